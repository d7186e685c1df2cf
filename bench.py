"""Benchmark: Poisson unknowns/s to relative residual 1e-10 on the
paper-scale spherical shell (192 r x 256 theta x 512 phi cells, tanh radial
clustering with stretching factor 2.0, cone walls at 0.05 and pi - 0.05,
right-hand side = seeded N(0,1) field smoothed by 3 Jacobi passes, mean
removed), one MI355X.

A step is one complete cps_solve (FP64 hierarchy, conjugate gradients
preconditioned by one V(2,2) cycle) from the right-hand side resident in HBM
to relative residual 1e-10.  The FP32-multigrid + FP64-refinement form is
timed on the same input and reported beside it, and so is the same solve
with the zebra (r, phi)-plane smoother (`plane`); the whole projection step
around the solve is timed under `project`, and the implicit line solves of
the ADI steps under `lines`; the 64-problem batched form under `batch`, the
cache-resident 32^3 shell under `config1`, and a 60 s stream of Poisson
arrivals at 200/s through the solve service under `serve`.  The CPU leg
then times the oracle on the host (`cpu_baseline`) and computes the exact
discrete solution of the paper-scale shell and of every batch problem, and
each form's answer is compared with it (`error_vs_oracle`).  Prints one JSON
line.

Roofline: the dominant kernel is the finest-level Gauss-Seidel colour pass.
Its duration is measured live with HIP events recorded on the solve stream
around each of its launches in the timed region.  `traffic` comes from
profiles/gs_pass_config2_traffic.json (FETCH_SIZE / WRITE_SIZE counter runs,
scaled by the same counters on a plain copy of known size) when that file
was taken on the current kernel source, else null.
"""
import argparse
import hashlib
import json
import os
import sys
import statistics
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Poisson unknowns/s to 1e-10 residual, FP64 vs FP32-MG+IR; serve p50/p99 ms"
HBM_PEAK_GBS = 8000.0
TOL = 1e-10
KERNEL_SRC = os.path.join(ROOT, "paper_2305_17875_amd", "csrc", "kernels.hpp")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "gs_pass_config2_traffic.json")
PLANE_SRC = os.path.join(ROOT, "paper_2305_17875_amd", "csrc", "plane.hpp")
PLANE_TRAFFIC_FILE = os.path.join(ROOT, "profiles", "plane_half_sweep_config2_traffic.json")
VCYCLE_TRAFFIC_FILE = os.path.join(ROOT, "profiles", "vcycle_config2_fp64_traffic.json")
TILE_SRC = os.path.join(ROOT, "paper_2305_17875_amd", "csrc", "tile.hpp")
KNAMES = ["gs_pass", "residual", "apply", "restrict", "prolong", "vcycle", "divergence",
          "correct"]
GS_KERNEL = "k_gs_march2<double, 0, 0>"


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def kernel_hash(path=KERNEL_SRC) -> str:
    return hashlib.sha256(open(path, "rb").read()).hexdigest()[:16]


def plane_traffic(key):
    """Counter bytes of one finest-level half-sweep (fetch + write, scaled
    by the copy yardstick) while they were taken on the current plane
    kernel source, else None."""
    try:
        d = json.load(open(PLANE_TRAFFIC_FILE))
    except (OSError, ValueError):
        return None
    if d.get("kernel_source_sha256_16") != kernel_hash(PLANE_SRC) or key not in d:
        return None
    return d[key]["bytes_per_half_sweep"]


def gs_bytes_per_launch(shape, ncol, word, phi_invariant, nterms):
    """Algorithmic HBM bytes of one finest-level Gauss-Seidel colour pass:
    each updated cell reads its right-hand side and writes itself once,
    every cell of the other colours is read once as a neighbour, and the
    metric arrays are read once (per (r, theta) when phi-invariant)."""
    nr, nt, np_ = shape
    n = nr * nt * np_
    upd = n // ncol
    field = upd * 2 * word + (n - upd) * word
    coef = nterms * (nr * nt if phi_invariant else n) * word
    return field + coef


def fused_transfer(f, c):
    """Whether the V-cycle forms the red residual of level f inside its
    restriction to c (one pass, r never stored): a row-pair level halved in
    every direction whose coarse ring is one or two segments of 64 phi pairs
    and whose coarse theta count splits into the kernel's row groups (4 rows
    for one segment, 2 for two)."""
    (nr, nt, np_), (cr, ct, cp) = f, c
    if (np_ // 2) % 64 or nt % 2 or nr != 2 * cr or nt != 2 * ct or np_ != 2 * cp:
        return False
    if (cp // 2) % 64:
        return False
    segs = cp // 2 // 64
    return segs in (1, 2) and ct % (4 if segs == 1 else 2) == 0


def vcycle_bytes(levels, word, phi_invariant=True, fused=False, red_prolong=False):
    """Algorithmic HBM bytes of one V(2,2) cycle from a zero iterate on the
    7-point hierarchy with point red-black smoothing: per smoothed level of n
    cells, the zero-iterate pass (b and x of one colour: n words), seven full
    colour passes (b and x of the updated colour, x of the other: 1.5 n
    words each), the residual, the restriction and the prolongation (n/8 in,
    x in and out: 2 n + n/8), plus the three metric arrays per (r, theta)
    read by each of the 8 passes and the residual; the coarsest level reads
    its FP64 dense inverse once.

    The pre-smoothing ends on the black pass, which leaves the black
    residual zero.  On row-pair levels (n_phi / 2 a multiple of 64, n_theta
    even) only the red residual is formed and restricted: residual x in,
    red b in, red r out (2 n), restriction red r in, n/8 out -- 16.25 n
    words a level.  Elsewhere the full residual (x, b in, r out: 3 n) and
    restriction (n in, n/8 out) -- 17.75 n.

    fused (the library's cycles): where fused_transfer holds, the red residual is
    formed inside the restriction: x in, red b in, n/8 out, and r is neither
    written nor read back -- 15.25 n words.

    red_prolong (the library's cycles): the prolongation corrects only the
    red cells (the black pass that follows overwrites the black ones): red x
    in and out, n/8 in -- n words a level less."""
    total = 0
    for k, (nr, nt, np_) in enumerate(levels[:-1]):
        n = nr * nt * np_
        coef = 3 * nr * nt * (1 if phi_invariant else np_)
        red = (np_ // 2) % 64 == 0 and nt % 2 == 0
        words = 16.25 if red else 17.75
        if fused and fused_transfer(levels[k], levels[k + 1]):
            words = 15.25
        if red_prolong:
            words -= 1.0
        total += (words * n + 9 * coef) * word
    nc = levels[-1][0] * levels[-1][1] * levels[-1][2]
    return int(round(total)) + nc * nc * 8 + 2 * nc * word


def plane_half_sweep_bytes(shape, word):
    """Algorithmic HBM bytes of one zebra half-sweep of the plane smoother
    (the theta rows of one parity), per kernel with no cross-kernel fusion:
    the forward transform reads b of the relaxed rows and x of the other
    parity and writes the spectra; the r-line elimination reads and writes
    the spectra twice (down and up) and reads the inverse pivots twice; the
    inverse transform reads the spectra and writes x of the relaxed rows."""
    nr, nt, np_ = shape
    half = nr * nt * np_ // 2
    spec = nr * (nt // 2) * (np_ // 2 + 1) * 2  # words: (n_phi/2 + 1) complex per ring
    piv = spec // 2
    return (2 * half + spec + 4 * spec + 2 * piv + spec + half) * word


PROF_STEPS = 2


def run_form(cps, torch, g, rhs, precision, steps, warmup, smoother=0, graph_vcycle=True):
    """The timed solves run on a stream of the solver's own, as a user would
    set it up.  Inside the timed region HIP events are recorded on that
    stream around every launch of the finest-level smoothing pass only (the
    roofline's kernel; events around every class would add ~6% to the
    solve); PROF_STEPS more solves with events around every finest-level
    class give the kernel table, and PROF_STEPS more with events around the
    cycles only give the V-cycle span."""
    stream = torch.cuda.Stream()
    # set-up (hierarchy, metrics, coarsest inverse, smoother tables) is timed
    # on its own, outside the solves
    torch.cuda.synchronize()
    t_setup = time.perf_counter()
    s = cps.Solver(g, precision=precision, accel=1, max_iters=400, smoother=smoother,
                   stream=stream)
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t_setup
    p = torch.empty_like(rhs)
    torch.cuda.synchronize()
    for i in range(warmup):
        res = s.solve(rhs, TOL, out=p)
        log(f"warmup {i}: status={res.status} iterations={res.iterations} "
            f"{res.seconds * 1e3:.1f} ms")
    torch.cuda.synchronize()
    cps.cps_profile_select(s.h, [cps.KERNEL_GS])
    cps.cps_profile_enable(s.h, True)
    t0 = time.perf_counter()
    iters, solve_s = [], []
    for i in range(steps):
        # a solve returns after its result is written: the host clock
        # around it is the solve's own time
        t1 = time.perf_counter()
        res = s.solve(rhs, TOL, out=p)
        solve_s.append(time.perf_counter() - t1)
        iters.append(res.iterations)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    log(f"precision={precision} smoother={smoother}: timed solves done")
    timed_gs = cps.cps_profile_read(s.h, cps.KERNEL_GS)
    cps.cps_profile_select(s.h, None)
    for k in range(len(KNAMES)):
        cps.cps_profile_read(s.h, k)
    for i in range(PROF_STEPS):
        s.solve(rhs, TOL, out=p)
        log(f"profiled solve {i + 1}/{PROF_STEPS} (every finest-level class) done")
    prof = {k: cps.cps_profile_read(s.h, k) for k in range(len(KNAMES))}
    # the V-cycle span from solves with events around the cycles only: the
    # events around the finest-level kernels inside a cycle add ~4% to it
    vc = KNAMES.index("vcycle")
    cps.cps_profile_select(s.h, [vc])
    for i in range(PROF_STEPS):
        s.solve(rhs, TOL, out=p)
        log(f"profiled solve {i + 1}/{PROF_STEPS} (V-cycle spans) done")
    prof[vc] = cps.cps_profile_read(s.h, vc)
    cps.cps_profile_select(s.h, None)
    cps.cps_profile_enable(s.h, False)
    # the V-cycle as the solve runs it: replayed from a hipGraph (the spans
    # above launch every kernel from the host, as profiling requires); only
    # where the line reports the cycle's rate
    vcycle_graph_us = None
    if graph_vcycle:
        vcycle_graph_us, _ = s.time_vcycle(cycles=10, reps=5)
        torch.cuda.synchronize()
        log(f"graph-replayed V-cycle: {vcycle_graph_us:.1f} us")
    log(f"precision={precision} smoother={smoother}: {dt * 1e3:.1f} ms/solve, iterations={iters}, "
        f"rel_residual={res.rel_residual:.3e}")
    return dict(solver=s, p=p, host_p=p.cpu().numpy().reshape(g.shape), res=res, sec=dt,
                iters=iters, prof=prof, prof_steps=PROF_STEPS, vcycle_graph_us=vcycle_graph_us,
                setup_s=setup_s, solve_ms_median=statistics.median(solve_s) * 1e3,
                solve_ms_min=min(solve_s) * 1e3,
                timed_gs=timed_gs)


def kernel_table(prof, steps):
    out = {}
    for k, name in enumerate(KNAMES):
        ms, cnt = prof[k]
        out[name] = {"launches_per_step": cnt / steps,
                     "avg_us": round(ms / cnt * 1e3, 2) if cnt else None}
    return out


def vcycle_rate(prof, levels, word, steps, graph_us=None, traffic=None):
    """HBM rate of the preconditioning V-cycle: the byte model of
    vcycle_bytes over the time of one cycle.  graph_us: the cycle replayed
    from a hipGraph as the solve runs it (cps_time_vcycle), the rate's
    time; the span of each cycle measured with HIP events in solves that
    launch every kernel from the host (profiling) is reported beside it
    (eager_*), and is the rate's time when graph_us is None."""
    ms, cnt = prof[KNAMES.index("vcycle")]
    if not cnt:
        return None
    eager = ms / cnt * 1e-3
    t = graph_us * 1e-6 if graph_us else eager
    b = vcycle_bytes(levels, word, fused=True, red_prolong=True)
    out = {"bytes_per_cycle": b, "avg_us": t * 1e6, "achieved_GBs": b / t / 1e9,
           "frac_of_peak": b / t / 1e9 / HBM_PEAK_GBS, "cycles_per_step": cnt / steps,
           "timing": ("hipGraph replay of 10 cycles, 5 launches between events "
                      "(cps_time_vcycle)") if graph_us else "HIP events around each cycle, "
                                                            "kernels launched from the host"}
    if graph_us:
        out["eager_avg_us"] = eager * 1e6
        out["eager_frac_of_peak"] = b / eager / 1e9 / HBM_PEAK_GBS
    # the bytes the counters saw in one cycle (halo re-reads included) over
    # the same time: the sustained HBM rate
    out["traffic"] = None if traffic is None else {
        "bytes_per_cycle": traffic, "achieved_GBs": traffic / t / 1e9,
        "frac_of_peak": traffic / t / 1e9 / HBM_PEAK_GBS,
        "source": os.path.relpath(VCYCLE_TRAFFIC_FILE, ROOT)}
    return out


def yardstick(cps, torch, n):
    """Plain device copy of n doubles: ten back-to-back copies timed with
    events on the stream they run on (no host round trip between them).
    The byte counters are scaled by the library's own copy kernel in the
    profiles; this rate is the reference the kernels' rates are read
    against."""
    a = torch.ones(n, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    reps = 10
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    e1.synchronize()
    dt = e0.elapsed_time(e1) / 1e3 / reps
    del a, b
    return 16.0 * n / dt / 1e9


def plane_form(cps, torch, g, rhs, x64, steps, warmup, answers):
    """The same solve with the zebra (r, phi)-plane smoother in place of
    point red-black Gauss-Seidel (cps_opts.smoother = 1): FP64 and FP32
    cycles, each with its half-sweep rate against the byte model of
    plane_half_sweep_bytes."""
    out = {"smoother": "zebra (r,phi)-plane block Gauss-Seidel: FFT along phi, "
                       "Thomas along r per mode; V(2,2), PCG"}
    for precision, key, word in ((0, "fp64", 8), (1, "mixed", 4)):
        f = run_form(cps, torch, g, rhs, precision, steps, warmup, smoother=1,
                     graph_vcycle=False)
        answers[("plane", key)] = f["host_p"]
        hs_ms, hs_n = f["timed_gs"]  # HIP events over the timed region
        hs_s = hs_ms / max(hs_n, 1) * 1e-3
        hb = plane_half_sweep_bytes(g.shape, word)
        err = float(torch.linalg.norm(f["p"] - x64) / torch.linalg.norm(x64))
        out[key] = {"value": g.cells / f["sec"], "unit": "unknowns/s",
                    "ms_per_step": f["sec"] * 1e3, "setup_ms": f["setup_s"] * 1e3,
                    "iterations": f["iters"][-1],
                    "rel_residual": f["res"].rel_residual, "rel_diff_vs_fp64_point": err,
                    "half_sweep": {"avg_us": hs_s * 1e6, "per_step": hs_n / steps,
                                   "algorithmic_bytes": hb, "achieved_GBs": hb / hs_s / 1e9,
                                   "frac_of_peak": hb / hs_s / 1e9 / HBM_PEAK_GBS,
                                   "traffic": plane_traffic("fp64" if precision == 0 else "fp32")},
                    "kernels": kernel_table(f["prof"], f["prof_steps"])}
        f["solver"].close()
        del f
        torch.cuda.empty_cache()
    return out


def project_form(cps, torch, inputs, g, steps, warmup):
    """One projection step (cps_project: divergence right-hand side of eq.
    (PC_6), the solve, the correction of eq. (PC_7)) on a synthetic
    intermediate velocity, with the FP64 point-smoother solve of the headline
    and with the plane smoother.  The velocity is restored before each step
    outside the timed region.  Kernel rates against per-cell byte models:
    divergence reads 3 velocity words and writes 1; the correction reads phi
    and 3 velocity words and writes 3 (the face tables of a map symmetric
    about the polar axis are one row per (r, theta))."""
    u0 = torch.from_numpy(inputs.velocity_field(g.shape, 40)).cuda().flatten()
    n = g.cells
    out = {"workload": "u*** = three smoothed N(0,1) fields (seeds 40-42) as Cartesian "
                       "components on the paper-scale shell; tol 1e-10"}
    for key, smoother in (("fp64_point", 0), ("fp64_plane", 1)):
        stream = torch.cuda.Stream()
        s = cps.Solver(g, precision=0, accel=1, max_iters=400, smoother=smoother, stream=stream)
        u = torch.empty_like(u0)
        phi = torch.empty(n, dtype=torch.float64, device="cuda")
        for _ in range(warmup):
            u.copy_(u0)
            torch.cuda.synchronize()
            s.project(u, TOL, phi=phi)
        torch.cuda.synchronize()
        total, its = 0.0, []
        for _ in range(steps):
            u.copy_(u0)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            r = s.project(u, TOL, phi=phi)
            torch.cuda.synchronize()
            total += time.perf_counter() - t0
            its.append(r.iterations)
        log(f"project {key}: timed steps done")
        u.copy_(u0)
        torch.cuda.synchronize()
        cps.cps_profile_enable(s.h, True)
        s.project(u, TOL, phi=phi)
        log(f"project {key}: profiled step done")
        prof = {k: cps.cps_profile_read(s.h, k) for k in range(len(KNAMES))}
        cps.cps_profile_enable(s.h, False)
        dt = total / steps
        rates = {}
        for name, cls, words in (("divergence", cps.KERNEL_DIVERGENCE, 4),
                                 ("correct", cps.KERNEL_CORRECT, 7)):
            ms, cnt = prof[cls]
            t = ms / max(cnt, 1) * 1e-3
            b = words * 8 * n
            rates[name] = {"avg_us": t * 1e6, "algorithmic_bytes": b,
                           "achieved_GBs": b / t / 1e9, "frac_of_peak": b / t / 1e9 / HBM_PEAK_GBS}
        out[key] = {"value": n / dt, "unit": "unknowns/s", "ms_per_step": dt * 1e3,
                    "iterations": its[-1], "status": r.status, "kernels": rates}
        log(f"project {key}: {dt * 1e3:.1f} ms/step, iterations {its}")
        s.close()
        del u, phi
    del u0
    torch.cuda.empty_cache()
    return out


def lines_form(cps, torch, inputs, g, steps, warmup):
    """The implicit line solves of the ADI steps (cps_line_solve) along each
    direction on the paper-scale shell, coef 1e-4, value 0 on the low wall
    and no flux on the high wall.  Timed with events on the solve stream;
    rates against the design's bytes per cell: open r- and theta-lines read
    the right-hand side and write psi on the way down, read and write psi on
    the way up (4 words); periodic phi-lines with a power-of-two ring are
    solved by one transform per ring in LDS (read once, written once: 2
    words), other rings by the split with a closing row (12 words)."""
    n = g.cells
    rhs = torch.from_numpy(inputs.smoothed_noise(g.shape, 50)).cuda().flatten()
    psi = torch.empty_like(rhs)
    s = cps.Solver(g, precision=0)
    out = {"workload": "paper-scale shell, smoothed N(0,1) rhs seed 50, coef 1e-4, "
                       "bc: value 0 at the low wall, no flux at the high wall"}
    bc = (1, 0.0, 0, 0.0)
    nh = g.n_phi // 2
    phi_words = 2 if nh >= 2 and nh & (nh - 1) == 0 and nh <= 1024 else 12
    for d, name, words in ((0, "r", 4), (1, "theta", 4), (2, "phi_periodic", phi_words)):
        for _ in range(warmup):
            s.line_solve(d, 1e-4, rhs, bc, out=psi)
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
        torch.cuda.synchronize()
        ev[0].record()
        for _ in range(steps):
            s.line_solve(d, 1e-4, rhs, bc, out=psi)
        ev[1].record()
        torch.cuda.synchronize()
        t = ev[0].elapsed_time(ev[1]) / steps * 1e-3
        b = words * 8 * n
        out[name] = {"avg_us": t * 1e6, "unknowns_per_s": n / t, "algorithmic_bytes": b,
                     "achieved_GBs": b / t / 1e9, "frac_of_peak": b / t / 1e9 / HBM_PEAK_GBS}
        log(f"lines {name}: {t * 1e6:.1f} us")
    s.close()
    del rhs, psi
    torch.cuda.empty_cache()
    return out


def config1_form(cps, torch, inputs, steps, warmup):
    """The cache-resident 32^3 shell (uniform radius, cone walls): a plain
    FP64 V(2,2) red-black iteration (`vcycle`, accel 0) and the same cycle
    under conjugate gradients (`pcg`), to relative residual 1e-10.  The
    right-hand side is A p_s for the manufactured p_s = cos(pi xi) sin(2 phi)
    sin(theta), formed by the library's own operator (cps_debug_apply), so
    the exact answer is p_s - mean(p_s).  The working set (a few MB) stays in
    the caches: the figures are time per solve, per iteration and per
    V-cycle, which show the launch overhead, not an HBM fraction."""
    g = inputs.config1()
    ps = inputs.manufactured_p(g)
    want = ps - ps.mean()
    out = {"workload": "sphere shell 32^3, r 1.5..2.5 uniform, theta 0.05..pi-0.05, "
                       "rhs = A p_s (p_s = cos(pi xi) sin(2 phi) sin(theta)), rel residual 1e-10"}
    stream = torch.cuda.Stream()
    for accel, key in ((0, "vcycle"), (1, "pcg")):
        s = cps.Solver(g, precision=0, accel=accel, max_iters=500, stream=stream)
        pd = torch.from_numpy(ps).cuda().flatten()
        b = torch.empty_like(pd)
        cps.cps_debug_apply(s.h, 0, pd, b)
        p = torch.empty_like(b)
        for _ in range(warmup):
            s.solve(b, TOL, out=p)
        times, its = [], []
        for _ in range(max(steps, 5)):
            t0 = time.perf_counter()
            res = s.solve(b, TOL, out=p)  # returns once p is written
            times.append(time.perf_counter() - t0)
            its.append(res.iterations)
        x = p.cpu().numpy().reshape(g.shape)
        err = float(np.linalg.norm(x - want) / np.linalg.norm(want))
        t = statistics.median(times)
        entry = {"solve_ms_median": t * 1e3, "solve_ms_min": min(times) * 1e3,
                 "iterations": its[-1], "ms_per_iteration": t * 1e3 / its[-1],
                 "rel_residual": res.rel_residual, "status": res.status,
                 "rel_error_vs_exact": err, "unknowns_per_s": g.cells / t}
        if accel == 1:
            # the preconditioning V-cycle alone, HIP events around each cycle
            # (profiling launches every kernel directly: no graph replay)
            vc = KNAMES.index("vcycle")
            cps.cps_profile_select(s.h, [vc])
            cps.cps_profile_enable(s.h, True)
            s.solve(b, TOL, out=p)
            ms, cnt = cps.cps_profile_read(s.h, vc)
            cps.cps_profile_enable(s.h, False)
            entry["vcycle_us_direct_launches"] = ms / max(cnt, 1) * 1e3
            # the same cycle replayed from a hipGraph, as the solve runs it,
            # and the kernel nodes one cycle's graph holds
            entry["vcycle_us_graph"], entry["launches_per_vcycle"] = s.time_vcycle(cycles=10, reps=5)
        out[key] = entry
        log(f"config1 {key}: {t * 1e3:.2f} ms/solve, {its[-1]} iterations, error {err:.2e}")
        s.close()
    return out


def cpu_model():
    """CPU model name and the logical CPUs this process may run on."""
    name = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                name = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return name, len(os.sched_getaffinity(0))


def cpu_baseline(g, rhs_np, answers, batch_ref):
    """The CPU leg: the oracle timed on this host, and the oracle's exact
    answers that every GPU result is compared with.

    Timing: the oracle's own multigrid (same level plan, V(2,2) red-black
    cycle, transfers, coarse solve and conjugate-gradient outer iteration as
    the FP64 form) built with gcc -O3 -march=native on this host, one full
    solve of the paper-scale shell to 1e-10 on every CPU this process may use
    (set-up timed apart), and one outer iteration on a single thread.
    Errors: the exact discrete solution of the paper-scale shell (rFFT in phi
    and sparse LU per azimuthal mode, oracle.direct) against the answer of
    each GPU form, and the same for every problem of the batched form."""
    import oracle as O
    from oracle import direct
    O.use_native_build()
    model, cpus = cpu_model()
    O.set_threads(cpus)
    threads = O.max_threads()
    og = O.Grid(g.n_r, g.n_theta, g.n_phi, map=g.map, r_inner=g.r_inner, r_outer=g.r_outer,
                theta0=g.theta0, theta1=g.theta1, radial_stretch=g.radial_stretch)
    t0 = time.perf_counter()
    mg = O.Multigrid(og)
    setup = time.perf_counter() - t0
    log(f"cpu baseline: oracle set-up {setup:.1f} s on {threads} threads ({model})")
    t0 = time.perf_counter()
    x, st, it, rel, _, _ = mg.solve(rhs_np, tol=TOL, max_iters=400, accel=1)
    solve_s = time.perf_counter() - t0
    log(f"cpu baseline: full solve {solve_s:.1f} s, {it} iterations, rel {rel:.2e}")
    O.set_threads(1)
    t0 = time.perf_counter()
    mg.solve(rhs_np, tol=1e-300, max_iters=1, accel=1)
    one = time.perf_counter() - t0
    O.set_threads(threads)
    del mg
    log(f"cpu baseline: one iteration on one thread {one:.1f} s")
    n = g.cells
    out = {"value": n / solve_s, "unit": "unknowns/s", "cores": threads, "kind": "oracle",
           "sample": f"one full solve of the paper-scale shell {g.n_r}x{g.n_theta}x{g.n_phi} to "
                     f"rel residual 1e-10 by the oracle's V(2,2) multigrid with conjugate "
                     f"gradients ({it} iterations, {solve_s:.1f} s; set-up {setup:.1f} s "
                     f"apart) on {threads} OpenMP threads",
           "status": st, "iterations": it, "rel_residual": rel, "seconds": solve_s,
           "setup_s": setup, "single_thread_s_per_iteration": one,
           "single_thread_unknowns_per_s_est": n / (one * it),
           "cpu_model": model, "logical_cpus": cpus, "build": "gcc -O3 -march=native -fopenmp"}
    # exact answers
    errors = {}
    workers = max(1, min(16, cpus))
    t0 = time.perf_counter()
    G = O.face_metrics(og)
    with direct.mode_pool(workers) as pool:
        xe = direct.solve_axisym(G, rhs_np, pool=pool)
        del G
        for key, xg in answers.items():
            errors[key] = error_stats(xg, xe)
        out["oracle_cpu_rel_error_vs_exact"] = error_stats(x, xe)["rel_l2"]
        worst = None
        for (grid, b, xg) in batch_ref:
            e = error_stats(xg, direct.solve_axisym(O.face_metrics(grid), b, pool=pool))
            if worst is None or e["rel_l2"] > worst["rel_l2"]:
                worst = dict(e, shape=list(grid.shape), map=grid.map)
        if worst is not None:
            errors["batch_worst"] = worst
    log(f"cpu baseline: exact answers in {time.perf_counter() - t0:.1f} s")
    return out, errors


def error_stats(x, want):
    """Relative L2 error, and the largest element error over max |want|."""
    return {"rel_l2": float(np.linalg.norm(x - want) / np.linalg.norm(want)),
            "max": float(np.abs(x - want).max() / np.abs(want).max())}


def batch_form(cps, torch, inputs, n_problems, steps, warmup, smoother, batch_ref):
    """64 uneven-size problems (half spherical, half oblate with flattening
    0.1) solved together by the batched form, against the same problems
    solved one after another by cps_solve with the same options.  smoother 2
    (automatic): the spheres run the plane smoother as a group of their own,
    the oblate shells the plane smoother with r-theta cross terms as
    another."""
    probs = inputs.batch_problems(n_problems)
    grids = [p.grid for p in probs]
    log(f"batch: generating {n_problems} right-hand sides")
    rhs = [torch.from_numpy(p.rhs()).cuda().flatten() for p in probs]
    cells = sum(g.cells for g in grids)
    t0 = time.perf_counter()
    B = cps.Batch(grids, tune=1, smoother=smoother)
    setup = time.perf_counter() - t0
    out = [torch.empty_like(r) for r in rhs]
    for _ in range(warmup):
        B.solve(rhs, TOL, out=out)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        st, _, infos = B.solve(rhs, TOL, out=out)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    B.close()
    for p, o in zip(probs, out):
        batch_ref.append((p.grid, p.rhs(), o.cpu().numpy().reshape(p.grid.shape)))
    its = [i.iterations for i in infos]
    worst = max(i.rel_residual for i in infos)
    log(f"batch: {dt * 1e3:.1f} ms per batch solve, status {st}, iterations {min(its)}..{max(its)}")
    # the same problems one at a time (hierarchies built beforehand)
    solvers = [cps.Solver(g, precision=1, accel=1, smoother=smoother) for g in grids]
    for s, r, o in zip(solvers, rhs, out):
        s.solve(r, TOL, out=o)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s, r, o in zip(solvers, rhs, out):
        s.solve(r, TOL, out=o)
    torch.cuda.synchronize()
    seq = time.perf_counter() - t0
    for s in solvers:
        s.close()
    log(f"batch: sequential {seq * 1e3:.1f} ms")
    return {"value": cells / dt, "unit": "unknowns/s", "ms_per_step": dt * 1e3,
            "problems": n_problems, "cells": cells, "status": st,
            "iterations_min": min(its), "iterations_max": max(its), "worst_rel_residual": worst,
            "setup_s": setup, "sequential_ms": seq * 1e3, "speedup_vs_sequential": seq / dt,
            "dtype": "f32 V-cycles, f64 outer",
            "smoother": {0: "point red-black", 2: "automatic: zebra plane for the spheres and "
                                                  "(with r-theta cross terms) the oblate "
                                                  "shells"}[smoother],
            "workload": f"{n_problems} shells, sizes by seed 4 from 16^3, 32^3, 64x64x128, "
                        "96x128x256, 128x128x256; even index sphere, odd oblate f=0.1; "
                        "smoothed N(0,1) rhs seeds 1000+i; rel residual 1e-10"}


def pinned(shape):
    """A host array in page-locked memory (a new pinned tensor), so that the
    service's host<->device copies run as DMA at full link speed."""
    import torch
    return torch.empty(shape, dtype=torch.float64, pin_memory=True).numpy()


def rhs_pool(inputs, shapes, per_shape):
    out = {}
    for s in shapes:
        out[s] = []
        for k in range(per_shape):
            a = pinned(s)
            a[...] = inputs.smoothed_noise(s, seed=10**6 + k)
            out[s].append(a)
    return out


class OutPool:
    """Pinned output arrays per shape, all allocated up front (taken at
    submission, returned once the request has been waited for).  No host
    memory is pinned while the stream runs: pinning memory on the submitting
    thread while a service worker captures a hipGraph has invalidated that
    capture.  take() waits for a returned array when none is free."""

    def __init__(self, shapes, per_shape):
        import threading
        self.free = {s: [pinned(s) for _ in range(per_shape)] for s in shapes}
        self.cv = threading.Condition()

    def take(self, shape, timeout=60.0):
        with self.cv:
            if not self.cv.wait_for(lambda: self.free[shape], timeout=timeout):
                raise RuntimeError(f"no free output array of shape {shape} in {timeout} s")
            return self.free[shape].pop()

    def give(self, a):
        with self.cv:
            self.free[a.shape].append(a)
            self.cv.notify_all()


# output arrays per request size: more than the requests of one size ever in
# flight at once (they complete in tens of ms at 200 arrivals/s)
OUT_PER_SHAPE = 24


def serve_form(cps, inputs, duration, rate, slots, budget_gib, comparator_s, smoother=2):
    """Poisson arrivals at `rate`/s for `duration` s submitted in real time
    to the solve service (FP32 V-cycles in FP64 refinement, hierarchies kept
    resident); then the requests that arrive in the first `comparator_s`
    seconds of the same stream served one at a time by a plain FP64
    cps_setup + cps_solve per request (a fixed sample: one at a time the
    plain solve serves a fifth of the stream's demand, so the whole stream
    would take minutes)."""
    import threading
    import numpy as np
    arr = inputs.arrival_stream(rate=rate, duration=duration)
    pool = rhs_pool(inputs, inputs.SIZE_SET, 4)
    demand = sum(a.problem.grid.cells for a in arr) / duration
    svc = cps.Service(budget_gib * (1 << 30), max_slots=slots, precision=1, accel=1,
                      smoother=smoother)
    # warm the code paths once per (size, class) so that start-up compiles
    # and tuning are not in the measured stream
    outs = OutPool(inputs.SIZE_SET, OUT_PER_SHAPE)
    for s in inputs.SIZE_SET:
        for g in (inputs.Shell(*s), inputs.Shell(*s, map=inputs.MAP_OBLATE, flattening=0.1)):
            o = outs.take(s)
            svc.wait(svc.submit(g, pool[s][0], TOL, out=o))
            outs.give(o)
    base = svc.stats()
    tickets = []
    lock = threading.Lock()
    results = []

    def waiter():
        k = 0
        while True:
            with lock:
                t = tickets[k] if k < len(tickets) else None
            if t is None:
                if k >= len(arr):
                    return
                time.sleep(0.0005)
                continue
            st, p, info = svc.wait(t)
            outs.give(p)
            results.append((st, info.iterations))
            k += 1

    th = threading.Thread(target=waiter)
    th.start()
    t0 = time.perf_counter()
    for a in arr:
        d = t0 + a.t - time.perf_counter()
        if d > 0:
            time.sleep(d)
        s = a.problem.grid.shape
        t = svc.submit(a.problem.grid, pool[s][a.rid % 4], TOL, out=outs.take(s))
        with lock:
            tickets.append(t)
    th.join()
    wall = time.perf_counter() - t0
    st = svc.stats()
    svc.close()
    fails = sum(1 for r in results if r[0] != cps.CPS_OK)
    cells = sum(a.problem.grid.cells for a in arr)
    out = {"rate_per_s": rate, "duration_s": duration, "requests": len(arr),
           "failed": fails, "p50_ms": st["p50_ms"], "p99_ms": st["p99_ms"],
           "mean_ms": st["mean_ms"], "max_ms": st["max_ms"],
           "unknowns_per_s": cells / wall, "demand_unknowns_per_s": demand,
           "drain_s": wall - duration, "slots": slots, "hbm_budget_gib": budget_gib,
           "peak_active": st["peak_active"],
           "hierarchies_built": st["hierarchies_built"] - base["hierarchies_built"],
           "hierarchies_reused": st["hierarchies_reused"] - base["hierarchies_reused"],
           "map_rebuilds": st["map_rebuilds"] - base["map_rebuilds"],
           "evictions": st["evictions"] - base["evictions"],
           "dtype": "f32 V-cycles, f64 outer",
           "smoother": {0: "point red-black", 1: "zebra plane",
                        2: "automatic: zebra plane where the hierarchy allows it (spheres, "
                           "oblate shells), point red-black otherwise"}[smoother],
           "workload": f"Poisson arrivals {rate}/s for {duration} s (seed 5), sizes uniform over "
                       "16^3, 32^3, 64x64x128, 96x128x256, 128x128x256, sphere or oblate "
                       "f~U(0,0.15); rhs from 4 smoothed N(0,1) fields per size; tol 1e-10; "
                       "host rhs in, host p out (pinned host arrays)"}
    out["p50_p99_note"] = ("latency = submission to completion, p50/p99 over this stream "
                           "(the latency percentiles include queueing: at this rate the stream "
                           "asks for more unknowns/s than one GPU serves)"
                           # work left queued when the arrivals stop, beyond the
                           # last requests' own latency
                           if wall - duration > max(0.05 * duration, 2e-3 * st["p99_ms"]) else
                           "latency = submission to completion, p50/p99 over this stream")
    log(f"serve: {len(arr)} requests, p50 {st['p50_ms']:.1f} ms p99 {st['p99_ms']:.1f} ms, "
        f"{cells / wall / 1e6:.1f} M unknowns/s (demand {demand / 1e6:.1f} M)")
    if comparator_s > 0:
        import torch
        lat = []
        sample = [a for a in arr if a.t < comparator_s]
        cells = sum(a.problem.grid.cells for a in sample)
        t0 = time.perf_counter()
        for a in sample:
            d = t0 + a.t - time.perf_counter()
            if d > 0:
                time.sleep(d)
            g = a.problem.grid
            s = cps.Solver(g, precision=0, accel=1)
            r = torch.from_numpy(pool[g.shape][a.rid % 4]).cuda().flatten()
            res = s.solve(r, TOL)
            p = outs.take(g.shape)
            torch.from_numpy(p).flatten().copy_(res.p)
            outs.give(p)
            s.close()
            lat.append(time.perf_counter() - (t0 + a.t))
        wall_c = time.perf_counter() - t0
        lat = np.array(lat) * 1e3
        out["comparator_fp64_per_request"] = {
            "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
            "mean_ms": float(lat.mean()), "unknowns_per_s": cells / wall_c,
            "requests": len(sample), "sample_s": comparator_s,
            "what": f"the requests arriving in the first {comparator_s:g} s of the same stream, "
                    "one at a time: FP64 cps_setup + cps_solve + cps_destroy per request, host "
                    "rhs in, host p out"}
        log(f"serve comparator: p50 {np.percentile(lat, 50):.1f} ms p99 "
            f"{np.percentile(lat, 99):.1f} ms, {cells / wall_c / 1e6:.1f} M unknowns/s")
    return out


def vcycle_traffic():
    """Counter bytes of one FP64 V-cycle (profiles/), if they were taken on
    the current kernel sources (kernels.hpp and tile.hpp)."""
    try:
        d = json.load(open(VCYCLE_TRAFFIC_FILE))
    except (OSError, ValueError):
        return None
    h = hashlib.sha256()
    for path in (KERNEL_SRC, TILE_SRC):
        h.update(open(path, "rb").read())
    if d.get("source_sha256_16") != h.hexdigest()[:16]:
        return None
    return d.get("bytes_per_cycle")


def traffic_for(kh):
    """Per-launch HBM bytes of the finest-level colour pass from the counter
    summary, if it was taken on this kernel source."""
    try:
        d = json.load(open(TRAFFIC_FILE))
    except (OSError, ValueError):
        return None
    if d.get("kernel_source_sha256_16") != kh:
        return None
    return d.get("bytes_per_launch")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--no-plane", action="store_true")
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--no-project", action="store_true")
    ap.add_argument("--no-lines", action="store_true")
    ap.add_argument("--batch-problems", type=int, default=64)
    ap.add_argument("--batch-smoother", type=int, default=2, choices=[0, 2])
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--serve-seconds", type=float, default=60.0)
    ap.add_argument("--serve-rate", type=float, default=200.0)
    ap.add_argument("--serve-slots", type=int, default=8)
    ap.add_argument("--serve-smoother", type=int, default=2,
                    help="0 point, 1 plane, 2 automatic (plane where the hierarchy allows it)")
    ap.add_argument("--serve-comparator-seconds", type=float, default=5.0,
                    help="serve the requests of the first this many seconds of the stream one "
                         "at a time with plain FP64 solves (0: skip)")
    ap.add_argument("--no-config1", action="store_true")
    a = ap.parse_args()
    if a.gpus != 1:
        print(f"bench.py measures one GPU (asked for --gpus {a.gpus}): a grid's solve runs on "
              "a single device; run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    # the autotuner's choices (the batched form tunes its shapes) land here
    import tempfile
    tune_cache = os.path.join(tempfile.mkdtemp(prefix="cps_tune_"), "tune.json")
    os.environ["CPS_TUNE_CACHE"] = tune_cache

    import torch
    from paper_2305_17875_amd import cps, inputs

    torch.cuda.set_device(0)
    g = inputs.config2()
    n = g.cells
    copy_gbs = yardstick(cps, torch, n)
    log(f"yardstick copy {copy_gbs:.0f} GB/s")
    log(f"generating rhs {g.shape}")
    rhs_np = inputs.smoothed_noise(g.shape, seed=0)
    rhs = torch.from_numpy(rhs_np).cuda().flatten()

    f64 = run_form(cps, torch, g, rhs, 0, a.steps, a.warmup)
    s64 = f64["solver"]
    gs_ms, gs_n = f64["timed_gs"]  # HIP events over the timed region
    avg_gs_s = gs_ms / max(gs_n, 1) * 1e-3
    nterms = {2: 3, 4: 5}[s64.ncolours] if s64.phi_invariant else 9
    gs_bytes = gs_bytes_per_launch(g.shape, s64.ncolours, 8, s64.phi_invariant, nterms)
    achieved = gs_bytes / avg_gs_s / 1e9
    kh = kernel_hash()
    line = {
        "metric": METRIC,
        "value": n / f64["sec"],
        "unit": "unknowns/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": f64["sec"] * 1e3,
        "setup_ms": f64["setup_s"] * 1e3,  # once per hierarchy; not in ms_per_step
        "solve_ms_median": f64["solve_ms_median"],
        "solve_ms_min": f64["solve_ms_min"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "spherical shell 192(r)x256(theta)x512(phi), tanh radial "
                               "clustering 2.0, smoothed N(0,1) rhs seed 0, rel residual 1e-10",
                   "cells": n, "levels": len(s64.levels), "outer": "pcg",
                   "colours": s64.ncolours},
        "iterations": f64["iters"][-1],
        "rel_residual": f64["res"].rel_residual,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic_for(kh),
                     "kernel": GS_KERNEL + " (finest-level red-black colour pass, row pairs; "
                               "the zero-iterate first pass of a cycle is a kernel of its own)",
                     "avg_us": avg_gs_s * 1e6, "algorithmic_bytes": gs_bytes,
                     "kernel_source_sha256_16": kh, "copy_yardstick_GBs": copy_gbs,
                     "frac_of_copy": achieved / copy_gbs if copy_gbs else None},
        "kernels_fp64": kernel_table(f64["prof"], f64["prof_steps"]),
        "vcycle_fp64": vcycle_rate(f64["prof"], s64.levels, 8, f64["prof_steps"],
                                   f64["vcycle_graph_us"], vcycle_traffic()),
    }
    x64 = f64["p"]
    answers = {("fp64",): f64["host_p"]}  # GPU answers, compared with the oracle's exact one
    if not a.no_mixed:
        mx = run_form(cps, torch, g, rhs, 1, a.steps, a.warmup)
        err = float(torch.linalg.norm(mx["p"] - x64) / torch.linalg.norm(x64))
        line["mixed"] = {"value": n / mx["sec"], "ms_per_step": mx["sec"] * 1e3,
                         "setup_ms": mx["setup_s"] * 1e3,
                         "solve_ms_median": mx["solve_ms_median"],
                         "solve_ms_min": mx["solve_ms_min"],
                         "iterations": mx["iters"][-1], "rel_residual": mx["res"].rel_residual,
                         "rel_diff_vs_fp64": err, "dtype": "f32 V-cycles, f64 outer",
                         "kernels": kernel_table(mx["prof"], mx["prof_steps"]),
                         "vcycle": vcycle_rate(mx["prof"], mx["solver"].levels, 4, mx["prof_steps"],
                                               mx["vcycle_graph_us"])}
        answers[("mixed",)] = mx["host_p"]
        mx["solver"].close()
        del mx
    s64.close()
    if not a.no_plane:
        torch.cuda.empty_cache()
        line["plane"] = plane_form(cps, torch, g, rhs, x64, a.steps, a.warmup, answers)
    del x64, f64, rhs
    torch.cuda.empty_cache()
    if not a.no_project:
        line["project"] = project_form(cps, torch, inputs, g, a.steps, a.warmup)
    if not a.no_lines:
        line["lines"] = lines_form(cps, torch, inputs, g, a.steps, a.warmup)
    batch_ref = []
    if not a.no_batch:
        line["batch"] = batch_form(cps, torch, inputs, a.batch_problems, a.steps, a.warmup,
                                   a.batch_smoother, batch_ref)
        try:  # "plane/f32/<stencil>/<dims>": 100 x rings per block + r-steps in flight
            line["batch"]["tuned_shapes"] = {k: v for k, v in json.load(open(tune_cache)).items()
                                             if k.startswith("plane/f32/")}
        except (OSError, ValueError):
            line["batch"]["tuned_shapes"] = None
        torch.cuda.empty_cache()
    if not a.no_config1:
        line["config1"] = config1_form(cps, torch, inputs, a.steps, a.warmup)
    if not a.no_serve:
        line["serve"] = serve_form(cps, inputs, a.serve_seconds, a.serve_rate, a.serve_slots,
                                   64, a.serve_comparator_seconds, a.serve_smoother)
    if not a.no_cpu_baseline:
        log("cpu baseline (oracle)")
        line["cpu_baseline"], errors = cpu_baseline(g, rhs_np, answers, batch_ref)
        # each form's error against the oracle's exact solution
        line["error_vs_oracle"] = errors.pop(("fp64",))
        if ("mixed",) in errors:
            line["mixed"]["error_vs_oracle"] = errors.pop(("mixed",))
        for key in ("fp64", "mixed"):
            if ("plane", key) in errors:
                line["plane"][key]["error_vs_oracle"] = errors.pop(("plane", key))
        if "batch_worst" in errors:
            line["batch"]["worst_error_vs_oracle"] = errors.pop("batch_worst")
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
