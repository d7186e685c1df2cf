"""Solve service: requests of mixed sizes and maps admitted by an HBM budget
and solved concurrently on worker streams.  Each result must equal the same
problem solved alone by cps_solve with the service's opts, bit for bit (the
service runs the same code), and the oracle's exact solution to 1e-9; a
pooled hierarchy reused for a new map (metrics and coarse inverse recomputed
in place, or rebuilt when the stencil class changes) must give the same bits
as a fresh one."""
import numpy as np
import pytest

import oracle as O
from oracle import direct
from paper_2305_17875_amd import cps, inputs
from paper_2305_17875_amd.inputs import Shell, MAP_OBLATE, MAP_TRIAXIAL
from gpu_util import needs_gpu, log, dev, host, rel

pytestmark = [pytest.mark.gpu, needs_gpu]

GiB = 1 << 30


def alone(g, b, precision=1):
    s = cps.Solver(g, precision=precision, accel=1)
    try:
        r = s.solve(dev(b).flatten())
        return host(r.p).reshape(g.shape), r
    finally:
        s.close()


def run(svc, reqs):
    tickets = [svc.submit(g, b) for g, b in reqs]
    return [svc.wait(t) for t in tickets]


def test_service_equals_alone_and_oracle():
    reqs = [
        (Shell(16, 16, 16), inputs.smoothed_noise((16, 16, 16), 1)),
        (Shell(32, 32, 64, map=MAP_OBLATE, flattening=0.1), inputs.smoothed_noise((32, 32, 64), 2)),
        (Shell(16, 16, 32, radial_stretch=2.0), inputs.smoothed_noise((16, 16, 32), 3)),
        (Shell(32, 32, 64, map=MAP_OBLATE, flattening=0.05), inputs.smoothed_noise((32, 32, 64), 4)),
        (Shell(16, 16, 16, map=MAP_TRIAXIAL, flattening=0.1, skew=0.1),
         inputs.smoothed_noise((16, 16, 16), 5)),
        (Shell(32, 32, 32), inputs.smoothed_noise((32, 32, 32), 6)),
        (Shell(32, 32, 64, map=MAP_OBLATE, flattening=0.12), inputs.smoothed_noise((32, 32, 64), 7)),
        (Shell(16, 16, 16), np.zeros((16, 16, 16))),
    ]
    log("service", len(reqs), "requests, 3 slots")
    svc = cps.Service(4 * GiB, max_slots=3)
    try:
        out = run(svc, reqs)
        st = svc.stats()
    finally:
        svc.close()
    for i, ((g, b), (status, p, info)) in enumerate(zip(reqs, out)):
        assert status == cps.CPS_OK, i
        xa, ra = alone(g, b)
        assert info.iterations == ra.iterations, i
        assert np.array_equal(p, xa), (i, np.abs(p - xa).max())
        if not b.any():
            assert info.iterations == 0 and not p.any()
        elif g.map != MAP_TRIAXIAL:
            want = direct.solve_axisym(O.face_metrics(g), b)
            assert rel(p, want) <= 1e-9, (i, rel(p, want))
        else:
            assert rel(p, direct.solve_sparse(O.face_metrics(g), b)) <= 1e-9, i
    assert st["submitted"] == st["completed"] == len(reqs) and st["failed"] == 0
    assert st["queued"] == 0 and st["active"] == 0
    assert 0 < st["p50_ms"] <= st["p99_ms"] <= st["max_ms"]
    assert st["hbm_in_use"] <= st["hbm_budget"]
    assert st["hierarchies_built"] + st["hierarchies_reused"] == len(reqs)


def test_service_reuses_and_remaps_hierarchies():
    """One slot: same dims with three oblate maps (two remaps in place), then
    flattening 0 (7-point class: the entry is rebuilt), then a sphere."""
    shape = (16, 16, 32)
    gs = [Shell(*shape, map=MAP_OBLATE, flattening=f) for f in (0.1, 0.05, 0.15, 0.0)]
    gs.append(Shell(*shape))
    reqs = [(g, inputs.smoothed_noise(shape, 20 + i)) for i, g in enumerate(gs)]
    log("service remap")
    svc = cps.Service(4 * GiB, max_slots=1)
    try:
        out = run(svc, reqs)
        st = svc.stats()
    finally:
        svc.close()
    for i, ((g, b), (status, p, info)) in enumerate(zip(reqs, out)):
        assert status == cps.CPS_OK, i
        xa, ra = alone(g, b)
        assert np.array_equal(p, xa), (i, np.abs(p - xa).max())
    assert st["hierarchies_built"] == 2, st  # oblate, and the sphere class
    assert st["hierarchies_reused"] == 3, st
    assert st["map_rebuilds"] == 2, st
    assert st["peak_active"] == 1


def test_service_budget_queues_evicts_and_rejects():
    """Room for one hierarchy of either of two shapes: alternating requests
    queue, evict the idle one and rebuild; a request that can never fit is
    rejected and the service stays usable."""
    ga = Shell(32, 32, 64, map=MAP_OBLATE, flattening=0.1)
    gb = Shell(32, 64, 32, map=MAP_OBLATE, flattening=0.1)
    huge = Shell(64, 64, 128)
    probe = cps.Service(GiB, max_slots=1)
    try:
        fa, fb, fh = probe.footprint(ga), probe.footprint(gb), probe.footprint(huge)
        probe.wait(probe.submit(ga, inputs.smoothed_noise(ga.shape, 1)))
        resident_a = probe.stats()["hbm_in_use"]  # ga's hierarchy after set-up
    finally:
        probe.close()
    budget = max(fa, fb) + min(fa, fb) // 5
    # the footprint covers the resident hierarchy (a service hierarchy keeps
    # the scratch of its coarsest inverse for remaps, so the two can be equal)
    assert 0 < resident_a <= fa and resident_a + fb > budget and fh > budget
    reqs = [(g, inputs.smoothed_noise(g.shape, 40 + i))
            for i, g in enumerate([ga, gb, ga, gb])]
    log("service budget", budget)
    svc = cps.Service(budget, max_slots=4)
    try:
        out = run(svc, reqs)
        st = svc.stats()
        t = svc.submit(huge, inputs.smoothed_noise(huge.shape, 9))
        with pytest.raises(cps.CpsError, match="budget"):
            svc.wait(t)
        st2, p2, _ = svc.wait(svc.submit(*reqs[0]))
    finally:
        svc.close()
    for i, ((g, b), (status, p, info)) in enumerate(zip(reqs, out)):
        assert status == cps.CPS_OK, i
        xa, _ = alone(g, b)
        assert np.array_equal(p, xa), i
    assert st["hierarchies_built"] == 4 and st["evictions"] == 3, st
    assert st["peak_active"] == 1 and st["hbm_in_use"] <= budget, st
    assert st2 == cps.CPS_OK and np.array_equal(p2, out[0][1])


def test_service_fp64_and_errors():
    g = Shell(16, 16, 32, radial_stretch=2.0)
    b = inputs.smoothed_noise(g.shape, 77)
    svc = cps.Service(GiB, max_slots=2, precision=0)
    try:
        status, p, info = svc.wait(svc.submit(g, b))
        bad = Shell(15, 16, 32)  # odd n_r: rejected at submission
        with pytest.raises(cps.CpsError):
            svc.submit(bad, np.zeros(bad.shape))
        nan = b.copy()
        nan[1, 2, 3] = np.nan
        st_nan, _, _ = svc.wait(svc.submit(g, nan))
        with pytest.raises(cps.CpsError, match="ticket"):
            cps.cps_service_wait(svc.h, 12345)
    finally:
        svc.close()
    xa, _ = alone(g, b, precision=0)
    assert status == cps.CPS_OK and np.array_equal(p, xa)
    assert st_nan == cps.CPS_E_DIVERGED


def test_autotuned_solve_gives_the_same_bits(tmp_path, monkeypatch):
    """Retuning the smoother's marching chunk (tune=2) changes no result;
    the choices land in the cache file."""
    cache = tmp_path / "tune.json"
    monkeypatch.setenv("CPS_TUNE_CACHE", str(cache))
    g = Shell(32, 32, 64, radial_stretch=2.0)
    b = dev(inputs.smoothed_noise(g.shape, 91)).flatten()
    out = []
    for tune in (2, 0):
        for precision in (0, 1):
            s = cps.Solver(g, precision=precision, accel=1, tune=tune)
            try:
                r = s.solve(b)
                out.append((host(r.p), r.iterations))
            finally:
                s.close()
    assert np.array_equal(out[0][0], out[2][0]) and out[0][1] == out[2][1]
    assert np.array_equal(out[1][0], out[3][0]) and out[1][1] == out[3][1]
    import json
    keys = json.loads(cache.read_text())
    assert "gs_march/f64/32x32x64" in keys and "gs_march/f32/32x32x64" in keys


@pytest.mark.parametrize("map_,f", [(inputs.MAP_SPHERE, 0.0), (inputs.MAP_OBLATE, 0.1)],
                         ids=["sphere", "oblate"])
def test_plane_launch_shapes_give_the_same_bits(tmp_path, monkeypatch, map_, f):
    """The plane smoother's launch shapes (rings per block of the transforms,
    r-steps in flight of the elimination) only schedule the same arithmetic:
    a solve with the shapes the autotuner picks (tune=2) equals one with the
    default shapes (tune=0 on a shape no earlier call has tuned), bit for
    bit, and the choices land in the cache file."""
    cache = tmp_path / "tune.json"
    monkeypatch.setenv("CPS_TUNE_CACHE", str(cache))
    g = Shell(24, 20, 64, map=map_, flattening=f, radial_stretch=1.5)
    b = dev(inputs.smoothed_noise(g.shape, 92)).flatten()
    for precision in (0, 1):
        out = []
        for tune in (0, 2):
            s = cps.Solver(g, precision=precision, accel=1, smoother=1, tune=tune)
            try:
                r = s.solve(b)
                out.append((host(r.p), r.iterations))
            finally:
                s.close()
        log("plane shapes", map_, precision, out[0][1], out[1][1])
        assert np.array_equal(out[0][0], out[1][0]) and out[0][1] == out[1][1]
    import json
    keys = json.loads(cache.read_text())
    cls = "rt" if map_ == inputs.MAP_OBLATE else "ortho"
    assert f"plane/f64/{cls}/24x20x64" in keys and f"plane/f32/{cls}/12x10x32" in keys


def test_service_concurrent_builds_captures_and_remaps():
    """Eight workers, all requests submitted at once: fresh hierarchies of
    several shapes (each first solve captures its iteration bodies into
    graphs) interleave with in-place remaps (every oblate request has its
    own flattening, so its coarsest inverse is recomputed) on the other
    workers.  Every request succeeds (no capture is invalidated by another
    worker's allocation, free or upload), and sampled results equal the
    same problems solved alone, bit for bit."""
    rng = np.random.default_rng(77)
    shapes = [(16, 16, 16), (16, 16, 32), (32, 16, 32), (16, 32, 64), (32, 32, 32), (32, 32, 64)]
    reqs = []
    for k in range(72):
        s = shapes[k % len(shapes)]
        if k % 2:
            g = Shell(*s, map=MAP_OBLATE, flattening=float(rng.uniform(0.02, 0.15)))
        else:
            g = Shell(*s, radial_stretch=float(rng.uniform(0.0, 2.0)))
        reqs.append((g, inputs.smoothed_noise(s, 500 + k)))
    log("service concurrency", len(reqs))
    for smoother in (0, 2):
        svc = cps.Service(4 * GiB, max_slots=8, precision=1, smoother=smoother)
        try:
            out = run(svc, reqs)
            st = svc.stats()
        finally:
            svc.close()
        assert all(o[0] == cps.CPS_OK for o in out), [o[0] for o in out]
        assert st["map_rebuilds"] > 0 and st["hierarchies_built"] >= len(shapes), st
        for i in (0, 7, 31, 70):
            g, b = reqs[i]
            s = cps.Solver(g, precision=1, accel=1, smoother=smoother)
            try:
                xa = host(s.solve(dev(b).flatten()).p).reshape(g.shape)
            finally:
                s.close()
            assert np.array_equal(out[i][1], xa), (smoother, i)
