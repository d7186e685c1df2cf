"""Summarise rocprofv3 result databases of bench.py into short text.

    python -m paper_2305_17875_amd.profsum --kt KT.db --fetch F.db --write W.db \\
        --cmd "<the rocprofv3 commands>" --md out.md --traffic out.json \\
        [--plane-md plane.md --plane-traffic plane.json]

--kt     database of `rocprofv3 --kernel-trace --stats -- python3 bench.py ...`
--fetch  database(s) of `rocprofv3 --pmc FETCH_SIZE -- python3 bench.py ...`
--write  database(s) of `rocprofv3 --pmc WRITE_SIZE -- python3 bench.py ...`
         (several runs, e.g. one per bench form, are merged kernel by kernel)

Counter values (KiB per dispatch) are scaled by what the same counter reads
on the library's plain copy kernel (k_copy) over 192*256*512 doubles
(201,326,592 bytes read and written; every solve copies its right-hand side
with it), which turns them into bytes.  The traffic JSON records
the finest-level Gauss-Seidel kernel's bytes per launch together with a hash
of the kernel source, so bench.py can tell whether it is still current.  The
plane outputs do the same for the three kernels of one zebra half-sweep of
the plane smoother on the finest level (largest grid of each), FP64 and
FP32, with a hash of the plane kernels' source.
"""
from __future__ import annotations

import argparse
import collections
import hashlib
import json
import os
import sqlite3

HERE = os.path.dirname(os.path.abspath(__file__))
KERNEL_SRC = os.path.join(HERE, "csrc", "kernels.hpp")
TILE_SRC = os.path.join(HERE, "csrc", "tile.hpp")
PLANE_SRC = os.path.join(HERE, "csrc", "plane.hpp")
PLANE_KERNELS = ("k_plane_fwd", "k_plane_tri", "k_plane_inv")
COPY_BYTES = 192 * 256 * 512 * 8
GS_FINEST = "k_gs_march2<double, 0, 0>"


def short(name: str) -> str:
    return name.split("(")[0].replace("void ", "").replace("cps::", "")


def durations(db):
    c = sqlite3.connect(db)
    rows = c.execute("select name, duration, grid_x from kernels").fetchall()
    agg = collections.defaultdict(list)
    for n, d, g in rows:
        agg[(short(n), g)].append(d)
    return agg


def counters(dbs):
    agg = collections.defaultdict(list)
    for db in dbs:
        c = sqlite3.connect(db)
        rows = c.execute("select kernel_name, grid_size, counter_name, value "
                         "from counters_collection").fetchall()
        for n, g, cn, v in rows:
            agg[(short(n), g, cn)].append(v)
    return agg


def mean(v):
    return sum(v) / len(v)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--kt", required=True)
    ap.add_argument("--fetch", required=True, nargs="+")
    ap.add_argument("--write", required=True, nargs="+")
    ap.add_argument("--cmd", required=True)
    ap.add_argument("--md", required=True)
    ap.add_argument("--traffic", required=True)
    ap.add_argument("--top", type=int, default=16)
    ap.add_argument("--plane-md")
    ap.add_argument("--plane-traffic")
    ap.add_argument("--step-md", help="projection step and ADI line-solve kernels")
    ap.add_argument("--vcycle-traffic", help="counter bytes of one FP64 V-cycle (JSON)")
    a = ap.parse_args()
    kh = hashlib.sha256(open(KERNEL_SRC, "rb").read()).hexdigest()[:16]
    dur = durations(a.kt)
    fe = counters(a.fetch)
    wr = counters(a.write)
    copy_f = mean([v for (n, g, cn), v in fe.items() if n.startswith("k_copy<double>")
                   and g == COPY_BYTES // 8][0])
    copy_w = mean([v for (n, g, cn), v in wr.items() if n.startswith("k_copy<double>")
                   and g == COPY_BYTES // 8][0])
    sf = COPY_BYTES / (copy_f * 1024.0)
    sw = COPY_BYTES / (copy_w * 1024.0)
    lines = [f"# rocprofv3 summary: bench.py (spherical shell 192x256x512, FP64 PCG-multigrid)",
             "", "Commands (run from the repository root on one MI355X):", "", "```",
             a.cmd, "```", "",
             f"kernel source sha256[:16] = `{kh}`", "",
             "## Kernel durations (--kernel-trace --stats)", "",
             "| kernel | grid (threads) | launches | avg us | total ms |", "|---|---|---|---|---|"]
    for (n, g), v in sorted(dur.items(), key=lambda kv: -sum(kv[1]))[:a.top]:
        lines.append(f"| `{n}` | {g} | {len(v)} | {mean(v) / 1e3:.1f} | {sum(v) / 1e6:.2f} |")
    lines += ["", "## HBM bytes per dispatch (FETCH_SIZE, WRITE_SIZE)", "",
              f"Scale: the copy kernel of {COPY_BYTES} bytes reads as {copy_f:.1f} KiB fetched "
              f"and {copy_w:.1f} KiB written, so fetch x{sf:.3f}, write x{sw:.3f}.", "",
              "| kernel | grid (threads) | fetch MB | write MB |", "|---|---|---|---|"]
    keys = sorted({(n, g) for (n, g, cn) in fe}, key=lambda k: -mean(fe[(k[0], k[1], 'FETCH_SIZE')]))
    gs = None
    for n, g in keys[:a.top]:
        f = mean(fe[(n, g, "FETCH_SIZE")]) * 1024 * sf
        w = mean(wr.get((n, g, "WRITE_SIZE"), [0.0])) * 1024 * sw
        lines.append(f"| `{n}` | {g} | {f / 1e6:.1f} | {w / 1e6:.1f} |")
        if n.startswith(GS_FINEST):
            gs = (f, w, g)
    if gs is None:
        for (n, g, cn), v in fe.items():
            if n.startswith(GS_FINEST):
                gs = (mean(v) * 1024 * sf, mean(wr[(n, g, "WRITE_SIZE")]) * 1024 * sw, g)
    gsd = [v for (n, g), v in dur.items() if n.startswith(GS_FINEST)]
    lines += ["", f"Finest-level Gauss-Seidel colour pass `{GS_FINEST}`: average "
              f"{mean(gsd[0]) / 1e3:.1f} us over {len(gsd[0])} launches; "
              f"{gs[0] / 1e6:.1f} MB fetched + {gs[1] / 1e6:.1f} MB written per launch.", ""]
    os.makedirs(os.path.dirname(os.path.abspath(a.md)), exist_ok=True)
    open(a.md, "w").write("\n".join(lines))
    json.dump({"kernel": GS_FINEST, "kernel_source_sha256_16": kh,
               "bytes_per_launch": gs[0] + gs[1], "fetch_bytes": gs[0], "write_bytes": gs[1],
               "fetch_scale": sf, "write_scale": sw, "avg_us_trace": mean(gsd[0]) / 1e3},
              open(a.traffic, "w"), indent=1)
    print("\n".join(lines))
    if a.plane_md:
        plane_summary(a, dur, fe, wr, sf, sw)
    if a.step_md:
        step_summary(a, dur, fe, wr, sf, sw)
    if a.vcycle_traffic:
        vcycle_traffic(a, fe, wr, sf, sw)


def vcycle_sources_hash() -> str:
    h = hashlib.sha256()
    for path in (KERNEL_SRC, TILE_SRC):
        h.update(open(path, "rb").read())
    return h.hexdigest()[:16]


def vcycle_traffic(a, fe, wr, sf, sw):
    """HBM bytes of one FP64 preconditioning V-cycle by the counters: the
    kernels of one cycle as the kernel trace shows it (from a zero-iterate
    finest-level pass to the next, with no outer-iteration kernel between:
    a cycle of the graph replays that time it), each at its mean FETCH_SIZE
    and WRITE_SIZE per dispatch."""
    c = sqlite3.connect(a.kt)
    rows = [(short(n), s, g) for n, s, g in
            c.execute("select name, start, grid_x from kernels order by start")]
    starts = [i for i, r in enumerate(rows) if r[0] == "k_gs_march2<double, 0, 1>"]
    outer = ("k_apply", "k_cg", "k_reduce", "k_cast", "k_dot", "k_copy")
    best = None
    for i0, i1 in zip(starts, starts[1:]):
        cyc = rows[i0:i1]
        if any(n.startswith(outer) for n, _, _ in cyc):
            continue
        span = (rows[i1][1] - rows[i0][1]) / 1e3
        if best is None or span < best[0]:
            best = (span, cyc)
    if best is None:
        raise SystemExit("no bare V-cycle in the kernel trace")
    span, cyc = best
    total = 0.0
    for n, _, g in cyc:
        f = fe.get((n, g, "FETCH_SIZE"))
        w = wr.get((n, g, "WRITE_SIZE"))
        if not f or not w:
            raise SystemExit(f"no counters for {n} grid {g}")
        total += mean(f) * 1024 * sf + mean(w) * 1024 * sw
    out = {"what": "HBM bytes of one FP64 V-cycle of the paper-scale shell by FETCH_SIZE "
                   "and WRITE_SIZE (scaled by the copy kernel), over the kernels of one "
                   "graph-replayed cycle",
           "bytes_per_cycle": total, "kernels_per_cycle": len(cyc),
           "trace_span_us": span, "fetch_scale": sf, "write_scale": sw,
           "source_sha256_16": vcycle_sources_hash()}
    json.dump(out, open(a.vcycle_traffic, "w"), indent=1)
    print(json.dumps(out, indent=1))


STEP_KERNELS = ("k_divergence", "k_divergence2", "k_correct", "k_line_factor", "k_line_open",
                "k_line_fft", "k_line_periodic")


def step_summary(a, dur, fe, wr, sf, sw):
    lines = ["# rocprofv3 summary: projection step and ADI line solves, spherical shell "
             "192x256x512", "", "Same runs as the Gauss-Seidel summary (bench.py's `project` and "
             "`lines` forms); commands:", "", "```", a.cmd, "```", "",
             "Largest grid of each kernel, per launch:", "",
             "| kernel | grid (threads) | launches | avg us | fetch MB | write MB |",
             "|---|---|---|---|---|---|"]
    for k in STEP_KERNELS:
        names = sorted({n for (n, g) in dur if n.startswith(k + "<") or n == k})
        for name in names:
            g = max(gg for (n, gg) in dur if n == name)
            d = dur[(name, g)]
            f = mean(fe.get((name, g, "FETCH_SIZE"), [0.0])) * 1024 * sf
            w = mean(wr.get((name, g, "WRITE_SIZE"), [0.0])) * 1024 * sw
            lines.append(f"| `{name}` | {g} | {len(d)} | {mean(d) / 1e3:.1f} | "
                         f"{f / 1e6:.1f} | {w / 1e6:.1f} |")
    lines.append("")
    open(a.step_md, "w").write("\n".join(lines))
    print("\n".join(lines))


def plane_summary(a, dur, fe, wr, sf, sw):
    ph = hashlib.sha256(open(PLANE_SRC, "rb").read()).hexdigest()[:16]
    lines = ["# rocprofv3 summary: plane-smoother half-sweep, spherical shell 192x256x512",
             "", "Same runs as the Gauss-Seidel summary (bench.py's `plane` form, FP64 and "
             "FP32 cycles); commands:", "", "```", a.cmd, "```", "",
             f"plane kernel source sha256[:16] = `{ph}`", "",
             "Finest level (largest grid of each kernel), per launch:", "",
             "| kernel | grid (threads) | launches | avg us | fetch MB | write MB |",
             "|---|---|---|---|---|---|"]
    out = {"kernel_source_sha256_16": ph, "fetch_scale": sf, "write_scale": sw}
    for prec in ("double", "float"):
        tot_us = tot_b = 0.0
        for k in PLANE_KERNELS:
            # k<prec> or k<prec, ring-size class>: the finest level's launch
            cands = [(g, n) for (n, g) in dur if n == f"{k}<{prec}>" or n.startswith(f"{k}<{prec},")]
            if not cands:
                continue
            g, name = max(cands)
            d = dur[(name, g)]
            f = mean(fe.get((name, g, "FETCH_SIZE"), [0.0])) * 1024 * sf
            w = mean(wr.get((name, g, "WRITE_SIZE"), [0.0])) * 1024 * sw
            lines.append(f"| `{name}` | {g} | {len(d)} | {mean(d) / 1e3:.1f} | "
                         f"{f / 1e6:.1f} | {w / 1e6:.1f} |")
            tot_us += mean(d) / 1e3
            tot_b += f + w
        if tot_us:
            lines.append(f"| **half-sweep {prec}** | | | **{tot_us:.1f}** | "
                         f"{tot_b / 1e6:.1f} (fetch + write) | |")
            out["fp64" if prec == "double" else "fp32"] = {"avg_us_trace": tot_us,
                                                            "bytes_per_half_sweep": tot_b}
    lines.append("")
    open(a.plane_md, "w").write("\n".join(lines))
    json.dump(out, open(a.plane_traffic, "w"), indent=1)
    print("\n".join(lines))


if __name__ == "__main__":
    main()
