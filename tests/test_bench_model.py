"""The byte models behind bench.py's roofline figures, pinned to brute-force
counts on small grids and to the paper-scale values the measurement quotes;
and the one-GPU contract of bench.py's command line.  CPU only."""
import importlib.util
import os
import subprocess
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PAPER_SCALE = (192, 256, 512)


@pytest.fixture(scope="module")
def bench():
    spec = importlib.util.spec_from_file_location("bench_model", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def colour_of(shape, ncol):
    """Red-black (a + b + c) mod 2, or the four colours ((a + c) mod 2,
    (b + c) mod 2) of the 19-point class."""
    a, b, c = np.meshgrid(*[np.arange(k) for k in shape], indexing="ij")
    if ncol == 2:
        return (a + b + c) % 2
    return ((a + c) % 2) * 2 + (b + c) % 2


@pytest.mark.parametrize("shape", [(4, 6, 8), (6, 4, 10)])
@pytest.mark.parametrize("ncol,nterms", [(2, 3), (4, 5)])
def test_colour_pass_bytes_count_every_access_once(bench, shape, ncol, nterms):
    """One pass of colour k: every cell of colour k reads b and writes x,
    every other cell is read once as a neighbour, the metric arrays once
    (per (r, theta)); counted cell by cell."""
    col = colour_of(shape, ncol)
    w = 8
    for k in range(ncol):
        upd = int((col == k).sum())
        other = col.size - upd
        want = upd * 2 * w + other * w + nterms * shape[0] * shape[1] * w
        got = bench.gs_bytes_per_launch(shape, ncol, w, True, nterms)
        # the model takes n / ncol cells per colour; the colour classes of
        # these grids have exactly that size
        assert upd == col.size // ncol
        assert got == want, (k, got, want)


def test_paper_scale_figures(bench):
    """The algorithmic bytes the roofline and the half-sweep rate use on the
    paper-scale shell (FP64)."""
    assert bench.gs_bytes_per_launch(PAPER_SCALE, 2, 8, True, 3) == 303_169_536
    assert bench.plane_half_sweep_bytes(PAPER_SCALE, 8) == 1_009_385_472
    levels = [(192, 256, 512), (96, 128, 256), (48, 64, 128), (24, 32, 64), (12, 16, 32),
              (6, 8, 16)]
    assert bench.vcycle_bytes(levels, 8) == 3_758_344_704
    # the cycle's fused transfers on the two finest levels: one word a
    # cell less there (25,165,824 + 3,145,728 cells)
    assert bench.vcycle_bytes(levels, 8, fused=True) == 3_758_344_704 - 8 * 28_311_552
    # and the red-only prolongation: one word a cell less on every smoothed
    # level (28,760,064 cells)
    assert bench.vcycle_bytes(levels, 8, fused=True, red_prolong=True) == \
        3_758_344_704 - 8 * 28_311_552 - 8 * 28_760_064


def test_vcycle_bytes_red_residual_levels(bench):
    """Row-pair levels (n_phi / 2 a multiple of 64, n_theta even) form and
    restrict only the red residual: 16.25 n words a level against 17.75 n
    on the others; the coarsest level's dense inverse is the same."""
    coarse = (2, 2, 4)
    nc = 16
    tail = nc * nc * 8 + 2 * nc * 8
    for shape, words in (((4, 8, 128), 16.25), ((4, 8, 64), 17.75), ((4, 7, 128), 17.75)):
        nr, nt, np_ = shape
        n = nr * nt * np_
        want = int(round((words * n + 9 * 3 * nr * nt) * 8)) + tail
        assert bench.vcycle_bytes([shape, coarse], 8) == want, shape
    # the fused transfer: 15.25 n words where the coarse ring is one or
    # two 64-pair segments and its theta count splits into row groups
    for shape, c, words in (((8, 8, 256), (4, 4, 128), 15.25), ((8, 8, 512), (4, 4, 256), 15.25),
                            ((8, 4, 256), (4, 2, 128), 16.25), ((8, 8, 1024), (4, 4, 512), 16.25),
                            ((8, 8, 256), (4, 8, 128), 16.25)):
        nr, nt, np_ = shape
        n = nr * nt * np_
        ncc = c[0] * c[1] * c[2]
        want = int(round((words * n + 9 * 3 * nr * nt) * 8)) + ncc * ncc * 8 + 2 * ncc * 8
        assert bench.vcycle_bytes([shape, c], 8, fused=True) == want, shape


def test_plane_half_sweep_counts_its_terms(bench):
    """Half-sweep = b and x in (n/2 each), spectra out, the elimination's two
    passes over the spectra (4 x) and pivots (2 x half of them), spectra in,
    x out; spectra are n_phi/2 + 1 complex values per relaxed ring."""
    nr, nt, np_ = 4, 6, 16
    rings = nr * (nt // 2)
    spec = rings * (np_ // 2 + 1) * 2
    half = nr * nt * np_ // 2
    words = 2 * half + spec + 4 * spec + spec + spec + half
    assert bench.plane_half_sweep_bytes((nr, nt, np_), 4) == words * 4


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and "--gpus 1" in r.stderr


def test_vcycle_rate_reports_cycles_per_solve(bench):
    """The V-cycle figure divides the byte model by the mean event span of a
    cycle, and counts cycles per profiled solve, not in total."""
    levels = [PAPER_SCALE, (96, 128, 256), (48, 64, 128), (24, 32, 64), (12, 16, 32), (6, 8, 16)]
    vc = bench.KNAMES.index("vcycle")
    prof = {k: (0.0, 0) for k in range(len(bench.KNAMES))}
    prof[vc] = (150 * 0.93, 150)  # 150 cycles of 930 us in 2 solves
    out = bench.vcycle_rate(prof, levels, 8, 2)
    assert out["cycles_per_step"] == 75
    assert out["bytes_per_cycle"] == bench.vcycle_bytes(levels, 8, fused=True, red_prolong=True)
    assert bench.vcycle_rate(prof, levels, 4, 2)["bytes_per_cycle"] == \
        bench.vcycle_bytes(levels, 4, fused=True, red_prolong=True)
    assert out["avg_us"] == pytest.approx(930.0)
    assert out["frac_of_peak"] == pytest.approx(out["bytes_per_cycle"] / 930e-6 / 1e9 / 8000.0)
    # with the graph-replayed time: the rate is on it, the eager span beside it
    g = bench.vcycle_rate(prof, levels, 8, 2, graph_us=800.0)
    assert g["avg_us"] == pytest.approx(800.0)
    assert g["frac_of_peak"] == pytest.approx(g["bytes_per_cycle"] / 800e-6 / 1e9 / 8000.0)
    assert g["eager_avg_us"] == pytest.approx(930.0)
    assert g["eager_frac_of_peak"] == pytest.approx(out["frac_of_peak"])
    assert g["traffic"] is None
    # with the counters' bytes of one cycle: their rate over the same time
    t = bench.vcycle_rate(prof, levels, 8, 2, graph_us=800.0, traffic=3.9e9)
    assert t["traffic"]["achieved_GBs"] == pytest.approx(3.9e9 / 800e-6 / 1e9)
    assert t["traffic"]["frac_of_peak"] == pytest.approx(3.9e9 / 800e-6 / 1e9 / 8000.0)
    prof[vc] = (0.0, 0)
    assert bench.vcycle_rate(prof, levels, 8, 2) is None


def test_vcycle_traffic_follows_the_kernel_sources(bench, tmp_path, monkeypatch):
    """Counter bytes of a V-cycle are used only while the hash of the kernel
    sources they were taken on (kernels.hpp, then tile.hpp) matches."""
    import hashlib
    import json
    h = hashlib.sha256()
    for path in (bench.KERNEL_SRC, bench.TILE_SRC):
        h.update(open(path, "rb").read())
    f = tmp_path / "t.json"
    monkeypatch.setattr(bench, "VCYCLE_TRAFFIC_FILE", str(f))
    f.write_text(json.dumps({"bytes_per_cycle": 3.9e9, "source_sha256_16": h.hexdigest()[:16]}))
    assert bench.vcycle_traffic() == 3.9e9
    f.write_text(json.dumps({"bytes_per_cycle": 3.9e9, "source_sha256_16": "0" * 16}))
    assert bench.vcycle_traffic() is None
    f.unlink()
    assert bench.vcycle_traffic() is None
