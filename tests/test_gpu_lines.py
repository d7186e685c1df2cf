"""Implicit line solves of the ADI steps on the GPU (cps_line_solve) against
the oracle's Thomas and periodic solves, entry by entry, for every
direction, both wall conditions and the phi-invariant maps; in place; the
paper-scale shell at sampled lines; and the rejections."""
import numpy as np
import pytest

import oracle as O
from paper_2305_17875_amd import cps, inputs
from paper_2305_17875_amd.inputs import Shell, MAP_OBLATE, MAP_TRIAXIAL, MAP_IDENTITY
from gpu_util import needs_gpu, log, dev, host, torch

pytestmark = [pytest.mark.gpu, needs_gpu]

GRIDS = [
    ("sphere-stretch-8x8x16", Shell(8, 8, 16, radial_stretch=2.0)),
    ("oblate-6x10x36", Shell(6, 10, 36, map=MAP_OBLATE, flattening=0.1)),  # ragged
    ("identity-8x6x12", Shell(8, 6, 12, map=MAP_IDENTITY)),
]
BCS = [(0, 0.0, 0, 0.0), (1, 0.4, 1, -1.1), (1, 0.0, 0, 0.0)]


@pytest.fixture(scope="module", params=GRIDS, ids=[c[0] for c in GRIDS])
def grid(request):
    name, g = request.param
    log("lines", name)
    s = cps.Solver(g, precision=0)
    yield name, g, s
    s.close()


@pytest.mark.parametrize("d", [0, 1, 2])
@pytest.mark.parametrize("bc", BCS, ids=["noflux", "values", "mixed"])
def test_line_solve_matches_oracle(grid, d, bc):
    """Per entry to 1e-12 of the largest (both sides eliminate in the same
    order; the GPU multiplies by stored inverse pivots)."""
    name, g, s = grid
    rhs = np.random.default_rng(30 + d).standard_normal(g.shape)
    coef = 1.7
    want = O.line_solve(g, d, coef, rhs, bc)
    got = host(s.line_solve(d, coef, dev(rhs).flatten(), bc)).reshape(g.shape)
    assert np.abs(got - want).max() <= 1e-12 * np.abs(want).max(), np.abs(got - want).max()


@pytest.mark.parametrize("np_", [512, 1024, 2048])
def test_long_phi_rings_match_oracle(np_):
    """Periodic phi-lines on rings of 512 to 2048 cells (the ring transform
    takes 4, 2 and 1 rings per block).  At coef 1e-3 the circulant systems
    are well conditioned, and the GPU matches the oracle per entry to 1e-11
    of the largest.  At coef 1.7 the symbols of modes n/2 and 0 differ by up
    to ~1e7 near the cone tips, so the forward error of either side is that
    large a multiple of rounding; there the check is the backward error: the
    GPU solution's residual in the oracle's operator stays within 10x the
    oracle's own."""
    g = Shell(8, 8, np_, radial_stretch=1.5)
    log("long phi rings", np_)
    rhs = np.random.default_rng(np_).standard_normal(g.shape)
    bc = (0, 0.0, 0, 0.0)
    s = cps.Solver(g, precision=0)
    try:
        got = {c: host(s.line_solve(2, c, dev(rhs).flatten(), bc)).reshape(g.shape)
               for c in (1e-3, 1.7)}
    finally:
        s.close()
    want = O.line_solve(g, 2, 1e-3, rhs, bc)
    assert np.abs(got[1e-3] - want).max() <= 1e-11 * np.abs(want).max()
    ref = O.line_solve(g, 2, 1.7, rhs, bc)
    r_gpu = np.abs(O.line_apply(g, 2, 1.7, got[1.7], bc) - rhs).max()
    r_orc = np.abs(O.line_apply(g, 2, 1.7, ref, bc) - rhs).max()
    log("backward error", np_, r_gpu, r_orc, np.abs(got[1.7] - ref).max() / np.abs(ref).max())
    assert r_gpu <= 10.0 * r_orc + 1e-14 * np.abs(rhs).max(), (r_gpu, r_orc)


@pytest.mark.parametrize("d", [0, 1, 2])
def test_in_place_equals_out_of_place(d):
    g = Shell(8, 8, 16, radial_stretch=2.0)
    s = cps.Solver(g, precision=0)
    try:
        r = dev(np.random.default_rng(40 + d).standard_normal(g.shape)).flatten()
        out = s.line_solve(d, 0.9, r, (1, 0.3, 1, 0.3))
        x = r.clone()
        s.line_solve(d, 0.9, x, (1, 0.3, 1, 0.3), out=x)
        assert np.array_equal(host(out), host(x))
    finally:
        s.close()


def test_rejections():
    s = cps.Solver(Shell(6, 8, 16, map=MAP_TRIAXIAL, flattening=0.1, skew=0.1), precision=0)
    try:
        r = torch.zeros(6 * 8 * 16, dtype=torch.float64, device="cuda")
        with pytest.raises(cps.CpsError, match="phi-invariant"):
            s.line_solve(0, 1.0, r)
    finally:
        s.close()
    s = cps.Solver(Shell(8, 8, 16), precision=0)
    try:
        r = torch.zeros(8 * 8 * 16, dtype=torch.float64, device="cuda")
        with pytest.raises(cps.CpsError, match="coef"):
            s.line_solve(0, -1.0, r)
        with pytest.raises(cps.CpsError, match="dir"):
            s.line_solve(3, 1.0, r)
        with pytest.raises(cps.CpsError, match="bc"):
            s.line_solve(0, 1.0, r, (2, 0.0, 0, 0.0))
    finally:
        s.close()


def test_paper_scale_sampled_lines():
    """192 x 256 x 512, stretching 2.0: each direction's solve on the whole
    field, checked at sampled lines (walls, cone tips, interior) that the
    oracle solves one by one.  coef = 1e-4 puts coef G_dd / |J^-1| at O(1-10)
    on these cells (|J^-1| ~ 3e-6); a much stiffer line with a no-flux end is
    nearly singular and both solvers' rounding is then amplified by its
    condition number."""
    g = inputs.config2()
    nr, nt, np_ = g.shape
    log("lines fullsize", g.shape)
    rhs = inputs.smoothed_noise(g.shape, 50)
    bc = (1, 0.5, 0, 0.0)
    s = cps.Solver(g, precision=0)
    try:
        rd = dev(rhs).flatten()
        outs = [host(s.line_solve(d, 1e-4, rd, bc)).reshape(g.shape) for d in range(3)]
    finally:
        s.close()
        torch.cuda.empty_cache()
    rng = np.random.default_rng(9)
    for d, got in enumerate(outs):
        span = (nt * np_, nr * np_, nr * nt)[d]
        lines = np.concatenate([[0, 1, span - 1], rng.integers(0, span, 24)])
        want = O.line_solve(g, d, 1e-4, rhs, bc, lines=lines)
        for line in lines:
            sl = {0: (slice(None), line // np_, line % np_), 1: (line // np_, slice(None), line % np_),
                  2: (line // nt, line % nt, slice(None))}[d]
            assert np.abs(got[sl] - want[sl]).max() <= 1e-12 * np.abs(want[sl]).max(), (d, line)


def test_degenerate_cases():
    """coef = 0: psi = g / |J^-1| exactly along every direction; a ring of 2
    phi cells (both neighbours are the same cell) and a zero field in the
    projection step."""
    g = Shell(8, 8, 16, radial_stretch=2.0)
    b = np.random.default_rng(60).standard_normal(g.shape)
    Jc = np.array([[O.cell_jdet(g, a, bb, 0) for bb in range(g.n_theta)] for a in range(g.n_r)])
    s = cps.Solver(g, precision=0)
    try:
        for d in range(3):
            got = host(s.line_solve(d, 0.0, dev(b).flatten())).reshape(g.shape)
            assert np.abs(got - b / Jc[:, :, None]).max() <= 1e-14 * np.abs(got).max(), d
        z = torch.zeros(3 * g.cells, dtype=torch.float64, device="cuda")
        assert not host(s.divergence(z)).any()
    finally:
        s.close()
    g2 = Shell(4, 4, 2)  # one level: phi ring of 2
    u = np.random.default_rng(61).standard_normal((3,) + g2.shape)
    s = cps.Solver(g2, precision=0)
    try:
        got = host(s.divergence(dev(u).flatten())).reshape(g2.shape)
        with pytest.raises(cps.CpsError, match="n_phi"):
            s.line_solve(2, 1.0, dev(u[0]).flatten())
    finally:
        s.close()
    want = O.divergence(g2, u)
    assert np.abs(got - want).max() <= 1e-13 * np.abs(want).max()
