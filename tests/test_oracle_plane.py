"""Pins of the oracle's zebra (r, phi)-plane smoother: block Gauss-Seidel
over theta rows with exact (r, phi)-plane solves."""
import numpy as np
import pytest

import oracle as O
from oracle import plane


def _grid(nr, nt, np_, **kw):
    return O.Grid(nr, nt, np_, **kw)


# the 7-point operator, and the oblate shell's 11-point one (r-theta cross
# terms), whose plane blocks are not symmetric
KINDS = {"sphere": dict(radial_stretch=2.0),
         "oblate": dict(map=O.MAP_OBLATE, flattening=0.15, radial_stretch=1.5)}


@pytest.mark.parametrize("kind", sorted(KINDS))
def test_half_sweep_solves_its_rows_exactly(kind):
    """After relaxing parity k, the rows of parity k satisfy their equations
    (residual 0 there, with the other parity as it was), and the other
    parity is untouched."""
    g = _grid(8, 8, 16, **KINDS[kind])
    G = O.face_metrics(g)
    rng = np.random.default_rng(3)
    b = rng.standard_normal(g.shape)
    x = rng.standard_normal(g.shape)
    sm = plane.PlaneSmoother(G)
    for k in (0, 1):
        y = sm.half_sweep(b, x, k)
        r = O.residual(G, b, y)
        assert np.abs(r[:, k::2, :]).max() < 1e-11 * np.abs(b).max()
        assert np.array_equal(y[:, 1 - k::2, :], x[:, 1 - k::2, :])


@pytest.mark.parametrize("kind", sorted(KINDS))
def test_half_sweep_matches_dense_block_gauss_seidel(kind):
    """The same block solves from the oracle's dense matrix (assembled by
    the C oracle, not by probing) and numpy's dense solver."""
    g = _grid(6, 6, 8, **KINDS[kind])
    G = O.face_metrics(g)
    A = O.dense_matrix(G)
    nr, nt, np_ = g.shape
    idx = np.arange(nr * nt * np_).reshape(g.shape)
    rng = np.random.default_rng(4)
    b = rng.standard_normal(g.shape)
    x = rng.standard_normal(g.shape)
    want = x.ravel().copy()
    for k in (0, 1):
        y = plane.PlaneSmoother(G).half_sweep(b, x if k == 0 else want.reshape(g.shape), k)
        old = want.copy()
        for row in range(k, nt, 2):
            rr = idx[:, row, :].ravel()
            rest = np.setdiff1d(np.arange(A.shape[0]), rr)
            rhs = b.ravel()[rr] - A[np.ix_(rr, rest)] @ old[rest]
            want[rr] = np.linalg.solve(A[np.ix_(rr, rr)], rhs)
        assert np.abs(y.ravel() - want).max() < 1e-12 * np.abs(want).max()


def test_plane_vcycle_is_a_symmetric_preconditioner():
    """Zebra forward before, backward after the coarse correction: on a
    symmetric operator the V-cycle from zero is a symmetric linear map."""
    g = _grid(8, 8, 16, radial_stretch=2.0)
    mg = O.Multigrid(g)
    pm = plane.PlaneMultigrid(mg, nu=1)
    rng = np.random.default_rng(5)
    u = rng.standard_normal(g.shape); u -= u.mean()
    v = rng.standard_normal(g.shape); v -= v.mean()
    mu = pm.vcycle(u, np.zeros_like(u))
    mv = pm.vcycle(v, np.zeros_like(v))
    a, c = float((v * mu).sum()), float((u * mv).sum())
    assert abs(a - c) <= 1e-11 * max(abs(a), abs(c))


def _rate(cycle, G, b, n=8):
    x = np.zeros_like(b)
    hist = []
    for _ in range(n):
        x = cycle(b, x)
        x -= x.mean()
        hist.append(np.linalg.norm(O.residual(G, b, x)))
    return hist[-1] / hist[-2]


def test_plane_smoothing_removes_the_shell_anisotropy():
    """On the stretched shell with cone walls at 0.05 (radial coupling up to
    ~40x the theta coupling, phi coupling at the cone tips ~15x the radial
    one) point red-black V(2,2) contracts by > 0.7 per cycle, the plane
    smoother's V(2,2) by < 0.2."""
    g = _grid(16, 16, 64, radial_stretch=2.0)
    mg = O.Multigrid(g)
    G = mg.metrics(0)
    b = np.random.default_rng(6).standard_normal(g.shape)
    b -= b.mean()
    point = _rate(lambda bb, xx: mg.vcycle(bb, xx), G, b)
    pm = plane.PlaneMultigrid(mg, nu=2)
    plane_rate = _rate(lambda bb, xx: pm.vcycle(bb, xx), G, b)
    assert point > 0.7, point
    assert plane_rate < 0.2, plane_rate
