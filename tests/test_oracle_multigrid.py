"""Pins of the oracle's multigrid pieces: level plan, colourings, grid
transfers and Gauss-Seidel colour passes.

Checked against: the transpose relation R = P^T (two independent loops),
exact reproduction of constants and of linear fields by cell-centred
trilinear interpolation, conservation of the sum by restriction, brute-force
colouring validity over every stencil offset, and textbook sequential
Gauss-Seidel written with a dense matrix.
"""
import itertools

import numpy as np
import pytest

import oracle as O


def test_level_plans():
    assert O.level_plan(32, 32, 32) == [(32, 32, 32), (16, 16, 16), (8, 8, 8)]
    assert O.level_plan(192, 256, 512) == [(192, 256, 512), (96, 128, 256), (48, 64, 128),
                                           (24, 32, 64), (12, 16, 32), (6, 8, 16)]
    assert len(O.level_plan(16, 16, 16)) == 2
    assert O.level_plan(64, 64, 128)[-1] == (8, 8, 16)
    assert O.level_plan(96, 128, 256)[-1] == (6, 8, 16)
    assert O.level_plan(128, 128, 256)[-1] == (8, 8, 16)
    assert O.level_plan(6, 6, 6) == [(6, 6, 6)]          # too small to halve
    assert O.level_plan(40, 40, 40)[-1] == (10, 10, 10)  # stops at odd dims
    assert len(O.level_plan(32, 32, 32, n_levels=2)) == 2
    with pytest.raises(ValueError):
        O.level_plan(12, 12, 12, n_levels=4)


FACE = [o for o in itertools.product((-1, 0, 1), repeat=3) if sum(map(abs, o)) == 1]
FACE_EDGE = [o for o in itertools.product((-1, 0, 1), repeat=3) if 1 <= sum(map(abs, o)) <= 2]


@pytest.mark.parametrize("ncol,offs", [(2, FACE), (4, FACE_EDGE)])
def test_colourings_separate_stencil_neighbours(ncol, offs):
    n = (6, 4, 8)
    for a, b, c in itertools.product(*map(range, n)):
        k = O.colour(ncol, a, b, c)
        assert 0 <= k < ncol
        for da, db, dc in offs:
            a2, b2, c2 = a + da, b + db, (c + dc) % n[2]
            if 0 <= a2 < n[0] and 0 <= b2 < n[1]:
                assert O.colour(ncol, a2, b2, c2) != k


def _matrices(nf):
    nc = tuple(v // 2 for v in nf)
    P = np.zeros((np.prod(nf), np.prod(nc)))
    for j in range(P.shape[1]):
        e = np.zeros(np.prod(nc)); e[j] = 1
        P[:, j] = O.prolong_add(e.reshape(nc), np.zeros(nf)).ravel()
    R = np.zeros((np.prod(nc), np.prod(nf)))
    for j in range(R.shape[1]):
        e = np.zeros(np.prod(nf)); e[j] = 1
        R[:, j] = O.restrict(e.reshape(nf)).ravel()
    return P, R


def test_restriction_is_transpose_of_prolongation():
    P, R = _matrices((4, 6, 8))
    np.testing.assert_allclose(R, P.T, rtol=0, atol=1e-15)
    np.testing.assert_allclose(P.sum(axis=1), 1.0, atol=1e-15)   # P 1 = 1


def test_restriction_conserves_sum_and_weights_interior_rows_by_eight():
    nf = (8, 8, 16)
    r = np.random.default_rng(2).standard_normal(nf)
    assert abs(O.restrict(r).sum() - r.sum()) <= 1e-12 * np.abs(r).sum()
    R1 = O.restrict(np.ones(nf))
    np.testing.assert_allclose(R1, 8.0, atol=1e-14)


def test_prolongation_reproduces_linear_fields():
    """Cell-centred linear interpolation: fine cell i sits at coarse index
    position i/2 - 1/4, so a coarse field linear in the index is reproduced
    exactly away from the walls (and the periodic seam)."""
    nf = (8, 8, 16)
    nc = (4, 4, 8)
    I, J, K = np.meshgrid(*[np.arange(n, dtype=float) for n in nc], indexing="ij")
    e = 1.0 + 2.0 * I - 0.5 * J + 0.25 * K
    x = O.prolong_add(e, np.zeros(nf))
    i, j, k = np.meshgrid(*[np.arange(n) / 2.0 - 0.25 for n in nf], indexing="ij")
    want = 1.0 + 2.0 * i - 0.5 * j + 0.25 * k
    np.testing.assert_allclose(x[1:-1, 1:-1, 1:-1], want[1:-1, 1:-1, 1:-1], atol=1e-13)


def _diag_sum(G):
    """-(sum of the six G_dd around each cell); high faces come from the
    neighbour's low face (zero past the walls, wrapped in phi)."""
    d = G[0] + G[4] + G[8] + np.roll(G[8], -1, axis=2)
    d[:-1] += G[0][1:]
    d[:, :-1] += G[4][:, 1:]
    return -d


@pytest.mark.parametrize("kw,ncol", [(dict(map=O.MAP_SPHERE), 2),
                                     (dict(map=O.MAP_TRIAXIAL, flattening=0.1, skew=0.2), 4)])
def test_colour_pass_is_sequential_gauss_seidel(kw, ncol):
    """Cells of the colour visited one at a time in index order, each
    updated with the current values of all others (dense matrix row)."""
    g = O.Grid(4, 4, 6, **kw)
    G = O.face_metrics(g)
    A = O.dense_matrix(G)
    D = _diag_sum(G).ravel()
    if ncol == 2:
        np.testing.assert_allclose(D, np.diag(A), rtol=1e-14)  # textbook diagonal
    rng = np.random.default_rng(5)
    b = rng.standard_normal(g.shape)
    x0 = rng.standard_normal(g.shape)
    for col in range(ncol):
        want = x0.ravel().copy()
        for i, (a, bb, c) in enumerate(itertools.product(*map(range, g.shape))):
            if O.colour(ncol, a, bb, c) == col:
                want[i] += (b.ravel()[i] - A[i] @ want) / D[i]
        got = O.gs_pass(G, b, x0, ncol, col)
        np.testing.assert_allclose(got.ravel(), want, rtol=1e-12, atol=1e-12)


def test_black_residual_vanishes_after_a_black_pass():
    """After a red-black sweep that ends on the black pass (colour 1), every
    black cell's own equation holds with its red neighbours as they stand:
    its residual is zero up to rounding, the red residual is not.  So the
    restriction of the red residual alone (black entries zeroed) equals the
    restriction of the whole residual up to rounding -- the fact that lets
    the V-cycle form and restrict only the red residual after
    pre-smoothing."""
    g = O.Grid(6, 8, 16, radial_stretch=2.0)
    G = O.face_metrics(g)
    rng = np.random.default_rng(11)
    b = rng.standard_normal(g.shape)
    x = rng.standard_normal(g.shape)
    for _ in range(2):
        for col in (0, 1):
            x = O.gs_pass(G, b, x, 2, col)
    r = O.residual(G, b, x)
    scale = np.abs(b).max() + np.abs(O.apply(G, x)).max()
    black = np.zeros(g.shape, dtype=bool)
    for a, bb, c in itertools.product(*map(range, g.shape)):
        black[a, bb, c] = O.colour(2, a, bb, c) == 1
    assert np.abs(r[black]).max() <= 1e-14 * scale
    assert np.abs(r[~black]).max() >= 1e-3 * scale
    red_only = np.where(black, 0.0, r)
    full, red = O.restrict(r), O.restrict(red_only)
    assert np.abs(full - red).max() <= 1e-13 * np.abs(full).max()


def test_coarse_solve_is_exact_on_zero_mean_data():
    g = O.Grid(8, 8, 16)
    mg = O.Multigrid(g)
    Gc = mg.metrics(len(mg.levels) - 1)
    Ac = O.dense_matrix(Gc)
    bc = np.random.default_rng(7).standard_normal(mg.levels[-1])
    e = mg.coarse_solve(bc)
    assert abs(e.sum()) < 1e-10
    np.testing.assert_allclose(Ac @ e.ravel(), (bc - bc.mean()).ravel(), atol=1e-10)
