"""Pins of caller-supplied face metrics in the oracle (the boundary's
CPS_METRICS_USER_FACE): level 0 is the caller's array with the low-wall
faces taken as zero, and each coarser level's face is half the sum of its
four child faces (coarsen_metrics).

Checked against what the geometry fixes, not against the rule retyped:
  * on a uniform box the face metric is h_u h_v / h_d, and the coarsened
    metrics equal those of the box with twice the spacings exactly;
  * on the sphere the coarsened metrics approach the ones formed from the
    map at the coarse spacing at second order (the error drops ~4x per
    refinement), for the diagonal and, on the oblate shell, the r-theta
    cross entries;
  * the coarse operator keeps the constants as its null space on both
    sides, and stays symmetric when the fine one is;
  * a multigrid built from the paper's vertex-averaged metrics handed in as
    caller metrics reaches the exact solution of that operator;
  * entries on the low-wall faces are ignored, and non-finite entries or a
    negative diagonal are rejected.
"""
import numpy as np
import pytest

import oracle as O
from oracle import direct


def test_box_coarsening_is_exact():
    kw = dict(map=O.MAP_IDENTITY, r_inner=0.0, r_outer=1.3, theta0=0.2, theta1=2.0)
    Gf = O.face_metrics(O.Grid(12, 8, 16, **kw))
    Gc = O.face_metrics(O.Grid(6, 4, 8, **kw))
    np.testing.assert_allclose(O.coarsen_metrics(Gf), Gc, rtol=1e-14, atol=1e-15)


@pytest.mark.parametrize("map_,f", [(O.MAP_SPHERE, 0.0), (O.MAP_OBLATE, 0.1)])
def test_shell_coarsening_is_second_order(map_, f):
    errs = {0: [], 1: []}
    for n in (8, 16, 32):
        kw = dict(map=map_, flattening=f, radial_stretch=1.5)
        Gf = O.face_metrics(O.Grid(2 * n, 2 * n, 4 * n, **kw))
        Gc = O.face_metrics(O.Grid(n, n, 2 * n, **kw))
        Gh = O.coarsen_metrics(Gf)
        for k in (0, 1):  # G_rr, and the r-theta cross entry on the r-faces
            scale = np.abs(Gc[0]).max()
            errs[k].append(np.abs(Gh[k] - Gc[k])[1:].max() / scale)
    q = [errs[0][i] / errs[0][i + 1] for i in range(2)]
    assert all(3.5 < v < 4.5 for v in q), (errs[0], q)
    if map_ == O.MAP_OBLATE:
        q = [errs[1][i] / errs[1][i + 1] for i in range(2)]
        assert all(3.0 < v < 5.0 for v in q), (errs[1], q)
    else:
        assert max(errs[1]) == 0.0


def test_coarse_operator_keeps_null_space_and_symmetry():
    g = O.Grid(8, 8, 16, radial_stretch=2.0)
    Gh = O.coarsen_metrics(O.face_metrics(g))
    A = O.dense_matrix(Gh)
    one = np.ones(A.shape[0])
    s = np.abs(A).max()
    assert np.abs(A @ one).max() <= 1e-13 * s and np.abs(one @ A).max() <= 1e-13 * s
    assert np.abs(A - A.T).max() <= 1e-13 * s


def test_vertex_metrics_as_caller_metrics_reach_the_exact_solution():
    g = O.Grid(16, 16, 64, radial_stretch=2.0)
    G0 = O.face_metrics(g, method=O.METRICS_VERTEX)
    assert np.abs(G0[1]).max() > 0  # the vertex metrics' r-theta cross entries
    mg = O.Multigrid(g, face_G=G0)
    assert len(mg.levels) == 3 and mg.ncol == 4
    np.testing.assert_array_equal(mg.metrics(0), G0)
    np.testing.assert_allclose(mg.metrics(1), O.coarsen_metrics(G0), rtol=0, atol=0)
    np.testing.assert_allclose(mg.metrics(2), O.coarsen_metrics(mg.metrics(1)), rtol=0, atol=0)
    b = np.random.default_rng(5).standard_normal(g.shape)
    want = direct.solve_axisym(G0, b)
    x, st, it, rel, _, _ = mg.solve(b, tol=1e-11, max_iters=300, accel=1)
    assert st == 0
    assert np.linalg.norm(x - want) <= 1e-9 * np.linalg.norm(want)


def test_wall_entries_ignored_and_bad_entries_rejected():
    g = O.Grid(8, 8, 32)
    G0 = O.face_metrics(g)
    noisy = G0.copy()
    noisy[0:3, 0] = 7.0   # low r-wall faces
    noisy[3:6, :, 0] = -3.0  # low theta-wall faces
    np.testing.assert_array_equal(O.Multigrid(g, face_G=noisy).metrics(0), G0)
    for bad in (np.nan, np.inf):
        B = G0.copy()
        B[2, 3, 4, 5] = bad
        with pytest.raises(ValueError):
            O.Multigrid(g, face_G=B)
    B = G0.copy()
    B[4, 3, 4, 5] = -1e-3
    with pytest.raises(ValueError):
        O.Multigrid(g, face_G=B)
