"""Pins of the full sphere (theta0 = 0, theta1 = pi) in the flux form: the
faces on the polar axis have zero area, so they carry no flux and no
coupling across the pole is needed (the paper's shell cut connects lines
through the pole for its finite differences; here the zero-area face is the
whole story).  Checked: the pole faces' rows and determinants vanish, the
operator keeps its null space and symmetry, and (A p) / |J^-1| converges
to the Cartesian Laplacian at second order, in the polar rows too."""
import numpy as np
import pytest

import oracle as O
from oracle import direct

PI = np.pi


def _sphere(n, **kw):
    return O.Grid(n, n, 2 * n, theta0=0.0, theta1=PI, **kw)


def test_pole_faces_have_zero_area():
    g = _sphere(8, radial_stretch=2.0)
    for a, c in [(0, 0), (3, 5), (7, 15)]:
        for b in (0, g.n_theta):
            C, det = O.face_crow(g, 1, a, b, c)
            assert np.abs(C).max() <= 1e-16 and abs(det) <= 1e-16
    G = O.face_metrics(g)
    assert np.isfinite(G).all() and not G[3:6, :, 0, :].any()
    assert np.all(G[4, :, 1:, :] > 0)
    # the line operator's G_dd at a pole face is 0, not 0/0
    psi = np.random.default_rng(2).standard_normal(g.shape)
    assert np.isfinite(O.line_apply(g, 1, 1.0, psi, (1, 0.5, 1, 0.5))).all()


def test_operator_null_space_and_symmetry():
    g = _sphere(6)
    A = O.dense_matrix(O.face_metrics(g))
    one = np.ones(A.shape[0])
    assert np.abs(A @ one).max() <= 1e-13 * np.abs(A).max()
    assert np.abs(one @ A).max() <= 1e-13 * np.abs(A).max()
    assert np.abs(A - A.T).max() <= 1e-13 * np.abs(A).max()


@pytest.mark.parametrize("map_,method", [(O.MAP_SPHERE, O.METRICS_CENTRAL),
                                         (O.MAP_OBLATE, O.METRICS_CENTRAL),
                                         (O.MAP_SPHERE, O.METRICS_VERTEX),
                                         (O.MAP_OBLATE, O.METRICS_VERTEX)],
                         ids=["sphere", "oblate", "sphere-vertex", "oblate-vertex"])
def test_second_order_including_the_poles(map_, method):
    """p = sin x1 cos 0.7 x2 + 0.3 x3^2 (smooth through the poles): the RMS of
    (A p)/|J^-1| - lap p over the cells off the r-walls, and its maximum over
    the two polar rows, both drop ~4x per refinement.  On the oblate shell
    (flattening 0.1) and with the paper's vertex-averaged metrics the r-faces
    next to the axis carry an r-theta cross metric, whose reads across the
    pole are mirrored onto the polar row itself (the cell across the axis is
    not read): that cross metric vanishes as the face approaches the axis,
    so the polar rows still converge at second order."""
    rms, pole = [], []
    f = 0.1 if map_ == O.MAP_OBLATE else 0.0
    for n in (8, 16, 32):
        g = _sphere(n, map=map_, flattening=f)
        G = O.face_metrics(g, method=method)
        if method == O.METRICS_VERTEX or map_ == O.MAP_OBLATE:
            assert np.abs(G[1, 1:, 0, :]).max() > 0  # r-theta cross metric in the polar row
        X = np.zeros((3,) + g.shape)
        for a in range(n):
            for b in range(n):
                for c in range(2 * n):
                    X[:, a, b, c] = O.map_point(g, (a + .5) / n, (b + .5) / n, (c + .5) / (2 * n))
        p = np.sin(X[0]) * np.cos(0.7 * X[1]) + 0.3 * X[2] ** 2
        lap = -1.49 * np.sin(X[0]) * np.cos(0.7 * X[1]) + 0.6
        J = np.array([[O.cell_jdet(g, a, b, 0, method=method) for b in range(n)]
                      for a in range(n)])[:, :, None]
        e = (O.apply(G, p) / J - lap)[1:-1]
        rms.append(np.sqrt((e ** 2).mean()))
        pole.append(np.abs(e[:, [0, -1], :]).max())
    q_rms = [rms[i] / rms[i + 1] for i in range(2)]
    q_pole = [pole[i] / pole[i + 1] for i in range(2)]
    assert all(3.5 < q < 4.5 for q in q_rms), (rms, q_rms)
    assert q_pole[0] > 2.5 and q_pole[1] > 3.2, (pole, q_pole)


def test_multigrid_reaches_the_exact_solution():
    g = _sphere(16, radial_stretch=2.0)
    G = O.face_metrics(g)
    b = np.random.default_rng(3).standard_normal(g.shape)
    want = direct.solve_axisym(G, b)
    x, st, it, rel, hist, mean = O.Multigrid(g).solve(b, tol=1e-10, max_iters=400, accel=1)
    assert st == 0 and rel <= 1e-10
    assert np.linalg.norm(x - want) <= 1e-9 * np.linalg.norm(want)
