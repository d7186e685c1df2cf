"""Pins of the oracle's face metrics (Sec. 3.2, eq. (jacobi), (skewness)).

Each check compares the oracle with something other than itself: a library
matrix inverse, closed forms of the spherical and box geometries, exact
symmetries of the maps, and the second-order agreement of the paper's
vertex-averaged metrics with the central-difference ones.
"""
import numpy as np
import pytest

import oracle as O


def shell(n_r, n_t, n_p, **kw):
    return O.Grid(n_r, n_t, n_p, **kw)


def radius(g, s):
    d = g.r_outer - g.r_inner
    if g.radial_stretch == 0:
        return g.r_inner + d * s
    k = g.radial_stretch
    return 0.5 * (g.r_inner + g.r_outer) + d * np.tanh(k * (s - 0.5)) / (2 * np.tanh(k / 2))


def test_metric_from_chords_matches_matrix_inverse():
    """G = det(M) M^-1 M^-T for M with columns t_q (numpy inverse)."""
    rng = np.random.default_rng(3)
    for _ in range(50):
        M = rng.standard_normal((3, 3)) + 3 * np.eye(3)
        if np.linalg.det(M) <= 0:
            M[:, 0] *= -1
        G, det = O.metric_from_chords(M.T)  # rows of the argument are the chords
        Minv = np.linalg.inv(M)
        np.testing.assert_allclose(det, np.linalg.det(M), rtol=1e-13)
        np.testing.assert_allclose(G, np.linalg.det(M) * Minv @ Minv.T, rtol=1e-12, atol=1e-13)


@pytest.mark.parametrize("stretch", [0.0, 2.0])
def test_sphere_central_metrics_closed_form(stretch):
    """Chords of a sphere across a face are mutually orthogonal, with lengths
    dr, 2 r sin(dtheta/2), 2 r sin(theta) sin(dphi/2); G follows in closed
    form and every cross entry vanishes."""
    g = shell(12, 10, 16, radial_stretch=stretch)
    G = O.face_metrics(g)
    nr, nt, np_ = g.shape
    dth = (g.theta1 - g.theta0) / nt
    dph = 2 * np.pi / np_
    rv = radius(g, np.arange(nr + 1) / nr)          # vertex radii r(a)
    rc = radius(g, (np.arange(-1, nr + 1) + 0.5) / nr)  # centre radii r(a+1/2), a=-1..nr
    thv = g.theta0 + np.arange(nt + 1) * dth
    thc = g.theta0 + (np.arange(nt) + 0.5) * dth
    # r-faces a = 1..nr-1
    a = np.arange(1, nr)[:, None]
    drf = rc[a + 1] - rc[a]  # r(a+1/2) - r(a-1/2)
    grr = 4 * rv[a] ** 2 * np.sin(thc)[None] * np.sin(dth / 2) * np.sin(dph / 2) / drf
    np.testing.assert_allclose(G[0, 1:, :, 0], grr, rtol=1e-12)
    # theta-faces b = 1..nt-1
    drc = (rv[1:] - rv[:-1])[:, None]
    gtt = drc * np.sin(thv[1:nt])[None] * np.sin(dph / 2) / np.sin(dth / 2)
    np.testing.assert_allclose(G[4, :, 1:, 0], gtt, rtol=1e-12)
    # phi-faces
    gpp = drc * np.sin(dth / 2) / (np.sin(thc)[None] * np.sin(dph / 2))
    np.testing.assert_allclose(G[8, :, :, 0], gpp, rtol=1e-12)
    # phi invariance and zero cross terms; zero wall faces
    np.testing.assert_allclose(G, np.repeat(G[:, :, :, :1], np_, axis=3), rtol=1e-12, atol=0)
    for k in (1, 2, 3, 5, 6, 7):
        assert not G[k].any()
    assert not G[0:3, 0].any() and not G[3:6, :, 0].any()


def test_identity_box_metrics():
    """Box with spacings h_r, h_t, h_p: G_dd = h_u h_v / h_d, no cross terms."""
    g = shell(6, 8, 10, map=O.MAP_IDENTITY)
    G = O.face_metrics(g)
    hr = (g.r_outer - g.r_inner) / 6
    ht = (g.theta1 - g.theta0) / 8
    hp = 2 * np.pi / 10
    np.testing.assert_allclose(G[0, 1:], ht * hp / hr, rtol=1e-12)
    np.testing.assert_allclose(G[4, :, 1:], hr * hp / ht, rtol=1e-12)
    np.testing.assert_allclose(G[8], hr * ht / hp, rtol=1e-12)
    for k in (1, 2, 3, 5, 6, 7):
        assert not G[k].any()


def test_oblate_axisymmetry():
    """Rotation about the polar axis maps the oblate shell onto itself: the
    metrics are phi-independent and r/theta never couple with phi; the
    r-theta coupling does not vanish."""
    g = shell(16, 16, 32, map=O.MAP_OBLATE, flattening=0.1)
    G = O.face_metrics(g)
    scale = np.abs(G).max()
    assert np.abs(G - G[:, :, :, :1]).max() <= 1e-13 * scale
    for k in (2, 5, 6, 7):
        assert not G[k].any()
    assert np.abs(G[1]).max() > 1e-3 * scale
    assert np.abs(G[3]).max() > 1e-3 * scale


def test_triaxial_has_all_couplings():
    g = shell(8, 8, 16, map=O.MAP_TRIAXIAL, flattening=0.1, skew=0.2)
    G = O.face_metrics(g)
    for k in range(9):
        assert np.abs(G[k]).max() > 0, k


def _rel_diff(g, n):
    gg = O.Grid(n, n, 2 * n, map=g.map, flattening=g.flattening, skew=g.skew,
                radial_stretch=g.radial_stretch)
    A = O.face_metrics(gg, method=O.METRICS_CENTRAL)
    B = O.face_metrics(gg, method=O.METRICS_VERTEX)
    return np.abs(A - B).max() / np.abs(A).max()


@pytest.mark.parametrize("mp", [O.MAP_SPHERE, O.MAP_TRIAXIAL])
def test_paper_vertex_metrics_agree_to_second_order(mp):
    """The paper's vertex-averaged metrics and the central-difference ones
    differ by O(h^2): the gap shrinks about 4x per refinement."""
    g = O.Grid(8, 8, 16, map=mp, flattening=0.1, skew=0.15)
    e = [_rel_diff(g, n) for n in (8, 16, 32)]
    assert e[0] > 0
    r1, r2 = e[0] / e[1], e[1] / e[2]
    assert 3.0 < r1 < 5.5 and 3.4 < r2 < 4.6, (e, r1, r2)


def test_degenerate_map_is_rejected():
    g = shell(4, 4, 4, theta0=1.0, theta1=1.0)
    with pytest.raises(ValueError):
        O.face_metrics(g)
