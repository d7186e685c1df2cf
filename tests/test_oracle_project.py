"""Pins of the oracle's projection step: the divergence right-hand side of
eq. (PC_6), d/ds_j [C_ji u_i], and the velocity correction of eq. (PC_7),
u_i - (1/|J^-1|) d/ds_j [C_ji phi], on the collocated grid (face values are
the mean of the two cells sharing the face, no flow through the r- and
theta-walls, phi mirrored at them).  Every expected value here comes from a
closed form or a geometric identity, not from the oracle's own formulas."""
import numpy as np
import pytest

import oracle as O

PI = np.pi


def centres(g):
    """Cell-centre computational coordinates of the box (identity map)."""
    d = g.r_outer - g.r_inner
    hr, ht, hp = d / g.n_r, (g.theta1 - g.theta0) / g.n_theta, 2 * PI / g.n_phi
    x1 = g.r_inner + hr * (np.arange(g.n_r) + 0.5)
    x2 = g.theta0 + ht * (np.arange(g.n_theta) + 0.5)
    x3 = hp * (np.arange(g.n_phi) + 0.5)
    return np.meshgrid(x1, x2, x3, indexing="ij"), (hr, ht, hp)


def cart_centres(g):
    """Cartesian cell centres X[3, n_r, n_theta, n_phi] from the oracle's map."""
    X = np.zeros((3,) + g.shape)
    for a in range(g.n_r):
        for b in range(g.n_theta):
            for c in range(g.n_phi):
                X[:, a, b, c] = O.map_point(g, (a + 0.5) / g.n_r, (b + 0.5) / g.n_theta,
                                            (c + 0.5) / g.n_phi)
    return X


def test_box_divergence_closed_form():
    """Identity map: C = diag(face areas).  For u = (sin k1 x1', sin k2 x2',
    cos m x3) the face mean of a sine is the sine at the face times
    cos(k h / 2), so the divergence is exactly
    A_r sin(k1 h_r) cos(k1 x1') + A_t sin(k2 h_t) cos(k2 x2')
    - A_p sin(m h_p) sin(m x3); the wall fluxes vanish with u1, u2."""
    g = O.Grid(8, 10, 16, map=O.MAP_IDENTITY)
    (x1, x2, x3), (hr, ht, hp) = centres(g)
    k1, k2, m = PI / (g.r_outer - g.r_inner), PI / (g.theta1 - g.theta0), 3
    u = np.stack([np.sin(k1 * (x1 - g.r_inner)), np.sin(k2 * (x2 - g.theta0)), np.cos(m * x3)])
    want = (ht * hp * np.sin(k1 * hr) * np.cos(k1 * (x1 - g.r_inner))
            + hr * hp * np.sin(k2 * ht) * np.cos(k2 * (x2 - g.theta0))
            - hr * ht * np.sin(m * hp) * np.sin(m * x3))
    got = O.divergence(g, u)
    assert np.abs(got - want).max() <= 1e-14 * np.abs(want).max() * 10


def test_box_correction_closed_form():
    """Identity map, u = 0, phi = cos k1 x1' + cos k2 x2' + sin m x3: in the
    interior the correction is minus the central difference of face means,
    -(1/h) sin(k h) sin(k x) along r and theta and (1/h_p) sin(m h_p) cos(m
    x3) along phi; in a wall cell the wall face takes the cell's own value."""
    g = O.Grid(8, 10, 16, map=O.MAP_IDENTITY)
    (x1, x2, x3), (hr, ht, hp) = centres(g)
    k1, k2, m = PI / (g.r_outer - g.r_inner), PI / (g.theta1 - g.theta0), 2
    p1, p2 = np.cos(k1 * (x1 - g.r_inner)), np.cos(k2 * (x2 - g.theta0))
    phi = p1 + p2 + np.sin(m * x3)
    out = O.correct(g, phi, np.zeros((3,) + g.shape))
    g1 = -np.sin(k1 * hr) * np.sin(k1 * (x1 - g.r_inner)) / hr
    g2 = -np.sin(k2 * ht) * np.sin(k2 * (x2 - g.theta0)) / ht
    g3 = np.sin(m * hp) * np.cos(m * x3) / hp
    # wall cells: one face mean replaced by the cell value
    g1[0] = (0.5 * (p1[1] + p1[0]) - p1[0]) / hr
    g1[-1] = (p1[-1] - 0.5 * (p1[-1] + p1[-2])) / hr
    g2[:, 0] = (0.5 * (p2[:, 1] + p2[:, 0]) - p2[:, 0]) / ht
    g2[:, -1] = (p2[:, -1] - 0.5 * (p2[:, -1] + p2[:, -2])) / ht
    for q, want in enumerate((g1, g2, g3)):
        assert np.abs(-out[q] - want).max() <= 1e-12, q


def test_sphere_face_rows_closed_form():
    """Sphere (polar axis x1): the chords across a face are the exact chords
    of circles, so C_r = 4 r_f^2 sin(theta) sin(dth/2) sin(dph/2) e_r,
    C_theta = 2 r dr sin(theta_f) sin(dph/2) e_theta, C_phi = 2 r dr
    sin(dth/2) e_phi, each det = (normal chord) . C, and |J^-1| of a cell is
    the mean of its six face dets; the high walls a = n_r, b = n_theta are
    faces like any other."""
    g = O.Grid(6, 8, 12, radial_stretch=2.0)
    nr, nt, np_ = g.shape
    dth, dph = (g.theta1 - g.theta0) / nt, 2 * PI / np_

    def rad(s):
        return np.linalg.norm(O.map_point(g, s, 0.5, 0.0))

    def er(t, p): return np.array([np.cos(t), np.sin(t) * np.cos(p), np.sin(t) * np.sin(p)])
    def eth(t, p): return np.array([-np.sin(t), np.cos(t) * np.cos(p), np.cos(t) * np.sin(p)])
    def eph(p): return np.array([0.0, -np.sin(p), np.cos(p)])

    for (a, b, c) in [(0, 0, 0), (2, 3, 5), (nr, 4, 11), (3, nt, 7), (5, 7, 0)]:
        th = lambda i: g.theta0 + dth * i
        ph = lambda i: dph * i
        if a <= nr - 1 or a == nr:
            rf = rad(a / nr)
            drf = rad((a + 0.5) / nr) - rad((a - 0.5) / nr)
            C, det = O.face_crow(g, 0, a, min(b, nt - 1), c)
            bb = min(b, nt - 1)
            wantC = 4 * rf**2 * np.sin(th(bb + 0.5)) * np.sin(dth / 2) * np.sin(dph / 2) \
                * er(th(bb + 0.5), ph(c + 0.5))
            assert np.allclose(C, wantC, rtol=1e-12, atol=1e-14 * np.abs(wantC).max())
            assert abs(det - drf * np.linalg.norm(wantC)) <= 1e-12 * det
        if a < nr:
            rc = rad((a + 0.5) / nr)
            drc = rad((a + 1) / nr) - rad(a / nr)
            C, det = O.face_crow(g, 1, a, b, c)
            wantC = 2 * rc * drc * np.sin(th(b)) * np.sin(dph / 2) * eth(th(b), ph(c + 0.5))
            assert np.allclose(C, wantC, rtol=1e-12, atol=1e-14 * np.abs(wantC).max())
            assert abs(det - 2 * rc * np.sin(dth / 2) * np.linalg.norm(wantC)) <= 1e-12 * det
            if b < nt:
                C, det = O.face_crow(g, 2, a, b, c)
                wantC = 2 * rc * drc * np.sin(dth / 2) * eph(ph(c))
                assert np.allclose(C, wantC, rtol=1e-12, atol=1e-14 * np.abs(wantC).max())
                want_det = 2 * rc * np.sin(th(b + 0.5)) * np.sin(dph / 2) * np.linalg.norm(wantC)
                assert abs(det - want_det) <= 1e-12 * det
    # cell |J^-1| = mean of the six face dets (Sec. 3.2 item 3), closed form
    a, b, c = 2, 3, 5
    r0, r1, rm = rad(a / nr), rad((a + 1) / nr), rad((a + 0.5) / nr)
    dr_a = lambda i: rad((i + 0.5) / nr) - rad((i - 0.5) / nr)
    s2 = np.sin(dth / 2) * np.sin(dph / 2)
    faces = [dr_a(a) * 4 * r0**2 * np.sin(th(b + 0.5)) * s2,
             dr_a(a + 1) * 4 * r1**2 * np.sin(th(b + 0.5)) * s2,
             4 * (r1 - r0) * rm**2 * np.sin(th(b)) * s2,
             4 * (r1 - r0) * rm**2 * np.sin(th(b + 1)) * s2,
             4 * (r1 - r0) * rm**2 * np.sin(th(b + 0.5)) * s2,
             4 * (r1 - r0) * rm**2 * np.sin(th(b + 0.5)) * s2]
    assert abs(O.cell_jdet(g, a, b, c) - np.mean(faces)) <= 1e-12 * np.mean(faces)


@pytest.mark.parametrize("kw", [dict(), dict(radial_stretch=2.0),
                                dict(map=O.MAP_OBLATE, flattening=0.1)])
def test_rigid_rotation_about_the_axis_is_divergence_free(kw):
    """u = e1 x X (rotation about the polar axis) is tangent to every r- and
    theta-surface of an axisymmetric map, and the chords of such a map lie
    in meridional planes or along e_phi: every r- and theta-face flux is 0
    and every phi-face carries the same flux, so the divergence vanishes to
    rounding.  The projection leaves it unchanged."""
    g = O.Grid(8, 8, 16, **kw)
    X = cart_centres(g)
    u = np.stack([np.zeros(g.shape), -X[2], X[1]])
    div = O.divergence(g, u)
    C, _ = O.face_crow(g, 2, 4, 4, 0)
    scale = np.linalg.norm(C) * np.abs(u).max()
    assert np.abs(div).max() <= 1e-13 * scale
    un, phi, rhs = O.project(g, u)
    assert np.abs(phi).max() <= 1e-11 * np.abs(u).max()
    assert np.abs(un - u).max() <= 1e-11 * np.abs(u).max()


def test_divergence_sums_to_zero():
    """No flow through the walls and a periodic phi: the fluxes telescope,
    so the divergence of any field sums to zero (triaxial map, random u)."""
    g = O.Grid(6, 8, 16, map=O.MAP_TRIAXIAL, flattening=0.1, skew=0.1)
    u = np.random.default_rng(3).standard_normal((3,) + g.shape)
    div = O.divergence(g, u)
    assert abs(div.sum()) <= 1e-13 * np.abs(div).sum()


def _grad_psi(g, X):
    """psi = cos(pi (r - r_i)/d) cos(pi (theta - theta0)/(theta1 - theta0))
    sin(2 phi) (zero normal derivative on every wall) and its Cartesian
    gradient psi_r e_r + psi_theta/r e_theta + psi_phi/(r sin theta) e_phi."""
    r = np.linalg.norm(X, axis=0)
    th = np.arccos(X[0] / r)
    ph = np.arctan2(X[2], X[1])
    d, L = g.r_outer - g.r_inner, g.theta1 - g.theta0
    kr, kt = PI / d, PI / L
    R, T, P = np.cos(kr * (r - g.r_inner)), np.cos(kt * (th - g.theta0)), np.sin(2 * ph)
    pr = -kr * np.sin(kr * (r - g.r_inner)) * T * P
    pt = -kt * R * np.sin(kt * (th - g.theta0)) * P
    pp = 2 * R * T * np.cos(2 * ph)
    er = np.stack([np.cos(th), np.sin(th) * np.cos(ph), np.sin(th) * np.sin(ph)])
    et = np.stack([-np.sin(th), np.cos(th) * np.cos(ph), np.cos(th) * np.sin(ph)])
    ep = np.stack([np.zeros_like(ph), -np.sin(ph), np.cos(ph)])
    return pr * er + pt / r * et + pp / (r * np.sin(th)) * ep


def test_projection_removes_a_gradient_field_at_second_order():
    """u = grad psi with psi Neumann on every wall: the projection leaves
    u - grad_h phi = O(h^2) (collocated, approximate projection); the
    remainder drops ~4x per refinement."""
    errs = []
    for n in (8, 16, 32):
        g = O.Grid(n, n, 2 * n)
        X = cart_centres(g)
        u = _grad_psi(g, X)
        un, phi, rhs = O.project(g, u)
        errs.append(np.sqrt((un**2).sum() / (u**2).sum()))
    ratios = [errs[i] / errs[i + 1] for i in range(2)]
    assert all(3.3 < q < 4.7 for q in ratios), (errs, ratios)


def test_correction_converges_to_the_cartesian_gradient():
    """(1/|J^-1|) d/ds_j [C_ji phi] -> d phi / d x_i at second order
    (phi = x1^2 + x2 x3 + sin x3 on the stretched sphere) in the band
    sin(theta) > 1/2 off the walls, and the sum of |J^-1| over the cells ->
    the shell volume at second order.  Next to the cone tips the chord faces
    of a cell close only to O(dtheta^2 / sin(theta)) of its volume (the
    discrete metric identity), which is first order where sin(theta) ~
    dtheta, so the band keeps a fixed distance from the axis."""
    errs, verrs = [], []
    for n in (8, 16, 32):
        g = O.Grid(n, n, 2 * n, radial_stretch=2.0)
        X = cart_centres(g)
        r = np.linalg.norm(X, axis=0)
        band = np.hypot(X[1], X[2]) / r > 0.5
        band[0] = band[-1] = False
        band[:, 0] = band[:, -1] = False
        phi = X[0] ** 2 + X[1] * X[2] + np.sin(X[2])
        grad = np.stack([2 * X[0], X[2], X[1] + np.cos(X[2])])
        got = -O.correct(g, phi, np.zeros((3,) + g.shape))
        errs.append(np.abs(got - grad).max(axis=0)[band].max())
        vol = sum(O.cell_jdet(g, a, b, 0) for a in range(n) for b in range(n)) * 2 * n
        exact = 2 * PI / 3 * (g.r_outer**3 - g.r_inner**3) * (np.cos(g.theta0) - np.cos(g.theta1))
        verrs.append(abs(vol - exact) / exact)
    for e in (errs, verrs):
        q = [e[i] / e[i + 1] for i in range(2)]
        assert all(3.0 < x < 4.7 for x in q), (e, q)
