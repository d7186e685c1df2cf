"""Pins of the oracle's implicit line solves (the ADI steps of eq.
(solve_2)-(solve_4)): |J^-1| psi - coef d/ds_d [G_dd d psi/ds_d] = g on every
line along one direction, no-flux or fixed-value wall faces, periodic phi.
The solves (Thomas; the periodic split with a closing row) are checked
against the plain operator, against numpy's dense solver on each line's
matrix probed from that operator, and against closed forms on the box."""
import numpy as np
import pytest

import oracle as O

PI = np.pi
BCS = [(0, 0.0, 0, 0.0), (1, 0.0, 1, 0.0), (1, 0.7, 0, 0.0), (0, 0.0, 1, -1.3)]


@pytest.mark.parametrize("d", [0, 1, 2])
@pytest.mark.parametrize("bc", BCS)
def test_solve_inverts_the_operator(d, bc):
    g = O.Grid(6, 8, 16, radial_stretch=2.0)
    rhs = np.random.default_rng(10 + d).standard_normal(g.shape)
    psi = O.line_solve(g, d, 0.37, rhs, bc)
    back = O.line_apply(g, d, 0.37, psi, bc)
    assert np.abs(back - rhs).max() <= 1e-12 * np.abs(rhs).max()


@pytest.mark.parametrize("d", [0, 1, 2])
def test_solve_matches_dense_solve_of_each_line(d):
    """Each line's matrix is probed column by column from the plain operator
    (homogeneous walls, unit vectors on that line only) and solved with
    numpy's LU; the oblate shell's lines vary with position."""
    g = O.Grid(5, 6, 8, map=O.MAP_OBLATE, flattening=0.1, radial_stretch=1.5)
    nr, nt, np_ = g.shape
    bc = (1, 0.0, 0, 0.0)
    rhs = np.random.default_rng(20 + d).standard_normal(g.shape)
    psi = O.line_solve(g, d, 2.5, rhs, bc)
    lines = {0: [(slice(None), b, c) for b in (0, 3) for c in (1, 7)],
             1: [(a, slice(None), c) for a in (0, 4) for c in (0, 5)],
             2: [(a, b, slice(None)) for a in (0, 2) for b in (1, 5)]}[d]
    for sl in lines:
        n = g.shape[d]
        A = np.zeros((n, n))
        for j in range(n):
            e = np.zeros(g.shape)
            idx = list(sl)
            idx[d] = j
            e[tuple(idx)] = 1.0
            A[:, j] = O.line_apply(g, d, 2.5, e, bc)[sl]
        want = np.linalg.solve(A, rhs[sl])
        assert np.abs(psi[sl] - want).max() <= 1e-12 * np.abs(want).max()


def _box():
    g = O.Grid(8, 10, 16, map=O.MAP_IDENTITY)
    hr, ht, hp = (g.r_outer - g.r_inner) / g.n_r, (g.theta1 - g.theta0) / g.n_theta, 2 * PI / g.n_phi
    return g, hr, ht, hp


def test_box_eigenvectors():
    """Identity map: constant coefficients, J = h_r h_t h_p, G_dd = (product
    of the other two h) / h_d.  cos(k pi (i + 1/2)/n) is an eigenvector of the
    no-flux line, sin(k pi (i + 1/2)/n) of the zero-value line and
    cos(2 pi m c/n + 0.3) of the periodic line, each with eigenvalue
    J + coef G_dd (2 - 2 cos(theta_k))."""
    g, hr, ht, hp = _box()
    J = hr * ht * hp
    coef = 0.8
    a = np.arange(g.n_r)[:, None, None] + 0.5
    b = np.arange(g.n_theta)[None, :, None] + 0.5
    c = np.arange(g.n_phi)[None, None, :]
    ones = np.ones(g.shape)
    cases = [(0, (0, 0.0, 0, 0.0), np.cos(3 * PI * a / g.n_r) * ones, ht * hp / hr, 3 * PI / g.n_r),
             (1, (1, 0.0, 1, 0.0), np.sin(2 * PI * b / g.n_theta) * ones, hr * hp / ht,
              2 * PI / g.n_theta),
             (2, (0, 0.0, 0, 0.0), np.cos(2 * PI * 3 * c / g.n_phi + 0.3) * ones, hr * ht / hp,
              2 * PI * 3 / g.n_phi)]
    for d, bc, v, G, th in cases:
        want = v / (J + coef * G * (2 - 2 * np.cos(th)))
        got = O.line_solve(g, d, coef, v, bc)
        assert np.abs(got - want).max() <= 1e-12 * np.abs(want).max(), d


@pytest.mark.parametrize("d", [0, 1])
def test_wall_values_hold_a_constant(d):
    """With the value v on both walls and g = |J^-1| v, every flux vanishes:
    psi = v exactly, on the stretched sphere's varying coefficients."""
    g = O.Grid(6, 8, 16, radial_stretch=2.0)
    Jc = np.array([[[O.cell_jdet(g, a, b, c) for c in range(g.n_phi)] for b in range(g.n_theta)]
                   for a in range(g.n_r)])
    psi = O.line_solve(g, d, 3.0, 1.7 * Jc, (1, 1.7, 1, 1.7))
    assert np.abs(psi - 1.7).max() <= 1e-12


def test_short_periodic_line_is_rejected():
    with pytest.raises(ValueError):
        O.line_solve(O.Grid(4, 4, 2), 2, 1.0, np.zeros((4, 4, 2)))
