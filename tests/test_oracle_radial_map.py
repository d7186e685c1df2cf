"""Pins of the oracle's radial clustering, eq. (stretching) (Sec. 4): the
radius of a vertex plane is the paper's r(j) shifted to the mid-radius and
scaled by the gap, with j - 1 = s n_r.  The oracle's radius is read back as
|X| of its spherical map, and checked against what the equation fixes
without retyping it:
  * the end vertices lie on the walls, r(0) = r_i and r(1) = r_o, and the
    middle one on the mid-radius;
  * the clustering is mirror-symmetric about mid-gap (r(s) - r_m is odd in
    s - 1/2) and monotone;
  * every cell's width equals the derivative of the map at the cell centre
    times the index spacing, to second order in the spacing (the derivative
    of tanh is sech^2, a different formula from the one integrated);
  * on the paper-scale grid (192 radial cells, stretching factor 2.0, gap
    1) the wall cells are 0.002895 wide and the mid-gap ones 0.006838
    (evaluated by hand to four figures from the second-order Taylor
    expansion of tanh about 1 and about 0), a ratio close to sech^2(1) =
    0.420, the slope ratio of tanh between the wall and the middle.
"""
import numpy as np
import pytest

import oracle as O


def radii(n, stretch, r_i=1.5, r_o=2.5):
    """Vertex radii a / n, a = 0..n, from the oracle's sphere map."""
    g = O.Grid(n, 4, 4, r_inner=r_i, r_outer=r_o, radial_stretch=stretch)
    return np.array([np.linalg.norm(O.map_point(g, a / n, 0.3, 0.1)) for a in range(n + 1)])


@pytest.mark.parametrize("stretch", [0.5, 2.0, 4.0])
def test_ends_middle_and_symmetry(stretch):
    r = radii(64, stretch)
    assert abs(r[0] - 1.5) <= 1e-14 and abs(r[-1] - 2.5) <= 1e-14
    assert abs(r[32] - 2.0) <= 1e-14
    np.testing.assert_allclose(r - 2.0, -(r[::-1] - 2.0), rtol=0, atol=1e-14)
    assert np.all(np.diff(r) > 0)
    # clustered toward both walls: the wall cells are the narrowest
    w = np.diff(r)
    assert w[0] == pytest.approx(w.min()) and w[31] == pytest.approx(w.max())


def test_uniform_without_stretching():
    r = radii(10, 0.0, 0.7, 1.9)
    np.testing.assert_allclose(np.diff(r), 0.12, rtol=0, atol=1e-14)


@pytest.mark.parametrize("stretch", [1.0, 2.0, 3.0])
def test_cell_width_is_the_derivative_times_the_spacing(stretch):
    """width_a / (h r'(s_a + h/2)) - 1 = O(h^2), with r'(s) = d k sech^2(k (s -
    1/2)) / (2 tanh(k / 2)) and h = 1/n: the error drops 4x per doubling."""
    k = stretch
    errs = []
    for n in (24, 48, 96):
        w = np.diff(radii(n, k))
        sc = (np.arange(n) + 0.5) / n
        slope = k / np.cosh(k * (sc - 0.5)) ** 2 / (2.0 * np.tanh(k / 2.0))
        errs.append(np.abs(w / (slope / n) - 1.0).max())
    assert errs[0] < 0.05
    assert 3.6 < errs[0] / errs[1] < 4.4 and 3.6 < errs[1] / errs[2] < 4.4, errs


def test_paper_scale_spacings():
    w = np.diff(radii(192, 2.0))
    for a in (0, 191):
        assert abs(w[a] - 0.002895) < 5e-7, (a, w[a])
    for a in (95, 96):
        assert abs(w[a] - 0.006838) < 5e-7, (a, w[a])
    assert abs(w[0] / w[95] - 1.0 / np.cosh(1.0) ** 2) < 0.01
