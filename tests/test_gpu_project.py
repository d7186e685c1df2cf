"""The projection step on the GPU against the oracle: the divergence
right-hand side of eq. (PC_6) and the velocity correction of eq. (PC_7)
entry by entry on seeded fields (several blocks and a ragged tail, every
map, both metric methods), the whole projection against the oracle's
projection with an exact solve, and sampled cells of the paper-scale shell
in the configuration bench.py times."""
import numpy as np
import pytest

import oracle as O
from paper_2305_17875_amd import cps, inputs
from paper_2305_17875_amd.inputs import Shell, MAP_OBLATE, MAP_TRIAXIAL, MAP_IDENTITY
from gpu_util import needs_gpu, log, dev, host, torch

pytestmark = [pytest.mark.gpu, needs_gpu]

CASES = [
    ("sphere-stretch-8x8x16", Shell(8, 8, 16, radial_stretch=2.0), 0),
    ("sphere-6x10x36", Shell(6, 10, 36), 0),  # 2160 cells: a ragged last block
    # odd n_theta: the divergence takes one row per thread, not row pairs
    ("sphere-4x7x128", Shell(4, 7, 128, radial_stretch=2.0), 0),
    # 12 row pairs (a ragged pair group), two 64-cell phi segments
    ("oblate-8x24x256", Shell(8, 24, 256, map=MAP_OBLATE, flattening=0.1), 0),
    ("oblate-8x8x16", Shell(8, 8, 16, map=MAP_OBLATE, flattening=0.1), 0),
    ("triaxial-6x8x16", Shell(6, 8, 16, map=MAP_TRIAXIAL, flattening=0.1, skew=0.1), 0),
    ("identity-8x8x16", Shell(8, 8, 16, map=MAP_IDENTITY), 0),
    ("sphere-vertex-8x8x16", Shell(8, 8, 16, radial_stretch=2.0), cps.METRICS_PAPER_VERTEX),
]


@pytest.fixture(scope="module", params=CASES, ids=[c[0] for c in CASES])
def case(request):
    name, g, method = request.param
    log("project", name)
    s = cps.Solver(g, precision=0, accel=1, metrics=method)
    yield name, g, method, s
    s.close()


def test_divergence_matches_oracle(case):
    """Per entry to 1e-13 of the largest: both sides sum the same six face
    fluxes; the C rows differ by rounding (and, on rotation-symmetric maps,
    by the GPU's rotation of the (r, theta) tables about the axis)."""
    name, g, method, s = case
    u = np.random.default_rng(5).standard_normal((3,) + g.shape)
    want = O.divergence(g, u, method=method)
    got = host(s.divergence(dev(u).flatten())).reshape(g.shape)
    assert np.abs(got - want).max() <= 1e-13 * np.abs(want).max(), np.abs(got - want).max()
    assert abs(got.sum()) <= 1e-12 * np.abs(got).sum()


def test_correction_matches_oracle(case):
    name, g, method, s = case
    rng = np.random.default_rng(6)
    u = rng.standard_normal((3,) + g.shape)
    phi = rng.standard_normal(g.shape)
    want = O.correct(g, phi, u, method=method)
    ud = dev(u).flatten()
    s.correct(dev(phi).flatten(), ud)
    got = host(ud).reshape((3,) + g.shape)
    scale = np.abs(want - u).max()
    assert np.abs(got - want).max() <= 1e-12 * scale, np.abs(got - want).max() / scale


@pytest.mark.parametrize("g", [Shell(16, 16, 32, radial_stretch=2.0),
                               Shell(16, 16, 32, map=MAP_OBLATE, flattening=0.1)],
                         ids=["sphere-stretch-16x16x32", "oblate-16x16x32"])
def test_projection_matches_oracle_with_exact_solve(g):
    """cps_project (divergence, multigrid solve to 1e-12, correction) against
    the oracle's projection with an exact solve: phi to 1e-9 of its norm,
    the corrected velocity to 1e-9 of the correction."""
    u = inputs.velocity_field(g.shape, 30)
    u_want, phi_want, rhs = O.project(g, u)
    s = cps.Solver(g, precision=0, accel=1)
    try:
        ud = dev(u).flatten()
        r = s.project(ud, tol=1e-12)
        phi = host(r.p).reshape(g.shape)
        got = host(ud).reshape((3,) + g.shape)
    finally:
        s.close()
    assert r.status == cps.CPS_OK and r.rel_residual <= 1e-12
    assert np.linalg.norm(phi - phi_want) <= 1e-9 * np.linalg.norm(phi_want)
    assert np.abs(got - u_want).max() <= 1e-9 * np.abs(u_want - u).max()


def test_rigid_rotation_passes_unchanged():
    """Rotation about the polar axis has zero discrete divergence on a
    rotation-symmetric map: the projection leaves it as it was."""
    g = Shell(16, 16, 32, radial_stretch=2.0)
    X = np.zeros((3,) + g.shape)
    for a in range(g.n_r):
        for b in range(g.n_theta):
            for c in range(g.n_phi):
                X[:, a, b, c] = O.map_point(g, (a + 0.5) / g.n_r, (b + 0.5) / g.n_theta,
                                            (c + 0.5) / g.n_phi)
    u = np.stack([np.zeros(g.shape), -X[2], X[1]])
    s = cps.Solver(g, precision=0, accel=1)
    try:
        ud = dev(u).flatten()
        rhs = host(s.divergence(ud))
        r = s.project(ud, tol=1e-10)
        got = host(ud).reshape(u.shape)
    finally:
        s.close()
    assert np.abs(rhs).max() <= 1e-13 * np.abs(u).max()
    assert r.status == cps.CPS_OK
    assert np.abs(got - u).max() <= 1e-12 * np.abs(u).max()


def test_overlapping_arguments_are_rejected():
    g = Shell(8, 8, 16)
    s = cps.Solver(g, precision=0)
    try:
        u = torch.zeros(3 * g.cells, dtype=torch.float64, device="cuda")
        phi = u[g.cells:2 * g.cells]  # a view into u's second component
        with pytest.raises(cps.CpsError, match="overlap"):
            cps._check(cps.lib().cps_correct(s.h, cps._ptr(phi), cps._ptr(u)))
        with pytest.raises(cps.CpsError, match="overlap"):
            cps._check(cps.lib().cps_divergence(s.h, cps._ptr(u), cps._ptr(phi)))
    finally:
        s.close()


def test_paper_scale_sampled_cells():
    """192 x 256 x 512, stretching 2.0 (bench.py's workload): the divergence
    and, after a full cps_project, the correction with the GPU's own phi, at
    sampled cells (walls, cone tips and random interior cells) against the
    oracle evaluated cell by cell."""
    g = inputs.config2()
    log("project fullsize", g.shape)
    u = inputs.velocity_field(g.shape, 40)
    nr, nt, np_ = g.shape
    rng = np.random.default_rng(8)
    pts = [(0, 0, 0), (nr - 1, nt - 1, np_ - 1), (0, nt // 2, 7), (nr - 1, 3, 500),
           (nr // 2, 0, 100), (nr // 3, nt - 1, 511)]
    pts += [tuple(int(v) for v in (rng.integers(nr), rng.integers(nt), rng.integers(np_)))
            for _ in range(400)]
    cells = np.array([(a * nt + b) * np_ + c for a, b, c in pts], dtype=np.int64)
    s = cps.Solver(g, precision=0, accel=1, max_iters=400)
    try:
        ud = dev(u).flatten()
        div = host(s.divergence(ud)).ravel()
        r = s.project(ud, tol=1e-10)
        phi = host(r.p).ravel()
        got = host(ud).reshape(3, -1)
    finally:
        s.close()
        torch.cuda.empty_cache()
    assert r.status == cps.CPS_OK
    want = O.divergence(g, u, cells=cells)
    assert np.abs(div[cells] - want).max() <= 1e-13 * np.abs(div).max()
    want_u = O.correct(g, phi.reshape(g.shape), u, cells=cells)
    corr = np.abs(want_u - u.reshape(3, -1)[:, cells].T).max()
    assert np.abs(got[:, cells].T - want_u).max() <= 1e-12 * corr
