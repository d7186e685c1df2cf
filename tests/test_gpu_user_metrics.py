"""Caller-supplied face metrics through the C ABI (CPS_METRICS_USER_FACE):
the finest level's metrics come from the caller, each coarser face is half
the sum of its four child faces.  The oracle builds the same hierarchy from
the same array (oracle.Multigrid(face_G=...), pinned in
test_oracle_user_metrics.py), and its exact solvers give the answer the
solve must reach.

Cases: the paper's vertex-averaged metrics of a stretched sphere (their
r-theta cross entries make an 11-point, phi-invariant operator), and the
central metrics of a triaxial shell (all nine entries, stored per cell)."""
import numpy as np
import pytest

import oracle as O
from oracle import direct
from paper_2305_17875_amd import cps, inputs
from paper_2305_17875_amd.inputs import Shell, MAP_TRIAXIAL
from gpu_util import needs_gpu, log, dev, host, rel, torch

pytestmark = [pytest.mark.gpu, needs_gpu]

CASES = [
    ("sphere-vertex-16x16x64", Shell(16, 16, 64, radial_stretch=2.0), O.METRICS_VERTEX),
    ("triaxial-8x8x16", Shell(8, 8, 16, map=MAP_TRIAXIAL, flattening=0.1, skew=0.2),
     O.METRICS_CENTRAL),
]


@pytest.mark.parametrize("name,g,method", CASES, ids=[c[0] for c in CASES])
def test_levels_follow_the_coarsening_rule(name, g, method):
    G0 = O.face_metrics(g, method=method)
    G0[3:6, :, 0] = 5.0  # low theta-wall entries: ignored
    mg = O.Multigrid(g, face_G=G0)
    log("user metrics levels", name)
    s = cps.Solver(g, precision=0, face_G=G0)
    try:
        assert s.levels == mg.levels
        assert s.ncolours == mg.ncol
        assert s.phi_invariant == (g.map != MAP_TRIAXIAL)
        for l, shp in enumerate(s.levels):
            G = torch.empty(9 * int(np.prod(shp)), dtype=torch.float64, device="cuda")
            cps.cps_debug_metrics(s.h, l, G)
            got = host(G).reshape((9,) + shp)
            want = mg.metrics(l)
            # phi-invariant metrics are stored once per ring from c = 0: the
            # oracle's own values vary along the ring by ~1e-14 (rounding)
            assert np.abs(got - want).max() <= 1e-13 * np.abs(want).max(), l
    finally:
        s.close()


@pytest.mark.parametrize("precision,smoother", [(0, 0), (1, 0), (0, 1), (1, 1)])
def test_vertex_metrics_solve_reaches_the_exact_solution(precision, smoother):
    name, g, method = CASES[0]
    G0 = O.face_metrics(g, method=method)
    b = inputs.smoothed_noise(g.shape, 90)
    want = direct.solve_axisym(G0, b)
    log("user metrics solve", precision, smoother)
    s = cps.Solver(g, precision=precision, accel=1, smoother=smoother, max_iters=300, face_G=G0)
    try:
        r = s.solve(dev(b).flatten())
        x = host(r.p).reshape(g.shape)
    finally:
        s.close()
    log("iterations", r.iterations, "rel", r.rel_residual, "error", rel(x, want))
    assert r.status == cps.CPS_OK and r.rel_residual <= 1e-10
    assert rel(x, want) <= 1e-9, rel(x, want)


def test_triaxial_metrics_solve_reaches_the_exact_solution():
    name, g, method = CASES[1]
    G0 = O.face_metrics(g, method=method)
    b = inputs.smoothed_noise(g.shape, 91)
    want = direct.solve_sparse(G0, b)
    s = cps.Solver(g, precision=0, accel=1, max_iters=300, face_G=G0)
    try:
        r = s.solve(dev(b).flatten())
        x = host(r.p).reshape(g.shape)
    finally:
        s.close()
    assert r.status == cps.CPS_OK and rel(x, want) <= 1e-9, rel(x, want)


def test_bad_metrics_and_map_calls_are_rejected():
    g = Shell(8, 8, 32)
    G0 = O.face_metrics(g)
    for k, v in ((2, np.nan), (4, -1e-3), (8, np.inf)):
        B = G0.copy()
        B[k, 3, 4, 5] = v
        with pytest.raises(cps.CpsError) as e:
            cps.Solver(g, precision=0, face_G=B)
        assert e.value.status == cps.CPS_E_INVALID
    s = cps.Solver(g, precision=0, face_G=G0)
    try:
        f = dev(np.ones(g.shape)).flatten()
        u = dev(np.ones((3,) + g.shape)).flatten()
        for call in (lambda: s.divergence(u), lambda: s.line_solve(0, 0.5, f),
                     lambda: cps.cps_line_solve_noalloc(s.h, 0, 0.5, f, torch.empty_like(f))):
            with pytest.raises(cps.CpsError) as e:
                call()
            assert e.value.status == cps.CPS_E_INVALID
    finally:
        s.close()
