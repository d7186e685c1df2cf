"""The zebra (r, phi)-plane smoother on the GPU (Fourier transform along phi
+ Thomas along r) against the oracle's exact block Gauss-Seidel solves
(sparse LU of every (r, phi) plane), its V-cycle against the oracle's plane
V-cycle, and solves against the oracle's exact solution; for the 7-point
operator and for the oblate shell's 11-point one (r-theta cross terms,
whose r-lines are tridiagonal but not symmetric)."""
import numpy as np
import pytest

import oracle as O
from oracle import direct, plane
from paper_2305_17875_amd import cps, inputs
from paper_2305_17875_amd.inputs import Shell, MAP_OBLATE, MAP_IDENTITY, MAP_TRIAXIAL
from gpu_util import needs_gpu, log, dev, host, rel, relmax, torch

pytestmark = [pytest.mark.gpu, needs_gpu]

CASES = [
    ("sphere-stretch-8x8x64", Shell(8, 8, 64, radial_stretch=2.0)),
    ("sphere-6x10x32", Shell(6, 10, 32)),           # 5 rows of each parity
    ("sphere-8x6x128", Shell(8, 6, 128, radial_stretch=2.0)),
    ("sphere-4x4x2048", Shell(4, 4, 2048)),         # the longest ring (1024 per parity)
    ("identity-8x8x32", Shell(8, 8, 32, map=MAP_IDENTITY)),
    ("oblate-8x8x32", Shell(8, 8, 32, map=MAP_OBLATE, flattening=0.1)),
    ("oblate-stretch-6x10x64", Shell(6, 10, 64, map=MAP_OBLATE, flattening=0.15,
                                     radial_stretch=1.5)),
    ("oblate-sphere-full-8x8x16", Shell(8, 8, 16, map=MAP_OBLATE, flattening=0.2,
                                        theta0=0.0, theta1=np.pi)),
    ("oblate-4x6x1024", Shell(4, 6, 1024, map=MAP_OBLATE, flattening=0.1)),
]


@pytest.fixture(scope="module", params=CASES, ids=[c[0] for c in CASES])
def case(request):
    name, g = request.param
    log("plane", name)
    s = cps.Solver(g, precision=0, accel=0, smoother=1)
    mg = O.Multigrid(g)
    yield name, g, s, mg
    s.close()


def test_half_sweeps_match_block_gauss_seidel(case):
    """Per entry to 1e-11 relative: the transform of a ring of up to 2048
    cells adds ~log2(n) roundings, amplified by the plane systems' condition
    (phi coupling ~1e3 x the theta coupling on the longest ring)."""
    name, g, s, mg = case
    rng = np.random.default_rng(11)
    for l, shp in enumerate(s.levels[:-1]):
        G = mg.metrics(l)
        sm = plane.PlaneSmoother(G)
        b = rng.standard_normal(shp)
        x = rng.standard_normal(shp)
        for parity in (0, 1):
            want = sm.half_sweep(b, x, parity)
            xd = dev(x).flatten()
            cps.cps_debug_plane_sweep(s.h, l, parity, dev(b).flatten(), xd)
            got = host(xd).reshape(shp)
            assert relmax(got, want) < 1e-11, (l, parity, relmax(got, want))
            x = want


def test_plane_vcycle_matches_oracle(case):
    name, g, s, mg = case
    pm = plane.PlaneMultigrid(mg, nu=2)
    rng = np.random.default_rng(12)
    b = rng.standard_normal(g.shape)
    b -= b.mean()
    x = rng.standard_normal(g.shape) * 0.1
    want = pm.vcycle(b, x)
    xd = dev(x).flatten()
    cps.cps_debug_vcycle(s.h, dev(b).flatten(), xd)
    got = host(xd).reshape(g.shape)
    assert relmax(got, want) < 1e-11, relmax(got, want)


@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("kind", ["sphere", "oblate"])
def test_plane_solve_against_exact_and_fewer_cycles(precision, kind):
    if kind == "sphere":
        g = Shell(32, 32, 64, radial_stretch=2.0)
    else:
        g = Shell(32, 32, 64, map=MAP_OBLATE, flattening=0.1, radial_stretch=2.0)
    b = inputs.smoothed_noise(g.shape, 21)
    want = direct.solve_axisym(O.face_metrics(g), b)
    out = {}
    for sm in (0, 1):
        s = cps.Solver(g, precision=precision, accel=1, smoother=sm, max_iters=400)
        try:
            r = s.solve(dev(b).flatten())
            out[sm] = (host(r.p).reshape(g.shape), r)
        finally:
            s.close()
    x, r = out[1]
    assert r.status == cps.CPS_OK and r.rel_residual <= 1e-10
    assert rel(x, want) <= 1e-9, rel(x, want)
    log("plane cycles", kind, precision, out[0][1].iterations, r.iterations)
    assert r.iterations * 3 <= out[0][1].iterations


def test_plane_smoother_rejects_what_it_cannot_do():
    with pytest.raises(cps.CpsError, match="phi-invariant"):
        cps.Solver(Shell(16, 16, 32, map=MAP_TRIAXIAL, flattening=0.1, skew=0.2), smoother=1)
    with pytest.raises(cps.CpsError, match="power of two"):
        cps.Solver(Shell(16, 16, 48), smoother=1)
    with pytest.raises(cps.CpsError, match="n_phi <= 512"):
        cps.cps_batch_setup([cps.make_grid(Shell(4, 4, 1024))], cps.cps_metrics(0),
                            cps.cps_opts(1, 200, 1, 0, 0, 1, None))


def test_plane_graph_replays_equal_eager():
    g = Shell(16, 16, 64, radial_stretch=2.0)
    side = torch.cuda.Stream()
    sg = cps.Solver(g, precision=1, accel=1, smoother=1, stream=side)
    se = cps.Solver(g, precision=1, accel=1, smoother=1, stream=side, eager=True)
    try:
        for k in range(3):
            b = dev(inputs.smoothed_noise(g.shape, 400 + k)).flatten()
            torch.cuda.synchronize()
            xg = host(sg.solve(b).p)
            xe = host(se.solve(b).p)
            assert np.array_equal(xg, xe), k
    finally:
        sg.close()
        se.close()


def test_service_with_plane_smoother_recomputes_pivots_on_remap():
    """The service with smoother = 1 and one slot: three sphere stretchings
    of one shape share a pooled hierarchy, whose metrics, coarse inverse and
    plane pivots are recomputed in place for each new map; every result
    equals a fresh solve bit for bit, and the footprint estimate covers the
    resident hierarchy."""
    shape = (16, 16, 64)
    gs = [Shell(*shape, radial_stretch=s) for s in (0.0, 2.0, 1.0)]
    reqs = [(g, inputs.smoothed_noise(shape, 60 + i)) for i, g in enumerate(gs)]
    log("plane service remap")
    svc = cps.Service(1 << 30, max_slots=1, precision=1, smoother=1)
    try:
        fp = svc.footprint(gs[0])
        out = [svc.wait(svc.submit(g, b)) for g, b in reqs]
        st = svc.stats()
    finally:
        svc.close()
    for i, ((g, b), (status, p, info)) in enumerate(zip(reqs, out)):
        assert status == cps.CPS_OK, i
        s = cps.Solver(g, precision=1, accel=1, smoother=1)
        try:
            r = s.solve(dev(b).flatten())
            xa = host(r.p).reshape(shape)
        finally:
            s.close()
        assert info.iterations == r.iterations, i
        assert np.array_equal(p, xa), (i, np.abs(p - xa).max())
    assert st["hierarchies_built"] == 1 and st["hierarchies_reused"] == 2, st
    assert st["map_rebuilds"] == 2, st
    assert 0 < st["hbm_in_use"] <= fp, (st["hbm_in_use"], fp)


def test_automatic_smoother_in_the_service():
    """smoother = 2: the hierarchies of a sphere and of an oblate shell (r-theta
    cross terms) take the plane smoother, a triaxial shell's the point
    smoother; each result equals the same problem solved alone with the same
    opts, bit for bit, and the axisymmetric ones need fewer cycles than with
    the point smoother."""
    reqs = [(Shell(16, 16, 32, radial_stretch=2.0), inputs.smoothed_noise((16, 16, 32), 70)),
            (Shell(16, 16, 32, map=MAP_OBLATE, flattening=0.1),
             inputs.smoothed_noise((16, 16, 32), 71)),
            (Shell(32, 32, 64, radial_stretch=2.0), inputs.smoothed_noise((32, 32, 64), 72)),
            (Shell(16, 16, 32, map=MAP_TRIAXIAL, flattening=0.1, skew=0.2),
             inputs.smoothed_noise((16, 16, 32), 73))]
    log("automatic smoother service")
    svc = cps.Service(1 << 30, max_slots=2, precision=1, smoother=2)
    try:
        out = [svc.wait(svc.submit(g, b)) for g, b in reqs]
    finally:
        svc.close()
    for i, ((g, b), (status, p, info)) in enumerate(zip(reqs, out)):
        assert status == cps.CPS_OK, i
        its = {}
        for sm in (2, 0):
            s = cps.Solver(g, precision=1, accel=1, smoother=sm)
            try:
                r = s.solve(dev(b).flatten())
                its[sm] = r.iterations
                if sm == 2:
                    assert np.array_equal(p, host(r.p).reshape(g.shape)), i
                    assert info.iterations == r.iterations, i
            finally:
                s.close()
        log("automatic smoother", g.map, its)
        if g.map == MAP_TRIAXIAL:
            assert its[2] == its[0], its
        else:
            assert 3 * its[2] <= its[0], its
