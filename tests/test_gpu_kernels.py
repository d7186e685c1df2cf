"""Kernel-level parity of the HIP library against the FP64 oracle, through
the C ABI's per-step entry points: face metrics (Sec. 3.2), the flux-form
operator and residual (eq. (PC_8)), one Gauss-Seidel colour pass,
restriction, prolongation, the coarsest solve and one V-cycle.

Grids span several 256-thread blocks with ragged tails, every map (7-, 11-
and 19-point stencils; phi-invariant and 3-D metric storage) and both metric
methods.  Tolerances: the GPU and the oracle evaluate the same formulas in
FP64 in different orders (and the device libm differs from glibc by an ulp),
so per-entry agreement is to a few 1e-15 relative; 1e-13 leaves room for
the cancellation in A x of a smooth field.
"""
import numpy as np
import pytest

import oracle as O
from paper_2305_17875_amd import cps
from paper_2305_17875_amd.inputs import Shell, MAP_SPHERE, MAP_OBLATE, MAP_TRIAXIAL, MAP_IDENTITY
from gpu_util import needs_gpu, log, dev, host, relmax, rel, torch

pytestmark = [pytest.mark.gpu, needs_gpu]

CASES = [
    ("sphere-12x10x14", Shell(12, 10, 14), 0),
    ("sphere-stretch-16x16x32", Shell(16, 16, 32, radial_stretch=2.0), 0),
    ("oblate-16x12x20", Shell(16, 12, 20, map=MAP_OBLATE, flattening=0.12), 0),
    ("triaxial-12x12x16", Shell(12, 12, 16, map=MAP_TRIAXIAL, flattening=0.1, skew=0.2), 0),
    ("identity-8x12x16", Shell(8, 12, 16, map=MAP_IDENTITY), 0),
    ("sphere-vertex-16x16x16", Shell(16, 16, 16), 1),
    ("triaxial-vertex-12x12x16", Shell(12, 12, 16, map=MAP_TRIAXIAL, flattening=0.1, skew=0.2), 1),
    # n_phi / 2 a multiple of 64: LDS-staged tiles of 4 theta rows x 64 phi;
    # one segment per row (phi wraps inside the wavefront), a tile row
    # group overhanging n_theta, and rows of 2 segments (phi halo loads)
    ("sphere-tile-8x6x128", Shell(8, 6, 128, radial_stretch=2.0), 0),
    ("sphere-tile-6x10x256", Shell(6, 10, 256), 0),
    # coarse rings of 128 phi pairs: two wavefronts per coarse row, so the
    # restriction's outer phi values cross a wavefront boundary inside a ring
    ("sphere-wide-8x8x512", Shell(8, 8, 512), 0),
    # the V-cycle's tile path: level 1 (12 x 10 x 32) in ragged 8^3 tiles
    # (r and theta) and four tiles around phi; then two tile levels in a row
    # (24 x 16 x 32 and 12 x 8 x 16), the second's post-smoothed iterate
    # being the first's coarse correction, and a ring of two tiles
    ("sphere-tiles-24x20x64", Shell(24, 20, 64, radial_stretch=2.0), 0),
    ("sphere-tiles-48x32x64", Shell(48, 32, 64), 0),
    # coarse rows of 64 phi pairs in groups of four: the restriction shares
    # its theta rows between the wavefronts of a block through LDS (two row
    # groups, mirrored rows at both theta walls)
    ("sphere-rows-6x16x256", Shell(6, 16, 256, radial_stretch=2.0), 0),
    # full spheres (theta from 0 to pi): the polar rows' r-faces carry an
    # r-theta cross metric on the oblate shell and with vertex metrics
    ("oblate-fullsphere-16x12x20",
     Shell(16, 12, 20, map=MAP_OBLATE, flattening=0.1, theta0=0.0, theta1=np.pi), 0),
    ("sphere-vertex-fullsphere-12x8x16", Shell(12, 8, 16, theta0=0.0, theta1=np.pi), 1),
]


@pytest.fixture(scope="module", params=CASES, ids=[c[0] for c in CASES])
def case(request):
    name, g, method = request.param
    log("kernels", name)
    s = cps.Solver(g, precision=0, accel=0, metrics=method)
    mg = O.Multigrid(g, method=method)
    yield name, g, s, mg
    s.close()


def test_levels_and_colouring_match_oracle(case):
    name, g, s, mg = case
    assert s.levels == mg.levels
    assert s.ncolours == mg.ncol
    assert s.phi_invariant == (g.map != MAP_TRIAXIAL)


def test_metrics(case):
    name, g, s, mg = case
    for l, shp in enumerate(s.levels):
        G = torch.empty(9 * int(np.prod(shp)), dtype=torch.float64, device="cuda")
        cps.cps_debug_metrics(s.h, l, G)
        want = mg.metrics(l)
        got = host(G).reshape(want.shape)
        assert relmax(got, want) < 1e-13, (l, relmax(got, want))
        # zero pattern identical (walls, thresholded cross terms)
        assert ((got == 0) == (want == 0)).all()


def test_apply_and_residual(case):
    name, g, s, mg = case
    rng = np.random.default_rng(1)
    for l, shp in enumerate(s.levels):
        G = mg.metrics(l)
        x = rng.standard_normal(shp)
        b = rng.standard_normal(shp)
        y = torch.empty(int(np.prod(shp)), dtype=torch.float64, device="cuda")
        cps.cps_debug_apply(s.h, l, dev(x).flatten(), y)
        want = O.apply(G, x)
        assert relmax(host(y).reshape(shp), want) < 1e-13
        r = torch.empty_like(y)
        n2 = cps.cps_debug_residual(s.h, l, dev(b).flatten(), dev(x).flatten(), r)
        wr = O.residual(G, b, x)
        assert relmax(host(r).reshape(shp), wr) < 1e-13
        assert abs(n2 - (wr ** 2).sum()) <= 1e-12 * (wr ** 2).sum()


def test_gs_passes(case):
    name, g, s, mg = case
    rng = np.random.default_rng(2)
    for l, shp in enumerate(s.levels[:-1]):
        G = mg.metrics(l)
        b = rng.standard_normal(shp)
        x = rng.standard_normal(shp)
        xd = dev(x).flatten()
        for col in range(s.ncolours):
            cps.cps_debug_gs_pass(s.h, l, col, dev(b).flatten(), xd)
            x = O.gs_pass(G, b, x, mg.ncol, col)
            assert relmax(host(xd).reshape(shp), x) < 1e-12, (l, col)


def test_transfers(case):
    name, g, s, mg = case
    rng = np.random.default_rng(3)
    for l in range(len(s.levels) - 1):
        shp, cshp = s.levels[l], s.levels[l + 1]
        r = rng.standard_normal(shp)
        bc = torch.empty(int(np.prod(cshp)), dtype=torch.float64, device="cuda")
        cps.cps_debug_restrict(s.h, l, dev(r).flatten(), bc)
        assert relmax(host(bc).reshape(cshp), O.restrict(r)) < 1e-14
        e = rng.standard_normal(cshp)
        x = rng.standard_normal(shp)
        xd = dev(x).flatten()
        cps.cps_debug_prolong(s.h, l, dev(e).flatten(), xd)
        assert relmax(host(xd).reshape(shp), O.prolong_add(e, x)) < 1e-14


def test_coarse_solve_and_vcycle(case):
    name, g, s, mg = case
    rng = np.random.default_rng(4)
    cshp = s.levels[-1]
    bc = rng.standard_normal(cshp)
    e = torch.empty(int(np.prod(cshp)), dtype=torch.float64, device="cuda")
    cps.cps_debug_coarse_solve(s.h, dev(bc).flatten(), e)
    assert rel(host(e).reshape(cshp), mg.coarse_solve(bc)) < 1e-11
    b = rng.standard_normal(s.levels[0])
    b -= b.mean()
    x = rng.standard_normal(s.levels[0])
    xd = dev(x).flatten()
    for k in range(3):
        cps.cps_debug_vcycle(s.h, dev(b).flatten(), xd)
        x = mg.vcycle(b, x)
        assert rel(host(xd).reshape(x.shape), x) < 1e-11, k


# Red-residual transfer of the FP64 V-cycle (one fused pass where the level
# allows it): rings of one and two 64-pair coarse segments, several chunks of
# coarse planes, both theta walls, and levels that take the two-kernel form;
# odd coarse plane counts (the last chunk one coarse plane, the top wall's
# fine plane counted twice) with one and two segments; three row groups.
RED_CASES = [
    ("sphere-wide-16x16x512", Shell(16, 16, 512, radial_stretch=2.0)),
    ("sphere-rows-12x32x256", Shell(12, 32, 256)),
    ("sphere-rows-40x16x256", Shell(40, 16, 256, radial_stretch=1.5)),
    ("sphere-tile-6x10x256", Shell(6, 10, 256)),
    ("sphere-odd-6x16x256", Shell(6, 16, 256, radial_stretch=2.0)),
    ("sphere-odd-6x8x512", Shell(6, 8, 512)),
    ("sphere-rows-12x24x256", Shell(12, 24, 256, radial_stretch=1.5)),
]


@pytest.mark.parametrize("name,g", RED_CASES, ids=[c[0] for c in RED_CASES])
def test_red_residual_transfer(name, g):
    """cps_debug_residual_restrict against the oracle: the residual b - A x
    with its black cells set to 0, then the restriction, at 1e-13 of the
    largest coarse value, on every level that forms a red residual."""
    log("red transfer", name)
    s = cps.Solver(g, precision=0, accel=1)
    mg = O.Multigrid(g)
    rng = np.random.default_rng(5)
    done = 0
    try:
        for l in range(len(s.levels) - 1):
            shp, cshp = s.levels[l], s.levels[l + 1]
            if shp[2] % 128 != 0 or shp[1] % 2 != 0:
                with pytest.raises(cps.CpsError):
                    cps.cps_debug_residual_restrict(
                        s.h, l, dev(np.zeros(shp)).flatten(), dev(np.zeros(shp)).flatten(),
                        torch.empty(int(np.prod(cshp)), dtype=torch.float64, device="cuda"))
                continue
            b = rng.standard_normal(shp)
            x = rng.standard_normal(shp)
            bc = torch.empty(int(np.prod(cshp)), dtype=torch.float64, device="cuda")
            cps.cps_debug_residual_restrict(s.h, l, dev(b).flatten(), dev(x).flatten(), bc)
            r = O.residual(mg.metrics(l), b, x)
            a, t, p = np.indices(shp)
            r[(a + t + p) % 2 == 1] = 0.0
            want = O.restrict(r)
            got = host(bc).reshape(cshp)
            err = np.abs(got - want).max() / np.abs(want).max()
            log("red transfer", name, l, shp, f"{err:.1e}")
            assert err < 1e-13, (l, err)
            done += 1
    finally:
        s.close()
    assert done >= 1
