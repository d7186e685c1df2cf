"""The grids of the paper's simulations (tests/golden/paper_grids.txt, from
its table of results) against the host-side plan: each has a level plan that
ends at a coarsest level of at most 1024 cells by halving every direction,
and the library's resident-footprint estimate for it fits one 288 GB GPU."""
import os

import pytest

import oracle as O
from paper_2305_17875_amd import cps
from paper_2305_17875_amd.inputs import Shell

HERE = os.path.dirname(os.path.abspath(__file__))
HBM = 288 * 10**9


def paper_grids():
    rows = []
    for line in open(os.path.join(HERE, "golden", "paper_grids.txt")):
        line = line.split("#")[0].split()
        if line:
            ra, nz, ne, nx = line
            # the paper's (zeta, eta, xi) are the build's (theta, r, phi)
            rows.append((float(ra), (int(ne), int(nz), int(nx))))
    return rows


def test_fixture_holds_the_three_simulations():
    rows = paper_grids()
    assert [ra for ra, _ in rows] == [1e5, 1e7, 1e8]
    assert rows[1][1] == rows[2][1] == (256, 512, 512)


@pytest.mark.parametrize("ra,shape", paper_grids(), ids=lambda v: str(v))
def test_paper_grid_plans_and_fits_one_gpu(ra, shape):
    plan = O.level_plan(*shape)
    nr, nt, nph = plan[-1]
    assert nr * nt * nph <= 1024
    for fine, coarse in zip(plan, plan[1:]):
        assert tuple(2 * c for c in coarse) == fine
    if not os.path.exists(cps.LIB_PATH):
        pytest.skip("libcps.so not built")
    for precision in (0, 1):
        opts = cps.cps_opts(precision=precision)
        b = cps.cps_service_footprint(cps.make_grid(Shell(*shape, radial_stretch=2.0)), opts)
        cells = shape[0] * shape[1] * shape[2]
        # at least the FP64 right-hand side, solution and search vectors
        assert 4 * 8 * cells <= b <= HBM, (precision, b)
