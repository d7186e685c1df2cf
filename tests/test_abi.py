"""Host-side checks of the C ABI: the library loads without a GPU, exports
every function that include/cps.h declares, and the ctypes structures match
the C layout (sizes and offsets printed by a gcc-compiled probe)."""
import os
import re
import subprocess
import ctypes

import pytest

from paper_2305_17875_amd import cps

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "cps.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(cps_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_the_entry_points():
    names = declared_functions()
    for want in ("cps_setup", "cps_solve", "cps_destroy", "cps_last_error", "cps_levels",
                 "cps_debug_residual", "cps_debug_gs_pass", "cps_debug_vcycle",
                 "cps_divergence", "cps_correct", "cps_project", "cps_line_solve"):
        assert want in names


def test_library_exports_every_declared_symbol():
    if not os.path.exists(cps.LIB_PATH):
        pytest.skip("libcps.so not built")
    out = subprocess.check_output(["nm", "-D", "--defined-only", cps.LIB_PATH], text=True)
    exported = {l.split()[-1] for l in out.splitlines() if " T " in l}
    missing = [n for n in declared_functions() if n not in exported]
    assert not missing, missing
    L = cps.lib()  # loads on a host without a GPU
    for n in declared_functions():
        assert hasattr(L, n)


def test_ctypes_layout_matches_c(tmp_path):
    probe = tmp_path / "probe.c"
    probe.write_text(
        '#include <stdio.h>\n#include <stddef.h>\n#include "cps.h"\n'
        "int main(void){\n"
        'printf("%zu %zu %zu %zu\\n", sizeof(cps_grid), sizeof(cps_metrics), sizeof(cps_opts), sizeof(cps_info));\n'
        'printf("%zu %zu %zu\\n", offsetof(cps_grid, r_inner), offsetof(cps_grid, skew), offsetof(cps_grid, n_levels));\n'
        'printf("%zu %zu\\n", offsetof(cps_opts, stream), offsetof(cps_info, seconds));\n'
        'printf("%zu %zu\\n", sizeof(cps_line_bc), offsetof(cps_line_bc, value_hi));\n'
        'printf("%zu\\n", offsetof(cps_metrics, face_G));\n'
        "return 0;}\n")
    exe = tmp_path / "probe"
    subprocess.check_call(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), str(probe),
                           "-o", str(exe)])
    vals = [int(v) for v in subprocess.check_output([str(exe)], text=True).split()]
    assert vals[:4] == [ctypes.sizeof(cps.cps_grid), ctypes.sizeof(cps.cps_metrics),
                        ctypes.sizeof(cps.cps_opts), ctypes.sizeof(cps.cps_info)]
    assert vals[4:7] == [cps.cps_grid.r_inner.offset, cps.cps_grid.skew.offset,
                         cps.cps_grid.n_levels.offset]
    assert vals[7:9] == [cps.cps_opts.stream.offset, cps.cps_info.seconds.offset]
    assert vals[9:11] == [ctypes.sizeof(cps.cps_line_bc), cps.cps_line_bc.value_hi.offset]
    assert vals[11:] == [cps.cps_metrics.face_G.offset]


def test_grid_default_and_invalid_setup_without_gpu():
    """cps_grid_default is pure host code; cps_setup rejects bad grids before
    touching the device."""
    if not os.path.exists(cps.LIB_PATH):
        pytest.skip("libcps.so not built")
    g = cps.cps_grid()
    cps.lib().cps_grid_default(ctypes.byref(g))
    assert (g.n_r, g.n_theta, g.n_phi, g.map) == (32, 32, 32, cps.MAP_SPHERE)
    assert abs(g.r_inner - 1.5) < 1e-15 and abs(g.theta1 - (3.141592653589793 - 0.05)) < 1e-15
    g.n_r = 0
    h = ctypes.c_void_p()
    st = cps.lib().cps_setup(ctypes.byref(g), None, None, ctypes.byref(h))
    assert st == cps.CPS_E_INVALID and not h.value
    assert "positive" in cps.last_error()


def test_service_report_layout_and_footprint(tmp_path):
    """cps_service_report matches the C layout; cps_service_footprint is host
    code: it grows with the grid, covers the FP64 metrics and vectors, and
    rejects grids the level plan cannot take."""
    probe = tmp_path / "probe2.c"
    probe.write_text(
        '#include <stdio.h>\n#include <stddef.h>\n#include "cps.h"\n'
        "int main(void){\n"
        'printf("%zu %zu %zu %zu %zu\\n", sizeof(cps_service_report),'
        " offsetof(cps_service_report, active), offsetof(cps_service_report, p50_ms),"
        " offsetof(cps_service_report, hbm_in_use), offsetof(cps_service_report, evictions));\n"
        "return 0;}\n")
    exe = tmp_path / "probe2"
    subprocess.check_call(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), str(probe),
                           "-o", str(exe)])
    vals = [int(v) for v in subprocess.check_output([str(exe)], text=True).split()]
    R = cps.cps_service_report
    assert vals == [ctypes.sizeof(R), R.active.offset, R.p50_ms.offset, R.hbm_in_use.offset,
                    R.evictions.offset]
    if not os.path.exists(cps.LIB_PATH):
        pytest.skip("libcps.so not built")
    from paper_2305_17875_amd.inputs import Shell, MAP_OBLATE
    opts = cps.cps_opts(1, 200, 1, 0, 0, 0, None)
    f = [cps.cps_service_footprint(cps.make_grid(Shell(*s)), opts)
         for s in [(16, 16, 16), (32, 32, 32), (64, 64, 128)]]
    assert f[0] < f[1] < f[2]
    n = 64 * 64 * 128
    assert f[2] > 8 * 5 * n  # at least the five FP64 vectors of the finest level
    bicg = cps.cps_opts(1, 200, 2, 0, 0, 0, None)
    fo = cps.cps_service_footprint(cps.make_grid(Shell(64, 64, 128, map=MAP_OBLATE,
                                                        flattening=0.1)), bicg)
    assert fo > f[2]  # BiCGStab's extra vectors
    with pytest.raises(cps.CpsError, match="coarsest"):
        cps.cps_service_footprint(cps.make_grid(Shell(15, 16, 32)), opts)
