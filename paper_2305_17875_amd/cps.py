"""ctypes binding of libcps.so -- argument marshalling only.

Every function here forwards to the C ABI of ``include/cps.h`` with the same
name; all computation runs in the HIP library.  Arrays are torch tensors on
the current HIP device (float64, contiguous, [r][theta][phi]); torch is used
only to own device memory and to provide the stream.  Loading fails loudly if
the library has not been built (``python -m paper_2305_17875_amd.build``).
"""
from __future__ import annotations

import ctypes
import math
import os
from dataclasses import dataclass

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libcps.so")

CPS_OK, CPS_E_INVALID, CPS_E_OOM, CPS_E_HIP, CPS_E_NOT_CONVERGED, CPS_E_DIVERGED = 0, -1, -2, -3, -4, -5
STATUS_NAMES = {0: "CPS_OK", -1: "CPS_E_INVALID", -2: "CPS_E_OOM", -3: "CPS_E_HIP",
                -4: "CPS_E_NOT_CONVERGED", -5: "CPS_E_DIVERGED"}
MAP_IDENTITY, MAP_SPHERE, MAP_OBLATE, MAP_TRIAXIAL = 0, 1, 2, 3
METRICS_MAP_CENTRAL, METRICS_PAPER_VERTEX, METRICS_USER_FACE = 0, 1, 2


class cps_grid(ctypes.Structure):
    _fields_ = [
        ("n_r", ctypes.c_int32), ("n_theta", ctypes.c_int32), ("n_phi", ctypes.c_int32),
        ("map", ctypes.c_int32),
        ("r_inner", ctypes.c_double), ("r_outer", ctypes.c_double),
        ("theta0", ctypes.c_double), ("theta1", ctypes.c_double),
        ("radial_stretch", ctypes.c_double), ("flattening", ctypes.c_double),
        ("skew", ctypes.c_double), ("n_levels", ctypes.c_int32),
    ]


class cps_metrics(ctypes.Structure):
    _fields_ = [("method", ctypes.c_int32), ("face_G", ctypes.c_void_p)]


class cps_opts(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int32), ("max_iters", ctypes.c_int32),
                ("accel", ctypes.c_int32), ("tune", ctypes.c_int32), ("eager", ctypes.c_int32),
                ("smoother", ctypes.c_int32), ("stream", ctypes.c_void_p)]


class cps_info(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int32), ("rel_residual", ctypes.c_double),
                ("rhs_mean_removed", ctypes.c_double), ("seconds", ctypes.c_double)]


class cps_service_report(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_uint64), ("completed", ctypes.c_uint64),
                ("failed", ctypes.c_uint64), ("queued", ctypes.c_uint64),
                ("active", ctypes.c_int32), ("peak_active", ctypes.c_int32),
                ("p50_ms", ctypes.c_double), ("p99_ms", ctypes.c_double),
                ("mean_ms", ctypes.c_double), ("max_ms", ctypes.c_double),
                ("unknowns_per_s", ctypes.c_double),
                ("hbm_in_use", ctypes.c_uint64), ("hbm_budget", ctypes.c_uint64),
                ("hierarchies_built", ctypes.c_uint64), ("hierarchies_reused", ctypes.c_uint64),
                ("map_rebuilds", ctypes.c_uint64), ("evictions", ctypes.c_uint64)]


_lib = None


class CpsError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


def lib():
    """The loaded library (raises if libcps.so is missing)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -m paper_2305_17875_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        P, I, D = ctypes.c_void_p, ctypes.c_int32, ctypes.c_double
        L.cps_grid_default.argtypes = [P]
        L.cps_grid_default.restype = None
        L.cps_last_error.restype = ctypes.c_char_p
        L.cps_setup.argtypes = [P, P, P, ctypes.POINTER(P)]
        L.cps_setup.restype = I
        L.cps_solve.argtypes = [P, P, P, D, P]
        L.cps_solve.restype = I
        L.cps_destroy.argtypes = [P]
        L.cps_destroy.restype = None
        L.cps_levels.argtypes = [P, P, P, P, P]
        L.cps_levels.restype = I
        L.cps_debug_metrics.argtypes = [P, I, P]
        L.cps_debug_apply.argtypes = [P, I, P, P]
        L.cps_debug_residual.argtypes = [P, I, P, P, P, P]
        L.cps_debug_gs_pass.argtypes = [P, I, I, P, P]
        L.cps_debug_restrict.argtypes = [P, I, P, P]
        L.cps_debug_residual_restrict.argtypes = [P, I, P, P, P]
        L.cps_debug_prolong.argtypes = [P, I, P, P]
        L.cps_debug_coarse_solve.argtypes = [P, P, P]
        L.cps_debug_vcycle.argtypes = [P, P, P]
        L.cps_debug_plane_sweep.argtypes = [P, I, I, P, P]
        L.cps_batch_setup.argtypes = [I, P, P, P, ctypes.POINTER(P)]
        L.cps_batch_setup.restype = I
        L.cps_batch_solve.argtypes = [P, P, P, D, P]
        L.cps_batch_solve.restype = I
        L.cps_batch_destroy.argtypes = [P]
        L.cps_batch_destroy.restype = None
        L.cps_service_create.argtypes = [ctypes.c_size_t, I, P, ctypes.POINTER(P)]
        L.cps_service_create.restype = I
        L.cps_service_submit.argtypes = [P, P, P, P, P, D, ctypes.POINTER(ctypes.c_uint64)]
        L.cps_service_submit.restype = I
        L.cps_service_wait.argtypes = [P, ctypes.c_uint64, P]
        L.cps_service_wait.restype = I
        L.cps_service_footprint.argtypes = [P, P, ctypes.POINTER(ctypes.c_uint64)]
        L.cps_service_footprint.restype = I
        L.cps_service_stats.argtypes = [P, P]
        L.cps_service_stats.restype = I
        L.cps_service_destroy.argtypes = [P]
        L.cps_service_destroy.restype = None
        L.cps_profile_enable.argtypes = [P, I]
        L.cps_profile_select.argtypes = [P, ctypes.c_uint32]
        L.cps_profile_read.argtypes = [P, I, P, P]
        L.cps_debug_copy.argtypes = [P, P, ctypes.c_int64, P]
        L.cps_time_vcycle.argtypes = [P, I, I, P, P]
        L.cps_divergence.argtypes = [P, P, P]
        L.cps_correct.argtypes = [P, P, P]
        L.cps_project.argtypes = [P, P, P, D, P]
        L.cps_line_solve.argtypes = [P, I, D, P, P, P]
        L.cps_line_solve_noalloc.argtypes = [P, I, D, P, P, P]
        for f in ("cps_divergence", "cps_correct", "cps_project", "cps_line_solve",
                  "cps_line_solve_noalloc",
                  "cps_profile_select", "cps_profile_enable", "cps_profile_read", "cps_debug_copy",
                  "cps_time_vcycle",
                  "cps_debug_metrics", "cps_debug_apply", "cps_debug_residual",
                  "cps_debug_gs_pass", "cps_debug_restrict", "cps_debug_residual_restrict",
                  "cps_debug_prolong",
                  "cps_debug_coarse_solve", "cps_debug_vcycle", "cps_debug_plane_sweep"):
            getattr(L, f).restype = I
        _lib = L
    return _lib


def last_error() -> str:
    return lib().cps_last_error().decode()


def _check(st: int):
    if st != CPS_OK:
        raise CpsError(st, last_error())


def _ptr(t) -> int:
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda or not t.is_contiguous():
        raise ValueError("expected a contiguous device tensor")
    return t.data_ptr()


def make_grid(g, n_levels: int = 0) -> cps_grid:
    """A cps_grid from any object with the shell attributes (inputs.Shell)."""
    c = cps_grid()
    lib().cps_grid_default(ctypes.byref(c))
    c.n_r, c.n_theta, c.n_phi = g.n_r, g.n_theta, g.n_phi
    c.map = g.map
    c.r_inner, c.r_outer = g.r_inner, g.r_outer
    c.theta0, c.theta1 = g.theta0, g.theta1
    c.radial_stretch = g.radial_stretch
    c.flattening, c.skew = g.flattening, g.skew
    c.n_levels = n_levels
    return c


def cps_setup(grid: cps_grid, metrics: cps_metrics, opts: cps_opts) -> ctypes.c_void_p:
    h = ctypes.c_void_p()
    _check(lib().cps_setup(ctypes.byref(grid), ctypes.byref(metrics), ctypes.byref(opts),
                           ctypes.byref(h)))
    return h


def cps_solve(h, rhs, p, tol: float):
    """Returns (status, cps_info); status CPS_E_NOT_CONVERGED is returned,
    every other error raises."""
    _, n = _dims(h, 0)
    _expect(rhs, n, "rhs"); _expect(p, n, "p")
    info = cps_info()
    st = lib().cps_solve(h, _ptr(rhs), _ptr(p), tol, ctypes.byref(info))
    if st not in (CPS_OK, CPS_E_NOT_CONVERGED, CPS_E_DIVERGED):
        _check(st)
    return st, info


def cps_divergence(h, u, rhs):
    """rhs = d/ds_j [C_ji u_i] (u: 3 x cells, rhs: cells; device FP64)."""
    _, n = _dims(h, 0)
    _expect(u, 3 * n, "u"); _expect(rhs, n, "rhs")
    _check(lib().cps_divergence(h, _ptr(u), _ptr(rhs)))


def cps_correct(h, phi, u):
    """u_i -= (1/|J^-1|) d/ds_j [C_ji phi] in place."""
    _, n = _dims(h, 0)
    _expect(phi, n, "phi"); _expect(u, 3 * n, "u")
    _check(lib().cps_correct(h, _ptr(phi), _ptr(u)))


def cps_project(h, u, phi, tol: float):
    """Divergence, solve, correction; returns (status, cps_info) like
    cps_solve (u is corrected only when the solve converged)."""
    _, n = _dims(h, 0)
    _expect(u, 3 * n, "u"); _expect(phi, n, "phi")
    info = cps_info()
    st = lib().cps_project(h, _ptr(u), _ptr(phi), tol, ctypes.byref(info))
    if st not in (CPS_OK, CPS_E_NOT_CONVERGED, CPS_E_DIVERGED):
        _check(st)
    return st, info


class cps_line_bc(ctypes.Structure):
    _fields_ = [("type_lo", ctypes.c_int32), ("type_hi", ctypes.c_int32),
                ("value_lo", ctypes.c_double), ("value_hi", ctypes.c_double)]


def cps_line_solve(h, d: int, coef: float, rhs, psi, bc=(0, 0.0, 0, 0.0)):
    """One ADI direction's implicit line solves (bc = (type_lo, value_lo,
    type_hi, value_hi)); rhs and psi may be the same tensor."""
    _, n = _dims(h, 0)
    _expect(rhs, n, "rhs"); _expect(psi, n, "psi")
    b = cps_line_bc(bc[0], bc[2], bc[1], bc[3])
    _check(lib().cps_line_solve(h, d, coef, ctypes.byref(b), _ptr(rhs), _ptr(psi)))


def cps_line_solve_noalloc(h, d: int, coef: float, rhs, psi, bc=(0, 0.0, 0, 0.0)):
    """cps_line_solve without allocation: its tables are formed on every
    call in the library's fixed device array (kernel launches only)."""
    _, n = _dims(h, 0)
    _expect(rhs, n, "rhs"); _expect(psi, n, "psi")
    b = cps_line_bc(bc[0], bc[2], bc[1], bc[3])
    _check(lib().cps_line_solve_noalloc(h, d, coef, ctypes.byref(b), _ptr(rhs), _ptr(psi)))


def cps_destroy(h):
    if h:
        lib().cps_destroy(h)


def cps_levels(h):
    nl = ctypes.c_int32()
    dims = (ctypes.c_int32 * 48)()
    nc = ctypes.c_int32()
    axi = ctypes.c_int32()
    _check(lib().cps_levels(h, ctypes.byref(nl), dims, ctypes.byref(nc), ctypes.byref(axi)))
    return [tuple(dims[3 * l:3 * l + 3]) for l in range(nl.value)], nc.value, bool(axi.value)


def _dims(h, level):
    levels, _, _ = cps_levels(h)
    if not 0 <= level < len(levels):
        raise ValueError(f"level {level} out of range")
    return levels, levels[level][0] * levels[level][1] * levels[level][2]


def _expect(t, n, what):
    import torch
    if t.dtype != torch.float64 or t.numel() != n:
        raise ValueError(f"{what}: expected {n} float64 values, got {t.numel()} {t.dtype}")


def cps_debug_metrics(h, level, G_out):
    _, n = _dims(h, level)
    _expect(G_out, 9 * n, "G_out")
    _check(lib().cps_debug_metrics(h, level, _ptr(G_out)))


def cps_debug_apply(h, level, x, y):
    _, n = _dims(h, level)
    _expect(x, n, "x"); _expect(y, n, "y")
    _check(lib().cps_debug_apply(h, level, _ptr(x), _ptr(y)))


def cps_debug_residual(h, level, b, x, r) -> float:
    _, n = _dims(h, level)
    for t, w in ((b, "b"), (x, "x"), (r, "r")):
        _expect(t, n, w)
    n2 = ctypes.c_double()
    _check(lib().cps_debug_residual(h, level, _ptr(b), _ptr(x), _ptr(r), ctypes.byref(n2)))
    return n2.value


def cps_debug_gs_pass(h, level, colour, b, x):
    _, n = _dims(h, level)
    _expect(b, n, "b"); _expect(x, n, "x")
    _check(lib().cps_debug_gs_pass(h, level, colour, _ptr(b), _ptr(x)))


def cps_debug_restrict(h, level, r, bc):
    levels, n = _dims(h, level)
    if level + 1 >= len(levels):
        raise ValueError("no coarser level")
    _expect(r, n, "r"); _expect(bc, n // 8, "bc")
    _check(lib().cps_debug_restrict(h, level, _ptr(r), _ptr(bc)))


def cps_debug_residual_restrict(h, level, b, x, bc):
    """bc = P^T r, r = b - A x on the red cells of level `level` and 0 on
    its black cells: the FP64 V-cycle's transfer after red-black smoothing."""
    levels, n = _dims(h, level)
    if level + 1 >= len(levels):
        raise ValueError("no coarser level")
    nc = math.prod(levels[level + 1])
    _expect(b, n, "b"); _expect(x, n, "x"); _expect(bc, nc, "bc")
    _check(lib().cps_debug_residual_restrict(h, level, _ptr(b), _ptr(x), _ptr(bc)))


def cps_debug_prolong(h, level, e, x):
    levels, n = _dims(h, level)
    if level + 1 >= len(levels):
        raise ValueError("no coarser level")
    _expect(e, n // 8, "e"); _expect(x, n, "x")
    _check(lib().cps_debug_prolong(h, level, _ptr(e), _ptr(x)))


def cps_debug_coarse_solve(h, b, e):
    levels, _ = _dims(h, 0)
    nc = levels[-1][0] * levels[-1][1] * levels[-1][2]
    _expect(b, nc, "b"); _expect(e, nc, "e")
    _check(lib().cps_debug_coarse_solve(h, _ptr(b), _ptr(e)))


def cps_debug_plane_sweep(h, level, parity, b, x):
    _, n = _dims(h, level)
    _expect(b, n, "b"); _expect(x, n, "x")
    _check(lib().cps_debug_plane_sweep(h, level, parity, _ptr(b), _ptr(x)))


def cps_debug_vcycle(h, b, x):
    _, n = _dims(h, 0)
    _expect(b, n, "b"); _expect(x, n, "x")
    _check(lib().cps_debug_vcycle(h, _ptr(b), _ptr(x)))


KERNEL_GS, KERNEL_RESIDUAL, KERNEL_APPLY, KERNEL_RESTRICT, KERNEL_PROLONG, KERNEL_VCYCLE, \
    KERNEL_DIVERGENCE, KERNEL_CORRECT = range(8)


def cps_profile_enable(h, enable: bool):
    _check(lib().cps_profile_enable(h, 1 if enable else 0))


def cps_profile_select(h, classes=None):
    """Record only these kernel classes (None: all)."""
    mask = 0xFFFFFFFF if classes is None else sum(1 << c for c in classes)
    _check(lib().cps_profile_select(h, mask))


def cps_profile_read(h, kernel_class: int):
    """(total_ms, launches) recorded for the class since the last read."""
    ms = ctypes.c_double()
    n = ctypes.c_int64()
    _check(lib().cps_profile_read(h, kernel_class, ctypes.byref(ms), ctypes.byref(n)))
    return ms.value, n.value


def cps_time_vcycle(h, cycles: int, reps: int):
    """(microseconds, kernel launches) per preconditioning V-cycle, replayed
    from a hipGraph of `cycles` cycles, `reps` launches timed with events."""
    us = ctypes.c_double()
    n = ctypes.c_int64()
    _check(lib().cps_time_vcycle(h, int(cycles), int(reps), ctypes.byref(us), ctypes.byref(n)))
    return us.value, n.value


def cps_debug_copy(src, dst, stream=None):
    if src.numel() != dst.numel():
        raise ValueError("size mismatch")
    _expect(src, src.numel(), "src")
    _expect(dst, src.numel(), "dst")
    st = ctypes.c_void_p(stream.cuda_stream) if stream is not None else None
    _check(lib().cps_debug_copy(_ptr(src), _ptr(dst), src.numel(), st))


@dataclass
class Result:
    p: object
    status: int
    iterations: int
    rel_residual: float
    rhs_mean_removed: float
    seconds: float


class Solver:
    """One hierarchy on the current device (owns a cps_handle)."""

    def __init__(self, grid, precision: int = 0, accel: int = 1, max_iters: int = 200,
                 metrics: int = METRICS_MAP_CENTRAL, n_levels: int = 0, stream=None,
                 tune: int = 0, eager: bool = False, smoother: int = 0, face_G=None):
        """face_G: the caller's own finest-level face metrics, a host float64
        array of shape (9, n_r, n_theta, n_phi) (metrics = METRICS_USER_FACE);
        read during set-up only."""
        import numpy as np
        import torch
        self.shape = (grid.n_r, grid.n_theta, grid.n_phi)
        s = stream if stream is not None else torch.cuda.current_stream()
        self.stream = s
        opts = cps_opts(precision, max_iters, accel, tune, 1 if eager else 0, smoother,
                        ctypes.c_void_p(s.cuda_stream))
        met = cps_metrics(metrics)
        if face_G is not None:
            fg = np.ascontiguousarray(face_G, dtype=np.float64)
            if fg.shape != (9,) + self.shape:
                raise ValueError(f"face_G must have shape {(9,) + self.shape}")
            met = cps_metrics(METRICS_USER_FACE, fg.ctypes.data_as(ctypes.c_void_p))
        self.h = cps_setup(make_grid(grid, n_levels), met, opts)
        self.levels, self.ncolours, self.phi_invariant = cps_levels(self.h)

    def _enter(self, *tensors):
        """The library runs on self.stream: order it after the work the
        caller's current stream has queued (which may still be writing the
        inputs), and tell torch's caching allocator that the tensors are in
        use on self.stream, so their memory is not handed out again before
        the library is done with it."""
        import torch
        cur = torch.cuda.current_stream()
        if cur != self.stream:
            self.stream.wait_stream(cur)
            for t in tensors:
                t.record_stream(self.stream)
        return cur

    def _leave(self, cur):
        """Later work on the caller's stream sees the library's results."""
        if cur != self.stream:
            cur.wait_stream(self.stream)

    def time_vcycle(self, cycles: int = 10, reps: int = 5):
        """(microseconds, kernel launches) per V-cycle as the solve replays
        it (cps_time_vcycle)."""
        cur = self._enter()
        try:
            return cps_time_vcycle(self.h, cycles, reps)
        finally:
            self._leave(cur)

    def solve(self, rhs, tol: float = 1e-10, out=None) -> Result:
        import torch
        p = out if out is not None else torch.empty_like(rhs)
        cur = self._enter(rhs, p)
        st, info = cps_solve(self.h, rhs, p, tol)
        self._leave(cur)
        return Result(p, st, info.iterations, info.rel_residual, info.rhs_mean_removed,
                      info.seconds)

    def divergence(self, u, out=None):
        """Right-hand side of eq. (PC_6) for the velocity u (3 x cells)."""
        import torch
        rhs = out if out is not None else torch.empty(u.numel() // 3, dtype=u.dtype,
                                                      device=u.device)
        cur = self._enter(u, rhs)
        cps_divergence(self.h, u, rhs)
        self._leave(cur)
        return rhs

    def correct(self, phi, u):
        """eq. (PC_7) in place on u."""
        cur = self._enter(phi, u)
        cps_correct(self.h, phi, u)
        self._leave(cur)
        return u

    def project(self, u, tol: float = 1e-10, phi=None) -> Result:
        """One projection step on u in place; Result.p is phi."""
        import torch
        phi = phi if phi is not None else torch.empty(u.numel() // 3, dtype=u.dtype,
                                                      device=u.device)
        cur = self._enter(u, phi)
        st, info = cps_project(self.h, u, phi, tol)
        self._leave(cur)
        return Result(phi, st, info.iterations, info.rel_residual, info.rhs_mean_removed,
                      info.seconds)

    def line_solve(self, d: int, coef: float, rhs, bc=(0, 0.0, 0, 0.0), out=None):
        """Implicit line solves along direction d (0 r, 1 theta, 2 phi)."""
        import torch
        psi = out if out is not None else torch.empty_like(rhs)
        cur = self._enter(rhs, psi)
        cps_line_solve(self.h, d, coef, rhs, psi, bc)
        self._leave(cur)
        return psi

    def close(self):
        if getattr(self, "h", None):
            cps_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def cps_batch_setup(grids, metrics: cps_metrics, opts: cps_opts):
    arr = (cps_grid * len(grids))(*grids)
    h = ctypes.c_void_p()
    _check(lib().cps_batch_setup(len(grids), arr, ctypes.byref(metrics), ctypes.byref(opts),
                                 ctypes.byref(h)))
    return h


def cps_batch_solve(h, rhs_list, p_list, sizes, tol: float):
    """rhs_list / p_list: device tensors (checked against sizes).  Returns
    (status, [cps_info])."""
    n = len(rhs_list)
    if len(p_list) != n or len(sizes) != n:
        raise ValueError("one rhs and one p per problem")
    for r, p, s in zip(rhs_list, p_list, sizes):
        _expect(r, s, "rhs")
        _expect(p, s, "p")
    rp = (ctypes.c_void_p * n)(*[_ptr(t) for t in rhs_list])
    pp = (ctypes.c_void_p * n)(*[_ptr(t) for t in p_list])
    infos = (cps_info * n)()
    st = lib().cps_batch_solve(h, rp, pp, tol, infos)
    if st not in (CPS_OK, CPS_E_NOT_CONVERGED, CPS_E_DIVERGED):
        _check(st)
    return st, list(infos)


def cps_batch_destroy(h):
    if h:
        lib().cps_batch_destroy(h)


class Batch:
    """Many problems solved together (FP32 V-cycles inside FP64 refinement)."""

    def __init__(self, grids, max_iters: int = 200, metrics: int = METRICS_MAP_CENTRAL,
                 stream=None, tune: int = 0, smoother: int = 0):
        import torch
        self.grids = list(grids)
        self.sizes = [g.n_r * g.n_theta * g.n_phi for g in self.grids]
        s = stream if stream is not None else torch.cuda.current_stream()
        opts = cps_opts(1, max_iters, 1, tune, 0, smoother, ctypes.c_void_p(s.cuda_stream))
        self.h = cps_batch_setup([make_grid(g) for g in self.grids], cps_metrics(metrics), opts)

    def solve(self, rhs_list, tol: float = 1e-10, out=None):
        import torch
        p = out if out is not None else [torch.empty_like(r) for r in rhs_list]
        # the batch may run on its own stream: inputs must be complete
        torch.cuda.current_stream().synchronize()
        st, infos = cps_batch_solve(self.h, rhs_list, p, self.sizes, tol)
        return st, p, infos

    def close(self):
        if getattr(self, "h", None):
            cps_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---- solve service (host arrays in and out) -------------------------------

def cps_service_create(hbm_budget_bytes: int, max_slots: int, opts: cps_opts):
    h = ctypes.c_void_p()
    _check(lib().cps_service_create(hbm_budget_bytes, max_slots, ctypes.byref(opts),
                                    ctypes.byref(h)))
    return h


def _host_f64(a, n, what):
    import numpy as np
    if not isinstance(a, np.ndarray) or a.dtype != np.float64 or not a.flags.c_contiguous:
        raise ValueError(f"{what}: expected a C-contiguous float64 numpy array")
    if a.size != n:
        raise ValueError(f"{what}: {a.size} elements, expected {n}")
    return a.ctypes.data


def cps_service_submit(h, grid: cps_grid, metrics: cps_metrics, rhs, p, tol: float) -> int:
    """rhs, p: host float64 arrays the caller keeps alive and untouched until
    the ticket's wait returns."""
    n = grid.n_r * grid.n_theta * grid.n_phi
    t = ctypes.c_uint64()
    _check(lib().cps_service_submit(h, ctypes.byref(grid), ctypes.byref(metrics),
                                    _host_f64(rhs, n, "rhs"), _host_f64(p, n, "p"), tol,
                                    ctypes.byref(t)))
    return t.value


def cps_service_wait(h, ticket: int):
    """Blocks (without the GIL) until the request ends.  Returns (status,
    cps_info); raises for argument and device errors."""
    info = cps_info()
    st = lib().cps_service_wait(h, ticket, ctypes.byref(info))
    if st not in (CPS_OK, CPS_E_NOT_CONVERGED, CPS_E_DIVERGED):
        _check(st)
    return st, info


def cps_service_footprint(grid: cps_grid, opts: cps_opts) -> int:
    b = ctypes.c_uint64()
    _check(lib().cps_service_footprint(ctypes.byref(grid), ctypes.byref(opts), ctypes.byref(b)))
    return b.value


def cps_service_stats(h) -> dict:
    r = cps_service_report()
    _check(lib().cps_service_stats(h, ctypes.byref(r)))
    return {k: getattr(r, k) for k, _ in cps_service_report._fields_}


def cps_service_destroy(h):
    if h:
        lib().cps_service_destroy(h)


class Service:
    """Continuous solve service on the current device: submit() queues a
    request and returns its ticket; wait() returns (status, p, info)."""

    def __init__(self, hbm_budget_bytes: int, max_slots: int = 4, precision: int = 1,
                 accel: int = 1, max_iters: int = 200, tune: int = 0, smoother: int = 0):
        self.opts = cps_opts(precision, max_iters, accel, tune, 0, smoother, None)
        self.h = cps_service_create(int(hbm_budget_bytes), max_slots, self.opts)
        self._held = {}  # ticket -> (rhs, p): alive until the wait returns

    def submit(self, grid, rhs, tol: float = 1e-10, metrics: int = METRICS_MAP_CENTRAL,
               n_levels: int = 0, out=None) -> int:
        import numpy as np
        rhs = np.ascontiguousarray(rhs, dtype=np.float64)
        p = out if out is not None else np.empty(rhs.shape, dtype=np.float64)
        t = cps_service_submit(self.h, make_grid(grid, n_levels), cps_metrics(metrics), rhs, p,
                               tol)
        self._held[t] = (rhs, p)
        return t

    def wait(self, ticket: int):
        try:
            st, info = cps_service_wait(self.h, ticket)
        finally:
            held = self._held.pop(ticket, None)
        return st, held[1], info

    def stats(self) -> dict:
        return cps_service_stats(self.h)

    def footprint(self, grid, n_levels: int = 0) -> int:
        return cps_service_footprint(make_grid(grid, n_levels), self.opts)

    def close(self):
        if getattr(self, "h", None):
            cps_service_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
