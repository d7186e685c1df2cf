"""FP64 CPU oracle for the pressure-correction Poisson solve -- TEST INFRASTRUCTURE.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The GPU library never does, and shares
no source with it.

* ``cps_oracle.c`` -- map, face metrics (Sec. 3.2), the nine-term flux-form
  operator of eq. (PC_8)/(PC_term1-3), Gauss-Seidel colour passes, grid
  transfers, dense coarse LU and the multigrid solve of eq. (PC_6).
  It also holds the two steps either side of the solve: the divergence
  right-hand side of eq. (PC_6) and the velocity correction of eq. (PC_7),
  and the implicit line solves of the ADI steps, eq. (solve_2)-(solve_4).
* ``direct.py`` -- exact solves (dense, DCT/FFT on the identity box, rFFT in
  phi with sparse LU per mode on axisymmetric maps) that pin the multigrid.

The C library is compiled with gcc on first use (or by ``build()``).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "cps_oracle.c")
_LIB_DEFAULT = os.path.join(_HERE, "libcps_oracle.so")
_lock = threading.Lock()
_lib = None

MAP_IDENTITY, MAP_SPHERE, MAP_OBLATE, MAP_TRIAXIAL = 0, 1, 2, 3
METRICS_CENTRAL, METRICS_VERTEX = 0, 1


_LIB_NATIVE = os.path.join(_HERE, "libcps_oracle_native.so")


def build(force: bool = True, native: bool = False) -> str:
    """Compile the oracle with gcc (-O2, OpenMP).  Returns the library path.
    native: a second build with -O3 -march=native (the same source, tuned
    for the host it is built on), for timing the oracle as a CPU baseline;
    it is built where it runs, never shipped."""
    lib, opt = (_LIB_NATIVE, ["-O3", "-march=native"]) if native else (_LIB_DEFAULT, ["-O2"])
    if force or not os.path.exists(lib) or os.path.getmtime(lib) < os.path.getmtime(_SRC):
        tmp = lib + ".tmp%d" % os.getpid()
        subprocess.check_call(
            ["gcc", *opt, "-std=c11", "-fopenmp", "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"]
        )
        os.replace(tmp, lib)
    return lib


_native = False


def use_native_build() -> None:
    """Load the -O3 -march=native build (compiled now, on this host) in place
    of the default one.  Must run before the first oracle call."""
    global _native
    with _lock:
        if _lib is not None:
            raise RuntimeError("the oracle library is already loaded")
        build(force=True, native=True)
        _native = True


def set_threads(n: int) -> None:
    """Threads of the oracle's OpenMP loops from now on."""
    _load().orc_set_threads(int(n))


class _Grid(ctypes.Structure):
    _fields_ = [
        ("n_r", ctypes.c_int32), ("n_theta", ctypes.c_int32), ("n_phi", ctypes.c_int32),
        ("map", ctypes.c_int32),
        ("r_inner", ctypes.c_double), ("r_outer", ctypes.c_double),
        ("theta0", ctypes.c_double), ("theta1", ctypes.c_double),
        ("radial_stretch", ctypes.c_double), ("flattening", ctypes.c_double),
        ("skew", ctypes.c_double),
    ]


def _load():
    global _lib
    with _lock:
        if _lib is None:
            lib = ctypes.CDLL(build(force=False, native=_native))
            P = ctypes.c_void_p
            I = ctypes.c_int
            D = ctypes.c_double
            lib.orc_max_threads.restype = I
            lib.orc_set_threads.argtypes = [I]
            lib.orc_set_threads.restype = None
            lib.orc_map.argtypes = [P, D, D, D, P]
            lib.orc_metric_from_chords.argtypes = [P, P]
            lib.orc_metric_from_chords.restype = D
            lib.orc_face_metrics.argtypes = [P, I, I, I, I, P]
            lib.orc_face_metrics.restype = I
            lib.orc_apply.argtypes = [I, I, I, P, P, P]
            lib.orc_residual.argtypes = [I, I, I, P, P, P, P]
            lib.orc_colour.argtypes = [I, I, I, I]
            lib.orc_colour.restype = I
            lib.orc_gs_pass.argtypes = [I, I, I, I, I, P, P, P]
            lib.orc_prolong_add.argtypes = [I, I, I, P, P]
            lib.orc_restrict.argtypes = [I, I, I, P, P]
            lib.orc_dense_matrix.argtypes = [I, I, I, P, P]
            lib.orc_level_plan.argtypes = [I, I, I, I, P]
            lib.orc_level_plan.restype = I
            lib.orc_mg_create.argtypes = [P, I, I, I]
            lib.orc_mg_create.restype = P
            lib.orc_mg_create_user.argtypes = [P, I, I, I, I, I]
            lib.orc_mg_create_user.restype = P
            lib.orc_coarsen_metrics.argtypes = [I, I, I, P, P]
            lib.orc_mg_destroy.argtypes = [P]
            lib.orc_mg_levels.argtypes = [P, P, P]
            lib.orc_mg_levels.restype = I
            lib.orc_mg_metrics.argtypes = [P, I]
            lib.orc_mg_metrics.restype = P
            lib.orc_mg_vcycle.argtypes = [P, P, P]
            lib.orc_mg_coarse_solve.argtypes = [P, P, P]
            lib.orc_mg_solve.argtypes = [P, P, P, D, I, I, P, P, P, P]
            lib.orc_mg_solve.restype = I
            L = ctypes.c_longlong
            lib.orc_face_crow.argtypes = [P, I, I, I, I, I, I, I, I, P]
            lib.orc_face_crow.restype = D
            lib.orc_cell_jdet.argtypes = [P, I, I, I, I, I, I, I]
            lib.orc_cell_jdet.restype = D
            lib.orc_divergence.argtypes = [P, I, I, I, I, P, L, P, P]
            lib.orc_correct.argtypes = [P, I, I, I, I, P, P, L, P, P]
            lib.orc_line_apply.argtypes = [P, I, I, I, I, I, D, I, D, I, D, P, P]
            lib.orc_line_solve.argtypes = [P, I, I, I, I, I, D, I, D, I, D, P, P, L, P]
            lib.orc_line_solve.restype = I
            _lib = lib
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


@dataclass
class Grid:
    """Shell (or box) grid: cells n_r x n_theta x n_phi, phi periodic."""
    n_r: int
    n_theta: int
    n_phi: int
    map: int = MAP_SPHERE
    r_inner: float = 1.5
    r_outer: float = 2.5
    theta0: float = 0.05
    theta1: float = np.pi - 0.05
    radial_stretch: float = 0.0
    flattening: float = 0.0
    skew: float = 0.0

    def c_struct(self) -> _Grid:
        return _Grid(self.n_r, self.n_theta, self.n_phi, self.map, self.r_inner, self.r_outer,
                     self.theta0, self.theta1, self.radial_stretch, self.flattening, self.skew)

    @property
    def shape(self):
        return (self.n_r, self.n_theta, self.n_phi)


def as_grid(g) -> Grid:
    """Accept an oracle Grid or any object with the same attribute names."""
    if isinstance(g, Grid):
        return g
    return Grid(**{k: getattr(g, k) for k in Grid.__dataclass_fields__})


def max_threads() -> int:
    return int(_load().orc_max_threads())


def map_point(grid, sr: float, st: float, sp: float) -> np.ndarray:
    g = as_grid(grid).c_struct()
    X = np.zeros(3)
    _load().orc_map(ctypes.byref(g), sr, st, sp, _p(X))
    return X


def metric_from_chords(t: np.ndarray):
    """t[q] = chord along q; returns (G[3][3], det)."""
    t = _f64(t).reshape(9)
    G = np.zeros(9)
    det = _load().orc_metric_from_chords(_p(t), _p(G))
    return G.reshape(3, 3), det


def face_metrics(grid, shape=None, method: int = METRICS_CENTRAL) -> np.ndarray:
    """G[9, n_r, n_theta, n_phi] of the level with the given dims."""
    g = as_grid(grid)
    nr, nt, np_ = shape or g.shape
    G = np.zeros((9, nr, nt, np_))
    rc = _load().orc_face_metrics(ctypes.byref(g.c_struct()), nr, nt, np_, method, _p(G))
    if rc != 0:
        raise ValueError("non-positive det on an interior face")
    return G


def apply(G: np.ndarray, x: np.ndarray) -> np.ndarray:
    G = _f64(G); x = _f64(x)
    y = np.empty_like(x)
    _load().orc_apply(*x.shape, _p(G), _p(x), _p(y))
    return y


def residual(G, b, x) -> np.ndarray:
    G = _f64(G); b = _f64(b); x = _f64(x)
    r = np.empty_like(x)
    _load().orc_residual(*x.shape, _p(G), _p(b), _p(x), _p(r))
    return r


def colour(ncol: int, a: int, b: int, c: int) -> int:
    return _load().orc_colour(ncol, a, b, c)


def gs_pass(G, b, x, ncol: int, col: int) -> np.ndarray:
    """Returns a new array: x after one Gauss-Seidel pass over colour col."""
    G = _f64(G); b = _f64(b)
    y = _f64(x).copy()
    _load().orc_gs_pass(*y.shape, ncol, col, _p(G), _p(b), _p(y))
    return y


def prolong_add(e, x) -> np.ndarray:
    """x + P e for fine x (new array)."""
    e = _f64(e)
    y = _f64(x).copy()
    _load().orc_prolong_add(*y.shape, _p(e), _p(y))
    return y


def restrict(r) -> np.ndarray:
    r = _f64(r)
    nr, nt, np_ = r.shape
    bc = np.zeros((nr // 2, nt // 2, np_ // 2))
    _load().orc_restrict(nr, nt, np_, _p(r), _p(bc))
    return bc


def coarsen_metrics(G) -> np.ndarray:
    """Face metrics of the next coarser level from a level's [9][n_r][n_t][n_p]
    metrics: each coarse face is half the sum of its four child faces."""
    G = _f64(G)
    nr, nt, np_ = G.shape[1:]
    Gc = np.zeros((9, nr // 2, nt // 2, np_ // 2))
    _load().orc_coarsen_metrics(nr, nt, np_, _p(G), _p(Gc))
    return Gc


def dense_matrix(G) -> np.ndarray:
    G = _f64(G)
    nr, nt, np_ = G.shape[1:]
    n = nr * nt * np_
    A = np.zeros((n, n))
    _load().orc_dense_matrix(nr, nt, np_, _p(G), _p(A))
    return A


def level_plan(nr: int, nt: int, np_: int, n_levels: int = 0):
    dims = np.zeros(48, dtype=np.int32)
    L = _load().orc_level_plan(nr, nt, np_, n_levels, _p(dims))
    if L < 1:
        raise ValueError("no level plan")
    return [tuple(int(v) for v in dims[3 * l:3 * l + 3]) for l in range(L)]


class Multigrid:
    """Oracle multigrid hierarchy for one grid (metrics from the map)."""

    def __init__(self, grid, method: int = METRICS_CENTRAL, n_levels: int = 0, ncol: int = 0,
                 face_G=None):
        """face_G: caller-given level-0 face metrics [9][n_r][n_t][n_p] (the
        low-wall faces taken as zero; coarse levels by coarsen_metrics) in
        place of metrics from the map."""
        self._lib = _load()
        self.grid = as_grid(grid)
        self._g = self.grid.c_struct()
        if face_G is None:
            self._h = self._lib.orc_mg_create(ctypes.byref(self._g), method, n_levels, ncol)
        else:
            self._G0 = _f64(face_G)
            if self._G0.shape != (9,) + self.grid.shape:
                raise ValueError("face_G must be [9][n_r][n_theta][n_phi]")
            self._h = self._lib.orc_mg_create_user(_p(self._G0), *self.grid.shape, n_levels,
                                                   ncol)
        if not self._h:
            raise ValueError("oracle multigrid setup failed")
        dims = np.zeros(48, dtype=np.int32)
        nc = ctypes.c_int(0)
        L = self._lib.orc_mg_levels(self._h, _p(dims), ctypes.byref(nc))
        self.levels = [tuple(int(v) for v in dims[3 * l:3 * l + 3]) for l in range(L)]
        self.ncol = nc.value

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            self._lib.orc_mg_destroy(h)
            self._h = None

    def metrics(self, level: int = 0) -> np.ndarray:
        nr, nt, np_ = self.levels[level]
        ptr = self._lib.orc_mg_metrics(self._h, level)
        buf = (ctypes.c_double * (9 * nr * nt * np_)).from_address(ptr)
        return np.frombuffer(buf, dtype=np.float64).reshape(9, nr, nt, np_).copy()

    def vcycle(self, b, x) -> np.ndarray:
        b = _f64(b)
        y = _f64(x).copy()
        self._lib.orc_mg_vcycle(self._h, _p(b), _p(y))
        return y

    def coarse_solve(self, b) -> np.ndarray:
        b = _f64(b)
        e = np.zeros_like(b)
        self._lib.orc_mg_coarse_solve(self._h, _p(b), _p(e))
        return e

    def solve(self, b, tol: float = 1e-10, max_iters: int = 200, accel: int = 0):
        """Returns (x, status, iterations, rel_residual, history, mean_removed)."""
        b = _f64(b)
        x = np.zeros_like(b)
        it = ctypes.c_int(0)
        rel = ctypes.c_double(0.0)
        mean = ctypes.c_double(0.0)
        hist = np.zeros(max(max_iters, 1))
        st = self._lib.orc_mg_solve(self._h, _p(b), _p(x), tol, max_iters, accel,
                                    ctypes.byref(it), ctypes.byref(rel), _p(hist),
                                    ctypes.byref(mean))
        return x, st, it.value, rel.value, hist[:it.value].copy(), mean.value


# ---------------------------------------------------------------------------
# Projection step: the right-hand side of eq. (PC_6) and eq. (PC_7)
# ---------------------------------------------------------------------------

def face_crow(grid, d: int, a: int, b: int, c: int, method: int = METRICS_CENTRAL):
    """(C_d., |J^-1|) at the LOW d-face of cell (a, b, c); a may be n_r and
    b may be n_theta (the high walls)."""
    g = as_grid(grid)
    C = np.zeros(3)
    det = _load().orc_face_crow(ctypes.byref(g.c_struct()), *g.shape, method, d, a, b, c, _p(C))
    return C, det


def cell_jdet(grid, a: int, b: int, c: int, method: int = METRICS_CENTRAL) -> float:
    """|J^-1| at the cell centre: mean of its six face determinants."""
    g = as_grid(grid)
    return _load().orc_cell_jdet(ctypes.byref(g.c_struct()), *g.shape, method, a, b, c)


def _cells(g, cells):
    if cells is None:
        return 0, None, int(np.prod(g.shape))
    idx = np.ascontiguousarray(cells, dtype=np.int64).ravel()
    return idx, _p(idx), idx.size


def divergence(grid, u, cells=None, method: int = METRICS_CENTRAL) -> np.ndarray:
    """d/ds_j [C_ji u_i] (u: [3, n_r, n_theta, n_phi]) at every cell
    (shape of the grid) or at the listed flat cell indices (1-D)."""
    g = as_grid(grid)
    u = _f64(u).reshape((3,) + g.shape)
    idx, ptr, n = _cells(g, cells)
    out = np.zeros(n)
    _load().orc_divergence(ctypes.byref(g.c_struct()), *g.shape, method, _p(u), n, ptr, _p(out))
    return out.reshape(g.shape) if cells is None else out


def correct(grid, phi, u, cells=None, method: int = METRICS_CENTRAL) -> np.ndarray:
    """u - (1/|J^-1|) d/ds_j [C_ji phi]: [3, n_r, n_theta, n_phi] for every
    cell, or [n, 3] at the listed flat cell indices."""
    g = as_grid(grid)
    u = _f64(u).reshape((3,) + g.shape)
    phi = _f64(phi).reshape(g.shape)
    idx, ptr, n = _cells(g, cells)
    out = np.zeros((n, 3))
    _load().orc_correct(ctypes.byref(g.c_struct()), *g.shape, method, _p(phi), _p(u), n, ptr,
                        _p(out))
    if cells is None:
        return np.moveaxis(out.reshape(g.shape + (3,)), -1, 0).copy()
    return out


def project(grid, u, method: int = METRICS_CENTRAL):
    """The projection step with an exact solve: rhs = d/ds_j [C_ji u_i],
    A phi = rhs - mean(rhs) with mean(phi) = 0 (``direct.solve_axisym`` for
    phi-invariant metrics, else ``direct.solve_sparse``), then eq. (PC_7).
    Returns (u_new, phi, rhs)."""
    from . import direct
    g = as_grid(grid)
    rhs = divergence(g, u, method=method)
    G = face_metrics(g, method=method)
    solve = direct.solve_axisym if direct.is_axisymmetric(G) else direct.solve_sparse
    phi = solve(G, rhs)
    return correct(g, phi, u, method=method), phi, rhs


# ---------------------------------------------------------------------------
# Implicit line solves of the ADI steps, eq. (solve_2)-(solve_4)
# ---------------------------------------------------------------------------

def line_apply(grid, d: int, coef: float, psi, bc=(0, 0.0, 0, 0.0),
               method: int = METRICS_CENTRAL) -> np.ndarray:
    """|J^-1| psi - coef [G_dd (psi_hi - psi_lo)] along direction d, the wall
    fluxes of bc = (type_lo, v_lo, type_hi, v_hi) (type 0 no flux, 1 value v
    on the wall face; phi is periodic)."""
    g = as_grid(grid)
    psi = _f64(psi).reshape(g.shape)
    out = np.zeros(g.shape)
    _load().orc_line_apply(ctypes.byref(g.c_struct()), *g.shape, method, d, coef, bc[0], bc[1],
                           bc[2], bc[3], _p(psi), _p(out))
    return out


def line_solve(grid, d: int, coef: float, rhs, bc=(0, 0.0, 0, 0.0),
               method: int = METRICS_CENTRAL, lines=None) -> np.ndarray:
    """psi with line_apply(psi) = rhs on every line along d: the Thomas
    algorithm, and for the periodic phi-lines the paper's split with a
    closing row.  lines: solve only these line indices (d = 0: b n_phi + c,
    d = 1: a n_phi + c, d = 2: a n_theta + b); psi is zero elsewhere."""
    g = as_grid(grid)
    rhs = _f64(rhs).reshape(g.shape)
    psi = np.zeros(g.shape)
    idx = None if lines is None else np.ascontiguousarray(lines, dtype=np.int64).ravel()
    rc = _load().orc_line_solve(ctypes.byref(g.c_struct()), *g.shape, method, d, coef, bc[0],
                                bc[1], bc[2], bc[3], _p(rhs), _p(psi),
                                0 if idx is None else idx.size,
                                None if idx is None else _p(idx))
    if rc != 0:
        raise ValueError("periodic lines need at least 3 cells")
    return psi
