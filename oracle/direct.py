"""Exact solves of eq. (PC_6) -- TEST INFRASTRUCTURE.

The solution of the discrete pressure-correction equation has a plain
definition: the unique x with A x = b and sum(x) = 0 (zero-flux walls make A
singular with the constants as null space, and 1^T A = 0 makes sum(b) = 0 the
solvability condition).  These solvers compute that x directly, without
multigrid, so that they pin the oracle's (and the GPU's) iterative solves:

* ``solve_sparse``   -- any map: sparse matrix (probed from the oracle
  operator) bordered with the constraint row, sparse LU.  Small grids.
* ``solve_axisym``   -- maps that are invariant under rotation about the
  polar axis (sphere, oblate): an rFFT in phi decouples one 2-D (r, theta)
  system per azimuthal mode; each is factored with sparse LU.
* ``solve_identity`` -- the uniform identity box: DCT-II in r and theta,
  DFT in phi, with the eigenvalues written out from the box spacings.
"""
from __future__ import annotations

import numpy as np
import scipy.fft as sfft
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import apply as _apply


def _probe_colours(shape):
    """Colour classes such that no two cells of one class lie in the 3x3x3
    neighbourhood of a common cell (mod 3 in r, theta; mod 4 in phi, or every
    cell its own class along phi when phi has fewer than 4 cells or is not a
    multiple of 4)."""
    nr, nt, np_ = shape
    kp = 4 if np_ % 4 == 0 else np_
    a = np.arange(nr)[:, None, None] % 3
    b = np.arange(nt)[None, :, None] % 3
    c = np.arange(np_)[None, None, :] % kp
    return (a * 3 + b) * kp + c, 9 * kp


def csr_matrix(G: np.ndarray) -> sp.csr_matrix:
    """Sparse A assembled by probing the oracle operator with colour
    indicator fields: for probe k, (A e_k)_i = A_ij for the unique cell j of
    class k inside the stencil of row i."""
    shape = G.shape[1:]
    n = int(np.prod(shape))
    col_of, ncls = _probe_colours(shape)
    col_of = col_of.ravel()
    nr, nt, np_ = shape
    idx = np.arange(n).reshape(shape)
    rows, cols, vals = [], [], []
    # neighbour offsets within the 3x3x3 block (clamped / wrapped)
    offs = [(i, j, k) for i in (-1, 0, 1) for j in (-1, 0, 1) for k in (-1, 0, 1)]
    for cls in range(ncls):
        e = (col_of == cls).astype(np.float64).reshape(shape)
        if not e.any():
            continue
        y = _apply(G, e).ravel()
        # for every row i, find the class-cls cell in its neighbourhood
        seen = np.full(n, -1, dtype=np.int64)
        for (i, j, k) in offs:
            a = np.clip(np.arange(nr) + i, 0, nr - 1)
            b = np.clip(np.arange(nt) + j, 0, nt - 1)
            c = (np.arange(np_) + k) % np_
            nb = idx[a][:, b][:, :, c].ravel()
            hit = (col_of[nb] == cls) & (seen < 0)
            seen[hit] = nb[hit]
        rr = np.nonzero(seen >= 0)[0]
        cc = seen[rr]
        vv = y[rr]
        keep = vv != 0.0
        rows.append(rr[keep]); cols.append(cc[keep]); vals.append(vv[keep])
    A = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(n, n))
    return A


def solve_sparse(G: np.ndarray, b: np.ndarray) -> np.ndarray:
    """x with A x = b - mean(b), sum(x) = 0, via the bordered system
    [[A, 1], [1^T, 0]] [x; lam] = [b; 0] and sparse LU."""
    A = csr_matrix(G)
    n = A.shape[0]
    one = sp.csr_matrix(np.ones((n, 1)))
    K = sp.bmat([[A, one], [one.T, None]], format="csc")
    rhs = np.concatenate([(b - b.mean()).ravel(), [0.0]])
    x = spla.splu(K).solve(rhs)[:n]
    return x.reshape(b.shape)


def _axisym_2d(G: np.ndarray):
    """The (r, theta) part of A on phi-constant fields, probed with 3x3
    colour classes; plus the phi-face metric per (r, theta)."""
    nr, nt, np_ = G.shape[1:]
    n2 = nr * nt
    idx = np.arange(n2).reshape(nr, nt)
    cls2 = (np.arange(nr)[:, None] % 3) * 3 + np.arange(nt)[None, :] % 3
    rows, cols, vals = [], [], []
    for cls in range(9):
        e2 = (cls2 == cls).astype(np.float64)
        if not e2.any():
            continue
        y = _apply(G, np.repeat(e2[:, :, None], np_, axis=2))[:, :, 0].ravel()
        seen = np.full(n2, -1, dtype=np.int64)
        for i in (-1, 0, 1):
            for j in (-1, 0, 1):
                a = np.clip(np.arange(nr) + i, 0, nr - 1)
                b = np.clip(np.arange(nt) + j, 0, nt - 1)
                nb = idx[a][:, b].ravel()
                hit = (cls2.ravel()[nb] == cls) & (seen < 0)
                seen[hit] = nb[hit]
        rr = np.nonzero(seen >= 0)[0]
        keep = y[rr] != 0.0
        rows.append(rr[keep]); cols.append(seen[rr][keep]); vals.append(y[rr][keep])
    A2 = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                       shape=(n2, n2))
    return A2, G[8, :, :, 0].ravel()


def is_axisymmetric(G: np.ndarray, rtol: float = 1e-12) -> bool:
    """Metrics independent of phi and no coupling between phi and r/theta."""
    ref = G[:, :, :, :1]
    scale = np.abs(G).max()
    if np.abs(G - ref).max() > rtol * scale:
        return False
    return not (G[2].any() or G[5].any() or G[6].any() or G[7].any())


def _mode_solve(A2, gpp, rhs: np.ndarray, m: int, np_: int) -> np.ndarray:
    """Azimuthal mode m of the solution: (A_2d - 4 sin^2(pi m / n_phi)
    diag(G_pp)) x_m = b_m by sparse LU; mode 0 bordered with sum(x_0) = 0.
    rhs: the complex mode of b, flattened over (r, theta)."""
    n2 = A2.shape[0]
    if m == 0:
        one = sp.csr_matrix(np.ones((n2, 1)))
        K = sp.bmat([[A2, one], [one.T, None]], format="csc")
        lu = spla.splu(K)
        xr = lu.solve(np.concatenate([rhs.real, [0.0]]))[:n2]
        xi = lu.solve(np.concatenate([rhs.imag, [0.0]]))[:n2]
    else:
        shift = -4.0 * np.sin(np.pi * m / np_) ** 2 * gpp
        lu = spla.splu((A2 + sp.diags(shift)).tocsc())
        xr = lu.solve(np.ascontiguousarray(rhs.real))
        xi = lu.solve(np.ascontiguousarray(rhs.imag))
    return xr + 1j * xi


def _mode_chunk(task):
    """Worker body: the modes of one chunk, as (m, x_m) pairs."""
    A2, gpp, np_, chunk = task
    return [(m, _mode_solve(A2, gpp, rhs, m, np_)) for m, rhs in chunk]


def mode_pool(workers: int):
    """A process pool for solve_axisym (spawned workers: they import numpy and
    scipy only); the caller closes it (use as a context manager)."""
    import concurrent.futures as cf
    import multiprocessing as mp
    return cf.ProcessPoolExecutor(max_workers=workers, mp_context=mp.get_context("spawn"))


def solve_axisym(G: np.ndarray, b: np.ndarray, workers: int = 1, progress=None,
                 pool=None) -> np.ndarray:
    """Exact solve for phi-invariant metrics with G_{r phi} = G_{theta phi} = 0.

    On each azimuthal mode m the phi-flux difference G_pp (x_{c+1} - 2 x_c +
    x_{c-1}) becomes -4 sin^2(pi m / n_phi) G_pp x_m, so A splits into
    (A_2d - 4 sin^2(pi m/n_phi) diag(G_pp)) x_m = b_m.  Mode 0 is singular and
    is solved bordered with sum(x_0) = 0.  The modes are independent systems:
    with workers > 1 (or a pool from mode_pool) they are solved in chunks in
    worker processes, the same arithmetic per mode.  progress(done, total)
    is called as modes finish."""
    if not is_axisymmetric(G):
        raise ValueError("metrics are not axisymmetric")
    nr, nt, np_ = b.shape
    A2, gpp = _axisym_2d(G)
    bh = np.fft.rfft(b - b.mean(), axis=2)
    xh = np.zeros_like(bh)
    nm = bh.shape[2]
    if workers <= 1 and pool is None:
        for m in range(nm):
            xh[:, :, m] = _mode_solve(A2, gpp, bh[:, :, m].ravel(), m, np_).reshape(nr, nt)
            if progress:
                progress(m + 1, nm)
    else:
        ex = pool if pool is not None else mode_pool(workers)
        try:
            nchunk = 4 * (workers if pool is None else ex._max_workers)
            modes = [(m, np.ascontiguousarray(bh[:, :, m].ravel())) for m in range(nm)]
            tasks = [(A2, gpp, np_, modes[k::nchunk]) for k in range(min(nchunk, nm))]
            done = 0
            for res in ex.map(_mode_chunk, tasks):
                for m, xm in res:
                    xh[:, :, m] = xm.reshape(nr, nt)
                done += len(res)
                if progress:
                    progress(done, nm)
        finally:
            if pool is None:
                ex.shutdown()
    x = np.fft.irfft(xh, n=np_, axis=2)
    return x - x.mean()


def solve_identity(grid, b: np.ndarray) -> np.ndarray:
    """Identity box with uniform spacing h_r = (r_o - r_i)/n_r, h_t = (theta1
    - theta0)/n_theta, h_p = 2 pi/n_phi: the face metrics are G_dd = h_u h_v /
    h_d, the operator is the tensor sum of three scaled second differences
    (zero-flux ends in r and theta, periodic in phi), and DCT-II / DFT
    diagonalise it with eigenvalues -G_dd 4 sin^2(pi k / (2 n)) (Neumann) and
    -G_pp 4 sin^2(pi m / n_phi) (periodic)."""
    nr, nt, np_ = b.shape
    hr = (grid.r_outer - grid.r_inner) / nr
    ht = (grid.theta1 - grid.theta0) / nt
    hp = 2.0 * np.pi / np_
    grr, gtt, gpp = ht * hp / hr, hr * hp / ht, hr * ht / hp
    lr = -grr * 4.0 * np.sin(np.pi * np.arange(nr) / (2 * nr)) ** 2
    lt = -gtt * 4.0 * np.sin(np.pi * np.arange(nt) / (2 * nt)) ** 2
    lp = -gpp * 4.0 * np.sin(np.pi * np.arange(np_) / np_) ** 2
    lam = lr[:, None, None] + lt[None, :, None] + lp[None, None, :]
    bh = sfft.fft(sfft.dctn(b - b.mean(), type=2, axes=(0, 1), norm="ortho"), axis=2)
    lam[0, 0, 0] = 1.0
    xh = bh / lam
    xh[0, 0, 0] = 0.0
    x = sfft.idctn(sfft.ifft(xh, axis=2).real, type=2, axes=(0, 1), norm="ortho")
    return x - x.mean()
