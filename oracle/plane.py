"""Zebra (r, phi)-plane relaxation and the V-cycle around it -- TEST
INFRASTRUCTURE (see the package docstring).

A block Gauss-Seidel smoother for the 7-point operator with phi-invariant
metrics (orthogonal maps).  The cells of one theta row b form a block: the
(r, phi) plane at that row.  A half-sweep of parity k relaxes every row with
b = k (mod 2) at once -- rows of one parity do not couple, their theta
neighbours are the other parity -- by solving each block exactly with the
other parity held fixed:

    x_B <- A_BB^-1 (b_B - A_B,rest x_rest).

That is the plain definition written out: the blocks come from the sparse
matrix of the flux-form operator (``direct.csr_matrix``) and each is solved
with a sparse LU; no FFT and no tridiagonal algebra, so it pins the GPU's
spectral plane solver.  The smoother treats the theta direction, the weakest
coupling of the shell everywhere, by zebra ordering, and the two strong ones
(r, and phi at the cone tips) exactly.  It is a design of this project, not
of the paper, which solves its implicit lines with the Thomas algorithm
(Sec. on the ADI steps); the r-direction solve here is such a line solve for
every azimuthal mode.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse.linalg as spla

from . import direct
from . import prolong_add, residual, restrict


class PlaneSmoother:
    """Exact block solves of the theta rows of one level."""

    def __init__(self, G: np.ndarray):
        self.shape = G.shape[1:]
        nr, nt, np_ = self.shape
        self.A = direct.csr_matrix(G).tocsr()
        idx = np.arange(nr * nt * np_).reshape(nr, nt, np_)
        self.rows = [idx[:, b, :].ravel() for b in range(nt)]
        self.lu = [spla.splu(self.A[r][:, r].tocsc()) for r in self.rows]

    def half_sweep(self, b: np.ndarray, x: np.ndarray, parity: int) -> np.ndarray:
        """Relax the rows b = parity (mod 2); returns the new x."""
        x = np.array(x, dtype=np.float64, copy=True)
        xf = x.ravel()
        bf = np.asarray(b, dtype=np.float64).ravel()
        nt = self.shape[1]
        old = xf.copy()  # rows of one parity only read the other parity
        for row in range(parity, nt, 2):
            r = self.rows[row]
            rhs = bf[r] - self.A[r] @ old + self.A[r][:, r] @ old[r]
            xf[r] = self.lu[row].solve(rhs)
        return x

    def sweep(self, b, x, reverse: bool = False):
        for parity in ((1, 0) if reverse else (0, 1)):
            x = self.half_sweep(b, x, parity)
        return x


class PlaneMultigrid:
    """V(nu, nu) cycle with zebra plane smoothing on every level above the
    coarsest (post-smoothing in reverse parity order, so the cycle is a
    symmetric preconditioner for a symmetric operator); transfers and the
    coarsest solve are the oracle's multigrid pieces."""

    def __init__(self, mg, nu: int = 2):
        self.mg = mg
        self.nu = nu
        self.L = len(mg.levels)
        self.sm = [PlaneSmoother(mg.metrics(l)) for l in range(self.L - 1)]

    def vcycle(self, b, x, level: int = 0):
        if level == self.L - 1:
            return self.mg.coarse_solve(b)
        G = self.mg.metrics(level)
        for _ in range(self.nu):
            x = self.sm[level].sweep(b, x)
        bc = restrict(residual(G, b, x))
        e = self.vcycle(bc, np.zeros_like(bc), level + 1)
        x = prolong_add(e, x)
        for _ in range(self.nu):
            x = self.sm[level].sweep(b, x, reverse=True)
        return x
