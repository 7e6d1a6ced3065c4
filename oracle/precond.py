"""Block preconditioners of Sec. 3.1 (oracle).

TEST INFRASTRUCTURE ONLY (see the package docstring).

    P1 = [A   0   ]        P2 = [A   0   ]        S_p = (tau + beta/K) C
         [B' -S_p ]             [0  -S_p ]            = tau C_K + C_beta

Applying P1^{-1} to r = [r_u; r_p]:   z_u = A^{-1} r_u,  z_p = S_p^{-1}(B' z_u - r_p).
Applying P2^{-1}:                      z_u = A^{-1} r_u,  z_p = -S_p^{-1} r_p.

The paper does not say how the two inner solves are carried out.  Two choices are
stated here: "exact" (sparse direct) and "gmg" (one multigrid V-cycle of
oracle.gmg for each of A and S_p), the latter being the fixed linear operator
that the device applies.

Prescribed dofs: their rows and columns are removed from A and S_p and replaced
by a unit diagonal, so their entries of z are zero whenever r is zero there.
Vectors are field-major ([u (node*dim+c); p (node)]).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import gmg


def deterministic_start(n: int) -> np.ndarray:
    """Start vector for the spectral-bound power iterations: SplitMix64 of the
    index, mapped to [0.5, 1.5).  (SplitMix64: Steele, Lea and Flood, OOPSLA 2014.)"""
    x = (np.arange(n, dtype=np.uint64) + np.uint64(1)) * np.uint64(0x9E3779B97F4A7C15)
    with np.errstate(over="ignore"):
        z = x.copy()
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        z = z ^ (z >> np.uint64(31))
    return 0.5 + (z >> np.uint64(11)).astype(np.float64) / float(1 << 53)


def power_bound(K: sp.csr_matrix, Dinv: np.ndarray, iters: int = 20) -> float:
    """Rayleigh-quotient estimate of lambda_max(D^{-1} K) after `iters` steps of
    power iteration from the deterministic start vector.  D^{-1}K is
    self-adjoint in the K inner product, hence the quotient x'K y / x'K x."""
    x = deterministic_start(K.shape[0])
    lam = 0.0
    for _ in range(iters):
        Kx = K @ x
        y = gmg.apply_blocks(Dinv, Kx)
        lam = float(y @ Kx) / float(x @ Kx)   # = x'K D^{-1} K x / x'K x
        x = y / np.linalg.norm(y)
    return lam


class BlockPreconditioner:
    """P1 (block lower triangular) or P2 (block diagonal) for one Biot problem."""

    def __init__(self, orc, kind: str = "P1", inner: str = "gmg", degree: int = 2,
                 ratio: float = 4.0, safety: float = 1.1, power_iters: int = 20,
                 pre: int = 1, post: int = 1, min_cells: int = 2):
        if kind not in ("P1", "P2"):
            raise ValueError(kind)
        self.kind = kind
        self.inner = inner
        self.pre, self.post = pre, post
        a = orc.asm
        nU = orc.nU
        self.nU = nU
        fixed = orc.fixed
        self.fu, self.fp = fixed[:nU], fixed[nU:]
        keep_u = sp.diags((~self.fu).astype(np.float64))
        keep_p = sp.diags((~self.fp).astype(np.float64))
        self.A = gmg.apply_fixed(a.A, self.fu)
        self.S = gmg.apply_fixed(orc.tau * a.CK + a.Cb, self.fp)
        self.Bt = (keep_p @ a.B.T @ keep_u).tocsr()
        if inner == "exact":
            la = spla.splu(self.A.tocsc())
            ls = spla.splu(self.S.tocsc())
            self._Ainv, self._Sinv = la.solve, ls.solve
        elif inner == "gmg":
            n = orc.problem.grid_n
            dim = orc.dim
            self.HA = self._hierarchy(self.A, self.fu, n, dim, dim, degree, ratio, safety,
                                      power_iters, min_cells)
            self.HS = self._hierarchy(self.S, self.fp, n, dim, 1, degree, ratio, safety,
                                      power_iters, min_cells)
            self._Ainv = lambda r: gmg.vcycle(self.HA, r, 0, pre, post)
            self._Sinv = lambda r: gmg.vcycle(self.HS, r, 0, pre, post)
        else:
            raise ValueError(inner)

    @staticmethod
    def _hierarchy(K, fixed, n, dim, comps, degree, ratio, safety, power_iters, min_cells):
        H = gmg.build(K, fixed, n, dim, comps, degree=degree, ratio=ratio,
                      min_cells=min_cells, lmax=[1.0] * 64)
        for lev in H.levels[:-1]:
            lev.lmax = safety * power_bound(lev.K, lev.Dinv, power_iters)
        return H

    def apply(self, r: np.ndarray) -> np.ndarray:
        ru, rp = r[: self.nU], r[self.nU:]
        zu = self._Ainv(ru)
        if self.kind == "P1":
            zp = self._Sinv(self.Bt @ zu - rp)
        else:
            zp = self._Sinv(-rp)
        return np.concatenate([zu, zp])
