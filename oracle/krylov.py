"""GMRES(k) as the per-unit solver K of Alg. 3 (oracle).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Alg. 3 writes one unit of the inverted iteration as
    X^{n,m} = K(P, AA, X^{n,m-1}, b^{n,m}, n_iter),
K being a Krylov method (the paper uses PETSc's GMRES) preconditioned by P.
Here K is restarted GMRES with left preconditioning (PETSc's default side for
GMRES), k iterations from the previous iterate (Saad, Iterative Methods for
Sparse Linear Systems, the left-preconditioned GMRES algorithm):
r0 = P^{-1}(b - A x0), v_1 = r0/||r0||, Arnoldi on P^{-1} A with modified
Gram-Schmidt, y minimizing ||beta e_1 - H_k y|| (here by numpy's least squares
on the small Hessenberg matrix), x = x0 + V_k y.  It minimizes the
preconditioned residual ||P^{-1}(b - A x)||, which weighs the displacement and
pressure rows (of very different scales) by the preconditioner.

All vectors live on the free (not prescribed) dofs: the operator and the
preconditioner outputs are zeroed on prescribed dofs.
"""
from __future__ import annotations

import numpy as np

from .inverted import norms, step_residual


def gmres_left(apply_A, apply_P, b: np.ndarray, x0: np.ndarray, k: int) -> np.ndarray:
    """k iterations of left-preconditioned GMRES for A x = b from x0."""
    r0 = apply_P(b - apply_A(x0))
    beta = np.linalg.norm(r0)
    if beta == 0.0:
        return x0.copy()
    V = [r0 / beta]
    H = np.zeros((k + 1, k))
    m = k
    for j in range(k):
        w = apply_P(apply_A(V[j]))
        for i in range(j + 1):
            H[i, j] = w @ V[i]
            w = w - H[i, j] * V[i]
        H[j + 1, j] = np.linalg.norm(w)
        if H[j + 1, j] == 0.0:          # the Krylov space is invariant: exact solution
            m = j + 1
            break
        V.append(w / H[j + 1, j])
    e1 = np.zeros(m + 1)
    e1[0] = beta
    y = np.linalg.lstsq(H[: m + 1, :m], e1, rcond=None)[0]
    return x0 + sum(y[j] * V[j] for j in range(m))


class GmresUnit:
    """One unit of Alg. 3 with K = GMRES(k) and the preconditioner `prec`."""

    def __init__(self, orc, prec, k: int):
        self.orc, self.prec, self.k = orc, prec, k

    def _A(self, v):
        w = self.orc.AA @ v
        w[self.orc.fixed] = 0.0
        return w

    def _P(self, r):
        z = self.prec.apply(r)
        z[self.orc.fixed] = 0.0
        return z

    def update(self, n: int, X_prev: np.ndarray, X_cur: np.ndarray):
        """(X^{n,m}, norms of the unit's residual before the update)."""
        b, r = step_residual(self.orc, n, X_prev, X_cur)
        return gmres_left(self._A, self._P, b, X_cur, self.k), norms(self.orc, b, r)


def sweep(orc, X: np.ndarray, unit, order: str = "gauss_seidel"):
    """One outer sweep with `unit` (see inverted.sweep for the orders)."""
    N = X.shape[0] - 1
    Xn = X.copy()
    out = np.zeros((N, 4))
    for n in range(1, N + 1):
        src = Xn[n - 1] if order == "gauss_seidel" else X[n - 1]
        Xn[n], out[n - 1] = unit.update(n, src, X[n])
    return Xn, out


def wavefront(orc, X: np.ndarray, unit, depth: int):
    """`depth` Gauss-Seidel sweeps with `unit`, as the wavefront of Alg. 4."""
    N = X.shape[0] - 1
    it = [X.copy()] + [X.copy() for _ in range(depth)]
    for w in range(1, N + depth):
        for s in range(depth):
            n = w - s
            if 1 <= n <= N:
                it[s + 1][n], _ = unit.update(n, it[s + 1][n - 1], it[s][n])
    return it[depth]
