"""The inverted time-stepping iteration (oracle).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Sec. 3.2, Alg. 2: with zero initial iterates X^{n,0}, for m = 1, 2, ... and
n = 1..N_time,
    b^{n,m} = A' X^{n-1,m} + f^n
    X^{n,m} = X^{n,m-1} + P^{-1}(b^{n,m} - AA X^{n,m-1}).
The step equation's unknown X^{n,m-1} enters the residual; the coupling uses the
previous step's iterate of the *same* sweep m ("gauss_seidel" order: within a
sweep, step n sees step n-1 already updated).  This module also states the order
in which every step of a sweep couples to the previous sweep's value X^{n-1,m-1}
("jacobi"), which updates all steps at once.  Both orders share the fixed point:
the backward-Euler trajectory (Sec. 3.2; a single thread in Alg. 3 is backward
Euler).

A damping factor omega multiplies the preconditioned correction; omega = 1 is the
update as printed.  (With the paper's P1 the undamped update diverges at small
time steps because S_p leaves out B'A^{-1}B; see the design notes.)

Residual norms.  For each step the sweep reports ||r_u||^2, ||r_p||^2,
||b_u||^2, ||b_p||^2 of r = b - AA X^{n,m-1}, with b the coupled right-hand side
used in that update.
"""
from __future__ import annotations

import numpy as np


def step_residual(orc, n: int, X_prev: np.ndarray, X_cur: np.ndarray):
    """b and r = b - AA x of step n's equation on the free dofs (prescribed
    values moved into b; prescribed rows zero)."""
    b = orc.rhs(n, X_prev)
    r = b - orc.AA @ orc.free_part(X_cur)
    r[orc.fixed] = 0.0
    return b, r


def norms(orc, b, r):
    nU = orc.nU
    return np.array([r[:nU] @ r[:nU], r[nU:] @ r[nU:], b[:nU] @ b[:nU], b[nU:] @ b[nU:]])


def sweep(orc, X: np.ndarray, prec, omega: float = 1.0, order: str = "gauss_seidel"):
    """One outer sweep over all steps; returns (X_new, norms [N, 4]).

    X is field-major [N+1, n_dof]; X[0] is the initial state and is not changed.
    """
    N = X.shape[0] - 1
    Xn = X.copy()
    out = np.zeros((N, 4))
    for n in range(1, N + 1):
        src = Xn[n - 1] if order == "gauss_seidel" else X[n - 1]
        b, r = step_residual(orc, n, src, X[n])
        out[n - 1] = norms(orc, b, r)
        Xn[n] = X[n] + omega * prec.apply(r)
    return Xn, out


def wavefront(orc, X: np.ndarray, prec, omega: float, depth: int):
    """`depth` Gauss-Seidel sweeps executed as a wavefront (Alg. 4's schedule).

    At wall step w, slot s (s = 0..depth-1) updates step n = w - s from its
    iterate of sweep s to sweep s+1.  The result equals `depth` calls of
    sweep(..., order="gauss_seidel"); the wavefront is stated separately so the
    device schedule can be compared with it as a schedule.
    """
    N = X.shape[0] - 1
    # iterates[s][n] = value of step n after s sweeps in this pass
    it = [X.copy()] + [X.copy() for _ in range(depth)]
    for w in range(1, N + depth):
        for s in range(depth):
            n = w - s
            if n < 1 or n > N:
                continue
            b, r = step_residual(orc, n, it[s + 1][n - 1], it[s][n])
            it[s + 1][n] = it[s][n] + omega * prec.apply(r)
    return it[depth]


def relative_residual(nrm: np.ndarray, floor: float = 1e-300) -> float:
    """max over fields of max_n ||r^n|| / max_n ||b^n|| (per field).

    A field whose right-hand side is zero at every step (e.g. the pressure rows
    of a single step from a zero initial state) is measured against the whole
    right-hand side instead."""
    ru = np.sqrt(nrm[:, 0].max())
    rp = np.sqrt(nrm[:, 1].max())
    bu = np.sqrt(nrm[:, 2].max())
    bp = np.sqrt(nrm[:, 3].max())
    both = np.sqrt(bu * bu + bp * bp)
    du = bu if bu > 0 else both
    dp = bp if bp > 0 else both
    return max(ru / max(du, floor), rp / max(dp, floor))
