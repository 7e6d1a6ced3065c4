"""Sequential backward-Euler time stepping with a sparse direct solve (oracle).

TEST INFRASTRUCTURE ONLY (see the package docstring).

This is the trajectory that the inverted iteration converges to: Alg. 3 with a
single thread is exactly backward Euler (Sec. 3.2), and for any convergent fixed
linear preconditioner the inverted iteration's fixed point solves every step
equation AA X^n = A' X^{n-1} + f^n of eq. (fullysystem) exactly.

Solve method (needed for a reference accurate to far below 1e-8):
  * homogeneous or prescribed Dirichlet values are eliminated (the reduced
    matrix is AA restricted to the free dofs);
  * symmetric diagonal scaling D = |diag AA|^{-1/2};
  * SuperLU of D AA D with a symmetric fill-reducing ordering and no pivoting.
    AA is symmetric quasi-definite ([A B; B' -S] with A and S positive definite
    once the Dirichlet dofs are removed), so every symmetric permutation has a
    stable LDL'-type factorization and diagonal pivots suffice;
  * one step of iterative refinement per time step.
AA does not change between steps, so it is factored once.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import fem


class StepSolver:
    """Factorization of the reduced step matrix; solves AA_ff x = rhs_f."""

    def __init__(self, AA: sp.csr_matrix, free: np.ndarray):
        K = AA[free][:, free].tocsc()
        d = np.abs(K.diagonal())
        if np.any(d == 0):
            raise ValueError("zero diagonal in the reduced step matrix")
        self.D = 1.0 / np.sqrt(d)
        Ds = sp.diags(self.D)
        M = (Ds @ K @ Ds).tocsc()
        self.K = K.tocsr()
        self.lu = spla.splu(M, permc_spec="MMD_AT_PLUS_A", diag_pivot_thresh=0.0,
                            options=dict(SymmetricMode=True))

    def solve(self, rhs: np.ndarray, refine: int = 1) -> np.ndarray:
        x = self.D * self.lu.solve(self.D * rhs)
        for _ in range(refine):
            r = rhs - self.K @ x
            x = x + self.D * self.lu.solve(self.D * r)
        return x


class BiotOracle:
    """Assembled Biot problem: step matrix, coupling, loads and boundary data."""

    def __init__(self, problem, asm: fem.Assembled | None = None):
        self.problem = problem
        self.dim = problem.dim
        self.n_nodes = problem.n_nodes
        self.tau = float(problem.dt)
        self.asm = fem.assemble(problem) if asm is None else asm
        self.AA, self.Ap = fem.block_system(self.asm, self.tau)
        self.fixed = fem.dirichlet_mask(problem)
        self.free = np.nonzero(~self.fixed)[0]
        nU = self.n_nodes * self.dim
        F = fem.traction_load(problem)
        self.F_unit = np.concatenate([F, np.zeros(self.n_nodes)])   # [F; 0], field-major
        self.nU = nU
        self._step = None
        # general right-hand side (Sec. 2.2, f^n = [F^n; -tau G^n]): assembled
        # load terms with per-step multipliers, prescribed values of the flagged
        # dofs as terms with per-step multipliers, and the initial state
        to_fm = fem.node_to_field_major
        self.terms = None if getattr(problem, "terms", None) is None else to_fm(problem.terms)
        self.pres = None
        if getattr(problem, "prescribed", None) is not None:
            self.pres = to_fm(problem.prescribed) * self.fixed[None, :]
        self.x0 = None if getattr(problem, "x0", None) is None else to_fm(problem.x0)

    @property
    def n_dof(self) -> int:
        return self.AA.shape[0]

    def load(self, n: int) -> np.ndarray:
        """f^n = [F^n; -tau G^n]: the traction times its multiplier plus the
        assembled terms times theirs (G = 0 for the consolidation column)."""
        f = self.problem.load_coef[n] * self.F_unit
        if self.terms is not None:
            f = f + self.problem.term_coef[n] @ self.terms
        return f

    def prescribed(self, n: int) -> np.ndarray:
        """g^n at the prescribed dofs, zero elsewhere (field-major)."""
        if self.pres is None:
            return np.zeros(self.n_dof)
        return self.problem.prescribed_coef[n] @ self.pres

    def initial_state(self) -> np.ndarray:
        """X^0: the problem's initial state, else g^0 at the prescribed dofs."""
        return self.x0.copy() if self.x0 is not None else self.prescribed(0)

    def free_part(self, X: np.ndarray) -> np.ndarray:
        Y = X.copy()
        Y[..., self.fixed] = 0.0
        return Y

    def step_solver(self) -> StepSolver:
        if self._step is None:
            self._step = StepSolver(self.AA, self.free)
        return self._step

    def rhs(self, n: int, X_prev: np.ndarray) -> np.ndarray:
        """Right-hand side of step n's equation for the free dofs, with the
        prescribed values g^n moved over: b^n = A' X^{n-1} + f^n - AA g^n,
        prescribed rows cleared.  (X^{n-1} carries g^{n-1}.)"""
        b = self.Ap @ X_prev + self.load(n)
        if self.pres is not None:
            b = b - self.AA @ self.prescribed(n)
        b[self.fixed] = 0.0
        return b

    def solve_sequential(self, X0: np.ndarray | None = None, n_steps: int | None = None,
                         refine: int = 1) -> np.ndarray:
        """Backward-Euler trajectory, field-major [n_steps+1, n_dof], with the
        prescribed values g^n at the prescribed dofs of every step n >= 1."""
        N = self.problem.n_steps if n_steps is None else n_steps
        X = np.zeros((N + 1, self.n_dof))
        X[0] = self.initial_state() if X0 is None else X0
        st = self.step_solver()
        for n in range(1, N + 1):
            b = self.rhs(n, X[n - 1])
            X[n] = self.prescribed(n)
            X[n, self.free] = st.solve(b[self.free], refine=refine)
        return X

    def trajectory_node_major(self, X: np.ndarray) -> np.ndarray:
        return fem.field_to_node_major(X, self.n_nodes, self.dim)

    def space_time_residual(self, X: np.ndarray):
        """R^n = A' X^{n-1} + f^n - AA X^n for n >= 1 (prescribed rows zero;
        X^n carries g^n at the prescribed dofs)."""
        N = X.shape[0] - 1
        R = np.zeros((N, self.n_dof))
        for n in range(1, N + 1):
            R[n - 1] = self.rhs(n, X[n - 1]) - self.AA @ self.free_part(X[n])
            R[n - 1, self.fixed] = 0.0
        return R


def relative_field_errors(X: np.ndarray, X_ref: np.ndarray, n_nodes: int, dim: int):
    """Per-field error max_n ||Y^n - Y_ref^n||_2 / max_n ||Y_ref^n||_2, Y in {U, P}
    (field-major trajectories)."""
    nU = n_nodes * dim
    out = {}
    for name, sl in (("u", slice(0, nU)), ("p", slice(nU, nU + n_nodes))):
        num = np.max(np.linalg.norm(X[:, sl] - X_ref[:, sl], axis=1))
        den = np.max(np.linalg.norm(X_ref[:, sl], axis=1))
        out[name] = num / den if den > 0 else num
    return out
