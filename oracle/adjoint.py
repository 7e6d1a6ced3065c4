"""Discrete adjoint of the backward-Euler Biot trajectory (oracle).

TEST INFRASTRUCTURE ONLY (see the package docstring).

The forward problem is the fully discrete system of eq. (fullysystem):
    AA X^n = A' X^{n-1} + f^n,   n = 1..N,   X^0 = 0,
with the prescribed (Dirichlet) dofs eliminated.  Stacked over the time steps
this is one block lower-bidiagonal space-time system  calA X = f, whose block
row n holds AA on the diagonal and -A' on the sub-diagonal.

Objective (pressure misfit at sensor nodes s, every step):
    J = sum_{n=1..N} sum_s (p^n_s - d^n_s)^2.

Adjoint.  With the Lagrangian L = J - sum_n Lam^n . (AA X^n - A' X^{n-1} - f^n),
stationarity in X^n gives calA^T Lam = dJ/dX, i.e. the backward recursion
    AA Lam^n = dJ/dX^n + A'^T Lam^{n+1},   Lam^{N+1} = 0
(AA is symmetric), and for any parameter theta that enters the matrices
    dJ/dtheta = - sum_n Lam^n . (dAA/dtheta X^n - dA'/dtheta X^{n-1}).

Parameters, per element e: log K_e, lambda_e, mu_e.
  * K enters only S = tau C_K + C_beta, so dAA/dlogK_e = [0 0; 0 -tau K_e L_e]
    with L_e the element stiffness of the unit-coefficient Laplacian.
  * lambda and mu enter A (the elasticity form) and, through the stabilization
    parameter beta_e = alpha^2 h^2 / (4 (lambda_e + 2 mu_e)), the C_beta block
    that appears with a minus sign both in AA and in A'.  Hence
        dAA/dlam_e X^n - dA'/dlam_e X^{n-1}
            = [A_e^lam U^n ;  -(dbeta_e/dlam_e) L_e (P^n - P^{n-1})]
    and the same for mu with A_e^mu and dbeta_e/dmu_e.
Prescribed dofs are zero in X and Lam, so the element matrices are contracted
without any boundary treatment.  The gradient with respect to a global lambda
or mu is the sum of the per-element entries.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from . import fem
from .sequential import BiotOracle


# ----------------------------------------------------------------------------
# problem with explicit (log K, lambda, mu) per element
# ----------------------------------------------------------------------------
def assemble_params(problem, logk: np.ndarray, lam: np.ndarray, mu: np.ndarray) -> fem.Assembled:
    """A, B, C_K, C_beta for per-element log-permeability and Lame parameters
    (default beta of the stabilization, Sec. 2)."""
    dim, n = problem.dim, problem.n_nodes
    lam = np.asarray(lam, dtype=np.float64)
    mu = np.asarray(mu, dtype=np.float64)
    K = np.exp(np.asarray(logk, dtype=np.float64))
    grads, vol = fem.simplex_gradients(problem.xyz, problem.conn)
    beta = problem.alpha ** 2 * problem.stab_h ** 2 / (4.0 * (lam + 2.0 * mu))
    conn = problem.conn.astype(np.int64)
    udofs = (conn[:, :, None] * dim + np.arange(dim)[None, None, :]).reshape(conn.shape[0], -1)
    A = fem._scatter(udofs, udofs, fem.element_elasticity(grads, vol, lam, mu), n * dim, n * dim)
    B = fem._scatter(udofs, conn, fem.element_coupling(grads, vol, problem.alpha), n * dim, n)
    CK = fem._scatter(conn, conn, fem.element_laplacian(grads, vol, K), n, n)
    Cb = fem._scatter(conn, conn, fem.element_laplacian(grads, vol, beta), n, n)
    return fem.Assembled(dim, n, A, B, CK, Cb, lam, mu, beta)


def oracle_for_params(problem, logk, lam, mu) -> BiotOracle:
    return BiotOracle(problem, asm=assemble_params(problem, logk, lam, mu))


def problem_params(problem):
    """(log K, lambda, mu) per element of a problem given by E, nu, K."""
    lam, mu = fem.lame(problem.young, problem.poisson)
    return np.log(problem.perm), lam, mu


# ----------------------------------------------------------------------------
# space-time solves
# ----------------------------------------------------------------------------
def space_time_solve(orc: BiotOracle, rhs: np.ndarray) -> np.ndarray:
    """X with AA X^n = A' X^{n-1} + rhs^n (n = 1..N, X^0 = 0); rhs is [N, n_dof]
    field-major, prescribed rows ignored.  Returns [N+1, n_dof]."""
    N = rhs.shape[0]
    st = orc.step_solver()
    X = np.zeros((N + 1, orc.n_dof))
    for n in range(1, N + 1):
        b = orc.Ap @ X[n - 1] + rhs[n - 1]
        X[n, orc.free] = st.solve(b[orc.free])
    return X


def adjoint_solve(orc: BiotOracle, g: np.ndarray) -> np.ndarray:
    """Lam with AA Lam^n = g^n + A'^T Lam^{n+1}, Lam^{N+1} = 0, on the free dofs
    (g is [N, n_dof]); returns [N, n_dof] with row n-1 = Lam^n."""
    N = g.shape[0]
    st = orc.step_solver()
    ApT = sp.csr_matrix(orc.Ap.T)
    Lam = np.zeros((N, orc.n_dof))
    nxt = np.zeros(orc.n_dof)
    for n in range(N, 0, -1):
        b = g[n - 1] + ApT @ nxt
        Lam[n - 1, orc.free] = st.solve(b[orc.free])
        nxt = Lam[n - 1]
    return Lam


# ----------------------------------------------------------------------------
# the pressure-misfit objective
# ----------------------------------------------------------------------------
def sensor_pressures(orc: BiotOracle, X: np.ndarray, sensors: np.ndarray) -> np.ndarray:
    """p^n at the sensor nodes for n = 1..N: [N, S]."""
    return X[1:, orc.nU + np.asarray(sensors, dtype=np.int64)]


def objective(orc: BiotOracle, X: np.ndarray, sensors, p_obs) -> float:
    r = sensor_pressures(orc, X, sensors) - p_obs
    return float(np.sum(r * r))


def objective_gradient_state(orc: BiotOracle, X: np.ndarray, sensors, p_obs) -> np.ndarray:
    """dJ/dX^n for n = 1..N as [N, n_dof] (zero on prescribed dofs)."""
    N = X.shape[0] - 1
    g = np.zeros((N, orc.n_dof))
    idx = orc.nU + np.asarray(sensors, dtype=np.int64)
    g[:, idx] = 2.0 * (X[1:, idx] - p_obs)
    g[:, orc.fixed] = 0.0
    return g


def parameter_gradient(orc: BiotOracle, X: np.ndarray, Lam: np.ndarray, perm: np.ndarray):
    """(dJ/dlogK_e, dJ/dlambda_e, dJ/dmu_e) from the forward states X [N+1, n_dof],
    the adjoint states Lam [N, n_dof] and the element permeabilities K_e."""
    pb = orc.problem
    dim, nn = orc.dim, orc.n_nodes
    N = X.shape[0] - 1
    tau = orc.tau
    asm = orc.asm
    grads, vol = fem.simplex_gradients(pb.xyz, pb.conn)
    ne = vol.shape[0]
    conn = pb.conn.astype(np.int64)
    Le = fem.element_laplacian(grads, vol, np.ones(ne))
    A_lam = fem.element_elasticity(grads, vol, np.ones(ne), np.zeros(ne))
    A_mu = fem.element_elasticity(grads, vol, np.zeros(ne), np.ones(ne))
    lam, mu, beta = asm.lam, asm.mu, asm.beta
    dbeta_dlam = -beta / (lam + 2.0 * mu)
    dbeta_dmu = -2.0 * beta / (lam + 2.0 * mu)
    Xn = fem.field_to_node_major(X, nn, dim)                  # [N+1, nn, d+1]
    Ln = fem.field_to_node_major(Lam, nn, dim)                # [N, nn, d+1]
    g_logk = np.zeros(ne)
    g_lam = np.zeros(ne)
    g_mu = np.zeros(ne)
    for n in range(1, N + 1):
        ue = Xn[n][conn, :dim].reshape(ne, -1)                # [ne, (d+1) d], local a*d + c
        pe = Xn[n][conn, dim]                                 # [ne, d+1]
        dpe = pe - Xn[n - 1][conn, dim]
        lu = Ln[n - 1][conn, :dim].reshape(ne, -1)
        lp = Ln[n - 1][conn, dim]
        g_logk += tau * np.einsum("ea,eab,eb->e", lp, Le, pe)
        LdP = np.einsum("ea,eab,eb->e", lp, Le, dpe)
        g_lam += -np.einsum("ea,eab,eb->e", lu, A_lam, ue) + dbeta_dlam * LdP
        g_mu += -np.einsum("ea,eab,eb->e", lu, A_mu, ue) + dbeta_dmu * LdP
    g_logk *= np.asarray(perm, dtype=np.float64)
    return g_logk, g_lam, g_mu


def forward(problem, logk, lam, mu):
    """Oracle for the parameters and its backward-Euler trajectory."""
    orc = oracle_for_params(problem, logk, lam, mu)
    rhs = np.stack([orc.load(n) for n in range(1, problem.n_steps + 1)])
    return orc, space_time_solve(orc, rhs)


def objective_value(problem, logk, lam, mu, sensors, p_obs) -> float:
    orc, X = forward(problem, logk, lam, mu)
    return objective(orc, X, sensors, p_obs)


def objective_and_gradient(problem, logk, lam, mu, sensors, p_obs):
    """J and (dJ/dlogK_e, dJ/dlambda_e, dJ/dmu_e), plus X and Lam."""
    orc, X = forward(problem, logk, lam, mu)
    J = objective(orc, X, sensors, p_obs)
    g = objective_gradient_state(orc, X, sensors, p_obs)
    Lam = adjoint_solve(orc, g)
    grads = parameter_gradient(orc, X, Lam, np.exp(np.asarray(logk, dtype=np.float64)))
    return J, grads, X, Lam


def observations(problem, logk_ref, sensors) -> np.ndarray:
    """Synthetic data: sensor pressures of the forward run with a reference
    log-permeability field (same Lame parameters as the problem)."""
    _, lam, mu = problem_params(problem)
    orc, X = forward(problem, logk_ref, lam, mu)
    return sensor_pressures(orc, X, sensors).copy()
