"""Stabilized P1-P1 finite elements for the two-field Biot model (oracle).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Follows Sec. 2 of the paper:
  * Lame parameters from E and nu (Sec. 2.1).
  * a(u, v) = int 2 mu eps(u):eps(v) + lambda div u div v.  The printed bilinear
    form omits the lambda term although the stress tensor of Sec. 2.1 contains
    it; the standard form with lambda is used.
  * b(v, q) = alpha int q div v; the block B is the matrix of -b (Sec. 2.2).
  * c(p, q) = K int grad p . grad q gives C_K.
  * The stabilization term (beta/K) c(dp/dt, q) = beta int grad dp/dt . grad q
    gives C_beta, with beta_e = alpha^2 h^2 / (4 (lambda_e + 2 mu_e)) per element
    (the printed formula lost the square on h and the alpha^2 factor; only h^2 is
    dimensionally consistent).
  * Backward Euler, eq. (diseq1)/(fullysystem):
        [A  B ] [U^m]   [0   0     ] [U^{m-1}]   [ F^m     ]
        [B' -S] [P^m] = [B'  -C_beta] [P^{m-1}] + [-tau G^m ]
    with S = tau C_K + C_beta.

P1 gradients are constant per simplex, so every volume integral here is exact
with the gradients and the simplex measure; int phi_i = |T| / (dim+1).

DOF orderings.  Internally the oracle keeps fields apart ("field-major"):
u-dof = node*dim + c, then p-dof = node.  Trajectories are returned node-major
([n_steps+1, n_nodes, dim+1], components u_x, u_y, (u_z), p), the layout of the
device library.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np
import scipy.sparse as sp


def lame(E, nu):
    """Lame parameters from Young's modulus and Poisson's ratio (Sec. 2.1)."""
    E = np.asarray(E, dtype=np.float64)
    nu = np.asarray(nu, dtype=np.float64)
    lam = E * nu / ((1.0 + nu) * (1.0 - 2.0 * nu))
    mu = E / (2.0 * (1.0 + nu))
    return lam, mu


def simplex_gradients(xyz: np.ndarray, conn: np.ndarray):
    """Gradients of the barycentric coordinates and the measure of every simplex.

    For vertices x_0..x_d, J = [x_1-x_0, ..., x_d-x_0]; the barycentric
    coordinates of 1..d are J^{-1}(x - x_0), so their gradients are the rows of
    J^{-1}; the gradient of coordinate 0 is minus their sum.
    Returns grads [ne, d+1, d] and vol [ne].
    """
    dim = xyz.shape[1]
    x = xyz[conn]                                   # [ne, d+1, d]
    J = np.transpose(x[:, 1:, :] - x[:, :1, :], (0, 2, 1))   # columns x_i - x_0
    det = np.linalg.det(J)
    if np.any(det <= 0):
        raise ValueError("mesh has inverted or degenerate simplices")
    Jinv = np.linalg.inv(J)                         # rows = grad lambda_1..d
    grads = np.empty((conn.shape[0], dim + 1, dim))
    grads[:, 1:, :] = Jinv
    grads[:, 0, :] = -Jinv.sum(axis=1)
    vol = det / math.factorial(dim)
    return grads, vol


def element_elasticity(grads, vol, lam, mu):
    """Element matrices of a(u,v) = int 2mu eps:eps + lam div div.

    Entry [(a,c),(b,d)] = vol (mu delta_cd g_a.g_b + mu g_a[d] g_b[c]
                              + lam g_a[c] g_b[d]).
    Returned as [ne, (d+1)*d, (d+1)*d] with local index a*d + c.
    """
    ne, nv, dim = grads.shape
    gg = np.einsum("eai,ebi->eab", grads, grads)             # g_a . g_b
    eye = np.eye(dim)
    K = (mu[:, None, None, None, None] * gg[:, :, None, :, None] * eye[None, None, :, None, :]
         + mu[:, None, None, None, None] * np.einsum("ead,ebc->eacbd", grads, grads)
         + lam[:, None, None, None, None] * np.einsum("eac,ebd->eacbd", grads, grads))
    K *= vol[:, None, None, None, None]
    return K.reshape(ne, nv * dim, nv * dim)


def element_coupling(grads, vol, alpha):
    """Element matrices of B = matrix of -b(v, q) = -alpha int q div v.

    Entry [(a,c), i] = -alpha g_a[c] vol/(d+1).  Shape [ne, (d+1)*d, d+1].
    """
    ne, nv, dim = grads.shape
    Be = -alpha * grads.reshape(ne, nv * dim)[:, :, None] * (vol / nv)[:, None, None]
    return np.repeat(Be, nv, axis=2)


def element_laplacian(grads, vol, coef):
    """Element matrices of coef int grad p . grad q.  Shape [ne, d+1, d+1]."""
    return coef[:, None, None] * vol[:, None, None] * np.einsum("eai,ebi->eab", grads, grads)


def _scatter(rows_local_to_global, cols_local_to_global, Ke, nrow, ncol):
    ne, r, c = Ke.shape
    I = np.repeat(rows_local_to_global[:, :, None], c, axis=2)
    J = np.repeat(cols_local_to_global[:, None, :], r, axis=1)
    M = sp.coo_matrix((Ke.ravel(), (I.ravel(), J.ravel())), shape=(nrow, ncol))
    return M.tocsr()


@dataclass
class Assembled:
    """Global matrices before boundary conditions (field-major numbering)."""
    dim: int
    n_nodes: int
    A: sp.csr_matrix        # [n*dim, n*dim]
    B: sp.csr_matrix        # [n*dim, n]
    CK: sp.csr_matrix       # [n, n]
    Cb: sp.csr_matrix       # [n, n]
    lam: np.ndarray
    mu: np.ndarray
    beta: np.ndarray


def assemble(problem) -> Assembled:
    """Global A, B, C_K, C_beta of the stabilized P1-P1 discretization."""
    dim = problem.dim
    n = problem.n_nodes
    grads, vol = simplex_gradients(problem.xyz, problem.conn)
    lam, mu = lame(problem.young, problem.poisson)
    beta = problem.alpha ** 2 * problem.stab_h ** 2 / (4.0 * (lam + 2.0 * mu))
    conn = problem.conn.astype(np.int64)
    udofs = (conn[:, :, None] * dim + np.arange(dim)[None, None, :]).reshape(conn.shape[0], -1)
    A = _scatter(udofs, udofs, element_elasticity(grads, vol, lam, mu), n * dim, n * dim)
    B = _scatter(udofs, conn, element_coupling(grads, vol, problem.alpha), n * dim, n)
    CK = _scatter(conn, conn, element_laplacian(grads, vol, problem.perm), n, n)
    Cb = _scatter(conn, conn, element_laplacian(grads, vol, beta), n, n)
    return Assembled(dim, n, A, B, CK, Cb, lam, mu, beta)


def traction_load(problem) -> np.ndarray:
    """u-part of the load vector, int_Gamma t . v ds, for a unit load multiplier.

    Each facet's traction is constant, so vertex a of a facet receives
    t * |facet| / dim.  Returned field-major over u-dofs, shape [n*dim].
    """
    dim = problem.dim
    x = problem.xyz[problem.facets]                 # [nf, dim, dim]
    if dim == 2:
        meas = np.linalg.norm(x[:, 1] - x[:, 0], axis=1)
    else:
        meas = 0.5 * np.linalg.norm(np.cross(x[:, 1] - x[:, 0], x[:, 2] - x[:, 0]), axis=1)
    F = np.zeros(problem.n_nodes * dim)
    share = (meas / dim)[:, None] * problem.traction      # [nf, dim]
    for a in range(dim):
        for c in range(dim):
            np.add.at(F, problem.facets[:, a].astype(np.int64) * dim + c, share[:, c])
    return F


def dirichlet_mask(problem) -> np.ndarray:
    """Boolean mask over field-major dofs: True where the value is prescribed."""
    dim = problem.dim
    fl = problem.flags.astype(np.int64)
    u_fixed = np.stack([(fl >> c) & 1 for c in range(dim)], axis=1).astype(bool).ravel()
    p_fixed = ((fl >> dim) & 1).astype(bool)
    return np.concatenate([u_fixed, p_fixed])


def block_system(asm: Assembled, tau: float):
    """The step matrix AA = [A B; B' -S] and the coupling A' = [0 0; B' -C_beta]
    of eq. (fullysystem), field-major, before boundary conditions."""
    S = tau * asm.CK + asm.Cb
    AA = sp.bmat([[asm.A, asm.B], [asm.B.T, -S]], format="csr")
    nU = asm.A.shape[0]
    Z = sp.csr_matrix((nU, nU))
    Ap = sp.bmat([[Z, sp.csr_matrix((nU, asm.n_nodes))], [asm.B.T, -asm.Cb]], format="csr")
    return AA, Ap


def field_to_node_major(X: np.ndarray, n_nodes: int, dim: int) -> np.ndarray:
    """[..., n*dim + n] field-major -> [..., n, dim+1] node-major."""
    lead = X.shape[:-1]
    u = X[..., : n_nodes * dim].reshape(*lead, n_nodes, dim)
    p = X[..., n_nodes * dim:].reshape(*lead, n_nodes, 1)
    return np.concatenate([u, p], axis=-1)


def node_to_field_major(Y: np.ndarray) -> np.ndarray:
    """[..., n, dim+1] node-major -> [..., n*dim + n] field-major."""
    lead = Y.shape[:-2]
    n, d1 = Y.shape[-2:]
    u = Y[..., :, : d1 - 1].reshape(*lead, n * (d1 - 1))
    return np.concatenate([u, Y[..., :, d1 - 1]], axis=-1)
