"""Closed-form solutions used to pin the oracle (oracle).

TEST INFRASTRUCTURE ONLY (see the package docstring).

* Terzaghi one-dimensional consolidation of a column of height H = 1 under a
  unit top load q, drained at the top (y = H), impermeable and fixed at the base,
  with Biot coefficient alpha and no storage (1/M = 0).  Consolidation
  coefficient c_v = K (lambda + 2 mu) / alpha^2; the classical Fourier series
      p(y, t) = (4 q / (alpha pi)) sum_k (-1)^k / (2k+1) cos((2k+1) pi y / 2)
                exp(-(2k+1)^2 pi^2 c_v t / 4)
  with u_y(y, t) = int_0^y (alpha p - q) / (lambda + 2 mu).
  Its t -> infinity limit u_y = -q y / (lambda + 2 mu), p = 0 is linear and hence
  reproduced exactly by P1 elements.

* The trigonometric manufactured solution of Sec. 4.1:
  u_1 = u_2 = p = cos t cos(3 pi x) cos(3 pi y) on the unit square with
  Dirichlet data on the whole boundary.  The body force is as printed; the source
  term is the one that makes the printed solution exact,
      g = 3 alpha pi sin t (sin 3pix cos 3piy + cos 3pix sin 3piy)
          + 18 K pi^2 cos t cos 3pix cos 3piy,
  (the printed g has the first bracket with a minus sign and its terms swapped,
  which the exact solution does not satisfy).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from . import fem
from .sequential import StepSolver


# ---------------------------------------------------------------------------
# Terzaghi
# ---------------------------------------------------------------------------
def terzaghi_pressure(y, t, cv, q=1.0, alpha=1.0, terms=400):
    y = np.asarray(y, dtype=np.float64)
    k = np.arange(terms)
    m = 2 * k + 1
    coef = (4.0 * q / (alpha * np.pi)) * ((-1.0) ** k) / m
    mode = np.cos(np.outer(y, m) * np.pi / 2.0)
    decay = np.exp(-(m ** 2) * np.pi ** 2 * cv * t / 4.0)
    return mode @ (coef * decay)


def terzaghi_displacement(y, t, cv, lam, mu, q=1.0, alpha=1.0, terms=400):
    """u_y(y, t) = int_0^y (alpha p - q)/(lam + 2 mu); the cosine modes integrate
    to sines."""
    y = np.asarray(y, dtype=np.float64)
    k = np.arange(terms)
    m = 2 * k + 1
    coef = (4.0 * q / (alpha * np.pi)) * ((-1.0) ** k) / m
    decay = np.exp(-(m ** 2) * np.pi ** 2 * cv * t / 4.0)
    integ = np.sin(np.outer(y, m) * np.pi / 2.0) / (m * np.pi / 2.0)
    int_p = integ @ (coef * decay)
    return (alpha * int_p - q * y) / (lam + 2.0 * mu)


# ---------------------------------------------------------------------------
# triangle quadrature: Dunavant's 6-point rule, exact for degree 4
# (D. A. Dunavant, Int. J. Numer. Meth. Eng. 21, 1985)
# ---------------------------------------------------------------------------
_A1, _B1, _W1 = 0.445948490915965, 0.108103018168070, 0.223381589678011
_A2, _B2, _W2 = 0.091576213509771, 0.816847572980459, 0.109951743655322
TRI_BARY = np.array([[_B1, _A1, _A1], [_A1, _B1, _A1], [_A1, _A1, _B1],
                     [_B2, _A2, _A2], [_A2, _B2, _A2], [_A2, _A2, _B2]])
TRI_W = np.array([_W1, _W1, _W1, _W2, _W2, _W2])


def tri_quadrature(xyz, conn):
    """Physical quadrature points [ne, nq, 2], weights [ne, nq] and barycentric
    values of the three hat functions at the points [nq, 3]."""
    x = xyz[conn]                                     # [ne, 3, 2]
    pts = np.einsum("qa,ead->eqd", TRI_BARY, x)
    _, vol = fem.simplex_gradients(xyz, conn)
    return pts, vol[:, None] * TRI_W[None, :], TRI_BARY


# ---------------------------------------------------------------------------
# manufactured solution
# ---------------------------------------------------------------------------
def mms_exact(x, y, t):
    return np.cos(t) * np.cos(3 * np.pi * x) * np.cos(3 * np.pi * y)


def mms_force(x, y, t, lam, mu, alpha):
    s3x, c3x = np.sin(3 * np.pi * x), np.cos(3 * np.pi * x)
    s3y, c3y = np.sin(3 * np.pi * y), np.cos(3 * np.pi * y)
    pi = np.pi
    fx = -3 * pi * np.cos(t) * (alpha * s3x * c3y - 3 * pi * (lam + 3 * mu) * c3x * c3y
                                + 3 * pi * (lam + mu) * s3x * s3y)
    fy = -3 * pi * np.cos(t) * (alpha * c3x * s3y - 3 * pi * (lam + 3 * mu) * c3x * c3y
                                + 3 * pi * (lam + mu) * s3x * s3y)
    return fx, fy


def mms_source(x, y, t, alpha, K):
    s3x, c3x = np.sin(3 * np.pi * x), np.cos(3 * np.pi * x)
    s3y, c3y = np.sin(3 * np.pi * y), np.cos(3 * np.pi * y)
    pi = np.pi
    return (3 * alpha * pi * np.sin(t) * (s3x * c3y + c3x * s3y)
            + 18 * K * pi ** 2 * np.cos(t) * c3x * c3y)


def mms_problem(n: int, dt: float, n_steps: int, E=1.0, nu=0.3, alpha=1.0, K=1.0):
    """Problem description for the manufactured solution (all-Dirichlet)."""
    from paper_2310_10430_amd import workloads as W
    xyz, conn = W.square_mesh(n)
    tol = 1e-12
    bnd = ((xyz[:, 0] < tol) | (xyz[:, 0] > 1 - tol) | (xyz[:, 1] < tol) | (xyz[:, 1] > 1 - tol))
    flags = np.where(bnd, 0b111, 0).astype(np.uint8)
    ne = conn.shape[0]
    return W.Problem(dim=2, grid_n=n, xyz=xyz, conn=conn, flags=flags,
                     young=np.full(ne, E), poisson=np.full(ne, nu), perm=np.full(ne, K),
                     alpha=alpha, stab_h=1.0 / n, facets=np.zeros((0, 2), np.int32),
                     traction=np.zeros((0, 2)), load_coef=np.zeros(n_steps + 1),
                     n_steps=n_steps, dt=dt)


def mms_solve(n: int, dt: float, n_steps: int, E=1.0, nu=0.3, alpha=1.0, K=1.0,
              trajectory: bool = False):
    """Sequential backward Euler for the manufactured solution.

    Returns (problem, X) with X the field-major state after n_steps steps, or
    with trajectory=True the states of all steps [n_steps+1, n_dof].
    Prescribed boundary values are the exact solution at each time level; they
    are lifted into the right-hand side.
    """
    pb = mms_problem(n, dt, n_steps, E, nu, alpha, K)
    asm = fem.assemble(pb)
    lam, mu = float(asm.lam[0]), float(asm.mu[0])
    AA, Ap = fem.block_system(asm, dt)
    fixed = fem.dirichlet_mask(pb)
    free = np.nonzero(~fixed)[0]
    fx_idx = np.nonzero(fixed)[0]
    nn = pb.n_nodes
    nU = 2 * nn
    pts, wts, bary = tri_quadrature(pb.xyz, pb.conn)
    conn = pb.conn.astype(np.int64)

    def nodal(t):
        v = mms_exact(pb.xyz[:, 0], pb.xyz[:, 1], t)
        return np.concatenate([np.repeat(v, 2), v])     # u_x, u_y interleaved, then p

    def loads(t):
        fx, fy = mms_force(pts[..., 0], pts[..., 1], t, lam, mu, alpha)
        g = mms_source(pts[..., 0], pts[..., 1], t, alpha, K)
        F = np.zeros(nU)
        G = np.zeros(nn)
        for a in range(3):
            phi = bary[:, a][None, :]
            np.add.at(F, conn[:, a] * 2, np.sum(wts * phi * fx, axis=1))
            np.add.at(F, conn[:, a] * 2 + 1, np.sum(wts * phi * fy, axis=1))
            np.add.at(G, conn[:, a], np.sum(wts * phi * g, axis=1))
        return np.concatenate([F, -dt * G])

    st = StepSolver(AA, free)
    AA_fD = AA[free][:, fx_idx]
    X = nodal(0.0)
    traj = [X] if trajectory else None
    for m in range(1, n_steps + 1):
        t = m * dt
        Xm = nodal(t)
        rhs = (Ap @ X + loads(t))[free] - AA_fD @ Xm[fx_idx]
        Xm[free] = st.solve(rhs)
        X = Xm
        if trajectory:
            traj.append(X)
    return pb, (np.array(traj) if trajectory else X)


def l2_error_p(pb, X: np.ndarray, t: float) -> float:
    """|| p_h(t) - p(t) ||_{L^2} by the degree-4 rule on every triangle."""
    nU = 2 * pb.n_nodes
    p = X[nU:]
    pts, wts, bary = tri_quadrature(pb.xyz, pb.conn)
    ph = np.einsum("qa,ea->eq", bary, p[pb.conn])
    pe = mms_exact(pts[..., 0], pts[..., 1], t)
    return float(np.sqrt(np.sum(wts * (ph - pe) ** 2)))
