"""Geometric multigrid on the nested structured meshes (oracle).

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper applies A^{-1} and S_p^{-1} inside its block preconditioners (Sec. 3.1)
without saying how.  The device path replaces each by a fixed linear multigrid
V-cycle; this module states that V-cycle plainly so that one device sweep can be
checked against it value by value.

Hierarchy.  Level 0 is the given structured mesh with n cells per side; level
l+1 has n/2^(l+1) cells and its nodes are the even-index nodes of level l.  The
right-triangle mesh of 2m cells is the midpoint refinement of the one of m cells
(Sec. 4.1), so the P1 spaces are nested and the prolongation is plain P1
interpolation: a fine node that is a coarse node takes its value; a fine node at
the midpoint of a coarse edge takes the mean of the edge's two ends.  The
coarse-level operators are Galerkin products K_{l+1} = P' K_l P.

Boundary conditions.  A coarse dof is prescribed iff the coincident fine dof is;
prolongation rows of prescribed fine dofs and columns of prescribed coarse dofs
are zero, and prescribed dofs keep a unit diagonal on every level.

Cycle.  Each level has node-block diagonal blocks D (the dim x dim displacement
block of a node, or the 1x1 pressure entry); the smoother is Chebyshev
iteration of a fixed degree preconditioned by D^{-1}, on the interval
[lmax/ratio, lmax] with lmax an upper bound of the spectrum of D^{-1}K.  The
coarsest level is solved exactly.  One application of the cycle to r is
    x = presmooth(0, r); x += P V_{l+1}(P'(r - K x)); x = postsmooth(x, r).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
import scipy.sparse as sp
import scipy.linalg as sla


def coarse_sizes(n: int, min_cells: int = 2):
    """Cells per side on every level: halve while even and above min_cells."""
    sizes = [n]
    while sizes[-1] % 2 == 0 and sizes[-1] // 2 >= min_cells:
        sizes.append(sizes[-1] // 2)
    return sizes


def prolongation_2d(nc: int, comps: int) -> sp.csr_matrix:
    """P1 interpolation from the (nc)^2-cell grid to the (2 nc)^2-cell grid.

    Node-major dofs: dof = node*comps + c.  Fine node (i, j) with both indices
    even is coarse node (i/2, j/2); with one or both odd it is the midpoint of a
    coarse edge: horizontal, vertical, or the (i,j)->(i+1,j+1) diagonal.
    """
    nf = 2 * nc
    mf = nf + 1
    mc = nc + 1
    rows, cols, vals = [], [], []
    for j in range(mf):
        for i in range(mf):
            f = j * mf + i
            I0, J0 = i // 2, j // 2
            if i % 2 == 0 and j % 2 == 0:
                src = [(J0 * mc + I0, 1.0)]
            elif i % 2 == 1 and j % 2 == 0:
                src = [(J0 * mc + I0, 0.5), (J0 * mc + I0 + 1, 0.5)]
            elif i % 2 == 0 and j % 2 == 1:
                src = [(J0 * mc + I0, 0.5), ((J0 + 1) * mc + I0, 0.5)]
            else:
                src = [(J0 * mc + I0, 0.5), ((J0 + 1) * mc + I0 + 1, 0.5)]
            for (c_node, w) in src:
                for c in range(comps):
                    rows.append(f * comps + c)
                    cols.append(c_node * comps + c)
                    vals.append(w)
    return sp.csr_matrix((vals, (rows, cols)), shape=(mf * mf * comps, mc * mc * comps))


def prolongation_3d(nc: int, comps: int) -> sp.csr_matrix:
    """P1 interpolation between nested Kuhn meshes: a fine node with odd indices
    is the midpoint of the coarse edge from (floor) to (floor + odd pattern)."""
    nf = 2 * nc
    mf = nf + 1
    mc = nc + 1
    rows, cols, vals = [], [], []
    for k in range(mf):
        for j in range(mf):
            for i in range(mf):
                f = (k * mf + j) * mf + i
                a = (k // 2, j // 2, i // 2)
                odd = (k % 2, j % 2, i % 2)
                c0 = (a[0] * mc + a[1]) * mc + a[2]
                if odd == (0, 0, 0):
                    src = [(c0, 1.0)]
                else:
                    b = (a[0] + odd[0], a[1] + odd[1], a[2] + odd[2])
                    c1 = (b[0] * mc + b[1]) * mc + b[2]
                    src = [(c0, 0.5), (c1, 0.5)]
                for (c_node, w) in src:
                    for c in range(comps):
                        rows.append(f * comps + c)
                        cols.append(c_node * comps + c)
                        vals.append(w)
    return sp.csr_matrix((vals, (rows, cols)), shape=(mf ** 3 * comps, mc ** 3 * comps))


def coarse_fixed(fixed_f: np.ndarray, nf: int, dim: int, comps: int) -> np.ndarray:
    """Prescribed mask on the coarse grid: injection from the coincident fine node."""
    mf = nf + 1
    nc = nf // 2
    mc = nc + 1
    ff = fixed_f.reshape(-1, comps)
    if dim == 2:
        J, I = np.meshgrid(np.arange(mc), np.arange(mc), indexing="ij")
        fine_nodes = (2 * J) * mf + 2 * I
    else:
        K, J, I = np.meshgrid(np.arange(mc), np.arange(mc), np.arange(mc), indexing="ij")
        fine_nodes = ((2 * K) * mf + 2 * J) * mf + 2 * I
    return ff[fine_nodes.ravel()].ravel()


def apply_fixed(K: sp.csr_matrix, fixed: np.ndarray) -> sp.csr_matrix:
    """Zero rows and columns of prescribed dofs and put 1 on their diagonal."""
    keep = sp.diags((~fixed).astype(np.float64))
    K = (keep @ K @ keep).tocsr()
    K = K + sp.diags(fixed.astype(np.float64))
    K.eliminate_zeros()
    return K.tocsr()


def block_diag_inverse(K: sp.csr_matrix, comps: int) -> np.ndarray:
    """Inverses of the comps x comps node blocks of K: [n_nodes, comps, comps]."""
    n = K.shape[0] // comps
    D = np.zeros((n, comps, comps))
    Kc = K.tocsr()
    for a in range(comps):
        for b in range(comps):
            rows = np.arange(n) * comps + a
            cols = np.arange(n) * comps + b
            D[:, a, b] = np.asarray(Kc[rows, cols]).ravel()
    return np.linalg.inv(D)


def apply_blocks(Dinv: np.ndarray, r: np.ndarray) -> np.ndarray:
    comps = Dinv.shape[1]
    return np.einsum("nab,nb->na", Dinv, r.reshape(-1, comps)).ravel()


def power_lmax(K, Dinv, iters: int = 30, seed: int = 0) -> float:
    """Estimate of the largest eigenvalue of D^{-1} K by power iteration
    (in the K-inner product, where D^{-1}K is self-adjoint)."""
    rng = np.random.default_rng(seed)
    x = rng.standard_normal(K.shape[0])
    lam = 0.0
    for _ in range(iters):
        y = apply_blocks(Dinv, K @ x)
        lam = float(x @ (K @ y)) / float(x @ (K @ x))
        x = y / np.linalg.norm(y)
    return lam


@dataclass
class Level:
    n: int
    K: sp.csr_matrix
    fixed: np.ndarray
    Dinv: np.ndarray
    lmax: float = 0.0
    P: sp.csr_matrix | None = None     # prolongation from the next (coarser) level


@dataclass
class Hierarchy:
    dim: int
    comps: int
    levels: list = field(default_factory=list)
    degree: int = 2
    ratio: float = 4.0
    coarse_lu: tuple | None = None


def build(K0: sp.csr_matrix, fixed0: np.ndarray, n: int, dim: int, comps: int,
          degree: int = 2, ratio: float = 4.0, lmax_safety: float = 1.05,
          min_cells: int = 2, lmax: list | None = None) -> Hierarchy:
    """Hierarchy for an SPD node-major operator K0 with `comps` dofs per node.

    `lmax` may give the per-level spectral bounds directly (used to mirror a
    bound computed elsewhere); otherwise they come from power iteration, scaled
    by `lmax_safety`.
    """
    H = Hierarchy(dim=dim, comps=comps, degree=degree, ratio=ratio)
    sizes = coarse_sizes(n, min_cells)
    K = apply_fixed(K0.tocsr(), fixed0)
    fixed = fixed0.copy()
    for li, nl in enumerate(sizes):
        lev = Level(n=nl, K=K, fixed=fixed, Dinv=block_diag_inverse(K, comps))
        H.levels.append(lev)
        if li + 1 < len(sizes):
            P = prolongation_2d(nl // 2, comps) if dim == 2 else prolongation_3d(nl // 2, comps)
            fc = coarse_fixed(fixed, nl, dim, comps)
            P = sp.diags((~fixed).astype(np.float64)) @ P @ sp.diags((~fc).astype(np.float64))
            lev.P = P.tocsr()
            K = apply_fixed((P.T @ K @ P).tocsr(), fc)
            fixed = fc
    for li, lev in enumerate(H.levels[:-1]):
        lev.lmax = lmax[li] if lmax is not None else lmax_safety * power_lmax(lev.K, lev.Dinv)
    Kc = H.levels[-1].K.toarray()
    H.coarse_lu = sla.lu_factor(Kc)
    return H


def chebyshev(lev: Level, x: np.ndarray, r: np.ndarray, degree: int, ratio: float) -> np.ndarray:
    """`degree` steps of Chebyshev iteration for K x = r, preconditioned by D^{-1},
    targeting the interval [lmax/ratio, lmax] (standard three-term recurrence)."""
    lmax = lev.lmax
    lmin = lmax / ratio
    theta = 0.5 * (lmax + lmin)
    delta = 0.5 * (lmax - lmin)
    sigma = theta / delta
    rho = 1.0 / sigma
    res = r - lev.K @ x
    d = apply_blocks(lev.Dinv, res) / theta
    x = x + d
    for _ in range(degree - 1):
        res = r - lev.K @ x
        rho_new = 1.0 / (2.0 * sigma - rho)
        d = rho_new * rho * d + (2.0 * rho_new / delta) * apply_blocks(lev.Dinv, res)
        x = x + d
        rho = rho_new
    return x


def vcycle(H: Hierarchy, r: np.ndarray, level: int = 0, pre: int = 1, post: int = 1) -> np.ndarray:
    """One V-cycle approximating K_level^{-1} r (zero initial guess)."""
    lev = H.levels[level]
    if level == len(H.levels) - 1:
        return sla.lu_solve(H.coarse_lu, r)
    x = np.zeros_like(r)
    for _ in range(pre):
        x = chebyshev(lev, x, r, H.degree, H.ratio)
    rc = lev.P.T @ (r - lev.K @ x)
    x = x + lev.P @ vcycle(H, rc, level + 1, pre, post)
    for _ in range(post):
        x = chebyshev(lev, x, r, H.degree, H.ratio)
    return x
