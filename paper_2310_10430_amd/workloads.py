"""Seeded synthetic inputs for the Biot parallel-in-time solver.

This module produces *inputs only*: mesh coordinates and connectivity, boundary
flags, the boundary facets that carry a load, per-element material fields and the
time profile of the load.  It contains none of the solver's arithmetic (no element
matrices, no Lame conversion, no time stepping), so both the device path and the
independent CPU reference can consume the same inputs without sharing any of the
method.

Mesh conventions (the paper's experiments use uniform right-triangle grids on the
unit square, Sec. 4.1):
  * 2D: an N x N grid of squares, node (i, j) has id j*(N+1)+i and sits at
    (i/N, j/N); every square is split along its (i,j)->(i+1,j+1) diagonal, so
    refining N -> 2N is the midpoint (red) refinement the paper describes.
  * 3D (not in the paper): an N^3 grid of cubes, node (i,j,k) has id
    (k*(N+1)+j)*(N+1)+i; every cube is split into the six Kuhn tetrahedra that
    share its (0,0,0)->(1,1,1) diagonal, which is conforming and nested under 2:1
    refinement.

Boundary flags are a per-node bit mask: bit d (d < dim) marks displacement
component d as prescribed, bit dim the pressure (zero unless a problem gives
prescribed values).

The manufactured-solution problem of Sec. 4.1 (`mms_problem`) is an input too:
its data (body force, fluid source, boundary and initial values of the exact
solution) are evaluated from their closed forms and integrated against the P1
hat functions with Dunavant's degree-4 rule, which gives the assembled load
vectors that the C ABI takes; the solver's own arithmetic (element matrices,
time stepping, lifting of prescribed values) is not here.
"""
from __future__ import annotations

import dataclasses
from typing import Optional

import numpy as np

U_BITS_2D = 0b011
P_BIT_2D = 0b100


# ----------------------------------------------------------------------------
# meshes
# ----------------------------------------------------------------------------
def square_mesh(n: int):
    """Structured right-triangle mesh of the unit square with n cells per side.

    Returns (xyz float64 [(n+1)^2, 2], conn int32 [2 n^2, 3]); triangles are
    counter-clockwise.  Triangle 2*(j*n+i) is the lower-right one of square
    (i, j), triangle 2*(j*n+i)+1 the upper-left one.
    """
    if n < 1:
        raise ValueError("n must be >= 1")
    i, j = np.meshgrid(np.arange(n + 1), np.arange(n + 1), indexing="xy")
    xyz = np.stack([i.ravel() / n, j.ravel() / n], axis=1).astype(np.float64)
    ci, cj = np.meshgrid(np.arange(n), np.arange(n), indexing="xy")
    ci = ci.ravel()
    cj = cj.ravel()
    v00 = cj * (n + 1) + ci
    v10 = v00 + 1
    v01 = v00 + (n + 1)
    v11 = v01 + 1
    lower = np.stack([v00, v10, v11], axis=1)
    upper = np.stack([v00, v11, v01], axis=1)
    conn = np.empty((2 * n * n, 3), dtype=np.int32)
    conn[0::2] = lower
    conn[1::2] = upper
    return xyz, conn


# the six axis orders that define the Kuhn simplices of a cube
_KUHN_PERMS = ((0, 1, 2), (0, 2, 1), (1, 0, 2), (1, 2, 0), (2, 0, 1), (2, 1, 0))


def cube_mesh(n: int):
    """Structured Kuhn tetrahedral mesh of the unit cube with n cells per side.

    Returns (xyz float64 [(n+1)^3, 3], conn int32 [6 n^3, 4]).  Each tetrahedron
    walks from the cube's (0,0,0) corner to its (1,1,1) corner one axis at a
    time; vertex order is fixed so that every tetrahedron has positive volume.
    """
    if n < 1:
        raise ValueError("n must be >= 1")
    m = n + 1
    g = np.arange(m)
    k, j, i = np.meshgrid(g, g, g, indexing="ij")
    xyz = np.stack([i.ravel() / n, j.ravel() / n, k.ravel() / n], axis=1).astype(np.float64)
    c = np.arange(n)
    ck, cj, ci = np.meshgrid(c, c, c, indexing="ij")
    base = np.stack([ci.ravel(), cj.ravel(), ck.ravel()], axis=1)
    tets = []
    for perm in _KUHN_PERMS:
        verts = [base.copy()]
        cur = base.copy()
        for ax in perm:
            cur = cur.copy()
            cur[:, ax] += 1
            verts.append(cur)
        ids = [(v[:, 2] * m + v[:, 1]) * m + v[:, 0] for v in verts]
        t = np.stack(ids, axis=1)
        # orientation: sign of the permutation decides the handedness
        sign = _perm_sign(perm)
        if sign < 0:
            t = t[:, [0, 2, 1, 3]]
        tets.append(t)
    # interleave so that the 6 tets of one cube are contiguous
    conn = np.stack(tets, axis=1).reshape(-1, 4).astype(np.int32)
    return xyz, conn


def _perm_sign(p):
    p = list(p)
    s = 1
    for a in range(len(p)):
        for b in range(a + 1, len(p)):
            if p[a] > p[b]:
                s = -s
    return s


# ----------------------------------------------------------------------------
# Terzaghi-type boundary data on the unit square / cube
# ----------------------------------------------------------------------------
def terzaghi_flags(xyz: np.ndarray) -> np.ndarray:
    """Per-node Dirichlet bit mask for the consolidation column.

    Fixed base (all displacement components zero on the bottom face), roller
    sides (the normal displacement component zero on the lateral faces), drained
    top (pressure zero on the top face).  Corners take the union.
    """
    dim = xyz.shape[1]
    up = dim - 1  # vertical axis
    tol = 1e-12
    flags = np.zeros(xyz.shape[0], dtype=np.uint8)
    bottom = xyz[:, up] < tol
    top = xyz[:, up] > 1 - tol
    flags[bottom] |= np.uint8((1 << dim) - 1)
    for ax in range(dim - 1):
        side = (xyz[:, ax] < tol) | (xyz[:, ax] > 1 - tol)
        flags[side] |= np.uint8(1 << ax)
    flags[top] |= np.uint8(1 << dim)
    return flags


def top_facets(n: int, dim: int) -> np.ndarray:
    """Boundary facets of the top face (y=1 in 2D, z=1 in 3D) as node tuples."""
    if dim == 2:
        j = n
        i = np.arange(n)
        a = j * (n + 1) + i
        return np.stack([a, a + 1], axis=1).astype(np.int32)
    m = n + 1
    k = n
    j, i = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    v00 = (k * m + j.ravel()) * m + i.ravel()
    v10 = v00 + 1
    v01 = v00 + m
    v11 = v01 + 1
    # each top square is the face of two Kuhn tets: split along (0,0)->(1,1)
    t1 = np.stack([v00, v10, v11], axis=1)
    t2 = np.stack([v00, v11, v01], axis=1)
    return np.concatenate([t1, t2], axis=0).astype(np.int32)


def step_load_profile(n_steps: int, magnitude: float = 1.0) -> np.ndarray:
    """Load multiplier per time level: zero at t=0, `magnitude` for every step n>=1."""
    c = np.full(n_steps + 1, magnitude, dtype=np.float64)
    c[0] = 0.0
    return c


# ----------------------------------------------------------------------------
# material fields
# ----------------------------------------------------------------------------
def smoothed_gaussian_cells(n: int, seed: int, ell: float) -> np.ndarray:
    """Unit-variance smooth Gaussian field on the n x n cells of the unit square.

    White noise per cell from numpy's PCG64 (`default_rng(seed)`), convolved with
    exp(-r^2 / (2 ell^2)) by a zero-padded FFT, then shifted and scaled to zero
    sample mean and unit sample standard deviation.  Returned as [n*n] in cell
    order j*n+i.
    """
    rng = np.random.default_rng(seed)
    w = rng.standard_normal((n, n))
    h = 1.0 / n
    m = 2 * n
    d = np.minimum(np.arange(m), m - np.arange(m)) * h
    kern = np.exp(-(d[:, None] ** 2 + d[None, :] ** 2) / (2 * ell * ell))
    pad = np.zeros((m, m))
    pad[:n, :n] = w
    z = np.real(np.fft.ifft2(np.fft.fft2(pad) * np.fft.fft2(kern)))[:n, :n]
    z = (z - z.mean()) / z.std()
    return z.ravel()


def lognormal_perm_2d(n: int, seed: int, k_mean: float = 1e-2, sigma: float = 1.0,
                      ell: float = 0.1) -> np.ndarray:
    """Per-element permeability exp(log k_mean + sigma z), z the smooth cell field;
    both triangles of a square share the square's value."""
    z = smoothed_gaussian_cells(n, seed, ell)
    k_cell = np.exp(np.log(k_mean) + sigma * z)
    return np.repeat(k_cell, 2)


def uniform_young(n_elems: int, seed: int, lo: float = 5e3, hi: float = 2e4) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return rng.uniform(lo, hi, size=n_elems)


# ----------------------------------------------------------------------------
# a complete problem description
# ----------------------------------------------------------------------------
@dataclasses.dataclass
class Problem:
    """Everything the solver needs, as plain arrays (inputs only)."""
    dim: int
    grid_n: int                 # cells per side of the structured grid
    xyz: np.ndarray             # [n_nodes, dim] float64
    conn: np.ndarray            # [n_elems, dim+1] int32
    flags: np.ndarray           # [n_nodes] uint8 Dirichlet bit mask (homogeneous values)
    young: np.ndarray           # [n_elems] E
    poisson: np.ndarray         # [n_elems] nu
    perm: np.ndarray            # [n_elems] K (permeability / viscosity)
    alpha: float                # Biot-Willis coefficient
    stab_h: float               # mesh size entering the stabilization parameter
    facets: np.ndarray          # [n_facets, dim] boundary facets carrying a traction
    traction: np.ndarray        # [n_facets, dim] traction vector per facet
    load_coef: np.ndarray       # [n_steps+1] multiplier of the traction at each time level
    n_steps: int
    dt: float
    # general right-hand side (optional; node-major [n_nodes, dim+1] vectors):
    # assembled load terms with per-step multipliers, prescribed-value terms
    # (read at the flagged dofs) with per-step multipliers, initial state
    terms: Optional[np.ndarray] = None            # [n_terms, n_nodes, dim+1]
    term_coef: Optional[np.ndarray] = None        # [n_steps+1, n_terms]
    prescribed: Optional[np.ndarray] = None       # [n_prescribed, n_nodes, dim+1]
    prescribed_coef: Optional[np.ndarray] = None  # [n_steps+1, n_prescribed]
    x0: Optional[np.ndarray] = None               # [n_nodes, dim+1]

    @property
    def n_nodes(self) -> int:
        return self.xyz.shape[0]

    @property
    def n_elems(self) -> int:
        return self.conn.shape[0]

    @property
    def n_dof(self) -> int:
        return self.n_nodes * (self.dim + 1)


def terzaghi_problem(n: int, n_steps: int, dim: int = 2, dt: Optional[float] = None,
                     young=1e4, poisson=0.3, perm=1e-2, alpha: float = 1.0,
                     load: float = 1.0) -> Problem:
    """Consolidation column: unit top load, drained top, fixed base, roller sides.

    `young`, `poisson` and `perm` may be scalars or per-element arrays.
    """
    if dim == 2:
        xyz, conn = square_mesh(n)
    elif dim == 3:
        xyz, conn = cube_mesh(n)
    else:
        raise ValueError("dim must be 2 or 3")
    ne = conn.shape[0]
    facets = top_facets(n, dim)
    tr = np.zeros((facets.shape[0], dim))
    tr[:, dim - 1] = -load
    return Problem(
        dim=dim, grid_n=n, xyz=xyz, conn=conn, flags=terzaghi_flags(xyz),
        young=np.broadcast_to(np.asarray(young, dtype=np.float64), (ne,)).copy(),
        poisson=np.broadcast_to(np.asarray(poisson, dtype=np.float64), (ne,)).copy(),
        perm=np.broadcast_to(np.asarray(perm, dtype=np.float64), (ne,)).copy(),
        alpha=float(alpha), stab_h=1.0 / n, facets=facets, traction=tr,
        load_coef=step_load_profile(n_steps), n_steps=n_steps,
        dt=(1.0 / n_steps) if dt is None else float(dt))


def heterogeneous_problem(n: int, n_steps: int, field_seed: int = 2, young_seed: int = 102,
                          sigma: float = 1.0, ell: float = 0.1) -> Problem:
    """Consolidation column with a log-normal permeability field and uniform-random E."""
    k = lognormal_perm_2d(n, field_seed, 1e-2, sigma, ell)
    e = uniform_young(2 * n * n, young_seed)
    return terzaghi_problem(n, n_steps, young=e, perm=k)


# ----------------------------------------------------------------------------
# named workloads
# ----------------------------------------------------------------------------
def small_terzaghi() -> Problem:
    """16 x 16 square, 289 nodes, 867 unknowns, 32 steps of dt = 1/32."""
    return terzaghi_problem(16, 32)


def large_terzaghi() -> Problem:
    """256 x 256 square, 66,049 nodes, 198,147 unknowns, 512 steps of dt = 1/512."""
    return terzaghi_problem(256, 512)


def large_heterogeneous() -> Problem:
    """256 x 256 square, log-normal permeability, E ~ U[5e3, 2e4], 512 steps."""
    return heterogeneous_problem(256, 512)


def adjoint_problem(n: int = 128, n_steps: int = 256, field_seed: int = 40) -> Problem:
    """Gradient workload: consolidation column with a log-normal permeability
    field (the point where the gradient is taken) and homogeneous E, nu."""
    return terzaghi_problem(n, n_steps, perm=lognormal_perm_2d(n, field_seed))


def adjoint_reference_logk(n: int = 128, seed: int = 41) -> np.ndarray:
    """Log-permeability of the reference field that generates the observations."""
    return np.log(lognormal_perm_2d(n, seed))


def fd_directions(n_elems: int, count: int = 32, seed: int = 43):
    """Seeded directions (d log K, d lambda / lambda, d mu / mu) per element."""
    rng = np.random.default_rng(seed)
    return [(rng.standard_normal(n_elems), rng.standard_normal(n_elems),
             rng.standard_normal(n_elems)) for _ in range(count)]


def batched_samples(count: int = 64, seed: int = 3):
    """(grid n, n_steps, field seed) for independent samples of uneven size."""
    rng = np.random.default_rng(seed)
    sizes = rng.choice(np.array([32, 48, 64, 96, 128]), size=count)
    steps = rng.choice(np.arange(128, 513, 16), size=count)
    return [(int(sizes[i]), int(steps[i]), 3000 + i) for i in range(count)]


def sensor_nodes(problem: Problem, count: int = 64, seed: int = 42) -> np.ndarray:
    """Distinct nodes whose pressure is free (not on the drained face)."""
    free = np.nonzero((problem.flags & (1 << problem.dim)) == 0)[0]
    rng = np.random.default_rng(seed)
    return np.sort(rng.choice(free, size=count, replace=False)).astype(np.int32)


# ----------------------------------------------------------------------------
# manufactured solution of Sec. 4.1 (inputs: assembled loads, boundary values)
# ----------------------------------------------------------------------------
# Dunavant's symmetric 6-point rule on a triangle, exact for degree 4
# (D. A. Dunavant, Int. J. Numer. Meth. Eng. 21, 1985): barycentric points
# (a, a, 1-2a) and permutations, with a weight per orbit (weights sum to 1)
_DUN_ORBITS = ((0.445948490915965, 0.223381589678011),
               (0.091576213509771, 0.109951743655322))


def _dunavant_points():
    pts, wts = [], []
    for a, w in _DUN_ORBITS:
        b = 1.0 - 2.0 * a
        for bary in ((b, a, a), (a, b, a), (a, a, b)):
            pts.append(bary)
            wts.append(w)
    return np.array(pts), np.array(wts)


def mms_problem(n: int, dt: float, n_steps: int, E: float = 1.0, nu: float = 0.3,
                alpha: float = 1.0, K: float = 1.0) -> Problem:
    """Sec. 4.1 on the n x n unit square: exact solution
    u_1 = u_2 = p = cos(t) cos(3 pi x) cos(3 pi y), prescribed on the whole
    boundary (all three fields), E = 1, nu = 0.3, alpha = 1, K = 1.

    Right-hand side, per step n at t_n = n dt, as two load terms:
      term 0 (multiplier cos t_n): u rows int f_c . v with the body force
        f = cos t [k^2((lam+3mu) c_x c_y - (lam+mu) s_x s_y) - alpha k s_x c_y,
                   k^2((lam+3mu) c_x c_y - (lam+mu) s_x s_y) - alpha k c_x s_y]
        (k = 3 pi, c_x = cos 3 pi x, s_x = sin 3 pi x), and p rows -dt int g_c q
        with the cos-part of the source, g_c = 2 k^2 K c_x c_y;
      term 1 (multiplier sin t_n): p rows -dt int g_s q,
        g_s = alpha k (s_x c_y + c_x s_y).
    (g is the source that makes the printed solution exact; the printed one
    has the first bracket's sign and order changed.)  Prescribed values: one
    term cos(3 pi x) cos(3 pi y) in all fields with multiplier cos t_n; X^0 the
    exact solution at t = 0.
    """
    xyz, conn = square_mesh(n)
    nn = xyz.shape[0]
    tol = 1e-12
    bnd = ((xyz[:, 0] < tol) | (xyz[:, 0] > 1 - tol) | (xyz[:, 1] < tol) | (xyz[:, 1] > 1 - tol))
    flags = np.where(bnd, 0b111, 0).astype(np.uint8)
    lam = E * nu / ((1.0 + nu) * (1.0 - 2.0 * nu))
    mu = E / (2.0 * (1.0 + nu))
    k = 3.0 * np.pi
    bary, w = _dunavant_points()
    x = xyz[conn]                                           # [ne, 3, 2]
    d1, d2 = x[:, 1] - x[:, 0], x[:, 2] - x[:, 0]
    area = 0.5 * np.abs(d1[:, 0] * d2[:, 1] - d1[:, 1] * d2[:, 0])
    qp = np.einsum("qa,ead->eqd", bary, x)                  # [ne, nq, 2]
    cx, cy = np.cos(k * qp[..., 0]), np.cos(k * qp[..., 1])
    sx, sy = np.sin(k * qp[..., 0]), np.sin(k * qp[..., 1])
    common = k * k * ((lam + 3 * mu) * cx * cy - (lam + mu) * sx * sy)
    f1 = common - alpha * k * sx * cy
    f2 = common - alpha * k * cx * sy
    gc = 2 * k * k * K * cx * cy
    gs = alpha * k * (sx * cy + cx * sy)
    terms = np.zeros((2, nn, 3))
    wa = area[:, None] * w[None, :]                         # [ne, nq]
    for a in range(3):
        phi = wa * bary[None, :, a]
        v = conn[:, a]
        np.add.at(terms[0, :, 0], v, np.sum(phi * f1, axis=1))
        np.add.at(terms[0, :, 1], v, np.sum(phi * f2, axis=1))
        np.add.at(terms[0, :, 2], v, -dt * np.sum(phi * gc, axis=1))
        np.add.at(terms[1, :, 2], v, -dt * np.sum(phi * gs, axis=1))
    t = dt * np.arange(n_steps + 1)
    shape = np.cos(k * xyz[:, 0]) * np.cos(k * xyz[:, 1])
    pres = np.repeat(shape[None, :, None], 3, axis=2)       # [1, nn, 3]
    ne = conn.shape[0]
    return Problem(dim=2, grid_n=n, xyz=xyz, conn=conn, flags=flags,
                   young=np.full(ne, E), poisson=np.full(ne, nu), perm=np.full(ne, K),
                   alpha=alpha, stab_h=1.0 / n, facets=np.zeros((0, 2), np.int32),
                   traction=np.zeros((0, 2)), load_coef=np.zeros(n_steps + 1),
                   n_steps=n_steps, dt=dt,
                   terms=terms, term_coef=np.stack([np.cos(t), np.sin(t)], axis=1),
                   prescribed=pres, prescribed_coef=np.cos(t)[:, None],
                   x0=pres[0].copy())


def general_rhs_problem(n: int, n_steps: int, seed: int, dim: int = 2, n_terms: int = 2,
                        n_prescribed: int = 2) -> Problem:
    """Consolidation-column mesh, boundary flags and materials (log-normal K,
    uniform E in 2D) with a seeded general right-hand side: the unit top
    traction with its step profile, `n_terms` random load vectors (all dofs,
    scaled like the traction's loads and -dt times a pressure source) with
    random smooth multipliers, `n_prescribed` random prescribed-value vectors
    with random smooth multipliers, and a random initial state."""
    rng = np.random.default_rng(seed)
    if dim == 2:
        pb = heterogeneous_problem(n, n_steps, field_seed=seed + 1, young_seed=seed + 2)
    else:
        pb = terzaghi_problem(n, n_steps, dim=3)
    nn, d1 = pb.n_nodes, dim + 1
    h = 1.0 / n
    t = np.arange(n_steps + 1) / n_steps
    terms = rng.standard_normal((n_terms, nn, d1)) * h ** (dim - 1)
    terms[..., dim] *= pb.dt
    tc = np.stack([np.cos(rng.uniform(0, 6) * t + rng.uniform(0, 6)) for _ in range(n_terms)], 1)
    pres = rng.standard_normal((n_prescribed, nn, d1)) * 1e-4
    pres[..., dim] *= 1e4
    pc = np.stack([np.sin(rng.uniform(0, 6) * t + rng.uniform(0, 6)) for _ in range(n_prescribed)], 1)
    x0 = rng.standard_normal((nn, d1)) * 1e-4
    x0[:, dim] *= 1e4
    pb.terms, pb.term_coef = terms, tc
    pb.prescribed, pb.prescribed_coef = pres, pc
    pb.x0 = x0
    return pb
