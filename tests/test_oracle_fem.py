"""Pins of the oracle's finite-element assembly (stabilized P1-P1, Sec. 2.2).

Every check here is fixed by mathematics independent of the oracle's own
formulas: closed-form stencils, rigid-body null spaces, the divergence theorem,
the Voigt form of the elasticity matrix, and load totals.
"""
import numpy as np
import pytest

from paper_2310_10430_amd import workloads as W
from oracle import fem


def test_square_mesh_counts_and_area():
    xyz, conn = W.square_mesh(16)
    assert xyz.shape == (289, 2) and conn.shape == (512, 3)
    g, vol = fem.simplex_gradients(xyz, conn)
    assert np.all(vol > 0)
    assert abs(vol.sum() - 1.0) < 1e-14


def test_cube_mesh_counts_and_volume():
    xyz, conn = W.cube_mesh(4)
    assert xyz.shape == (125, 3) and conn.shape == (384, 4)
    g, vol = fem.simplex_gradients(xyz, conn)
    assert np.all(vol > 0)
    assert abs(vol.sum() - 1.0) < 1e-13
    # conforming: every interior face is shared by exactly two tets
    faces = np.sort(np.concatenate([conn[:, [0, 1, 2]], conn[:, [0, 1, 3]],
                                    conn[:, [0, 2, 3]], conn[:, [1, 2, 3]]]), axis=1)
    _, counts = np.unique(faces, axis=0, return_counts=True)
    assert set(counts.tolist()) <= {1, 2}
    n_boundary = (counts == 1).sum()
    assert n_boundary == 6 * 2 * 16   # 6 faces x 16 squares x 2 triangles


def test_lame_parameters():
    lam, mu = fem.lame(1e4, 0.3)
    # E nu / ((1+nu)(1-2nu)) and E / (2(1+nu)) for E = 1e4, nu = 0.3
    assert abs(lam - 5769.230769230769) < 1e-9
    assert abs(mu - 3846.153846153846) < 1e-9


def test_laplacian_is_five_point_stencil():
    """P1 Laplacian on the right-triangle grid: interior row = (4, -1, -1, -1, -1)
    in the axis directions and exactly zero along the diagonal."""
    n = 8
    pb = W.terzaghi_problem(n, 4, perm=1.0)
    asm = fem.assemble(pb)
    C = asm.CK.toarray()
    m = n + 1
    for (i, j) in [(3, 3), (4, 5), (1, 6)]:
        r = j * m + i
        assert abs(C[r, r] - 4.0) < 1e-13
        for (di, dj) in [(1, 0), (-1, 0), (0, 1), (0, -1)]:
            assert abs(C[r, (j + dj) * m + i + di] + 1.0) < 1e-13
        assert abs(C[r, (j + 1) * m + i + 1]) < 1e-13
        assert abs(C[r, (j - 1) * m + i - 1]) < 1e-13
        assert abs(C[r].sum()) < 1e-13


@pytest.mark.parametrize("dim", [2, 3])
def test_rigid_modes_null_space(dim):
    n = 4 if dim == 3 else 6
    pb = W.terzaghi_problem(n, 2, dim=dim, young=np.random.default_rng(1).uniform(1, 3, 6 * n ** 3 if dim == 3 else 2 * n * n))
    asm = fem.assemble(pb)
    x = pb.xyz
    modes = []
    for c in range(dim):
        v = np.zeros_like(x)
        v[:, c] = 1.0
        modes.append(v)
    if dim == 2:
        modes.append(np.stack([-x[:, 1], x[:, 0]], axis=1))
    else:
        modes.append(np.stack([-x[:, 1], x[:, 0], 0 * x[:, 0]], axis=1))
        modes.append(np.stack([0 * x[:, 0], -x[:, 2], x[:, 1]], axis=1))
        modes.append(np.stack([x[:, 2], 0 * x[:, 0], -x[:, 0]], axis=1))
    scale = abs(asm.A).max()
    for v in modes:
        u = v.ravel()
        assert np.abs(asm.A @ u).max() < 1e-12 * scale
        assert np.abs(asm.B.T @ u).max() < 1e-14     # rigid motions are divergence free
    assert np.abs(asm.CK @ np.ones(pb.n_nodes)).max() < 1e-13
    assert np.abs(asm.Cb @ np.ones(pb.n_nodes)).max() < 1e-13 * abs(asm.Cb).max()


def test_divergence_theorem_for_coupling():
    """sum_i b(u, phi_i) = alpha int div u = alpha * (boundary flux of u);
    B' u = -(b(u, phi_i))_i."""
    pb = W.terzaghi_problem(8, 2, alpha=0.7)
    asm = fem.assemble(pb)
    x = pb.xyz
    u = np.stack([x[:, 0] ** 1, 0 * x[:, 1]], axis=1).ravel()      # div u = 1
    assert abs((asm.B.T @ u).sum() + 0.7) < 1e-13
    u2 = np.stack([x[:, 0] * x[:, 1], x[:, 1]], axis=1).ravel()   # flux: int_{x=1} y + int_{y=1} 1
    assert abs((asm.B.T @ u2).sum() + 0.7 * 1.5) < 1e-13


def test_divergence_theorem_for_coupling_3d():
    pb = W.terzaghi_problem(4, 2, dim=3, alpha=0.7)
    asm = fem.assemble(pb)
    x = pb.xyz
    u = np.stack([0 * x[:, 0], x[:, 1], 0 * x[:, 2]], axis=1).ravel()      # div u = 1
    assert abs((asm.B.T @ u).sum() + 0.7) < 1e-13
    # u = (x z, 0, y): div u = z, int_cube z = 1/2
    u2 = np.stack([x[:, 0] * x[:, 2], 0 * x[:, 1], x[:, 1]], axis=1).ravel()
    assert abs((asm.B.T @ u2).sum() + 0.7 * 0.5) < 1e-13


def test_elasticity_matches_voigt_form():
    """Element matrix equals vol * Bv' D Bv with the plane-strain Voigt matrices."""
    rng = np.random.default_rng(3)
    xyz = rng.uniform(size=(3, 2))
    conn = np.array([[0, 1, 2]])
    if np.linalg.det(np.stack([xyz[1] - xyz[0], xyz[2] - xyz[0]], 1)) < 0:
        conn = conn[:, [0, 2, 1]]
    g, vol = fem.simplex_gradients(xyz, conn)
    lam, mu = np.array([2.0]), np.array([0.7])
    K = fem.element_elasticity(g, vol, lam, mu)[0]
    Bv = np.zeros((3, 6))
    for a in range(3):
        Bv[0, 2 * a] = g[0, a, 0]
        Bv[1, 2 * a + 1] = g[0, a, 1]
        Bv[2, 2 * a] = g[0, a, 1]
        Bv[2, 2 * a + 1] = g[0, a, 0]
    D = np.array([[lam[0] + 2 * mu[0], lam[0], 0], [lam[0], lam[0] + 2 * mu[0], 0], [0, 0, mu[0]]])
    assert np.allclose(K, vol[0] * Bv.T @ D @ Bv, rtol=0, atol=1e-13)


def test_top_load_total():
    for dim, n in [(2, 16), (3, 4)]:
        pb = W.terzaghi_problem(n, 2, dim=dim)
        F = fem.traction_load(pb).reshape(-1, dim)
        assert abs(F[:, dim - 1].sum() + 1.0) < 1e-13
        assert np.abs(F[:, : dim - 1]).max() == 0.0


def test_matrices_symmetric():
    pb = W.heterogeneous_problem(16, 4)
    asm = fem.assemble(pb)
    AA, Ap = fem.block_system(asm, 0.01)
    assert abs(AA - AA.T).max() < 1e-12 * abs(AA).max()


def test_stabilization_parameter():
    """beta_e = alpha^2 h^2 / (4 (lambda_e + 2 mu_e)) with h the grid step."""
    pb = W.terzaghi_problem(16, 2, alpha=1.0)
    asm = fem.assemble(pb)
    lam, mu = fem.lame(1e4, 0.3)
    assert np.allclose(asm.beta, (1 / 16) ** 2 / (4 * (lam + 2 * mu)), rtol=1e-14)
