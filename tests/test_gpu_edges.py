"""GPU edge cases of the inverted iteration against the oracle's sequential
backward Euler (<= 1e-8 per field), through the C ABI:

* a single time step (no coupling to a previous iterate of the sweep);
* a wavefront deeper than the number of steps (every wave partial);
* the smallest grid, 2 x 2 cells, where the multigrid hierarchy is one level
  (the preconditioner is the dense coarsest solve);
* an odd grid whose hierarchy ends on an odd coarsest level (12 -> 6 -> 3);
* Jacobi batches that do not divide the step count (ragged last launch);
* a zero load: the zero trajectory is the exact solution and is reached at
  once, with a finite residual;
* a one-sample batch through the batch entry point equals the single handle;
* eight copies of one sample in a batch, whose tail launches take 256-thread
  workgroups, equal the single handle (1024-thread tails) bit for bit;
* smoother degree 3, where the stored increment d is used between steps;
* the fused two-step post-smoothing against the two separate steps
  (options.fuse_post = 0), bit for bit, for a single sample and for a batch;
* a single-level 3D hierarchy whose dense coarsest solve is large enough that
  fewer right-hand sides fit one workgroup's LDS (4 and 2 columns per group,
  with ragged last groups), against the oracle's preconditioner, and the same
  hierarchy in a two-sample batch against the oracle.
"""
import numpy as np
import pytest
import torch

from oracle import fem, sequential as seq
from paper_2310_10430_amd import workloads as W

pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("needs a ROCm GPU", allow_module_level=True)

from paper_2310_10430_amd.solver import BiotSolver  # noqa: E402


def _fm(Y):
    return fem.node_to_field_major(Y)


def _solve_and_check(pb, rtol=1e-11, max_sweeps=600, **kw):
    orc = seq.BiotOracle(pb)
    Xs = orc.solve_sequential()
    s = BiotSolver(pb, **kw)
    st = s.solve_to_tol(rtol, max_sweeps=max_sweeps, check_every=2)
    Xg = _fm(s.trajectory().cpu().numpy())
    s.close()
    assert st["converged"], st
    err = seq.relative_field_errors(Xg, Xs, orc.n_nodes, orc.dim)
    assert err["u"] < 1e-8 and err["p"] < 1e-8, (err, st)
    return st


@pytest.mark.parametrize("schedule,precision", [("jacobi", "fp64"), ("wavefront", "fp64"),
                                                ("wavefront", "mixed")])
def test_single_step(schedule, precision):
    _solve_and_check(W.heterogeneous_problem(16, 1), schedule=schedule, depth=4,
                     precision=precision)


def test_wavefront_deeper_than_steps():
    _solve_and_check(W.heterogeneous_problem(12, 3), schedule="wavefront", depth=16)


@pytest.mark.parametrize("schedule", ["jacobi", "wavefront"])
def test_smallest_grid_single_level(schedule):
    st = _solve_and_check(W.terzaghi_problem(2, 6), schedule=schedule, depth=4)
    assert st["sweeps"] > 0


def test_odd_coarsest_level():
    pb = W.heterogeneous_problem(12, 5, field_seed=11, young_seed=12)
    _solve_and_check(pb, schedule="wavefront", depth=4)


@pytest.mark.parametrize("max_batch", [1, 5])
def test_ragged_jacobi_batches(max_batch):
    _solve_and_check(W.heterogeneous_problem(16, 12), schedule="jacobi", max_batch=max_batch)


@pytest.mark.parametrize("schedule", ["jacobi", "wavefront"])
def test_zero_load_stays_zero(schedule):
    pb = W.terzaghi_problem(8, 6, load=0.0)
    s = BiotSolver(pb, schedule=schedule, depth=4)
    st = s.solve_to_tol(1e-11, max_sweeps=40, check_every=2)
    X = s.trajectory().cpu().numpy()
    s.close()
    assert st["converged"] and np.isfinite(st["rel_resid_u"]) and np.isfinite(st["rel_resid_p"])
    assert np.abs(X).max() == 0.0


def test_one_sample_batch_equals_single_handle():
    pb = W.heterogeneous_problem(16, 7)
    a = BiotSolver(pb, schedule="wavefront", depth=4)
    b = BiotSolver([pb], schedule="wavefront", depth=4)
    a.sweep(8)
    b.sweep(8)
    Xa = a.trajectory().cpu().numpy()
    Xb = b.sample_trajectory(0).cpu().numpy()
    a.close()
    b.close()
    assert np.array_equal(Xa, Xb)


def test_batch_tail_with_small_workgroups_equals_single_handle():
    """Eight copies of one sample with 32 columns per full wave launch 256 tail
    workgroups, enough for the tail's 256-thread instantiation; the sample
    alone (32 per launch) takes the 1024-thread one.  Same arithmetic (and the
    same smoother bounds: a batch takes the largest of its samples'): every
    copy equals the single handle bit for bit.  (Samples that differ share
    the batch's bounds and so differ from their single handles.)"""
    pb = W.heterogeneous_problem(16, 40, field_seed=50, young_seed=60)
    b = BiotSolver([pb] * 8, schedule="wavefront", depth=32)
    b.sweep(32)
    Xb = [b.sample_trajectory(i).cpu().numpy() for i in range(8)]
    b.close()
    a = BiotSolver(pb, schedule="wavefront", depth=32)
    a.sweep(32)
    Xa = a.trajectory().cpu().numpy()
    a.close()
    for i in range(8):
        assert np.array_equal(Xa, Xb[i]), i


@pytest.mark.parametrize("schedule", ["jacobi", "wavefront"])
def test_smoother_degree_three(schedule):
    _solve_and_check(W.heterogeneous_problem(16, 6), schedule=schedule, depth=4, cheb_degree=3)


@pytest.mark.parametrize("degree", [3, 4])
def test_preconditioner_higher_smoother_degree_matches_oracle(degree):
    from oracle import precond
    pb = W.heterogeneous_problem(24, 3)
    orc = seq.BiotOracle(pb)
    P = precond.BlockPreconditioner(orc, "P1", "gmg", degree=degree)
    rng = np.random.default_rng(8)
    R = rng.standard_normal((5, orc.n_dof))
    R[:, orc.fixed] = 0.0
    R[:, orc.nU:] *= 1e-6
    s = BiotSolver(pb, cheb_degree=degree, max_batch=3)   # batches of 3 + 2
    Z = _fm(s.apply_precond(torch.from_numpy(fem.field_to_node_major(R, orc.n_nodes, orc.dim)))
            .cpu().numpy())
    s.close()
    for c in range(R.shape[0]):
        Zo = P.apply(R[c])
        for sl in (slice(0, orc.nU), slice(orc.nU, None)):
            assert np.abs(Z[c, sl] - Zo[sl]).max() < 1e-11 * np.abs(Zo[sl]).max()


@pytest.mark.parametrize("n,coarse_cells", [(7, 2), (8, 8)])
def test_preconditioner_large_dense_coarsest_level_matches_oracle(n, coarse_cells):
    # one level: 512 nodes (1536 displacement dofs, 4 columns per workgroup) or
    # 729 nodes (2187 dofs, 2 per workgroup); 11 columns leave ragged groups
    from oracle import precond
    pb = W.terzaghi_problem(n, 3, dim=3)
    pb.perm = pb.perm * np.exp(0.5 * np.random.default_rng(n).standard_normal(pb.n_elems))
    orc = seq.BiotOracle(pb)
    P = precond.BlockPreconditioner(orc, "P1", "gmg", min_cells=coarse_cells)
    rng = np.random.default_rng(9)
    R = rng.standard_normal((11, orc.n_dof))
    R[:, orc.fixed] = 0.0
    R[:, orc.nU:] *= 1e-6
    s = BiotSolver(pb, coarse_cells=coarse_cells, max_batch=11)
    assert s.info()["n_levels"] == 1
    Z = _fm(s.apply_precond(torch.from_numpy(fem.field_to_node_major(R, orc.n_nodes, orc.dim)))
            .cpu().numpy())
    s.close()
    for c in range(R.shape[0]):
        Zo = P.apply(R[c])
        for sl in (slice(0, orc.nU), slice(orc.nU, None)):
            assert np.abs(Z[c, sl] - Zo[sl]).max() < 1e-11 * np.abs(Zo[sl]).max()


def test_batch_with_large_dense_coarsest_level_matches_oracle():
    # two copies of the single-level 512-node hierarchy: one coarsest solve per copy
    pbs = []
    for i, N in enumerate((5, 8)):
        pb = W.terzaghi_problem(7, N, dim=3)
        pb.perm = pb.perm * np.exp(0.5 * np.random.default_rng(70 + i).standard_normal(pb.n_elems))
        pbs.append(pb)
    s = BiotSolver(pbs, schedule="wavefront", depth=4)
    st = s.solve_to_tol(1e-11, max_sweeps=600, check_every=2)
    assert st["converged"], st
    for i, pb in enumerate(pbs):
        orc = seq.BiotOracle(pb)
        Xs = orc.solve_sequential()
        Xg = _fm(s.sample_trajectory(i).cpu().numpy())
        err = seq.relative_field_errors(Xg, Xs, orc.n_nodes, orc.dim)
        assert err["u"] < 1e-8 and err["p"] < 1e-8, (i, err)
    s.close()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_fused_post_smoothing_equals_separate_steps(precision):
    # both post-smoothing steps of each level in one launch against two launches
    pb = W.heterogeneous_problem(40, 9, field_seed=17, young_seed=18)
    for probs in (pb, [pb, W.heterogeneous_problem(40, 6, field_seed=19, young_seed=20)]):
        out = []
        for fuse in (True, False):
            s = BiotSolver(probs, schedule="wavefront", depth=4, precision=precision,
                           fuse_post=fuse)
            s.sweep(7)
            if isinstance(probs, list):
                out.append([s.sample_trajectory(i).cpu().numpy() for i in range(len(probs))])
            else:
                out.append([s.trajectory().cpu().numpy()])
            s.close()
        for x, y in zip(*out):
            assert np.array_equal(x, y)
