"""GPU parity of batched solves (biot_create_batch): several samples on one mesh,
with their own permeability fields, moduli, step counts and step sizes, solved
together in every launch.

* each sample of the batch against its own oracle (sequential backward Euler),
  <= 1e-8 per field, for both schedules and the mixed-precision preconditioner;
* the batch against the same samples solved one handle at a time;
* 3D samples;
* the per-sample residual norms match the single-sample ones;
* handles of several mesh sizes solved concurrently, each on a stream of its
  own, match the same handles solved one after another, bit for bit.
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


def _samples(n=16, steps=(12, 20, 16, 7), dim=2):
    if dim == 2:
        return [W.heterogeneous_problem(n, N, field_seed=3000 + i, young_seed=4000 + i)
                for i, N in enumerate(steps)]
    out = []
    for i, N in enumerate(steps):
        pb = W.terzaghi_problem(n, N, dim=3)
        pb.perm = pb.perm * np.exp(0.5 * np.random.default_rng(3000 + i).standard_normal(pb.n_elems))
        out.append(pb)
    return out


def _check_samples(s, pbs, tol=1e-8):
    for i, pb in enumerate(pbs):
        orc = seq.BiotOracle(pb)
        Xs = orc.solve_sequential()
        Xg = fem.node_to_field_major(s.sample_trajectory(i).cpu().numpy())
        assert Xg.shape == Xs.shape
        err = seq.relative_field_errors(Xg, Xs, orc.n_nodes, orc.dim)
        assert err["u"] < tol and err["p"] < tol, (i, err)


@pytest.mark.parametrize("schedule,depth,precision", [("wavefront", 8, "fp64"),
                                                      ("jacobi", 1, "fp64"),
                                                      ("wavefront", 8, "mixed")])
def test_batch_matches_oracle_per_sample(schedule, depth, precision):
    pbs = _samples()
    print(f"batch of {len(pbs)} samples, {schedule}, {precision}", flush=True)
    s = BiotSolver(pbs, schedule=schedule, depth=depth, precision=precision, max_batch=9)
    st = s.solve_to_tol(1e-11, max_sweeps=2000, check_every=4)
    assert st["converged"]
    _check_samples(s, pbs)
    s.close()


def test_batch_agrees_with_single_handles():
    pbs = _samples(n=16, steps=(10, 14, 6))
    s = BiotSolver(pbs, schedule="wavefront", depth=8)
    s.solve_to_tol(1e-12, max_sweeps=2000)
    for i, pb in enumerate(pbs):
        t = BiotSolver(pb, schedule="wavefront", depth=8)
        t.solve_to_tol(1e-12, max_sweeps=2000)
        a = s.sample_trajectory(i).cpu().numpy()
        b = t.trajectory().cpu().numpy()
        t.close()
        for sl in (slice(0, 2), slice(2, 3)):
            assert np.abs(a[..., sl] - b[..., sl]).max() <= 1e-9 * np.abs(b[..., sl]).max()
    s.close()


def test_batch_3d():
    pbs = _samples(n=4, steps=(6, 4), dim=3)
    s = BiotSolver(pbs, schedule="wavefront", depth=4)
    st = s.solve_to_tol(1e-11, max_sweeps=2000)
    assert st["converged"]
    _check_samples(s, pbs)
    s.close()


def test_batch_residual_norms_per_sample():
    pbs = _samples(n=8, steps=(6, 9))
    s = BiotSolver(pbs, schedule="jacobi")
    s.sweep(5)
    nb = s.residual_norms()
    assert nb.shape == (9, 2, 4)
    for i, pb in enumerate(pbs):
        t = BiotSolver(pb, schedule="jacobi")
        t.sweep(5)
        ns = t.residual_norms()
        t.close()
        # identical sweeps except for the smoothers' common spectral bound
        assert np.all(np.isfinite(nb[:, i]))
        np.testing.assert_allclose(nb[: pb.n_steps, i, 2], ns[:, 2], rtol=1e-12)  # ||b_u||^2
    s.close()


def test_concurrent_handles_on_own_streams_match_sequential():
    # handles of different mesh sizes, each bound to a stream of its own and
    # driven by a host thread of its own, give the same trajectories bit for bit
    from paper_2310_10430_amd import autotune
    groups = []
    for n, steps in ((8, (6, 9)), (12, (5, 7, 4)), (16, (8,))):
        groups.append([(len(sum(groups, [])) + k, W.heterogeneous_problem(n, N, field_seed=50 + k))
                       for k, N in enumerate(steps)])
    _, st_a, a = autotune.solve_groups(groups, 1e-11, "fp64", depth=4, keep=True)
    _, st_b, b = autotune.solve_groups(groups, 1e-11, "fp64", depth=4, keep=True, concurrent=True)
    assert [x["sweeps"] for x in st_a] == [x["sweeps"] for x in st_b]
    assert sorted(a) == sorted(b)
    for i in a:
        assert torch.equal(a[i], b[i]), i
    # and the concurrent trajectories are the backward-Euler ones
    for g in groups:
        for i, pb in g:
            orc = seq.BiotOracle(pb)
            err = seq.relative_field_errors(fem.node_to_field_major(b[i].cpu().numpy()),
                                            orc.solve_sequential(), orc.n_nodes, orc.dim)
            assert err["u"] < 1e-8 and err["p"] < 1e-8, (i, err)
