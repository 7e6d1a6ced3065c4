"""GPU parity of GMRES(k) per unit (options.inner = GMRES) against the oracle.

* one Jacobi-order sweep and one wavefront pass of GMRES units from a random
  trajectory, element by element against oracle.krylov with the oracle's own
  multigrid block preconditioner (the Krylov processes are mathematically the
  same; rounding differs, so the bar is 1e-9 of the largest entry);
* converged solves reach backward Euler (<= 1e-8 per field) for both
  schedules, FP64 and the mixed-precision preconditioner;
* the adjoint and a batch with GMRES units.
"""
import numpy as np
import pytest
import torch

from oracle import adjoint as adj, fem, krylov, precond, sequential as seq
from paper_2310_10430_amd import workloads as W

pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("needs a ROCm GPU", allow_module_level=True)

from paper_2310_10430_amd.solver import BiotSolver  # noqa: E402


def _nm(X, orc):
    return fem.field_to_node_major(X, orc.n_nodes, orc.dim)


def _fm(Y):
    return fem.node_to_field_major(Y)


def _random_state(orc, ncols, seed):
    rng = np.random.default_rng(seed)
    X = rng.standard_normal((ncols, orc.n_dof))
    X[:, orc.fixed] = 0.0
    X[:, : orc.nU] *= 1e-4
    X[0] = 0.0
    return X


def _rel(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


@pytest.mark.parametrize("k", [1, 3])
def test_gmres_jacobi_sweep_matches_oracle(k):
    pb = W.heterogeneous_problem(16, 6)
    orc = seq.BiotOracle(pb)
    unit = krylov.GmresUnit(orc, precond.BlockPreconditioner(orc, "P1", "gmg"), k)
    X = _random_state(orc, pb.n_steps + 1, 4)
    s = BiotSolver(pb, schedule="jacobi", inner="gmres", gmres_k=k, max_batch=4)
    s.set_trajectory(torch.from_numpy(_nm(X, orc)))
    s.sweep(1)
    Xg = _fm(s.trajectory().cpu().numpy())
    s.close()
    Xo, _ = krylov.sweep(orc, X, unit, "jacobi")
    assert _rel(Xg[:, : orc.nU], Xo[:, : orc.nU]) < 1e-9
    assert _rel(Xg[:, orc.nU:], Xo[:, orc.nU:]) < 1e-9


def test_gmres_wavefront_pass_matches_oracle():
    pb = W.heterogeneous_problem(16, 7)
    orc = seq.BiotOracle(pb)
    unit = krylov.GmresUnit(orc, precond.BlockPreconditioner(orc, "P1", "gmg"), 2)
    X = _random_state(orc, pb.n_steps + 1, 5)
    s = BiotSolver(pb, schedule="wavefront", depth=3, inner="gmres", gmres_k=2)
    s.set_trajectory(torch.from_numpy(_nm(X, orc)))
    s.sweep(3)
    Xg = _fm(s.trajectory().cpu().numpy())
    s.close()
    Xo = krylov.wavefront(orc, X, unit, 3)
    assert _rel(Xg[:, : orc.nU], Xo[:, : orc.nU]) < 1e-9
    assert _rel(Xg[:, orc.nU:], Xo[:, orc.nU:]) < 1e-9


@pytest.mark.parametrize("schedule,precision,k", [("wavefront", "fp64", 4), ("jacobi", "fp64", 2),
                                                  ("wavefront", "mixed", 4)])
def test_gmres_solve_reaches_backward_euler(schedule, precision, k):
    pb = W.heterogeneous_problem(16, 24)
    orc = seq.BiotOracle(pb)
    Xs = orc.solve_sequential()
    s = BiotSolver(pb, schedule=schedule, depth=8, inner="gmres", gmres_k=k, precision=precision)
    st = s.solve_to_tol(1e-11, max_sweeps=400, check_every=2)
    Xg = _fm(s.trajectory().cpu().numpy())
    s.close()
    assert st["converged"]
    err = seq.relative_field_errors(Xg, Xs, orc.n_nodes, orc.dim)
    assert err["u"] < 1e-8 and err["p"] < 1e-8, (err, st)


def test_gmres_adjoint_and_batch():
    pb = W.heterogeneous_problem(12, 10)
    theta = adj.problem_params(pb)
    sens = W.sensor_nodes(pb, 6, seed=42)
    p_obs = adj.observations(pb, theta[0] + 0.4, sens)
    J, grads, _, _ = adj.objective_and_gradient(pb, *theta, sens, p_obs)
    s = BiotSolver(pb, schedule="wavefront", depth=6, inner="gmres", gmres_k=3, adjoint=True,
                   ckpt_stride=4, replay_segments=2)
    s.solve_to_tol(1e-11, max_sweeps=400)
    out = s.adjoint(sens, p_obs, rtol=1e-11, max_sweeps=400)
    s.close()
    for key, g in zip(("grad_logk", "grad_lambda", "grad_mu"), grads):
        assert _rel(out[key].cpu().numpy(), g) < 1e-8, key
    pbs = [W.heterogeneous_problem(12, N, field_seed=3000 + i) for i, N in enumerate((8, 11))]
    b = BiotSolver(pbs, schedule="wavefront", depth=6, inner="gmres", gmres_k=3)
    b.solve_to_tol(1e-11, max_sweeps=400)
    for i, q in enumerate(pbs):
        orc = seq.BiotOracle(q)
        err = seq.relative_field_errors(_fm(b.sample_trajectory(i).cpu().numpy()),
                                        orc.solve_sequential(), orc.n_nodes, orc.dim)
        assert err["u"] < 1e-8 and err["p"] < 1e-8, (i, err)
    b.close()
