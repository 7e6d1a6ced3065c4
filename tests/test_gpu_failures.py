"""Failure detection of the solve (numerical divergence, never a device fault):

* a damping omega far above 2 / lambda_max of P^{-1}AA makes the outer
  iteration grow; biot_solve_to_tol stops with BIOT_EDIVERGED (residual grown
  by more than 1e6, or non-finite), in both schedules, and reports the sweeps
  it did;
* a NaN placed in the iterate from the host (biot_set_trajectory) gives a
  non-finite residual at the first check: BIOT_EDIVERGED;
* afterwards the same process solves a well-posed problem normally.
A NaN in the load itself is refused at set-up (host test)."""
import numpy as np
import pytest
import torch

from paper_2310_10430_amd import workloads as W

pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("needs a ROCm GPU", allow_module_level=True)

from paper_2310_10430_amd.solver import BiotSolver  # noqa: E402

DEV = "cuda:0"
EDIVERGED = -4


@pytest.mark.parametrize("sched", ["jacobi", "wavefront"])
def test_omega_far_above_the_stability_limit_reports_divergence(sched):
    pb = W.small_terzaghi()
    s = BiotSolver(pb, schedule=sched, depth=8, omega=6.0, device=DEV)
    st = s.solve_to_tol(1e-12, max_sweeps=2000, check_every=4, raise_on_failure=False)
    msg = s.lib.biot_last_error(s.h).decode()
    s.close()
    assert st["rc"] == EDIVERGED, (st, msg)
    assert "grew" in msg or "non-finite" in msg
    assert 0 < st["sweeps"] < 2000


def test_nan_in_the_iterate_reports_divergence():
    pb = W.small_terzaghi()
    s = BiotSolver(pb, schedule="jacobi", omega=0.6, device=DEV)
    X = torch.zeros((pb.n_steps + 1, pb.n_nodes, 3), dtype=torch.float64, device=DEV)
    X[5, 40, 1] = float("nan")
    s.set_trajectory(X)
    st = s.solve_to_tol(1e-12, max_sweeps=100, raise_on_failure=False)
    msg = s.lib.biot_last_error(s.h).decode()
    s.close()
    assert st["rc"] == EDIVERGED and "non-finite" in msg, (st, msg)
    assert st["sweeps"] == 0


def test_solve_after_a_divergent_one_is_normal():
    pb = W.small_terzaghi()
    s = BiotSolver(pb, schedule="jacobi", omega=6.0, device=DEV)
    s.solve_to_tol(1e-12, max_sweeps=400, raise_on_failure=False)
    s.close()
    s = BiotSolver(pb, schedule="wavefront", depth=8, omega=0.6, device=DEV)
    st = s.solve_to_tol(1e-11, max_sweeps=400)
    X = s.trajectory().cpu().numpy()
    s.close()
    assert st["converged"] and np.isfinite(X).all()
