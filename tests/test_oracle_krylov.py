"""Pins of the oracle's GMRES(k) unit (CPU only).

* with k equal to the system size, GMRES returns the solution of the system;
* for k below it, the result is the minimizer of ||P^{-1}(b - A x)|| over
  x0 + span{s0, (P^{-1}A) s0, ...} with s0 = P^{-1} r0, computed independently
  from the explicit Krylov matrix with numpy's least squares;
* GMRES units in the inverted iteration converge to backward Euler, in fewer
  sweeps than the damped Richardson units.
"""
import numpy as np

from oracle import inverted, krylov, precond, sequential as seq
from paper_2310_10430_amd import workloads as W


def _system(n=12, seed=0):
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((n, n)) + n * np.eye(n)
    M = rng.standard_normal((n, n)) * 0.3 + np.eye(n)       # a nonsymmetric preconditioner
    b = rng.standard_normal(n)
    x0 = rng.standard_normal(n)
    return A, M, b, x0


def test_full_dimension_gmres_solves_exactly():
    A, M, b, x0 = _system()
    Minv = np.linalg.inv(M)
    x = krylov.gmres_left(lambda v: A @ v, lambda v: Minv @ v, b, x0, k=12)
    np.testing.assert_allclose(x, np.linalg.solve(A, b), rtol=1e-10, atol=1e-12)


def test_gmres_is_the_krylov_least_squares_minimizer():
    # spectrum near 1 keeps the explicit (monomial) Krylov basis well conditioned
    n = 20
    rng = np.random.default_rng(3)
    A = np.eye(n) + 0.5 * rng.standard_normal((n, n)) / np.sqrt(n)
    M = np.eye(n) + 0.2 * rng.standard_normal((n, n)) / np.sqrt(n)
    b = rng.standard_normal(n)
    x0 = rng.standard_normal(n)
    Minv = np.linalg.inv(M)
    k = 5
    x = krylov.gmres_left(lambda v: A @ v, lambda v: Minv @ v, b, x0, k)
    s0 = Minv @ (b - A @ x0)
    cols, v = [], s0.copy()
    for _ in range(k):
        cols.append(v)
        v = Minv @ (A @ v)
    Kmat = np.stack(cols, axis=1)               # [s0, P^{-1}A s0, ...]
    c = np.linalg.lstsq(Minv @ A @ Kmat, s0, rcond=None)[0]
    x_ref = x0 + Kmat @ c
    np.testing.assert_allclose(x, x_ref, rtol=1e-9, atol=1e-12)
    assert np.linalg.norm(Minv @ (b - A @ x)) <= np.linalg.norm(s0)


def test_gmres_units_converge_to_backward_euler():
    pb = W.heterogeneous_problem(8, 10)
    orc = seq.BiotOracle(pb)
    Xs = orc.solve_sequential()
    P = precond.BlockPreconditioner(orc, "P1", "gmg")
    unit = krylov.GmresUnit(orc, P, k=4)
    X = np.zeros_like(Xs)
    sweeps_gmres = None
    for m in range(1, 60):
        X, nrm = krylov.sweep(orc, X, unit)
        if inverted.relative_residual(nrm) < 1e-11:
            sweeps_gmres = m
            break
    err = seq.relative_field_errors(X, Xs, orc.n_nodes, orc.dim)
    assert sweeps_gmres is not None and err["u"] < 1e-8 and err["p"] < 1e-8
    # the damped Richardson unit needs more outer sweeps to the same residual
    Y = np.zeros_like(Xs)
    for m in range(1, sweeps_gmres + 1):
        Y, nrm = inverted.sweep(orc, Y, P, omega=0.6)
    assert inverted.relative_residual(nrm) > 1e-11
