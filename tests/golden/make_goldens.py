"""Writes the stored expected values under tests/golden/ (calls only oracle/).

large_terzaghi.npz -- 256 x 256 consolidation column, 512 steps of dt = 1/512
(66,049 nodes, 198,147 unknowns), sequential backward Euler with the scaled
SuperLU solve and one refinement step per step:
    norm_u[n], norm_p[n]   ||U^n||_2, ||P^n||_2 for n = 0..512
    dofs[k]                node-major dof indices of 256 sampled free unknowns
                           (numpy default_rng(7), without replacement)
    samples[n, k]          X^n at those dofs

large_heterogeneous.npz -- the same mesh and steps with a log-normal
permeability field (sigma_log = 1, correlation length 0.1, field seed 2) and
E ~ U[5e3, 2e4] per element (seed 102); same contents.

adjoint_c4.npz -- gradient workload: 128 x 128 consolidation column, 256 steps
of dt = 1/256, log-normal permeability (field seed 40) where the gradient is
taken, homogeneous E = 1e4, nu = 0.3; 64 sensor nodes with free pressure
(seed 42); observations from the forward run with the reference field (seed 41):
    sensors[64], p_obs[256, 64]   objective data
    J                             objective at the evaluation point
    grad_logk, grad_lambda, grad_mu [32768]   oracle discrete adjoint
    fd[32]                        central differences, h = 1e-6, of J along the
                                  seeded directions (seed 43): d log K = v_k,
                                  d lambda = lambda v_l, d mu = mu v_m
    fd_scale[32]                  sum_i |g_i v_i| of each direction

Run:  python tests/golden/make_goldens.py [large_terzaghi] [large_heterogeneous] [adjoint_c4]
      (about 2 minutes each on one core; adjoint_c4 uses a process pool)
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from paper_2310_10430_amd import workloads as W  # noqa: E402
from oracle import adjoint as adj, fem, sequential as seq  # noqa: E402


def write(name, pb):
    t0 = time.time()
    orc = seq.BiotOracle(pb)
    X = orc.solve_sequential()
    Y = orc.trajectory_node_major(X)           # [513, nn, 3]
    nn, d1 = Y.shape[1], Y.shape[2]
    flat = Y.reshape(Y.shape[0], -1)
    fixed_nm = fem.field_to_node_major(orc.fixed.astype(float), nn, 2).reshape(-1) > 0.5
    free = np.nonzero(~fixed_nm)[0]
    dofs = np.sort(np.random.default_rng(7).choice(free, size=256, replace=False))
    np.savez_compressed(
        os.path.join(HERE, name + ".npz"),
        norm_u=np.linalg.norm(Y[..., :2].reshape(Y.shape[0], -1), axis=1),
        norm_p=np.linalg.norm(Y[..., 2], axis=1),
        dofs=dofs.astype(np.int64), samples=flat[:, dofs])
    print(f"{name}.npz written in {time.time() - t0:.1f} s")


def _fd_one(args):
    pb, theta, sensors, p_obs, v, h = args
    (logk, lam, mu), (vk, vl, vm) = theta, v
    jp = adj.objective_value(pb, logk + h * vk, lam + h * lam * vl, mu + h * mu * vm, sensors, p_obs)
    jm = adj.objective_value(pb, logk - h * vk, lam - h * lam * vl, mu - h * mu * vm, sensors, p_obs)
    return (jp - jm) / (2 * h)


def write_adjoint(name="adjoint_c4", workers=6):
    from multiprocessing import Pool
    t0 = time.time()
    pb = W.adjoint_problem()
    theta = adj.problem_params(pb)
    sensors = W.sensor_nodes(pb, 64, seed=42)
    p_obs = adj.observations(pb, W.adjoint_reference_logk(), sensors)
    J, (gk, gl, gm), _, _ = adj.objective_and_gradient(pb, *theta, sensors, p_obs)
    print(f"  gradient in {time.time() - t0:.1f} s", flush=True)
    dirs = W.fd_directions(pb.n_elems, 32, seed=43)
    with Pool(workers) as pool:
        fd = pool.map(_fd_one, [(pb, theta, sensors, p_obs, v, 1e-6) for v in dirs])
    lam, mu = theta[1], theta[2]
    scale = [np.abs(gk * vk).sum() + np.abs(gl * lam * vl).sum() + np.abs(gm * mu * vm).sum()
             for vk, vl, vm in dirs]
    np.savez_compressed(os.path.join(HERE, name + ".npz"), sensors=sensors, p_obs=p_obs,
                        J=np.float64(J), grad_logk=gk, grad_lambda=gl, grad_mu=gm,
                        fd=np.asarray(fd), fd_scale=np.asarray(scale))
    print(f"{name}.npz written in {time.time() - t0:.1f} s")


WORKLOADS = {"large_terzaghi": W.large_terzaghi, "large_heterogeneous": W.large_heterogeneous}

if __name__ == "__main__":
    for name in (sys.argv[1:] or list(WORKLOADS) + ["adjoint_c4"]):
        if name == "adjoint_c4":
            write_adjoint()
        else:
            write(name, WORKLOADS[name]())
