"""Writes the stored expected values under tests/golden/ (calls only oracle/).

large_terzaghi.npz -- 256 x 256 consolidation column, 512 steps of dt = 1/512
(66,049 nodes, 198,147 unknowns), sequential backward Euler with the scaled
SuperLU solve and one refinement step per step:
    norm_u[n], norm_p[n]   ||U^n||_2, ||P^n||_2 for n = 0..512
    dofs[k]                node-major dof indices of 256 sampled free unknowns
                           (numpy default_rng(7), without replacement)
    samples[n, k]          X^n at those dofs

cube40.npz -- 40^3 unit cube on Kuhn tetrahedra (68,921 nodes, 275,684
unknowns), 256 steps of dt = 1/256, homogeneous materials, the 3D column;
same contents (dofs index the node-major [nn][4] layout).

large_terzaghi_dt32.npz, large_terzaghi_dt0.1.npz -- the 256 x 256 column with
512 steps of dt = 1/32 and of dt = 0.1 (the larger time steps where the block
preconditioners P1 and P2 are compared, Table 3's regime); same contents.

large_heterogeneous.npz -- the same mesh and steps with a log-normal
permeability field (sigma_log = 1, correlation length 0.1, field seed 2) and
E ~ U[5e3, 2e4] per element (seed 102); same contents.

batched64.npz -- the 64 samples of the batched workload (grid n, steps and
field seed from workloads.batched_samples(64, seed=3); log-normal permeability
with field seed 3000+i and E ~ U[5e3, 2e4] with seed 4000+i), each solved by
the sequential oracle:
    grid_n[64], n_steps[64], offsets[65]   sample i's rows are
                                           offsets[i] .. offsets[i+1]-1 (steps 0..N_i)
    norm_u, norm_p                         ||U^n||_2, ||P^n||_2 per sample and step
    dofs[64, 8]                            sampled free unknowns of each sample
                                           (numpy default_rng(100 + i))
    samples[rows, 8]                       X^n at those unknowns
    amax_u[64], amax_p[64]                 largest |u| and |p| of each sample's trajectory
                                           (the scale of its relative errors)

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

Run:  python tests/golden/make_goldens.py [large_terzaghi] [large_terzaghi_dt32]
        [large_terzaghi_dt0.1] [large_heterogeneous] [cube40] [batched64] [adjoint_c4]
      (about 2 minutes each on one core; cube40's 3D factorization takes far longer;
      batched64 and adjoint_c4 use a process pool)
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
    Y = orc.trajectory_node_major(X)           # [N+1, nn, dim+1]
    nn, dim = Y.shape[1], Y.shape[2] - 1
    flat = Y.reshape(Y.shape[0], -1)
    fixed_nm = fem.field_to_node_major(orc.fixed.astype(float), nn, dim).reshape(-1) > 0.5
    free = np.nonzero(~fixed_nm)[0]
    dofs = np.sort(np.random.default_rng(7).choice(free, size=256, replace=False))
    np.savez_compressed(
        os.path.join(HERE, name + ".npz"),
        norm_u=np.linalg.norm(Y[..., :dim].reshape(Y.shape[0], -1), axis=1),
        norm_p=np.linalg.norm(Y[..., dim], axis=1),
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


def _batched_one(args):
    i, n, steps, seed = args
    pb = W.heterogeneous_problem(n, steps, field_seed=seed, young_seed=seed + 1000)
    orc = seq.BiotOracle(pb)
    Y = orc.trajectory_node_major(orc.solve_sequential())
    nn = Y.shape[1]
    fixed_nm = fem.field_to_node_major(orc.fixed.astype(float), nn, 2).reshape(-1) > 0.5
    free = np.nonzero(~fixed_nm)[0]
    dofs = np.sort(np.random.default_rng(100 + i).choice(free, size=8, replace=False))
    flat = Y.reshape(Y.shape[0], -1)
    return (np.linalg.norm(Y[..., :2].reshape(Y.shape[0], -1), axis=1),
            np.linalg.norm(Y[..., 2], axis=1), dofs, flat[:, dofs],
            np.abs(Y[..., :2]).max(), np.abs(Y[..., 2]).max())


def write_batched(name="batched64", workers=6):
    from multiprocessing import Pool
    t0 = time.time()
    specs = W.batched_samples(64, seed=3)
    with Pool(workers) as pool:
        out = pool.map(_batched_one, [(i, n, N, sd) for i, (n, N, sd) in enumerate(specs)])
    steps = np.array([N for _, N, _ in specs], dtype=np.int64)
    np.savez_compressed(
        os.path.join(HERE, name + ".npz"), grid_n=np.array([n for n, _, _ in specs]),
        n_steps=steps, offsets=np.concatenate([[0], np.cumsum(steps + 1)]).astype(np.int64),
        norm_u=np.concatenate([o[0] for o in out]), norm_p=np.concatenate([o[1] for o in out]),
        dofs=np.stack([o[2] for o in out]).astype(np.int64),
        samples=np.concatenate([o[3] for o in out]),
        amax_u=np.array([o[4] for o in out]), amax_p=np.array([o[5] for o in out]))
    print(f"{name}.npz written in {time.time() - t0:.1f} s")


WORKLOADS = {"large_terzaghi": W.large_terzaghi, "large_heterogeneous": W.large_heterogeneous,
             "cube40": lambda: W.terzaghi_problem(40, 256, dim=3),
             "large_terzaghi_dt32": lambda: W.terzaghi_problem(256, 512, dt=1 / 32),
             "large_terzaghi_dt0.1": lambda: W.terzaghi_problem(256, 512, dt=0.1)}

if __name__ == "__main__":
    for name in (sys.argv[1:] or list(WORKLOADS) + ["adjoint_c4"]):
        if name == "adjoint_c4":
            write_adjoint()
        elif name == "batched64":
            write_batched()
        else:
            write(name, WORKLOADS[name]())
