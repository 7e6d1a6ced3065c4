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

Run:  python tests/golden/make_goldens.py [large_terzaghi] [large_heterogeneous]
      (about 2 minutes each on one core)
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from paper_2310_10430_amd import workloads as W  # noqa: E402
from oracle import fem, sequential as seq  # noqa: E402


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


WORKLOADS = {"large_terzaghi": W.large_terzaghi, "large_heterogeneous": W.large_heterogeneous}

if __name__ == "__main__":
    for name in (sys.argv[1:] or list(WORKLOADS)):
        write(name, WORKLOADS[name]())
