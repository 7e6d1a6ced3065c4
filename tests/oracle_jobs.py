"""Oracle jobs that GPU tests run in separate processes (spawned, so they never
touch the GPU): the sequential backward-Euler oracle for a full-size workload,
written to a .npy file, or solved for one batched sample and compared there
with the GPU trajectory the test saved.  Imports only numpy, the oracle and
the input generators."""
import numpy as np

from oracle import sequential as seq
from paper_2310_10430_amd import workloads as W


def _field_errors(Y, Yo, dim):
    """Per field: max_n ||Y^n - Yo^n|| / max_n ||Yo^n|| (the method's 1e-8
    error) and the worst element relative to the field's largest value."""
    out = {}
    for name, sl in (("u", slice(0, dim)), ("p", slice(dim, dim + 1))):
        a = np.asarray(Y[..., sl]).reshape(Y.shape[0], -1)
        b = np.asarray(Yo[..., sl]).reshape(Yo.shape[0], -1)
        out[f"q12_{name}"] = float(np.linalg.norm(a - b, axis=1).max()
                                   / np.linalg.norm(b, axis=1).max())
        out[f"elem_{name}"] = float(np.abs(a - b).max() / np.abs(b).max())
    return out


def full_trajectory(name, path):
    """Oracle trajectory of a named workload (node-major) saved to `path`."""
    pb = getattr(W, name)()
    orc = seq.BiotOracle(pb)
    Y = orc.trajectory_node_major(orc.solve_sequential())
    np.save(path, Y)
    return path


def batched_sample_errors(args):
    """Oracle of batched sample i, compared with the GPU trajectory in gpu_path
    at every unknown of every step of that sample."""
    i, n, steps, seed, gpu_path = args
    pb = W.heterogeneous_problem(n, steps, field_seed=seed, young_seed=seed + 1000)
    orc = seq.BiotOracle(pb)
    Yo = orc.trajectory_node_major(orc.solve_sequential())
    Y = np.load(gpu_path)
    return i, _field_errors(Y, Yo, 2)
