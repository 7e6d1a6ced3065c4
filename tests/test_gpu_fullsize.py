"""GPU parity at the full workload sizes, in the launch configuration the
bench times (wavefront, depth 64, omega 0.6, rtol 2e-9), against the stored
oracle values of tests/golden/ (written by make_goldens.py from the oracle):

* the 256 x 256 consolidation column (512 steps), FP64 and mixed precision:
  256 sampled unknowns at every step and the per-step field norms, and the
  final step against the closed-form steady state;
* the heterogeneous 256 x 256 workload, FP64 and mixed;
* the 40^3 cube on Kuhn tetrahedra (256 steps), FP64 and mixed;
* all 64 batched samples on uneven meshes, one batch handle per mesh size,
  FP64 and mixed, each sample against its own oracle values.

The bar is the 1e-8 relative error of the method's target, per field, each
error relative to the largest oracle value of that field (of the samples for
the single workloads, of the whole trajectory for the batched samples).
"""
import os

import numpy as np
import pytest
import torch

from oracle import fem
from paper_2310_10430_amd import workloads as W

pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("needs a ROCm GPU", allow_module_level=True)

from paper_2310_10430_amd.solver import BiotSolver  # noqa: E402

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
RTOL = 2e-9
BAR = 1e-8


def _solve(pb, precision, depth=64):
    s = BiotSolver(pb, schedule="wavefront", depth=depth, omega=0.6, precision=precision)
    st = s.solve_to_tol(RTOL, max_sweeps=600, check_every=8)
    return s, st


def _errors(X, dofs, samp, norm_u, norm_p, scale=None):
    d1 = X.shape[2]
    flat = X.reshape(X.shape[0], -1)
    got = flat[:, dofs]
    is_p = (dofs % d1) == d1 - 1
    out = {}
    for f, (name, m) in enumerate((("u", ~is_p), ("p", is_p))):
        if m.any():
            ref = samp[:, m]
            den = np.abs(ref).max() if scale is None else scale[f]
            out["sampled_" + name] = float(np.abs(got[:, m] - ref).max() / den)
    nu = np.linalg.norm(X[..., : d1 - 1].reshape(X.shape[0], -1), axis=1)
    npn = np.linalg.norm(X[..., d1 - 1], axis=1)
    out["norms_u"] = float(np.abs(nu - norm_u).max() / norm_u.max())
    out["norms_p"] = float(np.abs(npn - norm_p).max() / norm_p.max())
    return out


def _steady_error(X, pb):
    lam, mu = fem.lame(1e4, 0.3)
    up = pb.dim - 1
    ref = -pb.xyz[:, up] / (lam + 2 * mu)
    e = max(np.abs(X[-1, :, up] - ref).max(), np.abs(X[-1, :, :up]).max())
    return max(e / np.abs(ref).max(), np.abs(X[-1, :, pb.dim]).max())


@pytest.mark.parametrize("name,precision", [("large_terzaghi", "fp64"),
                                            ("large_terzaghi", "mixed"),
                                            ("large_heterogeneous", "fp64"),
                                            ("large_heterogeneous", "mixed")])
def test_full_size_square_against_oracle_golden(name, precision):
    pb = getattr(W, name)()
    s, st = _solve(pb, precision)
    X = s.trajectory().cpu().numpy()
    s.close()
    assert st["converged"], st
    g = np.load(os.path.join(GOLDEN, name + ".npz"))
    err = _errors(X, g["dofs"], g["samples"], g["norm_u"], g["norm_p"])
    if name == "large_terzaghi":
        err["steady"] = _steady_error(X, pb)
    assert max(err.values()) < BAR, err


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_full_size_cube_against_oracle_golden(precision):
    pb = W.terzaghi_problem(40, 256, dim=3)
    s, st = _solve(pb, precision)
    X = s.trajectory().cpu().numpy()
    s.close()
    assert st["converged"], st
    g = np.load(os.path.join(GOLDEN, "cube40.npz"))
    err = _errors(X, g["dofs"], g["samples"], g["norm_u"], g["norm_p"])
    err["steady"] = _steady_error(X, pb)
    assert max(err.values()) < BAR, err


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_full_size_batched_samples_against_oracle_golden(precision):
    g = np.load(os.path.join(GOLDEN, "batched64.npz"))
    specs = W.batched_samples(64, seed=3)
    worst = {}
    for n in sorted({n for n, _, _ in specs}):
        ids = [i for i, (m, _, _) in enumerate(specs) if m == n]
        probs = [W.heterogeneous_problem(n, specs[i][1], field_seed=specs[i][2],
                                         young_seed=specs[i][2] + 1000) for i in ids]
        s, st = _solve(probs, precision)
        assert st["converged"], (n, st)
        for k, i in enumerate(ids):
            X = s.sample_trajectory(k).cpu().numpy()
            a, b = int(g["offsets"][i]), int(g["offsets"][i + 1])
            e = _errors(X, g["dofs"][i], g["samples"][a:b], g["norm_u"][a:b], g["norm_p"][a:b],
                        scale=(g["amax_u"][i], g["amax_p"][i]))
            for key, v in e.items():
                worst[key] = max(worst.get(key, 0.0), v)
        s.close()
    assert max(worst.values()) < BAR, worst
