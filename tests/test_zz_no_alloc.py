"""biot_apply_precond_noalloc against biot_apply_precond, through the C ABI.

The allocation-free entry point runs the same kernels with the V-cycle work
vectors in the library's static device scratch instead of the bound workspace,
so its output must equal the workspace entry point's.  Each case makes two
calls in a row, the second with fewer columns, so the second runs on scratch
that still holds the first call's contents.  Covered: FP64 and mixed precision,
2D and 3D, a two-sample batch handle, the 256^2 headline mesh (more columns
than the scratch holds at once, so the call runs in several batches), and the
size limit (a 640^2 mesh, whose single column of work vectors exceeds the
scratch, is rejected with BIOT_ENOMEM before any device work).
"""
import numpy as np
import pytest
import torch

from paper_2310_10430_amd import workloads as W

pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("needs a ROCm GPU", allow_module_level=True)

from paper_2310_10430_amd import _lib  # noqa: E402
from paper_2310_10430_amd.solver import BiotSolver  # noqa: E402

DEV = "cuda:0"


def _random_cols(pb, n_nodes, ncols, seed):
    rng = np.random.default_rng(seed)
    R = rng.standard_normal((ncols, n_nodes, pb.dim + 1))
    R[..., : pb.dim] *= 1.0
    R[..., pb.dim] *= 1e-6
    return torch.from_numpy(R).to(DEV)


def _check_pair(s, pb, ncols_list, seed, bound):
    n_nodes = s.info()["n_nodes"]
    for k, nc in enumerate(ncols_list):
        R = _random_cols(pb, n_nodes, nc, seed + k)
        Zref = s.apply_precond(R)
        Z = torch.full_like(R, float("nan"))
        s.apply_precond_noalloc(R, Z)
        torch.cuda.synchronize()
        a, b = Z.cpu().numpy(), Zref.cpu().numpy()
        assert np.isfinite(a).all()
        err = np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)
        print(f"noalloc vs workspace apply: {nc} columns, rel diff {err:.3e}", flush=True)
        assert err <= bound, (nc, err)


@pytest.mark.parametrize("precision,bound", [("fp64", 0.0), ("mixed", 0.0)])
def test_noalloc_matches_workspace_apply_2d(precision, bound):
    pb = W.heterogeneous_problem(48, 3, field_seed=21, young_seed=22)
    s = BiotSolver(pb, precision=precision, max_batch=3, device=DEV)
    _check_pair(s, pb, [7, 2], 100, bound)
    s.close()


def test_noalloc_matches_workspace_apply_3d_and_batch():
    pb = W.terzaghi_problem(8, 3, dim=3)
    s = BiotSolver(pb, precond="P2", device=DEV)
    _check_pair(s, pb, [5, 1], 200, 0.0)
    s.close()
    pbs = [W.heterogeneous_problem(32, 4, field_seed=31), W.heterogeneous_problem(32, 6, field_seed=32)]
    s = BiotSolver(pbs, device=DEV)
    _check_pair(s, pbs[0], [4, 3], 300, 0.0)
    s.close()


def test_noalloc_headline_mesh_in_several_batches():
    pb = W.terzaghi_problem(256, 2)
    s = BiotSolver(pb, schedule="wavefront", depth=8, device=DEV)
    _check_pair(s, pb, [9, 4], 400, 0.0)
    s.close()


def test_noalloc_rejects_a_column_larger_than_the_scratch():
    pb = W.terzaghi_problem(640, 1)
    s = BiotSolver(pb, device=DEV)
    n = s.info()["n_nodes"]
    R = torch.zeros((1, n, 3), dtype=torch.float64, device=DEV)
    Z = torch.zeros_like(R)
    with pytest.raises(_lib.BiotError) as ei:
        s.apply_precond_noalloc(R, Z)
    assert ei.value.code == -2 and "static scratch" in str(ei.value)
    s.close()
