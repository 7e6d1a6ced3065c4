"""CPU checks of the batched-solve autotuner's host logic (no GPU needed): the
cache key (workload, library build and device) and the cache round trip."""
import json

from paper_2310_10430_amd import autotune as at
from paper_2310_10430_amd import workloads as W


def _samples():
    return [W.terzaghi_problem(n, N) for n, N in ((8, 128), (16, 512), (8, 256), (12, 144))]


def test_batch_key_names_workload_build_and_device():
    probs = _samples()
    k1 = at.batch_key(probs, "mixed", 2e-9, "devA", lib_hash="abc")
    assert k1.startswith("2d-S4-n8_16-") and k1.endswith("-mixed-rtol2e-09-libabc-devA")
    assert at.batch_key(probs, "mixed", 2e-9, "devB", lib_hash="abc") != k1
    assert at.batch_key(probs, "mixed", 2e-9, "devA", lib_hash="abd") != k1
    assert at.batch_key(probs, "fp64", 2e-9, "devA", lib_hash="abc") != k1
    other = _samples()
    other[2] = W.terzaghi_problem(8, 272)
    assert at.batch_key(other, "mixed", 2e-9, "devA", lib_hash="abc") != k1


def test_cache_hit_needs_no_gpu(tmp_path, monkeypatch):
    probs = _samples()
    key = at.batch_key(probs, "mixed", 2e-9, "devA")
    cache = tmp_path / "tune.json"
    monkeypatch.setenv("BIOT_TUNE_CACHE", str(cache))
    cache.write_text(json.dumps({key: {"key": key, "depth": 48, "wg_per_cu": 2, "trials": []}}))
    out = at.tune_batch(probs, precision="mixed", rtol=2e-9, device_name="devA")
    assert out["cached"] and out["depth"] == 48 and out["wg_per_cu"] == 2


def test_batch_key_names_materials_and_solver_options():
    """Two workloads of the same sizes and steps but other material fields, or
    the same workload under other solver options, get other keys."""
    a = [W.terzaghi_problem(16, 64)]
    b = [W.heterogeneous_problem(16, 64, field_seed=1, young_seed=2)]
    assert (a[0].grid_n, a[0].n_steps, a[0].dt) == (b[0].grid_n, b[0].n_steps, b[0].dt)
    ka = at.batch_key(a, "fp64", 2e-9, "devA", lib_hash="abc")
    assert at.batch_key(b, "fp64", 2e-9, "devA", lib_hash="abc") != ka
    assert at.batch_key(a, "fp64", 2e-9, "devA", lib_hash="abc", omega=1.3) != ka
    kp = at.batch_key(a, "fp64", 2e-9, "devA", lib_hash="abc", solver_kw={"precond": "P2"})
    assert kp != ka and "precond=P2" in kp
    assert at.batch_key(a, "fp64", 2e-9, "devA", lib_hash="abc", solver_kw={}) == ka
