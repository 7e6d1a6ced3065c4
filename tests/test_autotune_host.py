"""CPU checks of the batched-solve autotuner's host logic (no GPU needed):
the split of a bucket by step count, the bucket key, and the cache round trip."""
import json

from paper_2310_10430_amd import autotune as at
from paper_2310_10430_amd import workloads as W


def _bucket():
    return [W.terzaghi_problem(8, N) for N in (128, 512, 256, 144, 496, 300, 200)]


def test_split_groups_partition_by_steps():
    probs = _bucket()
    for split in (1, 2, 3, 7, 10):
        groups = at.split_groups(probs, split)
        flat = sorted(i for g in groups for i in g)
        assert flat == list(range(len(probs)))                  # a partition
        assert len(groups) == min(split, len(probs))
        steps = [[probs[i].n_steps for i in g] for g in groups]
        # longest samples first, groups ordered by decreasing steps
        for a, b in zip(steps, steps[1:]):
            assert min(a) >= max(b)


def test_split_balances_work():
    probs = _bucket()
    groups = at.split_groups(probs, 2)
    work = [sum(probs[i].n_steps for i in g) for g in groups]
    total = sum(work)
    assert abs(work[0] - work[1]) <= max(p.n_steps for p in probs)
    assert sum(work) == total


def test_bucket_key_and_cache_hit(tmp_path, monkeypatch):
    probs = _bucket()
    key = at.bucket_key(probs, "mixed", 64)
    assert key.startswith("2d-n8-S7-steps128_512")
    cache = tmp_path / "tune.json"
    monkeypatch.setenv("BIOT_TUNE_CACHE", str(cache))
    cache.write_text(json.dumps({key: {"key": key, "split": 2, "wg_per_cu": 1, "trials": []}}))
    out = at.tune(probs, precision="mixed", depth=64)      # served from the cache, no GPU
    assert out["cached"] and out["split"] == 2 and out["wg_per_cu"] == 1
    groups = at.tuned_groups(list(enumerate(probs)), out)
    assert sorted(i for g in groups for i, _ in g) == list(range(len(probs)))
