"""Autotuner for batched solves of many samples on uneven meshes.

Samples on the same mesh size form a bucket; a bucket is solved by one or more
batch handles (biot_create_batch), every launch of a handle covering all of
its samples.  Per bucket the tuner chooses

  * how to split the bucket into handles: samples sorted by their step count
    and cut into `split` groups (a handle runs as many steps as its longest
    sample, so splitting trades padding steps for more, smaller launches);
  * the workgroups per compute unit of the node-blocked kernels (0 = each
    kernel's occupancy).

Each candidate is timed on one full wavefront pass of every handle of the
split (after one untimed pass that also captures the HIP graphs); the pass time
is what a solve repeats, since the number of passes to a tolerance does not
depend on these choices.  Results are cached per bucket key in a JSON file
(BIOT_TUNE_CACHE, default ~/.cache/biot_pint/autotune.json).
"""
from __future__ import annotations

import json
import os
import time
from concurrent.futures import ThreadPoolExecutor

import torch

from .solver import BiotSolver

DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "biot_pint", "autotune.json")


def cache_path() -> str:
    return os.environ.get("BIOT_TUNE_CACHE", DEFAULT_CACHE)


def bucket_key(problems, precision: str, depth: int) -> str:
    pb = problems[0]
    steps = sorted(p.n_steps for p in problems)
    return (f"{pb.dim}d-n{pb.grid_n}-S{len(problems)}-steps{steps[0]}_{steps[-1]}"
            f"_{sum(steps)}-{precision}-D{depth}")


def split_groups(problems, split: int):
    """Samples sorted by step count (longest first) and cut into `split` groups
    of about equal total work."""
    order = sorted(range(len(problems)), key=lambda i: -problems[i].n_steps)
    split = max(1, min(split, len(order)))
    total = sum(problems[i].n_steps for i in order)
    groups, cur, acc = [], [], 0
    for pos, i in enumerate(order):
        left = len(order) - pos                 # samples not yet placed, i included
        need = split - 1 - len(groups)          # cuts still to make
        if cur and need > 0:
            target = total * (len(groups) + 1) / split
            # cut before sample i when that lands closer to the group's share,
            # or when every remaining sample must start a group of its own
            if abs(acc + problems[i].n_steps - target) > abs(acc - target) or left <= need:
                groups.append(cur)
                cur = []
        cur.append(i)
        acc += problems[i].n_steps
    if cur:
        groups.append(cur)
    return groups


def _load_cache():
    try:
        with open(cache_path()) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _store_cache(cache):
    path = cache_path()
    try:
        os.makedirs(os.path.dirname(path), exist_ok=True)
        tmp = path + ".tmp"
        with open(tmp, "w") as f:
            json.dump(cache, f, indent=1, sort_keys=True)
        os.replace(tmp, path)
    except OSError:
        pass


def time_pass(problems, groups, wpc: int, depth: int, precision: str, device="cuda:0") -> float:
    """Seconds for one wavefront pass of every handle of the split."""
    total = 0.0
    for g in groups:
        batch = [problems[i] for i in g]
        s = BiotSolver(batch if len(batch) > 1 else batch[0], schedule="wavefront", depth=depth,
                       wg_per_cu=wpc, precision=precision, device=device)
        s.sweep(depth)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s.sweep(depth)
        torch.cuda.synchronize()
        total += time.perf_counter() - t0
        s.close()
    return total


def tune(problems, precision: str = "mixed", depth: int = 64, splits=(1, 2), wpcs=(0, 2),
         use_cache: bool = True, device="cuda:0") -> dict:
    """Best (split, wg_per_cu) for one bucket; returns the choice, every
    candidate's pass time and whether it came from the cache."""
    key = bucket_key(problems, precision, depth)
    cache = _load_cache() if use_cache else {}
    if key in cache:
        out = dict(cache[key])
        out["cached"] = True
        return out
    t0 = time.perf_counter()
    trials = []
    for split in splits:
        if split > len(problems):
            continue
        groups = split_groups(problems, split)
        for wpc in wpcs:
            t = time_pass(problems, groups, wpc, depth, precision, device)
            trials.append({"split": split, "wg_per_cu": wpc, "pass_s": t})
    best = min(trials, key=lambda r: r["pass_s"])
    out = {"key": key, "split": best["split"], "wg_per_cu": best["wg_per_cu"],
           "trials": trials, "tuning_s": time.perf_counter() - t0}
    if use_cache:
        cache = _load_cache()
        cache[key] = out
        _store_cache(cache)
    out = dict(out)
    out["cached"] = False
    return out


def solve_groups(groups, rtol: float, precision: str, depth: int = 64, wpcs=None,
                 max_sweeps: int = 2000, device="cuda:0", keep=False, concurrent=False):
    """Solves each group of (sample number, problem) pairs as one handle (a
    batch if it has several samples).  Handles are created, bound and warmed up
    (one pass, which captures the graphs) before the timed region; the timed
    region resets and solves every handle to rtol, in turn, or with
    `concurrent`, all at once: each handle then runs on a stream of its own
    (default priority) and is driven by a host thread of its own, so the small
    launches of different mesh sizes overlap on the GPU.  Returns the wall
    time, the stats per handle and, with keep, {sample number: trajectory}."""
    handles = []
    for k, g in enumerate(groups):
        batch = [pb for _, pb in g]
        wpc = 0 if wpcs is None else wpcs[k]
        stream = torch.cuda.Stream(device=device) if concurrent else None
        with torch.cuda.stream(stream) if concurrent else _nullctx():
            s = BiotSolver(batch if len(batch) > 1 else batch[0], schedule="wavefront",
                           depth=depth, wg_per_cu=wpc, precision=precision, device=device)
            s.sweep(depth)
        handles.append((s, [i for i, _ in g]))
    torch.cuda.synchronize()

    def run(s):
        s.reset()
        return s.solve_to_tol(rtol, max_sweeps=max_sweeps)

    t0 = time.perf_counter()
    if concurrent:
        with ThreadPoolExecutor(max_workers=len(handles)) as ex:
            stats = list(ex.map(run, [s for s, _ in handles]))
    else:
        stats = [run(s) for s, _ in handles]
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    trajs = {}
    if keep:
        for s, ids in handles:
            for k, i in enumerate(ids):
                trajs[i] = s.sample_trajectory(k) if s.batch else s.trajectory()
    for s, _ in handles:
        s.close()
    return wall, stats, trajs


class _nullctx:
    def __enter__(self):
        return None

    def __exit__(self, *exc):
        return False


def tuned_groups(bucket, choice):
    """(sample number, problem) groups of a bucket under a tuner choice."""
    probs = [pb for _, pb in bucket]
    return [[bucket[i] for i in g] for g in split_groups(probs, choice["split"])]
