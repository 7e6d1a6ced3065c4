"""Autotuner for one batched solve of many samples on uneven meshes.

All samples go into one batch handle (biot_create_batch with a mesh per
sample): every launch covers the samples that take part in it, and each
sample skips the steps past its own count.  For that handle the tuner picks

  * the wavefront depth: the columns of one launch and the sweeps one pass
    gives every step (more columns amortize a launch's operator reads over
    more columns and fill the chip better; fewer make a pass, N + depth - 1
    waves, shorter and the convergence checks between passes more frequent; a
    single problem is fastest at about the smallest depth at which one pass
    reaches the tolerance: 256^2 consolidation column, 383 ms at depth 60
    against 403 ms at 64 and 506 ms at 58, which needs a partial second
    pass), and
  * the workgroups per compute unit of the node-blocked kernels' grids
    (0 = each kernel's occupancy, capped at 3 per CU),

by timing a whole solve to the tolerance for every candidate pair (after one
untimed pass that captures the HIP graphs).  The time is not smooth in the
depth (64-sample batch, FP64, 4 workgroups per CU: 2.93, 2.61, 2.57, 2.64,
2.72, 2.81 s at depths 72, 76, 80, 84, 88, 96, and depths past the sweeps the
samples need add passes), hence the grid of depths around the usual sweep
counts.  Results are cached in a JSON file
(BIOT_TUNE_CACHE, default ~/.cache/biot_pint/autotune.json) under a key made of
the workload (dimension, sizes, step counts, precision, tolerance), the library
build (a hash of libbiot_pint.so) and the device name, so that a rebuilt
library or another device is tuned again.
"""
from __future__ import annotations

import hashlib
import json
import os
import time
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import torch

from . import _lib
from .solver import BiotSolver

DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "biot_pint", "autotune.json")


def cache_path() -> str:
    return os.environ.get("BIOT_TUNE_CACHE", DEFAULT_CACHE)


def library_hash() -> str:
    """Hash of the built library (the kernels the choice was measured with)."""
    h = hashlib.sha256()
    with open(_lib.LIB_PATH, "rb") as f:
        for chunk in iter(lambda: f.read(1 << 20), b""):
            h.update(chunk)
    return h.hexdigest()[:16]


def batch_key(problems, precision: str, rtol: float, device_name: str,
              lib_hash: str | None = None, omega: float = 0.6, solver_kw=None) -> str:
    """Cache key: the workload (sizes, steps, time step and material fields;
    the damping when it is not the default 0.6 and any further solver
    options), the library build and the device."""
    sig = hashlib.sha256()
    for pb in problems:
        sig.update(f"{pb.dim}:{pb.grid_n}:{pb.n_steps}:{pb.dt!r}:{pb.alpha!r};".encode())
        for a in (pb.young, pb.poisson, pb.perm):
            sig.update(np.ascontiguousarray(a, dtype=np.float64).tobytes())
    sizes = sorted({pb.grid_n for pb in problems})
    w = "" if omega == 0.6 else f"-w{omega:g}"
    if solver_kw:
        w += "-" + ",".join(f"{k}={solver_kw[k]}" for k in sorted(solver_kw))
    return (f"{problems[0].dim}d-S{len(problems)}-n{sizes[0]}_{sizes[-1]}-{sig.hexdigest()[:12]}"
            f"-{precision}{w}-rtol{rtol:g}-lib{lib_hash or library_hash()}-{device_name}")


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


def time_solve(problems, depth: int, wpc: int, precision: str, rtol: float,
               max_sweeps: int = 2000, device="cuda:0", omega: float = 0.6,
               solver_kw=None) -> float:
    """Seconds of one solve to rtol of all samples in one handle (`solver_kw`:
    further BiotSolver options, e.g. the preconditioner)."""
    s = BiotSolver(problems if len(problems) > 1 else problems[0], schedule="wavefront",
                   depth=depth, wg_per_cu=wpc, precision=precision, device=device, omega=omega,
                   **(solver_kw or {}))
    try:
        s.sweep(depth)                      # captures the graphs
        torch.cuda.synchronize()
        s.reset()
        t0 = time.perf_counter()
        s.solve_to_tol(rtol, max_sweeps=max_sweeps)
        torch.cuda.synchronize()
        return time.perf_counter() - t0
    finally:
        s.close()


def tune_batch(problems, precision: str = "mixed", rtol: float = 2e-9,
               depths=(64, 72, 80, 88, 96), wpcs=(0, 4), use_cache: bool = True, device="cuda:0",
               device_name: str | None = None, omega: float = 0.6, solver_kw=None) -> dict:
    """Best (depth, wg_per_cu) for one handle over all samples; returns the
    choice, every candidate's solve time and whether it came from the cache."""
    if device_name is None:
        device_name = torch.cuda.get_device_name(device).replace(" ", "_")
    key = batch_key(problems, precision, rtol, device_name, omega=omega, solver_kw=solver_kw)
    cache = _load_cache() if use_cache else {}
    if key in cache:
        out = dict(cache[key])
        out["cached"] = True
        return out
    t0 = time.perf_counter()
    trials = []
    for depth in depths:
        for wpc in wpcs:
            t = time_solve(problems, depth, wpc, precision, rtol, device=device, omega=omega,
                           solver_kw=solver_kw)
            trials.append({"depth": depth, "wg_per_cu": wpc, "solve_s": t})
    best = min(trials, key=lambda r: r["solve_s"])
    out = {"key": key, "depth": best["depth"], "wg_per_cu": best["wg_per_cu"],
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
    (default priority) and is driven by a host thread of its own.  Returns the
    wall time, the stats per handle and, with keep, {sample number:
    trajectory}."""
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
