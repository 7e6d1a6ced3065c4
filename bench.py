"""Benchmark: preconditioned parallel-in-time Biot solve on one MI355X.

One bench "step" is one complete solve of the headline workload from the zero
initial iterate to the residual tolerance: the inverted time-stepping iteration
(every sweep = fused residual/coupling/norms, P1 block preconditioner with two
multigrid V-cycles, damped update) over all time steps, on the GPU through the
C ABI.  Inputs (operators, load) are resident in HBM before the timed region.

Workload: 256 x 256 unit-square P1-P1 mesh (66,049 nodes, 198,147 unknowns),
consolidation column (unit top load, drained top, fixed base, roller sides),
E = 1e4, nu = 0.3, alpha = 1, K = 1e-2, 512 backward-Euler steps of dt = 1/512,
FP64.  value = unknowns x steps / (wall time of one solve), with the accuracy of
the converged trajectory against the FP64 sequential oracle reported beside it.

Also reported: the seconds for one gradient of a pressure-misfit objective
(forward + adjoint, 128 x 128 mesh, 256 steps; checkpoints every 16 steps and,
for comparison, the whole forward trajectory kept), the mixed-precision and
heterogeneous variants, and the CPU oracle's times on one host core.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E

# HBM traffic per probed kernel from two rocprofv3 counter passes (FETCH_SIZE
# x 2.00 + WRITE_SIZE x 1.00, the factors of a plain 1 GiB copy) over
# 64-column launches, averaged over the kernel's dispatches, and the kernel
# source they were taken with; see profiles/level0_kernels_large_terzaghi_hbm_counters.md
TRAFFIC = {
    # k_residual<2, double, false>: 8 dispatches; a Jacobi batch reads 65
    # distinct state columns for its 64 (the coupling overlaps the iterates)
    "residual": {"kernels_sha256_prefix": "958ea774ab53d6d8", "bytes_per_launch": 308.1e6,
                 "launch_columns": 64, "algorithmic_bytes_per_launch": 244.9e6},
    # k_post2<2, false, double> (coarse-grid correction and both post-smoothing
    # steps): 24 dispatches (levels 0-2 of 8 batches), average
    "post_u": {"kernels_sha256_prefix": "958ea774ab53d6d8", "bytes_per_launch": 122.7e6,
               "launch_columns": 64, "algorithmic_bytes_per_launch": 104.8e6},
}
METRIC = "dof-timestep updates/s to 1e-8 rel err; HBM GB/s fraction; adjoint grad s"
# candidate wavefront depths of the variants' Richardson solves (the headline's
# come from --depths)
VARIANT_DEPTHS = (32, 40, 48, 56, 60, 64, 72, 80, 96)
ADJOINT_DEPTHS = (64, 72, 80, 88)
CUBE_DEPTHS = (56, 60, 64, 72)


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def traffic_fields(probe, algo_bytes_avg):
    """`traffic`: counter-measured HBM bytes per 64-column launch of the probed
    kernel (None when no counters were taken for it or the kernel source changed
    since), with the launch shape it was measured on and the same
    measured/algorithmic ratio applied to the bench's average launch."""
    import hashlib
    out = {"traffic": None}
    t = TRAFFIC.get(probe)
    if t is None:
        return out
    src = os.path.join(ROOT, "paper_2310_10430_amd", "csrc", "kernels.hip")
    with open(src, "rb") as f:
        h = hashlib.sha256(f.read()).hexdigest()
    if not h.startswith(t["kernels_sha256_prefix"]):
        return out
    ratio = t["bytes_per_launch"] / t["algorithmic_bytes_per_launch"]
    out.update(traffic=t["bytes_per_launch"], traffic_launch_columns=t["launch_columns"],
               traffic_over_algorithmic=ratio, traffic_per_average_launch=ratio * algo_bytes_avg)
    return out


def sampled_errors(X, dofs, samp, norm_u, norm_p, scale=None):
    """Errors of the GPU trajectory X [N+1, nn, dim+1] at stored oracle samples
    (unknowns `dofs` of the node-major layout, values samp[n, k]) and in the
    per-step field norms; each relative to the largest oracle value (of the
    samples, or scale = (largest |u|, largest |p|) of the whole trajectory)."""
    d1 = X.shape[2]
    flat = X.reshape(X.shape[0], -1)
    got = flat[:, dofs]
    is_p = (dofs % d1) == d1 - 1
    out = {}
    for f, (name, m) in enumerate((("u", ~is_p), ("p", is_p))):
        if m.any():
            ref = samp[:, m]
            den = np.abs(ref).max() if scale is None else scale[f]
            out[f"sampled_{name}"] = float(np.abs(got[:, m] - ref).max() / den)
    nu = np.linalg.norm(X[..., : d1 - 1].reshape(X.shape[0], -1), axis=1)
    npn = np.linalg.norm(X[..., d1 - 1], axis=1)
    out["norms_u"] = float(np.abs(nu - norm_u).max() / norm_u.max())
    out["norms_p"] = float(np.abs(npn - norm_p).max() / norm_p.max())
    return out


def accuracy_vs_golden(X, golden):
    """Errors of the GPU trajectory at the stored oracle samples of a workload."""
    return sampled_errors(X, golden["dofs"], golden["samples"], golden["norm_u"],
                          golden["norm_p"])


def steady_state_error(X, pb):
    """The consolidation column's final state against its closed form: the
    vertical displacement -x_up / (lambda + 2 mu), zero lateral displacement and
    zero pressure (homogeneous materials, E = 1e4, nu = 0.3)."""
    lam = 1e4 * 0.3 / (1.3 * 0.4)
    mu = 1e4 / 2.6
    up = pb.dim - 1
    ref = -pb.xyz[:, up] / (lam + 2 * mu)
    err = np.abs(X[-1, :, up] - ref).max()
    err = max(err, np.abs(X[-1, :, :up]).max())
    return float(max(err / np.abs(ref).max(), np.abs(X[-1, :, pb.dim]).max()))


def host_cpu():
    """Logical CPUs of the host and its CPU model (from /proc/cpuinfo)."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return os.cpu_count(), model


def cpu_baseline(pb, X_gpu):
    """Time the oracle (sequential BE, scaled SuperLU + one refinement step) on
    one host core over the whole solve (factorization and every step), and
    compare the GPU trajectory with it at every unknown of every step: per
    field max_n ||Y^n - Y_o^n|| / max_n ||Y_o^n|| and the worst element."""
    from oracle import sequential as seq
    try:
        prev = os.sched_getaffinity(0)
        os.sched_setaffinity(0, {min(prev)})
        cores = 1
    except (AttributeError, OSError):
        prev = None
        cores = os.cpu_count()
    try:
        t0 = time.perf_counter()
        orc = seq.BiotOracle(pb)
        t_asm = time.perf_counter() - t0
        t0 = time.perf_counter()
        orc.step_solver()
        t_fact = time.perf_counter() - t0
        t0 = time.perf_counter()
        Xo = orc.solve_sequential()
        t_steps = time.perf_counter() - t0
    finally:
        if prev is not None:
            os.sched_setaffinity(0, prev)
    t_full = t_fact + t_steps
    value = pb.n_dof * pb.n_steps / t_full
    Yo = orc.trajectory_node_major(Xo)
    del Xo
    err = {}
    d = pb.dim
    for name, sl in (("u", slice(0, d)), ("p", slice(d, d + 1))):
        a = X_gpu[..., sl].reshape(X_gpu.shape[0], -1)
        b = Yo[..., sl].reshape(Yo.shape[0], -1)
        num = np.linalg.norm(a - b, axis=1).max()
        den = np.linalg.norm(b, axis=1).max()
        err[f"all_steps_q12_{name}"] = float(num / den)
        err[f"all_steps_max_elem_{name}"] = float(np.abs(a - b).max() / np.abs(b).max())
    nproc, model = host_cpu()
    info = {"value": value, "unit": "dof-timestep updates/s", "cores": cores, "kind": "oracle",
            "host_nproc": nproc, "host_cpu": model,
            "sample": (f"the whole solve on one core: SuperLU factorization {t_fact:.1f} s + "
                       f"all {pb.n_steps} steps {t_steps:.1f} s = {t_full:.1f} s "
                       f"(assembly {t_asm:.1f} s excluded)")}
    return info, err


def run_variant(BiotSolver, pb, golden_name, precision, args, reps=2, **kw):
    """Solve one workload variant to the same tolerance; time `reps` solves
    after one warm-up and report throughput and the error at the stored oracle
    samples.  `kw` overrides solver options (inner solver, preconditioner,
    depth)."""
    import torch
    opts = dict(schedule=args.schedule, depth=args.variant_depth, omega=args.omega,
                wg_per_cu=args.wg_per_cu, precision=precision)
    opts.update(kw)
    tuned = None
    if args.depth_auto and args.schedule == "wavefront" and "depth" not in kw:
        # Richardson units: the depth tuned like the headline's, over depths
        # that cover these variants' sweep counts (about 32-96)
        from paper_2310_10430_amd import autotune
        extra = {k: v for k, v in kw.items() if k != "omega"}
        ch = autotune.tune_batch([pb], precision=precision, rtol=args.rtol,
                                 depths=VARIANT_DEPTHS, wpcs=(args.wg_per_cu,),
                                 omega=opts["omega"], solver_kw=extra)
        opts["depth"] = ch["depth"]
        tuned = {"over": list(VARIANT_DEPTHS), "trials": ch.get("trials")}
    s = BiotSolver(pb, **opts)
    s.reset()
    s.solve_to_tol(args.rtol, max_sweeps=args.max_sweeps, check_every=args.check_every)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        s.reset()
        st = s.solve_to_tol(args.rtol, max_sweeps=args.max_sweeps, check_every=args.check_every)
    torch.cuda.synchronize()
    per = (time.perf_counter() - t0) / reps
    X = s.trajectory().cpu().numpy()
    s.close()
    gpath = os.path.join(ROOT, "tests", "golden", golden_name + ".npz")
    acc = accuracy_vs_golden(X, np.load(gpath)) if os.path.exists(gpath) else {}
    if pb.n_steps * pb.dt >= 8 and np.all(pb.young == pb.young[0]):
        acc["final_step_vs_steady_state"] = steady_state_error(X, pb)
    return {"value": pb.n_dof * pb.n_steps / per, "unit": "dof-timestep updates/s",
            "ms_per_solve": 1e3 * per, "precision": precision, "options": kw, "dt": pb.dt,
            "depth": opts["depth"], "depth_tuned": tuned, "sweeps": st["sweeps"],
            "rel_resid": max(st["rel_resid_u"], st["rel_resid_p"]),
            "max_rel_err_vs_oracle_samples": max(acc.values()), "accuracy": acc}


def adjoint_errors(grads, golden, pb, lam, mu):
    """Gradient errors against the stored oracle gradient and central FD."""
    from paper_2310_10430_amd import workloads as W
    out = {}
    for g, key in zip(grads, ("grad_logk", "grad_lambda", "grad_mu")):
        ref = golden[key]
        out[key] = float(np.linalg.norm(g - ref) / np.linalg.norm(ref))
    worst = 0.0
    for (vk, vl, vm), fd, sc in zip(W.fd_directions(pb.n_elems, 32, seed=43), golden["fd"],
                                    golden["fd_scale"]):
        an = grads[0] @ vk + grads[1] @ (lam * vl) + grads[2] @ (mu * vm)
        worst = max(worst, abs(an - fd) / sc)
    out["fd_32_directions"] = worst
    return out


def run_adjoint(BiotSolver, args, reps=2):
    """Seconds for one gradient (forward solve + objective + adjoint solve +
    gradient contraction) of the pressure misfit on the gradient workload, with
    checkpoints every 16 steps and with the whole forward trajectory kept."""
    import torch
    from paper_2310_10430_amd import workloads as W
    golden = np.load(os.path.join(ROOT, "tests", "golden", "adjoint_c4.npz"))
    sensors, p_obs = golden["sensors"], golden["p_obs"]
    pb = W.adjoint_problem()
    E, nu = pb.young, pb.poisson
    lam = E * nu / ((1 + nu) * (1 - 2 * nu))
    mu = E / (2 * (1 + nu))
    res = {"workload": "adjoint_c4: 128x128 consolidation column, 49923 unknowns, 256 steps "
                       "dt=1/256, log-normal K (field seed 40), 64 pressure sensors, "
                       "observations from reference field seed 41; gradient w.r.t. 32768 "
                       "log K_e and lambda_e, mu_e",
           "rtol": args.rtol}

    def make(depth, stride):
        return BiotSolver(pb, schedule=args.schedule, depth=depth, omega=args.omega,
                          wg_per_cu=args.wg_per_cu, adjoint=True, ckpt_stride=stride,
                          replay_segments=4, max_sensors=64)

    def grad_of(s):
        s.reset()
        st = s.solve_to_tol(args.rtol, max_sweeps=args.max_sweeps, check_every=args.check_every)
        out = s.adjoint(sensors, p_obs, rtol=args.rtol, max_sweeps=args.max_sweeps)
        return st, out

    depth = args.variant_depth
    if args.depth_auto and args.schedule == "wavefront":
        # one depth for the forward and the adjoint solve (80 and 76 sweeps at
        # depth 64): the fastest gradient with checkpoints, timed
        trials = []
        for d in ADJOINT_DEPTHS:
            s = make(d, 16)
            grad_of(s)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            grad_of(s)
            torch.cuda.synchronize()
            trials.append({"depth": d, "seconds": time.perf_counter() - t0})
            s.close()
        depth = min(trials, key=lambda r: r["seconds"])["depth"]
        res["depth_tuned"] = {"over": list(ADJOINT_DEPTHS), "trials": trials}
    res["depth"] = depth
    for stride in (16, 0):
        s = make(depth, stride)

        def grad():
            return grad_of(s)
        grad()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            st, out = grad()
        torch.cuda.synchronize()
        per = (time.perf_counter() - t0) / reps
        grads = [out[k].cpu().numpy() for k in ("grad_logk", "grad_lambda", "grad_mu")]
        s.close()
        key = f"ckpt_{stride}" if stride else "full_trajectory"
        res[key] = {"seconds": per, "forward_s": st["seconds"],
                    "adjoint_s": out["seconds_adjoint"], "replay_and_contraction_s":
                    out["seconds_replay"], "forward_sweeps": st["sweeps"],
                    "adjoint_sweeps": out["adjoint_sweeps"],
                    "replay_sweeps": out["replay_sweeps"], "replay_groups": out["replay_groups"],
                    "J": out["J"], "rel_err_vs_oracle": adjoint_errors(grads, golden, pb, lam, mu)}
        log(f"bench: adjoint ckpt_stride={stride}: {per:.3f} s per gradient")
    res["seconds"] = res["ckpt_16"]["seconds"]
    return res


def _max_rel_diff(a, b):
    """per field max_n |a - b| / max_n |b| over a node-major trajectory pair"""
    d = a.shape[-1] - 1
    return max(float(((a[..., sl] - b[..., sl]).abs().max() / b[..., sl].abs().max()).item())
               for sl in (slice(0, d), slice(d, d + 1)))


def batched_oracle_errors(trajs):
    """Worst error over the 64 samples at their stored oracle samples and step
    norms (None when the stored values are absent)."""
    gpath = os.path.join(ROOT, "tests", "golden", "batched64.npz")
    if not os.path.exists(gpath):
        return None
    g = np.load(gpath)
    worst = {}
    for i, X in trajs.items():
        a, b = int(g["offsets"][i]), int(g["offsets"][i + 1])
        e = sampled_errors(X.cpu().numpy(), g["dofs"][i], g["samples"][a:b], g["norm_u"][a:b],
                           g["norm_p"][a:b], scale=(g["amax_u"][i], g["amax_p"][i]))
        for k, v in e.items():
            worst[k] = max(worst.get(k, 0.0), v)
    worst["max"] = max(worst.values())
    return worst


def run_batched(args):
    """64 independent samples on uneven meshes (sizes from {32,48,64,96,128},
    128..512 steps, own permeability field and moduli each), solved to the same
    tolerance: one handle per sample in FP64, one after another (the plain GPU
    method), and all 64 samples in ONE batch handle, whose every launch covers
    all samples that take part in it and whose samples skip the steps past
    their own counts, with the wavefront depth and workgroups per CU chosen by
    the autotuner, in FP64 and with the mixed-precision preconditioner."""
    from paper_2310_10430_amd import autotune
    from paper_2310_10430_amd import workloads as W
    specs = W.batched_samples(64, seed=3)
    probs = [W.heterogeneous_problem(n, N, field_seed=seed, young_seed=seed + 1000)
             for n, N, seed in specs]
    real = float(sum(pb.n_dof * pb.n_steps for pb in probs))
    sizes = sorted({pb.grid_n for pb in probs})
    res = {"workload": "64 samples: grid n from {32,48,64,96,128} and steps from 128..512 "
                       "(seeded), log-normal K and E~U[5e3,2e4] per sample (seeds 3000+i, "
                       "4000+i), dt = 1/steps",
           "samples_per_size": {str(n): sum(pb.grid_n == n for pb in probs) for n in sizes},
           "dof_steps": real, "rtol": args.rtol}
    log("bench: batched: one handle per sample, FP64")
    wall, st, ref = autotune.solve_groups([[(i, pb)] for i, pb in enumerate(probs)], args.rtol,
                                          "fp64", max_sweeps=args.max_sweeps, keep=True)
    res["per_sample_fp64"] = {"seconds": wall, "value": real / wall, "handles": len(probs),
                              "sweeps_max": max(x["sweeps"] for x in st),
                              "max_rel_err_vs_oracle": batched_oracle_errors(ref)}
    for prec in ("fp64", "mixed"):
        t0 = time.perf_counter()
        ch = autotune.tune_batch(probs, precision=prec, rtol=args.rtol)
        tune_s = time.perf_counter() - t0
        log(f"bench: batched {prec}: one handle, depth {ch['depth']}, "
            f"wg_per_cu {ch['wg_per_cu']} (tuning {tune_s:.1f} s)")
        wall, st, tr = autotune.solve_groups([list(enumerate(probs))], args.rtol, prec,
                                             depth=ch["depth"], wpcs=[ch["wg_per_cu"]],
                                             max_sweeps=args.max_sweeps, keep=True)
        diff = max(_max_rel_diff(tr[i], ref[i]) for i in ref)
        res[f"batched_{prec}"] = {
            "seconds": wall, "value": real / wall, "handles": 1,
            "sweeps": st[0]["sweeps"], "alg_bytes": st[0]["alg_bytes"],
            "sweep_GBps": st[0]["alg_bytes"] / st[0]["seconds"] / 1e9,
            "computed_dof_steps": real, "phantom_dof_steps": 0.0,
            "max_rel_diff_vs_per_sample_fp64": diff, "tuning_s": tune_s,
            "max_rel_err_vs_oracle": batched_oracle_errors(tr),
            "choice": {k: ch[k] for k in ("depth", "wg_per_cu", "cached", "key")},
            "trials": ch.get("trials")}
        del tr
    del ref
    res["unit"] = "dof-timestep updates/s"
    return res


def run_cube(args):
    """3D unit cube, 40^3 Kuhn tetrahedra (68,921 nodes, 275,684 unknowns),
    256 steps of dt = 1/256, homogeneous materials, FP64 and mixed."""
    import torch
    from paper_2310_10430_amd import workloads as W
    from paper_2310_10430_amd.solver import BiotSolver
    pb = W.terzaghi_problem(40, 256, dim=3)
    res = {"workload": "cube40: 40^3 unit cube, Kuhn tetrahedra, 275684 unknowns, 256 steps "
                       "dt=1/256, E=1e4 nu=0.3 K=1e-2", "rtol": args.rtol}
    gpath = os.path.join(ROOT, "tests", "golden", "cube40.npz")
    golden = np.load(gpath) if os.path.exists(gpath) else None
    res["oracle_golden"] = golden is not None
    for prec in ("fp64", "mixed"):
        depth, tuned = args.variant_depth, None
        if args.depth_auto:
            from paper_2310_10430_amd import autotune
            ch = autotune.tune_batch([pb], precision=prec, rtol=args.rtol, depths=CUBE_DEPTHS,
                                     wpcs=(args.wg_per_cu,), omega=args.omega)
            depth, tuned = ch["depth"], {"over": list(CUBE_DEPTHS), "trials": ch.get("trials")}
        t0 = time.perf_counter()
        s = BiotSolver(pb, schedule="wavefront", depth=depth, omega=args.omega,
                       precision=prec)
        setup = time.perf_counter() - t0
        s.solve_to_tol(args.rtol, max_sweeps=args.max_sweeps, check_every=args.check_every)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s.reset()
        st = s.solve_to_tol(args.rtol, max_sweeps=args.max_sweeps, check_every=args.check_every)
        torch.cuda.synchronize()
        per = time.perf_counter() - t0
        X = s.trajectory()
        s.close()
        res[prec] = {"seconds": per, "value": pb.n_dof * pb.n_steps / per, "setup_s": setup,
                     "depth": depth, "depth_tuned": tuned, "sweeps": st["sweeps"],
                     "rel_resid": max(st["rel_resid_u"], st["rel_resid_p"])}
        Xn = X.cpu().numpy()
        acc = {"final_step_vs_steady_state": steady_state_error(Xn, pb)}
        if golden is not None:
            acc.update(accuracy_vs_golden(Xn, golden))
        res[prec]["accuracy"] = acc
        res[prec]["max_rel_err_vs_oracle"] = max(acc.values())
        del Xn
        if prec == "fp64":
            Xf = X
        else:
            res[prec]["max_rel_diff_vs_fp64"] = _max_rel_diff(X, Xf)
        log(f"bench: cube40 {prec}: {per:.3f} s per solve")
    res["unit"] = "dof-timestep updates/s"
    return res


def cpu_adjoint_baseline():
    """The oracle's gradient (factorization, 256 forward and 256 adjoint direct
    solves, element contraction) of the gradient workload on one host core."""
    from oracle import adjoint as adj
    from paper_2310_10430_amd import workloads as W
    golden = np.load(os.path.join(ROOT, "tests", "golden", "adjoint_c4.npz"))
    pb = W.adjoint_problem()
    try:
        prev = os.sched_getaffinity(0)
        os.sched_setaffinity(0, {min(prev)})
        cores = 1
    except (AttributeError, OSError):
        prev = None
        cores = os.cpu_count()
    try:
        t0 = time.perf_counter()
        adj.objective_and_gradient(pb, *adj.problem_params(pb), golden["sensors"], golden["p_obs"])
        t = time.perf_counter() - t0
    finally:
        if prev is not None:
            os.sched_setaffinity(0, prev)
    return {"seconds": t, "cores": cores, "kind": "oracle",
            "sample": "one whole gradient of the gradient workload (assembly included)"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--schedule", default="wavefront", choices=["wavefront", "jacobi"])
    ap.add_argument("--depth", type=int, default=0,
                    help="wavefront depth; 0: the fastest of --depths, timed by the autotuner")
    ap.add_argument("--depths", default="56,58,60,62,64",
                    help="candidate depths when --depth is 0")
    ap.add_argument("--omega", type=float, default=0.6)
    ap.add_argument("--wg-per-cu", type=int, default=0,
                    help="workgroups per CU of the node-blocked kernels (0: occupancy)")
    ap.add_argument("--rtol", type=float, default=2e-9)
    ap.add_argument("--check-every", type=int, default=8)
    ap.add_argument("--max-sweeps", type=int, default=600)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run a plain 1 GiB device copy (reference for HBM counters)")
    ap.add_argument("--pmc-run", action="store_true",
                    help="hardware-counter run: one Jacobi-schedule sweep of the workload in "
                         "batches of --depth columns (the bench's full-wave launch shape, few "
                         "dispatches), no timing")
    ap.add_argument("--probe-stride", type=int, default=8,
                    help="probe every k-th wave of a pass in the timed region, replaying the "
                         "others as graphs (1: every wave, all eager)")
    ap.add_argument("--probe", default="auto",
                    help="kernel timed with HIP events in the timed region; auto: of the probes "
                         "that each time one kernel, the one with the most time in a probed "
                         "solve before the timed region")
    ap.add_argument("--no-variants", action="store_true",
                    help="skip the mixed-precision and heterogeneous-permeability variants")
    ap.add_argument("--no-adjoint", action="store_true",
                    help="skip the gradient (adjoint) measurement")
    ap.add_argument("--no-batched", action="store_true",
                    help="skip the 64-sample batched measurement")
    ap.add_argument("--no-cube", action="store_true",
                    help="skip the 3D 40^3 measurement")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (got --gpus {args.gpus}); the library has no "
              "multi-GPU path. Run with --gpus 1.", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2310_10430_amd import workloads as W
    from paper_2310_10430_amd.solver import BiotSolver

    if not torch.cuda.is_available():
        print("bench.py needs a ROCm GPU", file=sys.stderr)
        sys.exit(1)
    if args.calibrate_copy:
        src = torch.ones(1 << 27, dtype=torch.float64, device="cuda")   # 1 GiB
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
        log("bench: 1 GiB copy done (counter reference: 1 GiB read, 1 GiB written)")
    pb = W.large_terzaghi()
    if args.pmc_run:
        # the wavefront's full-wave launch shape (64 columns) in few dispatches:
        # one Jacobi sweep in batches of 64 time-step columns
        cols = args.depth if args.depth > 0 else 64
        s = BiotSolver(pb, schedule="jacobi", omega=args.omega, wg_per_cu=args.wg_per_cu,
                       max_batch=cols)
        s.sweep(1)
        torch.cuda.synchronize()
        s.close()
        log(f"bench: counter run done (1 Jacobi sweep in batches of {cols} columns)")
        return
    depth_choice = None
    # with --depth 0 the variants' Richardson solves, the adjoint and the cube
    # tune their depths too; a given depth applies to every leg
    args.variant_depth = args.depth if args.depth > 0 else 64
    args.depth_auto = args.depth <= 0
    if args.schedule == "wavefront" and args.depth <= 0:
        # a pass gives every step `depth` sweeps: the fastest depth is about the
        # smallest at which one pass reaches the tolerance (a shallower one
        # needs further, partial passes); timed, not assumed
        from paper_2310_10430_amd import autotune
        t0 = time.perf_counter()
        ch = autotune.tune_batch([pb], precision="fp64", rtol=args.rtol,
                                 depths=tuple(int(x) for x in args.depths.split(",")),
                                 wpcs=(args.wg_per_cu,), omega=args.omega)
        args.depth = ch["depth"]
        depth_choice = {"tuned_over": args.depths, "tuning_s": time.perf_counter() - t0,
                        "trials": ch.get("trials"), "cached": ch["cached"]}
        log(f"bench: depth {args.depth} (tuned over {args.depths}, {depth_choice['tuning_s']:.1f} s)")
    elif args.depth <= 0:
        args.depth = 64
    log(f"bench: workload 256x256, {pb.n_steps} steps, {pb.n_dof} unknowns; "
        f"schedule={args.schedule} depth={args.depth} omega={args.omega} rtol={args.rtol}")
    t0 = time.perf_counter()
    s = BiotSolver(pb, schedule=args.schedule, depth=args.depth, omega=args.omega,
                   wg_per_cu=args.wg_per_cu)
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0
    log(f"bench: setup {setup_s:.2f} s, workspace {s.workspace_bytes / 1e9:.2f} GB")

    def solve():
        s.reset()
        return s.solve_to_tol(args.rtol, max_sweeps=args.max_sweeps, check_every=args.check_every)

    for i in range(args.warmup):
        st = solve()
        log(f"bench: warmup {i}: {st['sweeps']} sweeps, {st['seconds'] * 1e3:.1f} ms")
    # breakdown of the probed kernels from one probed (untimed) solve, which
    # also names the dominant kernel: the single-kernel probe with the most time
    s.profile(True)
    st_b = solve()
    prof = s.profile_read()
    if args.probe == "auto":
        # post_p times two kernels (level 0 writes the outer update)
        single = [k for k in prof if k != "post_p"]
        args.probe = max(single, key=lambda k: prof[k]["ms"])
    # timed region: HIP events bracket the probed launches of that kernel on
    # the solver's stream, in every probe_stride-th wave of a pass (the waves
    # between them replay captured graphs; 1: every wave, all eager); one
    # untimed solve first captures the graphs of that layout, and enabling
    # again clears the accumulators
    s.profile(True, probes=[args.probe], stride=args.probe_stride)
    if args.probe_stride > 1:
        solve()
        s.profile(True, probes=[args.probe], stride=args.probe_stride)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    stats = []
    for i in range(args.steps):
        stats.append(solve())
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    prof_main = s.profile_read()
    s.profile(False)
    ms_per_step = 1e3 * elapsed / args.steps
    value = pb.n_dof * pb.n_steps / (elapsed / args.steps)
    log(f"bench: {args.steps} solves in {elapsed:.3f} s ({ms_per_step:.1f} ms each, "
        f"{stats[-1]['sweeps']} sweeps)")

    # whole-solve figure: the algorithmic bytes of every kernel a solve
    # enqueues (all levels, tails, transfers, pressure stage, residual checks)
    # over the solve's wall time
    solve_bytes = sum(x["alg_bytes"] for x in stats) / len(stats)
    solve_s = sum(x["seconds"] for x in stats) / len(stats)
    sweep_gbs = solve_bytes / solve_s / 1e9
    log(f"bench: whole solve moves {solve_bytes / 1e9:.1f} GB algorithmic in {solve_s * 1e3:.1f} ms: "
        f"{sweep_gbs:.0f} GB/s = {sweep_gbs / HBM_PEAK_GBS:.3f} of peak")
    p = prof_main[args.probe]
    dominant = max(prof, key=lambda k: prof[k]["ms"])
    avg_ms = p["ms"] / max(p["launches"], 1)
    bytes_per_launch = p["bytes"] / max(p["launches"], 1)
    achieved = bytes_per_launch / (avg_ms * 1e-3) / 1e9
    solve_ms = st_b["seconds"] * 1e3
    kernels = {k: {"launches": v["launches"], "avg_us": 1e3 * v["ms"] / max(v["launches"], 1),
                   "GBps": (v["bytes"] / max(v["ms"], 1e-30)) / 1e6,
                   "share_of_solve": v["ms"] / solve_ms} for k, v in prof.items()}
    kernels["largest_probe"] = dominant   # a probe may cover several kernels
    kernels["roofline_kernel"] = args.probe

    X = s.trajectory().cpu().numpy()
    s.close()
    golden = np.load(os.path.join(ROOT, "tests", "golden", "large_terzaghi.npz"))
    acc = accuracy_vs_golden(X, golden)
    acc["final_step_vs_steady_state"] = steady_state_error(X, pb)

    cpu = None
    if not args.no_cpu_baseline:
        log("bench: timing the CPU oracle over the whole solve on one core (about 45 s)")
        cpu, err = cpu_baseline(pb, X)
        acc.update(err)
    acc["max_rel_err"] = max(v for k, v in acc.items())

    variants = None
    if not args.no_variants:
        variants = {}
        het = W.large_heterogeneous()
        gm = dict(inner="gmres", gmres_k=4, depth=8)
        # P1 against P2 (Sec. 3.1, eqs. (p1)/(p2); Table 3 compares them at
        # tau = 0.1): the same mesh and 512 steps at dt = 1/32 and dt = 0.1,
        # Richardson with the omega that minimizes the step operator's spectral
        # radius (eigenvalues of P^{-1}AA on a 16^2 copy), and GMRES(4)
        big = {32: W.terzaghi_problem(256, 512, dt=1 / 32), 10: W.terzaghi_problem(256, 512, dt=0.1)}
        runs = [("large_terzaghi_mixed", pb, "large_terzaghi", "mixed", {}),
                ("large_heterogeneous_fp64", het, "large_heterogeneous", "fp64", {}),
                ("large_heterogeneous_mixed", het, "large_heterogeneous", "mixed", {}),
                ("large_terzaghi_gmres4_P1", pb, "large_terzaghi", "fp64", gm)]
        for key, gname in ((32, "large_terzaghi_dt32"), (10, "large_terzaghi_dt0.1")):
            runs += [(f"{gname}_P1", big[key], gname, "fp64", dict(omega=1.4)),
                     (f"{gname}_P2", big[key], gname, "fp64", dict(precond="P2", omega=1.3)),
                     (f"{gname}_gmres4_P1", big[key], gname, "fp64", gm),
                     (f"{gname}_gmres4_P2", big[key], gname, "fp64", dict(gm, precond="P2"))]
        for name, prob, gname, prec, kw in runs:
            log(f"bench: variant {name}")
            try:
                variants[name] = run_variant(BiotSolver, prob, gname, prec, args, **kw)
            except RuntimeError as e:      # a variant that does not converge is reported
                variants[name] = {"error": str(e), "options": kw, "precision": prec}

    adjoint = None
    if not args.no_adjoint:
        log("bench: adjoint gradient workload")
        adjoint = run_adjoint(BiotSolver, args)
        if not args.no_cpu_baseline:
            log("bench: timing the CPU oracle's gradient (about half a minute)")
            adjoint["cpu_oracle"] = cpu_adjoint_baseline()

    batched = None if args.no_batched else run_batched(args)
    cube = None if args.no_cube else run_cube(args)

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "dof-timestep updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": "large_terzaghi: 256x256 unit-square P1-P1 consolidation column, "
                        "198147 unknowns, 512 backward-Euler steps dt=1/512, E=1e4 nu=0.3 "
                        "alpha=1 K=1e-2, X^0=0, FP64",
            "schedule": args.schedule, "depth": args.depth if args.schedule == "wavefront" else None,
            "omega": args.omega, "precond": "P1 with one multigrid V-cycle per inner solve",
            "rtol": args.rtol, "sweeps": stats[-1]["sweeps"],
            "rel_resid": max(stats[-1]["rel_resid_u"], stats[-1]["rel_resid_p"]),
            "setup_s": setup_s, "wg_per_cu": args.wg_per_cu, "depth_choice": depth_choice,
        },
        "accuracy": acc,
        "roofline": {
            "bound": "hbm", "kernel": p["name"], "achieved": achieved, "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, **traffic_fields(args.probe,
                                                                             bytes_per_launch),
            "avg_launch_us": 1e3 * avg_ms, "algorithmic_bytes_per_launch": bytes_per_launch,
            "launches": p["launches"], "probed_wave_stride": args.probe_stride,
            "sweep_achieved": sweep_gbs, "sweep_frac": sweep_gbs / HBM_PEAK_GBS,
            "sweep_bytes_per_solve": solve_bytes, "sweep_seconds_per_solve": solve_s,
        },
        "kernels": kernels,
        "cpu_baseline": cpu,
        "variants": variants,
        "adjoint": adjoint,
        "batched": batched,
        "cube40": cube,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
