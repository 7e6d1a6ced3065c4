"""Python front end of the HIP library: argument marshalling and device memory.

Every step of the solver runs in the HIP kernels of libbiot_pint.so; this module
only converts a `workloads.Problem` into the C structures, allocates the device
workspace as a torch tensor and binds the handle to torch's current stream at
construction (create it under `torch.cuda.stream(...)` to give it a stream of
its own; tensors passed in and out are then ordered against the caller's
stream).  It raises if the library is not built; there is no other code path.
"""
from __future__ import annotations

import ctypes as C

import numpy as np
import torch

from . import _lib


def _mesh_struct(problem, keep):
    xyz = np.ascontiguousarray(problem.xyz, dtype=np.float64)
    conn = np.ascontiguousarray(problem.conn, dtype=np.int32)
    flags = np.ascontiguousarray(problem.flags, dtype=np.uint8)
    keep += [xyz, conn, flags]
    return _lib.Mesh(problem.dim, problem.n_nodes, problem.n_elems, problem.grid_n,
                     _lib.dptr(xyz), _lib.iptr(conn), _lib.uptr(flags))


def _sample_structs(problem, beta, lame, keep):
    """biot_materials and biot_load of one problem (arrays kept alive in `keep`)."""
    young = np.ascontiguousarray(problem.young, dtype=np.float64)
    pois = np.ascontiguousarray(problem.poisson, dtype=np.float64)
    perm = np.ascontiguousarray(problem.perm, dtype=np.float64)
    beta_a = None if beta is None else np.ascontiguousarray(beta, dtype=np.float64)
    lam_a = mu_a = None
    if lame is not None:
        lam_a = np.ascontiguousarray(lame[0], dtype=np.float64)
        mu_a = np.ascontiguousarray(lame[1], dtype=np.float64)
        if lam_a.shape != (problem.n_elems,) or mu_a.shape != (problem.n_elems,):
            raise ValueError("lame arrays must have one entry per element")
    facets = np.ascontiguousarray(problem.facets, dtype=np.int32)
    tr = np.ascontiguousarray(problem.traction, dtype=np.float64)
    coef = np.ascontiguousarray(problem.load_coef, dtype=np.float64)
    keep += [young, pois, perm, beta_a, lam_a, mu_a, facets, tr, coef]
    mat = _lib.Materials(_lib.dptr(young), _lib.dptr(pois), _lib.dptr(perm),
                         _lib.dptr(beta_a), float(problem.alpha), float(problem.stab_h),
                         _lib.dptr(lam_a), _lib.dptr(mu_a))
    load = _lib.Load(facets.shape[0], _lib.iptr(facets) if facets.size else None,
                     _lib.dptr(tr) if tr.size else None, _lib.dptr(coef))
    n_nodes, d1, ns = problem.n_nodes, problem.dim + 1, problem.n_steps + 1

    def arr(a, shape):
        a = np.ascontiguousarray(a, dtype=np.float64)
        if a.shape != shape:
            raise ValueError(f"expected shape {shape}, got {a.shape}")
        keep.append(a)
        return a
    if getattr(problem, "terms", None) is not None:
        t = np.asarray(problem.terms)
        nt = t.shape[0]
        load.n_terms = nt
        load.terms = _lib.dptr(arr(t, (nt, n_nodes, d1)))
        load.term_coef = _lib.dptr(arr(problem.term_coef, (ns, nt)))
    if getattr(problem, "prescribed", None) is not None:
        g = np.asarray(problem.prescribed)
        npr = g.shape[0]
        load.n_prescribed = npr
        load.prescribed = _lib.dptr(arr(g, (npr, n_nodes, d1)))
        load.prescribed_coef = _lib.dptr(arr(problem.prescribed_coef, (ns, npr)))
    if getattr(problem, "x0", None) is not None:
        load.x0 = _lib.dptr(arr(problem.x0, (n_nodes, d1)))
    return mat, load


def create_handle(problem, schedule="jacobi", depth=8, precond="P1", omega=0.6, cheb_degree=2,
                  cheb_ratio=4.0, lmax_safety=1.1, power_iters=20, max_batch=0, beta=None,
                  wg_per_cu=0, coarse_cells=2, use_graph=True, precision="fp64", lame=None,
                  adjoint=False, ckpt_stride=16, replay_segments=4, max_sensors=256,
                  inner="richardson", gmres_k=4, fuse_post=True):
    """biot_create (one problem) or biot_create_batch (a list of problems on the
    same mesh) on the host, no device work; returns (handle, options).

    `lame` = (lambda_e, mu_e) per element replaces the problem's E and nu (one
    problem only)."""
    lib = _lib.load()
    opt = _lib.Options()
    lib.biot_default_options(C.byref(opt))
    opt.schedule = _lib.SCHED[schedule]
    opt.depth = depth
    opt.precond = _lib.PRECOND[precond]
    opt.cheb_degree = cheb_degree
    opt.cheb_ratio = cheb_ratio
    opt.lmax_safety = lmax_safety
    opt.power_iters = power_iters
    opt.max_batch = max_batch
    opt.omega = omega
    opt.wg_per_cu = wg_per_cu
    opt.coarse_cells = coarse_cells
    opt.use_graph = 1 if use_graph else 0
    opt.precision = _lib.PRECISION[precision]
    opt.adjoint = 1 if adjoint else 0
    opt.ckpt_stride = ckpt_stride
    opt.replay_segments = replay_segments
    opt.max_sensors = max_sensors
    opt.inner = _lib.INNER[inner]
    opt.gmres_k = gmres_k
    opt.fuse_post = int(fuse_post)
    keep = []
    h = C.c_void_p()
    if isinstance(problem, (list, tuple)):
        if beta is not None or lame is not None:
            raise ValueError("beta and lame are per problem; not supported for batches")
        S = len(problem)
        meshes = (_lib.Mesh * S)()
        mats = (_lib.Materials * S)()
        loads = (_lib.Load * S)()
        for i, pb in enumerate(problem):
            meshes[i] = _mesh_struct(pb, keep)
            mats[i], loads[i] = _sample_structs(pb, None, None, keep)
        dts = np.ascontiguousarray([float(pb.dt) for pb in problem], dtype=np.float64)
        steps = np.ascontiguousarray([int(pb.n_steps) for pb in problem], dtype=np.int32)
        _lib.check(lib, lib.biot_create_batch(meshes, S, mats, loads, _lib.dptr(dts),
                                              _lib.iptr(steps), C.byref(opt), C.byref(h)), None)
    else:
        mesh = _mesh_struct(problem, keep)
        mat, load = _sample_structs(problem, beta, lame, keep)
        _lib.check(lib, lib.biot_create(C.byref(mesh), C.byref(mat), C.byref(load),
                                        float(problem.dt), problem.n_steps, C.byref(opt),
                                        C.byref(h)), None)
    return h, opt


def handle_info(lib, h) -> dict:
    inf = _lib.Info()
    _lib.check(lib, lib.biot_get_info(h, C.byref(inf)), h)
    L = inf.n_levels
    return dict(dim=inf.dim, n_nodes=inf.n_nodes, n_steps=inf.n_steps, n_levels=L,
                level_cells=list(inf.level_cells[:L]), level_nodes=list(inf.level_nodes[:L]),
                slots=inf.slots, lmax_A=list(inf.lmax_A[:L]), lmax_S=list(inf.lmax_S[:L]),
                workspace_bytes=int(inf.workspace_bytes), n_samples=inf.n_samples,
                nodes_per_sample=inf.nodes_per_sample)


def export_level(lib, h, level: int) -> dict:
    """Host copies of a level's node-blocked operators (see biot_export_level)."""
    info = handle_info(lib, h)
    nn = info["level_nodes"][level]
    W = info["slots"]
    d = info["dim"]
    out = dict(nbr=np.zeros((W, nn), np.int32), A=np.zeros((W, d * d, nn)), S=np.zeros((W, nn)))
    ptr = lambda a: C.c_void_p(a.ctypes.data)
    if level == 0:
        out.update(B=np.zeros((W, d, nn)), Bt=np.zeros((W, d, nn)), Cb=np.zeros((W, nn)),
                   F=np.zeros((nn, d + 1)))
        args = [ptr(out[k]) for k in ("nbr", "A", "S", "B", "Bt", "Cb", "F")]
    else:
        args = [ptr(out[k]) for k in ("nbr", "A", "S")] + [None] * 4
    _lib.check(lib, lib.biot_export_level(h, level, *args), h)
    return out


class BiotSolver:
    """Handle on one Biot problem bound to a GPU workspace."""

    def __init__(self, problem, schedule: str = "jacobi", depth: int = 8, precond: str = "P1",
                 omega: float = 0.6, cheb_degree: int = 2, cheb_ratio: float = 4.0,
                 lmax_safety: float = 1.1, power_iters: int = 20, max_batch: int = 0,
                 device: str = "cuda:0", beta=None, wg_per_cu: int = 0, coarse_cells: int = 2,
                 use_graph: bool = True, precision: str = "fp64", lame=None,
                 adjoint: bool = False, ckpt_stride: int = 16, replay_segments: int = 4,
                 max_sensors: int = 256, inner: str = "richardson", gmres_k: int = 4,
                 fuse_post: bool = True):
        if not torch.cuda.is_available():
            raise RuntimeError("BiotSolver needs a ROCm GPU (torch.cuda is not available)")
        self.lib = _lib.load()
        self.device = torch.device(device)
        h, opt = create_handle(problem, schedule=schedule, depth=depth, precond=precond,
                               omega=omega, cheb_degree=cheb_degree, cheb_ratio=cheb_ratio,
                               lmax_safety=lmax_safety, power_iters=power_iters,
                               max_batch=max_batch, beta=beta, wg_per_cu=wg_per_cu,
                               coarse_cells=coarse_cells, use_graph=use_graph,
                               precision=precision, lame=lame, adjoint=adjoint,
                               ckpt_stride=ckpt_stride, replay_segments=replay_segments,
                               max_sensors=max_sensors, inner=inner, gmres_k=gmres_k,
                               fuse_post=fuse_post)
        self.problem = problem
        self.batch = isinstance(problem, (list, tuple))
        first = problem[0] if self.batch else problem
        self.dim = first.dim
        self.n_samples = len(problem) if self.batch else 1
        self.sample_steps = [pb.n_steps for pb in problem] if self.batch else [problem.n_steps]
        self.n_steps = max(self.sample_steps)
        self.options = opt
        lib = self.lib
        self.h = h
        nbytes = C.c_uint64()
        self._check(lib.biot_workspace_size(h, C.byref(nbytes)))
        self.workspace_bytes = int(nbytes.value)
        self.workspace = torch.empty(self.workspace_bytes, dtype=torch.uint8, device=self.device)
        self.stream = torch.cuda.current_stream(self.device)
        self._check(lib.biot_bind(h, C.c_void_p(self.workspace.data_ptr()), self.workspace_bytes,
                                  C.c_void_p(self.stream.cuda_stream)))
        inf = handle_info(lib, h)
        # nodes of each sample's grid; all nodes of the handle (batches: the
        # samples side by side, largest grids first, each padded)
        self.sample_nodes = [pb.n_nodes for pb in problem] if self.batch else [first.n_nodes]
        self.grid_nodes = first.n_nodes
        self.n_nodes = inf["n_nodes"]

    # ------------------------------------------------------------------
    def _check(self, rc):
        return _lib.check(self.lib, rc, self.h)

    # The library enqueues on the stream the handle was bound to; tensors that
    # cross between it and the caller's current stream are ordered both ways.
    def _inputs_ready(self, *tensors):
        """The handle's stream waits for the caller's work on `tensors`."""
        cur = torch.cuda.current_stream(self.device)
        if cur != self.stream:
            self.stream.wait_stream(cur)
            for t in tensors:
                t.record_stream(self.stream)

    def _outputs_ready(self, *tensors):
        """The caller's stream waits for the handle's writes to `tensors`."""
        cur = torch.cuda.current_stream(self.device)
        if cur != self.stream:
            for t in tensors:
                t.record_stream(self.stream)
            cur.wait_stream(self.stream)

    def close(self):
        if getattr(self, "h", None):
            torch.cuda.synchronize(self.device)
            self.lib.biot_destroy(self.h)
            self.h = None
            self.workspace = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ------------------------------------------------------------------
    def reset(self):
        self._check(self.lib.biot_reset(self.h))

    def sweep(self, n: int = 1):
        self._check(self.lib.biot_sweep(self.h, int(n)))

    def residual_norms(self) -> np.ndarray:
        """[n_steps, 4] (one problem) or [n_steps, n_samples, 4] (batch)."""
        out = np.zeros((self.n_steps, self.n_samples, 4))
        self._check(self.lib.biot_residual_norms(self.h, _lib.dptr(out)))
        return out if self.batch else out[:, 0, :]

    def sample_trajectory(self, sample: int, n0: int = 0, n1: int | None = None) -> torch.Tensor:
        """Steps n0..n1-1 of one sample of a batch, [n1-n0, grid nodes, dim+1]."""
        n1 = self.sample_steps[sample] + 1 if n1 is None else n1
        out = torch.empty((n1 - n0, self.sample_nodes[sample], self.dim + 1),
                          dtype=torch.float64, device=self.device)
        self._inputs_ready(out)
        self._check(self.lib.biot_get_sample_trajectory(self.h, int(sample), n0, n1,
                                                        C.c_void_p(out.data_ptr()), 1))
        self._outputs_ready(out)
        return out

    def sample_layout(self, sample: int):
        """(first node, grid nodes) of a sample in the handle's node numbering."""
        first, n = C.c_int32(), C.c_int32()
        self._check(self.lib.biot_sample_layout(self.h, int(sample), C.byref(first), C.byref(n)))
        return first.value, n.value

    def solve_to_tol(self, rtol: float, max_sweeps: int = 1000, check_every: int = 4,
                     raise_on_failure: bool = True) -> dict:
        st = _lib.Stats()
        rc = self.lib.biot_solve_to_tol(self.h, float(rtol), int(max_sweeps), int(check_every),
                                        C.byref(st))
        if rc != 0 and raise_on_failure:
            self._check(rc)
        return dict(sweeps=st.sweeps, converged=bool(st.converged), rel_resid_u=st.rel_resid_u,
                    rel_resid_p=st.rel_resid_p, seconds=st.seconds, alg_bytes=st.alg_bytes, rc=rc)

    def trajectory(self, n0: int = 0, n1: int | None = None) -> torch.Tensor:
        n1 = self.n_steps + 1 if n1 is None else n1
        out = torch.empty((n1 - n0, self.n_nodes, self.dim + 1), dtype=torch.float64,
                          device=self.device)
        self._inputs_ready(out)
        self._check(self.lib.biot_get_trajectory(self.h, n0, n1, C.c_void_p(out.data_ptr()), 1))
        self._outputs_ready(out)
        return out

    def set_trajectory(self, X: torch.Tensor, n0: int = 0):
        X = X.to(self.device, torch.float64).contiguous()
        self._inputs_ready(X)
        self._check(self.lib.biot_set_trajectory(self.h, n0, n0 + X.shape[0],
                                                 C.c_void_p(X.data_ptr()), 1))

    def apply_operator(self, X: torch.Tensor) -> torch.Tensor:
        X = X.to(self.device, torch.float64).contiguous()
        Y = torch.empty_like(X)
        self._inputs_ready(X, Y)
        self._check(self.lib.biot_apply_operator(self.h, C.c_void_p(X.data_ptr()),
                                                 C.c_void_p(Y.data_ptr()), X.shape[0]))
        self._outputs_ready(Y)
        return Y

    def apply_precond(self, R: torch.Tensor) -> torch.Tensor:
        R = R.to(self.device, torch.float64).contiguous()
        Z = torch.empty_like(R)
        self._inputs_ready(R, Z)
        self._check(self.lib.biot_apply_precond(self.h, C.c_void_p(R.data_ptr()),
                                                C.c_void_p(Z.data_ptr()), R.shape[0]))
        self._outputs_ready(Z)
        return Z

    def apply_precond_noalloc(self, R: torch.Tensor, Z: torch.Tensor) -> torch.Tensor:
        """Z = P^{-1} R through biot_apply_precond_noalloc: the caller passes both
        device tensors ([ncols][n_nodes][dim+1] FP64); the library's work vectors
        are its static device scratch, so nothing is allocated."""
        if R.dtype != torch.float64 or Z.dtype != torch.float64 or R.shape != Z.shape:
            raise ValueError("R and Z must be float64 tensors of the same shape")
        if not (R.is_contiguous() and Z.is_contiguous()):
            raise ValueError("R and Z must be contiguous")
        self._inputs_ready(R, Z)
        self._check(self.lib.biot_apply_precond_noalloc(self.h, C.c_void_p(R.data_ptr()),
                                                        C.c_void_p(Z.data_ptr()), R.shape[0]))
        self._outputs_ready(Z)
        return Z

    def info(self) -> dict:
        return handle_info(self.lib, self.h)

    # ------------------------------------------------------------------
    @staticmethod
    def _objective(sensors, p_obs):
        nodes = np.ascontiguousarray(np.asarray(sensors), dtype=np.int32)
        obs = np.ascontiguousarray(np.asarray(p_obs), dtype=np.float64)
        if obs.ndim != 2 or obs.shape[1] != nodes.size:
            raise ValueError("p_obs must be [n_steps, n_sensors]")
        return _lib.Objective(nodes.size, _lib.iptr(nodes), _lib.dptr(obs)), (nodes, obs)

    def objective(self, sensors, p_obs) -> float:
        """J = sum_n sum_s (p^n_s - p_obs[n-1, s])^2 at the current trajectory."""
        obj, keep = self._objective(sensors, p_obs)
        J = C.c_double()
        self._check(self.lib.biot_objective_value(self.h, C.byref(obj), C.byref(J)))
        return J.value

    def adjoint(self, sensors, p_obs, rtol: float = 1e-10, max_sweeps: int = 2000) -> dict:
        """Gradient of the pressure misfit w.r.t. log K_e, lambda_e, mu_e (device
        tensors) by biot_adjoint; the trajectory must be the converged forward."""
        obj, keep = self._objective(sensors, p_obs)
        ne = self.problem.n_elems
        g = torch.empty((3, ne), dtype=torch.float64, device=self.device)
        st = _lib.AdjointStats()
        ptr = lambda i: C.c_void_p(g[i].data_ptr())
        self._inputs_ready(g)
        self._check(self.lib.biot_adjoint(self.h, C.byref(obj), float(rtol), int(max_sweeps),
                                          ptr(0), ptr(1), ptr(2), 1, C.byref(st)))
        self._outputs_ready(g)
        return dict(J=st.J, grad_logk=g[0], grad_lambda=g[1], grad_mu=g[2],
                    adjoint_sweeps=st.adjoint_sweeps, replay_sweeps=st.replay_sweeps,
                    replay_groups=st.replay_groups, adjoint_rel_resid=st.adjoint_rel_resid,
                    replay_rel_resid=st.replay_rel_resid, seconds_adjoint=st.seconds_adjoint,
                    seconds_replay=st.seconds_replay, seconds=st.seconds)

    def adjoint_states(self, n0: int = 1, n1: int | None = None) -> torch.Tensor:
        """Lam^n for n = n0..n1-1 of the last adjoint call, [n1-n0, nn, dim+1]."""
        n1 = self.n_steps + 1 if n1 is None else n1
        out = torch.empty((n1 - n0, self.n_nodes, self.dim + 1), dtype=torch.float64,
                          device=self.device)
        self._inputs_ready(out)
        self._check(self.lib.biot_get_adjoint(self.h, n0, n1, C.c_void_p(out.data_ptr()), 1))
        self._outputs_ready(out)
        return out

    def profile(self, enable: bool = True, probes=None, stride: int = 0):
        """Start (or stop) the HIP-event probes around level-0 launches; `probes`
        selects a subset by name (see _lib.PROBES), default all.  `stride` k > 1
        probes only every k-th wave of a wavefront pass and replays the waves
        between them as captured graphs; otherwise a probed pass runs eagerly."""
        if not 0 <= stride <= 255:
            raise ValueError("stride must be in 0..255")
        if not enable:
            mask = 0
        elif probes is None:
            mask = (1 << len(_lib.PROBES)) - 1
        else:
            mask = sum(1 << _lib.PROBES.index(p) for p in probes)
        if enable:
            mask |= stride << _lib.PROBE_STRIDE_SHIFT
        self._check(self.lib.biot_profile_enable(self.h, mask))

    def profile_read(self) -> dict:
        out = {}
        for i, key in enumerate(_lib.PROBES):
            n = C.c_uint64()
            ms = C.c_double()
            by = C.c_double()
            nm = C.c_char_p()
            self._check(self.lib.biot_profile_read(self.h, i, C.byref(n), C.byref(ms), C.byref(by),
                                                   C.byref(nm)))
            out[key] = dict(name=nm.value.decode(), launches=int(n.value), ms=ms.value,
                            bytes=by.value)
        return out
