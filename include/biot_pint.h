/*
 * biot_pint -- preconditioned parallel-in-time solver for the quasi-static
 * two-field Biot model on one AMD Instinct MI355X (gfx950).
 *
 * The method is the inverted time-stepping iteration of Zhou, Gu, Ju and Xing,
 * "A Parallel-in-time Method Based on Preconditioner for Biot's Model"
 * (arXiv 2310.10430):
 *   - Sec. 2.2, eq. (diseq1)/(fullysystem): stabilized P1-P1 finite elements
 *     and backward Euler give, per time step n,
 *         AA X^n = A' X^{n-1} + f^n,
 *         AA = [A  B; B' -S],  S = tau C_K + C_beta,  A' = [0 0; B' -C_beta],
 *         f^n = [F^n; -tau G^n];
 *   - Sec. 3.1, eqs. (p1)/(p2): block preconditioners P1 = [A 0; B' -S_p],
 *     P2 = [A 0; 0 -S_p] with the approximate Schur complement
 *     S_p = (tau + beta/K) C;
 *   - Sec. 3.2, Alg. 2 and Alg. 3: the outer loop iterates
 *         X^{n,m} = X^{n,m-1} + omega P^{-1}(A' X^{n-1,m} + f^n - AA X^{n,m-1})
 *     over all time steps, starting from X^{n,0} = 0; Alg. 4 runs the
 *     iterations as a pipeline ("wavefront") lagging one step each.
 * The two inner solves with A and S_p inside P are each replaced by one
 * geometric-multigrid V-cycle (Galerkin coarse operators on the nested
 * structured meshes, Chebyshev smoothing preconditioned by node-block Jacobi,
 * dense solve on the coarsest level).  The fixed point of the iteration is the
 * backward-Euler trajectory.
 *
 * Conventions
 *   - Every function returns BIOT_OK (0) or a negative error code; the message
 *     of the last error on a handle is available from biot_last_error().
 *     No C++ exception crosses this interface.
 *   - Host arrays passed in are only read during the call (they are copied).
 *   - Device memory is owned by the caller: the library computes how much it
 *     needs (biot_workspace_size) and the caller binds one buffer of that size
 *     (biot_bind).  The library never allocates or frees device memory.
 *   - All device work is enqueued on the stream given to biot_bind.  Calls that
 *     return host values synchronize that stream; the others do not.
 *   - Degrees of freedom are node-major: dof = node*(dim+1) + c with
 *     c = 0..dim-1 the displacement components and c = dim the pressure.  A
 *     trajectory is [n_steps+1][n_nodes][dim+1] doubles; row 0 is X^0.
 *   - Prescribed (Dirichlet) dofs are flagged per node (biot_mesh.dirichlet);
 *     their values come from biot_load (zero unless prescribed terms are given)
 *     and are part of the trajectory.
 *   - Meshes must be the structured unit-square (2D, right triangles split
 *     along (i,j)->(i+1,j+1)) or unit-cube (3D, Kuhn tetrahedra) grids with
 *     lexicographic node numbering; grid_n gives the cells per side.
 *
 * Calls on one handle must not overlap; different handles are independent.
 */
#ifndef BIOT_PINT_H
#define BIOT_PINT_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define BIOT_OK 0
#define BIOT_EINVAL (-1)        /* bad argument or mesh                        */
#define BIOT_ENOMEM (-2)        /* workspace too small                          */
#define BIOT_EHIP (-3)          /* a HIP runtime call failed                    */
#define BIOT_EDIVERGED (-4)     /* residual became non-finite or grew too much  */
#define BIOT_ENOTCONVERGED (-5) /* max_sweeps reached above tolerance           */
#define BIOT_ESTATE (-6)        /* call out of order (e.g. not bound yet)       */

#define BIOT_SCHED_JACOBI 0     /* every step couples to the previous sweep     */
#define BIOT_SCHED_WAVEFRONT 1  /* Alg. 2 order: step n couples to step n-1 of  */
                                /* the same sweep; `depth` sweeps per pass run  */
                                /* as a pipeline (Alg. 4)                       */
#define BIOT_PRECOND_P1 1       /* eq. (p1), block lower triangular             */
#define BIOT_PRECOND_P2 2       /* eq. (p2), block diagonal                     */
#define BIOT_PRECISION_FP64 0   /* everything in FP64                           */
#define BIOT_PRECISION_MIXED 1  /* residual, coupling and update in FP64; the   */
                                /* preconditioner (both V-cycles, the pressure  */
                                /* stage) in FP32.  Each sweep is one step of   */
                                /* iterative refinement, so the fixed point is  */
                                /* the FP64 one                                 */
#define BIOT_INNER_RICHARDSON 0  /* unit = one damped preconditioned update     */
#define BIOT_INNER_GMRES 1       /* unit = GMRES(k) on AA x = b^{n,m} from      */
                                 /* X^{n,m-1}, left-preconditioned by P (the    */
                                 /* Krylov solver K of Alg. 3; PETSc's default  */
                                 /* side), minimizing ||P^{-1}(b - AA x)||      */

typedef struct biot_handle biot_handle;

/* Mesh and boundary description (Sec. 2.1 boundary conditions). */
typedef struct {
  int32_t dim;               /* 2 or 3                                          */
  int32_t n_nodes;           /* (grid_n+1)^dim                                  */
  int32_t n_elems;           /* simplices                                       */
  int32_t grid_n;            /* cells per side of the structured grid (>= 1)    */
  const double* xyz;         /* [n_nodes][dim], node (i,j,k) at (i,j,k)/grid_n  */
  const int32_t* conn;       /* [n_elems][dim+1], positively oriented           */
  const uint8_t* dirichlet;  /* [n_nodes]; bit c<dim: u_c prescribed, bit dim: */
                             /* p prescribed (values: biot_load)               */
} biot_mesh;

/* Materials per element (Sec. 2.1: Lame parameters from E and nu). */
typedef struct {
  const double* young;    /* [n_elems] Young's modulus E > 0                      */
  const double* poisson;  /* [n_elems] Poisson ratio, -1 < nu < 0.5                */
  const double* perm;     /* [n_elems] K = permeability / viscosity >= 0           */
  const double* beta;     /* [n_elems] stabilization parameter, or NULL for         */
                          /* beta_e = alpha^2 stab_h^2 / (4 (lambda_e + 2 mu_e))     */
  double alpha;           /* Biot-Willis coefficient                               */
  double stab_h;          /* mesh size entering the default beta                    */
  const double* lame_lambda; /* [n_elems] lambda_e, or NULL: both given together   */
  const double* lame_mu;     /* [n_elems] mu_e > 0; when set, young and poisson     */
                             /* are ignored (they may be NULL)                      */
} biot_materials;

/* Right-hand side of eq. (fullysystem) (Sec. 2.2): per step n,
 *     f^n = [F^n; -tau G^n] = c(n) F_traction + sum_j c_j(n) F_j,
 * the prescribed (Dirichlet) values g^n = sum_k d_k(n) G_k at the flagged dofs,
 * and the initial state X^0.
 *   - Traction: constant per boundary facet, |facet|/dim of it to each vertex.
 *   - Load terms F_j: assembled vectors in the trajectory layout, e.g. a body
 *     force int f.v on the displacement rows and -tau int g q of a fluid source
 *     on the pressure rows.  Entries at prescribed dofs are ignored.
 *   - Prescribed values: G_k in the trajectory layout; only the entries at the
 *     flagged dofs are read.  The library lifts them into the right-hand side
 *     with the assembled operators: on the free rows the step equation becomes
 *         AA_ff x^n = f^n_f - (AA g^n)_f + (A' g^{n-1})_f + (A' X^{n-1})_f-part,
 *     i.e. two more internal load terms per G_k, with multipliers d_k(n) and
 *     d_k(n-1); the values themselves are written into the trajectory at every
 *     step (biot_bind, biot_reset) and never changed by a sweep.
 *   - X^0 (NULL: g^0 at the prescribed dofs, zero elsewhere): row 0 of the
 *     trajectory; where its prescribed part differs from g^0 the difference is
 *     lifted into step 1.
 * Arrays are read during biot_create only. */
typedef struct {
  int32_t n_facets;            /* may be 0                                       */
  const int32_t* facet_nodes;  /* [n_facets][dim]                                */
  const double* traction;      /* [n_facets][dim]                                */
  const double* coef;          /* [n_steps+1]: multiplier c(n) of the traction   */
                               /* (may be NULL when n_facets = 0)                */
  int32_t n_terms;             /* 0..8 assembled load terms                      */
  const double* terms;         /* [n_terms][n_nodes][dim+1]                      */
  const double* term_coef;     /* [n_steps+1][n_terms]: c_j(n)                   */
  int32_t n_prescribed;        /* 0..3 prescribed-value terms                    */
  const double* prescribed;    /* [n_prescribed][n_nodes][dim+1]                 */
  const double* prescribed_coef; /* [n_steps+1][n_prescribed]: d_k(n)            */
  const double* x0;            /* [n_nodes][dim+1] initial state, or NULL        */
} biot_load;

typedef struct {
  int32_t schedule;     /* BIOT_SCHED_*  (default JACOBI)                          */
  int32_t depth;        /* wavefront: sweeps per pass = iterations in flight (8)   */
  int32_t precond;      /* BIOT_PRECOND_* (default P1)                             */
  int32_t cheb_degree;  /* Chebyshev smoother degree per smoothing call, 2..8 (2)  */
  double cheb_ratio;    /* smoother interval [lmax/ratio, lmax] (4)                */
  double lmax_safety;   /* factor on the power-iteration estimate of lmax (1.1)    */
  int32_t power_iters;  /* power iterations for lmax per level (20)                */
  int32_t max_batch;    /* Jacobi: columns per launch, <= 0 for all steps (0)      */
  double omega;         /* damping of the outer update (0.6)                       */
  int32_t wg_per_cu;    /* workgroups per compute unit of the node-blocked kernels' */
                        /* grids, 0..32; 0: each kernel's occupancy, at most 3   */
                        /* (3D level-0 residual and smoother: 4) (0); the fused  */
                        /* post-smoothing sizes its own grid (fuse_post)         */
  int32_t coarse_cells; /* multigrid: halve the grid while it is even and the half */
                        /* still has >= coarse_cells cells per side (2); the last  */
                        /* level is solved with a dense inverse                    */
  int32_t use_graph;    /* wavefront: replay each pass as a captured HIP graph (1) */
  int32_t precision;    /* BIOT_PRECISION_* (default FP64)                          */
  /* adjoint (biot_adjoint); its buffers count in the workspace only when on    */
  int32_t adjoint;         /* 1: reserve the adjoint buffers (0)                   */
  int32_t ckpt_stride;     /* 0: keep the whole forward trajectory; s > 0: keep    */
                           /* X^{ks} and X^N only, overwrite the forward           */
                           /* trajectory with the adjoint one and recompute each   */
                           /* segment from its checkpoint for the gradient (16)    */
  int32_t replay_segments; /* segments recomputed together (4)                     */
  int32_t max_sensors;     /* capacity of the objective's sensor list (256)        */
  int32_t inner;           /* BIOT_INNER_* : what one unit does (RICHARDSON)       */
  int32_t gmres_k;         /* GMRES iterations per unit, 1..8 (4); omega unused    */
  int32_t fuse_post;       /* 1: in 2D with smoother degree 2, run a level's      */
                           /* coarse-grid correction and both post-smoothing      */
                           /* steps in one launch (same result bit for bit);      */
                           /* 0: three launches (1)                               */
} biot_options;

/* Pressure-misfit objective J = sum_{n=1..N} sum_s (p^n(node_s) - p_obs[n-1][s])^2. */
typedef struct {
  int32_t n_sensors;        /* 1..max_sensors                                     */
  const int32_t* nodes;     /* [n_sensors] distinct node ids (host)               */
  const double* p_obs;      /* [n_steps][n_sensors] observed pressure (host)      */
} biot_objective;

typedef struct {
  double J;                 /* objective at the forward trajectory                */
  int32_t adjoint_sweeps;   /* outer sweeps of the adjoint solve                  */
  int32_t replay_sweeps;    /* outer sweeps summed over the replayed groups       */
  int32_t replay_groups;    /* groups of segments recomputed (0 without ckpt)     */
  double adjoint_rel_resid; /* max over fields of the adjoint's relative residual */
  double replay_rel_resid;  /* worst over groups of the replays' residuals        */
  double seconds_adjoint;   /* wall time of the adjoint solve                     */
  double seconds_replay;    /* wall time of replays and gradient contraction      */
  double seconds;           /* wall time of the call                              */
} biot_adjoint_stats;

typedef struct {
  int32_t sweeps;       /* outer sweeps performed                                  */
  int32_t converged;    /* 1 if rel_resid <= rtol                                  */
  double rel_resid_u;   /* max_n ||r_u^n|| / max_n ||b_u^n||                       */
  double rel_resid_p;   /* max_n ||r_p^n|| / max_n ||b_p^n||; a field whose b is   */
                        /* zero at every step is divided by max_n ||b_u^n|| and  */
                        /* max_n ||b_p^n|| combined (root of the sum of squares) */
  double seconds;       /* wall time of the call                                   */
  double alg_bytes;     /* algorithmic bytes of all kernels the call enqueued:     */
                        /* each launch's distinct global inputs and outputs once  */
                        /* (operators once per launch, vectors once per column);  */
                        /* alg_bytes / seconds is the solve's effective bandwidth */
} biot_stats;

typedef struct {
  int32_t dim, n_nodes, n_steps, n_levels;
  int32_t level_cells[16];   /* cells per side per multigrid level                */
  int32_t level_nodes[16];   /* nodes per level                                    */
  int32_t slots;             /* node-blocked ELL slots per node (7 in 2D, 15 in 3D) */
  double lmax_A[16];         /* spectral bounds used by the smoothers (with safety) */
  double lmax_S[16];
  uint64_t workspace_bytes;
  int32_t n_samples;         /* samples of a batch handle (1 otherwise)             */
  int32_t nodes_per_sample;  /* node stride of a sample in the trajectory layout    */
} biot_info_t;

/* Fills *opt with the defaults listed above. */
int biot_default_options(biot_options* opt);

/* Assembles the step matrix, the coupling, the load and the multigrid
 * hierarchy on the host (FP64).  dt = tau > 0, n_steps >= 1.  On success
 * *out is a new handle that must be released with biot_destroy(). */
int biot_create(const biot_mesh* mesh, const biot_materials* mat, const biot_load* load,
                double dt, int32_t n_steps, const biot_options* opt, biot_handle** out);

/* A batch of n_samples independent problems, each on its own structured mesh
 * (meshes[i]; grids may differ in size), with its own materials, load, dt and
 * number of steps, solved together: the samples are stored as disconnected
 * grids side by side, largest grid first (stable; biot_sample_layout gives a
 * sample's nodes), each padded to a multiple of 256 nodes with inert
 * prescribed nodes, so that no workgroup's node block straddles two samples.
 * Every launch of the sweep works on all samples that take part in it: a
 * multigrid level on the samples whose hierarchy reaches it as its own
 * launches, the fused coarse end on every sample at once (each from its own
 * first fused level; batches of different grids need one for every sample),
 * and a sample skips the columns of steps past its own n_steps (nothing is
 * computed for them).  The handle's step count is the largest n_steps.  A
 * larger grid must not have a shallower hierarchy.  Convergence is the worst
 * sample's relative residual over its own steps.  All samples must have the
 * same right-hand-side structure (traction or not, n_terms, n_prescribed, x0
 * given or not) and their multipliers (coef, term_coef, prescribed_coef) must
 * agree on their common steps.  The spectral bounds of a multigrid level are
 * the maximum over its samples.  meshes, mats, loads, dts and n_steps have
 * n_samples entries.  Trajectory calls see [n_steps+1][n_nodes][dim+1] with
 * all samples' nodes (biot_get_info); biot_get_sample_trajectory extracts one
 * sample and biot_residual_norms reports samples in the order given.  The
 * adjoint needs n_samples = 1. */
int biot_create_batch(const biot_mesh* meshes, int32_t n_samples, const biot_materials* mats,
                      const biot_load* loads, const double* dts, const int32_t* n_steps,
                      const biot_options* opt, biot_handle** out);

/* Where sample `sample` of a handle sits in the node numbering of its
 * trajectory: nodes first_node .. first_node + n_nodes - 1 (its grid nodes; a
 * single-problem handle has one sample at node 0). */
int biot_sample_layout(const biot_handle* h, int32_t sample, int32_t* first_node,
                       int32_t* n_nodes);

/* Device bytes the handle needs (operators, two trajectories, work vectors). */
int biot_workspace_size(const biot_handle* h, uint64_t* bytes);

/* Binds caller-owned device memory (>= biot_workspace_size bytes, 256-byte
 * aligned) and the HIP stream (hipStream_t, NULL for the default stream),
 * uploads the operators and sets the trajectory to zero. */
int biot_bind(biot_handle* h, void* device_ptr, uint64_t bytes, void* hip_stream);

/* The initial iterate of Alg. 2: X^{n,0} = 0 for n >= 1 except the prescribed
 * values, X^0 as given in biot_load (zero by default). */
int biot_reset(biot_handle* h);

/* n_sweeps outer sweeps.  JACOBI: each sweep updates every step from the
 * previous sweep.  WAVEFRONT: floor(n_sweeps/depth) passes of `depth`
 * Gauss-Seidel-in-time sweeps, each run as N+depth-1 pipelined waves, then one
 * shallower pass for the remainder. */
int biot_sweep(biot_handle* h, int32_t n_sweeps);

/* Space-time residual of the current trajectory: for every step n >= 1 the
 * squared norms [||r_u||^2, ||r_p||^2, ||b_u||^2, ||b_p||^2] of
 * r = A' X^{n-1} + f^n - AA X^n and b = A' X^{n-1} + f^n, written to
 * norms[n_steps][n_samples][4] (host).  Synchronizes the stream. */
int biot_residual_norms(biot_handle* h, double* norms);

/* Sweeps until max(rel_resid_u, rel_resid_p) <= rtol or max_sweeps.  JACOBI
 * checks every `check_every` sweeps; WAVEFRONT checks after each pass, the
 * first of full depth and later ones sized from the contraction observed so
 * far.  Returns BIOT_ENOTCONVERGED if the
 * tolerance was not met, BIOT_EDIVERGED on non-finite residuals.  stats may be
 * NULL.  Synchronizes the stream. */
int biot_solve_to_tol(biot_handle* h, double rtol, int32_t max_sweeps, int32_t check_every,
                      biot_stats* stats);

/* Copies steps n0..n1-1 of the trajectory to dst ([n1-n0][n_nodes][dim+1]),
 * a device pointer if dst_on_device else host (host copies synchronize). */
int biot_get_trajectory(biot_handle* h, int32_t n0, int32_t n1, double* dst, int32_t dst_on_device);

/* Steps n0..n1-1 (n1 <= that sample's n_steps + 1) of one sample's trajectory,
 * [n1-n0][n_nodes][dim+1] (its grid nodes only), to host or device memory. */
int biot_get_sample_trajectory(biot_handle* h, int32_t sample, int32_t n0, int32_t n1, double* dst,
                               int32_t dst_on_device);

/* Overwrites steps n0..n1-1 of the trajectory (warm start / resume).  The
 * values at prescribed dofs are taken as given (sweeps keep them), so src
 * should carry the prescribed values, e.g. a trajectory read back earlier. */
int biot_set_trajectory(biot_handle* h, int32_t n0, int32_t n1, const double* src,
                        int32_t src_on_device);

/* Y = AA X for ncols device columns [ncols][n_nodes][dim+1] (diagnostic). */
int biot_apply_operator(biot_handle* h, const double* X, double* Y, int32_t ncols);

/* Z = P^{-1} R with the multigrid inner solves, for ncols device columns. */
int biot_apply_precond(biot_handle* h, const double* R, double* Z, int32_t ncols);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * Z = P^{-1} R as biot_apply_precond, for ncols device columns
 * [ncols][n_nodes][dim+1] (R read, Z written, both caller-owned), but the
 * V-cycle work vectors live in a static device array of the library (64 MiB
 * per device, held until the process ends) instead of the bound workspace.
 * Columns are processed in batches of as many as that array holds; the part of
 * it a batch uses is zeroed first by a fill kernel (no memset node).  The call
 * allocates nothing and calls no allocating library routine.  BIOT_ENOMEM when
 * one column's work vectors exceed 64 MiB (about 1.5e6 nodes in 2D, FP64).
 * All calls on one device share that array: calls that overlap on one device
 * (from any handle or thread) race and must be serialized by the caller.  The
 * handle must be bound; the work is enqueued on its stream. */
int biot_apply_precond_noalloc(biot_handle* h, const double* R, double* Z, int32_t ncols);

int biot_get_info(const biot_handle* h, biot_info_t* info);

/* Probes: HIP events recorded on the handle's stream around every level-0
 * launch (every launch for POST_U and POST_P) of the selected kernels below,
 * with the algorithmic bytes each launch
 * moves (distinct global inputs and outputs counted once).  `mask` has bit p
 * set for probe p (0 disables); enabling or disabling clears the accumulators;
 * reading synchronizes the stream.  While probes are on, wavefront passes run
 * their launches eagerly instead of replaying a captured graph, unless bits
 * BIOT_PROBE_STRIDE_SHIFT.. +7 of `mask` hold a stride k > 1: then only the
 * waves w with w mod k = k/2 run eagerly and are probed, and the waves between
 * them replay captured graphs (so a timed solve keeps most of the graph
 * replay's speed while its probes sample every k-th wave). */
#define BIOT_PROBE_RESIDUAL 0     /* fused residual + coupling + norms           */
#define BIOT_PROBE_CHEB_U 1       /* displacement Chebyshev smoothing steps      */
#define BIOT_PROBE_CHEB_P 2       /* pressure Chebyshev smoothing steps          */
#define BIOT_PROBE_LEVRES_U 3     /* displacement residual before restriction    */
#define BIOT_PROBE_LEVRES_P 4     /* pressure residual before restriction        */
#define BIOT_PROBE_PSTAGE 5       /* P1 pressure stage t = B' z_u - r_p          */
#define BIOT_PROBE_POST_U 6       /* displacement coarse-grid correction and     */
                                  /* post-smoothing, both steps in one launch   */
                                  /* (2D, degree 2, fuse_post), on every level  */
                                  /* outside the fused tail                     */
#define BIOT_PROBE_POST_P 7       /* the same for the pressure field (on level 0 */
                                  /* in sweeps the last step writes the outer   */
                                  /* update)                                    */
#define BIOT_PROBE_COUNT 8
#define BIOT_PROBE_ALL 0xFF
#define BIOT_PROBE_STRIDE_SHIFT 16
int biot_profile_enable(biot_handle* h, int32_t mask);
int biot_profile_read(biot_handle* h, int32_t probe, uint64_t* launches, double* total_ms,
                      double* total_bytes, const char** name);

/* Host copies of the operators of multigrid level `level` as assembled by
 * biot_create (after the boundary conditions), in the node-blocked layout:
 *   nbr [W][nn]           neighbour node of each slot (slot 0 = the node)
 *   A   [W][dim*dim][nn]  displacement blocks, entry a*dim+b
 *   S   [W][nn]           tau C_K + C_beta (coarse levels: Galerkin products)
 * and, for level 0 only,
 *   B   [W][dim][nn]      matrix of -b(v,q): u-row, p-column
 *   Bt  [W][dim][nn]      its transpose: p-row, u-column
 *   Cb  [W][nn]           C_beta
 *   F   [nn][dim+1]       load for a unit multiplier.
 * Any pointer may be NULL.  Sizes follow biot_get_info (W = slots). */
int biot_export_level(const biot_handle* h, int32_t level, int32_t* nbr, double* A, double* S,
                      double* B, double* Bt, double* Cb, double* F);

/* J of the objective at the current trajectory (host value; synchronizes). */
int biot_objective_value(biot_handle* h, const biot_objective* obj, double* J);

/* Gradient of the pressure misfit J with respect to the per-element parameters
 * log K_e, lambda_e and mu_e, by the discrete adjoint of the backward-Euler
 * trajectory (the fixed point of the inverted iteration, Sec. 3.2).  With the
 * space-time system calA X = f of eq. (fullysystem) (block row n: AA on the
 * diagonal, -A' below it), the adjoint states solve calA^T Lam = dJ/dX, i.e.
 *     AA Lam^n = dJ/dX^n + A'^T Lam^{n+1},   Lam^{N+1} = 0,
 * which is run through the same inverted iteration, schedule and preconditioner
 * as the forward problem, backward in time (AA is symmetric).  Then
 *     dJ/dtheta = -sum_n Lam^n . (dAA/dtheta X^n - dA'/dtheta X^{n-1}),
 * contracted element by element: log K through S = tau C_K + C_beta, lambda and
 * mu through A and through the default beta_e (no beta term when the caller
 * gave beta).  A global lambda or mu has the sum of the entries as gradient.
 * The trajectory in the handle is taken as the converged forward solution
 * (call biot_solve_to_tol first) and the call needs options.adjoint = 1;
 * such handles take homogeneous prescribed values only (biot_create rejects
 * prescribed terms and an X^0 that is nonzero at prescribed dofs).
 * With ckpt_stride s > 0 the forward trajectory is overwritten (afterwards
 * biot_sweep, biot_solve_to_tol and biot_get_trajectory return BIOT_ESTATE until
 * biot_reset); each segment of s steps is recomputed from its checkpoint,
 * replay_segments at a time, to rtol.  rtol and max_sweeps apply to the adjoint
 * solve and to every replay.  grad_* are [n_elems] doubles, device pointers if
 * grads_on_device else host; any may be NULL.  stats may be NULL; when the
 * adjoint solve or a replay fails, stats still reports how far it got.
 * Synchronizes the stream. */
int biot_adjoint(biot_handle* h, const biot_objective* obj, double rtol, int32_t max_sweeps,
                 double* grad_logk, double* grad_lambda, double* grad_mu, int32_t grads_on_device,
                 biot_adjoint_stats* stats);

/* Copies the adjoint states Lam^n, n = n0..n1-1 (1 <= n0 <= n1 <= n_steps+1) of
 * the last biot_adjoint call to dst ([n1-n0][n_nodes][dim+1], node-major). */
int biot_get_adjoint(biot_handle* h, int32_t n0, int32_t n1, double* dst, int32_t dst_on_device);

/* Message of the last failed call on h (or of the last failed biot_create when
 * h is NULL).  Valid until the next call on the same handle. */
const char* biot_last_error(const biot_handle* h);

const char* biot_version(void);

void biot_destroy(biot_handle* h);

#ifdef __cplusplus
}
#endif

#endif /* BIOT_PINT_H */
