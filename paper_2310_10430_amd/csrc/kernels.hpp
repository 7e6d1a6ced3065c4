// Device-side views and kernel launchers of the Biot parallel-in-time sweep.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace biot {

constexpr int kBlock = 256;   // threads per workgroup (4 wave64)
// fused post-smoothing patches: 16 x 16 nodes, stepping by the 14 x 14 interior
constexpr int kPatchInterior = 14;

// One multigrid level on the device (node-blocked ELL, see setup.hpp), with
// operator values of type T (double, or float for the mixed-precision
// preconditioner).
struct ColDesc;

template <typename T>
struct LevelView {
  int nn, W, n_cells;
  int copies, nn1, nreal;  // disconnected copies of the grid (samples of a batch),
                           // nodes per copy with padding, grid nodes per copy
                           // (those of copy 0 when the copies differ)
  // Copies (samples) may be grids of different sizes, largest first.  A launch
  // works on the first `nact` nodes (whole copies); vectors keep the stride nn.
  int nact;
  const int32_t* cbase;   // [copies+1] first node of each copy (multiples of 256)
  const int32_t* ccells;  // [copies] cells per side of each copy
  const int32_t* bcopy;   // [nn/256] copy of each node block
  // steps of each copy and, when set, the launch's column descriptors: column
  // c is skipped for copy cp when act[c].step > csteps[cp] (the sample has
  // fewer steps); the active columns of a launch are contiguous for each copy
  const int32_t* csteps;
  const ColDesc* act;
  // fused post-smoothing patches of this level (k_post2): patch p covers
  // patch ptab[2p+1] of copy ptab[2p]; npatch of them (whole copies, like nact)
  const int32_t* ptab;
  int npatch;
  const int32_t* nbr;    // [W][nn]
  const T* A;            // [W][dim*dim][nn]
  const T* S;            // [W][nn]
  const T* Ainv;         // [dim*dim][nn]
  const T* Sinv;         // [nn]
  const uint8_t* fixed;  // [nn]
  const T* AD;           // [W][dim*dim][nn]  A_k(i) Ainv(nbr_k(i))
  const T* SD;           // [W][nn]           S_k(i) Sinv(nbr_k(i))
};
using LevelDev = LevelView<double>;

// Fine-level coupling blocks and load (level 0 only, FP64).
struct FineDev {
  const double* B;      // [W][dim][nn]
  const double* Bt;     // [W][dim][nn]
  const double* Cb;     // [W][nn]
  const double* F;      // load terms [nt][nn][dim+1] (zero at prescribed dofs)
  int nt;               // number of load terms (0 in the adjoint recursion)
  const double* gload;  // adjoint only: pressure-row load [N][nn] per column step
};

// One (time step, iteration) column of a batch.
struct ColDesc {
  const double* xcur;   // X^{n,m-1}            [nn][dim+1]
  const double* xprev;  // coupling source X^{n-1,*}
  double* xout;         // X^{n,m}
  double* xout2;        // optional second copy (may be null)
  const double* tc;     // load-term multipliers of step n: f^n = sum_j tc[j] F_j
  double c0;            // tc[0], kept here so that kernels read it with the
                        // descriptor (one scalar load) rather than through tc
  int step;             // n
  int pad;
};

// Probing: the next node-blocked launch issued by this host thread records
// `start` and `stop` with its own dispatch (the kernel's begin and end), then
// the pair is disarmed; launch_events_armed() tells whether it is still pending.
void set_launch_events(hipEvent_t start, hipEvent_t stop);
bool launch_events_armed();

// Launchers (all asynchronous on `st`).  `nc` = number of columns in the batch;
// per-column work vectors are contiguous with stride nn*comps.  The node-blocked
// kernels split their (node block, column) units evenly over a grid of one
// workgroup per resident slot of the device; `wpc` > 0 fixes the workgroups per
// compute unit instead of the kernel's occupancy.  T is the type of the
// preconditioner's vectors and operators (double or float); the residual and
// the state update always run in FP64.

// `adj`: the adjoint recursion (coupling A'^T, load F.gload; see k_residual)
template <typename T>
void launch_residual(int dim, const LevelDev& L, const FineDev& F, const ColDesc* cols, int nc,
                     T* ru, T* rp, double* partials, int partial_stride, int wpc, bool adj,
                     hipStream_t st);
// Chebyshev step d <- c1 d + c2 D^{-1}(b - K xin), xout = xin + d.  With `upd`
// (pressure field, level 0) the step writes the outer update
// X^{n,m} = X^{n,m-1} + omega [zu; xin + d] through the descriptors instead.
// wd = false skips storing d; dx: where the previous d comes from (0: d;
// 1: xin, after a first step from zero; 2: xin - xout, after the first
// post-smoothing step, xout still holding that step's input).  first = true:
// the step after the first step from zero, which is never stored: xin =
// it D^{-1} b is formed on the fly through the folded operators (L.AD, L.SD);
// xin is then unused.
template <typename T>
void launch_cheb(int dim, int comps, const LevelView<T>& L, bool is_A, const T* b, const T* xin,
                 T* xout, T* d, int nc, double c1, double c2, bool wd, int dx, bool first,
                 double it, const ColDesc* upd, const T* zu, double omega, int wpc, bool fine,
                 hipStream_t st);
template <typename T>
void launch_level_residual(int dim, int comps, const LevelView<T>& L, bool is_A, const T* b,
                           const T* x, T* r, int nc, int wpc, hipStream_t st);
template <typename T>
void launch_restrict(int dim, int comps, const LevelView<T>& Lf, const LevelView<T>& Lc,
                     bool is_A, const T* rf, T* bc, int nc, hipStream_t st);
template <typename T>
void launch_prolong(int dim, int comps, const LevelView<T>& Lf, const LevelView<T>& Lc, bool is_A,
                    const T* xin, const T* xc, T* xout, int nc, int wpc, hipStream_t st);
// the coarse-grid correction x2 = x + P xc and the two post-smoothing steps of
// degree 2, fused (2D, any number of samples): x, xc -> x4, with the first
// step's c2 and the second step's c1, c2 (k_post2); x2 is not stored.  With
// `upd` (pressure field, level 0) the last step writes the outer update
// X^{n,m} = X^{n,m-1} + omega [zu; x4] through the descriptors instead of x4.
template <typename T>
void launch_post2(int comps, const LevelView<T>& L, const LevelView<T>& Lc, bool is_A, const T* b,
                  const T* xin, const T* xc, T* x4, int nc, double c2a, double c1b, double c2b,
                  const ColDesc* upd, const T* zu, double omega, int wpc, hipStream_t st);
// dense coarsest solve per column and copy: n grid dofs per copy, `stride` dofs
// per copy with padding, Minv = copies dense inverses
template <typename T>
void launch_coarse_solve(int n, int stride, int copies, const T* Minv, const T* b, T* x, int nc,
                         hipStream_t st);

// The coarse end of a V-cycle (levels t..last) in one launch, one workgroup
// per column with the vectors in LDS (k_vcycle_tail).  L[0] is level t, whose
// right-hand side b (no first Chebyshev step yet) is read and whose V-cycle
// result is written to x; L[nlev-1] is the densely solved coarsest level.
constexpr int kTailMaxLevels = 8;
constexpr int kMaxLevels = 16;
// LDS budget of the fused V-cycle tail: gfx950's 160 KB per workgroup (capped
// at bind by what the device reports)
constexpr size_t kTailMaxLds = 160 * 1024;
// the tail of one copy: its levels t0 .. t0+nlev-1 (global level numbers), the
// LDS offset (in values) of each of them, and the offset of its dense inverse
struct TailCopy {
  int t0, nlev;
  int off[kTailMaxLevels];
  long long moff;
};
template <typename T>
struct TailDev {
  int degree;
  int cp0, copies;                // the launch covers copies cp0 .. cp0+copies-1
  LevelView<T> L[kMaxLevels];     // every level of the hierarchy
  double theta[kMaxLevels], delta[kMaxLevels], sigma[kMaxLevels];
  const TailCopy* tc;             // [copies]
  const T* Minv;
  const T* b[kMaxLevels];         // per level: right-hand sides (read at a copy's t0)
  T* x[kMaxLevels];               // per level: results (written at a copy's t0)
};
// LDS vectors per (non-coarsest) tail level for a smoother degree, and the
// tail's LDS bytes
int tail_vectors(int degree);
// threads of a tail workgroup (one workgroup per column and sample copy)
int tail_block_threads(int dim);
size_t tail_lds_bytes(const int* level_nn, int nlev, int comps, int tbytes, int degree);
// one workgroup per (column, copy with a tail); each copy reads TD.b and
// writes TD.x at its own first tail level; `lds` = the largest copy's bytes
template <typename T>
void launch_vcycle_tail(int dim, int comps, const TailDev<T>& TD, int nc, size_t lds,
                        hipStream_t st);
template <typename T>
void launch_pstage(int dim, const LevelView<T>& L, const T* Bt, bool p1, const T* zu, const T* rp,
                   T* t, int nc, int wpc, hipStream_t st);
// csteps/bcopy (may be null): columns past a copy's steps are skipped
template <typename T>
void launch_update(int dim, int nn, const ColDesc* cols, const T* zu, const T* zp, double omega,
                   int nc, const int32_t* csteps, const int32_t* bcopy, hipStream_t st);
template <typename T>
void launch_unpack(int dim, int nn, const double* X, T* ru, T* rp, int nc, hipStream_t st);
template <typename T>
void launch_pack(int dim, int nn, const T* zu, const T* zp, double* Z, int nc, hipStream_t st);

// forward initial iterate with prescribed values (k_init_traj): columns
// 0..ncols-1 of X; x0 may be null
void launch_init_traj(double* X, int ncols, int nn, int D1, const double* x0, const double* pres,
                      const double* pcoef, int npres, const uint8_t* fixed, hipStream_t st);
// zeroes `bytes` (a multiple of 16; p 16-byte aligned) with a fill kernel, which
// unlike a memset node may sit in a captured graph
void launch_zero(void* p, size_t bytes, hipStream_t st);

// norms[c][copy][4] = sums of the block partials of each copy (the blocks of
// copy cp are those of nodes cbase[cp] .. cbase[cp+1]-1)
void launch_reduce_norms(const double* partials, const int32_t* cbase, int copies,
                         int partial_stride, double* norms, int nc, hipStream_t st);
void launch_apply_operator(int dim, const LevelDev& L, const FineDev& F, const double* X,
                           double* Y, int nc, hipStream_t st);

// ---- adjoint (adjoint.hip) ----
// Element data of the gradient contraction (see HostProblem::geo / conn_t).
struct ElemDev {
  int ne;
  const int32_t* conn;   // [dim+1][ne]
  const double* geo;     // [(dim+1)*dim + 1][ne]: vertex gradients, then |e|
  const double* coefK;   // [ne] tau K_e
  const double* dbl;     // [ne] d beta_e / d lambda_e (0 if beta was given)
  const double* dbm;     // [ne] d beta_e / d mu_e
};
// dJ/dX of the pressure misfit: gload[(m-1)*nn + node_s] = 2 (p^n_s - d^n_s)
// with n = N+1-m (reversed time) for free pressures, and misfit^2 per entry in
// jpart[(n-1)*S + s].  gload must be zero elsewhere beforehand.
void launch_sensor_load(int dim, int nn, int N, int S, const double* X, const int32_t* sens,
                        const double* pobs, const uint8_t* fixed, double* gload, double* jpart,
                        hipStream_t st);
// out[0] = sum of x[0..n) in a fixed order (one workgroup)
void launch_sum(const double* x, int n, double* out, hipStream_t st);
// replay start values for steps n0..n0+L of a group: X^{n0} from its checkpoint,
// the others linearly interpolated between the checkpoints around them
// (checkpoint k holds X^{k s} for k < K = ceil(N/s), checkpoint K holds X^N)
void launch_lerp_init(size_t col, const double* ck, int s, int N, int n0, int L, double* out,
                      hipStream_t st);
// per-element partial sums over steps [n_beg, n_end) in chunks of `chunk` steps:
// part[(kbase + y)][4][ne] = sum over chunk y of (grad lp . grad p,
//   div lu div u, 2 eps(lu):eps(u), grad lp . grad (p - p_prev)) |e|,
// with X^n at xbase + (n - xstep0) col and Lam^n at lam_top - n col
void launch_grad_partial(int dim, const ElemDev& E, size_t col, const double* xbase, int xstep0,
                         const double* lam_top, int n_beg, int n_end, int chunk, int kbase,
                         double* part, hipStream_t st);
// gradients from the partials of nchunks chunks (summed in chunk order)
void launch_grad_finish(const ElemDev& E, const double* part, int nchunks, double* g_logk,
                        double* g_lam, double* g_mu, hipStream_t st);

// ---- GMRES(k) per unit (gmres.hip) ----
// Per batch column c: basis vectors V_i at base + i*stride_v + c*col (node-major
// FP64 columns of `col` values); Hessenberg H[c][i][j] at ((c*(K+1)+i)*K + j),
// g[c][i] at c*(K+1)+i, rotations and y at c*K + j, with K = kGmresMaxK.
constexpr int kGmresMaxK = 8;
struct GmresVecs {
  const double* base;
  size_t stride_v;
  size_t col;
};
// <V_i[c], W[c]> for i < nvec into out[c*ocs + i*ois]: mode 0 store, 1 add,
// 2 store the square root (a norm); out2 (optional) += the same values.
// `part` holds [nc][120][K+1] partial sums.
void gmres_dot(const GmresVecs& V, int nvec, const double* W, double* part, double* out,
               size_t ocs, size_t ois, int mode, double* out2, size_t ocs2, size_t ois2, int nc,
               hipStream_t st);
// W[c] -= sum_{i < nvec} coef[c*ccs + i*cis] V_i[c]
void gmres_axpy(const GmresVecs& V, int nvec, const double* coef, size_t ccs, size_t cis, double* W,
                int nc, hipStream_t st);
// X[c] /= s[c*s_stride] (times zero when s is zero)
void gmres_scale(double* X, size_t col, const double* s, size_t s_stride, int nc, hipStream_t st);
// g[c] = (beta[c*beta_stride], 0, ...)
void gmres_start(const double* beta, size_t beta_stride, double* g, int nc, hipStream_t st);
// Givens rotation j on every column's Hessenberg column j and g
void gmres_givens(double* H, double* g, double* cs, double* sn, int j, int nc, hipStream_t st);
// y = R^{-1} g and X^{n,m} = X^{n,m-1} + V y through the descriptors
void gmres_finish(int dim, int nn, const ColDesc* cols, const GmresVecs& Z, int k, const double* H,
                  const double* g, double* y, int nc, hipStream_t st);
constexpr int kGmresDotBlocks = 120;

__host__ __device__ inline int num_node_blocks(int nn) { return (nn + kBlock - 1) / kBlock; }

}  // namespace biot
