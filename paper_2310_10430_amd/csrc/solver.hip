// Runtime of the Biot parallel-in-time solver and its C ABI (include/biot_pint.h).
//
// Schedules (Sec. 3.2 and 3.3 of the paper):
//   JACOBI     one sweep updates all N_time steps at once from the previous
//              sweep's trajectory; batches of steps are columns of one launch.
//   WAVEFRONT  Alg. 2's Gauss-Seidel-in-time order run as the pipeline of
//              Alg. 4: `depth` iterations are in flight, slot s working on step
//              w - s at wall step w.  Each slot keeps a ping-pong pair of
//              columns, so no slot reads what another writes in the same wave.
// One unit (step n, iteration m) is
//   r   = c(n) F + A' X^{n-1} - AA X^{n,m-1}                  (k_residual)
//   z_u = V_A(r_u)                                            (multigrid V-cycle)
//   t   = B' z_u - r_p   (P1)   or   -r_p   (P2)              (k_pstage)
//   z_p = V_S(t)                                              (multigrid V-cycle)
//   X^{n,m} = X^{n,m-1} + omega [z_u; z_p]                    (k_update)
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <type_traits>
#include <vector>

#include "../../include/biot_pint.h"
#include "kernels.hpp"
#include "setup.hpp"

using namespace biot;

// Static device scratch of biot_apply_precond_noalloc (64 MiB per device; see
// scratch_address below).
constexpr size_t kScratchBytes = size_t(64) << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

thread_local std::string g_create_error;

template <typename T>
struct Field {  // work vectors of one V-cycle family per level
  std::vector<T*> b, x0, x1, d, r;
};

// Preconditioner state in precision T: multigrid levels (operator values of
// type T; neighbour lists and boundary flags shared with the FP64 levels), the
// fine-level B' for the P1 pressure stage, dense coarsest inverses and the work
// vectors of the two V-cycle families.
template <typename T>
struct Prec {
  std::vector<LevelView<T>> L;
  const T* Bt = nullptr;
  T* coarseA = nullptr;
  T* coarseS = nullptr;
  Field<T> fa, fs;
  T* rp = nullptr;
  // fused coarse end of the V-cycles (k_vcycle_tail), per copy: 1 when every
  // copy has one (-1: none has; the coarsest level is then its own launch)
  int tailA = -1, tailS = -1;
  TailDev<T> tdA{}, tdS{};
  std::vector<TailCopy> tcA, tcS;     // host copies of the per-copy descriptors
  size_t ldsA = 0, ldsS = 0;          // LDS bytes of a tail workgroup (largest copy)
  // tail launches: runs of consecutive copies with the same tail shape, each
  // launched with its own LDS size (first copy, copies, LDS bytes)
  struct TailGroup { int cp0, n; size_t lds; };
  std::vector<TailGroup> tgA, tgS;
  // per level: copies (a prefix) that run the level as their own launches
  std::vector<int> standA, standS;
};

struct ChebCoef {
  double theta = 0, delta = 0, sigma = 0;
};

// One space-time problem that the schedules iterate: the forward problem, the
// adjoint recursion in reversed time, or a group of checkpointed segments that
// is recomputed.  Columns 1..N of the trajectory pair T are the unknowns;
// column 0 is the initial value.  pin[n] (if set) replaces X^{n-1} as the
// coupling source of step n (a segment that starts from a checkpoint).
struct Sched {
  bool adj = false;
  int N = 0, cap = 0;                 // steps now / table capacity in steps
  double* T[2] = {nullptr, nullptr};
  int cur = 0;
  std::vector<int> gstep;             // [N+1] global step of each column (descriptors'
                                      // step and load-coefficient row)
  std::vector<const double*> pin;     // [N+1]
  ColDesc* desc_jac[2] = {nullptr, nullptr};
  ColDesc* desc_k4[2] = {nullptr, nullptr};
  ColDesc* desc_wave[2] = {nullptr, nullptr};
  ColDesc* desc_part = nullptr;       // table of a partial (shallower) pass
  std::vector<ColDesc> h_jac[2], h_k4[2], h_wave[2], h_part;
  std::vector<int> wave_off, wave_cnt, part_off, part_cnt;
  int part_key = -1;                  // (parity, depth) of the uploaded partial table
  // wavefront passes captured as HIP graphs, per trajectory parity, each pass
  // as a few graphs of consecutive waves; valid for the step count graph_N
  // (the tables' contents may change between replays)
  std::vector<hipGraph_t> graph[2];
  std::vector<hipGraphExec_t> gexec[2];
  std::vector<size_t> gfirst[2], gend[2];  // waves [first, end) of each graph, in wave order
  double gbytes[2] = {0.0, 0.0};      // algorithmic bytes of one replay of a pass
  int graph_N = -1;
  int graph_stride = 0;               // probe stride the graphs leave out (0: none)
};

}  // namespace

struct biot_handle {
  std::string err;
  HostProblem P;
  biot_options opt{};
  int dim = 2, D1 = 3, nn = 0, N = 0, nlev = 0;
  int ncmax = 0;  // batch capacity (columns)
  int S = 1;                     // samples (copies of the grid) in the handle
  std::vector<int> steps;        // steps of each sample (<= N; later ones are padding)
  size_t col = 0; // doubles per state column
  // device state
  bool bound = false;
  hipStream_t st = nullptr;
  char* ws = nullptr;
  uint64_t ws_need = 0;
  std::vector<LevelDev> L;       // FP64 levels (level 0 also feeds the residual)
  std::vector<std::vector<int>> ppre;  // per level: fused post-smoothing patches of
                                       // the first k copies, k = 0..copies
  std::vector<std::vector<int32_t>> ptab_h;  // per level: (copy, patch) pairs
  std::vector<int> copy_of;      // copy (node order) of each sample
  FineDev F{};
  double* tcoef = nullptr;       // [N+1][nterms] load-term multipliers (device)
  double* pres = nullptr;        // [npres][nn][dim+1] prescribed-value terms (device)
  double* pcoef = nullptr;       // [N+1][npres]
  double* x0 = nullptr;          // [nn][dim+1] initial state (device), if given
  Prec<double> pd;               // FP64 preconditioner (precision FP64)
  Prec<float> pf;                // FP32 preconditioner (precision MIXED)
  Sched fw;                      // forward problem (the trajectory of the ABI)
  Sched bw;                      // adjoint recursion, reversed time
  Sched rp;                      // replay of checkpointed segments
  bool fw_valid = true;          // false once a checkpointed adjoint overwrote fw.T
  bool adj_valid = false;        // bw.T holds the states of the last biot_adjoint
  double* slots = nullptr;
  double* partials = nullptr;
  int nblk = 0;
  double* norms = nullptr;
  std::vector<ChebCoef> chA, chS;
  // adjoint buffers (options.adjoint)
  int ckK = 0;                   // checkpointed segments ceil(N / ckpt_stride)
  int n_chunks = 0;              // chunks of the gradient partial sums
  double* ck = nullptr;          // [ckK+1] checkpoint columns
  double* gload = nullptr;       // [N][nn] adjoint pressure-row load
  int32_t* sens = nullptr;       // [max_sensors]
  double* pobs = nullptr;        // [N][max_sensors]
  double* jpart = nullptr;       // [N][max_sensors]
  double* jval = nullptr;        // [1]
  double* gpart = nullptr;       // [n_chunks][4][ne]
  double* gout = nullptr;        // [3][ne] staging for host gradients
  ElemDev E{};
  // GMRES(k) per unit (options.inner = GMRES), per batch column
  double* gV = nullptr;          // basis V_0..V_k        [k+1][ncmax][col]
  double* gT = nullptr;          // operator products     [ncmax][col]
  double* gru = nullptr;         // r0 in field layout    [ncmax][nn][dim]
  double* grp = nullptr;         //                       [ncmax][nn]
  double* kpart = nullptr;       // dot partials
  double* gH = nullptr;          // Hessenberg            [ncmax][K+1][K]
  double* gg = nullptr;          // rotated rhs           [ncmax][K+1]
  double* gcs = nullptr;         // rotations, y          [ncmax][K]
  double* gsn = nullptr;
  double* gy = nullptr;
  double* gbeta = nullptr;       // ||r0||                [ncmax]
  double* gcorr = nullptr;       // second Gram-Schmidt pass [ncmax][K+1]
  // HIP-event probes around level-0 launches (biot_profile_enable)
  struct Pending { hipEvent_t a, b; int id; double bytes; };
  struct Acc { uint64_t launches = 0; double ms = 0, bytes = 0; };
  bool prof = false;
  unsigned prof_mask = 0;  // which probes record events
  int prof_stride = 0;     // > 1: only every prof_stride-th wave of a pass is probed
  size_t tail_lds = kTailMaxLds;  // LDS a fused tail may use (device limit, at bind)
  std::vector<hipEvent_t> ev_pool;
  size_t ev_next = 0;
  std::vector<Pending> pending;
  Acc acc[BIOT_PROBE_COUNT];
  int cur_copies = 0;  // columns of the current batch that also write a second copy
  // algorithmic bytes (each launch's distinct global inputs and outputs, once)
  // of every kernel enqueued on the handle's stream, replayed graphs included
  double acct = 0.0;
  hipStream_t cap_stream = nullptr;  // stream used for graph capture
  // allocation-free preconditioner apply: the device the handle was bound on,
  // that device's address of the static scratch array, and host-side field
  // tables (sized at bind) that point into it during a call
  int dev = 0;
  char* scratch_dev = nullptr;
  Field<double> sfa_d, sfs_d;
  Field<float> sfa_f, sfs_f;
};

namespace {

// steps per chunk of the gradient partial sums when the whole forward
// trajectory is kept (with checkpoints a chunk is one segment)
constexpr int kGradChunk = 16;

int fail(biot_handle* h, int code, const std::string& msg) {
  if (h) h->err = msg;
  else g_create_error = msg;
  return code;
}

#define HIPCHK(h, call)                                                               \
  do {                                                                                \
    hipError_t e_ = (call);                                                           \
    if (e_ != hipSuccess)                                                             \
      return fail(h, BIOT_EHIP, std::string(#call) + ": " + hipGetErrorString(e_));   \
  } while (0)

#define LAUNCHCHK(h)                                                                  \
  do {                                                                                \
    hipError_t e_ = hipGetLastError();                                                \
    if (e_ != hipSuccess)                                                             \
      return fail(h, BIOT_EHIP, std::string("kernel launch: ") + hipGetErrorString(e_)); \
  } while (0)

// bump allocator over the workspace; with base == nullptr it only counts bytes
struct Bump {
  char* base;
  uint64_t off = 0;
  template <class T>
  T* take(size_t count) {
    off = (off + 255) & ~uint64_t(255);
    T* p = base ? reinterpret_cast<T*>(base + off) : nullptr;
    off += uint64_t(count) * sizeof(T);
    return p;
  }
};

// Device scratch of biot_apply_precond_noalloc: the V-cycle work vectors of
// that entry point live here instead of in the bound workspace.  Every device
// the library runs on holds one copy until the process ends; host code reaches
// a device's copy only through the address hipGetSymbolAddress returns for it
// (kept per device in g_scratch_addr), never through the array's name.
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
char* g_scratch_addr[kMaxDevices] = {};

// address of the current device's scratch array (looked up once per device)
int scratch_address(biot_handle* h, int dev, char** out) {
  if (dev < 0 || dev >= kMaxDevices) return fail(h, BIOT_EINVAL, "device ordinal out of range");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_addr[dev]) {
    void* p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fail(h, BIOT_EHIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_scratch_addr[dev] = static_cast<char*>(p);
  }
  *out = g_scratch_addr[dev];
  return BIOT_OK;
}

// Vector that holds a level's V-cycle result, whether the level runs as its
// own launches (not the level-0 pressure field, which writes the outer update)
// or in the fused tail: with the fused coarse-grid correction and
// post-smoothing (2D, degree 2) the level's residual buffer, free after the
// restriction; otherwise x0 or x1, as each smoothing step and the
// prolongation swap the iterates.
template <typename T>
T* result_vec(const biot_handle* h, const Field<T>& f, int l) {
  const int deg = h->opt.cheb_degree;
  if (h->opt.fuse_post && deg == 2 && h->dim == 2) return f.r[l];
  int cur = 0;
  for (int j = 2; j <= deg; ++j) cur ^= 1;  // pre-smoothing
  cur ^= 1;                                 // coarse-grid correction
  for (int j = 1; j <= deg; ++j) cur ^= 1;
  return cur ? f.x1[l] : f.x0[l];
}

// The coarsest levels of a copy whose V-cycle vectors fit in the LDS of one
// workgroup (kTailMaxLds, or less if the device allows less) run as one fused
// launch; level 0 never does (its steps are fused with the residual and the
// update).  A level joins only if it has at most two nodes per tail thread:
// the tail runs one workgroup per column, so a larger level is faster as its
// own launches, which spread over the whole chip.  Each copy (sample) gets its
// own first tail level; either every copy has a tail or none has.
template <typename T>
void plan_tail(biot_handle* h, Bump& b, Prec<T>& p, bool is_A) {
  const int C = is_A ? h->dim : 1;
  const int copies = h->P.levels[0].copies;
  int& t = is_A ? p.tailA : p.tailS;
  TailDev<T>& td = is_A ? p.tdA : p.tdS;
  std::vector<TailCopy>& tcs = is_A ? p.tcA : p.tcS;
  size_t& lds = is_A ? p.ldsA : p.ldsS;
  std::vector<int>& stand = is_A ? p.standA : p.standS;
  auto& groups = is_A ? p.tgA : p.tgS;
  groups.clear();
  const size_t budget = std::min(kTailMaxLds, h->tail_lds);
  tcs.assign(copies, TailCopy{});
  lds = 0;
  int with = 0;
  auto grid_nodes = [&](int cells) {
    const int m = cells + 1;
    return h->dim == 2 ? m * m : m * m * m;
  };
  for (int cp = 0; cp < copies; ++cp) {
    const int last = h->P.clast[cp];
    TailCopy& tc = tcs[cp];
    tc.t0 = -1;
    for (int l = 1; l < last; ++l) {
      const int n = last - l + 1;
      if (n > kTailMaxLevels) continue;
      if (grid_nodes(h->P.levels[l].ccells[cp]) > 2 * tail_block_threads(h->dim)) continue;
      int nnl[kTailMaxLevels];
      for (int i = 0; i < n; ++i) nnl[i] = grid_nodes(h->P.levels[l + i].ccells[cp]);
      const size_t bytes = tail_lds_bytes(nnl, n, C, int(sizeof(T)), h->opt.cheb_degree);
      if (bytes > budget) continue;
      tc.t0 = l;
      tc.nlev = n;
      int off = 0;
      for (int i = 0; i < n; ++i) {
        tc.off[i] = off;
        off += nnl[i] * C * (i + 1 < n ? tail_vectors(h->opt.cheb_degree) : 2);
      }
      tc.moff = is_A ? h->P.cAoff[cp] : h->P.cSoff[cp];
      lds = std::max(lds, bytes);
      ++with;
      // copies are ordered largest first: a new group where the shape changes
      if (groups.empty() || groups.back().lds != bytes ||
          tcs[groups.back().cp0].t0 != tc.t0 || groups.back().cp0 + groups.back().n != cp)
        groups.push_back({cp, 0, bytes});
      groups.back().n += 1;
      break;
    }
  }
  t = (with > 0 && with == copies) ? 1 : -1;
  // per level, the copies that run it as their own launches: with a tail, the
  // levels above it; without, the levels above the copy's last one (which is
  // then solved densely, when no copy runs that level as launches)
  stand.assign(h->nlev, 0);
  for (int l = 0; l < h->nlev; ++l)
    for (int cp = 0; cp < copies; ++cp) {
      const bool own = t > 0 ? l < tcs[cp].t0 : l < h->P.clast[cp];
      if (own) stand[l] = cp + 1;
    }
  td = TailDev<T>{};
  td.degree = h->opt.cheb_degree;
  td.cp0 = 0;
  td.copies = copies;
  for (int l = 0; l < h->nlev && l < kMaxLevels; ++l) {
    td.L[l] = p.L[l];
    const ChebCoef& cc = is_A ? h->chA[l] : h->chS[l];
    td.theta[l] = cc.theta;
    td.delta[l] = cc.delta;
    td.sigma[l] = cc.sigma;
  }
  td.Minv = is_A ? p.coarseA : p.coarseS;
  td.tc = b.take<TailCopy>(copies);
}

template <typename T>
void plan_prec(biot_handle* h, Bump& b, Prec<T>& p) {
  const int dim = h->dim;
  p.L.assign(h->nlev, LevelView<T>{});
  for (int l = 0; l < h->nlev; ++l) {
    const HostLevel& H = h->P.levels[l];
    LevelView<T>& D = p.L[l];
    D.nn = H.nn;
    D.W = H.W;
    D.n_cells = H.n_cells;
    D.copies = H.copies;
    D.nn1 = H.nn1;
    D.nreal = H.nreal;
    D.nact = H.nn;
    D.cbase = h->L[l].cbase;
    D.ccells = h->L[l].ccells;
    D.bcopy = h->L[l].bcopy;
    D.csteps = h->L[l].csteps;
    D.act = nullptr;
    D.ptab = h->L[l].ptab;
    D.npatch = h->L[l].npatch;
    D.nbr = h->L[l].nbr;
    D.fixed = h->L[l].fixed;
    if constexpr (std::is_same<T, double>::value) {
      D.A = h->L[l].A;
      D.S = h->L[l].S;
      D.Ainv = h->L[l].Ainv;
      D.Sinv = h->L[l].Sinv;
      D.AD = h->L[l].AD;
      D.SD = h->L[l].SD;
    } else {
      D.A = b.take<T>(H.A.size());
      D.S = b.take<T>(H.S.size());
      D.Ainv = b.take<T>(H.Ainv.size());
      D.Sinv = b.take<T>(H.Sinv.size());
      D.AD = b.take<T>(H.AD.size());
      D.SD = b.take<T>(H.SD.size());
    }
  }
  if constexpr (std::is_same<T, double>::value) p.Bt = h->F.Bt;
  else p.Bt = b.take<T>(h->P.levels[0].Bt.size());
  p.coarseA = b.take<T>(h->P.coarseAinv.size());
  p.coarseS = b.take<T>(h->P.coarseSinv.size());
  const int nc = h->ncmax;
  for (Field<T>* f : {&p.fa, &p.fs}) {
    const int C = (f == &p.fa) ? dim : 1;
    f->b.assign(h->nlev, nullptr);
    f->x0.assign(h->nlev, nullptr);
    f->x1.assign(h->nlev, nullptr);
    f->d.assign(h->nlev, nullptr);
    f->r.assign(h->nlev, nullptr);
    for (int l = 0; l < h->nlev; ++l) {
      const size_t n = size_t(nc) * h->P.levels[l].nn * C;
      f->b[l] = b.take<T>(n);
      f->x0[l] = b.take<T>(n);
      f->x1[l] = b.take<T>(n);
      f->d[l] = b.take<T>(n);
      f->r[l] = b.take<T>(n);
    }
  }
  p.rp = b.take<T>(size_t(nc) * h->nn);
  plan_tail(h, b, p, true);
  plan_tail(h, b, p, false);
}

// fused post-smoothing patches (2D): per level, (copy, patch) for every patch
// of every copy in copy order, and the patch count of the first k copies
void build_patches(biot_handle* h) {
  h->ppre.assign(h->nlev, {});
  h->ptab_h.assign(h->nlev, {});
  for (int l = 0; l < h->nlev; ++l) {
    const HostLevel& H = h->P.levels[l];
    std::vector<int>& pre = h->ppre[l];
    pre.assign(size_t(H.copies) + 1, 0);
    for (int c = 0; c < H.copies; ++c) {
      const int per_side = h->dim == 2 ? (H.ccells[c] + 1 + kPatchInterior - 1) / kPatchInterior : 0;
      for (int q = 0; q < per_side * per_side; ++q) {
        h->ptab_h[l].push_back(c);
        h->ptab_h[l].push_back(q);
      }
      pre[c + 1] = pre[c] + per_side * per_side;
    }
  }
}

void plan(biot_handle* h, char* base) {
  Bump b{base};
  h->L.assign(h->nlev, LevelDev{});
  for (int l = 0; l < h->nlev; ++l) {
    const HostLevel& H = h->P.levels[l];
    LevelDev& D = h->L[l];
    D.nn = H.nn;
    D.W = H.W;
    D.n_cells = H.n_cells;
    D.copies = H.copies;
    D.nn1 = H.nn1;
    D.nreal = H.nreal;
    D.nact = H.nn;
    D.cbase = b.take<int32_t>(H.cbase.size());
    D.ccells = b.take<int32_t>(H.ccells.size());
    D.bcopy = b.take<int32_t>(H.bcopy.size());
    D.csteps = l == 0 ? b.take<int32_t>(h->P.csteps.size()) : h->L[0].csteps;
    D.act = nullptr;
    D.ptab = b.take<int32_t>(h->ptab_h[l].size());
    D.npatch = int(h->ptab_h[l].size() / 2);
    D.nbr = b.take<int32_t>(H.nbr.size());
    D.A = b.take<double>(H.A.size());
    D.S = b.take<double>(H.S.size());
    D.Ainv = b.take<double>(H.Ainv.size());
    D.Sinv = b.take<double>(H.Sinv.size());
    D.fixed = b.take<uint8_t>(H.fixed.size());
    D.AD = b.take<double>(H.AD.size());
    D.SD = b.take<double>(H.SD.size());
  }
  const HostLevel& H0 = h->P.levels[0];
  h->F.B = b.take<double>(H0.B.size());
  h->F.Bt = b.take<double>(H0.Bt.size());
  h->F.Cb = b.take<double>(H0.Cb.size());
  h->F.F = b.take<double>(h->P.terms.size());
  h->F.nt = h->P.nterms;
  h->F.gload = nullptr;
  h->tcoef = b.take<double>(h->P.tcoef.size());
  h->pres = b.take<double>(h->P.pres.size());
  h->pcoef = b.take<double>(h->P.pcoef.size());
  h->x0 = h->P.x0.empty() ? nullptr : b.take<double>(h->P.x0.size());
  const bool wave = h->opt.schedule == BIOT_SCHED_WAVEFRONT;
  auto traj_pair = [&](Sched& S, int cap) {
    S.T[0] = b.take<double>(size_t(cap + 1) * h->col);
    S.T[1] = b.take<double>(size_t(cap + 1) * h->col);
  };
  auto tables = [&](Sched& S) {
    for (int c = 0; c < 2; ++c) {
      S.desc_jac[c] = b.take<ColDesc>(S.cap);
      S.desc_k4[c] = b.take<ColDesc>(S.cap);
      if (wave) S.desc_wave[c] = b.take<ColDesc>(size_t(S.cap) * h->opt.depth);
    }
    if (wave) S.desc_part = b.take<ColDesc>(size_t(S.cap) * h->opt.depth);
  };
  h->fw.cap = h->N;
  traj_pair(h->fw, h->N);
  tables(h->fw);
  if (h->opt.adjoint) {
    const int s = h->opt.ckpt_stride;
    h->bw.cap = h->N;
    if (s > 0) {
      // the adjoint reuses the forward trajectory pair; the forward states are
      // kept at the checkpoints and recomputed segment group by group
      h->bw.T[0] = h->fw.T[0];
      h->bw.T[1] = h->fw.T[1];
      h->ckK = (h->N + s - 1) / s;
      h->ck = b.take<double>(size_t(h->ckK + 1) * h->col);
      h->rp.cap = std::min(h->N, h->opt.replay_segments * s);
      traj_pair(h->rp, h->rp.cap);
      tables(h->rp);
      h->n_chunks = h->ckK;
    } else {
      traj_pair(h->bw, h->N);
      h->n_chunks = (h->N + kGradChunk - 1) / kGradChunk;
    }
    tables(h->bw);
    const size_t ne = size_t(h->P.ne), ms = size_t(h->opt.max_sensors);
    h->gload = b.take<double>(size_t(h->N) * h->nn);
    h->sens = b.take<int32_t>(ms);
    h->pobs = b.take<double>(size_t(h->N) * ms);
    h->jpart = b.take<double>(size_t(h->N) * ms);
    h->jval = b.take<double>(1);
    h->E.ne = h->P.ne;
    h->E.conn = b.take<int32_t>(h->P.conn_t.size());
    h->E.geo = b.take<double>(h->P.geo.size());
    h->E.coefK = b.take<double>(ne);
    h->E.dbl = b.take<double>(ne);
    h->E.dbm = b.take<double>(ne);
    h->gpart = b.take<double>(size_t(h->n_chunks) * 4 * ne);
    h->gout = b.take<double>(3 * ne);
  }
  if (wave) h->slots = b.take<double>(size_t(2) * h->opt.depth * h->col);
  if (h->opt.inner == BIOT_INNER_GMRES) {
    const size_t nc = size_t(h->ncmax), K = kGmresMaxK, k = size_t(h->opt.gmres_k);
    h->gV = b.take<double>((k + 1) * nc * h->col);
    h->gT = b.take<double>(nc * h->col);
    h->gru = b.take<double>(nc * h->nn * h->dim);
    h->grp = b.take<double>(nc * h->nn);
    h->kpart = b.take<double>(nc * kGmresDotBlocks * (K + 1));
    h->gH = b.take<double>(nc * (K + 1) * K);
    h->gg = b.take<double>(nc * (K + 1));
    h->gcs = b.take<double>(nc * K);
    h->gsn = b.take<double>(nc * K);
    h->gy = b.take<double>(nc * K);
    h->gbeta = b.take<double>(nc);
    h->gcorr = b.take<double>(nc * (K + 1));
  }
  if (h->opt.precision == BIOT_PRECISION_MIXED) plan_prec<float>(h, b, h->pf);
  else plan_prec<double>(h, b, h->pd);
  h->nblk = num_node_blocks(h->nn);
  h->partials = b.take<double>(size_t(std::max(h->ncmax, h->N)) * h->nblk * 4);
  h->norms = b.take<double>(size_t(h->N) * h->S * 4);
  h->ws_need = b.off + 256;
}

// multiplier of load term 0 at column n of a schedule (0 for the adjoint)
double term0(const biot_handle* h, const Sched& S, int n) {
  if (S.adj || h->P.nterms == 0) return 0.0;
  return h->P.tcoef[size_t(S.gstep[n]) * h->P.nterms];
}

// Wavefront table of a pass of depth d (<= the configured depth) reading
// trajectory T[c] and writing T[1-c]: at wave w, slot s updates step w - s
// from its iterate of sweep s to sweep s+1.  Slot s reads its input from slot
// s-1's output of the previous wave (slot 0: the trajectory) and its coupling
// from its own previous output (step 1, or a pinned step: the fixed source);
// outputs alternate between two buffers per slot; slot d-1 also writes the
// trajectory.
void wave_table(biot_handle* h, const Sched& S, int c, int d, std::vector<ColDesc>& tab,
                std::vector<int>& off, std::vector<int>& cnt) {
  const size_t col = h->col;
  const int D = h->opt.depth;
  double* Tin = S.T[c];
  double* Tout = S.T[1 - c];
  auto slot = [&](int s, int parity) { return h->slots + (size_t(parity) * D + s) * col; };
  tab.clear();
  off.clear();
  cnt.clear();
  for (int w = 1; w <= S.N + d - 1; ++w) {
    off.push_back(int(tab.size()));
    int k = 0;
    for (int s = 0; s < d; ++s) {
      const int n = w - s;
      if (n < 1 || n > S.N) continue;
      ColDesc e{};
      e.xcur = s == 0 ? Tin + n * col : slot(s - 1, (w - 1) & 1);
      e.xprev = S.pin[n] ? S.pin[n] : (n == 1 ? Tin : slot(s, (w - 1) & 1));
      e.xout = slot(s, w & 1);
      e.xout2 = s == d - 1 ? Tout + n * col : nullptr;
      e.tc = S.adj ? nullptr : h->tcoef + size_t(S.gstep[n]) * h->P.nterms;
      e.c0 = term0(h, S, n);
      e.step = S.gstep[n];
      tab.push_back(e);
      ++k;
    }
    cnt.push_back(k);
  }
}

// descriptor tables of both parities on the host (Jacobi, residual, wavefront)
void build_tables(biot_handle* h, Sched& S) {
  const size_t col = h->col;
  for (int c = 0; c < 2; ++c) {
    double* Tin = S.T[c];
    double* Tout = S.T[1 - c];
    S.h_jac[c].resize(S.N);
    S.h_k4[c].resize(S.N);
    for (int n = 1; n <= S.N; ++n) {
      ColDesc d{};
      d.xcur = Tin + n * col;
      d.xprev = S.pin[n] ? S.pin[n] : Tin + (n - 1) * col;
      d.xout = Tout + n * col;
      d.xout2 = nullptr;
      d.tc = S.adj ? nullptr : h->tcoef + size_t(S.gstep[n]) * h->P.nterms;
      d.c0 = term0(h, S, n);
      d.step = S.gstep[n];
      S.h_jac[c][n - 1] = d;
      d.xout = nullptr;
      S.h_k4[c][n - 1] = d;
    }
    if (h->opt.schedule == BIOT_SCHED_WAVEFRONT)
      wave_table(h, S, c, h->opt.depth, S.h_wave[c], S.wave_off, S.wave_cnt);
  }
  S.part_key = -1;
}

int upload_tables(biot_handle* h, Sched& S) {
  for (int c = 0; c < 2; ++c) {
    HIPCHK(h, hipMemcpyAsync(S.desc_jac[c], S.h_jac[c].data(), S.h_jac[c].size() * sizeof(ColDesc),
                             hipMemcpyHostToDevice, h->st));
    HIPCHK(h, hipMemcpyAsync(S.desc_k4[c], S.h_k4[c].data(), S.h_k4[c].size() * sizeof(ColDesc),
                             hipMemcpyHostToDevice, h->st));
    if (S.desc_wave[c])
      HIPCHK(h, hipMemcpyAsync(S.desc_wave[c], S.h_wave[c].data(),
                               S.h_wave[c].size() * sizeof(ColDesc), hipMemcpyHostToDevice, h->st));
  }
  return BIOT_OK;
}

// set the step count and per-column data of a schedule
void shape_sched(Sched& S, int N, bool adj) {
  S.adj = adj;
  S.N = N;
  S.gstep.resize(N + 1);
  for (int n = 0; n <= N; ++n) S.gstep[n] = n;
  S.pin.assign(N + 1, nullptr);
}

ChebCoef cheb_of(double lmax, double ratio) {
  ChebCoef c;
  const double lmin = lmax / ratio;
  c.theta = 0.5 * (lmax + lmin);
  c.delta = 0.5 * (lmax - lmin);
  c.sigma = c.theta / c.delta;
  return c;
}


const char* kProbeNames[BIOT_PROBE_COUNT] = {
    "k_residual (fused residual, coupling, norms; level 0)",
    "k_cheb displacement smoothing (level 0)",
    "k_cheb pressure smoothing (level 0)",
    "k_level_residual displacement (level 0)",
    "k_level_residual pressure (level 0)",
    "k_pstage (P1 pressure stage; level 0)",
    "k_post2 displacement post-smoothing, two steps (levels 0-2)",
    "k_post2 pressure post-smoothing, two steps (levels 1-2)"};

int harvest(biot_handle* h) {
  if (h->pending.empty()) {
    h->ev_next = 0;
    return BIOT_OK;
  }
  HIPCHK(h, hipEventSynchronize(h->pending.back().b));
  for (const auto& p : h->pending) {
    float ms = 0.f;
    HIPCHK(h, hipEventElapsedTime(&ms, p.a, p.b));
    h->acc[p.id].launches += 1;
    h->acc[p.id].ms += ms;
    h->acc[p.id].bytes += p.bytes;
  }
  h->pending.clear();
  h->ev_next = 0;
  return BIOT_OK;
}

// times the one node-blocked launch issued inside it when probing: the event
// pair is recorded by that launch's own dispatch (kernel begin and end), so the
// time excludes the event packets; `bytes` = the launch's algorithmic bytes
struct ProbeScope {
  biot_handle* h;
  int id;
  double bytes;
  hipEvent_t a = nullptr, b = nullptr;
  int rc = BIOT_OK;
  bool live = true;
  ProbeScope(biot_handle* h_, int id_, double bytes_) : h(h_), id(id_), bytes(bytes_) {
    if (!h->prof || id < 0 || bytes <= 0 || !((h->prof_mask >> id) & 1u)) {
      live = false;
      return;
    }
    if (h->ev_next + 2 > h->ev_pool.size()) {
      if (h->st == h->cap_stream) {
        rc = fail(h, BIOT_EHIP, "probe event pool exhausted during graph capture");
        return;
      }
      rc = harvest(h);
    }
    if (rc) return;
    a = h->ev_pool[h->ev_next++];
    b = h->ev_pool[h->ev_next++];
    set_launch_events(a, b);
  }
  ~ProbeScope() {
    // a scope left before its launch (an error path) must not hand its events
    // to an unrelated launch
    if (live && !rc && a && launch_events_armed()) set_launch_events(nullptr, nullptr);
  }
  int end() {
    if (!live || rc) return rc;
    if (launch_events_armed()) {
      set_launch_events(nullptr, nullptr);
      return fail(h, BIOT_EHIP, "probe scope without a node-blocked launch");
    }
    h->pending.push_back({a, b, id, bytes});
    return BIOT_OK;
  }
};

// Algorithmic bytes of each launch: its distinct global inputs and outputs,
// each counted once (operators once per launch, vectors once per column);
// `t` = bytes per value of the preconditioner precision.  The probes report
// these, and every launch adds them to h->acct.
double bytes_residual(const biot_handle* h, int nc, bool write_r, int t) {
  const double nn = h->nn, W = h->P.levels[0].W, d = h->dim, D1 = d + 1;
  double per_col = 8 * D1 * 2 + (write_r ? t * (d + 1) : 0);
  // operator blocks, neighbour indices, load terms, prescribed-dof flags
  double mat = W * (d * d + 2 * d + 2) * 8 + 4 * W + 8 * D1 * h->P.nterms + 1;
  return nc * nn * per_col + nn * mat;
}
// `first`: the step after the unstored first step reads only b (the gathered
// vector) and no separate iterate
// (k = copies in the launch: a level's launch covers its first k copies)
double act_nodes(const biot_handle* h, int l, int k) { return h->P.levels[l].cbase[k]; }
int grid_nodes_host(const biot_handle* h, int cells) {
  const int m = cells + 1;
  return h->dim == 2 ? m * m : m * m * m;
}
double bytes_cheb(const biot_handle* h, int l, int k, int C, int nc, bool c1, bool upd, bool wd,
                  bool first, int t) {
  const double nn = act_nodes(h, l, k), W = h->P.levels[l].W, d = h->dim, D1 = d + 1;
  double per_col =
      double(t) * C * ((first ? 1 : 2) + (c1 ? 1 : 0) + (upd ? 0 : 1 + (wd ? 1 : 0)));
  if (upd) per_col += 8 * D1 * 2 + t * d;
  double total = nc * nn * per_col + (upd ? h->cur_copies * nn * 8 * D1 : 0);
  total += nn * (W * C * C * t + 4 * W + C * C * t);
  return total;
}
double bytes_levres(const biot_handle* h, int l, int k, int C, int nc, int t) {
  const double nn = act_nodes(h, l, k), W = h->P.levels[l].W;
  return nc * nn * C * t * 3 + nn * (W * C * C * t + 4 * W);
}
// the coarse-grid correction and both post-smoothing steps: b, x, xc in, x4
// out; the operator row, D^{-1}, indices and the fine and coarse flags once
double bytes_post2(const biot_handle* h, int l, int k, int C, int nc, int t, bool upd) {
  const double nn = act_nodes(h, l, k), ncs = act_nodes(h, l + 1, k), W = h->P.levels[l].W;
  const double d = h->dim, D1 = d + 1;
  // with the outer update: no x4, but X^{m-1} and z_u in, X^m out (and the
  // trajectory copy of the last slot)
  const double per_col = upd ? nn * (C * t * 2 + 8 * D1 * 2 + t * d) : nn * C * t * 3;
  return nc * (per_col + ncs * C * t) + nn * (W * C * C * t + 4 * W + C * C * t) + (nn + ncs) +
         (upd ? h->cur_copies * nn * 8 * D1 : 0.0);
}
double bytes_pstage(const biot_handle* h, int nc, int t) {
  const double nn = h->nn, W = h->P.levels[0].W, d = h->dim;
  return nc * nn * t * (d + 2) + nn * (W * d * t + 4 * W);
}
// restriction l -> l+1: fine residual in, coarse right-hand side out, flags
double bytes_restrict(const biot_handle* h, int l, int k, int C, int nc, int t) {
  const double nf = act_nodes(h, l, k), ncs = act_nodes(h, l + 1, k);
  return nc * (nf + ncs) * C * t + (nf + ncs);
}
// prolongation l+1 -> l: fine iterate and coarse correction in, fine out, flags
double bytes_prolong(const biot_handle* h, int l, int k, int C, int nc, int t) {
  const double nf = act_nodes(h, l, k), ncs = act_nodes(h, l + 1, k);
  return nc * (2 * nf + ncs) * C * t + (nf + ncs);
}
// fused tail: per copy, its first tail level's b in and x out per column;
// the operators of its tail levels (A or S, the folded copy, D^{-1}, indices,
// flags) and its dense coarsest inverse once
double bytes_tail(const biot_handle* h, const std::vector<TailCopy>& tcs, int C, int nc, int t) {
  double total = 0;
  for (size_t cp = 0; cp < tcs.size(); ++cp) {
    const TailCopy& tc = tcs[cp];
    auto nodes = [&](int l) {
      const double m = h->P.levels[l].ccells[cp] + 1;
      return h->dim == 2 ? m * m : m * m * m;
    };
    for (int i = 0; i + 1 < tc.nlev; ++i) {
      const double W = h->P.levels[tc.t0 + i].W;
      total += nodes(tc.t0 + i) * (2 * W * C * C * t + 4 * W + C * C * t + 1);
    }
    const double n = nodes(tc.t0 + tc.nlev - 1) * C;
    total += n * n * t + nc * nodes(tc.t0) * C * t * 2;
  }
  return total;
}
double bytes_coarse(const biot_handle* h, int l, int C, int nc, int t) {
  const HostLevel& L = h->P.levels[l];
  const double n = double(L.nreal) * C;
  return L.copies * n * n * t + nc * L.copies * n * t * 2;
}
double bytes_update(const biot_handle* h, int nc, int t) {
  const double nn = h->nn, D1 = h->D1;
  return nc * nn * (8 * D1 * 2 + t * D1) + h->cur_copies * nn * 8 * D1;
}
double bytes_norms(const biot_handle* h, int nc) {
  return nc * (double(h->nblk) * 4 * 8 + double(h->S) * 4 * 8);
}
double bytes_apply_op(const biot_handle* h, int nc) {
  const double nn = h->nn, W = h->P.levels[0].W, d = h->dim, D1 = d + 1;
  return nc * nn * 8 * D1 * 2 + nn * (W * (d * d + 2 * d + 1) * 8 + 4 * W);
}
double bytes_pack(const biot_handle* h, int nc, int t) {
  return nc * double(h->nn) * h->D1 * (8 + t);
}

// A level's view for a launch over its first k copies, with the launch's
// column descriptors (batches: a sample skips the columns past its steps).
template <typename T>
LevelView<T> view_of(const biot_handle* h, const LevelView<T>& L, int l, int k,
                     const ColDesc* act) {
  LevelView<T> v = L;
  v.nact = h->P.levels[l].cbase[k];
  v.npatch = h->ppre.empty() ? 0 : h->ppre[l][k];
  v.act = act;
  return v;
}

// One V-cycle for field A (is_A) or S from level l down, for nc columns.  On
// entry b[l] holds the right-hand side; the first Chebyshev step from zero is
// pointwise and never stored (the second step forms it from b).  A level runs
// as its own launches for the copies (a prefix) whose coarse end lies below
// it; the first level where no copy does launches the fused tail of every copy
// (each from its own first tail level; the result goes to the result buffer
// of that level) or, without tails, the dense coarsest solve.  The result is
// returned in *out; when `upd` is given (pressure field, level 0) the last
// smoothing step writes the outer update through those descriptors instead
// and *out is null.  `act`: the column descriptors that let the samples of a
// batch skip the columns past their steps (null: every column is active).
template <typename T>
int vcycle(biot_handle* h, Prec<T>& p, bool is_A, int l, int nc, T** out, const ColDesc* upd,
           const T* zu, const ColDesc* act) {
  Field<T>& f = is_A ? p.fa : p.fs;
  const int C = is_A ? h->dim : 1;
  const int wpc = h->opt.wg_per_cu;
  const int tb = int(sizeof(T));
  hipStream_t st = h->st;
  const bool has_tail = (is_A ? p.tailA : p.tailS) > 0;
  const int k = (is_A ? p.standA : p.standS)[l];
  if (k == 0 && has_tail) {
    // the work vectors in use now (a caller-less apply may swap in others)
    TailDev<T> td = is_A ? p.tdA : p.tdS;
    for (int i = 0; i < h->nlev && i < kMaxLevels; ++i) {
      td.L[i].act = act;
      td.b[i] = f.b[i];
      td.x[i] = result_vec(h, f, i);
    }
    // one launch per run of copies with the same tail shape, each with the
    // LDS its copies need (small grids then keep more workgroups resident)
    for (const auto& g : is_A ? p.tgA : p.tgS) {
      td.cp0 = g.cp0;
      td.copies = g.n;
      launch_vcycle_tail<T>(h->dim, C, td, nc, g.lds, st);
      LAUNCHCHK(h);
    }
    h->acct += bytes_tail(h, is_A ? p.tcA : p.tcS, C, nc, tb);
    *out = result_vec(h, f, l);
    return BIOT_OK;
  }
  if (k == 0) {
    // no tails: every copy's coarsest level is this one (equal grids)
    const HostLevel& H = h->P.levels[l];
    launch_coarse_solve<T>(grid_nodes_host(h, H.ccells[0]) * C, (H.cbase[1] - H.cbase[0]) * C,
                           H.copies, is_A ? p.coarseA : p.coarseS, f.b[l], f.x0[l], nc, st);
    LAUNCHCHK(h);
    h->acct += bytes_coarse(h, l, C, nc, tb);
    if (upd) {
      launch_update<T>(h->dim, h->nn, upd, zu, f.x0[l], h->opt.omega, nc,
                       act ? h->L[0].csteps : nullptr, h->L[0].bcopy, st);
      LAUNCHCHK(h);
      h->acct += bytes_update(h, nc, tb);
      *out = nullptr;
    } else {
      *out = f.x0[l];
    }
    return BIOT_OK;
  }
  if (l + 1 >= h->nlev) return fail(h, BIOT_EINVAL, "internal: no coarser level below a smoothed one");
  const LevelView<T> Lv = view_of(h, p.L[l], l, k, act);
  const ChebCoef& cc = is_A ? h->chA[l] : h->chS[l];
  const int deg = h->opt.cheb_degree;
  T* cur = f.x0[l];
  T* oth = f.x1[l];
  // pre-smoothing: the first step was done by the producer of b[l]
  double rho = 1.0 / cc.sigma;
  const bool fine = l == 0;
  const int pid_cheb = is_A ? BIOT_PROBE_CHEB_U : BIOT_PROBE_CHEB_P;
  for (int j = 2; j <= deg; ++j) {
    const double rn = 1.0 / (2.0 * cc.sigma - rho);
    // d after the last pre-smoothing step is dead: the first post-smoothing
    // step does not read it.  The first step from zero (x = D^{-1} b / theta)
    // is never stored: step 2 forms it from b.
    const bool wd = j < deg;
    const bool first = j == 2;
    const double by = bytes_cheb(h, l, k, C, nc, j > 2, false, wd, first, tb);
    ProbeScope ps(h, fine ? pid_cheb : -1, fine ? by : 0);
    launch_cheb<T>(h->dim, C, Lv, is_A, f.b[l], first ? f.b[l] : cur, oth, f.d[l], nc,
                   rn * rho, 2.0 * rn / cc.delta, wd, first ? 1 : 0, first, 1.0 / cc.theta,
                   nullptr, nullptr, 0.0, wpc, fine, st);
    LAUNCHCHK(h);
    h->acct += by;
    if (fine && ps.end()) return BIOT_EHIP;
    rho = rn;
    std::swap(cur, oth);
  }
  {
    const double by = bytes_levres(h, l, k, C, nc, tb);
    ProbeScope ps(h, is_A ? BIOT_PROBE_LEVRES_U : BIOT_PROBE_LEVRES_P, fine ? by : 0);
    launch_level_residual<T>(h->dim, C, Lv, is_A, f.b[l], cur, f.r[l], nc, wpc, st);
    LAUNCHCHK(h);
    h->acct += by;
    if (fine && ps.end()) return BIOT_EHIP;
  }
  const LevelView<T> Lc = view_of(h, p.L[l + 1], l + 1, k, act);
  launch_restrict<T>(h->dim, C, Lv, Lc, is_A, f.r[l], f.b[l + 1], nc, st);
  LAUNCHCHK(h);
  h->acct += bytes_restrict(h, l, k, C, nc, tb);
  T* xc = nullptr;
  int rc = vcycle<T>(h, p, is_A, l + 1, nc, &xc, nullptr, nullptr, act);
  if (rc) return rc;
  // coarse-grid correction x += P xc, then deg post-smoothing steps
  rho = 1.0 / cc.sigma;
  if (h->opt.fuse_post && deg == 2 && h->dim == 2) {
    // the correction and both post-smoothing steps in one launch, into the
    // residual buffer (free after the restriction); on the pressure field's
    // level 0 the last step writes the outer update
    const double rn = 1.0 / (2.0 * cc.sigma - rho);
    // probed on every level, as a kernel trace averages this kernel
    const double by = bytes_post2(h, l, k, C, nc, tb, upd != nullptr);
    ProbeScope ps(h, is_A ? BIOT_PROBE_POST_U : BIOT_PROBE_POST_P, by);
    launch_post2<T>(C, Lv, Lc, is_A, f.b[l], cur, xc, f.r[l], nc, 1.0 / cc.theta, rn * rho,
                    2.0 * rn / cc.delta, upd, zu, h->opt.omega, wpc, st);
    LAUNCHCHK(h);
    h->acct += by;
    if (ps.end()) return BIOT_EHIP;
    *out = upd ? nullptr : f.r[l];
    return BIOT_OK;
  }
  launch_prolong<T>(h->dim, C, Lv, Lc, is_A, cur, xc, oth, nc, wpc, st);
  LAUNCHCHK(h);
  h->acct += bytes_prolong(h, l, k, C, nc, tb);
  std::swap(cur, oth);
  for (int j = 1; j <= deg; ++j) {
    double c1 = 0.0, c2 = 1.0 / cc.theta, rn = rho;
    if (j > 1) {
      rn = 1.0 / (2.0 * cc.sigma - rho);
      c1 = rn * rho;
      c2 = 2.0 * rn / cc.delta;
    }
    const bool final_upd = upd && j == deg;
    // d after the last step is dead, and the step after the first one (c1 = 0)
    // recovers it as its input minus the buffer it overwrites, which still
    // holds the first step's input
    const bool wd = j > 1 && j < deg;
    const int dx = j == 2 ? 2 : 0;
    const double by = bytes_cheb(h, l, k, C, nc, j > 1, final_upd, wd, false, tb);
    ProbeScope ps(h, fine ? pid_cheb : -1, fine ? by : 0);
    launch_cheb<T>(h->dim, C, Lv, is_A, f.b[l], cur, oth, f.d[l], nc, c1, c2, wd, dx, false,
                   0.0, final_upd ? upd : nullptr, zu, h->opt.omega, wpc, fine, st);
    LAUNCHCHK(h);
    h->acct += by;
    if (fine && ps.end()) return BIOT_EHIP;
    rho = rn;
    std::swap(cur, oth);
  }
  *out = upd ? nullptr : cur;
  return BIOT_OK;
}

// P^{-1} applied to the batch whose residual is in fa.b[0] (r_u) and rp (r_p).
// With `upd`, the outer update is written through those descriptors.
template <typename T>
int precond_batch(biot_handle* h, Prec<T>& p, int nc, T** zu, T** zp, const ColDesc* upd) {
  // a batch's samples skip the columns past their own steps
  const ColDesc* act = h->S > 1 ? upd : nullptr;
  int rc = vcycle<T>(h, p, true, 0, nc, zu, nullptr, nullptr, act);
  if (rc) return rc;
  {
    const double by = bytes_pstage(h, nc, int(sizeof(T)));
    ProbeScope ps(h, BIOT_PROBE_PSTAGE, by);
    launch_pstage<T>(h->dim, view_of(h, p.L[0], 0, h->P.levels[0].copies, act), p.Bt,
                     h->opt.precond == BIOT_PRECOND_P1, *zu, p.rp, p.fs.b[0], nc,
                     h->opt.wg_per_cu, h->st);
    LAUNCHCHK(h);
    h->acct += by;
    if (ps.end()) return BIOT_EHIP;
  }
  return vcycle<T>(h, p, false, 0, nc, zp, upd, *zu, act);
}

// one unit for every column of a descriptor batch: FP64 residual, P^{-1} in
// precision T, FP64 update
// level 0 for a residual launch over descriptor columns (the samples of a
// batch skip the columns past their own steps)
LevelDev fine_level(const biot_handle* h, const ColDesc* cols) {
  LevelDev L = h->L[0];
  if (h->S > 1) L.act = cols;
  return L;
}

// level-0 coupling data for a schedule (the adjoint adds its pressure load)
FineDev fine_of(const biot_handle* h, const Sched& S) {
  FineDev f = h->F;
  f.gload = S.adj ? h->gload : nullptr;
  if (S.adj) f.nt = 0;  // the adjoint's only load is gload
  return f;
}

template <typename T>
int unit_batch_t(biot_handle* h, const Sched& S, Prec<T>& p, const ColDesc* cols, int nc) {
  {
    const double by = bytes_residual(h, nc, true, int(sizeof(T)));
    ProbeScope ps(h, BIOT_PROBE_RESIDUAL, by);
    launch_residual<T>(h->dim, fine_level(h, cols), fine_of(h, S), cols, nc, p.fa.b[0], p.rp,
                       nullptr, h->nblk, h->opt.wg_per_cu, S.adj, h->st);
    LAUNCHCHK(h);
    h->acct += by;
    if (ps.end()) return BIOT_EHIP;
  }
  T *zu = nullptr, *zp = nullptr;
  return precond_batch<T>(h, p, nc, &zu, &zp, cols);
}


// Z = P^{-1} R for caller columns (diagnostic path)
template <typename T>
int apply_precond_t(biot_handle* h, Prec<T>& p, const double* R, double* Z, int ncols) {
  for (int c0 = 0; c0 < ncols; c0 += h->ncmax) {
    const int nc = std::min(h->ncmax, ncols - c0);
    launch_unpack<T>(h->dim, h->nn, R + size_t(c0) * h->col, p.fa.b[0], p.rp, nc, h->st);
    LAUNCHCHK(h);
    T *zu = nullptr, *zp = nullptr;
    int rc = precond_batch<T>(h, p, nc, &zu, &zp, nullptr);
    if (rc) return rc;
    launch_pack<T>(h->dim, h->nn, zu, zp, Z + size_t(c0) * h->col, nc, h->st);
    LAUNCHCHK(h);
    h->acct += 2 * bytes_pack(h, nc, int(sizeof(T)));
  }
  return BIOT_OK;
}

// Work-vector bytes of the preconditioner for nc columns, laid out as in
// plan_prec (every vector 256-byte aligned); with base != nullptr the fields
// fa, fs and rp are pointed into base.
template <typename T>
size_t precond_vectors(const biot_handle* h, int nc, char* base, Field<T>* fa, Field<T>* fs,
                       T** rp) {
  Bump b{base};
  for (int fi = 0; fi < 2; ++fi) {
    Field<T>* f = fi == 0 ? fa : fs;
    const int C = fi == 0 ? h->dim : 1;
    for (int l = 0; l < h->nlev; ++l) {
      const size_t n = size_t(nc) * h->P.levels[l].nn * C;
      T* pb = b.take<T>(n);
      T* p0 = b.take<T>(n);
      T* p1 = b.take<T>(n);
      T* pd = b.take<T>(n);
      T* pr = b.take<T>(n);
      if (base) {
        f->b[l] = pb;
        f->x0[l] = p0;
        f->x1[l] = p1;
        f->d[l] = pd;
        f->r[l] = pr;
      }
    }
  }
  T* q = b.take<T>(size_t(nc) * h->nn);
  if (base) *rp = q;
  return size_t((b.off + 255) & ~uint64_t(255));
}

// Z = P^{-1} R with the work vectors in the static scratch array: the same
// kernels as apply_precond_t, in batches of as many columns as the scratch
// holds.  The used part of the scratch is zeroed (fill kernel) before each
// batch, so a call does not depend on what an earlier call left there.
template <typename T>
int apply_precond_scratch_t(biot_handle* h, Prec<T>& p, Field<T>& sfa, Field<T>& sfs,
                            const double* R, double* Z, int ncols) {
  const size_t one = precond_vectors<T>(h, 1, nullptr, nullptr, nullptr, nullptr);
  if (one > kScratchBytes)
    return fail(h, BIOT_ENOMEM,
                "biot_apply_precond_noalloc: one column needs " + std::to_string(one) +
                    " bytes of work vectors; the static scratch holds " +
                    std::to_string(kScratchBytes));
  int nb = 1;
  while (nb < ncols && nb < 4096 &&
         precond_vectors<T>(h, nb + 1, nullptr, nullptr, nullptr, nullptr) <= kScratchBytes)
    ++nb;
  // swap the handle's work-vector tables for tables into the scratch (host
  // pointers only; nothing is allocated) and restore them on every path
  struct Swap {
    Prec<T>& p;
    Field<T>& a;
    Field<T>& s;
    T* rp;
    Swap(Prec<T>& p_, Field<T>& a_, Field<T>& s_) : p(p_), a(a_), s(s_), rp(p_.rp) {
      std::swap(p.fa, a);
      std::swap(p.fs, s);
    }
    ~Swap() {
      std::swap(p.fa, a);
      std::swap(p.fs, s);
      p.rp = rp;
    }
  } sw(p, sfa, sfs);
  for (int c0 = 0; c0 < ncols; c0 += nb) {
    const int nc = std::min(nb, ncols - c0);
    const size_t used = precond_vectors<T>(h, nc, h->scratch_dev, &p.fa, &p.fs, &p.rp);
    launch_zero(h->scratch_dev, used, h->st);
    LAUNCHCHK(h);
    launch_unpack<T>(h->dim, h->nn, R + size_t(c0) * h->col, p.fa.b[0], p.rp, nc, h->st);
    LAUNCHCHK(h);
    T *zu = nullptr, *zp = nullptr;
    int rc = precond_batch<T>(h, p, nc, &zu, &zp, nullptr);
    if (rc) return rc;
    launch_pack<T>(h->dim, h->nn, zu, zp, Z + size_t(c0) * h->col, nc, h->st);
    LAUNCHCHK(h);
  }
  return BIOT_OK;
}

// One unit as GMRES(k) on AA x = b (b = coupling + load of each column),
// left-preconditioned by P (PETSc's default side for GMRES, the Krylov solver
// K of Alg. 3) and started from X^{n,m-1}: v_0 = P^{-1}(b - AA x0)/beta; for
// j < k: w = P^{-1} AA v_j orthogonalized against v_0..v_j (classical
// Gram-Schmidt applied twice), v_{j+1} = w/||w||, Givens rotation of the
// Hessenberg column; then X^{n,m} = x0 + V y with y minimizing
// ||beta e_1 - H y||, i.e. the preconditioned residual ||P^{-1}(b - AA x)||,
// which weighs the displacement and pressure rows by the preconditioner.
template <typename T>
int gmres_batch_t(biot_handle* h, const Sched& S, Prec<T>& p, const ColDesc* cols, int nc) {
  const size_t K = kGmresMaxK, col = h->col, sv = size_t(h->ncmax) * col;
  const int k = h->opt.gmres_k;
  hipStream_t st = h->st;
  const GmresVecs Vv{h->gV, sv, col};
  launch_residual<double>(h->dim, fine_level(h, cols), fine_of(h, S), cols, nc, h->gru, h->grp,
                          nullptr, h->nblk, h->opt.wg_per_cu, S.adj, st);
  LAUNCHCHK(h);
  launch_pack<double>(h->dim, h->nn, h->gru, h->grp, h->gT, nc, st);
  LAUNCHCHK(h);
  h->acct += bytes_residual(h, nc, true, 8) + bytes_pack(h, nc, 8);
  int rc = apply_precond_t<T>(h, p, h->gT, h->gV, nc);
  if (rc) return rc;
  // Krylov vector traffic: a dot over v vectors reads v + 1 columns, an axpy
  // reads v + 1 and writes one, a scale reads and writes one
  const double cb = double(nc) * col * 8;
  gmres_dot(GmresVecs{h->gV, 0, col}, 1, h->gV, h->kpart, h->gbeta, 1, 0, 2, nullptr, 0, 0, nc, st);
  gmres_scale(h->gV, col, h->gbeta, 1, nc, st);
  gmres_start(h->gbeta, 1, h->gg, nc, st);
  LAUNCHCHK(h);
  h->acct += 3 * cb;  // the norm of v_0 (one column read) and its scale
  const size_t hcs = (K + 1) * K;
  for (int j = 0; j < k; ++j) {
    double* Vj = h->gV + j * sv;
    double* W = h->gV + (j + 1) * sv;
    launch_apply_operator(h->dim, h->L[0], h->F, Vj, h->gT, nc, st);
    LAUNCHCHK(h);
    h->acct += bytes_apply_op(h, nc);
    if ((rc = apply_precond_t<T>(h, p, h->gT, W, nc))) return rc;
    gmres_dot(Vv, j + 1, W, h->kpart, h->gH + j, hcs, K, 0, nullptr, 0, 0, nc, st);
    gmres_axpy(Vv, j + 1, h->gH + j, hcs, K, W, nc, st);
    gmres_dot(Vv, j + 1, W, h->kpart, h->gcorr, K + 1, 1, 0, h->gH + j, hcs, K, nc, st);
    gmres_axpy(Vv, j + 1, h->gcorr, K + 1, 1, W, nc, st);
    double* hn = h->gH + (j + 1) * K + j;
    gmres_dot(GmresVecs{W, 0, col}, 1, W, h->kpart, hn, hcs, 0, 2, nullptr, 0, 0, nc, st);
    gmres_scale(W, col, hn, hcs, nc, st);
    gmres_givens(h->gH, h->gg, h->gcs, h->gsn, j, nc, st);
    LAUNCHCHK(h);
    // two dot/axpy pairs over j + 1 vectors, the norm and the scale
    h->acct += 2 * ((j + 2) * cb + (j + 3) * cb) + 3 * cb;
  }
  gmres_finish(h->dim, h->nn, cols, Vv, k, h->gH, h->gg, h->gy, nc, st);
  LAUNCHCHK(h);
  h->acct += (k + 3) * cb + h->cur_copies * double(col) * 8;  // V, X in, X out
  return BIOT_OK;
}

int unit_batch(biot_handle* h, const Sched& S, const ColDesc* cols, int nc) {
  const bool mixed = h->opt.precision == BIOT_PRECISION_MIXED;
  if (h->opt.inner == BIOT_INNER_GMRES)
    return mixed ? gmres_batch_t<float>(h, S, h->pf, cols, nc)
                 : gmres_batch_t<double>(h, S, h->pd, cols, nc);
  return mixed ? unit_batch_t<float>(h, S, h->pf, cols, nc) : unit_batch_t<double>(h, S, h->pd, cols, nc);
}

int jacobi_sweep(biot_handle* h, Sched& S) {
  ColDesc* tab = S.desc_jac[S.cur];
  for (int n0 = 0; n0 < S.N; n0 += h->ncmax) {
    const int nc = std::min(h->ncmax, S.N - n0);
    int rc = unit_batch(h, S, tab + n0, nc);
    if (rc) return rc;
  }
  S.cur = 1 - S.cur;
  return BIOT_OK;
}

int run_waves(biot_handle* h, const Sched& S, const ColDesc* tab, const std::vector<int>& off,
              const std::vector<int>& cnt, int d, size_t w0 = 0, size_t w1 = size_t(-1)) {
  w1 = std::min(w1, off.size());
  for (size_t w = w0; w < w1; ++w) {
    const int wave = int(w) + 1, last_step = wave - d + 1;
    h->cur_copies = (last_step >= 1 && last_step <= S.N) ? 1 : 0;
    int rc = unit_batch(h, S, tab + off[w], cnt[w]);
    if (rc) return rc;
  }
  h->cur_copies = 0;
  return BIOT_OK;
}

int wavefront_pass_eager(biot_handle* h, Sched& S) {
  return run_waves(h, S, S.desc_wave[S.cur], S.wave_off, S.wave_cnt, h->opt.depth);
}

// a pass shallower than the configured depth (eager; table built on demand)
int wavefront_partial(biot_handle* h, Sched& S, int d) {
  const int key = S.cur * 65536 + d;
  if (S.part_key != key) {
    wave_table(h, S, S.cur, d, S.h_part, S.part_off, S.part_cnt);
    HIPCHK(h, hipMemcpyAsync(S.desc_part, S.h_part.data(), S.h_part.size() * sizeof(ColDesc),
                             hipMemcpyHostToDevice, h->st));
    HIPCHK(h, hipStreamSynchronize(h->st));
    S.part_key = key;
  }
  int rc = run_waves(h, S, S.desc_part, S.part_off, S.part_cnt, d);
  if (rc) return rc;
  S.cur = 1 - S.cur;
  return BIOT_OK;
}

void destroy_graphs(Sched& S) {
  for (int c = 0; c < 2; ++c) {
    for (auto e : S.gexec[c]) (void)hipGraphExecDestroy(e);
    for (auto g : S.graph[c]) (void)hipGraphDestroy(g);
    S.gexec[c].clear();
    S.graph[c].clear();
    S.gfirst[c].clear();
    S.gend[c].clear();
    S.gbytes[c] = 0.0;
  }
  S.graph_N = -1;
  S.graph_stride = 0;
}

// kernel nodes per captured graph: a pass of several hundred waves, each of up
// to a few hundred launches (GMRES units), is split into graphs of consecutive
// waves of about this size
constexpr size_t kGraphNodeBudget = 8192;

// captures waves [w0, w1) of the pass of parity c into one graph
int capture_waves(biot_handle* h, Sched& S, int c, size_t w0, size_t w1, size_t* nodes) {
  hipStream_t user = h->st;
  h->st = h->cap_stream;
  HIPCHK(h, hipStreamBeginCapture(h->st, hipStreamCaptureModeThreadLocal));
  // capture enqueues nothing: the bytes are counted per replay instead
  const double acct0 = h->acct;
  int rc = run_waves(h, S, S.desc_wave[c], S.wave_off, S.wave_cnt, h->opt.depth, w0, w1);
  S.gbytes[c] += h->acct - acct0;
  h->acct = acct0;
  hipGraph_t g = nullptr;
  hipError_t e = hipStreamEndCapture(h->st, &g);
  h->st = user;
  if (rc) {
    if (g) (void)hipGraphDestroy(g);
    return rc;
  }
  if (e != hipSuccess) return fail(h, BIOT_EHIP, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
  S.graph[c].push_back(g);
  S.gfirst[c].push_back(w0);
  S.gend[c].push_back(w1);
  if (nodes) HIPCHK(h, hipGraphGetNodes(g, nullptr, nodes));
  hipGraphExec_t x = nullptr;
  HIPCHK(h, hipGraphInstantiate(&x, g, nullptr, nullptr, 0));
  S.gexec[c].push_back(x);
  return BIOT_OK;
}

// One pass = N + depth - 1 waves.  With use_graph the launch sequence of a
// pass is captured once per trajectory parity (the descriptor tables, whose
// device buffers are fixed, hold every pointer) and replayed: the first wave
// alone, which measures the launches per wave, then chunks of waves of about
// kGraphNodeBudget launches.  Probes read HIP events recorded by a launch's
// own dispatch, which a replayed graph cannot carry: with probes on, a pass
// runs eagerly, or with a probe stride k > 1 only its waves w = k/2 (mod k)
// run eagerly (and are probed) and the waves between them are replayed.
bool probed_wave(int stride, size_t w) { return stride > 1 && int(w % size_t(stride)) == stride / 2; }

int wavefront_pass(biot_handle* h, Sched& S) {
  const int stride = h->prof ? h->prof_stride : 0;
  if (!h->opt.use_graph || (h->prof && stride < 2)) {
    int rc = wavefront_pass_eager(h, S);
    if (rc) return rc;
    S.cur = 1 - S.cur;
    return BIOT_OK;
  }
  if (S.graph_N != S.N || S.graph_stride != stride) destroy_graphs(S);
  const int c = S.cur;
  const size_t waves = S.wave_off.size();
  if (S.gexec[c].empty()) {
    // captured without probes; each run of unprobed waves becomes graphs of
    // at most `chunk` waves
    const bool prof = h->prof;
    h->prof = false;
    size_t per_wave = 0, chunk = 1;
    int rc = BIOT_OK;
    size_t w = 0;
    while (!rc && w < waves) {
      if (probed_wave(stride, w)) {
        ++w;
        continue;
      }
      size_t w1 = w + 1;
      if (per_wave > 0)
        while (w1 < waves && w1 - w < chunk && !probed_wave(stride, w1)) ++w1;
      rc = capture_waves(h, S, c, w, w1, per_wave == 0 ? &per_wave : nullptr);
      if (!rc && chunk == 1) chunk = std::max<size_t>(1, kGraphNodeBudget / std::max<size_t>(per_wave, 1));
      w = w1;
    }
    h->prof = prof;
    if (rc) {
      destroy_graphs(S);
      return rc;
    }
    S.graph_N = S.N;
    S.graph_stride = stride;
  }
  // replay, with the probed waves (those no graph covers) run eagerly
  size_t w = 0;
  for (size_t i = 0; i < S.gexec[c].size(); ++i) {
    for (; w < S.gfirst[c][i]; ++w) {
      int rc = run_waves(h, S, S.desc_wave[c], S.wave_off, S.wave_cnt, h->opt.depth, w, w + 1);
      if (rc) return rc;
    }
    HIPCHK(h, hipGraphLaunch(S.gexec[c][i], h->st));
    w = S.gend[c][i];
  }
  for (; w < waves; ++w) {
    int rc = run_waves(h, S, S.desc_wave[c], S.wave_off, S.wave_cnt, h->opt.depth, w, w + 1);
    if (rc) return rc;
  }
  h->acct += S.gbytes[c];
  S.cur = 1 - S.cur;
  return BIOT_OK;
}

// global space-time residual norms of the current trajectory into h->norms
int global_residual(biot_handle* h, const Sched& S) {
  ColDesc* tab = S.desc_k4[S.cur];
  const int chunk = std::max(h->ncmax, 1);
  const FineDev f = fine_of(h, S);
  for (int n0 = 0; n0 < S.N; n0 += chunk) {
    const int nc = std::min(chunk, S.N - n0);
    launch_residual<double>(h->dim, fine_level(h, tab + n0), f, tab + n0, nc, nullptr, nullptr,
                            h->partials, h->nblk, h->opt.wg_per_cu, S.adj, h->st);
    LAUNCHCHK(h);
    launch_reduce_norms(h->partials, h->L[0].cbase, h->S, h->nblk,
                        h->norms + size_t(n0) * h->S * 4, nc, h->st);
    LAUNCHCHK(h);
    h->acct += bytes_residual(h, nc, false, 8) + double(nc) * h->nblk * 4 * 8 * 2;
  }
  return BIOT_OK;
}

int sweep_sched(biot_handle* h, Sched& S, int n_sweeps) {
  int rc = BIOT_OK;
  if (h->opt.schedule == BIOT_SCHED_WAVEFRONT) {
    for (int p = 0; p < n_sweeps / h->opt.depth; ++p)
      if ((rc = wavefront_pass(h, S))) return rc;
    if (n_sweeps % h->opt.depth)
      if ((rc = wavefront_partial(h, S, n_sweeps % h->opt.depth))) return rc;
  } else {
    for (int s = 0; s < n_sweeps; ++s)
      if ((rc = jacobi_sweep(h, S))) return rc;
  }
  return BIOT_OK;
}

// Relative residual per field: max_n ||r^n|| / max_n ||b^n|| of each sample over
// its own steps (nr is [N][S][4]); the worst sample is returned.  A field
// whose right-hand side vanishes at every step (the pressure rows of a single
// step from rest, the displacement rows of a one-step adjoint) is measured
// against the whole right-hand side.
void rel_resid(const std::vector<double>& nr, int N, int S, const std::vector<int>& steps,
               double& ru, double& rp, std::vector<double>* per_u = nullptr,
               std::vector<double>* per_p = nullptr) {
  ru = rp = 0.0;
  for (int sm = 0; sm < S; ++sm) {
    const int Ns = S == 1 ? N : std::min(N, steps[sm]);
    double mu = 0, mp = 0, bu = 0, bp = 0;
    for (int n = 0; n < Ns; ++n) {
      const double* q = &nr[(size_t(n) * S + sm) * 4];
      for (int k = 0; k < 4; ++k)
        if (!std::isfinite(q[k])) {
          ru = rp = NAN;
          return;
        }
      mu = std::max(mu, q[0]);
      mp = std::max(mp, q[1]);
      bu = std::max(bu, q[2]);
      bp = std::max(bp, q[3]);
    }
    const double both = std::sqrt(bu + bp);
    const double du = bu > 0 ? std::sqrt(bu) : both, dp = bp > 0 ? std::sqrt(bp) : both;
    const double cu = std::sqrt(mu) / std::max(du, 1e-300), cpv = std::sqrt(mp) / std::max(dp, 1e-300);
    if (per_u) (*per_u)[sm] = cu;
    if (per_p) (*per_p)[sm] = cpv;
    ru = std::max(ru, cu);
    rp = std::max(rp, cpv);
  }
}

int check_bound(biot_handle* h) {
  if (!h) return BIOT_EINVAL;
  if (!h->bound) return fail(h, BIOT_ESTATE, "workspace not bound");
  return BIOT_OK;
}

int check_forward(biot_handle* h) {
  int rc = check_bound(h);
  if (rc) return rc;
  if (!h->fw_valid)
    return fail(h, BIOT_ESTATE,
                "the forward trajectory was overwritten by a checkpointed biot_adjoint; call biot_reset");
  return BIOT_OK;
}

struct SolveOut {
  int sweeps = 0;
  bool conv = false;
  double ru = 0, rp = 0;
};

// Sweeps schedule S until the worst relative residual is <= rtol (see
// biot_solve_to_tol for the policy).
// Sets the steps a copy takes part in on the device (0: none; the copy is
// frozen).  Graph replays read the table when they run.
int upload_csteps(biot_handle* h, const std::vector<int32_t>& cs) {
  HIPCHK(h, hipMemcpyAsync(const_cast<int32_t*>(h->L[0].csteps), cs.data(), cs.size() * 4,
                           hipMemcpyHostToDevice, h->st));
  HIPCHK(h, hipStreamSynchronize(h->st));  // the host vector must outlive the copy
  return BIOT_OK;
}

int solve_sched(biot_handle* h, Sched& S, double rtol, int max_sweeps, int check_every,
                SolveOut& out) {
  int rc = BIOT_OK;
  int step = check_every;
  if (h->opt.schedule == BIOT_SCHED_WAVEFRONT) step = h->opt.depth;  // first pass: full depth
  std::vector<double> nr(size_t(S.N) * h->S * 4);
  int done = 0;
  double first = -1;
  out = SolveOut{};
  // A sample of a batch that has reached the tolerance is frozen: its copy's
  // state is made the same in both trajectory buffers and its step count on
  // the device set to zero, so that every kernel skips it from then on; its
  // residual stays what it was.  (Richardson units only: a GMRES unit's
  // update would read the skipped residual.)
  const int ncp = h->S;
  const bool can_freeze = &S == &h->fw && ncp > 1 && h->opt.inner == BIOT_INNER_RICHARDSON;
  std::vector<double> cu(ncp, 0.0), cpv(ncp, 0.0), fu(ncp, 0.0), fp(ncp, 0.0);
  std::vector<char> frozen(ncp, 0);
  std::vector<int32_t> cs(h->P.csteps.begin(), h->P.csteps.end());
  int nfrozen = 0;
  while (true) {
    if ((rc = global_residual(h, S))) break;
    HIPCHK(h, hipMemcpyAsync(nr.data(), h->norms, nr.size() * 8, hipMemcpyDeviceToHost, h->st));
    HIPCHK(h, hipStreamSynchronize(h->st));
    rel_resid(nr, S.N, h->S, h->P.csteps, out.ru, out.rp, &cu, &cpv);
    if (nfrozen > 0) {
      // frozen copies were skipped by this check: their last values hold
      out.ru = out.rp = 0.0;
      bool finite = true;
      for (int c = 0; c < ncp; ++c) {
        if (frozen[c]) {
          cu[c] = fu[c];
          cpv[c] = fp[c];
        }
        finite = finite && std::isfinite(cu[c]) && std::isfinite(cpv[c]);
        out.ru = std::max(out.ru, cu[c]);
        out.rp = std::max(out.rp, cpv[c]);
      }
      if (!finite) out.ru = out.rp = NAN;
    }
    if (!std::isfinite(out.ru) || !std::isfinite(out.rp)) {
      rc = fail(h, BIOT_EDIVERGED, "non-finite residual");
      break;
    }
    const double worst = std::max(out.ru, out.rp);
    if (first < 0) first = worst;
    if (worst <= rtol) {
      out.conv = true;
      break;
    }
    if (done > 0 && worst > 1e6 * std::max(first, 1e-300)) {
      rc = fail(h, BIOT_EDIVERGED, "residual grew by more than 1e6");
      break;
    }
    if (done >= max_sweeps) {
      rc = fail(h, BIOT_ENOTCONVERGED, "max_sweeps reached above tolerance");
      break;
    }
    if (can_freeze) {
      bool any = false;
      for (int c = 0; c < ncp; ++c) {
        if (frozen[c] || std::max(cu[c], cpv[c]) > rtol) continue;
        const HostLevel& L0 = h->P.levels[0];
        const size_t off = size_t(L0.cbase[c]) * h->D1;
        const size_t width = size_t(L0.cbase[c + 1] - L0.cbase[c]) * h->D1 * 8;
        double* src = S.T[S.cur] + off;
        double* dst = S.T[1 - S.cur] + off;
        if (hipMemcpy2DAsync(dst, h->col * 8, src, h->col * 8, width, size_t(S.N) + 1,
                             hipMemcpyDeviceToDevice, h->st) != hipSuccess) {
          rc = fail(h, BIOT_EHIP, "hipMemcpy2DAsync (freezing a converged sample)");
          break;
        }
        frozen[c] = 1;
        fu[c] = cu[c];
        fp[c] = cpv[c];
        cs[c] = 0;
        ++nfrozen;
        any = true;
      }
      if (rc) break;
      if (any && (rc = upload_csteps(h, cs))) break;
    }
    int kk = std::min(step, max_sweeps - done);
    if (h->opt.schedule == BIOT_SCHED_WAVEFRONT && done > 0) {
      // size the next pass from the observed contraction per sweep, with margin
      const double rate = std::pow(worst / std::max(first, 1e-300), 1.0 / done);
      if (rate > 0 && rate < 0.999) {
        const double need = std::log(rtol / worst) / std::log(rate);
        const int k = int(std::ceil(1.15 * need)) + 2;
        kk = std::min({std::max(4, (k + 3) / 4 * 4), h->opt.depth, max_sweeps - done});
      }
    }
    if ((rc = sweep_sched(h, S, kk))) break;
    done += kk;
  }
  out.sweeps = done;
  if (nfrozen > 0) {
    // every sample takes part in later calls again (both buffers agree for
    // the frozen ones)
    const int r2 = upload_csteps(h, std::vector<int32_t>(h->P.csteps.begin(), h->P.csteps.end()));
    if (!rc) rc = r2;
  }
  return rc;
}

// Initial iterate X^{n,0} in both buffers of a trajectory pair: zero, or for
// the forward problem (`forward`) with prescribed values or X^0, the prescribed
// values g^n at the prescribed dofs of every step and X^0 in column 0.  Sweeps
// never change prescribed dofs (their residual and update are zero).
int zero_traj(biot_handle* h, Sched& S, bool forward = false) {
  if (forward && (h->P.npres > 0 || h->x0)) {
    for (int c = 0; c < 2; ++c) {
      launch_init_traj(S.T[c], S.N + 1, h->nn, h->D1, h->x0, h->pres, h->pcoef, h->P.npres,
                       h->L[0].fixed, h->st);
      LAUNCHCHK(h);
    }
  } else {
    const size_t bytes = size_t(S.N + 1) * h->col * 8;
    HIPCHK(h, hipMemsetAsync(S.T[0], 0, bytes, h->st));
    HIPCHK(h, hipMemsetAsync(S.T[1], 0, bytes, h->st));
  }
  S.cur = 0;
  return BIOT_OK;
}

// device data of the gradient contraction (element geometry and coefficients)
int upload_adjoint_data(biot_handle* h, std::vector<std::vector<double>>& keep) {
  const HostProblem& P = h->P;
  const size_t ne = size_t(P.ne);
  std::vector<double> cK(ne), dbl(ne), dbm(ne);
  for (size_t e = 0; e < ne; ++e) {
    cK[e] = P.dt * P.perm_e[e];
    const double den = P.lambda_e[e] + 2.0 * P.mu_e[e];
    dbl[e] = P.beta_given ? 0.0 : -P.beta_e[e] / den;
    dbm[e] = P.beta_given ? 0.0 : -2.0 * P.beta_e[e] / den;
  }
  keep.push_back(std::move(cK));
  keep.push_back(std::move(dbl));
  keep.push_back(std::move(dbm));
  const size_t n3 = keep.size();
  HIPCHK(h, hipMemcpyAsync(const_cast<int32_t*>(h->E.conn), P.conn_t.data(), P.conn_t.size() * 4,
                           hipMemcpyHostToDevice, h->st));
  HIPCHK(h, hipMemcpyAsync(const_cast<double*>(h->E.geo), P.geo.data(), P.geo.size() * 8,
                           hipMemcpyHostToDevice, h->st));
  HIPCHK(h, hipMemcpyAsync(const_cast<double*>(h->E.coefK), keep[n3 - 3].data(), ne * 8,
                           hipMemcpyHostToDevice, h->st));
  HIPCHK(h, hipMemcpyAsync(const_cast<double*>(h->E.dbl), keep[n3 - 2].data(), ne * 8,
                           hipMemcpyHostToDevice, h->st));
  HIPCHK(h, hipMemcpyAsync(const_cast<double*>(h->E.dbm), keep[n3 - 1].data(), ne * 8,
                           hipMemcpyHostToDevice, h->st));
  return BIOT_OK;
}

// validates the objective and evaluates J and the adjoint load from fw.T
int objective_load(biot_handle* h, const biot_objective* obj, double* J) {
  if (!h->opt.adjoint) return fail(h, BIOT_ESTATE, "handle created without options.adjoint");
  if (!obj || !obj->nodes || !obj->p_obs) return fail(h, BIOT_EINVAL, "NULL objective arrays");
  const int S = obj->n_sensors;
  if (S < 1 || S > h->opt.max_sensors)
    return fail(h, BIOT_EINVAL, "n_sensors must be in 1..max_sensors");
  std::vector<char> seen(h->nn, 0);
  for (int i = 0; i < S; ++i) {
    const int v = obj->nodes[i];
    if (v < 0 || v >= h->nn) return fail(h, BIOT_EINVAL, "sensor node out of range");
    if (seen[v]) return fail(h, BIOT_EINVAL, "sensor nodes must be distinct");
    seen[v] = 1;
  }
  const size_t NS = size_t(h->N) * S;
  for (size_t i = 0; i < NS; ++i)
    if (!std::isfinite(obj->p_obs[i])) return fail(h, BIOT_EINVAL, "non-finite p_obs");
  HIPCHK(h, hipMemcpyAsync(h->sens, obj->nodes, size_t(S) * 4, hipMemcpyHostToDevice, h->st));
  HIPCHK(h, hipMemcpyAsync(h->pobs, obj->p_obs, NS * 8, hipMemcpyHostToDevice, h->st));
  HIPCHK(h, hipMemsetAsync(h->gload, 0, size_t(h->N) * h->nn * 8, h->st));
  launch_sensor_load(h->dim, h->nn, h->N, S, h->fw.T[h->fw.cur], h->sens, h->pobs, h->L[0].fixed,
                     h->gload, h->jpart, h->st);
  LAUNCHCHK(h);
  launch_sum(h->jpart, int(NS), h->jval, h->st);
  LAUNCHCHK(h);
  HIPCHK(h, hipMemcpyAsync(J, h->jval, 8, hipMemcpyDeviceToHost, h->st));
  HIPCHK(h, hipStreamSynchronize(h->st));  // host sources must outlive the copies
  return BIOT_OK;
}

}  // namespace

extern "C" {

int biot_default_options(biot_options* o) {
  if (!o) return BIOT_EINVAL;
  o->schedule = BIOT_SCHED_JACOBI;
  o->depth = 8;
  o->precond = BIOT_PRECOND_P1;
  o->cheb_degree = 2;
  o->cheb_ratio = 4.0;
  o->lmax_safety = 1.1;
  o->power_iters = 20;
  o->max_batch = 0;
  o->omega = 0.6;
  o->wg_per_cu = 0;
  o->coarse_cells = 2;
  o->use_graph = 1;
  o->precision = BIOT_PRECISION_FP64;
  o->adjoint = 0;
  o->ckpt_stride = 16;
  o->replay_segments = 4;
  o->max_sensors = 256;
  o->inner = BIOT_INNER_RICHARDSON;
  o->gmres_k = 4;
  o->fuse_post = 1;
  return BIOT_OK;
}

int biot_create(const biot_mesh* mesh, const biot_materials* mat, const biot_load* load,
                double dt, int32_t n_steps, const biot_options* opt, biot_handle** out) {
  return biot_create_batch(mesh, 1, mat, load, &dt, &n_steps, opt, out);
}

int biot_create_batch(const biot_mesh* meshes, int32_t n_samples, const biot_materials* mats,
                      const biot_load* loads, const double* dts, const int32_t* n_steps,
                      const biot_options* opt, biot_handle** out) {
  const biot_mesh* mesh = meshes;
  if (!out) return fail(nullptr, BIOT_EINVAL, "out is NULL");
  *out = nullptr;
  if (!mesh || !mats || !loads || !dts || !n_steps)
    return fail(nullptr, BIOT_EINVAL, "NULL mesh, materials, load, dt or n_steps");
  if (n_samples < 1 || n_samples > 4096) return fail(nullptr, BIOT_EINVAL, "n_samples must be in 1..4096");
  biot_options o;
  biot_default_options(&o);
  if (opt) o = *opt;
  if (o.schedule != BIOT_SCHED_JACOBI && o.schedule != BIOT_SCHED_WAVEFRONT)
    return fail(nullptr, BIOT_EINVAL, "unknown schedule");
  if (o.precond != BIOT_PRECOND_P1 && o.precond != BIOT_PRECOND_P2)
    return fail(nullptr, BIOT_EINVAL, "unknown preconditioner");
  if (o.schedule == BIOT_SCHED_WAVEFRONT && (o.depth < 1 || o.depth > 4096))
    return fail(nullptr, BIOT_EINVAL, "depth must be in 1..4096");
  if (!(o.omega > 0.0) || !std::isfinite(o.omega)) return fail(nullptr, BIOT_EINVAL, "omega must be > 0");
  if (o.power_iters < 1) return fail(nullptr, BIOT_EINVAL, "power_iters must be >= 1");
  if (!(o.lmax_safety >= 1.0)) return fail(nullptr, BIOT_EINVAL, "lmax_safety must be >= 1");
  if (o.cheb_degree < 2 || o.cheb_degree > 8) return fail(nullptr, BIOT_EINVAL, "cheb_degree must be in 2..8");
  if (o.wg_per_cu < 0 || o.wg_per_cu > 32) return fail(nullptr, BIOT_EINVAL, "wg_per_cu must be in 0..32");
  if (o.coarse_cells < 1 || o.coarse_cells > 64) return fail(nullptr, BIOT_EINVAL, "coarse_cells must be in 1..64");
  if (o.precision != BIOT_PRECISION_FP64 && o.precision != BIOT_PRECISION_MIXED)
    return fail(nullptr, BIOT_EINVAL, "unknown precision");
  if (o.adjoint != 0 && o.adjoint != 1) return fail(nullptr, BIOT_EINVAL, "adjoint must be 0 or 1");
  if (o.adjoint && (o.ckpt_stride < 0 || o.replay_segments < 1 || o.max_sensors < 1))
    return fail(nullptr, BIOT_EINVAL, "need ckpt_stride >= 0, replay_segments >= 1, max_sensors >= 1");
  if (o.adjoint && n_samples > 1) return fail(nullptr, BIOT_EINVAL, "the adjoint takes one sample per handle");
  if (o.inner != BIOT_INNER_RICHARDSON && o.inner != BIOT_INNER_GMRES)
    return fail(nullptr, BIOT_EINVAL, "unknown inner solver");
  if (o.inner == BIOT_INNER_GMRES && (o.gmres_k < 1 || o.gmres_k > kGmresMaxK))
    return fail(nullptr, BIOT_EINVAL, "gmres_k must be in 1..8");
  if (o.fuse_post != 0 && o.fuse_post != 1) return fail(nullptr, BIOT_EINVAL, "fuse_post must be 0 or 1");
  biot_handle* h = new (std::nothrow) biot_handle();
  if (!h) return fail(nullptr, BIOT_ENOMEM, "out of host memory");
  h->opt = o;
  MeshIn m{mesh->dim, mesh->n_nodes, mesh->n_elems, mesh->grid_n, mesh->xyz, mesh->conn, mesh->dirichlet};
  HostOptions ho;
  ho.cheb_degree = o.cheb_degree;
  ho.cheb_ratio = o.cheb_ratio;
  ho.lmax_safety = o.lmax_safety;
  ho.power_iters = o.power_iters;
  ho.min_cells = o.coarse_cells;
  std::string e;
  int nmax = 0;
  try {
    if (n_samples == 1) {
      MaterialsIn mi{mats->young,  mats->poisson, mats->perm,        mats->beta,
                     mats->alpha,  mats->stab_h,  mats->lame_lambda, mats->lame_mu};
      LoadIn li{loads->n_facets,  loads->facet_nodes, loads->traction,
                loads->coef,      loads->n_terms,     loads->terms,
                loads->term_coef, loads->n_prescribed, loads->prescribed,
                loads->prescribed_coef, loads->x0};
      e = build_problem(m, mi, li, dts[0], n_steps[0], ho, h->P);
      nmax = n_steps[0];
    } else {
      std::vector<HostProblem> parts(n_samples);
      for (int sm = 0; sm < n_samples && e.empty(); ++sm) {
        const biot_materials& mt = mats[sm];
        const biot_load& ld = loads[sm];
        MaterialsIn mi{mt.young, mt.poisson, mt.perm, mt.beta, mt.alpha, mt.stab_h,
                       mt.lame_lambda, mt.lame_mu};
        LoadIn li{ld.n_facets, ld.facet_nodes, ld.traction, ld.coef, ld.n_terms, ld.terms,
                  ld.term_coef, ld.n_prescribed, ld.prescribed, ld.prescribed_coef, ld.x0};
        const biot_mesh& ms = meshes[sm];
        MeshIn mm{ms.dim, ms.n_nodes, ms.n_elems, ms.grid_n, ms.xyz, ms.conn, ms.dirichlet};
        e = build_problem(mm, mi, li, dts[sm], n_steps[sm], ho, parts[sm]);
        if (!e.empty()) e = "sample " + std::to_string(sm) + ": " + e;
        nmax = std::max(nmax, n_steps[sm]);
      }
      if (e.empty()) e = concat_problems(parts, kBlock, h->P);
    }
    if (e.empty()) fold_first_step(h->P);
  } catch (const std::exception& ex) {
    e = std::string("set-up failed: ") + ex.what();
  }
  if (!e.empty()) {
    delete h;
    return fail(nullptr, BIOT_EINVAL, e);
  }
  h->S = n_samples;
  h->steps.assign(n_steps, n_steps + n_samples);
  h->copy_of.assign(n_samples, 0);
  for (int c = 0; c < n_samples; ++c) h->copy_of[h->P.sample_of[c]] = c;
  h->dim = h->P.dim;
  h->D1 = h->dim + 1;
  h->nn = h->P.nn;
  h->N = nmax;
  h->nlev = int(h->P.levels.size());
  if (h->nlev > 16) {
    delete h;
    return fail(nullptr, BIOT_EINVAL, "too many multigrid levels");
  }
  h->col = size_t(h->nn) * h->D1;
  h->ncmax = o.schedule == BIOT_SCHED_WAVEFRONT
                 ? std::max(o.depth, 1)
                 : (o.max_batch > 0 ? std::min<int>(o.max_batch, nmax) : nmax);
  h->chA.resize(h->nlev);
  h->chS.resize(h->nlev);
  for (int l = 0; l + 1 < h->nlev; ++l) {
    h->chA[l] = cheb_of(h->P.levels[l].lmaxA, o.cheb_ratio);
    h->chS[l] = cheb_of(h->P.levels[l].lmaxS, o.cheb_ratio);
  }
  if (o.adjoint) {
    // the checkpoint replays start inner steps from interpolated checkpoints,
    // which is exact at prescribed dofs only when their values are zero
    bool nz = h->P.npres > 0;
    for (int v = 0; v < h->nn && !nz; ++v)
      for (int c = 0; c < h->D1; ++c)
        if (((h->P.levels[0].fixed[v] >> c) & 1) && !h->P.x0.empty() &&
            h->P.x0[size_t(v) * h->D1 + c] != 0.0)
          nz = true;
    if (nz) {
      delete h;
      return fail(nullptr, BIOT_EINVAL, "the adjoint needs zero prescribed values (no prescribed "
                                        "terms, X^0 zero at prescribed dofs)");
    }
  }
  shape_sched(h->fw, nmax, false);
  shape_sched(h->bw, nmax, true);  // load is gload, no traction
  build_patches(h);
  plan(h, nullptr);
  {
    // copies of different grids need every copy's coarse end in a fused tail
    bool uneven = false;
    for (const HostLevel& Hl : h->P.levels)
      for (int c = 1; c < Hl.copies; ++c) uneven = uneven || Hl.ccells[c] != Hl.ccells[0];
    const bool mixed = o.precision == BIOT_PRECISION_MIXED;
    const int ta = mixed ? h->pf.tailA : h->pd.tailA, ts = mixed ? h->pf.tailS : h->pd.tailS;
    if (uneven && (ta < 0 || ts < 0)) {
      delete h;
      return fail(nullptr, BIOT_EINVAL, "a batch of different grids needs the coarse end of "
                                        "every sample in the fused tail (use smaller grids)");
    }
  }
  *out = h;
  return BIOT_OK;
}

int biot_sample_layout(const biot_handle* h, int32_t sample, int32_t* first_node,
                       int32_t* n_nodes) {
  if (!h || !first_node || !n_nodes || sample < 0 || sample >= h->S) return BIOT_EINVAL;
  const HostLevel& L0 = h->P.levels[0];
  const int cp = h->copy_of[sample];
  *first_node = L0.cbase[cp];
  *n_nodes = grid_nodes_host(h, L0.ccells[cp]);
  return BIOT_OK;
}

int biot_workspace_size(const biot_handle* h, uint64_t* bytes) {
  if (!h || !bytes) return BIOT_EINVAL;
  *bytes = h->ws_need;
  return BIOT_OK;
}

int biot_bind(biot_handle* h, void* device_ptr, uint64_t bytes, void* stream) {
  if (!h) return BIOT_EINVAL;
  if (!device_ptr) return fail(h, BIOT_EINVAL, "device_ptr is NULL");
  if (reinterpret_cast<uintptr_t>(device_ptr) % 256 != 0)
    return fail(h, BIOT_EINVAL, "workspace must be 256-byte aligned");
  if (bytes < h->ws_need) return fail(h, BIOT_ENOMEM, "workspace smaller than biot_workspace_size");
  for (Sched* S : {&h->fw, &h->bw, &h->rp}) destroy_graphs(*S);
  {
    int dev = 0, lds = 0;
    HIPCHK(h, hipGetDevice(&dev));
    HIPCHK(h, hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
    h->tail_lds = std::min(kTailMaxLds, size_t(lds));
    h->dev = dev;
    int rc = scratch_address(h, dev, &h->scratch_dev);
    if (rc) return rc;
    for (auto* f : {&h->sfa_d, &h->sfs_d}) {
      f->b.assign(h->nlev, nullptr); f->x0.assign(h->nlev, nullptr); f->x1.assign(h->nlev, nullptr);
      f->d.assign(h->nlev, nullptr); f->r.assign(h->nlev, nullptr);
    }
    for (auto* f : {&h->sfa_f, &h->sfs_f}) {
      f->b.assign(h->nlev, nullptr); f->x0.assign(h->nlev, nullptr); f->x1.assign(h->nlev, nullptr);
      f->d.assign(h->nlev, nullptr); f->r.assign(h->nlev, nullptr);
    }
  }
  h->ws = static_cast<char*>(device_ptr);
  h->st = static_cast<hipStream_t>(stream);
  plan(h, h->ws);
  build_tables(h, h->fw);
  if (h->opt.adjoint) build_tables(h, h->bw);
  hipStream_t st = h->st;
  for (int l = 0; l < h->nlev; ++l) {
    const HostLevel& H = h->P.levels[l];
    const LevelDev& D = h->L[l];
    HIPCHK(h, hipMemcpyAsync(const_cast<int32_t*>(D.nbr), H.nbr.data(), H.nbr.size() * 4, hipMemcpyHostToDevice, st));
    HIPCHK(h, hipMemcpyAsync(const_cast<double*>(D.A), H.A.data(), H.A.size() * 8, hipMemcpyHostToDevice, st));
    HIPCHK(h, hipMemcpyAsync(const_cast<double*>(D.S), H.S.data(), H.S.size() * 8, hipMemcpyHostToDevice, st));
    HIPCHK(h, hipMemcpyAsync(const_cast<double*>(D.Ainv), H.Ainv.data(), H.Ainv.size() * 8, hipMemcpyHostToDevice, st));
    HIPCHK(h, hipMemcpyAsync(const_cast<double*>(D.Sinv), H.Sinv.data(), H.Sinv.size() * 8, hipMemcpyHostToDevice, st));
    HIPCHK(h, hipMemcpyAsync(const_cast<uint8_t*>(D.fixed), H.fixed.data(), H.fixed.size(), hipMemcpyHostToDevice, st));
    HIPCHK(h, hipMemcpyAsync(const_cast<double*>(D.AD), H.AD.data(), H.AD.size() * 8, hipMemcpyHostToDevice, st));
    HIPCHK(h, hipMemcpyAsync(const_cast<double*>(D.SD), H.SD.data(), H.SD.size() * 8, hipMemcpyHostToDevice, st));
    HIPCHK(h, hipMemcpyAsync(const_cast<int32_t*>(D.cbase), H.cbase.data(), H.cbase.size() * 4, hipMemcpyHostToDevice, st));
    HIPCHK(h, hipMemcpyAsync(const_cast<int32_t*>(D.ccells), H.ccells.data(), H.ccells.size() * 4, hipMemcpyHostToDevice, st));
    HIPCHK(h, hipMemcpyAsync(const_cast<int32_t*>(D.bcopy), H.bcopy.data(), H.bcopy.size() * 4, hipMemcpyHostToDevice, st));
    if (!h->ptab_h[l].empty())
      HIPCHK(h, hipMemcpyAsync(const_cast<int32_t*>(D.ptab), h->ptab_h[l].data(), h->ptab_h[l].size() * 4,
                               hipMemcpyHostToDevice, st));
  }
  HIPCHK(h, hipMemcpyAsync(const_cast<int32_t*>(h->L[0].csteps), h->P.csteps.data(), h->P.csteps.size() * 4,
                           hipMemcpyHostToDevice, st));
  auto up_tails = [&](auto& pr) -> hipError_t {
    hipError_t e = hipMemcpyAsync(const_cast<TailCopy*>(pr.tdA.tc), pr.tcA.data(),
                                  pr.tcA.size() * sizeof(TailCopy), hipMemcpyHostToDevice, st);
    if (e != hipSuccess) return e;
    return hipMemcpyAsync(const_cast<TailCopy*>(pr.tdS.tc), pr.tcS.data(),
                          pr.tcS.size() * sizeof(TailCopy), hipMemcpyHostToDevice, st);
  };
  if (h->opt.precision == BIOT_PRECISION_MIXED) HIPCHK(h, up_tails(h->pf));
  else HIPCHK(h, up_tails(h->pd));
  const HostLevel& H0 = h->P.levels[0];
  HIPCHK(h, hipMemcpyAsync(const_cast<double*>(h->F.B), H0.B.data(), H0.B.size() * 8, hipMemcpyHostToDevice, st));
  HIPCHK(h, hipMemcpyAsync(const_cast<double*>(h->F.Bt), H0.Bt.data(), H0.Bt.size() * 8, hipMemcpyHostToDevice, st));
  HIPCHK(h, hipMemcpyAsync(const_cast<double*>(h->F.Cb), H0.Cb.data(), H0.Cb.size() * 8, hipMemcpyHostToDevice, st));
  auto up64 = [&](const double* dst, const std::vector<double>& src) -> hipError_t {
    if (src.empty()) return hipSuccess;
    return hipMemcpyAsync(const_cast<double*>(dst), src.data(), src.size() * 8,
                          hipMemcpyHostToDevice, st);
  };
  HIPCHK(h, up64(h->F.F, h->P.terms));
  HIPCHK(h, up64(h->tcoef, h->P.tcoef));
  HIPCHK(h, up64(h->pres, h->P.pres));
  HIPCHK(h, up64(h->pcoef, h->P.pcoef));
  if (h->x0) HIPCHK(h, up64(h->x0, h->P.x0));
  std::vector<std::vector<float>> staging;  // FP32 copies must outlive the async copies
  auto up32 = [&](const float* dst, const std::vector<double>& src) -> hipError_t {
    staging.emplace_back(src.begin(), src.end());
    return hipMemcpyAsync(const_cast<float*>(dst), staging.back().data(), src.size() * 4,
                          hipMemcpyHostToDevice, st);
  };
  if (h->opt.precision == BIOT_PRECISION_MIXED) {
    for (int l = 0; l < h->nlev; ++l) {
      const HostLevel& H = h->P.levels[l];
      const LevelView<float>& D = h->pf.L[l];
      HIPCHK(h, up32(D.A, H.A));
      HIPCHK(h, up32(D.S, H.S));
      HIPCHK(h, up32(D.Ainv, H.Ainv));
      HIPCHK(h, up32(D.Sinv, H.Sinv));
      HIPCHK(h, up32(D.AD, H.AD));
      HIPCHK(h, up32(D.SD, H.SD));
    }
    HIPCHK(h, up32(h->pf.Bt, h->P.levels[0].Bt));
    HIPCHK(h, up32(h->pf.coarseA, h->P.coarseAinv));
    HIPCHK(h, up32(h->pf.coarseS, h->P.coarseSinv));
  } else {
    HIPCHK(h, hipMemcpyAsync(h->pd.coarseA, h->P.coarseAinv.data(), h->P.coarseAinv.size() * 8, hipMemcpyHostToDevice, st));
    HIPCHK(h, hipMemcpyAsync(h->pd.coarseS, h->P.coarseSinv.data(), h->P.coarseSinv.size() * 8, hipMemcpyHostToDevice, st));
  }
  int rc = upload_tables(h, h->fw);
  if (!rc && h->opt.adjoint) rc = upload_tables(h, h->bw);
  std::vector<std::vector<double>> keep;
  if (!rc && h->opt.adjoint) rc = upload_adjoint_data(h, keep);
  if (rc) return rc;
  if ((rc = zero_traj(h, h->fw, true))) return rc;
  if (h->opt.adjoint && h->opt.ckpt_stride == 0 && (rc = zero_traj(h, h->bw))) return rc;
  if (h->slots) HIPCHK(h, hipMemsetAsync(h->slots, 0, size_t(2) * h->opt.depth * h->col * 8, st));
  HIPCHK(h, hipStreamSynchronize(st));  // host sources must outlive the copies
  if (h->opt.schedule == BIOT_SCHED_WAVEFRONT && h->opt.use_graph && !h->cap_stream)
    HIPCHK(h, hipStreamCreateWithFlags(&h->cap_stream, hipStreamNonBlocking));
  h->fw_valid = true;
  h->adj_valid = false;
  h->bound = true;
  return BIOT_OK;
}

int biot_reset(biot_handle* h) {
  int rc = check_bound(h);
  if (rc) return rc;
  if ((rc = zero_traj(h, h->fw, true))) return rc;
  h->fw_valid = true;
  if (h->opt.ckpt_stride > 0) h->adj_valid = false;  // shared buffers
  return BIOT_OK;
}

int biot_sweep(biot_handle* h, int32_t n_sweeps) {
  int rc = check_forward(h);
  if (rc) return rc;
  if (n_sweeps < 0) return fail(h, BIOT_EINVAL, "n_sweeps < 0");
  if (h->opt.ckpt_stride > 0) h->adj_valid = false;
  return sweep_sched(h, h->fw, n_sweeps);
}

int biot_residual_norms(biot_handle* h, double* norms) {
  int rc = check_forward(h);
  if (rc) return rc;
  if (!norms) return fail(h, BIOT_EINVAL, "norms is NULL");
  if ((rc = global_residual(h, h->fw))) return rc;
  std::vector<double> byc(size_t(h->N) * h->S * 4);  // per copy (largest grids first)
  HIPCHK(h, hipMemcpyAsync(byc.data(), h->norms, byc.size() * 8, hipMemcpyDeviceToHost, h->st));
  HIPCHK(h, hipStreamSynchronize(h->st));
  for (int n = 0; n < h->N; ++n)
    for (int sm = 0; sm < h->S; ++sm)
      for (int q = 0; q < 4; ++q)
        norms[(size_t(n) * h->S + sm) * 4 + q] = byc[(size_t(n) * h->S + h->copy_of[sm]) * 4 + q];
  return BIOT_OK;
}

int biot_solve_to_tol(biot_handle* h, double rtol, int32_t max_sweeps, int32_t check_every,
                      biot_stats* stats) {
  int rc = check_forward(h);
  if (rc) return rc;
  if (!(rtol > 0) || max_sweeps < 0 || check_every < 1)
    return fail(h, BIOT_EINVAL, "need rtol > 0, max_sweeps >= 0, check_every >= 1");
  if (h->opt.ckpt_stride > 0) h->adj_valid = false;
  auto t0 = std::chrono::steady_clock::now();
  const double acct0 = h->acct;
  SolveOut so;
  rc = solve_sched(h, h->fw, rtol, max_sweeps, check_every, so);
  if (stats) {
    stats->alg_bytes = h->acct - acct0;
    stats->sweeps = so.sweeps;
    stats->converged = so.conv ? 1 : 0;
    stats->rel_resid_u = so.ru;
    stats->rel_resid_p = so.rp;
    stats->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  }
  return rc;
}

int biot_get_trajectory(biot_handle* h, int32_t n0, int32_t n1, double* dst, int32_t dst_on_device) {
  int rc = check_forward(h);
  if (rc) return rc;
  if (!dst || n0 < 0 || n1 > h->N + 1 || n0 > n1) return fail(h, BIOT_EINVAL, "bad range or NULL dst");
  const size_t bytes = size_t(n1 - n0) * h->col * 8;
  HIPCHK(h, hipMemcpyAsync(dst, h->fw.T[h->fw.cur] + size_t(n0) * h->col, bytes,
                           dst_on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, h->st));
  if (!dst_on_device) HIPCHK(h, hipStreamSynchronize(h->st));
  return BIOT_OK;
}

int biot_get_sample_trajectory(biot_handle* h, int32_t sample, int32_t n0, int32_t n1, double* dst,
                               int32_t dst_on_device) {
  int rc = check_forward(h);
  if (rc) return rc;
  if (sample < 0 || sample >= h->S) return fail(h, BIOT_EINVAL, "sample out of range");
  if (!dst || n0 < 0 || n1 > h->steps[sample] + 1 || n0 > n1)
    return fail(h, BIOT_EINVAL, "bad range or NULL dst");
  if (n1 == n0) return BIOT_OK;
  const HostLevel& L0 = h->P.levels[0];
  const int cp = h->copy_of[sample];
  const size_t width = size_t(grid_nodes_host(h, L0.ccells[cp])) * h->D1 * 8;
  const double* src = h->fw.T[h->fw.cur] + size_t(n0) * h->col + size_t(L0.cbase[cp]) * h->D1;
  HIPCHK(h, hipMemcpy2DAsync(dst, width, src, h->col * 8, width, size_t(n1 - n0),
                             dst_on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, h->st));
  if (!dst_on_device) HIPCHK(h, hipStreamSynchronize(h->st));
  return BIOT_OK;
}

int biot_set_trajectory(biot_handle* h, int32_t n0, int32_t n1, const double* src, int32_t src_on_device) {
  int rc = check_bound(h);
  if (rc) return rc;
  if (!src || n0 < 0 || n1 > h->N + 1 || n0 > n1) return fail(h, BIOT_EINVAL, "bad range or NULL src");
  if (!h->fw_valid && !(n0 == 0 && n1 == h->N + 1))
    return fail(h, BIOT_ESTATE, "forward trajectory overwritten: set all steps or call biot_reset");
  const size_t bytes = size_t(n1 - n0) * h->col * 8;
  for (int c = 0; c < 2; ++c)  // both buffers: X^0 must be the same in either
    HIPCHK(h, hipMemcpyAsync(h->fw.T[c] + size_t(n0) * h->col, src, bytes,
                             src_on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, h->st));
  if (!src_on_device) HIPCHK(h, hipStreamSynchronize(h->st));
  h->fw_valid = true;
  if (h->opt.ckpt_stride > 0) h->adj_valid = false;
  return BIOT_OK;
}

int biot_objective_value(biot_handle* h, const biot_objective* obj, double* J) {
  int rc = check_forward(h);
  if (rc) return rc;
  if (!J) return fail(h, BIOT_EINVAL, "J is NULL");
  return objective_load(h, obj, J);
}

int biot_adjoint(biot_handle* h, const biot_objective* obj, double rtol, int32_t max_sweeps,
                 double* grad_logk, double* grad_lambda, double* grad_mu, int32_t grads_on_device,
                 biot_adjoint_stats* stats) {
  int rc = check_forward(h);
  if (rc) return rc;
  if (!(rtol > 0) || max_sweeps < 0) return fail(h, BIOT_EINVAL, "need rtol > 0, max_sweeps >= 0");
  const auto t0 = std::chrono::steady_clock::now();
  biot_adjoint_stats out{};
  // J and dJ/dX from the forward trajectory
  if ((rc = objective_load(h, obj, &out.J))) return rc;
  const size_t col = h->col;
  const int N = h->N, s = h->opt.ckpt_stride;
  const bool ckpt = s > 0;
  const double* X = h->fw.T[h->fw.cur];
  if (ckpt) {
    for (int k = 0; k < h->ckK; ++k)
      HIPCHK(h, hipMemcpyAsync(h->ck + size_t(k) * col, X + size_t(k) * s * col, col * 8,
                               hipMemcpyDeviceToDevice, h->st));
    HIPCHK(h, hipMemcpyAsync(h->ck + size_t(h->ckK) * col, X + size_t(N) * col, col * 8,
                             hipMemcpyDeviceToDevice, h->st));
    h->fw_valid = false;  // the adjoint now overwrites the forward pair
  }
  // adjoint states: the recursion in reversed time, from zero
  h->adj_valid = false;
  if ((rc = zero_traj(h, h->bw))) return rc;
  SolveOut so;
  rc = solve_sched(h, h->bw, rtol, max_sweeps, 4, so);
  out.adjoint_sweeps = so.sweeps;
  out.adjoint_rel_resid = std::max(so.ru, so.rp);
  const auto t1 = std::chrono::steady_clock::now();
  out.seconds_adjoint = std::chrono::duration<double>(t1 - t0).count();
  if (rc) {
    if (stats) *stats = out;  // how far the adjoint solve got
    return rc;
  }
  h->adj_valid = true;
  const double* lam_top = h->bw.T[h->bw.cur] + size_t(N + 1) * col;
  if (!ckpt) {
    launch_grad_partial(h->dim, h->E, col, X, 0, lam_top, 1, N + 1, kGradChunk, 0, h->gpart, h->st);
    LAUNCHCHK(h);
  } else {
    const int gs = h->opt.replay_segments;
    double worst = 0.0;
    for (int k0 = 0; k0 < h->ckK; k0 += gs) {
      const int n0 = k0 * s;
      const int L = std::min(gs * s, N - n0);
      Sched& R = h->rp;
      HIPCHK(h, hipStreamSynchronize(h->st));  // the previous group's table uploads are done
      shape_sched(R, L, false);
      for (int j = 1; j <= L; ++j) {
        const int n = n0 + j;
        R.gstep[j] = n;
        if ((n - 1) % s == 0) R.pin[j] = h->ck + size_t((n - 1) / s) * col;
      }
      build_tables(h, R);
      if ((rc = upload_tables(h, R))) return rc;
      // start values: X^{n0} in both buffers, interpolated checkpoints inside
      launch_lerp_init(col, h->ck, s, N, n0, L, R.T[0], h->st);
      LAUNCHCHK(h);
      HIPCHK(h, hipMemcpyAsync(R.T[1], R.T[0], col * 8, hipMemcpyDeviceToDevice, h->st));
      R.cur = 0;
      SolveOut sr;
      rc = solve_sched(h, R, rtol, max_sweeps, 4, sr);
      out.replay_sweeps += sr.sweeps;
      out.replay_groups += 1;
      worst = std::max(worst, std::max(sr.ru, sr.rp));
      if (rc) {
        out.replay_rel_resid = worst;
        if (stats) *stats = out;
        return rc;
      }
      launch_grad_partial(h->dim, h->E, col, R.T[R.cur], n0, lam_top, n0 + 1, n0 + L + 1, s, k0,
                          h->gpart, h->st);
      LAUNCHCHK(h);
    }
    out.replay_rel_resid = worst;
  }
  double* gk = grads_on_device ? grad_logk : (grad_logk ? h->gout : nullptr);
  double* gl = grads_on_device ? grad_lambda : (grad_lambda ? h->gout + h->P.ne : nullptr);
  double* gm = grads_on_device ? grad_mu : (grad_mu ? h->gout + 2 * size_t(h->P.ne) : nullptr);
  launch_grad_finish(h->E, h->gpart, h->n_chunks, gk, gl, gm, h->st);
  LAUNCHCHK(h);
  if (!grads_on_device) {
    const size_t b = size_t(h->P.ne) * 8;
    if (grad_logk) HIPCHK(h, hipMemcpyAsync(grad_logk, gk, b, hipMemcpyDeviceToHost, h->st));
    if (grad_lambda) HIPCHK(h, hipMemcpyAsync(grad_lambda, gl, b, hipMemcpyDeviceToHost, h->st));
    if (grad_mu) HIPCHK(h, hipMemcpyAsync(grad_mu, gm, b, hipMemcpyDeviceToHost, h->st));
  }
  HIPCHK(h, hipStreamSynchronize(h->st));
  const auto t2 = std::chrono::steady_clock::now();
  out.seconds_replay = std::chrono::duration<double>(t2 - t1).count();
  out.seconds = std::chrono::duration<double>(t2 - t0).count();
  if (stats) *stats = out;
  return BIOT_OK;
}

int biot_get_adjoint(biot_handle* h, int32_t n0, int32_t n1, double* dst, int32_t dst_on_device) {
  int rc = check_bound(h);
  if (rc) return rc;
  if (!h->adj_valid) return fail(h, BIOT_ESTATE, "no adjoint states (call biot_adjoint)");
  if (!dst || n0 < 1 || n1 > h->N + 1 || n0 > n1) return fail(h, BIOT_EINVAL, "bad range or NULL dst");
  const size_t col = h->col;
  const double* top = h->bw.T[h->bw.cur] + size_t(h->N + 1) * col;
  for (int n = n0; n < n1; ++n)  // stored in reversed time: Lam^n at column N+1-n
    HIPCHK(h, hipMemcpyAsync(dst + size_t(n - n0) * col, top - size_t(n) * col, col * 8,
                             dst_on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, h->st));
  if (!dst_on_device) HIPCHK(h, hipStreamSynchronize(h->st));
  return BIOT_OK;
}

int biot_apply_operator(biot_handle* h, const double* X, double* Y, int32_t ncols) {
  int rc = check_bound(h);
  if (rc) return rc;
  if (!X || !Y || ncols < 0) return fail(h, BIOT_EINVAL, "bad arguments");
  if (ncols == 0) return BIOT_OK;
  launch_apply_operator(h->dim, h->L[0], h->F, X, Y, ncols, h->st);
  LAUNCHCHK(h);
  h->acct += bytes_apply_op(h, ncols);
  return BIOT_OK;
}

int biot_apply_precond(biot_handle* h, const double* R, double* Z, int32_t ncols) {
  int rc = check_bound(h);
  if (rc) return rc;
  if (!R || !Z || ncols < 0) return fail(h, BIOT_EINVAL, "bad arguments");
  if (h->opt.precision == BIOT_PRECISION_MIXED) return apply_precond_t<float>(h, h->pf, R, Z, ncols);
  return apply_precond_t<double>(h, h->pd, R, Z, ncols);
}

int biot_apply_precond_noalloc(biot_handle* h, const double* R, double* Z, int32_t ncols) {
  int rc = check_bound(h);
  if (rc) return rc;
  if (!R || !Z || ncols < 0) return fail(h, BIOT_EINVAL, "bad arguments");
  if (ncols == 0) return BIOT_OK;
  if (!h->scratch_dev) return fail(h, BIOT_ESTATE, "no scratch address for the bound device");
  if (h->opt.precision == BIOT_PRECISION_MIXED)
    return apply_precond_scratch_t<float>(h, h->pf, h->sfa_f, h->sfs_f, R, Z, ncols);
  return apply_precond_scratch_t<double>(h, h->pd, h->sfa_d, h->sfs_d, R, Z, ncols);
}

int biot_profile_enable(biot_handle* h, int32_t mask) {
  const int32_t enable = mask;
  int rc = check_bound(h);
  if (rc) return rc;
  if ((rc = harvest(h))) return rc;
  for (auto& a : h->acc) a = biot_handle::Acc{};
  const size_t waves = std::max(h->fw.wave_off.size(), h->bw.wave_off.size());
  const size_t want = std::max<size_t>(16384, 20 * (waves + 1) + 64);
  if (enable && h->ev_pool.size() < want) {
    const size_t old = h->ev_pool.size();
    h->ev_pool.resize(want);
    for (size_t i = old; i < want; ++i) HIPCHK(h, hipEventCreate(&h->ev_pool[i]));
  }
  h->prof = enable != 0;
  h->prof_mask = unsigned(mask) & ((1u << BIOT_PROBE_COUNT) - 1);
  h->prof_stride = int((unsigned(mask) >> BIOT_PROBE_STRIDE_SHIFT) & 0xFFu);
  return BIOT_OK;
}

int biot_profile_read(biot_handle* h, int32_t probe, uint64_t* launches, double* total_ms,
                      double* total_bytes, const char** name) {
  int rc = check_bound(h);
  if (rc) return rc;
  if (probe < 0 || probe >= BIOT_PROBE_COUNT) return fail(h, BIOT_EINVAL, "unknown probe");
  if ((rc = harvest(h))) return rc;
  if (launches) *launches = h->acc[probe].launches;
  if (total_ms) *total_ms = h->acc[probe].ms;
  if (total_bytes) *total_bytes = h->acc[probe].bytes;
  if (name) *name = kProbeNames[probe];
  return BIOT_OK;
}

int biot_get_info(const biot_handle* h, biot_info_t* info) {
  if (!h || !info) return BIOT_EINVAL;
  std::memset(info, 0, sizeof(*info));
  info->dim = h->dim;
  info->n_nodes = h->nn;
  info->n_steps = h->N;
  info->n_levels = h->nlev;
  for (int l = 0; l < h->nlev && l < 16; ++l) {
    info->level_cells[l] = h->P.levels[l].n_cells;
    info->level_nodes[l] = h->P.levels[l].nn;
    info->lmax_A[l] = h->P.levels[l].lmaxA;
    info->lmax_S[l] = h->P.levels[l].lmaxS;
  }
  info->slots = h->P.levels[0].W;
  info->workspace_bytes = h->ws_need;
  info->n_samples = h->S;
  info->nodes_per_sample = h->P.levels[0].nn1;
  return BIOT_OK;
}

int biot_export_level(const biot_handle* h, int32_t level, int32_t* nbr, double* A, double* S,
                      double* B, double* Bt, double* Cb, double* F) {
  if (!h || level < 0 || level >= h->nlev) return BIOT_EINVAL;
  const HostLevel& H = h->P.levels[level];
  if (nbr) std::memcpy(nbr, H.nbr.data(), H.nbr.size() * sizeof(int32_t));
  if (A) std::memcpy(A, H.A.data(), H.A.size() * sizeof(double));
  if (S) std::memcpy(S, H.S.data(), H.S.size() * sizeof(double));
  if (level == 0) {
    if (B) std::memcpy(B, H.B.data(), H.B.size() * sizeof(double));
    if (Bt) std::memcpy(Bt, H.Bt.data(), H.Bt.size() * sizeof(double));
    if (Cb) std::memcpy(Cb, H.Cb.data(), H.Cb.size() * sizeof(double));
    if (F) std::memcpy(F, h->P.F.data(), h->P.F.size() * sizeof(double));
  }
  return BIOT_OK;
}

const char* biot_last_error(const biot_handle* h) {
  return h ? h->err.c_str() : g_create_error.c_str();
}

const char* biot_version(void) {
  return "biot_pint 0.3 (gfx950; FP64 and FP32/FP64 mixed; discrete adjoint)";
}

void biot_destroy(biot_handle* h) {
  if (!h) return;
  for (Sched* S : {&h->fw, &h->bw, &h->rp}) destroy_graphs(*S);
  if (h->cap_stream) (void)hipStreamDestroy(h->cap_stream);
  for (auto& e : h->ev_pool) (void)hipEventDestroy(e);
  delete h;
}

}  // extern "C"
