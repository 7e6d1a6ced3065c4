// HIP kernels (gfx950) of the preconditioned inverted time-stepping sweep.
//
// Every kernel processes a batch of columns (time steps / iterations) at once.
//
// Thread mapping of the node-blocked kernels ("operator-stationary"): a thread
// owns one node, loads that node's operator row (all stencil slots) into
// registers once, and then loops over a run of time-step columns two at a
// time.  The operator is read once per run while the column data streams
// through.  Work is split evenly over a grid sized to the chip (see
// for_each_piece): the (node block, column) units of a launch are dealt out as
// contiguous ranges, so no workgroup is left over for a last partial round, and
// the ranges of the workgroups on one XCD are contiguous, so the rows above and
// below a node block (the stencil's other neighbours) sit in the same L2.
// Rows too large for registers (3D displacement blocks) are re-read per column
// pair, from L1/L2.
//
// Layouts (see setup.hpp): operator values [slot][entry][node]; state columns
// node-major [node][u_x, u_y, (u_z), p] in FP64; multigrid work vectors
// node-major [node][comp], one contiguous vector per column of the batch, of
// type T (double, or float in the mixed-precision preconditioner).
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <functional>
#include <mutex>
#include <unordered_map>

#include "kernels.hpp"

// waves per SIMD the 2D Chebyshev kernels are compiled for (register budget)
#ifndef BIOT_CHEB_MIN_WAVES
#define BIOT_CHEB_MIN_WAVES 2
#endif

namespace biot {
namespace {

__constant__ int c_off2[7][3] = {{0, 0, 0}, {1, 0, 0}, {-1, 0, 0}, {0, 1, 0},
                                 {0, -1, 0}, {1, 1, 0}, {-1, -1, 0}};
__constant__ int c_off3[15][3] = {{0, 0, 0},  {1, 0, 0},  {-1, 0, 0},  {0, 1, 0},  {0, -1, 0},
                                  {0, 0, 1},  {0, 0, -1}, {1, 1, 0},   {-1, -1, 0}, {1, 0, 1},
                                  {-1, 0, -1}, {0, 1, 1}, {0, -1, -1}, {1, 1, 1},  {-1, -1, -1}};

template <int DIM>
__device__ inline void node_coords(int id, int m, int& i, int& j, int& k) {
  i = id % m;
  j = (id / m) % m;
  k = DIM == 2 ? 0 : id / (m * m);
}
template <int DIM>
__device__ inline int node_id(int i, int j, int k, int m) {
  return DIM == 2 ? j * m + i : (k * m + j) * m + i;
}

// grid nodes of a copy with `cells` cells per side
template <int DIM>
__device__ inline int grid_nodes(int cells) {
  const int m = cells + 1;
  return DIM == 2 ? m * m : m * m * m;
}

// Copy of a node block, a copy's first node and its cells per side; a level
// with one copy (a single problem) takes them from the kernel arguments
// rather than from the tables, which saves a dependent load per piece.
template <typename T>
__device__ inline int block_copy(const LevelView<T>& L, int nblk) {
  return L.copies == 1 ? 0 : L.bcopy[nblk];
}
template <typename T>
__device__ inline int copy_base(const LevelView<T>& L, int cp) {
  return L.copies == 1 ? 0 : L.cbase[cp];
}
template <typename T>
__device__ inline int copy_cells(const LevelView<T>& L, int cp) {
  return L.copies == 1 ? L.n_cells : L.ccells[cp];
}

// Loads and stores through pointers read from memory (the column
// descriptors' state columns) in the global address space: through a generic
// pointer they compile to flat operations, which a wait for LDS traffic
// (lgkmcnt) also waits for.
template <typename V>
__device__ inline V gld(const V* p) {
  return *(const __attribute__((address_space(1))) V*)p;
}
template <typename V>
__device__ inline void gst(V* p, V v) {
  *(__attribute__((address_space(1))) V*)p = v;
}

// Shrinks the column range [cbeg, cend) of a launch to the columns active for
// copy cp (a sample skips the steps past its own count); they are contiguous.
template <typename T>
__device__ inline void active_cols(const LevelView<T>& L, int cp, int& cbeg, int& cend) {
  if (!L.act) return;
  const int ns = L.csteps[cp];
  while (cbeg < cend && L.act[cbeg].step > ns) ++cbeg;
  while (cend > cbeg && L.act[cend - 1].step > ns) --cend;
}
template <typename T>
__device__ inline bool col_active(const LevelView<T>& L, int cp, int c) {
  return !L.act || L.act[c].step <= L.csteps[cp];
}

// Balanced split of a launch's work over its grid.  The units are the pairs
// (node block of kBlock nodes, column), ordered block-major; workgroup slot l
// takes units [U l / P, U (l+1) / P) and calls f(node_block, c_begin, c_end)
// for each node block its range touches (at most a few), so every workgroup
// does the same amount of work to within one unit.  The hardware deals
// workgroups to the 8 XCDs round-robin (workgroup i on XCD i % 8); the slot of
// workgroup i is chosen so that each XCD holds one contiguous run of slots,
// i.e. neighbouring node blocks, whose shared stencil rows then hit one L2.
// The range depends only on blockIdx, so f's control flow is uniform across a
// workgroup (f may use __syncthreads).
// ALIGNED (the grid is nblocks * groups, see balanced_grid): each workgroup
// takes one node block and one of `groups` equal runs of its columns, so that
// neighbouring blocks walk through the same columns at the same time and
// share the stencil rows they gather in L2; used by the 3D displacement
// kernels, whose rows are re-read per group of columns anyway (40^3 cube:
// 707 -> 660 ms; the 2D kernels and the 3D pressure kernels were slower).
template <bool ALIGNED = false, typename F>
__device__ inline void for_each_piece(int nblocks, int nc, F&& f) {
  const int P = gridDim.x, i = blockIdx.x;
  if constexpr (ALIGNED) {
    if (P >= nblocks) {  // (otherwise the balanced split below covers the work)
      const int q = P >> 3;
      const int l = i < 8 * q ? (i & 7) * q + (i >> 3) : i;
      const int groups = P / nblocks, run = (nc + groups - 1) / groups;
      const int nb = l / groups, c0 = (l % groups) * run, c1 = min(nc, c0 + run);
      if (nb < nblocks && c0 < c1) f(nb, c0, c1);
      return;
    }
  }
  const int l = (P & 7) == 0 ? (i & 7) * (P >> 3) + (i >> 3) : i;
  const long U = long(nblocks) * nc;
  long u = U * l / P;
  const long u1 = U * (l + 1) / P;
  while (u < u1) {
    const int nb = int(u / nc), c0 = int(u % nc);
    const int c1 = int(min(long(nc), c0 + (u1 - u)));
    u += c1 - c0;
    f(nb, c0, c1);
  }
}

// Deterministic block sum of Q values per thread (wave64 shuffles, then LDS
// across the 4 waves in a fixed order).  Result valid in thread 0.  Every
// thread of the block must call it.
template <int Q>
__device__ inline void block_sum(double (&v)[Q], double* lds /* [4][Q] */) {
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    double x = v[q];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) x += __shfl_down(x, off, 64);
    v[q] = x;
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0)
#pragma unroll
    for (int q = 0; q < Q; ++q) lds[wave * Q + q] = v[q];
  __syncthreads();
  if (threadIdx.x == 0)
#pragma unroll
    for (int q = 0; q < Q; ++q) v[q] = ((lds[q] + lds[Q + q]) + lds[2 * Q + q]) + lds[3 * Q + q];
  __syncthreads();
}

// ---------------------------------------------------------------------------
// fine-level residual r = c(n) F + A' X^{n-1} - AA X^{n,m-1} (FP64), the
// coupled right-hand side norms; r is stored as T.  The displacement V-cycle's
// first Chebyshev step from zero (x = D^{-1} r / theta, pointwise) is not
// stored: the next step forms it on the fly (see k_cheb's `first`).
// ADJ: the adjoint recursion run forward in reversed time, whose coupling is
// A'^T = [0 B; 0 -C_beta] applied to the previous column and whose load is the
// pressure-row vector gload[step-1] (no traction load):
//   r = [B p'; -C_beta p' + g] - AA X^{m-1}.
// ---------------------------------------------------------------------------
template <int DIM, typename T, bool ADJ>
__global__ __launch_bounds__(kBlock) void k_residual(LevelDev L, FineDev F,
                                                     const ColDesc* __restrict__ cols, int nc,
                                                     T* __restrict__ ru, T* __restrict__ rp,
                                                     double* __restrict__ partials, int pstride) {
  // columns per iteration: two in 2D, whose rows stay in registers; eight in 3D,
  // whose rows are re-read from the caches once per group of columns
  constexpr bool STAT = DIM == 2;
  constexpr int NQ = STAT ? 2 : 8;
  constexpr int D1 = DIM + 1;
  constexpr int W = DIM == 2 ? 7 : 15;
  constexpr int RS = STAT ? W : 1;
  constexpr int SU = STAT ? W : 3;  // slot-loop unrolling (full when the row is in registers)
  __shared__ double lds[4 * 4 * NQ];
  const int nn = L.nn;
  for_each_piece<!STAT>(num_node_blocks(L.nact), nc, [&](int nblk, int cbeg, int cend) {
    if (L.act) active_cols(L, L.bcopy[nblk], cbeg, cend);
    if (cbeg >= cend) return;
    const int v = nblk * kBlock + threadIdx.x;
    const bool active = v < L.nact;
    const int vv = active ? v : nn - 1;
    int nb[RS];
    if constexpr (STAT) {
#pragma unroll
      for (int s = 0; s < W; ++s) nb[s] = L.nbr[size_t(s) * nn + vv];
    }
    double rA[RS][DIM * DIM], rB[RS][DIM], rBt[RS][DIM], rS[RS], rCb[RS];
    if constexpr (STAT) {
#pragma unroll
      for (int s = 0; s < W; ++s) {
#pragma unroll
        for (int e = 0; e < DIM * DIM; ++e) rA[s][e] = L.A[(size_t(s) * DIM * DIM + e) * nn + vv];
#pragma unroll
        for (int c = 0; c < DIM; ++c) {
          rB[s][c] = F.B[(size_t(s) * DIM + c) * nn + vv];
          rBt[s][c] = F.Bt[(size_t(s) * DIM + c) * nn + vv];
        }
        rS[s] = L.S[size_t(s) * nn + vv];
        rCb[s] = F.Cb[size_t(s) * nn + vv];
      }
    }
    // load f^n = sum_j c_j(n) F_j: term 0 stays in registers, further terms
    // are read per column pair (from the caches); prescribed dofs are masked
    const int nt = ADJ ? 0 : F.nt;
    const unsigned fx = active ? unsigned(L.fixed[vv]) : 0u;
    double Fu[DIM], Fp = 0.0;
#pragma unroll
    for (int a = 0; a < DIM; ++a) Fu[a] = (active && nt > 0) ? F.F[size_t(vv) * D1 + a] : 0.0;
    if (active && nt > 0) Fp = F.F[size_t(vv) * D1 + DIM];
#pragma unroll 1
    for (int c = cbeg; c < cend; c += NQ) {
      // columns past the end of the run repeat the last one (computed, not stored)
      int cc[NQ];
#pragma unroll
      for (int q = 0; q < NQ; ++q) cc[q] = min(c + q, cend - 1);
      const double* xc[NQ];
      const double* xp[NQ];
      double lb[NQ], au[NQ][DIM], ap[NQ], bp[NQ], cu[NQ][DIM];
#pragma unroll
      for (int q = 0; q < NQ; ++q) {
        xc[q] = cols[cc[q]].xcur;
        xp[q] = cols[cc[q]].xprev;
#pragma unroll
        for (int a = 0; a < DIM; ++a) cu[q][a] = 0.0;
        if constexpr (ADJ) {
          const double g = active ? F.gload[size_t(cols[cc[q]].step - 1) * nn + vv] : 0.0;
#pragma unroll
          for (int a = 0; a < DIM; ++a) au[q][a] = 0.0;
          ap[q] = g;
          bp[q] = g;
          lb[q] = 0.0;
        } else {
          const double* tc = cols[cc[q]].tc;
          const double c0 = cols[cc[q]].c0;
#pragma unroll
          for (int a = 0; a < DIM; ++a) au[q][a] = c0 * Fu[a];
          ap[q] = c0 * Fp;
#pragma unroll 1
          for (int j = 1; j < nt; ++j) {
            const double cj = tc[j];
            const double* Tj = F.F + (size_t(j) * nn + vv) * D1;
#pragma unroll
            for (int a = 0; a < DIM; ++a) au[q][a] += cj * Tj[a];
            ap[q] += cj * Tj[DIM];
          }
          bp[q] = ap[q];
          double sl = 0.0;
#pragma unroll
          for (int a = 0; a < DIM; ++a) sl += au[q][a] * au[q][a];
          lb[q] = sl;
        }
      }
#pragma unroll SU
      for (int s = 0; s < W; ++s) {
        const int w = STAT ? nb[s] : L.nbr[size_t(s) * nn + vv];
        double Ab[DIM * DIM], Bb[DIM], Btb[DIM], Sv, Cbv;
        if constexpr (STAT) {
#pragma unroll
          for (int e = 0; e < DIM * DIM; ++e) Ab[e] = rA[s][e];
#pragma unroll
          for (int k = 0; k < DIM; ++k) {
            Bb[k] = rB[s][k];
            Btb[k] = rBt[s][k];
          }
          Sv = rS[s];
          Cbv = rCb[s];
        } else {
#pragma unroll
          for (int e = 0; e < DIM * DIM; ++e) Ab[e] = L.A[(size_t(s) * DIM * DIM + e) * nn + vv];
#pragma unroll
          for (int k = 0; k < DIM; ++k) {
            Bb[k] = F.B[(size_t(s) * DIM + k) * nn + vv];
            Btb[k] = F.Bt[(size_t(s) * DIM + k) * nn + vv];
          }
          Sv = L.S[size_t(s) * nn + vv];
          Cbv = F.Cb[size_t(s) * nn + vv];
        }
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
          double xw[D1], xpw[D1];
#pragma unroll
          for (int k = 0; k < D1; ++k) {
            xw[k] = gld(xc[q] + size_t(w) * D1 + k);
            xpw[k] = gld(xp[q] + size_t(w) * D1 + k);
          }
#pragma unroll
          for (int a = 0; a < DIM; ++a) {
            double acc = Bb[a] * xw[DIM];
#pragma unroll
            for (int k = 0; k < DIM; ++k) acc += Ab[a * DIM + k] * xw[k];
            au[q][a] -= acc;
          }
          double btc = 0.0;
#pragma unroll
          for (int k = 0; k < DIM; ++k) btc += Btb[k] * xw[k];
          double coup;
          if constexpr (ADJ) {
#pragma unroll
            for (int a = 0; a < DIM; ++a) {
              const double c = Bb[a] * xpw[DIM];
              cu[q][a] += c;
              au[q][a] += c;
            }
            coup = -Cbv * xpw[DIM];
          } else {
            double btp = 0.0;
#pragma unroll
            for (int k = 0; k < DIM; ++k) btp += Btb[k] * xpw[k];
            coup = btp - Cbv * xpw[DIM];
          }
          bp[q] += coup;
          ap[q] += coup - btc + Sv * xw[DIM];
        }
      }
      // prescribed rows: zero residual (their values are kept in the state)
#pragma unroll
      for (int q = 0; q < NQ; ++q) {
#pragma unroll
        for (int a = 0; a < DIM; ++a)
          if ((fx >> a) & 1u) au[q][a] = 0.0;
        if ((fx >> DIM) & 1u) ap[q] = 0.0;
      }
#pragma unroll
      for (int q = 0; q < NQ; ++q) {
        if (!active || c + q >= cend) break;
        const size_t cu = size_t(cc[q]) * nn * DIM;
        if (ru) {
#pragma unroll
          for (int a = 0; a < DIM; ++a) ru[cu + size_t(v) * DIM + a] = T(au[q][a]);
          rp[size_t(cc[q]) * nn + v] = T(ap[q]);
        }
      }
      if (partials) {
        double qv[4 * NQ];
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
          double su = 0.0, sb = lb[q];
#pragma unroll
          for (int a = 0; a < DIM; ++a) {
            su += au[q][a] * au[q][a];
            if constexpr (ADJ) sb += cu[q][a] * cu[q][a];
          }
          qv[4 * q + 0] = active ? su : 0.0;
          qv[4 * q + 1] = active ? ap[q] * ap[q] : 0.0;
          qv[4 * q + 2] = active ? sb : 0.0;
          qv[4 * q + 3] = active ? bp[q] * bp[q] : 0.0;
        }
        block_sum<4 * NQ>(qv, lds);
        if (threadIdx.x == 0)
#pragma unroll
          for (int q = 0; q < NQ; ++q) {
            if (c + q >= cend) break;
#pragma unroll
            for (int k = 0; k < 4; ++k)
              partials[(size_t(cc[q]) * pstride + nblk) * 4 + k] = qv[4 * q + k];
          }
      }
    }
  });
}

// ---------------------------------------------------------------------------
// Prolongation of fine node f: parents p0, p1 on the coarse grid and a bit mask
// of the components that receive each parent (bit a: p0, bit C+a: p1, bit 2C:
// edge midpoint with weight 1/2; otherwise a coincident node with weight 1).
// A component is masked when the fine or the coarse dof is prescribed.
// ---------------------------------------------------------------------------
// f is a node of copy cp on the fine level (global numbering); the parents
// are returned in the coarse level's global numbering.
template <int DIM, int C, typename T>
__device__ inline void prolong_parents(const LevelView<T>& Lf, const LevelView<T>& Lc, int bit0,
                                       int cp, int f, int& p0, int& p1, unsigned& mask) {
  const int cf = copy_cells(Lf, cp);
  const int mf = cf + 1, mc = copy_cells(Lc, cp) + 1;
  const int fb = copy_base(Lf, cp), cb = copy_base(Lc, cp);
  const int lf = f - fb;  // node within the copy
  if (lf >= grid_nodes<DIM>(cf)) {  // padding node: no parents
    p0 = p1 = cb;
    mask = 0u;
    return;
  }
  int i, j, k;
  node_coords<DIM>(lf, mf, i, j, k);
  const int ai = i >> 1, aj = j >> 1, ak = k >> 1;
  const int oi = i & 1, oj = j & 1, ok = k & 1;
  const bool two = (oi | oj | ok) != 0;
  p0 = cb + node_id<DIM>(ai, aj, ak, mc);
  p1 = two ? cb + node_id<DIM>(ai + oi, aj + oj, ak + ok, mc) : p0;
  const unsigned ff = Lf.fixed[f], f0 = Lc.fixed[p0], f1 = Lc.fixed[p1];
  mask = two ? (1u << 2 * C) : 0u;
#pragma unroll
  for (int a = 0; a < C; ++a) {
    const bool fm = !((ff >> (bit0 + a)) & 1u);
    if (fm && !((f0 >> (bit0 + a)) & 1u)) mask |= 1u << a;
    if (two && fm && !((f1 >> (bit0 + a)) & 1u)) mask |= 1u << (C + a);
  }
}

// ---------------------------------------------------------------------------
// Chebyshev step on one level:  d <- c1 d + c2 D^{-1}(b - K xin);  xout = xin + d.
// wd = 0 leaves d unwritten (the last step before a residual or at the end of
// the smoothing, after which d is dead, and the first step after a coarse-grid
// correction).  dx selects where the previous increment comes from:
//   0: d;
//   1: xin itself (the step after a first step from zero);
//   2: xin - xout, xout still holding the previous step's input (the step
//      after the first post-smoothing step, which stores no d); the node's
//      own xout value is read before it is overwritten.
// first = 1: this is the step after the first step from zero, which is not
// stored: xin = it D^{-1} b is formed on the fly, K xin as it * KD b with the
// folded operator KD_k = K_k D^{-1}(nbr_k) (L.AD / L.SD); use with dx = 1.
// UPD (pressure field, level 0, last step): instead of xout, writes the outer
// update X^{n,m} = X^{n,m-1} + omega [z_u; xin + d] (FP64) through the column
// descriptors.  FINE only makes the level-0 launches a distinct symbol.
// ---------------------------------------------------------------------------
template <int DIM, int C, bool UPD, bool FINE, typename T>
__global__ __launch_bounds__(kBlock, DIM == 2 ? BIOT_CHEB_MIN_WAVES : 1) void k_cheb(LevelView<T> L, int isA,
                                                 const T* __restrict__ b,
                                                 const T* __restrict__ xin,
                                                 T* xout, T* __restrict__ d, int nc,
                                                 T c1, T c2, int wd, int dx, int first, T it,
                                                 const ColDesc* __restrict__ cols,
                                                 const T* __restrict__ zu, double omega) {
  // columns per iteration: when the row stays in registers two, or one for the
  // FP64 pressure field (measured); otherwise (3D displacement) the row is
  // re-read from the caches once per group of eight FP64 or four FP32 columns
  // (measured on the 40^3 cube: in FP32 the smaller group's higher occupancy
  // outweighs the extra row reads)
  constexpr int W = DIM == 2 ? 7 : 15;
  constexpr bool STAT = W * C * C <= 64;
  constexpr int NQ = STAT ? (C == 1 && sizeof(T) == 8 ? 1 : 2) : (sizeof(T) == 4 ? 4 : 8);
  constexpr int RS = STAT ? W : 1;
  constexpr int SU = STAT ? W : 3;  // slot-loop unrolling (full when the row is in registers)
  const int nn = L.nn;
  for_each_piece<!STAT>(num_node_blocks(L.nact), nc, [&](int nblk, int cbeg, int cend) {
    if (L.act) active_cols(L, L.bcopy[nblk], cbeg, cend);
    const int v = nblk * kBlock + threadIdx.x;
    if (v >= L.nact || cbeg >= cend) return;
    // C > 1 is the displacement field (A), C == 1 the pressure field (S)
    const T* K = first ? (C > 1 ? L.AD : L.SD) : (C > 1 ? L.A : L.S);
    const T* Dg = C > 1 ? L.Ainv : L.Sinv;
    const T* src = first ? b : xin;       // the gathered vector
    const T sc = first ? it : T(1);       // its scale in K xin
    const size_t stride = size_t(nn) * C;
    int nb[RS];
    if constexpr (STAT) {
#pragma unroll
      for (int s = 0; s < W; ++s) nb[s] = L.nbr[size_t(s) * nn + v];
    }
    T kr[RS][C * C];
    if constexpr (STAT) {
#pragma unroll
      for (int s = 0; s < W; ++s)
#pragma unroll
        for (int e = 0; e < C * C; ++e) kr[s][e] = K[(size_t(s) * C * C + e) * nn + v];
    }
    T Di[C * C];
#pragma unroll
    for (int e = 0; e < C * C; ++e) Di[e] = Dg[size_t(e) * nn + v];
#pragma unroll 1
    for (int c = cbeg; c < cend; c += NQ) {
      // columns past the end of the run repeat the last one (computed, not stored)
      int cc[NQ];
#pragma unroll
      for (int q = 0; q < NQ; ++q) cc[q] = min(c + q, cend - 1);
      // column base pointers; offsets within a column fit in 32 bits
      const T* xq[NQ];
#pragma unroll
      for (int q = 0; q < NQ; ++q) xq[q] = src + size_t(cc[q]) * stride;
      T acc[NQ][C], xs[NQ][C];
#pragma unroll
      for (int q = 0; q < NQ; ++q)
#pragma unroll
        for (int a = 0; a < C; ++a) acc[q][a] = b[size_t(cc[q]) * stride + v * C + a];
#pragma unroll SU
      for (int s = 0; s < W; ++s) {
        const int w = STAT ? nb[s] : L.nbr[size_t(s) * nn + v];
        T blk[C * C];
#pragma unroll
        for (int e = 0; e < C * C; ++e) {
          if constexpr (STAT) blk[e] = kr[s][e];
          else blk[e] = K[(size_t(s) * C * C + e) * nn + v];
        }
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
          T xw[C];
#pragma unroll
          for (int k = 0; k < C; ++k) xw[k] = xq[q][w * C + k];
          if (s == 0) {
            if (first) {
#pragma unroll
              for (int a = 0; a < C; ++a) {
                T z = T(0);
#pragma unroll
                for (int k = 0; k < C; ++k) z += Di[a * C + k] * xw[k];
                xs[q][a] = z * it;
              }
            } else {
#pragma unroll
              for (int k = 0; k < C; ++k) xs[q][k] = xw[k];
            }
          }
#pragma unroll
          for (int a = 0; a < C; ++a) {
            T s2 = T(0);
#pragma unroll
            for (int k = 0; k < C; ++k) s2 += blk[a * C + k] * xw[k];
            acc[q][a] -= sc * s2;
          }
        }
      }
#pragma unroll
      for (int q = 0; q < NQ; ++q) {
        if (c + q >= cend) break;
        const size_t base = size_t(cc[q]) * stride + size_t(v) * C;
        T xn[C];
#pragma unroll
        for (int a = 0; a < C; ++a) {
          T z = T(0);
#pragma unroll
          for (int k = 0; k < C; ++k) z += Di[a * C + k] * acc[q][k];
          const T dp = c1 == T(0) ? T(0)
                       : dx == 1 ? xs[q][a]
                       : dx == 2 ? xs[q][a] - xout[base + a]
                                 : d[base + a];
          // one rounding order for the update, shared with k_post2
          const T dn = fma(c2, z, c1 * dp);
          if (!UPD && wd) d[base + a] = dn;
          xn[a] = xs[q][a] + dn;
        }
        if constexpr (!UPD) {
#pragma unroll
          for (int a = 0; a < C; ++a) xout[base + a] = xn[a];
        } else {
          // pressure field on level 0 (C == 1): write the updated state column
          constexpr int D1 = DIM + 1;
          const ColDesc cd = cols[cc[q]];
          double out[D1];
#pragma unroll
          for (int a = 0; a < DIM; ++a)
            out[a] = gld(cd.xcur + size_t(v) * D1 + a) +
                     omega * double(zu[(size_t(cc[q]) * nn + v) * DIM + a]);
          out[DIM] = gld(cd.xcur + size_t(v) * D1 + DIM) + omega * double(xn[0]);
#pragma unroll
          for (int a = 0; a < D1; ++a) gst(cd.xout + size_t(v) * D1 + a, out[a]);
          if (cd.xout2)
#pragma unroll
            for (int a = 0; a < D1; ++a) gst(cd.xout2 + size_t(v) * D1 + a, out[a]);
        }
      }
    }
  });
}

// A workgroup barrier for LDS traffic only: waits for this wave's LDS
// operations, not for its global stores (which __syncthreads also waits for,
// to publish them to the workgroup; nothing here reads them back).
__device__ inline void lds_barrier() {
  asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
}

// The coarse-grid correction and the two post-smoothing steps of degree 2 on
// a structured 2D level, fused (each sample copy of a batch has its own
// patches; the padding nodes of a copy are not written, and hold the zeros the
// level residual wrote to x4's buffer there):
//   x2 = x + P xc                                   (coarse-grid correction)
//   x3 = x2 + c2a D^{-1}(b - K x2)                  (first step, no increment)
//   x4 = x3 + c1b (x3 - x2) + c2b D^{-1}(b - K x3)  (second step)
// with the arithmetic of k_prolong and two k_cheb launches, so the result is
// the same bit for bit.  A workgroup takes a kPatch x kPatch patch of grid
// nodes, one per thread, whose operator rows stay in registers over the
// columns.  Per column, the workgroup forms x2 over the patch and one more
// ring (kReg x kReg nodes, into LDS; x2 never goes to global memory), then
// every node of the patch forms x3 from x2 there (into LDS), then the interior
// (the patch without its outer ring) forms x4 from its neighbours' x3.
// Patches step by the interior width, so each node is the interior of exactly
// one patch.  x and x4 are different buffers (other patches read x around
// their rings).
// Columns are software-pipelined: between two barriers a workgroup loads and
// forms x2 of the next column while it forms x4 of the current one, so the
// loads' latency overlaps the second step; x3 sits in two LDS buffers.
// Work split: the columns of each patch are cut into `groups` runs of `run`
// columns, one workgroup each, all resident at once, so that neighbouring
// patches walk through the same columns together and share the ring rows they
// read in L2; workgroup i goes to XCD i % 8, and each XCD is given a
// contiguous range of (patch, run) pairs, i.e. neighbouring patches.
constexpr int kPatch = 16;
constexpr int kPatchIn = kPatchInterior;
constexpr int kReg = kPatch + 2;  // x2 region: the patch and one more ring
static_assert(kPatchIn == kPatch - 2, "a patch's interior drops its outer ring");
static_assert(kPatch * kPatch == kBlock, "one patch node per thread");
static_assert(kReg * kReg <= 2 * kBlock, "two x2 region nodes per thread at most");

template <int DIM, int C, typename T>
__device__ inline void prolong_parents(const LevelView<T>& Lf, const LevelView<T>& Lc, int bit0,
                                       int cp, int f, int& p0, int& p1, unsigned& mask);

// UPD (pressure field, level 0, C == 1): instead of storing x4, write the
// outer update X^{n,m} = X^{n,m-1} + omega [z_u; x4] through the column
// descriptors, as k_cheb's last step does (the copies' padding nodes get
// X^{n,m-1} + omega [z_u; 0]).
template <int C, bool UPD, typename T>
__global__ __launch_bounds__(kBlock) void k_post2(LevelView<T> L, LevelView<T> Lc, int isA,
                                                  const T* __restrict__ b,
                                                  const T* __restrict__ xin,
                                                  const T* __restrict__ xc,
                                                  T* __restrict__ x4, int nc, T c2a, T c1b,
                                                  T c2b, int groups, int run,
                                                  const ColDesc* __restrict__ cols,
                                                  const T* __restrict__ zu, double omega) {
  constexpr int W = 7, DIM = 2, D1 = 3;
  static_assert(!UPD || C == 1, "the outer update follows the pressure field");
  // per buffer: x3, and the node's own x2 and b, of the patch's nodes
  __shared__ T sh[2][3][kBlock][C];
  __shared__ T sx2[kReg * kReg][C];  // x2 over the region
  const int nn = L.nn;
  const int li = threadIdx.x % kPatch, lj = threadIdx.x / kPatch;
  const T* K = isA ? L.A : L.S;
  const T* Dg = isA ? L.Ainv : L.Sinv;
  const size_t stride = size_t(nn) * C, cstride = size_t(Lc.nn) * C;
  int buf = 0;
  {
    const int P = gridDim.x, i = blockIdx.x;  // P is a multiple of 8
    const int slot = (i & 7) * (P >> 3) + (i >> 3);
    if (slot >= L.npatch * groups) return;
    // patch of a copy (sample of a batch; copies may differ in size)
    const int gp = slot / groups;
    const bool one = L.copies == 1;
    const int cp = one ? 0 : L.ptab[2 * gp], patch = one ? gp : L.ptab[2 * gp + 1];
    const int m = copy_cells(L, cp) + 1, base = copy_base(L, cp);
    const int per_side = (m + kPatchIn - 1) / kPatchIn;
    int cbeg = (slot % groups) * run, cend = min(nc, cbeg + run);
    if (L.act) active_cols(L, cp, cbeg, cend);
    if (cbeg >= cend) return;
    const int i0 = (patch % per_side) * kPatchIn - 1, j0 = (patch / per_side) * kPatchIn - 1;
    const int gi = i0 + li, gj = j0 + lj;
    const bool node = gi >= 0 && gi < m && gj >= 0 && gj < m;
    const bool inner = node && li >= 1 && li <= kPatchIn && lj >= 1 && lj <= kPatchIn;
    const int v = base + (node ? gj * m + gi : 0);
    int nb[W];
    T kr[W][C * C], Di[C * C];
#pragma unroll
    for (int s = 0; s < W; ++s) {
      nb[s] = node ? L.nbr[size_t(s) * nn + v] : 0;
#pragma unroll
      for (int e = 0; e < C * C; ++e) kr[s][e] = node ? K[(size_t(s) * C * C + e) * nn + v] : T(0);
    }
#pragma unroll
    for (int e = 0; e < C * C; ++e) Di[e] = node ? Dg[size_t(e) * nn + v] : T(0);
    // neighbours in the patch (x3) and in the region (x2), and the node's own
    // place in the region
    int ls[W], lr[W];
#pragma unroll
    for (int s = 0; s < W; ++s) {
      const int ni = (nb[s] - base) % m, nj = (nb[s] - base) / m;
      ls[s] = (ni - i0) + (nj - j0) * kPatch;
      lr[s] = (ni - i0 + 1) + (nj - j0 + 1) * kReg;
    }
    const int own = (li + 1) + (lj + 1) * kReg;
    // this thread's region nodes (r = threadIdx.x, threadIdx.x + kBlock) and
    // their parents on the coarse level, for every column
    int rf[2], rp0[2], rp1[2];
    unsigned rpm[2];
    bool rv[2];
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      const int r = threadIdx.x + k * kBlock;
      const int ri = i0 - 1 + r % kReg, rj = j0 - 1 + r / kReg;
      rv[k] = r < kReg * kReg && ri >= 0 && ri < m && rj >= 0 && rj < m;
      rf[k] = base + (rv[k] ? rj * m + ri : 0);
      rp0[k] = rp1[k] = copy_base(Lc, cp);
      rpm[k] = 0u;
      if (rv[k]) prolong_parents<2, C>(L, Lc, isA ? 0 : 2, cp, rf[k], rp0[k], rp1[k], rpm[k]);
    }
    // x2 = x + P xc over the region (k_prolong's arithmetic): the loads, with
    // the node's b (kept for phase1, which runs after a barrier), are issued
    // before phase2 of the previous column and the sums stored after it
    T bnext[C], xv[2][C], q0[2][C], q1[2][C];
    auto phase0_load = [&](int c) {
#pragma unroll
      for (int a = 0; a < C; ++a) bnext[a] = node ? b[size_t(c) * stride + size_t(v) * C + a] : T(0);
      // unconditional (a region node outside the grid reads the copy's first
      // node and its value is not used), so that all are in flight together
#pragma unroll
      for (int k = 0; k < 2; ++k)
#pragma unroll
        for (int a = 0; a < C; ++a) {
          xv[k][a] = xin[size_t(c) * stride + size_t(rf[k]) * C + a];
          q0[k][a] = xc[size_t(c) * cstride + size_t(rp0[k]) * C + a];
          q1[k][a] = xc[size_t(c) * cstride + size_t(rp1[k]) * C + a];
        }
    };
    auto phase0_store = [&]() {
#pragma unroll
      for (int k = 0; k < 2; ++k) {
        if (!rv[k]) continue;
        const T wt = (rpm[k] >> (2 * C)) ? T(0.5) : T(1);
#pragma unroll
        for (int a = 0; a < C; ++a) {
          T x = xv[k][a];
          if ((rpm[k] >> a) & 1u) x += wt * q0[k][a];
          if ((rpm[k] >> (C + a)) & 1u) x += wt * q1[k][a];
          sx2[threadIdx.x + k * kBlock][a] = x;
        }
      }
    };
    // UPD: the state column and z_u of the node for phase2 of column c,
    // loaded by phase1(c) (after phase2 of the previous column)
    double xold[D1], zun[DIM];
    // x3 of the patch's nodes from x2 in LDS
    auto phase1 = [&](int c, int bb) {
      if (!node) return;
      if constexpr (UPD) {
        const double* xcur = cols[c].xcur;
#pragma unroll
        for (int a = 0; a < D1; ++a) xold[a] = gld(xcur + size_t(v) * D1 + a);
#pragma unroll
        for (int a = 0; a < DIM; ++a) zun[a] = double(zu[(size_t(c) * nn + v) * DIM + a]);
      }
      T acc[C], x2o[C];
#pragma unroll
      for (int a = 0; a < C; ++a) {
        const T bv = bnext[a];  // b of column c, loaded by phase0(c)
        acc[a] = bv;
        sh[bb][2][threadIdx.x][a] = bv;
        x2o[a] = sx2[own][a];
      }
#pragma unroll
      for (int s = 0; s < W; ++s) {
        T xw[C];
#pragma unroll
        for (int k = 0; k < C; ++k) xw[k] = sx2[lr[s]][k];
#pragma unroll
        for (int a = 0; a < C; ++a) {
          T s2 = T(0);
#pragma unroll
          for (int k = 0; k < C; ++k) s2 += kr[s][a * C + k] * xw[k];
          acc[a] -= T(1) * s2;
        }
      }
#pragma unroll
      for (int a = 0; a < C; ++a) {
        T z = T(0);
#pragma unroll
        for (int k = 0; k < C; ++k) z += Di[a * C + k] * acc[k];
        const T dn = fma(c2a, z, T(0) * T(0));
        sh[bb][0][threadIdx.x][a] = x2o[a] + dn;
        sh[bb][1][threadIdx.x][a] = x2o[a];
      }
    };
    // x4 of the interior from x3 in LDS
    auto phase2 = [&](int c, int bb) {
      if (!inner) return;
      T acc[C];
#pragma unroll
      for (int a = 0; a < C; ++a) acc[a] = sh[bb][2][threadIdx.x][a];
#pragma unroll
      for (int s = 0; s < W; ++s) {
        T xw[C];
#pragma unroll
        for (int k = 0; k < C; ++k) xw[k] = sh[bb][0][ls[s]][k];
#pragma unroll
        for (int a = 0; a < C; ++a) {
          T s2 = T(0);
#pragma unroll
          for (int k = 0; k < C; ++k) s2 += kr[s][a * C + k] * xw[k];
          acc[a] -= T(1) * s2;
        }
      }
#pragma unroll
      for (int a = 0; a < C; ++a) {
        T z = T(0);
#pragma unroll
        for (int k = 0; k < C; ++k) z += Di[a * C + k] * acc[k];
        const T x3 = sh[bb][0][threadIdx.x][a];
        const T dp = x3 - sh[bb][1][threadIdx.x][a];
        const T dn = fma(c2b, z, c1b * dp);
        if constexpr (UPD) {
          const ColDesc cd = cols[c];
          double out[D1];
#pragma unroll
          for (int k = 0; k < DIM; ++k) out[k] = xold[k] + omega * zun[k];
          out[DIM] = xold[DIM] + omega * double(x3 + dn);
#pragma unroll
          for (int k = 0; k < D1; ++k) gst(cd.xout + size_t(v) * D1 + k, out[k]);
          if (cd.xout2)
#pragma unroll
            for (int k = 0; k < D1; ++k) gst(cd.xout2 + size_t(v) * D1 + k, out[k]);
        } else {
          x4[size_t(c) * stride + size_t(v) * C + a] = x3 + dn;
        }
      }
    };
    // UPD: the copy's padding nodes, by the workgroups of its first patch
    auto padding = [&](int c) {
      if constexpr (UPD) {
        if (one || patch != 0) return;
        const int p0 = base + m * m, p1 = L.cbase[cp + 1];
        const ColDesc cd = cols[c];
        for (int u = p0 + int(threadIdx.x); u < p1; u += kBlock) {
          double out[D1];
#pragma unroll
          for (int k = 0; k < DIM; ++k)
            out[k] = gld(cd.xcur + size_t(u) * D1 + k) + omega * double(zu[(size_t(c) * nn + u) * DIM + k]);
          out[DIM] = gld(cd.xcur + size_t(u) * D1 + DIM) + omega * double(T(0));
#pragma unroll
          for (int k = 0; k < D1; ++k) gst(cd.xout + size_t(u) * D1 + k, out[k]);
          if (cd.xout2)
#pragma unroll
            for (int k = 0; k < D1; ++k) gst(cd.xout2 + size_t(u) * D1 + k, out[k]);
        }
      }
    };
    // prologue: x2 and x3 of the first column; then per column, x2 of the next
    // column with x4 of this one, and after a barrier x3 of the next column
    phase0_load(cbeg);
    phase0_store();
    __syncthreads();
    phase1(cbeg, buf);
#pragma unroll 1
    for (int c = cbeg; c < cend; ++c) {
      lds_barrier();
      const bool more = c + 1 < cend;
      if (more) phase0_load(c + 1);
      phase2(c, buf);
      padding(c);
      if (more) phase0_store();
      lds_barrier();
      if (more) phase1(c + 1, buf ^ 1);
      buf ^= 1;
    }
  }
}

// xout = xin + P xc (P1 interpolation, masked) for a group of columns; the
// parents of the node are found once and reused for every column
template <int DIM, int C, typename T>
__global__ __launch_bounds__(kBlock) void k_prolong(LevelView<T> Lf, LevelView<T> Lc, int isA,
                                                    const T* __restrict__ xin,
                                                    const T* __restrict__ xc,
                                                    T* __restrict__ xout, int nc) {
  const int nn = Lf.nn;
  for_each_piece(num_node_blocks(Lf.nact), nc, [&](int nblk, int cbeg, int cend) {
    const int cp = block_copy(Lf, nblk);
    if (Lf.act) active_cols(Lf, cp, cbeg, cend);
    const int v = nblk * kBlock + threadIdx.x;
    if (v >= Lf.nact || cbeg >= cend) return;
    int p0, p1;
    unsigned pm;
    prolong_parents<DIM, C>(Lf, Lc, isA ? 0 : DIM, cp, v, p0, p1, pm);
    const T wt = (pm >> (2 * C)) ? T(0.5) : T(1);
    const size_t stride = size_t(nn) * C, cstride = size_t(Lc.nn) * C;
#pragma unroll 2
    for (int c = cbeg; c < cend; ++c) {
      // all loads first (p0, p1 are valid nodes even when masked), then the
      // masked sums
      T xv[C], c0[C], c1[C];
#pragma unroll
      for (int a = 0; a < C; ++a) {
        xv[a] = xin[size_t(c) * stride + size_t(v) * C + a];
        c0[a] = xc[size_t(c) * cstride + size_t(p0) * C + a];
        c1[a] = xc[size_t(c) * cstride + size_t(p1) * C + a];
      }
#pragma unroll
      for (int a = 0; a < C; ++a) {
        T x = xv[a];
        if ((pm >> a) & 1u) x += wt * c0[a];
        if ((pm >> (C + a)) & 1u) x += wt * c1[a];
        xout[size_t(c) * stride + size_t(v) * C + a] = x;
      }
    }
  });
}

// r = b - K x on one level
template <int DIM, int C, typename T>
__global__ __launch_bounds__(kBlock) void k_level_residual(LevelView<T> L, int isA,
                                                           const T* __restrict__ b,
                                                           const T* __restrict__ x,
                                                           T* __restrict__ r, int nc) {
  // columns per iteration: two when the row stays in registers; otherwise (3D
  // displacement) the row is re-read from the caches once per group of eight
  // FP64 or four FP32 columns (measured on the 40^3 cube: in FP32 the smaller
  // group's higher occupancy outweighs the extra row reads)
  constexpr int W = DIM == 2 ? 7 : 15;
  constexpr bool STAT = W * C * C <= 64;
  constexpr int NQ = STAT ? 2 : (sizeof(T) == 4 ? 4 : 8);
  constexpr int RS = STAT ? W : 1;
  constexpr int SU = STAT ? W : 3;  // slot-loop unrolling (full when the row is in registers)
  const int nn = L.nn;
  for_each_piece<!STAT>(num_node_blocks(L.nact), nc, [&](int nblk, int cbeg, int cend) {
    if (L.act) active_cols(L, L.bcopy[nblk], cbeg, cend);
    const int v = nblk * kBlock + threadIdx.x;
    if (v >= L.nact || cbeg >= cend) return;
    const T* K = isA ? L.A : L.S;
    const size_t stride = size_t(nn) * C;
    int nb[RS];
    if constexpr (STAT) {
#pragma unroll
      for (int s = 0; s < W; ++s) nb[s] = L.nbr[size_t(s) * nn + v];
    }
    T kr[RS][C * C];
    if constexpr (STAT) {
#pragma unroll
      for (int s = 0; s < W; ++s)
#pragma unroll
        for (int e = 0; e < C * C; ++e) kr[s][e] = K[(size_t(s) * C * C + e) * nn + v];
    }
#pragma unroll 1
    for (int c = cbeg; c < cend; c += NQ) {
      // columns past the end of the run repeat the last one (computed, not stored)
      int cc[NQ];
#pragma unroll
      for (int q = 0; q < NQ; ++q) cc[q] = min(c + q, cend - 1);
      T acc[NQ][C];
#pragma unroll
      for (int q = 0; q < NQ; ++q)
#pragma unroll
        for (int a = 0; a < C; ++a) acc[q][a] = b[size_t(cc[q]) * stride + size_t(v) * C + a];
#pragma unroll SU
      for (int s = 0; s < W; ++s) {
        const int w = STAT ? nb[s] : L.nbr[size_t(s) * nn + v];
        T blk[C * C];
#pragma unroll
        for (int e = 0; e < C * C; ++e) {
          if constexpr (STAT) blk[e] = kr[s][e];
          else blk[e] = K[(size_t(s) * C * C + e) * nn + v];
        }
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
#pragma unroll
          for (int a = 0; a < C; ++a) {
            T s2 = T(0);
#pragma unroll
            for (int k = 0; k < C; ++k) s2 += blk[a * C + k] * x[size_t(cc[q]) * stride + size_t(w) * C + k];
            acc[q][a] -= s2;
          }
        }
      }
#pragma unroll
      for (int q = 0; q < NQ; ++q) {
        if (c + q >= cend) break;
#pragma unroll
        for (int a = 0; a < C; ++a) r[size_t(cc[q]) * stride + size_t(v) * C + a] = acc[q][a];
      }
    }
  });
}

// coarse b = P' r_fine (P1 interpolation transpose, masked)
template <int DIM, int C, typename T>
__global__ __launch_bounds__(kBlock) void k_restrict(LevelView<T> Lf, LevelView<T> Lc, int isA,
                                                     const T* __restrict__ rf,
                                                     T* __restrict__ bc, int nc) {
  constexpr int W = DIM == 2 ? 7 : 15;
  const int I = blockIdx.y * kBlock + threadIdx.x;
  const int c = blockIdx.x;
  const int cp = block_copy(Lc, blockIdx.y);
  if (I >= Lc.nact || !col_active(Lc, cp, c)) return;
  const int ccl = copy_cells(Lc, cp);
  const int mc = ccl + 1, mf = copy_cells(Lf, cp) + 1;
  const int lI = I - copy_base(Lc, cp);  // node within the copy
  const bool real = lI < grid_nodes<DIM>(ccl);
  const int fbase = copy_base(Lf, cp);
  int ci = 0, cj = 0, ck = 0;
  if (real) node_coords<DIM>(lI, mc, ci, cj, ck);
  const uint8_t fc = Lc.fixed[I];
  const int bit0 = isA ? 0 : DIM;
  const size_t sf = size_t(Lf.nn) * C, sc = size_t(Lc.nn) * C;
  // fine node under each slot (a missing one is replaced by the copy's first
  // node and masked out); every load is issued before the masked sums
  int fs[W];
  unsigned ok = 0u;
#pragma unroll
  for (int s = 0; s < W; ++s) {
    const int* o = DIM == 2 ? c_off2[s] : c_off3[s];
    const int fi = 2 * ci + o[0], fj = 2 * cj + o[1], fk = 2 * ck + o[2];
    const bool in = real && fi >= 0 && fi < mf && fj >= 0 && fj < mf && fk >= 0 && fk < mf;
    fs[s] = fbase + (in ? node_id<DIM>(fi, fj, fk, mf) : 0);
    ok |= unsigned(in) << s;
  }
  unsigned ff[W];
  T rv[W][C];
#pragma unroll
  for (int s = 0; s < W; ++s) {
    ff[s] = Lf.fixed[fs[s]];
#pragma unroll
    for (int a = 0; a < C; ++a) rv[s][a] = rf[size_t(c) * sf + size_t(fs[s]) * C + a];
  }
  T acc[C];
#pragma unroll
  for (int a = 0; a < C; ++a) acc[a] = T(0);
#pragma unroll
  for (int s = 0; s < W; ++s) {
    if (!((ok >> s) & 1u)) continue;
    const T wgt = s == 0 ? T(1) : T(0.5);
#pragma unroll
    for (int a = 0; a < C; ++a)
      if (!((ff[s] >> (bit0 + a)) & 1u)) acc[a] += wgt * rv[s][a];
  }
#pragma unroll
  for (int a = 0; a < C; ++a) {
    if ((fc >> (bit0 + a)) & 1) acc[a] = T(0);
    bc[size_t(c) * sc + size_t(I) * C + a] = acc[a];
  }
}

// ---------------------------------------------------------------------------
// The coarse end of a V-cycle in one launch: levels t..last of the hierarchy
// for one column per workgroup, every vector in LDS.  The steps are exactly
// those of the per-level kernels (k_cheb with its folded first step and
// recovered increments, k_level_residual, k_restrict, k_coarse_solve,
// k_prolong), in the same order and with the same summation order, so the
// result is the same as running them one launch at a time; only the launches
// (each a few microseconds on a level of a few hundred nodes) are saved.
// ---------------------------------------------------------------------------
namespace tail {

// workgroup size of the fused tail for a few columns: the levels are small, so
// a phase is one or two nodes per thread and its cost is the latency of the
// operator loads; more threads keep more of them in flight (3D rows need the
// registers of 256).  Launches of many workgroups (batches) take fewer threads
// (kTailSmallBlock).
template <int DIM>
constexpr int block() { return DIM == 2 ? 1024 : 256; }

// All routines work on one copy of the grid (one sample of a batch): `base`
// is the copy's first node in the level's arrays; LDS vectors hold only the
// copy's grid nodes (local numbering).

// One Chebyshev step xout = xin + d, d <- c1 dp + c2 D^{-1}(b - K xin), with
// the previous increment dp and the storing of d chosen as in k_cheb:
//   first: the step after the (unstored) first step from zero, xin formed as
//          it D^{-1} b through the folded operators, dp = xin;
//   dx = 2: dp = xin - xout at the node (xout holds the previous step's input
//          and is overwritten in place);
//   else dp = d (when c1 != 0); wd: store d.
template <int DIM, int C, bool FIRST, typename T, int BS>
__device__ inline void cheb(const LevelView<T>& L, int base, int nreal, const T* b, const T* xin,
                            T* xout, T* d, T c1, T c2, T it, int dx, bool wd) {
  constexpr bool first = FIRST;
  constexpr int W = DIM == 2 ? 7 : 15;
  const T* K = first ? (C > 1 ? L.AD : L.SD) : (C > 1 ? L.A : L.S);
  const T* Dg = C > 1 ? L.Ainv : L.Sinv;
  const T* src = first ? b : xin;
  const T sc = first ? it : T(1);
  const int nn = L.nn;
  for (int v = threadIdx.x; v < nreal; v += BS) {
    const int g = base + v;
    T acc[C], xs[C];
#pragma unroll
    for (int a = 0; a < C; ++a) acc[a] = b[v * C + a];
#pragma unroll
    for (int s = 0; s < W; ++s) {
      const int w = L.nbr[size_t(s) * nn + g] - base;
      T xw[C];
#pragma unroll
      for (int k = 0; k < C; ++k) xw[k] = src[w * C + k];
      if (s == 0) {
#pragma unroll
        for (int a = 0; a < C; ++a) {
          if (first) {
            T z = T(0);
#pragma unroll
            for (int k = 0; k < C; ++k) z += Dg[size_t(a * C + k) * nn + g] * xw[k];
            xs[a] = z * it;
          } else {
            xs[a] = xw[a];
          }
        }
      }
#pragma unroll
      for (int a = 0; a < C; ++a) {
        T s2 = T(0);
#pragma unroll
        for (int k = 0; k < C; ++k) s2 += K[(size_t(s) * C * C + a * C + k) * nn + g] * xw[k];
        acc[a] -= sc * s2;
      }
    }
#pragma unroll
    for (int a = 0; a < C; ++a) {
      T z = T(0);
#pragma unroll
      for (int k = 0; k < C; ++k) z += Dg[size_t(a * C + k) * nn + g] * acc[k];
      const T dp = c1 == T(0) ? T(0) : first ? xs[a] : dx == 2 ? xs[a] - xout[v * C + a] : d[v * C + a];
      const T dn = c1 * dp + c2 * z;
      if (wd) d[v * C + a] = dn;
      xout[v * C + a] = xs[a] + dn;
    }
  }
}

template <int DIM, int C, typename T, int BS>
__device__ inline void residual(const LevelView<T>& L, int base, int nreal, const T* b, const T* x,
                                T* r) {
  constexpr int W = DIM == 2 ? 7 : 15;
  const T* K = C > 1 ? L.A : L.S;
  const int nn = L.nn;
  for (int v = threadIdx.x; v < nreal; v += BS) {
    const int g = base + v;
    T acc[C];
#pragma unroll
    for (int a = 0; a < C; ++a) acc[a] = b[v * C + a];
#pragma unroll
    for (int s = 0; s < W; ++s) {
      const int w = L.nbr[size_t(s) * nn + g] - base;
#pragma unroll
      for (int a = 0; a < C; ++a) {
        T s2 = T(0);
#pragma unroll
        for (int k = 0; k < C; ++k) s2 += K[(size_t(s) * C * C + a * C + k) * nn + g] * x[w * C + k];
        acc[a] -= s2;
      }
    }
#pragma unroll
    for (int a = 0; a < C; ++a) r[v * C + a] = acc[a];
  }
}

// bc = P' rf (masked)
template <int DIM, int C, typename T, int BS>
__device__ inline void restrict_to(const LevelView<T>& Lf, int basef, int cellsf,
                                   const LevelView<T>& Lc, int basec, int cellsc, const T* rf,
                                   T* bc) {
  constexpr int W = DIM == 2 ? 7 : 15;
  const int mc = cellsc + 1, mf = cellsf + 1;
  const int bit0 = C > 1 ? 0 : DIM;
  const int nrc = grid_nodes<DIM>(cellsc);
  for (int I = threadIdx.x; I < nrc; I += BS) {
    int ci, cj, ck;
    node_coords<DIM>(I, mc, ci, cj, ck);
    T acc[C];
#pragma unroll
    for (int a = 0; a < C; ++a) acc[a] = T(0);
#pragma unroll
    for (int s = 0; s < W; ++s) {
      const int* o = DIM == 2 ? c_off2[s] : c_off3[s];
      const int fi = 2 * ci + o[0], fj = 2 * cj + o[1], fk = 2 * ck + o[2];
      if (fi < 0 || fi >= mf || fj < 0 || fj >= mf || fk < 0 || fk >= mf) continue;
      const int f = node_id<DIM>(fi, fj, fk, mf);
      const T wgt = s == 0 ? T(1) : T(0.5);
      const uint8_t ff = Lf.fixed[basef + f];
#pragma unroll
      for (int a = 0; a < C; ++a)
        if (!((ff >> (bit0 + a)) & 1)) acc[a] += wgt * rf[f * C + a];
    }
    const uint8_t fc = Lc.fixed[basec + I];
#pragma unroll
    for (int a = 0; a < C; ++a) {
      if ((fc >> (bit0 + a)) & 1) acc[a] = T(0);
      bc[I * C + a] = acc[a];
    }
  }
}

template <int DIM, int C, typename T, int BS>
__device__ inline void prolong(const LevelView<T>& Lf, int basef, int nrealf,
                               const LevelView<T>& Lc, int basec, int cp, const T* xin,
                               const T* xc, T* xout) {
  for (int v = threadIdx.x; v < nrealf; v += BS) {
    int p0, p1;
    unsigned pm;
    prolong_parents<DIM, C>(Lf, Lc, C > 1 ? 0 : DIM, cp, basef + v, p0, p1, pm);
    p0 -= basec;
    p1 -= basec;
    const T wt = (pm >> (2 * C)) ? T(0.5) : T(1);
#pragma unroll
    for (int a = 0; a < C; ++a) {
      T x = xin[v * C + a];
      if ((pm >> a) & 1u) x += wt * xc[p0 * C + a];
      if ((pm >> (C + a)) & 1u) x += wt * xc[p1 * C + a];
      xout[v * C + a] = x;
    }
  }
}

}  // namespace tail

// one workgroup per (column, copy); each copy runs its own tail levels
// t0..t0+nlev-1 (copies of a batch may be grids of different sizes)
template <int DIM, int C, typename T, int BS>
__global__ __launch_bounds__(BS) __attribute__((amdgpu_waves_per_eu(DIM == 2 ? 4 : 1)))
void k_vcycle_tail(TailDev<T> TD) {
  extern __shared__ double tail_raw[];
  T* lds = reinterpret_cast<T*>(tail_raw);
  __shared__ int s_nr[kTailMaxLevels], s_base[kTailMaxLevels], s_cells[kTailMaxLevels],
      s_off[kTailMaxLevels];
  const int copies = TD.copies;
  const int c = blockIdx.x / copies, cp = TD.cp0 + (blockIdx.x - c * copies);
  const TailCopy* tcp = TD.tc + cp;
  const int t0 = tcp->t0, nl = tcp->nlev;  // the last one is solved densely
  if (!col_active(TD.L[t0], cp, c)) return;  // past this sample's steps
  if (threadIdx.x < nl) {
    const LevelView<T>& Li = TD.L[t0 + threadIdx.x];
    s_cells[threadIdx.x] = Li.ccells[cp];
    s_nr[threadIdx.x] = grid_nodes<DIM>(Li.ccells[cp]);
    s_base[threadIdx.x] = Li.cbase[cp];
    s_off[threadIdx.x] = tcp->off[threadIdx.x];
  }
  __syncthreads();
  const int deg = TD.degree;
  // level i's LDS block at s_off[i]: b, two iterates (the free one also holds
  // the residual) and, for degree > 2, d (coarsest: b, x), each s_nr[i] * C
  // values; bit i of `alt` set when level i's current iterate is the second
  auto vec = [&](int i, int k) { return lds + s_off[i] + k * s_nr[i] * C; };
  T* const dnull = nullptr;
  unsigned alt = 0;
  const int n0 = s_nr[0] * C;
  const size_t g0 = (size_t(c) * TD.L[t0].nn + s_base[0]) * C;
  const T* b_t = TD.b[t0];
  for (int i = threadIdx.x; i < n0; i += BS) vec(0, 0)[i] = b_t[g0 + i];
  __syncthreads();
  // descend: pre-smoothing (its first step folded into the second), residual
  // into the free iterate, restriction
  for (int i = 0; i + 1 < nl; ++i) {
    const LevelView<T>& L = TD.L[t0 + i];
    const double theta = TD.theta[t0 + i], delta = TD.delta[t0 + i], sigma = TD.sigma[t0 + i];
    T* d = deg > 2 ? vec(i, 3) : dnull;
    int xi = 1;
    double rho = 1.0 / sigma;
    for (int j = 2; j <= deg; ++j) {
      const double rn = 1.0 / (2.0 * sigma - rho);
      const bool first = j == 2;
      if (first)
        tail::cheb<DIM, C, true, T, BS>(L, s_base[i], s_nr[i], vec(i, 0), vec(i, xi), vec(i, 1),
                                        d, T(rn * rho), T(2.0 * rn / delta), T(1.0 / theta), 0,
                                        j < deg);
      else
        tail::cheb<DIM, C, false, T, BS>(L, s_base[i], s_nr[i], vec(i, 0), vec(i, xi),
                                         vec(i, 3 - xi), d, T(rn * rho), T(2.0 * rn / delta), T(0),
                                         0, j < deg);
      __syncthreads();
      rho = rn;
      if (!first) xi = 3 - xi;
    }
    if (xi == 2) alt |= 1u << i;
    tail::residual<DIM, C, T, BS>(L, s_base[i], s_nr[i], vec(i, 0), vec(i, xi), vec(i, 3 - xi));
    __syncthreads();
    tail::restrict_to<DIM, C, T, BS>(L, s_base[i], s_cells[i], TD.L[t0 + i + 1], s_base[i + 1],
                                     s_cells[i + 1], vec(i, 3 - xi), vec(i + 1, 0));
    __syncthreads();
  }
  // coarsest level: dense inverse of this copy
  {
    const int n = s_nr[nl - 1] * C;
    const T* bb = vec(nl - 1, 0);
    T* xx = vec(nl - 1, 1);
    const T* M = TD.Minv + tcp->moff;
    for (int r = threadIdx.x; r < n; r += BS) {
      T acc = T(0);
      const T* row = M + size_t(r) * n;
      for (int j = 0; j < n; ++j) acc += row[j] * bb[j];
      xx[r] = acc;
    }
    __syncthreads();
  }
  // ascend: coarse-grid correction into the free iterate, then the
  // post-smoothing steps (the second recovers the first one's increment from
  // the buffer it overwrites)
  for (int i = nl - 2; i >= 0; --i) {
    const LevelView<T>& L = TD.L[t0 + i];
    const double theta = TD.theta[t0 + i], delta = TD.delta[t0 + i], sigma = TD.sigma[t0 + i];
    T* d = deg > 2 ? vec(i, 3) : dnull;
    int xi = ((alt >> i) & 1u) ? 2 : 1;
    const int xci = (i + 2 == nl) ? 1 : (((alt >> (i + 1)) & 1u) ? 2 : 1);
    tail::prolong<DIM, C, T, BS>(L, s_base[i], s_nr[i], TD.L[t0 + i + 1], s_base[i + 1], cp,
                                 vec(i, xi), vec(i + 1, xci), vec(i, 3 - xi));
    __syncthreads();
    xi = 3 - xi;
    double rho = 1.0 / sigma;
    for (int j = 1; j <= deg; ++j) {
      double c1 = 0.0, c2 = 1.0 / theta, rn = rho;
      if (j > 1) {
        rn = 1.0 / (2.0 * sigma - rho);
        c1 = rn * rho;
        c2 = 2.0 * rn / delta;
      }
      tail::cheb<DIM, C, false, T, BS>(L, s_base[i], s_nr[i], vec(i, 0), vec(i, xi),
                                       vec(i, 3 - xi), d, T(c1), T(c2), T(0), j == 2 ? 2 : 0,
                                       j > 1 && j < deg);
      __syncthreads();
      rho = rn;
      xi = 3 - xi;
    }
    alt = (alt & ~(1u << i)) | (xi == 2 ? 1u << i : 0u);
  }
  const T* res = vec(0, ((alt & 1u) ? 2 : 1));
  T* x_t = TD.x[t0];
  for (int i = threadIdx.x; i < n0; i += BS) x_t[g0 + i] = res[i];
  // padding nodes of the copy keep a zero correction
  const int npad = (TD.L[t0].cbase[cp + 1] - s_base[0] - s_nr[0]) * C;
  for (int i = threadIdx.x; i < npad; i += BS) x_t[g0 + n0 + i] = T(0);
}

// coarsest level: x = M^{-1} b with the dense inverses (row-major, one per
// copy).  A workgroup stages the right-hand sides of NCB columns of one copy in
// LDS ([NCB][n]); each of its waves takes kCoarseRows rows, its lanes striding
// over j (consecutive addresses of a row), and sums each product over the
// lanes in a fixed tree.  Grid (row blocks of 4 kCoarseRows, column groups,
// copies).  n = grid dofs of a copy, stride = dofs of a copy with padding,
// copies of a column contiguous; the padding dofs are set to zero.
constexpr int kCoarseRows = 4;
template <int NCB, typename T>
__global__ __launch_bounds__(kBlock) void k_coarse_solve(int n, int stride, int copies, int nc,
                                                         const T* __restrict__ Minv,
                                                         const T* __restrict__ b,
                                                         T* __restrict__ x) {
  constexpr int R = kCoarseRows;
  extern __shared__ double sb_raw[];
  T* sb = reinterpret_cast<T*>(sb_raw);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int cp = blockIdx.z, c0 = blockIdx.y * NCB;
  const int ncb = min(NCB, nc - c0);
  const T* M = Minv + size_t(cp) * n * n;
#pragma unroll
  for (int q = 0; q < NCB; ++q) {
    // columns past the end stage zeros (computed, not stored)
    const size_t base = (size_t(c0 + min(q, ncb - 1)) * copies + cp) * stride;
    for (int i = threadIdx.x; i < n; i += kBlock) sb[q * n + i] = q < ncb ? b[base + i] : T(0);
  }
  __syncthreads();
  const int r0 = (blockIdx.x * (kBlock / 64) + wave) * R;
  const T* row[R];
#pragma unroll
  for (int k = 0; k < R; ++k) row[k] = M + size_t(min(r0 + k, n - 1)) * n;  // past the end: not stored
  T acc[R][NCB];
#pragma unroll
  for (int k = 0; k < R; ++k)
#pragma unroll
    for (int q = 0; q < NCB; ++q) acc[k][q] = T(0);
#pragma unroll 2
  for (int j = lane; j < n; j += 64) {
    T bv[NCB];
#pragma unroll
    for (int q = 0; q < NCB; ++q) bv[q] = sb[q * n + j];
#pragma unroll
    for (int k = 0; k < R; ++k) {
      const T m = row[k][j];
#pragma unroll
      for (int q = 0; q < NCB; ++q) acc[k][q] += m * bv[q];
    }
  }
#pragma unroll
  for (int k = 0; k < R; ++k)
#pragma unroll
    for (int q = 0; q < NCB; ++q) {
      T v = acc[k][q];
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
      if (lane == 0 && r0 + k < n && q < ncb) x[(size_t(c0 + q) * copies + cp) * stride + r0 + k] = v;
    }
  if (blockIdx.x == 0)
    for (int q = 0; q < ncb; ++q)
      for (int i = n + threadIdx.x; i < stride; i += kBlock)
        x[(size_t(c0 + q) * copies + cp) * stride + i] = T(0);
}

// pressure stage of P1: t = B' z_u - r_p (P2: t = -r_p), the right-hand side
// of the pressure V-cycle
template <int DIM, typename T>
__global__ __launch_bounds__(kBlock) void k_pstage(LevelView<T> L, const T* __restrict__ Bt,
                                                   int p1, const T* __restrict__ zu,
                                                   const T* __restrict__ rp,
                                                   T* __restrict__ t_out, int nc) {
  // one column per iteration (the Bt row stays in registers; two per
  // iteration measured 44.5 against 40.8 us per level-0 launch)
  constexpr int NQ = 1;
  constexpr int W = DIM == 2 ? 7 : 15;
  const int nn = L.nn;
  for_each_piece(num_node_blocks(L.nact), nc, [&](int nblk, int cbeg, int cend) {
    if (L.act) active_cols(L, L.bcopy[nblk], cbeg, cend);
    const int v = nblk * kBlock + threadIdx.x;
    if (v >= L.nact || cbeg >= cend) return;
    int nb[W];
    T bt[W][DIM];
#pragma unroll
    for (int s = 0; s < W; ++s) {
      nb[s] = L.nbr[size_t(s) * nn + v];
#pragma unroll
      for (int k = 0; k < DIM; ++k) bt[s][k] = p1 ? Bt[(size_t(s) * DIM + k) * nn + v] : T(0);
    }
#pragma unroll 1
    for (int c = cbeg; c < cend; c += NQ) {
      // columns past the end of the run repeat the last one (computed, not stored)
      int cc[NQ];
#pragma unroll
      for (int q = 0; q < NQ; ++q) cc[q] = min(c + q, cend - 1);
      T acc[NQ];
#pragma unroll
      for (int q = 0; q < NQ; ++q) acc[q] = -rp[size_t(cc[q]) * nn + v];
      if (p1) {
        // all neighbour loads first: left to itself the compiler interleaves
        // them with the sums (to stay within the registers of 8 waves per
        // SIMD), one load in flight at a time (35.7 against 43.4 us per
        // level-0 launch of 64 columns)
        T z[W][NQ][DIM];
#pragma unroll
        for (int s = 0; s < W; ++s)
#pragma unroll
          for (int q = 0; q < NQ; ++q) {
            const size_t base = size_t(cc[q]) * nn * DIM + size_t(nb[s]) * DIM;
#pragma unroll
            for (int k = 0; k < DIM; ++k) z[s][q][k] = zu[base + k];
          }
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int s = 0; s < W; ++s)
#pragma unroll
          for (int q = 0; q < NQ; ++q)
#pragma unroll
            for (int k = 0; k < DIM; ++k) acc[q] += bt[s][k] * z[s][q][k];
      }
#pragma unroll
      for (int q = 0; q < NQ; ++q) {
        if (c + q >= cend) break;
        t_out[size_t(cc[q]) * nn + v] = acc[q];
      }
    }
  });
}

// X^{n,m} = X^{n,m-1} + omega [z_u; z_p]   (used when the coarsest level is 0)
template <int DIM, typename T>
__global__ __launch_bounds__(kBlock) void k_update(int nn, const ColDesc* __restrict__ cols,
                                                   const T* __restrict__ zu,
                                                   const T* __restrict__ zp, double omega,
                                                   const int32_t* __restrict__ csteps,
                                                   const int32_t* __restrict__ bcopy) {
  constexpr int D1 = DIM + 1;
  const int v = blockIdx.y * kBlock + threadIdx.x;
  if (v >= nn) return;
  const int c = blockIdx.x;
  if (csteps && cols[c].step > csteps[bcopy[blockIdx.y]]) return;  // past the sample's steps
  const double* xc = cols[c].xcur;
  double* xo = cols[c].xout;
  double* xo2 = cols[c].xout2;
  double out[D1];
#pragma unroll
  for (int a = 0; a < DIM; ++a)
    out[a] = xc[size_t(v) * D1 + a] + omega * double(zu[(size_t(c) * nn + v) * DIM + a]);
  out[DIM] = xc[size_t(v) * D1 + DIM] + omega * double(zp[size_t(c) * nn + v]);
#pragma unroll
  for (int a = 0; a < D1; ++a) xo[size_t(v) * D1 + a] = out[a];
  if (xo2)
#pragma unroll
    for (int a = 0; a < D1; ++a) xo2[size_t(v) * D1 + a] = out[a];
}

// per-column sums of the block partials in a fixed order
__global__ __launch_bounds__(kBlock) void k_reduce_norms(const double* __restrict__ partials,
                                                         const int32_t* __restrict__ cbase,
                                                         int copies, int pstride,
                                                         double* __restrict__ norms) {
  __shared__ double lds[16];
  const int c = blockIdx.x / copies, cp = blockIdx.x - c * copies;
  double q[4] = {0.0, 0.0, 0.0, 0.0};
  const int b0 = cbase[cp] / kBlock, b1 = (cbase[cp + 1] + kBlock - 1) / kBlock;
  for (int b = b0 + threadIdx.x; b < b1; b += kBlock)
#pragma unroll
    for (int k = 0; k < 4; ++k) q[k] += partials[(size_t(c) * pstride + b) * 4 + k];
  block_sum<4>(q, lds);
  if (threadIdx.x == 0)
#pragma unroll
    for (int k = 0; k < 4; ++k) norms[(size_t(c) * copies + cp) * 4 + k] = q[k];
}

// Y = AA X (diagnostic path)
template <int DIM>
__global__ __launch_bounds__(kBlock) void k_apply_operator(LevelDev L, FineDev F,
                                                           const double* __restrict__ X,
                                                           double* __restrict__ Y) {
  constexpr int D1 = DIM + 1;
  const int nn = L.nn;
  const int v = blockIdx.y * kBlock + threadIdx.x;
  if (v >= nn) return;
  const int c = blockIdx.x;
  const double* x = X + size_t(c) * nn * D1;
  double yu[DIM] = {}, yp = 0.0;
  for (int s = 0; s < L.W; ++s) {
    const int w = L.nbr[size_t(s) * nn + v];
    double xw[D1];
#pragma unroll
    for (int k = 0; k < D1; ++k) xw[k] = x[size_t(w) * D1 + k];
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
      double acc = F.B[(size_t(s) * DIM + a) * nn + v] * xw[DIM];
#pragma unroll
      for (int b = 0; b < DIM; ++b) acc += L.A[(size_t(s) * DIM * DIM + a * DIM + b) * nn + v] * xw[b];
      yu[a] += acc;
    }
    double acc = -L.S[size_t(s) * nn + v] * xw[DIM];
#pragma unroll
    for (int a = 0; a < DIM; ++a) acc += F.Bt[(size_t(s) * DIM + a) * nn + v] * xw[a];
    yp += acc;
  }
  double* y = Y + size_t(c) * nn * D1;
#pragma unroll
  for (int a = 0; a < DIM; ++a) y[size_t(v) * D1 + a] = yu[a];
  y[size_t(v) * D1 + DIM] = yp;
}

template <int DIM, typename T>
__global__ __launch_bounds__(kBlock) void k_unpack(int nn, const double* __restrict__ X,
                                                   T* __restrict__ ru, T* __restrict__ rp) {
  constexpr int D1 = DIM + 1;
  const int v = blockIdx.y * kBlock + threadIdx.x;
  if (v >= nn) return;
  const size_t c = blockIdx.x;
#pragma unroll
  for (int a = 0; a < DIM; ++a) ru[(c * nn + v) * DIM + a] = T(X[(c * nn + v) * D1 + a]);
  rp[c * nn + v] = T(X[(c * nn + v) * D1 + DIM]);
}

template <int DIM, typename T>
__global__ __launch_bounds__(kBlock) void k_pack(int nn, const T* __restrict__ zu,
                                                 const T* __restrict__ zp,
                                                 double* __restrict__ Z) {
  constexpr int D1 = DIM + 1;
  const int v = blockIdx.y * kBlock + threadIdx.x;
  if (v >= nn) return;
  const size_t c = blockIdx.x;
#pragma unroll
  for (int a = 0; a < DIM; ++a) Z[(c * nn + v) * D1 + a] = double(zu[(c * nn + v) * DIM + a]);
  Z[(c * nn + v) * D1 + DIM] = double(zp[c * nn + v]);
}

// zero n16 16-byte words (grid-stride)
__global__ __launch_bounds__(kBlock) void k_zero16(uint4* __restrict__ p, size_t n16) {
  const size_t stride = size_t(gridDim.x) * kBlock;
  for (size_t i = size_t(blockIdx.x) * kBlock + threadIdx.x; i < n16; i += stride)
    p[i] = make_uint4(0u, 0u, 0u, 0u);
}

// initial iterate of the forward trajectory with prescribed values: column
// blockIdx.x (step n) gets g^n = sum_k pcoef[n][k] pres[k] at the prescribed
// dofs and zero elsewhere; column 0 is x0 when given (else g^0 as above)
__global__ __launch_bounds__(kBlock) void k_init_traj(double* __restrict__ X, int nn, int D1,
                                                      const double* __restrict__ x0,
                                                      const double* __restrict__ pres,
                                                      const double* __restrict__ pcoef, int npres,
                                                      const uint8_t* __restrict__ fixed) {
  const int v = blockIdx.y * kBlock + threadIdx.x;
  if (v >= nn) return;
  const int n = blockIdx.x;
  const size_t nd = size_t(nn) * D1;
  double* out = X + size_t(n) * nd + size_t(v) * D1;
  const unsigned fx = fixed[v];
  for (int c = 0; c < D1; ++c) {
    double val = 0.0;
    if (n == 0 && x0) {
      val = x0[size_t(v) * D1 + c];
    } else if ((fx >> c) & 1u) {
      for (int k = 0; k < npres; ++k) val += pcoef[size_t(n) * npres + k] * pres[k * nd + size_t(v) * D1 + c];
    }
    out[c] = val;
  }
}

inline dim3 col_grid(int nc, int nn) { return dim3(nc, num_node_blocks(nn)); }

// Grid of a balanced launch (for_each_piece): one workgroup per resident
// workgroup slot of the device (compute units x the kernel's occupancy, or x
// `wpc` when wpc > 0), and no more than there are (node block, column) units.
// Occupancies are queried once per kernel and device and cached.
struct OccKey {
  const void* fn;
  int dev;
  bool operator==(const OccKey& o) const { return fn == o.fn && dev == o.dev; }
};
struct OccHash {
  size_t operator()(const OccKey& k) const {
    return std::hash<const void*>()(k.fn) ^ (size_t(k.dev) * 0x9E3779B97F4A7C15ull);
  }
};

// default cap on resident workgroups per CU of a balanced launch (measured on
// the 256^2 workload: 2, 3 and 4 give 487, 482 and 491 ms per solve)
constexpr int kDefaultMaxWgPerCu = 3;
// grids of the 3D level-0 residual and smoother launches: four workgroups per
// CU whatever the occupancy (two or three resident in FP64), i.e. smaller
// pieces of work (40^3 cube: 742 -> 707 ms per solve; the coarse levels and the
// level residual gain nothing)
constexpr int kWgPerCu3dFine = 4;

dim3 balanced_grid(const void* fn, int nn, int nc, int wpc, bool aligned = false) {
  static std::mutex mu;
  static std::unordered_map<OccKey, int, OccHash> occ;
  static std::unordered_map<int, int> cus;
  int dev = 0;
  (void)hipGetDevice(&dev);
  int per_cu = wpc, ncu = 0;
  {
    std::lock_guard<std::mutex> lock(mu);
    auto ic = cus.find(dev);
    if (ic == cus.end()) {
      int n = 0;
      if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n < 1) n = 256;
      ic = cus.emplace(dev, n).first;
    }
    ncu = ic->second;
    if (per_cu <= 0) {
      auto io = occ.find(OccKey{fn, dev});
      if (io == occ.end()) {
        int o = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&o, fn, kBlock, 0) != hipSuccess || o < 1) o = 1;
        io = occ.emplace(OccKey{fn, dev}, o).first;
      }
      // at most kDefaultMaxWgPerCu: light kernels reach high occupancy, but
      // more, smaller pieces re-read each node's operator row more often
      per_cu = std::min(io->second, kDefaultMaxWgPerCu);
    }
  }
  if (aligned) {  // one workgroup per (node block, run of columns)
    const int nblocks = num_node_blocks(nn);
    const int groups = std::max(1, std::min(nc, ncu * per_cu / nblocks));
    return dim3(unsigned(nblocks * groups));
  }
  const long units = long(num_node_blocks(nn)) * nc;
  return dim3(unsigned(std::max(1L, std::min(long(ncu) * per_cu, units))));
}

// Events armed by set_launch_events are recorded by the next balanced launch's
// own dispatch (kernel start and end), then disarmed.
thread_local hipEvent_t g_ev_start = nullptr, g_ev_stop = nullptr;

#define BIOT_LAUNCH_BALANCED(kern, nn, nc, wpc, st, ...)                                          \
  BIOT_LAUNCH_BALANCED_AL(kern, nn, nc, wpc, false, st, __VA_ARGS__)
#define BIOT_LAUNCH_BALANCED_AL(kern, nn, nc, wpc, aligned, st, ...)                              \
  do {                                                                                           \
    const dim3 grid_ = balanced_grid(reinterpret_cast<const void*>(kern), nn, nc, wpc, aligned); \
    if (g_ev_start) {                                                                            \
      hipExtLaunchKernelGGL(kern, grid_, dim3(kBlock), 0, st, g_ev_start, g_ev_stop, 0,          \
                            __VA_ARGS__);                                                        \
      g_ev_start = g_ev_stop = nullptr;                                                          \
    } else {                                                                                     \
      hipLaunchKernelGGL(kern, grid_, dim3(kBlock), 0, st, __VA_ARGS__);                         \
    }                                                                                            \
  } while (0)

// the same for a launch with a grid of its own
#define BIOT_LAUNCH_GRID(kern, grid, st, ...)                                                     \
  do {                                                                                           \
    if (g_ev_start) {                                                                            \
      hipExtLaunchKernelGGL(kern, grid, dim3(kBlock), 0, st, g_ev_start, g_ev_stop, 0,           \
                            __VA_ARGS__);                                                        \
      g_ev_start = g_ev_stop = nullptr;                                                          \
    } else {                                                                                     \
      hipLaunchKernelGGL(kern, grid, dim3(kBlock), 0, st, __VA_ARGS__);                          \
    }                                                                                            \
  } while (0)

// compute units of the current device
int num_cus() {
  static std::mutex mu;
  static std::unordered_map<int, int> cus;
  int dev = 0;
  (void)hipGetDevice(&dev);
  std::lock_guard<std::mutex> lock(mu);
  auto it = cus.find(dev);
  if (it == cus.end()) {
    int n = 0;
    if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n < 1)
      n = 256;
    it = cus.emplace(dev, n).first;
  }
  return it->second;
}

}  // namespace

void set_launch_events(hipEvent_t start, hipEvent_t stop) {
  g_ev_start = start;
  g_ev_stop = stop;
}

bool launch_events_armed() { return g_ev_start != nullptr; }

template <int DIM, bool ADJ, typename T>
static void residual_dispatch(const LevelDev& L, const FineDev& F, const ColDesc* cols, int nc,
                              T* ru, T* rp, double* partials, int pstride, int wpc,
                              hipStream_t st) {
  if (DIM == 3 && wpc <= 0) wpc = kWgPerCu3dFine;
  BIOT_LAUNCH_BALANCED_AL((k_residual<DIM, T, ADJ>), L.nact, nc, wpc, DIM == 3, st, L, F, cols, nc,
                          ru, rp, partials, pstride);
}

template <typename T>
void launch_residual(int dim, const LevelDev& L, const FineDev& F, const ColDesc* cols, int nc,
                     T* ru, T* rp, double* partials, int pstride, int wpc, bool adj,
                     hipStream_t st) {
  if (dim == 2) {
    if (adj) residual_dispatch<2, true, T>(L, F, cols, nc, ru, rp, partials, pstride, wpc, st);
    else residual_dispatch<2, false, T>(L, F, cols, nc, ru, rp, partials, pstride, wpc, st);
  } else {
    if (adj) residual_dispatch<3, true, T>(L, F, cols, nc, ru, rp, partials, pstride, wpc, st);
    else residual_dispatch<3, false, T>(L, F, cols, nc, ru, rp, partials, pstride, wpc, st);
  }
}

template <int DIM, int C, bool UPD, typename T>
static void cheb_dispatch(const LevelView<T>& L, bool is_A, const T* b, const T* xin, T* xout,
                          T* d, int nc, double c1, double c2, bool wd, int dx, bool first,
                          double it, const ColDesc* cols, const T* zu, double omega, int wpc,
                          bool fine, hipStream_t st) {
  constexpr bool aligned = DIM == 3 && C == 3;  // k_cheb's rows re-read per column group
  if (fine) {
    if (DIM == 3 && wpc <= 0) wpc = kWgPerCu3dFine;
    BIOT_LAUNCH_BALANCED_AL((k_cheb<DIM, C, UPD, true, T>), L.nact, nc, wpc, aligned, st, L,
                            int(is_A), b, xin, xout, d, nc, T(c1), T(c2), int(wd), dx, int(first),
                            T(it), cols, zu, omega);
  } else if constexpr (!UPD) {
    BIOT_LAUNCH_BALANCED_AL((k_cheb<DIM, C, UPD, false, T>), L.nact, nc, wpc, aligned, st, L,
                            int(is_A), b, xin, xout, d, nc, T(c1), T(c2), int(wd), dx, int(first),
                            T(it), cols, zu, omega);
  }
}

template <typename T>
void launch_cheb(int dim, int comps, const LevelView<T>& L, bool is_A, const T* b, const T* xin,
                 T* xout, T* d, int nc, double c1, double c2, bool wd, int dx, bool first,
                 double it, const ColDesc* upd, const T* zu, double omega, int wpc, bool fine,
                 hipStream_t st) {
  if (dim == 2) {
    if (comps == 1) {
      if (upd) cheb_dispatch<2, 1, true, T>(L, is_A, b, xin, xout, d, nc, c1, c2, wd, dx, first, it, upd, zu, omega, wpc, fine, st);
      else cheb_dispatch<2, 1, false, T>(L, is_A, b, xin, xout, d, nc, c1, c2, wd, dx, first, it, upd, zu, omega, wpc, fine, st);
    } else {
      cheb_dispatch<2, 2, false, T>(L, is_A, b, xin, xout, d, nc, c1, c2, wd, dx, first, it, upd, zu, omega, wpc, fine, st);
    }
  } else {
    if (comps == 1) {
      if (upd) cheb_dispatch<3, 1, true, T>(L, is_A, b, xin, xout, d, nc, c1, c2, wd, dx, first, it, upd, zu, omega, wpc, fine, st);
      else cheb_dispatch<3, 1, false, T>(L, is_A, b, xin, xout, d, nc, c1, c2, wd, dx, first, it, upd, zu, omega, wpc, fine, st);
    } else {
      cheb_dispatch<3, 3, false, T>(L, is_A, b, xin, xout, d, nc, c1, c2, wd, dx, first, it, upd, zu, omega, wpc, fine, st);
    }
  }
}

template <typename T>
void launch_post2(int comps, const LevelView<T>& L, const LevelView<T>& Lc, bool is_A, const T* b,
                  const T* xin, const T* xc, T* x4, int nc, double c2a, double c1b, double c2b,
                  const ColDesc* upd, const T* zu, double omega, int wpc, hipStream_t st) {
  const int patches = L.npatch;
  // runs per patch: as many as keep about one wave of resident workgroups
  // (3 per CU) busy, at most one per column
  const int resident = 3 * num_cus(), groups = std::max(1, std::min(nc, resident / patches));
  const int run = (nc + groups - 1) / groups;
  const dim3 grid(unsigned((patches * groups + 7) / 8 * 8));
  (void)wpc;
  if (upd)
    BIOT_LAUNCH_GRID((k_post2<1, true, T>), grid, st, L, Lc, int(is_A), b, xin, xc, x4, nc,
                     T(c2a), T(c1b), T(c2b), groups, run, upd, zu, omega);
  else if (comps == 1)
    BIOT_LAUNCH_GRID((k_post2<1, false, T>), grid, st, L, Lc, int(is_A), b, xin, xc, x4, nc,
                     T(c2a), T(c1b), T(c2b), groups, run, upd, zu, omega);
  else
    BIOT_LAUNCH_GRID((k_post2<2, false, T>), grid, st, L, Lc, int(is_A), b, xin, xc, x4, nc,
                     T(c2a), T(c1b), T(c2b), groups, run, upd, zu, omega);
}

template <typename T>
void launch_level_residual(int dim, int comps, const LevelView<T>& L, bool is_A, const T* b,
                           const T* x, T* r, int nc, int wpc, hipStream_t st) {
  if (dim == 2) {
    if (comps == 1) BIOT_LAUNCH_BALANCED((k_level_residual<2, 1, T>), L.nact, nc, wpc, st, L, int(is_A), b, x, r, nc);
    else BIOT_LAUNCH_BALANCED((k_level_residual<2, 2, T>), L.nact, nc, wpc, st, L, int(is_A), b, x, r, nc);
  } else {
    if (comps == 1) BIOT_LAUNCH_BALANCED((k_level_residual<3, 1, T>), L.nact, nc, wpc, st, L, int(is_A), b, x, r, nc);
    else BIOT_LAUNCH_BALANCED_AL((k_level_residual<3, 3, T>), L.nact, nc, wpc, true, st, L, int(is_A), b, x, r, nc);
  }
}

template <typename T>
void launch_restrict(int dim, int comps, const LevelView<T>& Lf, const LevelView<T>& Lc,
                     bool is_A, const T* rf, T* bc, int nc, hipStream_t st) {
  const dim3 g = col_grid(nc, Lc.nact);
  if (dim == 2) {
    if (comps == 1) hipLaunchKernelGGL((k_restrict<2, 1, T>), g, dim3(kBlock), 0, st, Lf, Lc, int(is_A), rf, bc, nc);
    else hipLaunchKernelGGL((k_restrict<2, 2, T>), g, dim3(kBlock), 0, st, Lf, Lc, int(is_A), rf, bc, nc);
  } else {
    if (comps == 1) hipLaunchKernelGGL((k_restrict<3, 1, T>), g, dim3(kBlock), 0, st, Lf, Lc, int(is_A), rf, bc, nc);
    else hipLaunchKernelGGL((k_restrict<3, 3, T>), g, dim3(kBlock), 0, st, Lf, Lc, int(is_A), rf, bc, nc);
  }
}

template <typename T>
void launch_prolong(int dim, int comps, const LevelView<T>& Lf, const LevelView<T>& Lc, bool is_A,
                    const T* xin, const T* xc, T* xout, int nc, int wpc, hipStream_t st) {
  if (dim == 2) {
    if (comps == 1) BIOT_LAUNCH_BALANCED((k_prolong<2, 1, T>), Lf.nact, nc, wpc, st, Lf, Lc, int(is_A), xin, xc, xout, nc);
    else BIOT_LAUNCH_BALANCED((k_prolong<2, 2, T>), Lf.nact, nc, wpc, st, Lf, Lc, int(is_A), xin, xc, xout, nc);
  } else {
    if (comps == 1) BIOT_LAUNCH_BALANCED((k_prolong<3, 1, T>), Lf.nact, nc, wpc, st, Lf, Lc, int(is_A), xin, xc, xout, nc);
    else BIOT_LAUNCH_BALANCED((k_prolong<3, 3, T>), Lf.nact, nc, wpc, st, Lf, Lc, int(is_A), xin, xc, xout, nc);
  }
}

template <typename T>
void launch_coarse_solve(int n, int stride, int copies, const T* Minv, const T* b, T* x, int nc,
                         hipStream_t st) {
  // columns per workgroup: as many as fit 64 KB of staged right-hand sides
  const size_t col_bytes = size_t(n) * sizeof(T);
  const int ncb = col_bytes * 8 <= 65536 ? 8 : col_bytes * 4 <= 65536 ? 4 : col_bytes * 2 <= 65536 ? 2 : 1;
  const int rows = (kBlock / 64) * kCoarseRows;
  const dim3 g((n + rows - 1) / rows, (nc + ncb - 1) / ncb, copies);
  const size_t lds = col_bytes * ncb;
  if (ncb == 8) hipLaunchKernelGGL((k_coarse_solve<8, T>), g, dim3(kBlock), lds, st, n, stride, copies, nc, Minv, b, x);
  else if (ncb == 4) hipLaunchKernelGGL((k_coarse_solve<4, T>), g, dim3(kBlock), lds, st, n, stride, copies, nc, Minv, b, x);
  else if (ncb == 2) hipLaunchKernelGGL((k_coarse_solve<2, T>), g, dim3(kBlock), lds, st, n, stride, copies, nc, Minv, b, x);
  else hipLaunchKernelGGL((k_coarse_solve<1, T>), g, dim3(kBlock), lds, st, n, stride, copies, nc, Minv, b, x);
}

int tail_vectors(int degree) { return degree > 2 ? 4 : 3; }

int tail_block_threads(int dim) { return dim == 2 ? tail::block<2>() : tail::block<3>(); }

// 2D tails launched with at least as many workgroups as compute units (a
// batch of samples) use workgroups of kTailSmallBlock threads: four of them
// are resident per compute unit, and fewer threads idle on the levels of a few
// hundred nodes (64-sample batch: 2.81 s against 3.03 s with 1024 threads,
// 2.87 s with 128 and 3.06 s with 64, whose LDS then limits residency)
constexpr int kTailSmallBlock = 256;

size_t tail_lds_bytes(const int* level_nn, int nlev, int comps, int tbytes, int degree) {
  size_t n = 0;
  for (int i = 0; i < nlev; ++i)
    n += size_t(level_nn[i]) * comps * (i + 1 < nlev ? tail_vectors(degree) : 2);
  return n * tbytes;
}

template <typename T>
void launch_vcycle_tail(int dim, int comps, const TailDev<T>& TD, int nc, size_t lds,
                        hipStream_t st) {
  const dim3 g(nc * TD.copies);
  if (dim == 2) {
    // a few columns: one workgroup of 1024 threads each, whose phases are
    // latency-bound; many (a batch of samples): kTailSmallBlock threads each
    if (int(g.x) >= num_cus()) {
      constexpr int bs = kTailSmallBlock;
      if (comps == 1) hipLaunchKernelGGL((k_vcycle_tail<2, 1, T, bs>), g, dim3(bs), lds, st, TD);
      else hipLaunchKernelGGL((k_vcycle_tail<2, 2, T, bs>), g, dim3(bs), lds, st, TD);
    } else {
      constexpr int bs = tail::block<2>();
      if (comps == 1) hipLaunchKernelGGL((k_vcycle_tail<2, 1, T, bs>), g, dim3(bs), lds, st, TD);
      else hipLaunchKernelGGL((k_vcycle_tail<2, 2, T, bs>), g, dim3(bs), lds, st, TD);
    }
  } else {
    constexpr int bs = tail::block<3>();
    if (comps == 1) hipLaunchKernelGGL((k_vcycle_tail<3, 1, T, bs>), g, dim3(bs), lds, st, TD);
    else hipLaunchKernelGGL((k_vcycle_tail<3, 3, T, bs>), g, dim3(bs), lds, st, TD);
  }
}

template <typename T>
void launch_pstage(int dim, const LevelView<T>& L, const T* Bt, bool p1, const T* zu, const T* rp,
                   T* t, int nc, int wpc, hipStream_t st) {
  if (dim == 2) BIOT_LAUNCH_BALANCED((k_pstage<2, T>), L.nact, nc, wpc, st, L, Bt, int(p1), zu, rp, t, nc);
  else BIOT_LAUNCH_BALANCED((k_pstage<3, T>), L.nact, nc, wpc, st, L, Bt, int(p1), zu, rp, t, nc);
}

template <typename T>
void launch_update(int dim, int nn, const ColDesc* cols, const T* zu, const T* zp, double omega,
                   int nc, const int32_t* csteps, const int32_t* bcopy, hipStream_t st) {
  const dim3 g = col_grid(nc, nn);
  if (dim == 2)
    hipLaunchKernelGGL((k_update<2, T>), g, dim3(kBlock), 0, st, nn, cols, zu, zp, omega, csteps, bcopy);
  else
    hipLaunchKernelGGL((k_update<3, T>), g, dim3(kBlock), 0, st, nn, cols, zu, zp, omega, csteps, bcopy);
}

template <typename T>
void launch_unpack(int dim, int nn, const double* X, T* ru, T* rp, int nc, hipStream_t st) {
  const dim3 g = col_grid(nc, nn);
  if (dim == 2) hipLaunchKernelGGL((k_unpack<2, T>), g, dim3(kBlock), 0, st, nn, X, ru, rp);
  else hipLaunchKernelGGL((k_unpack<3, T>), g, dim3(kBlock), 0, st, nn, X, ru, rp);
}

template <typename T>
void launch_pack(int dim, int nn, const T* zu, const T* zp, double* Z, int nc, hipStream_t st) {
  const dim3 g = col_grid(nc, nn);
  if (dim == 2) hipLaunchKernelGGL((k_pack<2, T>), g, dim3(kBlock), 0, st, nn, zu, zp, Z);
  else hipLaunchKernelGGL((k_pack<3, T>), g, dim3(kBlock), 0, st, nn, zu, zp, Z);
}

void launch_init_traj(double* X, int ncols, int nn, int D1, const double* x0, const double* pres,
                      const double* pcoef, int npres, const uint8_t* fixed, hipStream_t st) {
  hipLaunchKernelGGL(k_init_traj, col_grid(ncols, nn), dim3(kBlock), 0, st, X, nn, D1, x0, pres,
                     pcoef, npres, fixed);
}

void launch_zero(void* p, size_t bytes, hipStream_t st) {
  const size_t n16 = bytes / 16;
  if (n16 == 0) return;
  const unsigned grid = unsigned(std::min<size_t>((n16 + kBlock - 1) / kBlock, size_t(4096)));
  hipLaunchKernelGGL(k_zero16, dim3(grid), dim3(kBlock), 0, st, static_cast<uint4*>(p), n16);
}

void launch_reduce_norms(const double* partials, const int32_t* cbase, int copies, int pstride,
                         double* norms, int nc, hipStream_t st) {
  hipLaunchKernelGGL(k_reduce_norms, dim3(nc * copies), dim3(kBlock), 0, st, partials, cbase, copies,
                     pstride, norms);
}

void launch_apply_operator(int dim, const LevelDev& L, const FineDev& F, const double* X,
                           double* Y, int nc, hipStream_t st) {
  const dim3 g = col_grid(nc, L.nn);
  if (dim == 2) hipLaunchKernelGGL(k_apply_operator<2>, g, dim3(kBlock), 0, st, L, F, X, Y);
  else hipLaunchKernelGGL(k_apply_operator<3>, g, dim3(kBlock), 0, st, L, F, X, Y);
}

// explicit instantiations for the two preconditioner precisions
#define BIOT_INSTANTIATE(T)                                                                      \
  template void launch_residual<T>(int, const LevelDev&, const FineDev&, const ColDesc*, int, T*, \
                                   T*, double*, int, int, bool, hipStream_t);                    \
  template void launch_cheb<T>(int, int, const LevelView<T>&, bool, const T*, const T*, T*, T*,  \
                               int, double, double, bool, int, bool, double, const ColDesc*,     \
                               const T*, double, int, bool, hipStream_t);                         \
  template void launch_post2<T>(int, const LevelView<T>&, const LevelView<T>&, bool, const T*,  \
                                const T*, const T*, T*, int, double, double, double,              \
                                const ColDesc*, const T*, double, int, hipStream_t);              \
  template void launch_level_residual<T>(int, int, const LevelView<T>&, bool, const T*,          \
                                         const T*, T*, int, int, hipStream_t);                    \
  template void launch_restrict<T>(int, int, const LevelView<T>&, const LevelView<T>&, bool,     \
                                   const T*, T*, int, hipStream_t);                               \
  template void launch_prolong<T>(int, int, const LevelView<T>&, const LevelView<T>&, bool,      \
                                  const T*, const T*, T*, int, int, hipStream_t);                 \
  template void launch_coarse_solve<T>(int, int, int, const T*, const T*, T*, int, hipStream_t); \
  template void launch_vcycle_tail<T>(int, int, const TailDev<T>&, int, size_t, hipStream_t);     \
  template void launch_pstage<T>(int, const LevelView<T>&, const T*, bool, const T*, const T*,   \
                                 T*, int, int, hipStream_t);                                      \
  template void launch_update<T>(int, int, const ColDesc*, const T*, const T*, double, int,      \
                                 const int32_t*, const int32_t*, hipStream_t);                    \
  template void launch_unpack<T>(int, int, const double*, T*, T*, int, hipStream_t);             \
  template void launch_pack<T>(int, int, const T*, const T*, double*, int, hipStream_t);

BIOT_INSTANTIATE(double)
BIOT_INSTANTIATE(float)

}  // namespace biot
