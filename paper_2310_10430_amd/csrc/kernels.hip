// HIP kernels (gfx950) of the preconditioned inverted time-stepping sweep.
//
// Every kernel processes a batch of columns (time steps / iterations) at once.
// A thread owns one node and a tile of CT columns: the node's matrix blocks
// are loaded once per slot and applied to all CT columns, so the operator is
// read once per column tile while the column data streams through.  The grid
// is (column tiles, node blocks) with the column tile fastest, so the
// workgroups that share a node block -- and its matrix rows -- are dispatched
// back to back and hit in L2/MALL.
//
// Layouts (see setup.hpp): operator values [slot][entry][node]; state columns
// node-major [node][u_x, u_y, (u_z), p]; multigrid work vectors node-major
// [node][comp], one contiguous vector per column of the batch.
#include <hip/hip_runtime.h>

#include "kernels.hpp"

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

// XCD-aware workgroup order for the (column tile, node block) grid: workgroups
// are dealt to the 8 XCDs round-robin, so workgroup i runs on XCD i % 8.  All
// column tiles of node block b are given ids that land on XCD b % 8 back to
// back, so the block's operator rows are fetched into that XCD's L2 once and
// reused by every column tile.
__device__ inline void tile_coords(int ntiles, int& tile, int& nblk) {
  const int i = blockIdx.x;
  const int j = i >> 3;
  nblk = (j / ntiles) * 8 + (i & 7);
  tile = j % ntiles;
}

// Deterministic block sum of Q values per thread (wave64 shuffles, then LDS
// across the 4 waves in a fixed order).  Result valid in thread 0.
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
// Thread mapping of the node-blocked kernels ("operator-stationary"): a thread
// owns one node, loads that node's operator row (all slots) into registers
// once, and then loops over a group of G time-step columns two at a time.  The
// operator is read once per column group, the column data streams through,
// and the grid is (column groups) x (node blocks) in XCD-aware order.  Rows too
// large for registers (3D) are re-read per column pair from L1/L2 instead.
// ---------------------------------------------------------------------------

// fine-level residual r = c(n) F + A' X^{n-1} - AA X^{n,m-1}, the coupled
// right-hand side norms, and the first (pointwise) Chebyshev step of the
// displacement V-cycle
template <int DIM, int G>
__global__ __launch_bounds__(kBlock) void k_residual(LevelDev L, FineDev F,
                                                     const ColDesc* __restrict__ cols, int nc,
                                                     double* __restrict__ ru,
                                                     double* __restrict__ rp,
                                                     double* __restrict__ xa,
                                                     double* __restrict__ d, double inv_theta,
                                                     double* __restrict__ partials, int pstride) {
  constexpr int D1 = DIM + 1;
  constexpr int W = DIM == 2 ? 7 : 15;
  constexpr bool STAT = DIM == 2;
  constexpr int RS = STAT ? W : 1;
  __shared__ double lds[4 * 8];
  const int nn = L.nn;
  int tile, nblk;
  tile_coords((nc + G - 1) / G, tile, nblk);
  if (nblk * kBlock >= nn) return;  // padding workgroup (uniform exit)
  const int v = nblk * kBlock + threadIdx.x;
  const bool active = v < nn;
  const int vv = active ? v : nn - 1;
  int nb[W];
#pragma unroll
  for (int s = 0; s < W; ++s) nb[s] = L.nbr[size_t(s) * nn + vv];
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
  double Fu[DIM], Di[DIM * DIM];
#pragma unroll
  for (int a = 0; a < DIM; ++a) Fu[a] = active ? F.F[size_t(vv) * D1 + a] : 0.0;
#pragma unroll
  for (int e = 0; e < DIM * DIM; ++e) Di[e] = xa ? L.Ainv[size_t(e) * nn + vv] : 0.0;
  const int cbeg = tile * G, cend = min(nc, cbeg + G);
#pragma unroll 1
  for (int c = cbeg; c < cend; c += 2) {
    const bool two = c + 1 < cend;
    const int cc[2] = {c, two ? c + 1 : c};
    const double* xc[2];
    const double* xp[2];
    double coef[2], au[2][DIM], ap[2], bp[2];
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      xc[q] = cols[cc[q]].xcur;
      xp[q] = cols[cc[q]].xprev;
      coef[q] = cols[cc[q]].coef;
#pragma unroll
      for (int a = 0; a < DIM; ++a) au[q][a] = coef[q] * Fu[a];
      ap[q] = 0.0;
      bp[q] = 0.0;
    }
#pragma unroll
    for (int s = 0; s < W; ++s) {
      const int w = nb[s];
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
      for (int q = 0; q < 2; ++q) {
        double xw[D1], xpw[D1];
#pragma unroll
        for (int k = 0; k < D1; ++k) {
          xw[k] = xc[q][size_t(w) * D1 + k];
          xpw[k] = xp[q][size_t(w) * D1 + k];
        }
#pragma unroll
        for (int a = 0; a < DIM; ++a) {
          double acc = Bb[a] * xw[DIM];
#pragma unroll
          for (int k = 0; k < DIM; ++k) acc += Ab[a * DIM + k] * xw[k];
          au[q][a] -= acc;
        }
        double btc = 0.0, btp = 0.0;
#pragma unroll
        for (int k = 0; k < DIM; ++k) {
          btc += Btb[k] * xw[k];
          btp += Btb[k] * xpw[k];
        }
        const double coup = btp - Cbv * xpw[DIM];
        bp[q] += coup;
        ap[q] += coup - btc + Sv * xw[DIM];
      }
    }
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      if (!active || (q == 1 && !two)) break;
      const size_t cu = size_t(cc[q]) * nn * DIM;
      if (ru) {
#pragma unroll
        for (int a = 0; a < DIM; ++a) ru[cu + size_t(v) * DIM + a] = au[q][a];
        rp[size_t(cc[q]) * nn + v] = ap[q];
      }
      if (xa) {
#pragma unroll
        for (int a = 0; a < DIM; ++a) {
          double z = 0.0;
#pragma unroll
          for (int k = 0; k < DIM; ++k) z += Di[a * DIM + k] * au[q][k];
          z *= inv_theta;
          xa[cu + size_t(v) * DIM + a] = z;
          d[cu + size_t(v) * DIM + a] = z;
        }
      }
    }
    if (partials) {
      double qv[8];
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        double su = 0.0, sb = 0.0;
#pragma unroll
        for (int a = 0; a < DIM; ++a) {
          su += au[q][a] * au[q][a];
          const double ba = coef[q] * Fu[a];
          sb += ba * ba;
        }
        qv[4 * q + 0] = active ? su : 0.0;
        qv[4 * q + 1] = active ? ap[q] * ap[q] : 0.0;
        qv[4 * q + 2] = active ? sb : 0.0;
        qv[4 * q + 3] = active ? bp[q] * bp[q] : 0.0;
      }
      block_sum<8>(qv, lds);
      if (threadIdx.x == 0)
#pragma unroll
        for (int q = 0; q < 2; ++q) {
          if (q == 1 && !two) break;
#pragma unroll
          for (int k = 0; k < 4; ++k)
            partials[(size_t(cc[q]) * pstride + nblk) * 4 + k] = qv[4 * q + k];
        }
    }
  }
}

// ---------------------------------------------------------------------------
// Prolongation of fine node f: parents p0, p1 on the coarse grid and a bit mask
// of the components that receive each parent (bit a: p0, bit C+a: p1); the
// weight is 1 for a coincident node, 1/2 for an edge midpoint.
// ---------------------------------------------------------------------------
template <int DIM, int C>
__device__ inline void prolong_parents(const LevelDev& Lf, const LevelDev& Lc, int bit0, int f,
                                       int& p0, int& p1, unsigned& mask) {
  const int mf = Lf.n_cells + 1, mc = Lc.n_cells + 1;
  int i, j, k;
  node_coords<DIM>(f, mf, i, j, k);
  const int ai = i >> 1, aj = j >> 1, ak = k >> 1;
  const int oi = i & 1, oj = j & 1, ok = k & 1;
  const bool two = (oi | oj | ok) != 0;
  p0 = node_id<DIM>(ai, aj, ak, mc);
  p1 = two ? node_id<DIM>(ai + oi, aj + oj, ak + ok, mc) : p0;
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
// Chebyshev step on one level:
//     x  = xin               (PRO: x = xin + P xc, the coarse correction fused in)
//     d <- c1 d + c2 D^{-1}(b - K x);   xout = x + d
// UPD (pressure field, level 0, last step): instead of xout, writes the outer
// update X^{n,m} = X^{n,m-1} + omega [z_u; x + d] through the column descriptors.
// ---------------------------------------------------------------------------
template <int DIM, int C, int G, bool PRO, bool UPD, bool FINE>
__global__ __launch_bounds__(kBlock) void k_cheb(LevelDev L, LevelDev Lc, int isA,
                                                 const double* __restrict__ b,
                                                 const double* __restrict__ xin,
                                                 const double* __restrict__ xc,
                                                 double* __restrict__ xout, double* __restrict__ d,
                                                 int nc, double c1, double c2,
                                                 const ColDesc* __restrict__ cols,
                                                 const double* __restrict__ zu, double omega) {
  constexpr int W = DIM == 2 ? 7 : 15;
  constexpr bool STAT = W * C * C <= 64;
  constexpr int RS = STAT ? W : 1;
  const int nn = L.nn;
  int tile, nblk;
  tile_coords((nc + G - 1) / G, tile, nblk);
  const int v = nblk * kBlock + threadIdx.x;
  if (v >= nn) return;
  const double* K = isA ? L.A : L.S;
  const double* Dg = isA ? L.Ainv : L.Sinv;
  const int bit0 = isA ? 0 : DIM;
  const size_t stride = size_t(nn) * C;
  const size_t cstride = PRO ? size_t(Lc.nn) * C : 0;
  int nb[W];
#pragma unroll
  for (int s = 0; s < W; ++s) nb[s] = L.nbr[size_t(s) * nn + v];
  double kr[RS][C * C];
  if constexpr (STAT) {
#pragma unroll
    for (int s = 0; s < W; ++s)
#pragma unroll
      for (int e = 0; e < C * C; ++e) kr[s][e] = K[(size_t(s) * C * C + e) * nn + v];
  }
  int pp0[PRO ? W : 1], pp1[PRO ? W : 1];
  unsigned pm[PRO ? W : 1];
  if constexpr (PRO) {
#pragma unroll
    for (int s = 0; s < W; ++s) prolong_parents<DIM, C>(L, Lc, bit0, nb[s], pp0[s], pp1[s], pm[s]);
  }
  double Di[C * C];
#pragma unroll
  for (int e = 0; e < C * C; ++e) Di[e] = Dg[size_t(e) * nn + v];
  const int cbeg = tile * G, cend = min(nc, cbeg + G);
#pragma unroll 1
  for (int c = cbeg; c < cend; c += 2) {
    const bool two = c + 1 < cend;
    const int cc[2] = {c, two ? c + 1 : c};
    double acc[2][C], xs[2][C];
#pragma unroll
    for (int q = 0; q < 2; ++q)
#pragma unroll
      for (int a = 0; a < C; ++a) acc[q][a] = b[size_t(cc[q]) * stride + size_t(v) * C + a];
#pragma unroll
    for (int s = 0; s < W; ++s) {
      const int w = nb[s];
      double blk[C * C];
#pragma unroll
      for (int e = 0; e < C * C; ++e) {
        if constexpr (STAT) blk[e] = kr[s][e];
        else blk[e] = K[(size_t(s) * C * C + e) * nn + v];
      }
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        double xw[C];
#pragma unroll
        for (int k = 0; k < C; ++k) {
          xw[k] = xin[size_t(cc[q]) * stride + size_t(w) * C + k];
          if constexpr (PRO) {
            const double wt = (pm[s] >> (2 * C)) ? 0.5 : 1.0;
            const size_t cb = size_t(cc[q]) * cstride;
            if ((pm[s] >> k) & 1u) xw[k] += wt * xc[cb + size_t(pp0[s]) * C + k];
            if ((pm[s] >> (C + k)) & 1u) xw[k] += wt * xc[cb + size_t(pp1[s]) * C + k];
          }
        }
        if (s == 0)
#pragma unroll
          for (int k = 0; k < C; ++k) xs[q][k] = xw[k];
#pragma unroll
        for (int a = 0; a < C; ++a) {
          double s2 = 0.0;
#pragma unroll
          for (int k = 0; k < C; ++k) s2 += blk[a * C + k] * xw[k];
          acc[q][a] -= s2;
        }
      }
    }
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      if (q == 1 && !two) break;
      const size_t base = size_t(cc[q]) * stride + size_t(v) * C;
      double xn[C];
#pragma unroll
      for (int a = 0; a < C; ++a) {
        double z = 0.0;
#pragma unroll
        for (int k = 0; k < C; ++k) z += Di[a * C + k] * acc[q][k];
        const double dn = (c1 != 0.0 ? c1 * d[base + a] : 0.0) + c2 * z;
        if (!UPD) d[base + a] = dn;
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
          out[a] = cd.xcur[size_t(v) * D1 + a] + omega * zu[(size_t(cc[q]) * nn + v) * DIM + a];
        out[DIM] = cd.xcur[size_t(v) * D1 + DIM] + omega * xn[0];
#pragma unroll
        for (int a = 0; a < D1; ++a) cd.xout[size_t(v) * D1 + a] = out[a];
        if (cd.xout2)
#pragma unroll
          for (int a = 0; a < D1; ++a) cd.xout2[size_t(v) * D1 + a] = out[a];
      }
    }
  }
}

// xout = xin + P xc (P1 interpolation, masked) for a group of columns; the
// parents of the node are found once and reused for every column
template <int DIM, int C, int G>
__global__ __launch_bounds__(kBlock) void k_prolong(LevelDev Lf, LevelDev Lc, int isA,
                                                    const double* __restrict__ xin,
                                                    const double* __restrict__ xc,
                                                    double* __restrict__ xout, int nc) {
  const int nn = Lf.nn;
  int tile, nblk;
  tile_coords((nc + G - 1) / G, tile, nblk);
  const int v = nblk * kBlock + threadIdx.x;
  if (v >= nn) return;
  int p0, p1;
  unsigned pm;
  prolong_parents<DIM, C>(Lf, Lc, isA ? 0 : DIM, v, p0, p1, pm);
  const double wt = (pm >> (2 * C)) ? 0.5 : 1.0;
  const size_t stride = size_t(nn) * C, cstride = size_t(Lc.nn) * C;
  const int cbeg = tile * G, cend = min(nc, cbeg + G);
#pragma unroll 2
  for (int c = cbeg; c < cend; ++c) {
#pragma unroll
    for (int a = 0; a < C; ++a) {
      double x = xin[size_t(c) * stride + size_t(v) * C + a];
      if ((pm >> a) & 1u) x += wt * xc[size_t(c) * cstride + size_t(p0) * C + a];
      if ((pm >> (C + a)) & 1u) x += wt * xc[size_t(c) * cstride + size_t(p1) * C + a];
      xout[size_t(c) * stride + size_t(v) * C + a] = x;
    }
  }
}

// r = b - K x on one level
template <int DIM, int C, int G>
__global__ __launch_bounds__(kBlock) void k_level_residual(LevelDev L, int isA,
                                                           const double* __restrict__ b,
                                                           const double* __restrict__ x,
                                                           double* __restrict__ r, int nc) {
  constexpr int W = DIM == 2 ? 7 : 15;
  constexpr bool STAT = W * C * C <= 64;
  constexpr int RS = STAT ? W : 1;
  const int nn = L.nn;
  int tile, nblk;
  tile_coords((nc + G - 1) / G, tile, nblk);
  const int v = nblk * kBlock + threadIdx.x;
  if (v >= nn) return;
  const double* K = isA ? L.A : L.S;
  const size_t stride = size_t(nn) * C;
  int nb[W];
#pragma unroll
  for (int s = 0; s < W; ++s) nb[s] = L.nbr[size_t(s) * nn + v];
  double kr[RS][C * C];
  if constexpr (STAT) {
#pragma unroll
    for (int s = 0; s < W; ++s)
#pragma unroll
      for (int e = 0; e < C * C; ++e) kr[s][e] = K[(size_t(s) * C * C + e) * nn + v];
  }
  const int cbeg = tile * G, cend = min(nc, cbeg + G);
#pragma unroll 1
  for (int c = cbeg; c < cend; c += 2) {
    const bool two = c + 1 < cend;
    const int cc[2] = {c, two ? c + 1 : c};
    double acc[2][C];
#pragma unroll
    for (int q = 0; q < 2; ++q)
#pragma unroll
      for (int a = 0; a < C; ++a) acc[q][a] = b[size_t(cc[q]) * stride + size_t(v) * C + a];
#pragma unroll
    for (int s = 0; s < W; ++s) {
      const int w = nb[s];
      double blk[C * C];
#pragma unroll
      for (int e = 0; e < C * C; ++e) {
        if constexpr (STAT) blk[e] = kr[s][e];
        else blk[e] = K[(size_t(s) * C * C + e) * nn + v];
      }
#pragma unroll
      for (int q = 0; q < 2; ++q) {
#pragma unroll
        for (int a = 0; a < C; ++a) {
          double s2 = 0.0;
#pragma unroll
          for (int k = 0; k < C; ++k) s2 += blk[a * C + k] * x[size_t(cc[q]) * stride + size_t(w) * C + k];
          acc[q][a] -= s2;
        }
      }
    }
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      if (q == 1 && !two) break;
#pragma unroll
      for (int a = 0; a < C; ++a) r[size_t(cc[q]) * stride + size_t(v) * C + a] = acc[q][a];
    }
  }
}

// coarse b = P' r_fine (P1 interpolation transpose, masked), plus the first
// Chebyshev step of the coarse level when it is not the coarsest
template <int DIM, int C>
__global__ __launch_bounds__(kBlock) void k_restrict(LevelDev Lf, LevelDev Lc, int isA,
                                                     const double* __restrict__ rf,
                                                     double* __restrict__ bc,
                                                     double* __restrict__ xa,
                                                     double* __restrict__ d, double inv_theta,
                                                     int nc) {
  constexpr int W = DIM == 2 ? 7 : 15;
  const int I = blockIdx.y * kBlock + threadIdx.x;
  if (I >= Lc.nn) return;
  const int c = blockIdx.x;
  const int mc = Lc.n_cells + 1, mf = Lf.n_cells + 1;
  int ci, cj, ck;
  node_coords<DIM>(I, mc, ci, cj, ck);
  const uint8_t fc = Lc.fixed[I];
  const int bit0 = isA ? 0 : DIM;
  const size_t sf = size_t(Lf.nn) * C, sc = size_t(Lc.nn) * C;
  double acc[C];
#pragma unroll
  for (int a = 0; a < C; ++a) acc[a] = 0.0;
#pragma unroll
  for (int s = 0; s < W; ++s) {
    const int* o = DIM == 2 ? c_off2[s] : c_off3[s];
    const int fi = 2 * ci + o[0], fj = 2 * cj + o[1], fk = 2 * ck + o[2];
    if (fi < 0 || fi >= mf || fj < 0 || fj >= mf || fk < 0 || fk >= mf) continue;
    const int f = node_id<DIM>(fi, fj, fk, mf);
    const double wgt = s == 0 ? 1.0 : 0.5;
    const uint8_t ff = Lf.fixed[f];
#pragma unroll
    for (int a = 0; a < C; ++a)
      if (!((ff >> (bit0 + a)) & 1)) acc[a] += wgt * rf[size_t(c) * sf + size_t(f) * C + a];
  }
#pragma unroll
  for (int a = 0; a < C; ++a) {
    if ((fc >> (bit0 + a)) & 1) acc[a] = 0.0;
    bc[size_t(c) * sc + size_t(I) * C + a] = acc[a];
  }
  if (xa) {
    const double* Dg = isA ? Lc.Ainv : Lc.Sinv;
#pragma unroll
    for (int a = 0; a < C; ++a) {
      double z = 0.0;
#pragma unroll
      for (int k = 0; k < C; ++k) z += Dg[size_t(a * C + k) * Lc.nn + I] * acc[k];
      z *= inv_theta;
      xa[size_t(c) * sc + size_t(I) * C + a] = z;
      d[size_t(c) * sc + size_t(I) * C + a] = z;
    }
  }
}

// coarsest level: x = M^{-1} b with the dense inverse, one workgroup per column
__global__ __launch_bounds__(kBlock) void k_coarse_solve(int n, const double* __restrict__ Minv,
                                                         const double* __restrict__ b,
                                                         double* __restrict__ x) {
  extern __shared__ double sb[];
  const int c = blockIdx.x;
  for (int i = threadIdx.x; i < n; i += kBlock) sb[i] = b[size_t(c) * n + i];
  __syncthreads();
  for (int r = threadIdx.x; r < n; r += kBlock) {
    double acc = 0.0;
    const double* row = Minv + size_t(r) * n;
    for (int j = 0; j < n; ++j) acc += row[j] * sb[j];
    x[size_t(c) * n + r] = acc;
  }
}

// pressure stage of P1: t = B' z_u - r_p (P2: t = -r_p), and the first
// Chebyshev step of the pressure V-cycle
template <int DIM, int G>
__global__ __launch_bounds__(kBlock) void k_pstage(LevelDev L, FineDev F, int p1,
                                                   const double* __restrict__ zu,
                                                   const double* __restrict__ rp,
                                                   double* __restrict__ t_out,
                                                   double* __restrict__ xa,
                                                   double* __restrict__ d, double inv_theta,
                                                   int nc) {
  constexpr int W = DIM == 2 ? 7 : 15;
  const int nn = L.nn;
  int tile, nblk;
  tile_coords((nc + G - 1) / G, tile, nblk);
  const int v = nblk * kBlock + threadIdx.x;
  if (v >= nn) return;
  int nb[W];
  double bt[W][DIM];
#pragma unroll
  for (int s = 0; s < W; ++s) {
    nb[s] = L.nbr[size_t(s) * nn + v];
#pragma unroll
    for (int k = 0; k < DIM; ++k) bt[s][k] = p1 ? F.Bt[(size_t(s) * DIM + k) * nn + v] : 0.0;
  }
  const double si = L.Sinv[v];
  const int cbeg = tile * G, cend = min(nc, cbeg + G);
#pragma unroll 1
  for (int c = cbeg; c < cend; c += 2) {
    const bool two = c + 1 < cend;
    const int cc[2] = {c, two ? c + 1 : c};
    double acc[2];
#pragma unroll
    for (int q = 0; q < 2; ++q) acc[q] = -rp[size_t(cc[q]) * nn + v];
    if (p1) {
#pragma unroll
      for (int s = 0; s < W; ++s) {
        const int w = nb[s];
#pragma unroll
        for (int q = 0; q < 2; ++q) {
          const size_t base = size_t(cc[q]) * nn * DIM + size_t(w) * DIM;
#pragma unroll
          for (int k = 0; k < DIM; ++k) acc[q] += bt[s][k] * zu[base + k];
        }
      }
    }
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      if (q == 1 && !two) break;
      const size_t idx = size_t(cc[q]) * nn + v;
      t_out[idx] = acc[q];
      const double z = si * acc[q] * inv_theta;
      xa[idx] = z;
      d[idx] = z;
    }
  }
}

// X^{n,m} = X^{n,m-1} + omega [z_u; z_p]
template <int DIM>
__global__ __launch_bounds__(kBlock) void k_update(int nn, const ColDesc* __restrict__ cols,
                                                   const double* __restrict__ zu,
                                                   const double* __restrict__ zp, double omega) {
  constexpr int D1 = DIM + 1;
  const int v = blockIdx.y * kBlock + threadIdx.x;
  if (v >= nn) return;
  const int c = blockIdx.x;
  const double* xc = cols[c].xcur;
  double* xo = cols[c].xout;
  double* xo2 = cols[c].xout2;
  double out[D1];
#pragma unroll
  for (int a = 0; a < DIM; ++a)
    out[a] = xc[size_t(v) * D1 + a] + omega * zu[(size_t(c) * nn + v) * DIM + a];
  out[DIM] = xc[size_t(v) * D1 + DIM] + omega * zp[size_t(c) * nn + v];
#pragma unroll
  for (int a = 0; a < D1; ++a) xo[size_t(v) * D1 + a] = out[a];
  if (xo2)
#pragma unroll
    for (int a = 0; a < D1; ++a) xo2[size_t(v) * D1 + a] = out[a];
}

// per-column sums of the block partials in a fixed order
__global__ __launch_bounds__(kBlock) void k_reduce_norms(const double* __restrict__ partials,
                                                         int nblk, int pstride,
                                                         double* __restrict__ norms) {
  __shared__ double lds[16];
  const int c = blockIdx.x;
  double q[4] = {0.0, 0.0, 0.0, 0.0};
  for (int b = threadIdx.x; b < nblk; b += kBlock)
#pragma unroll
    for (int k = 0; k < 4; ++k) q[k] += partials[(size_t(c) * pstride + b) * 4 + k];
  block_sum<4>(q, lds);
  if (threadIdx.x == 0)
#pragma unroll
    for (int k = 0; k < 4; ++k) norms[size_t(c) * 4 + k] = q[k];
}

// Y = AA X (test/diagnostic path)
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

template <int DIM>
__global__ __launch_bounds__(kBlock) void k_unpack(int nn, const double* __restrict__ X,
                                                   double* __restrict__ ru,
                                                   double* __restrict__ rp) {
  constexpr int D1 = DIM + 1;
  const int v = blockIdx.y * kBlock + threadIdx.x;
  if (v >= nn) return;
  const size_t c = blockIdx.x;
#pragma unroll
  for (int a = 0; a < DIM; ++a) ru[(c * nn + v) * DIM + a] = X[(c * nn + v) * D1 + a];
  rp[c * nn + v] = X[(c * nn + v) * D1 + DIM];
}

template <int DIM>
__global__ __launch_bounds__(kBlock) void k_pack(int nn, const double* __restrict__ zu,
                                                 const double* __restrict__ zp,
                                                 double* __restrict__ Z) {
  constexpr int D1 = DIM + 1;
  const int v = blockIdx.y * kBlock + threadIdx.x;
  if (v >= nn) return;
  const size_t c = blockIdx.x;
#pragma unroll
  for (int a = 0; a < DIM; ++a) Z[(c * nn + v) * D1 + a] = zu[(c * nn + v) * DIM + a];
  Z[(c * nn + v) * D1 + DIM] = zp[c * nn + v];
}

// first Chebyshev step from a zero iterate: xa = d = D^{-1} b / theta
template <int C>
__global__ __launch_bounds__(kBlock) void k_pre1(LevelDev L, int isA, const double* __restrict__ b,
                                                 double* __restrict__ xa, double* __restrict__ d,
                                                 double inv_theta) {
  const int v = blockIdx.y * kBlock + threadIdx.x;
  if (v >= L.nn) return;
  const size_t base = size_t(blockIdx.x) * L.nn * C + size_t(v) * C;
  const double* Dg = isA ? L.Ainv : L.Sinv;
#pragma unroll
  for (int a = 0; a < C; ++a) {
    double z = 0.0;
#pragma unroll
    for (int k = 0; k < C; ++k) z += Dg[size_t(a * C + k) * L.nn + v] * b[base + k];
    z *= inv_theta;
    xa[base + a] = z;
    d[base + a] = z;
  }
}

inline dim3 tiled_grid(int nc, int nn, int ct) {
  const int nb8 = (num_node_blocks(nn) + 7) / 8 * 8;
  return dim3(nb8 * ((nc + ct - 1) / ct));
}
inline dim3 col_grid(int nc, int nn) { return dim3(nc, num_node_blocks(nn)); }

// runtime column group -> template instantiation
#define BIOT_CT_SWITCH(ct, ...)                              \
  switch (ct) {                                              \
    case 1: { constexpr int CTT = 1; __VA_ARGS__; } break;   \
    case 2: { constexpr int CTT = 2; __VA_ARGS__; } break;   \
    case 4: { constexpr int CTT = 4; __VA_ARGS__; } break;   \
    case 8: { constexpr int CTT = 8; __VA_ARGS__; } break;   \
    case 32: { constexpr int CTT = 32; __VA_ARGS__; } break; \
    default: { constexpr int CTT = 16; __VA_ARGS__; } break; \
  }

}  // namespace

bool valid_col_tile(int ct) {
  return ct == 1 || ct == 2 || ct == 4 || ct == 8 || ct == 16 || ct == 32;
}

// largest column group <= gmax that still gives the grid enough workgroups
int pick_group(int nc, int nn, int gmax) {
  const long nb8 = (num_node_blocks(nn) + 7) / 8 * 8;
  int g = gmax;
  while (g > 1 && nb8 * ((nc + g - 1) / g) < 1024) g >>= 1;
  return g;
}

void launch_residual(int dim, const LevelDev& L, const FineDev& F, const ColDesc* cols, int nc,
                     double* ru, double* rp, double* xa, double* d, double inv_theta,
                     double* partials, int pstride, int ct, hipStream_t st) {
  ct = pick_group(nc, L.nn, ct);
  const dim3 g = tiled_grid(nc, L.nn, ct);
  if (dim == 2) {
    BIOT_CT_SWITCH(ct, hipLaunchKernelGGL((k_residual<2, CTT>), g, dim3(kBlock), 0, st, L, F, cols,
                                          nc, ru, rp, xa, d, inv_theta, partials, pstride))
  } else {
    BIOT_CT_SWITCH(ct, hipLaunchKernelGGL((k_residual<3, CTT>), g, dim3(kBlock), 0, st, L, F, cols,
                                          nc, ru, rp, xa, d, inv_theta, partials, pstride))
  }
}

template <int DIM, int C, bool PRO, bool UPD>
static void cheb_dispatch(const LevelDev& L, const LevelDev& Lc, bool is_A, const double* b,
                          const double* xin, const double* xc, double* xout, double* d, int nc,
                          double c1, double c2, const ColDesc* cols, const double* zu,
                          double omega, int ct, bool fine, hipStream_t st) {
  ct = pick_group(nc, L.nn, ct);
  const dim3 g = tiled_grid(nc, L.nn, ct);
  if (fine) {
    BIOT_CT_SWITCH(ct, hipLaunchKernelGGL((k_cheb<DIM, C, CTT, PRO, UPD, true>), g, dim3(kBlock), 0,
                                          st, L, Lc, int(is_A), b, xin, xc, xout, d, nc, c1, c2,
                                          cols, zu, omega))
  } else if (!UPD) {
    BIOT_CT_SWITCH(ct, hipLaunchKernelGGL((k_cheb<DIM, C, CTT, PRO, UPD, false>), g, dim3(kBlock), 0,
                                          st, L, Lc, int(is_A), b, xin, xc, xout, d, nc, c1, c2,
                                          cols, zu, omega))
  }
}

void launch_cheb(int dim, int comps, const LevelDev& L, const LevelDev* Lc, bool is_A,
                 const double* b, const double* xin, const double* xc, double* xout, double* d,
                 int nc, double c1, double c2, const ColDesc* cols, const double* zu,
                 double omega, int ct, bool fine, hipStream_t st) {
  const bool pro = xc != nullptr;
  const bool upd = cols != nullptr;
  const LevelDev& C2 = Lc ? *Lc : L;
  if (dim == 2) {
    if (comps == 1) {
      if (upd) cheb_dispatch<2, 1, false, true>(L, C2, is_A, b, xin, xc, xout, d, nc, c1, c2, cols, zu, omega, ct, fine, st);
      else if (pro) cheb_dispatch<2, 1, true, false>(L, C2, is_A, b, xin, xc, xout, d, nc, c1, c2, cols, zu, omega, ct, fine, st);
      else cheb_dispatch<2, 1, false, false>(L, C2, is_A, b, xin, xc, xout, d, nc, c1, c2, cols, zu, omega, ct, fine, st);
    } else {
      if (pro) cheb_dispatch<2, 2, true, false>(L, C2, is_A, b, xin, xc, xout, d, nc, c1, c2, cols, zu, omega, ct, fine, st);
      else cheb_dispatch<2, 2, false, false>(L, C2, is_A, b, xin, xc, xout, d, nc, c1, c2, cols, zu, omega, ct, fine, st);
    }
  } else {
    if (comps == 1) {
      if (upd) cheb_dispatch<3, 1, false, true>(L, C2, is_A, b, xin, xc, xout, d, nc, c1, c2, cols, zu, omega, ct, fine, st);
      else if (pro) cheb_dispatch<3, 1, true, false>(L, C2, is_A, b, xin, xc, xout, d, nc, c1, c2, cols, zu, omega, ct, fine, st);
      else cheb_dispatch<3, 1, false, false>(L, C2, is_A, b, xin, xc, xout, d, nc, c1, c2, cols, zu, omega, ct, fine, st);
    } else {
      if (pro) cheb_dispatch<3, 3, true, false>(L, C2, is_A, b, xin, xc, xout, d, nc, c1, c2, cols, zu, omega, ct, fine, st);
      else cheb_dispatch<3, 3, false, false>(L, C2, is_A, b, xin, xc, xout, d, nc, c1, c2, cols, zu, omega, ct, fine, st);
    }
  }
}

void launch_level_residual(int dim, int comps, const LevelDev& L, bool is_A, const double* b,
                           const double* x, double* r, int nc, int ct, hipStream_t st) {
  ct = pick_group(nc, L.nn, ct);
  const dim3 g = tiled_grid(nc, L.nn, ct);
  if (dim == 2) {
    if (comps == 1) { BIOT_CT_SWITCH(ct, hipLaunchKernelGGL((k_level_residual<2, 1, CTT>), g, dim3(kBlock), 0, st, L, int(is_A), b, x, r, nc)) }
    else { BIOT_CT_SWITCH(ct, hipLaunchKernelGGL((k_level_residual<2, 2, CTT>), g, dim3(kBlock), 0, st, L, int(is_A), b, x, r, nc)) }
  } else {
    if (comps == 1) { BIOT_CT_SWITCH(ct, hipLaunchKernelGGL((k_level_residual<3, 1, CTT>), g, dim3(kBlock), 0, st, L, int(is_A), b, x, r, nc)) }
    else { BIOT_CT_SWITCH(ct, hipLaunchKernelGGL((k_level_residual<3, 3, CTT>), g, dim3(kBlock), 0, st, L, int(is_A), b, x, r, nc)) }
  }
}

void launch_restrict(int dim, int comps, const LevelDev& Lf, const LevelDev& Lc, bool is_A,
                     const double* rf, double* bc, double* xa_c, double* d_c, double inv_theta_c,
                     int nc, hipStream_t st) {
  dim3 g = col_grid(nc, Lc.nn);
  if (dim == 2) {
    if (comps == 1) hipLaunchKernelGGL((k_restrict<2, 1>), g, dim3(kBlock), 0, st, Lf, Lc, int(is_A), rf, bc, xa_c, d_c, inv_theta_c, nc);
    else hipLaunchKernelGGL((k_restrict<2, 2>), g, dim3(kBlock), 0, st, Lf, Lc, int(is_A), rf, bc, xa_c, d_c, inv_theta_c, nc);
  } else {
    if (comps == 1) hipLaunchKernelGGL((k_restrict<3, 1>), g, dim3(kBlock), 0, st, Lf, Lc, int(is_A), rf, bc, xa_c, d_c, inv_theta_c, nc);
    else hipLaunchKernelGGL((k_restrict<3, 3>), g, dim3(kBlock), 0, st, Lf, Lc, int(is_A), rf, bc, xa_c, d_c, inv_theta_c, nc);
  }
}


void launch_prolong(int dim, int comps, const LevelDev& Lf, const LevelDev& Lc, bool is_A,
                    const double* xin, const double* xc, double* xout, int nc, int ct,
                    hipStream_t st) {
  ct = pick_group(nc, Lf.nn, ct);
  const dim3 g = tiled_grid(nc, Lf.nn, ct);
  if (dim == 2) {
    if (comps == 1) { BIOT_CT_SWITCH(ct, hipLaunchKernelGGL((k_prolong<2, 1, CTT>), g, dim3(kBlock), 0, st, Lf, Lc, int(is_A), xin, xc, xout, nc)) }
    else { BIOT_CT_SWITCH(ct, hipLaunchKernelGGL((k_prolong<2, 2, CTT>), g, dim3(kBlock), 0, st, Lf, Lc, int(is_A), xin, xc, xout, nc)) }
  } else {
    if (comps == 1) { BIOT_CT_SWITCH(ct, hipLaunchKernelGGL((k_prolong<3, 1, CTT>), g, dim3(kBlock), 0, st, Lf, Lc, int(is_A), xin, xc, xout, nc)) }
    else { BIOT_CT_SWITCH(ct, hipLaunchKernelGGL((k_prolong<3, 3, CTT>), g, dim3(kBlock), 0, st, Lf, Lc, int(is_A), xin, xc, xout, nc)) }
  }
}

void launch_coarse_solve(int n, const double* Minv, const double* b, double* x, int nc,
                         hipStream_t st) {
  hipLaunchKernelGGL(k_coarse_solve, dim3(nc), dim3(kBlock), size_t(n) * sizeof(double), st, n,
                     Minv, b, x);
}

void launch_pstage(int dim, const LevelDev& L, const FineDev& F, bool p1, const double* zu,
                   const double* rp, double* t, double* xa, double* d, double inv_theta, int nc,
                   int ct, hipStream_t st) {
  ct = pick_group(nc, L.nn, ct);
  const dim3 g = tiled_grid(nc, L.nn, ct);
  if (dim == 2) {
    BIOT_CT_SWITCH(ct, hipLaunchKernelGGL((k_pstage<2, CTT>), g, dim3(kBlock), 0, st, L, F, int(p1), zu, rp, t, xa, d, inv_theta, nc))
  } else {
    BIOT_CT_SWITCH(ct, hipLaunchKernelGGL((k_pstage<3, CTT>), g, dim3(kBlock), 0, st, L, F, int(p1), zu, rp, t, xa, d, inv_theta, nc))
  }
}

void launch_update(int dim, int nn, const ColDesc* cols, const double* zu, const double* zp,
                   double omega, int nc, hipStream_t st) {
  dim3 g = col_grid(nc, nn);
  if (dim == 2) hipLaunchKernelGGL(k_update<2>, g, dim3(kBlock), 0, st, nn, cols, zu, zp, omega);
  else hipLaunchKernelGGL(k_update<3>, g, dim3(kBlock), 0, st, nn, cols, zu, zp, omega);
}

void launch_reduce_norms(const double* partials, int nblk, int pstride, double* norms, int nc,
                         hipStream_t st) {
  hipLaunchKernelGGL(k_reduce_norms, dim3(nc), dim3(kBlock), 0, st, partials, nblk, pstride, norms);
}

void launch_apply_operator(int dim, const LevelDev& L, const FineDev& F, const double* X,
                           double* Y, int nc, hipStream_t st) {
  dim3 g = col_grid(nc, L.nn);
  if (dim == 2) hipLaunchKernelGGL(k_apply_operator<2>, g, dim3(kBlock), 0, st, L, F, X, Y);
  else hipLaunchKernelGGL(k_apply_operator<3>, g, dim3(kBlock), 0, st, L, F, X, Y);
}

void launch_unpack(int dim, int nn, const double* X, double* ru, double* rp, int nc, hipStream_t st) {
  dim3 g = col_grid(nc, nn);
  if (dim == 2) hipLaunchKernelGGL(k_unpack<2>, g, dim3(kBlock), 0, st, nn, X, ru, rp);
  else hipLaunchKernelGGL(k_unpack<3>, g, dim3(kBlock), 0, st, nn, X, ru, rp);
}

void launch_pre1(int comps, const LevelDev& L, bool is_A, const double* b, double* xa, double* d,
                 double inv_theta, int nc, hipStream_t st) {
  dim3 g = col_grid(nc, L.nn);
  switch (comps) {
    case 1: hipLaunchKernelGGL(k_pre1<1>, g, dim3(kBlock), 0, st, L, int(is_A), b, xa, d, inv_theta); break;
    case 2: hipLaunchKernelGGL(k_pre1<2>, g, dim3(kBlock), 0, st, L, int(is_A), b, xa, d, inv_theta); break;
    default: hipLaunchKernelGGL(k_pre1<3>, g, dim3(kBlock), 0, st, L, int(is_A), b, xa, d, inv_theta); break;
  }
}

void launch_pack(int dim, int nn, const double* zu, const double* zp, double* Z, int nc,
                 hipStream_t st) {
  dim3 g = col_grid(nc, nn);
  if (dim == 2) hipLaunchKernelGGL(k_pack<2>, g, dim3(kBlock), 0, st, nn, zu, zp, Z);
  else hipLaunchKernelGGL(k_pack<3>, g, dim3(kBlock), 0, st, nn, zu, zp, Z);
}

}  // namespace biot
