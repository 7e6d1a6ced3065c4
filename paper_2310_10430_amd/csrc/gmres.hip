// HIP kernels (gfx950) of GMRES(k) per unit: the Krylov inner solver of the
// paper's Alg. 3, where each (time step, outer iteration) unit applies k
// iterations of preconditioned GMRES to AA x = b^{n,m} starting from X^{n,m-1}.
//
// All columns of a batch run their own Krylov process side by side; every
// vector is a node-major FP64 column [nn][dim+1] and every small quantity
// (Hessenberg matrix, rotations, right-hand side g) lives per column on the
// device, so a unit never waits for the host.  Reductions are deterministic:
// fixed per-thread element sets, wave64 shuffles, a fixed LDS order, and a
// second pass over the block partials in block order.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

#include "kernels.hpp"

namespace biot {
namespace {

constexpr int kDotBlocks = kGmresDotBlocks;  // partial sums per column

// the vectors of one batch column: vec(i) = base + (i * stride_v) + c * col
struct ColVecs {
  const double* base;
  size_t stride_v;  // between consecutive basis vectors
  size_t col;       // values per column
};

// out[c][blk][i] = partial of <V_i[c], W[c]>, i < nvec (W may be V_j itself)
__global__ __launch_bounds__(kBlock) void k_multi_dot(ColVecs V, int nvec, const double* __restrict__ W,
                                                      double* __restrict__ part) {
  __shared__ double lds[4][kGmresMaxK + 1];
  const int c = blockIdx.y, blk = blockIdx.x;
  const size_t n = V.col;
  const size_t per = (n + kDotBlocks - 1) / kDotBlocks;
  const size_t lo = blk * per, hi = min(n, lo + per);
  const double* w = W + size_t(c) * n;
  double acc[kGmresMaxK + 1];
#pragma unroll
  for (int i = 0; i <= kGmresMaxK; ++i) acc[i] = 0.0;
  for (size_t e = lo + threadIdx.x; e < hi; e += kBlock) {
    const double we = w[e];
#pragma unroll
    for (int i = 0; i <= kGmresMaxK; ++i)
      if (i < nvec) acc[i] += V.base[i * V.stride_v + size_t(c) * n + e] * we;
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int i = 0; i <= kGmresMaxK; ++i) {
    double x = acc[i];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) x += __shfl_down(x, off, 64);
    if (lane == 0) lds[wave][i] = x;
  }
  __syncthreads();
  if (int(threadIdx.x) < nvec) {
    const int i = threadIdx.x;
    part[(size_t(c) * kDotBlocks + blk) * (kGmresMaxK + 1) + i] =
        ((lds[0][i] + lds[1][i]) + lds[2][i]) + lds[3][i];
  }
}

// value_i = sum of the partials of column c in block order; then
//   mode 0: out[c*ocs + i*ois] = value_i
//   mode 1: out[...] += value_i
//   mode 2: out[...] = sqrt(value_i)          (a norm)
// and, when out2 is given, out2[c*ocs2 + i*ois2] += value_i as well
__global__ __launch_bounds__(64) void k_dot_finish(const double* __restrict__ part, int nvec,
                                                   double* __restrict__ out, size_t ocs, size_t ois,
                                                   int mode, double* __restrict__ out2, size_t ocs2,
                                                   size_t ois2, int nc) {
  const int c = blockIdx.x * 64 + threadIdx.x;
  if (c >= nc) return;
  for (int i = 0; i < nvec; ++i) {
    double s = 0.0;
    for (int b = 0; b < kDotBlocks; ++b) s += part[(size_t(c) * kDotBlocks + b) * (kGmresMaxK + 1) + i];
    double* o = out + size_t(c) * ocs + size_t(i) * ois;
    if (mode == 0) *o = s;
    else if (mode == 1) *o += s;
    else *o = std::sqrt(s);
    if (out2) out2[size_t(c) * ocs2 + size_t(i) * ois2] += s;
  }
}

// W[c] -= sum_{i < nvec} coef[c*ccs + i*cis] V_i[c]
__global__ __launch_bounds__(kBlock) void k_multi_axpy(ColVecs V, int nvec, const double* __restrict__ coef,
                                                       size_t ccs, size_t cis, double* __restrict__ W) {
  const int c = blockIdx.y;
  const size_t n = V.col;
  double a[kGmresMaxK + 1];
#pragma unroll
  for (int i = 0; i <= kGmresMaxK; ++i) a[i] = i < nvec ? coef[size_t(c) * ccs + size_t(i) * cis] : 0.0;
  double* w = W + size_t(c) * n;
  for (size_t e = size_t(blockIdx.x) * kBlock + threadIdx.x; e < n; e += size_t(gridDim.x) * kBlock) {
    double x = w[e];
#pragma unroll
    for (int i = 0; i <= kGmresMaxK; ++i)
      if (i < nvec) x -= a[i] * V.base[i * V.stride_v + size_t(c) * n + e];
    w[e] = x;
  }
}

// V[c] *= 1 / s[c] (0 when s[c] is zero: a column that has converged exactly)
__global__ __launch_bounds__(kBlock) void k_col_scale(double* __restrict__ X, size_t n,
                                                      const double* __restrict__ s, size_t s_stride) {
  const int c = blockIdx.y;
  const double v = s[size_t(c) * s_stride];
  const double inv = v > 0.0 ? 1.0 / v : 0.0;
  double* x = X + size_t(c) * n;
  for (size_t e = size_t(blockIdx.x) * kBlock + threadIdx.x; e < n; e += size_t(gridDim.x) * kBlock)
    x[e] *= inv;
}

// Givens step j for every column: rotate H[:, j] by the earlier rotations,
// make the new rotation that zeroes H[j+1][j], and rotate g.
__global__ __launch_bounds__(64) void k_givens(double* __restrict__ H, double* __restrict__ g,
                                               double* __restrict__ cs, double* __restrict__ sn,
                                               int j, int nc) {
  const int c = blockIdx.x * 64 + threadIdx.x;
  if (c >= nc) return;
  double* Hc = H + size_t(c) * (kGmresMaxK + 1) * kGmresMaxK;
  double* gc = g + size_t(c) * (kGmresMaxK + 1);
  double* cc = cs + size_t(c) * kGmresMaxK;
  double* ss = sn + size_t(c) * kGmresMaxK;
  for (int i = 0; i < j; ++i) {
    const double a = Hc[i * kGmresMaxK + j], b = Hc[(i + 1) * kGmresMaxK + j];
    Hc[i * kGmresMaxK + j] = cc[i] * a + ss[i] * b;
    Hc[(i + 1) * kGmresMaxK + j] = -ss[i] * a + cc[i] * b;
  }
  const double a = Hc[j * kGmresMaxK + j], b = Hc[(j + 1) * kGmresMaxK + j];
  const double r = std::hypot(a, b);
  const double co = r > 0.0 ? a / r : 1.0, si = r > 0.0 ? b / r : 0.0;
  cc[j] = co;
  ss[j] = si;
  Hc[j * kGmresMaxK + j] = r;
  Hc[(j + 1) * kGmresMaxK + j] = 0.0;
  const double gj = gc[j];
  gc[j] = co * gj;
  gc[j + 1] = -si * gj;
}

// g = (||r0||, 0, ..., 0) from the norm stored in beta[c]
__global__ __launch_bounds__(64) void k_gmres_start(const double* __restrict__ beta, size_t beta_stride,
                                                    double* __restrict__ g, int nc) {
  const int c = blockIdx.x * 64 + threadIdx.x;
  if (c >= nc) return;
  double* gc = g + size_t(c) * (kGmresMaxK + 1);
  gc[0] = beta[size_t(c) * beta_stride];
  for (int i = 1; i <= kGmresMaxK; ++i) gc[i] = 0.0;
}

// y = R^{-1} g (R = the rotated k x k upper triangle); a zero pivot (exact
// convergence earlier in the process) drops that direction
__global__ __launch_bounds__(64) void k_gmres_solve(const double* __restrict__ H,
                                                    const double* __restrict__ g, int k,
                                                    double* __restrict__ y, int nc) {
  const int c = blockIdx.x * 64 + threadIdx.x;
  if (c >= nc) return;
  const double* Hc = H + size_t(c) * (kGmresMaxK + 1) * kGmresMaxK;
  const double* gc = g + size_t(c) * (kGmresMaxK + 1);
  double* yc = y + size_t(c) * kGmresMaxK;
  for (int i = k - 1; i >= 0; --i) {
    double s = gc[i];
    for (int l = i + 1; l < k; ++l) s -= Hc[i * kGmresMaxK + l] * yc[l];
    const double d = Hc[i * kGmresMaxK + i];
    yc[i] = d != 0.0 ? s / d : 0.0;
  }
}

// X^{n,m} = X^{n,m-1} + sum_j y_j V_j through the column descriptors
template <int DIM>
__global__ __launch_bounds__(kBlock) void k_gmres_update(int nn, const ColDesc* __restrict__ cols,
                                                         ColVecs Z, int k, const double* __restrict__ y) {
  constexpr int D1 = DIM + 1;
  const int v = blockIdx.y * kBlock + threadIdx.x;
  if (v >= nn) return;
  const int c = blockIdx.x;
  const ColDesc cd = cols[c];
  double yc[kGmresMaxK];
  for (int j = 0; j < k; ++j) yc[j] = y[size_t(c) * kGmresMaxK + j];
  double out[D1];
#pragma unroll
  for (int a = 0; a < D1; ++a) {
    double x = cd.xcur[size_t(v) * D1 + a];
    for (int j = 0; j < k; ++j) x += yc[j] * Z.base[j * Z.stride_v + size_t(c) * Z.col + size_t(v) * D1 + a];
    out[a] = x;
  }
#pragma unroll
  for (int a = 0; a < D1; ++a) cd.xout[size_t(v) * D1 + a] = out[a];
  if (cd.xout2)
#pragma unroll
    for (int a = 0; a < D1; ++a) cd.xout2[size_t(v) * D1 + a] = out[a];
}

inline dim3 stream_grid(size_t n, int nc) {
  const size_t b = (n + kBlock - 1) / kBlock;
  return dim3(unsigned(std::min<size_t>(b, 256)), unsigned(nc));
}

}  // namespace

void gmres_dot(const GmresVecs& V, int nvec, const double* W, double* part, double* out,
               size_t ocs, size_t ois, int mode, double* out2, size_t ocs2, size_t ois2, int nc,
               hipStream_t st) {
  const ColVecs cv{V.base, V.stride_v, V.col};
  hipLaunchKernelGGL(k_multi_dot, dim3(kDotBlocks, nc), dim3(kBlock), 0, st, cv, nvec, W, part);
  hipLaunchKernelGGL(k_dot_finish, dim3((nc + 63) / 64), dim3(64), 0, st, part, nvec, out, ocs, ois,
                     mode, out2, ocs2, ois2, nc);
}

void gmres_axpy(const GmresVecs& V, int nvec, const double* coef, size_t ccs, size_t cis, double* W,
                int nc, hipStream_t st) {
  const ColVecs cv{V.base, V.stride_v, V.col};
  hipLaunchKernelGGL(k_multi_axpy, stream_grid(V.col, nc), dim3(kBlock), 0, st, cv, nvec, coef, ccs,
                     cis, W);
}

void gmres_scale(double* X, size_t col, const double* s, size_t s_stride, int nc, hipStream_t st) {
  hipLaunchKernelGGL(k_col_scale, stream_grid(col, nc), dim3(kBlock), 0, st, X, col, s, s_stride);
}

void gmres_start(const double* beta, size_t beta_stride, double* g, int nc, hipStream_t st) {
  hipLaunchKernelGGL(k_gmres_start, dim3((nc + 63) / 64), dim3(64), 0, st, beta, beta_stride, g, nc);
}

void gmres_givens(double* H, double* g, double* cs, double* sn, int j, int nc, hipStream_t st) {
  hipLaunchKernelGGL(k_givens, dim3((nc + 63) / 64), dim3(64), 0, st, H, g, cs, sn, j, nc);
}

void gmres_finish(int dim, int nn, const ColDesc* cols, const GmresVecs& Z, int k, const double* H,
                  const double* g, double* y, int nc, hipStream_t st) {
  hipLaunchKernelGGL(k_gmres_solve, dim3((nc + 63) / 64), dim3(64), 0, st, H, g, k, y, nc);
  const ColVecs cz{Z.base, Z.stride_v, Z.col};
  const dim3 grid(nc, num_node_blocks(nn));
  if (dim == 2) hipLaunchKernelGGL(k_gmres_update<2>, grid, dim3(kBlock), 0, st, nn, cols, cz, k, y);
  else hipLaunchKernelGGL(k_gmres_update<3>, grid, dim3(kBlock), 0, st, nn, cols, cz, k, y);
}

}  // namespace biot
