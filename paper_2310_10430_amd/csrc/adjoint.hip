// HIP kernels (gfx950) of the adjoint: the pressure-misfit load, replay start
// values and the element-by-element gradient contraction.
//
// The adjoint states themselves are computed by the sweep kernels (k_residual
// with its adjoint coupling, the multigrid preconditioner and the update), run
// over the time-reversed recursion.
#include <hip/hip_runtime.h>

#include "kernels.hpp"

namespace biot {
namespace {

__global__ __launch_bounds__(kBlock) void k_sensor_load(int nn, int N, int S, int D1,
                                                        const double* __restrict__ X,
                                                        const int32_t* __restrict__ sens,
                                                        const double* __restrict__ pobs,
                                                        const uint8_t* __restrict__ fixed,
                                                        double* __restrict__ gload,
                                                        double* __restrict__ jpart) {
  const long i = long(blockIdx.x) * kBlock + threadIdx.x;
  if (i >= long(N) * S) return;
  const int n = int(i / S) + 1, s = int(i % S);
  const int node = sens[s];
  const size_t col = size_t(nn) * D1;
  const double r = X[size_t(n) * col + size_t(node) * D1 + (D1 - 1)] - pobs[i];
  jpart[i] = r * r;
  const bool free_p = ((fixed[node] >> (D1 - 1)) & 1) == 0;
  const int m = N + 1 - n;  // reversed-time column of step n
  gload[size_t(m - 1) * nn + node] = free_p ? 2.0 * r : 0.0;
}

// one workgroup: strided partial sums, then a fixed-order tree over the block
__global__ __launch_bounds__(kBlock) void k_sum(const double* __restrict__ x, int n,
                                                double* __restrict__ out) {
  __shared__ double lds[kBlock];
  double acc = 0.0;
  for (int i = threadIdx.x; i < n; i += kBlock) acc += x[i];
  lds[threadIdx.x] = acc;
  __syncthreads();
  for (int w = kBlock / 2; w > 0; w >>= 1) {
    if (int(threadIdx.x) < w) lds[threadIdx.x] += lds[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = lds[0];
}

__device__ inline int ckpt_index(int step, int s, int N, int K) {
  return step == N ? K : step / s;
}

__global__ __launch_bounds__(kBlock) void k_lerp_init(size_t col, const double* __restrict__ ck,
                                                      int s, int N, int n0,
                                                      double* __restrict__ out) {
  const size_t i = size_t(blockIdx.x) * kBlock + threadIdx.x;
  if (i >= col) return;
  const int j = blockIdx.y;
  const int n = n0 + j;
  const int K = (N + s - 1) / s;
  double v;
  if (j == 0 || n % s == 0 || n == N) {
    v = ck[size_t(ckpt_index(n, s, N, K)) * col + i];
  } else {
    const int k = (n - 1) / s;
    const int a = k * s, b = min((k + 1) * s, N);
    const double th = double(n - a) / double(b - a);
    const double va = ck[size_t(ckpt_index(a, s, N, K)) * col + i];
    const double vb = ck[size_t(ckpt_index(b, s, N, K)) * col + i];
    v = (1.0 - th) * va + th * vb;
  }
  out[size_t(j) * col + i] = v;
}

// Thread per element, loop over the steps of one chunk.  Vertex gradients g_a
// are constant on a simplex, so for a P1 field the element gradient is
// sum_a v_a g_a; the four sums are
//   tK = grad lp . grad p,  tL = div lu div u,  tM = grad lu : (grad u + grad u^T),
//   tB = grad lp . grad (p - p_prev),
// times |e| (the element matrices of C_K, the lambda and the mu parts of A).
template <int DIM>
__global__ __launch_bounds__(kBlock) void k_grad_partial(ElemDev E, size_t col,
                                                         const double* __restrict__ xbase,
                                                         int xstep0,
                                                         const double* __restrict__ lam_top,
                                                         int n_beg, int n_end, int chunk,
                                                         int kbase, double* __restrict__ part) {
  constexpr int D1 = DIM + 1;
  const int ne = E.ne;
  const int e = blockIdx.x * kBlock + threadIdx.x;
  if (e >= ne) return;
  const int y = blockIdx.y;
  const int nb = n_beg + y * chunk, nend = min(nb + chunk, n_end);
  int vid[D1];
  double g[D1][DIM];
#pragma unroll
  for (int a = 0; a < D1; ++a) {
    vid[a] = E.conn[size_t(a) * ne + e];
#pragma unroll
    for (int c = 0; c < DIM; ++c) g[a][c] = E.geo[size_t(a * DIM + c) * ne + e];
  }
  const double vol = E.geo[size_t(D1 * DIM) * ne + e];
  double gp_prev[DIM] = {};
  {
    const double* xp = xbase + size_t(nb - 1 - xstep0) * col;
#pragma unroll
    for (int a = 0; a < D1; ++a) {
      const double p = xp[size_t(vid[a]) * D1 + DIM];
#pragma unroll
      for (int c = 0; c < DIM; ++c) gp_prev[c] += p * g[a][c];
    }
  }
  double tK = 0.0, tL = 0.0, tM = 0.0, tB = 0.0;
#pragma unroll 1
  for (int n = nb; n < nend; ++n) {
    const double* x = xbase + size_t(n - xstep0) * col;
    const double* l = lam_top - size_t(n) * col;
    double gp[DIM] = {}, glp[DIM] = {}, Gu[DIM][DIM] = {}, Gl[DIM][DIM] = {};
#pragma unroll
    for (int a = 0; a < D1; ++a) {
      double xv[D1], lv[D1];
#pragma unroll
      for (int k = 0; k < D1; ++k) {
        xv[k] = x[size_t(vid[a]) * D1 + k];
        lv[k] = l[size_t(vid[a]) * D1 + k];
      }
#pragma unroll
      for (int d = 0; d < DIM; ++d) {
        gp[d] += xv[DIM] * g[a][d];
        glp[d] += lv[DIM] * g[a][d];
#pragma unroll
        for (int c = 0; c < DIM; ++c) {
          Gu[c][d] += xv[c] * g[a][d];
          Gl[c][d] += lv[c] * g[a][d];
        }
      }
    }
    double du = 0.0, dl = 0.0;
#pragma unroll
    for (int c = 0; c < DIM; ++c) {
      tK += glp[c] * gp[c];
      tB += glp[c] * (gp[c] - gp_prev[c]);
      gp_prev[c] = gp[c];
      du += Gu[c][c];
      dl += Gl[c][c];
#pragma unroll
      for (int d = 0; d < DIM; ++d) tM += Gl[c][d] * (Gu[c][d] + Gu[d][c]);
    }
    tL += dl * du;
  }
  double* o = part + size_t(kbase + y) * 4 * ne;
  o[e] = vol * tK;
  o[size_t(ne) + e] = vol * tL;
  o[size_t(2) * ne + e] = vol * tM;
  o[size_t(3) * ne + e] = vol * tB;
}

__global__ __launch_bounds__(kBlock) void k_grad_finish(ElemDev E, const double* __restrict__ part,
                                                        int nchunks, double* __restrict__ gk,
                                                        double* __restrict__ gl,
                                                        double* __restrict__ gm) {
  const int ne = E.ne;
  const int e = blockIdx.x * kBlock + threadIdx.x;
  if (e >= ne) return;
  double sK = 0.0, sL = 0.0, sM = 0.0, sB = 0.0;
  for (int k = 0; k < nchunks; ++k) {
    const double* p = part + size_t(k) * 4 * ne;
    sK += p[e];
    sL += p[size_t(ne) + e];
    sM += p[size_t(2) * ne + e];
    sB += p[size_t(3) * ne + e];
  }
  if (gk) gk[e] = E.coefK[e] * sK;
  if (gl) gl[e] = -sL + E.dbl[e] * sB;
  if (gm) gm[e] = -sM + E.dbm[e] * sB;
}

}  // namespace

void launch_sensor_load(int dim, int nn, int N, int S, const double* X, const int32_t* sens,
                        const double* pobs, const uint8_t* fixed, double* gload, double* jpart,
                        hipStream_t st) {
  const long total = long(N) * S;
  const dim3 g(unsigned((total + kBlock - 1) / kBlock));
  hipLaunchKernelGGL(k_sensor_load, g, dim3(kBlock), 0, st, nn, N, S, dim + 1, X, sens, pobs,
                     fixed, gload, jpart);
}

void launch_sum(const double* x, int n, double* out, hipStream_t st) {
  hipLaunchKernelGGL(k_sum, dim3(1), dim3(kBlock), 0, st, x, n, out);
}

void launch_lerp_init(size_t col, const double* ck, int s, int N, int n0, int L, double* out,
                      hipStream_t st) {
  const dim3 g(unsigned((col + kBlock - 1) / kBlock), unsigned(L + 1));
  hipLaunchKernelGGL(k_lerp_init, g, dim3(kBlock), 0, st, col, ck, s, N, n0, out);
}

void launch_grad_partial(int dim, const ElemDev& E, size_t col, const double* xbase, int xstep0,
                         const double* lam_top, int n_beg, int n_end, int chunk, int kbase,
                         double* part, hipStream_t st) {
  const int nchunk = (n_end - n_beg + chunk - 1) / chunk;
  const dim3 g(unsigned((E.ne + kBlock - 1) / kBlock), unsigned(nchunk));
  if (dim == 2)
    hipLaunchKernelGGL(k_grad_partial<2>, g, dim3(kBlock), 0, st, E, col, xbase, xstep0, lam_top,
                       n_beg, n_end, chunk, kbase, part);
  else
    hipLaunchKernelGGL(k_grad_partial<3>, g, dim3(kBlock), 0, st, E, col, xbase, xstep0, lam_top,
                       n_beg, n_end, chunk, kbase, part);
}

void launch_grad_finish(const ElemDev& E, const double* part, int nchunks, double* g_logk,
                        double* g_lam, double* g_mu, hipStream_t st) {
  const dim3 g(unsigned((E.ne + kBlock - 1) / kBlock));
  hipLaunchKernelGGL(k_grad_finish, g, dim3(kBlock), 0, st, E, part, nchunks, g_logk, g_lam, g_mu);
}

}  // namespace biot
