// Device-side views and kernel launchers of the Biot parallel-in-time sweep.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace biot {

constexpr int kBlock = 256;   // threads per workgroup (4 wave64)

// One multigrid level on the device (node-blocked ELL, see setup.hpp).
struct LevelDev {
  int nn, W, n_cells;
  const int32_t* nbr;    // [W][nn]
  const double* A;       // [W][dim*dim][nn]
  const double* S;       // [W][nn]
  const double* Ainv;    // [dim*dim][nn]
  const double* Sinv;    // [nn]
  const uint8_t* fixed;  // [nn]
};

// Fine-level coupling blocks (level 0 only).
struct FineDev {
  const double* B;   // [W][dim][nn]
  const double* Bt;  // [W][dim][nn]
  const double* Cb;  // [W][nn]
  const double* F;   // [nn][dim+1]
};

// One (time step, iteration) column of a batch.
struct ColDesc {
  const double* xcur;   // X^{n,m-1}            [nn][dim+1]
  const double* xprev;  // coupling source X^{n-1,*}
  double* xout;         // X^{n,m}
  double* xout2;        // optional second copy (may be null)
  double coef;          // load multiplier of step n
  int step;             // n
  int pad;
};

// Launchers (all asynchronous on `st`).  `nc` = number of columns in the batch;
// per-column work vectors are contiguous with stride nn*comps.  `ct` = columns
// per thread in the node-blocked kernels (1, 2, 4 or 8).
bool valid_col_tile(int ct);
void launch_residual(int dim, const LevelDev& L, const FineDev& F, const ColDesc* cols, int nc,
                     double* ru, double* rp, double* xa, double* d, double inv_theta,
                     double* partials, int partial_stride, int ct, hipStream_t st);
// Chebyshev step; xc != null fuses the coarse-grid correction x += P xc (Lc =
// the coarse level); cols != null (pressure field, level 0) writes the outer
// update X^{n,m} = X^{n,m-1} + omega [zu; x_new] instead of xout.
void launch_cheb(int dim, int comps, const LevelDev& L, const LevelDev* Lc, bool is_A,
                 const double* b, const double* xin, const double* xc, double* xout, double* d,
                 int nc, double c1, double c2, const ColDesc* cols, const double* zu,
                 double omega, int ct, bool fine, hipStream_t st);
void launch_level_residual(int dim, int comps, const LevelDev& L, bool is_A, const double* b,
                           const double* x, double* r, int nc, int ct, hipStream_t st);
void launch_restrict(int dim, int comps, const LevelDev& Lf, const LevelDev& Lc, bool is_A,
                     const double* rf, double* bc, double* xa_c, double* d_c, double inv_theta_c,
                     int nc, hipStream_t st);
void launch_prolong(int dim, int comps, const LevelDev& Lf, const LevelDev& Lc, bool is_A,
                    const double* xin, const double* xc, double* xout, int nc, int ct,
                    hipStream_t st);
void launch_coarse_solve(int n, const double* Minv, const double* b, double* x, int nc,
                         hipStream_t st);
void launch_pstage(int dim, const LevelDev& L, const FineDev& F, bool p1, const double* zu,
                   const double* rp, double* t, double* xa, double* d, double inv_theta, int nc,
                   int ct, hipStream_t st);
void launch_update(int dim, int nn, const ColDesc* cols, const double* zu, const double* zp,
                   double omega, int nc, hipStream_t st);
void launch_reduce_norms(const double* partials, int nblk, int partial_stride, double* norms,
                         int nc, hipStream_t st);
void launch_apply_operator(int dim, const LevelDev& L, const FineDev& F, const double* X,
                           double* Y, int nc, hipStream_t st);
void launch_unpack(int dim, int nn, const double* X, double* ru, double* rp, int nc, hipStream_t st);
void launch_pre1(int comps, const LevelDev& L, bool is_A, const double* b, double* xa, double* d,
                 double inv_theta, int nc, hipStream_t st);
void launch_pack(int dim, int nn, const double* zu, const double* zp, double* Z, int nc,
                 hipStream_t st);

inline int num_node_blocks(int nn) { return (nn + kBlock - 1) / kBlock; }

}  // namespace biot
