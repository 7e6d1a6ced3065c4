// Host-side set-up of the Biot parallel-in-time solver: finite-element assembly,
// node-blocked ELL packing and the multigrid hierarchy.  Plain C++17, FP64.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

namespace biot {

// One level of the structured hierarchy, stored node-blocked: every node owns W
// slots; slot 0 is the node itself, unused slots point at the node and hold
// zero blocks.  Values are "slot-major, entry-major, node-minor": value e of
// slot k of node i lives at [(k*E + e)*nn + i], so consecutive threads (nodes)
// read consecutive addresses.
struct HostLevel {
  int n_cells = 0;           // cells per side
  int nn = 0;                // nodes (all copies, padding included)
  int copies = 1;            // samples stored as disconnected copies of the grid
  int nn1 = 0;               // nodes per copy, padding included (nn = copies * nn1)
  int nreal = 0;             // grid nodes per copy ((n_cells+1)^dim); the rest of a
                             // copy's nn1 are inert prescribed padding nodes
  int W = 0;                 // slots per node
  std::vector<int32_t> nbr;  // [W][nn]
  std::vector<double> A;     // [W][dim*dim][nn]  displacement block, entry a*dim+b
  std::vector<double> S;     // [W][nn]           pressure operator tau*C_K + C_beta
  std::vector<double> Ainv;  // [dim*dim][nn]     inverse of the node's A block
  std::vector<double> Sinv;  // [nn]
  std::vector<uint8_t> fixed;// [nn] bit c (<dim): u_c prescribed, bit dim: p prescribed
  // the operators with the neighbour's block-Jacobi inverse folded in, for the
  // smoothing step that follows a first step from zero (x = D^{-1} b / theta at
  // every node): AD_k(i) = A_k(i) Ainv(nbr_k(i)), SD_k(i) = S_k(i) Sinv(nbr_k(i))
  std::vector<double> AD;    // [W][dim*dim][nn]
  std::vector<double> SD;    // [W][nn]
  double lmaxA = 0, lmaxS = 0;  // spectral bounds of D^{-1}A and D^{-1}S (with safety)
  // fine level only
  std::vector<double> B;     // [W][dim][nn]  u-row / p-column coupling (matrix of -b)
  std::vector<double> Bt;    // [W][dim][nn]  p-row / u-column (transpose of B)
  std::vector<double> Cb;    // [W][nn]       stabilization matrix C_beta
};

struct HostOptions {
  int cheb_degree = 2;
  double cheb_ratio = 4.0;
  double lmax_safety = 1.1;
  int power_iters = 20;
  int min_cells = 2;
};

struct HostProblem {
  int dim = 2;
  int nn = 0, ne = 0;
  int n_steps = 0;
  double dt = 0, alpha = 1;
  std::vector<HostLevel> levels;
  std::vector<double> F;          // [nn][dim+1] load for a unit multiplier (p part zero)
  std::vector<double> coef;       // [n_steps+1]
  std::vector<double> coarseAinv; // dense inverse of the coarsest A (node-major dofs), per copy
  std::vector<double> coarseSinv; // dense inverse of the coarsest S, per copy
  std::vector<double> lambda_e, mu_e, beta_e, perm_e;  // per element
  bool beta_given = false;        // beta supplied by the caller (no lambda/mu dependence)
  // element geometry for the adjoint's gradient contraction, element-minor:
  // geo[(a*dim + c)*ne + e] = d(phi_a)/dx_c, geo[(dim+1)*dim*ne + e] = |e|
  std::vector<double> geo;
  std::vector<int32_t> conn_t;    // [dim+1][ne] vertex a of element e at [a*ne + e]
};

struct MeshIn {
  int dim, nn, ne, grid_n;
  const double* xyz;
  const int32_t* conn;
  const uint8_t* flags;
};
struct MaterialsIn {
  const double *young, *poisson, *perm, *beta;  // beta may be null
  double alpha, stab_h;
  const double *lame_lambda, *lame_mu;          // both null, or both set (override E, nu)
};
struct LoadIn {
  int n_facets;
  const int32_t* facet_nodes;
  const double* traction;
  const double* coef;
};

// Returns an empty string on success, an error message otherwise.
std::string build_problem(const MeshIn& m, const MaterialsIn& mat, const LoadIn& ld,
                          double dt, int n_steps, const HostOptions& opt, HostProblem& out);

// Joins single-sample problems on the same structured mesh into one problem of
// parts.size() disconnected copies.  Each copy's nodes are padded to a multiple
// of `pad` with inert nodes (prescribed in every component, identity diagonal,
// no neighbours, no load), so that blocks of `pad` nodes never straddle copies.
// Spectral bounds become the maximum over the copies.  The load multipliers of
// all parts must agree on their common steps (the result keeps the longest).
std::string concat_problems(const std::vector<HostProblem>& parts, int pad, HostProblem& out);

// Fills AD and SD of every level from A, S, their block inverses and nbr.
void fold_first_step(HostProblem& p);

// SplitMix64-based start vector in [0.5, 1.5) shared by the spectral bounds.
double splitmix_unit(uint64_t index);

}  // namespace biot
