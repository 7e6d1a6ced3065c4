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
                             // (n_cells, nn1, nreal: those of copy 0; copies of a
                             // batch of uneven samples differ, see the tables below)
  // per copy (sample) on this level, largest grids first: first node (padded to
  // a multiple of 256 nodes, so no node block straddles two copies), cells per
  // side; and the copy of each block of 256 nodes
  std::vector<int32_t> cbase;  // [copies+1]
  std::vector<int32_t> ccells; // [copies]
  std::vector<int32_t> bcopy;  // [nn / 256]
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
  // right-hand side f^n = sum_j coef[n][j] terms[j] on the free dofs (Sec. 2.2:
  // f^n = [F^n; -tau G^n]), with the prescribed values lifted in: the kernels'
  // operators have the prescribed rows and columns eliminated, so the terms
  // carry -AA g^n and A' g^{n-1} of the prescribed values g (see build_problem)
  int nterms = 0;
  std::vector<double> terms;      // [nterms][nn][dim+1], zero at prescribed dofs
  std::vector<double> tcoef;      // [n_steps+1][nterms]
  // prescribed values g^n = sum_k pcoef[n][k] pres[k] at the prescribed dofs,
  // kept in the trajectory; X^0 = x0 (empty: g^0 at prescribed dofs, 0 elsewhere)
  int npres = 0;
  std::vector<double> pres;       // [npres][nn][dim+1] (values at prescribed dofs only)
  std::vector<double> pcoef;      // [n_steps+1][npres]
  std::vector<double> x0;         // [nn][dim+1] or empty
  std::vector<double> F;          // [nn][dim+1] traction load of a unit multiplier (export)
  std::vector<double> coarseAinv; // dense inverse of the coarsest A (node-major dofs), per copy
  std::vector<double> coarseSinv; // dense inverse of the coarsest S, per copy
  // batches: copy c holds sample sample_of[c] (largest grids first); per copy
  // its steps, its last (densely solved) level and the offsets of its dense
  // inverses in coarseAinv / coarseSinv
  std::vector<int32_t> sample_of; // [copies]
  std::vector<int32_t> csteps;    // [copies]
  std::vector<int32_t> clast;     // [copies]
  std::vector<int64_t> cAoff, cSoff;  // [copies]
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
  const double* coef;            // [n_steps+1] traction multiplier (may be null without facets)
  int n_terms;
  const double* terms;           // [n_terms][nn][dim+1]
  const double* term_coef;       // [n_steps+1][n_terms]
  int n_prescribed;
  const double* prescribed;      // [n_prescribed][nn][dim+1]
  const double* prescribed_coef; // [n_steps+1][n_prescribed]
  const double* x0;              // [nn][dim+1] or null
};
constexpr int kMaxUserTerms = 8;
constexpr int kMaxPrescribed = 3;
constexpr int kMaxTerms = 1 + kMaxUserTerms + 2 * kMaxPrescribed + 1;

// Returns an empty string on success, an error message otherwise.
std::string build_problem(const MeshIn& m, const MaterialsIn& mat, const LoadIn& ld,
                          double dt, int n_steps, const HostOptions& opt, HostProblem& out);

// Joins single-sample problems on structured meshes (of equal or different
// sizes) into one problem of parts.size() disconnected copies, largest grids
// first (stable).  Level l holds the copies whose hierarchy has a level l
// (their number is non-increasing with l, so they are a prefix).  Each copy's
// nodes are padded to a multiple of `pad` with inert nodes (prescribed in
// every component, identity diagonal, no neighbours, no load), so that blocks
// of `pad` nodes never straddle copies.  Spectral bounds of a level become the
// maximum over its copies.  All parts must have the
// same right-hand-side structure (number of load and prescribed terms, X^0
// given or not) and their coefficient tables must agree on their common steps
// (the result keeps the longest).
std::string concat_problems(const std::vector<HostProblem>& parts, int pad, HostProblem& out);

// Fills AD and SD of every level from A, S, their block inverses and nbr.
void fold_first_step(HostProblem& p);

// SplitMix64-based start vector in [0.5, 1.5) shared by the spectral bounds.
double splitmix_unit(uint64_t index);

}  // namespace biot
