// Host-side set-up: stabilized P1-P1 assembly of the Biot step matrix
// (paper Sec. 2.2, eq. (fullysystem)), node-blocked ELL packing, and the
// structured Galerkin multigrid hierarchy used to apply A^{-1} and S_p^{-1}
// inside the block preconditioners of Sec. 3.1.
#include "setup.hpp"

#include <algorithm>
#include <array>
#include <cmath>
#include <cstring>
#include <sstream>

namespace biot {
namespace {

// Stencil offsets of the P1 graph on the structured meshes.  2D: the grid is
// split along (i,j)->(i+1,j+1); 3D: Kuhn tetrahedra along (0,0,0)->(1,1,1).
// Slot 0 is the node itself.
constexpr int kOff2[7][3] = {{0, 0, 0}, {1, 0, 0}, {-1, 0, 0}, {0, 1, 0},
                             {0, -1, 0}, {1, 1, 0}, {-1, -1, 0}};
constexpr int kOff3[15][3] = {{0, 0, 0},  {1, 0, 0},  {-1, 0, 0},  {0, 1, 0},  {0, -1, 0},
                              {0, 0, 1},  {0, 0, -1}, {1, 1, 0},   {-1, -1, 0}, {1, 0, 1},
                              {-1, 0, -1}, {0, 1, 1}, {0, -1, -1}, {1, 1, 1},  {-1, -1, -1}};

struct Grid {
  int dim, n, m;  // cells, nodes per side
  int nn() const { return dim == 2 ? m * m : m * m * m; }
  void coords(int id, int& i, int& j, int& k) const {
    i = id % m;
    j = (id / m) % m;
    k = dim == 2 ? 0 : id / (m * m);
  }
  int id(int i, int j, int k) const { return dim == 2 ? j * m + i : (k * m + j) * m + i; }
  bool inside(int i, int j, int k) const {
    return i >= 0 && i < m && j >= 0 && j < m && k >= 0 && k < m;
  }
  int W() const { return dim == 2 ? 7 : 15; }
  const int* off(int s) const { return dim == 2 ? kOff2[s] : kOff3[s]; }
  // slot holding neighbour (di,dj,dk), or -1
  int slot_of(int di, int dj, int dk) const {
    for (int s = 0; s < W(); ++s) {
      const int* o = off(s);
      if (o[0] == di && o[1] == dj && o[2] == dk) return s;
    }
    return -1;
  }
};

void set_single_copy(HostLevel& L) {
  L.copies = 1;
  L.nn1 = L.nn;
  L.nreal = L.nn;
  L.cbase = {0, L.nn};
  L.ccells = {L.n_cells};
  L.bcopy.assign(size_t((L.nn + 255) / 256), 0);
}

void init_level(HostLevel& L, const Grid& g, int dim) {
  L.n_cells = g.n;
  L.nn = g.nn();
  set_single_copy(L);
  L.W = g.W();
  L.nbr.assign(size_t(L.W) * L.nn, 0);
  for (int v = 0; v < L.nn; ++v) {
    int i, j, k;
    g.coords(v, i, j, k);
    for (int s = 0; s < L.W; ++s) {
      const int* o = g.off(s);
      int ii = i + o[0], jj = j + o[1], kk = k + o[2];
      L.nbr[size_t(s) * L.nn + v] = g.inside(ii, jj, kk) ? g.id(ii, jj, kk) : v;
    }
  }
  const size_t dd = size_t(dim) * dim;
  L.A.assign(L.W * dd * L.nn, 0.0);
  L.S.assign(size_t(L.W) * L.nn, 0.0);
  L.fixed.assign(L.nn, 0);
}

inline double& Aat(HostLevel& L, int dim, int s, int a, int b, int v) {
  return L.A[(size_t(s) * dim * dim + a * dim + b) * L.nn + v];
}
inline double& Sat(HostLevel& L, int s, int v) { return L.S[size_t(s) * L.nn + v]; }

// inverse of a small dense matrix (Gauss-Jordan, partial pivoting); false if singular
bool invert(std::vector<double>& M, int n) {
  std::vector<double> I(size_t(n) * n, 0.0);
  for (int i = 0; i < n; ++i) I[size_t(i) * n + i] = 1.0;
  for (int c = 0; c < n; ++c) {
    int p = c;
    for (int r = c + 1; r < n; ++r)
      if (std::fabs(M[size_t(r) * n + c]) > std::fabs(M[size_t(p) * n + c])) p = r;
    if (M[size_t(p) * n + c] == 0.0) return false;
    if (p != c)
      for (int k = 0; k < n; ++k) {
        std::swap(M[size_t(p) * n + k], M[size_t(c) * n + k]);
        std::swap(I[size_t(p) * n + k], I[size_t(c) * n + k]);
      }
    double inv = 1.0 / M[size_t(c) * n + c];
    for (int k = 0; k < n; ++k) {
      M[size_t(c) * n + k] *= inv;
      I[size_t(c) * n + k] *= inv;
    }
    for (int r = 0; r < n; ++r) {
      if (r == c) continue;
      double f = M[size_t(r) * n + c];
      if (f == 0.0) continue;
      for (int k = 0; k < n; ++k) {
        M[size_t(r) * n + k] -= f * M[size_t(c) * n + k];
        I[size_t(r) * n + k] -= f * I[size_t(c) * n + k];
      }
    }
  }
  M.swap(I);
  return true;
}

// Zero rows and columns of prescribed dofs, unit diagonal (A part).
void fix_A(HostLevel& L, int dim) {
  for (int v = 0; v < L.nn; ++v)
    for (int s = 0; s < L.W; ++s) {
      int w = L.nbr[size_t(s) * L.nn + v];
      for (int a = 0; a < dim; ++a)
        for (int b = 0; b < dim; ++b) {
          bool rf = (L.fixed[v] >> a) & 1, cf = (L.fixed[w] >> b) & 1;
          if (rf || cf) Aat(L, dim, s, a, b, v) = 0.0;
        }
    }
  for (int v = 0; v < L.nn; ++v)
    for (int a = 0; a < dim; ++a)
      if ((L.fixed[v] >> a) & 1) Aat(L, dim, 0, a, a, v) = 1.0;
}

void fix_S(HostLevel& L, int dim) {
  for (int v = 0; v < L.nn; ++v)
    for (int s = 0; s < L.W; ++s) {
      int w = L.nbr[size_t(s) * L.nn + v];
      if (((L.fixed[v] >> dim) & 1) || ((L.fixed[w] >> dim) & 1)) Sat(L, s, v) = 0.0;
    }
  for (int v = 0; v < L.nn; ++v)
    if ((L.fixed[v] >> dim) & 1) Sat(L, 0, v) = 1.0;
}

// the slot-0 (boundary-padded) neighbours must not contribute: padded slots carry
// zero values by construction, so y = K x just loops over all slots.
void matvec_A(const HostLevel& L, int dim, const std::vector<double>& x, std::vector<double>& y) {
  y.assign(size_t(L.nn) * dim, 0.0);
  for (int v = 0; v < L.nn; ++v)
    for (int s = 0; s < L.W; ++s) {
      int w = L.nbr[size_t(s) * L.nn + v];
      for (int a = 0; a < dim; ++a) {
        double acc = 0;
        for (int b = 0; b < dim; ++b)
          acc += L.A[(size_t(s) * dim * dim + a * dim + b) * L.nn + v] * x[size_t(w) * dim + b];
        y[size_t(v) * dim + a] += acc;
      }
    }
}

void matvec_S(const HostLevel& L, const std::vector<double>& x, std::vector<double>& y) {
  y.assign(L.nn, 0.0);
  for (int v = 0; v < L.nn; ++v)
    for (int s = 0; s < L.W; ++s) y[v] += L.S[size_t(s) * L.nn + v] * x[L.nbr[size_t(s) * L.nn + v]];
}

// Power iteration for lambda_max(D^{-1}K): Rayleigh quotient in the K inner
// product after `iters` steps from the SplitMix64 start vector.
double power_A(const HostLevel& L, int dim, int iters) {
  size_t n = size_t(L.nn) * dim;
  std::vector<double> x(n), Kx, y(n);
  for (size_t i = 0; i < n; ++i) x[i] = splitmix_unit(i);
  double lam = 0;
  for (int it = 0; it < iters; ++it) {
    matvec_A(L, dim, x, Kx);
    for (int v = 0; v < L.nn; ++v)
      for (int a = 0; a < dim; ++a) {
        double acc = 0;
        for (int b = 0; b < dim; ++b)
          acc += L.Ainv[size_t(a * dim + b) * L.nn + v] * Kx[size_t(v) * dim + b];
        y[size_t(v) * dim + a] = acc;
      }
    double num = 0, den = 0, nrm = 0;
    for (size_t i = 0; i < n; ++i) {
      num += y[i] * Kx[i];
      den += x[i] * Kx[i];
      nrm += y[i] * y[i];
    }
    lam = num / den;
    nrm = std::sqrt(nrm);
    for (size_t i = 0; i < n; ++i) x[i] = y[i] / nrm;
  }
  return lam;
}

double power_S(const HostLevel& L, int iters) {
  size_t n = L.nn;
  std::vector<double> x(n), Kx, y(n);
  for (size_t i = 0; i < n; ++i) x[i] = splitmix_unit(i);
  double lam = 0;
  for (int it = 0; it < iters; ++it) {
    matvec_S(L, x, Kx);
    double num = 0, den = 0, nrm = 0;
    for (size_t i = 0; i < n; ++i) {
      y[i] = L.Sinv[i] * Kx[i];
      num += y[i] * Kx[i];
      den += x[i] * Kx[i];
      nrm += y[i] * y[i];
    }
    lam = num / den;
    nrm = std::sqrt(nrm);
    for (size_t i = 0; i < n; ++i) x[i] = y[i] / nrm;
  }
  return lam;
}

void block_inverses(HostLevel& L, int dim) {
  L.Ainv.assign(size_t(dim) * dim * L.nn, 0.0);
  L.Sinv.assign(L.nn, 0.0);
  std::vector<double> M(size_t(dim) * dim);
  for (int v = 0; v < L.nn; ++v) {
    for (int a = 0; a < dim; ++a)
      for (int b = 0; b < dim; ++b) M[a * dim + b] = L.A[(size_t(a * dim + b)) * L.nn + v];
    if (!invert(M, dim)) M.assign(M.size(), 0.0);
    for (int e = 0; e < dim * dim; ++e) L.Ainv[size_t(e) * L.nn + v] = M[e];
    double d = L.S[v];
    L.Sinv[v] = d != 0.0 ? 1.0 / d : 0.0;
  }
}

// Parents of a fine node under 2:1 P1 coarsening: fine index f = 2a + o per
// axis; the parents are coarse a (and a+o when o != 0), weight 1 or 1/2 each.
int parents(const Grid& gf, const Grid& gc, int v, int* pid, double* pw) {
  int i, j, k;
  gf.coords(v, i, j, k);
  int ai = i >> 1, aj = j >> 1, ak = k >> 1;
  int oi = i & 1, oj = j & 1, ok = k & 1;
  pid[0] = gc.id(ai, aj, ak);
  if (oi == 0 && oj == 0 && ok == 0) {
    pw[0] = 1.0;
    return 1;
  }
  pw[0] = 0.5;
  pid[1] = gc.id(ai + oi, aj + oj, ak + ok);
  pw[1] = 0.5;
  return 2;
}

std::string coarsen(const HostLevel& F, const Grid& gf, HostLevel& C, const Grid& gc, int dim) {
  init_level(C, gc, dim);
  // coarse prescribed flags: injection from the coincident fine node
  for (int v = 0; v < C.nn; ++v) {
    int i, j, k;
    gc.coords(v, i, j, k);
    C.fixed[v] = F.fixed[gf.id(2 * i, 2 * j, 2 * k)];
  }
  int pid_f[2], pid_g[2];
  double pw_f[2], pw_g[2];
  for (int f = 0; f < F.nn; ++f) {
    int np_f = parents(gf, gc, f, pid_f, pw_f);
    for (int s = 0; s < F.W; ++s) {
      int g = F.nbr[size_t(s) * F.nn + f];
      if (s != 0 && g == f) continue;  // padded slot
      int np_g = parents(gf, gc, g, pid_g, pw_g);
      for (int pi = 0; pi < np_f; ++pi) {
        int I = pid_f[pi];
        int Ii, Ij, Ik;
        gc.coords(I, Ii, Ij, Ik);
        for (int pj = 0; pj < np_g; ++pj) {
          int J = pid_g[pj];
          int Ji, Jj, Jk;
          gc.coords(J, Ji, Jj, Jk);
          int cs = gc.slot_of(Ji - Ii, Jj - Ij, Jk - Ik);
          double w = pw_f[pi] * pw_g[pj];
          // A part, per component pair with the prolongation masks
          for (int a = 0; a < dim; ++a)
            for (int b = 0; b < dim; ++b) {
              double val = F.A[(size_t(s) * dim * dim + a * dim + b) * F.nn + f];
              if (val == 0.0) continue;
              bool m = ((F.fixed[f] >> a) & 1) || ((F.fixed[g] >> b) & 1) ||
                       ((C.fixed[I] >> a) & 1) || ((C.fixed[J] >> b) & 1);
              if (m) continue;
              if (cs < 0) return "Galerkin product leaves the coarse stencil";
              Aat(C, dim, cs, a, b, I) += w * val;
            }
          double sv = F.S[size_t(s) * F.nn + f];
          if (sv != 0.0) {
            bool m = ((F.fixed[f] >> dim) & 1) || ((F.fixed[g] >> dim) & 1) ||
                     ((C.fixed[I] >> dim) & 1) || ((C.fixed[J] >> dim) & 1);
            if (!m) {
              if (cs < 0) return "Galerkin product leaves the coarse stencil";
              Sat(C, cs, I) += w * sv;
            }
          }
        }
      }
    }
  }
  fix_A(C, dim);
  fix_S(C, dim);
  return "";
}

// Simplex gradients and measure (P1): rows of J^{-1}, J = [x1-x0, ..., xd-x0].
bool simplex(int dim, const double* xv, double* grads, double& vol) {
  double J[3][3] = {{0}};
  for (int c = 0; c < dim; ++c)        // column c = x_{c+1} - x_0
    for (int r = 0; r < dim; ++r) J[r][c] = xv[(c + 1) * dim + r] - xv[r];
  double det, inv[3][3];
  if (dim == 2) {
    det = J[0][0] * J[1][1] - J[0][1] * J[1][0];
    if (!(det > 0)) return false;
    inv[0][0] = J[1][1] / det;
    inv[0][1] = -J[0][1] / det;
    inv[1][0] = -J[1][0] / det;
    inv[1][1] = J[0][0] / det;
    vol = det / 2.0;
  } else {
    det = J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1]) -
          J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0]) +
          J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
    if (!(det > 0)) return false;
    inv[0][0] = (J[1][1] * J[2][2] - J[1][2] * J[2][1]) / det;
    inv[0][1] = (J[0][2] * J[2][1] - J[0][1] * J[2][2]) / det;
    inv[0][2] = (J[0][1] * J[1][2] - J[0][2] * J[1][1]) / det;
    inv[1][0] = (J[1][2] * J[2][0] - J[1][0] * J[2][2]) / det;
    inv[1][1] = (J[0][0] * J[2][2] - J[0][2] * J[2][0]) / det;
    inv[1][2] = (J[0][2] * J[1][0] - J[0][0] * J[1][2]) / det;
    inv[2][0] = (J[1][0] * J[2][1] - J[1][1] * J[2][0]) / det;
    inv[2][1] = (J[0][1] * J[2][0] - J[0][0] * J[2][1]) / det;
    inv[2][2] = (J[0][0] * J[1][1] - J[0][1] * J[1][0]) / det;
    vol = det / 6.0;
  }
  // gradient of barycentric coordinate a (a>=1) = row a-1 of J^{-1}
  for (int c = 0; c < dim; ++c) {
    double s = 0;
    for (int a = 1; a <= dim; ++a) {
      grads[a * dim + c] = inv[a - 1][c];
      s += inv[a - 1][c];
    }
    grads[c] = -s;
  }
  return true;
}

}  // namespace

double splitmix_unit(uint64_t index) {
  uint64_t z = (index + 1) * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  z = z ^ (z >> 31);
  return 0.5 + double(z >> 11) / 9007199254740992.0;
}

std::string build_problem(const MeshIn& m, const MaterialsIn& mat, const LoadIn& ld, double dt,
                          int n_steps, const HostOptions& opt, HostProblem& P) {
  const int dim = m.dim;
  if (dim != 2 && dim != 3) return "dim must be 2 or 3";
  if (m.nn <= 0 || m.ne <= 0 || !m.xyz || !m.conn || !m.flags) return "empty or null mesh arrays";
  if (!mat.perm) return "null permeability array";
  if ((mat.lame_lambda == nullptr) != (mat.lame_mu == nullptr))
    return "lame_lambda and lame_mu must be given together";
  if (!mat.lame_lambda && (!mat.young || !mat.poisson)) return "null material arrays";
  if (!(dt > 0) || n_steps < 1) return "dt must be > 0 and n_steps >= 1";
  if (m.grid_n < 1) return "only structured meshes (grid_n >= 1) are supported";
  if (!(mat.stab_h >= 0) || !std::isfinite(mat.alpha)) return "bad alpha or stab_h";
  if (ld.n_facets < 0 || (ld.n_facets > 0 && (!ld.facet_nodes || !ld.traction)))
    return "bad load facets";
  if (ld.n_facets > 0 && !ld.coef) return "null load coefficients";
  if (ld.n_terms < 0 || ld.n_terms > kMaxUserTerms) return "n_terms must be in 0..8";
  if (ld.n_terms > 0 && (!ld.terms || !ld.term_coef)) return "null load terms or term coefficients";
  if (ld.n_prescribed < 0 || ld.n_prescribed > kMaxPrescribed) return "n_prescribed must be in 0..3";
  if (ld.n_prescribed > 0 && (!ld.prescribed || !ld.prescribed_coef))
    return "null prescribed values or their coefficients";
  {
    const size_t nd = size_t(m.nn) * (dim + 1), ns = size_t(n_steps) + 1;
    auto finite = [](const double* a, size_t n) {
      for (size_t i = 0; i < n; ++i)
        if (!std::isfinite(a[i])) return false;
      return true;
    };
    if ((ld.n_facets > 0 && !finite(ld.coef, ns)) ||
        (ld.n_terms > 0 && (!finite(ld.terms, nd * ld.n_terms) ||
                            !finite(ld.term_coef, ns * ld.n_terms))) ||
        (ld.n_prescribed > 0 && (!finite(ld.prescribed, nd * ld.n_prescribed) ||
                                 !finite(ld.prescribed_coef, ns * ld.n_prescribed))) ||
        (ld.x0 && !finite(ld.x0, nd)))
      return "non-finite load, prescribed value, coefficient or initial state";
  }
  if (opt.cheb_degree < 1 || opt.cheb_degree > 8) return "cheb_degree must be in 1..8";
  if (!(opt.cheb_ratio > 1.0)) return "cheb_ratio must be > 1";

  Grid g0{dim, m.grid_n, m.grid_n + 1};
  if (g0.nn() != m.nn) return "n_nodes does not match grid_n";
  // the nodes must be the lexicographic structured grid on the unit square/cube
  for (int v = 0; v < m.nn; ++v) {
    int i, j, k;
    g0.coords(v, i, j, k);
    double e[3] = {double(i) / g0.n, double(j) / g0.n, double(k) / g0.n};
    for (int c = 0; c < dim; ++c)
      if (std::fabs(m.xyz[size_t(v) * dim + c] - e[c]) > 1e-9) return "mesh nodes are not the structured grid";
  }
  P.dim = dim;
  P.nn = m.nn;
  P.ne = m.ne;
  P.n_steps = n_steps;
  P.dt = dt;
  P.alpha = mat.alpha;
  P.levels.clear();
  P.levels.emplace_back();
  HostLevel& L = P.levels[0];
  init_level(L, g0, dim);
  for (int v = 0; v < m.nn; ++v) L.fixed[v] = m.flags[v] & uint8_t((1u << (dim + 1)) - 1);
  L.B.assign(size_t(L.W) * dim * L.nn, 0.0);
  L.Bt.assign(size_t(L.W) * dim * L.nn, 0.0);
  L.Cb.assign(size_t(L.W) * L.nn, 0.0);
  std::vector<double> CK(size_t(L.W) * L.nn, 0.0);

  P.lambda_e.resize(m.ne);
  P.mu_e.resize(m.ne);
  P.beta_e.resize(m.ne);
  P.perm_e.resize(m.ne);
  P.beta_given = mat.beta != nullptr;
  P.geo.assign(size_t((dim + 1) * dim + 1) * m.ne, 0.0);
  P.conn_t.assign(size_t(dim + 1) * m.ne, 0);
  const int nv = dim + 1;
  double xv[12], gr[12];
  int slot[4][4];
  for (int e = 0; e < m.ne; ++e) {
    const int32_t* cv = m.conn + size_t(e) * nv;
    for (int a = 0; a < nv; ++a) {
      if (cv[a] < 0 || cv[a] >= m.nn) return "connectivity out of range";
      for (int c = 0; c < dim; ++c) xv[a * dim + c] = m.xyz[size_t(cv[a]) * dim + c];
    }
    double vol;
    if (!simplex(dim, xv, gr, vol)) return "inverted or degenerate element";
    for (int a = 0; a < nv; ++a) {
      int ia, ja, ka;
      g0.coords(cv[a], ia, ja, ka);
      for (int b = 0; b < nv; ++b) {
        int ib, jb, kb;
        g0.coords(cv[b], ib, jb, kb);
        slot[a][b] = g0.slot_of(ib - ia, jb - ja, kb - ka);
        if (slot[a][b] < 0) return "element edge is not on the structured stencil";
      }
    }
    const double K = mat.perm[e];
    double lam, mu;
    if (mat.lame_lambda) {
      lam = mat.lame_lambda[e];
      mu = mat.lame_mu[e];
      if (!(mu > 0) || !(lam > -2.0 * mu / dim) || !(K >= 0) || !std::isfinite(lam) ||
          !std::isfinite(mu))
        return "bad material value";
    } else {
      double E = mat.young[e], nu = mat.poisson[e];
      if (!(E > 0) || !(nu > -1 && nu < 0.5) || !(K >= 0)) return "bad material value";
      lam = E * nu / ((1 + nu) * (1 - 2 * nu));
      mu = E / (2 * (1 + nu));
    }
    double beta = mat.beta ? mat.beta[e]
                           : mat.alpha * mat.alpha * mat.stab_h * mat.stab_h / (4 * (lam + 2 * mu));
    P.lambda_e[e] = lam;
    P.mu_e[e] = mu;
    P.beta_e[e] = beta;
    P.perm_e[e] = K;
    for (int a = 0; a < nv; ++a) {
      P.conn_t[size_t(a) * m.ne + e] = cv[a];
      for (int c = 0; c < dim; ++c) P.geo[size_t(a * dim + c) * m.ne + e] = gr[a * dim + c];
    }
    P.geo[size_t(nv * dim) * m.ne + e] = vol;
    for (int a = 0; a < nv; ++a) {
      const double* ga = gr + a * dim;
      int va = cv[a];
      for (int b = 0; b < nv; ++b) {
        const double* gb = gr + b * dim;
        int s = slot[a][b];
        double gg = 0;
        for (int c = 0; c < dim; ++c) gg += ga[c] * gb[c];
        // a(u,v) = int 2mu eps:eps + lam div div
        for (int c = 0; c < dim; ++c)
          for (int d = 0; d < dim; ++d) {
            double val = mu * ga[d] * gb[c] + lam * ga[c] * gb[d];
            if (c == d) val += mu * gg;
            Aat(L, dim, s, c, d, va) += vol * val;
          }
        // B[(a,c), b] = -alpha g_a[c] vol/(d+1); B' [b, (a,c)] is its transpose
        for (int c = 0; c < dim; ++c) {
          L.B[(size_t(s) * dim + c) * L.nn + va] += -mat.alpha * ga[c] * vol / nv;
          // row b (p), column a (u): stored in row cv[b] at the slot of a in b's list
          L.Bt[(size_t(slot[b][a]) * dim + c) * L.nn + cv[b]] += -mat.alpha * ga[c] * vol / nv;
        }
        CK[size_t(s) * L.nn + va] += K * vol * gg;
        L.Cb[size_t(s) * L.nn + va] += beta * vol * gg;
      }
    }
  }
  for (size_t i = 0; i < L.S.size(); ++i) L.S[i] = dt * CK[i] + L.Cb[i];
  // Prescribed values are lifted into the right-hand side with the operators
  // as assembled (before the elimination below): on the free rows, step n's
  // equation AA X^n = A' X^{n-1} + f^n holds with X^n = (x_free, g^n), so
  //   AA_ff x_free = f^n_f - (AA g^n)_f + (A' g^{n-1})_f + A'_ff X^{n-1}_free.
  // Each prescribed term k (g^n = sum_k d_k(n) G_k) gives two load terms,
  // -AA G_k with coefficient d_k(n) and A' G_k with d_k(n-1); an X^0 whose
  // prescribed part differs from g^0 adds A' (X^0 - g^0) at step 1 only.
  std::vector<std::vector<double>> tv;   // load terms [nn][dim+1]
  std::vector<std::vector<double>> tc;   // their coefficients [n_steps+1]
  const int D1 = dim + 1;
  const size_t nd = size_t(m.nn) * D1;
  auto fixed_dof = [&](int v, int c) { return ((L.fixed[v] >> c) & 1) != 0; };
  // y = AA g and yp = A' g with the unreduced level-0 blocks
  auto apply_full = [&](const std::vector<double>& g, std::vector<double>& y,
                        std::vector<double>& yp) {
    y.assign(nd, 0.0);
    yp.assign(nd, 0.0);
    for (int v = 0; v < L.nn; ++v)
      for (int sl = 0; sl < L.W; ++sl) {
        const int w = L.nbr[size_t(sl) * L.nn + v];
        const double* gw = &g[size_t(w) * D1];
        for (int a = 0; a < dim; ++a) {
          double acc = L.B[(size_t(sl) * dim + a) * L.nn + v] * gw[dim];
          for (int b = 0; b < dim; ++b) acc += Aat(L, dim, sl, a, b, v) * gw[b];
          y[size_t(v) * D1 + a] += acc;
        }
        double btg = 0.0;
        for (int c = 0; c < dim; ++c) btg += L.Bt[(size_t(sl) * dim + c) * L.nn + v] * gw[c];
        y[size_t(v) * D1 + dim] += btg - L.S[size_t(sl) * L.nn + v] * gw[dim];
        yp[size_t(v) * D1 + dim] += btg - L.Cb[size_t(sl) * L.nn + v] * gw[dim];
      }
  };
  auto masked = [&](const double* src, bool keep_fixed) {  // keep only fixed or only free dofs
    std::vector<double> out(nd, 0.0);
    for (int v = 0; v < m.nn; ++v)
      for (int c = 0; c < D1; ++c)
        if (fixed_dof(v, c) == keep_fixed) out[size_t(v) * D1 + c] = src[size_t(v) * D1 + c];
    return out;
  };
  const size_t ns = size_t(n_steps) + 1;
  P.npres = ld.n_prescribed;
  P.pres.assign(nd * P.npres, 0.0);
  P.pcoef.assign(ns * P.npres, 0.0);
  std::vector<double> gz(nd, 0.0);  // g^0
  for (int k = 0; k < P.npres; ++k) {
    std::vector<double> G = masked(ld.prescribed + nd * k, true);
    std::copy(G.begin(), G.end(), P.pres.begin() + nd * k);
    std::vector<double> d(ns);
    for (size_t n = 0; n < ns; ++n) {
      d[n] = ld.prescribed_coef[n * P.npres + k];
      P.pcoef[n * P.npres + k] = d[n];
    }
    for (size_t i = 0; i < nd; ++i) gz[i] += d[0] * G[i];
    std::vector<double> y, yp;
    apply_full(G, y, yp);
    for (double& x : y) x = -x;
    std::vector<double> dprev(ns, 0.0);
    for (size_t n = 1; n < ns; ++n) dprev[n] = d[n - 1];
    tv.push_back(masked(y.data(), false));
    tc.push_back(d);
    tv.push_back(masked(yp.data(), false));
    tc.push_back(dprev);
  }
  P.x0.clear();
  if (ld.x0) {
    P.x0.assign(ld.x0, ld.x0 + nd);
    std::vector<double> dx = masked(ld.x0, true);
    bool nz = false;
    for (size_t i = 0; i < nd; ++i) {
      dx[i] -= gz[i];
      nz = nz || dx[i] != 0.0;
    }
    if (nz && n_steps >= 1) {
      std::vector<double> y, yp;
      apply_full(dx, y, yp);
      std::vector<double> c1(ns, 0.0);
      c1[1] = 1.0;
      tv.push_back(masked(yp.data(), false));
      tc.push_back(c1);
    }
  }
  // prescribed dofs: zero rows/columns of every block touching them
  for (int v = 0; v < L.nn; ++v)
    for (int s = 0; s < L.W; ++s) {
      int w = L.nbr[size_t(s) * L.nn + v];
      bool pv = (L.fixed[v] >> dim) & 1, pw = (L.fixed[w] >> dim) & 1;
      for (int c = 0; c < dim; ++c) {
        bool uv = (L.fixed[v] >> c) & 1, uw = (L.fixed[w] >> c) & 1;
        if (uv || pw) L.B[(size_t(s) * dim + c) * L.nn + v] = 0.0;
        if (pv || uw) L.Bt[(size_t(s) * dim + c) * L.nn + v] = 0.0;
      }
      if (pv || pw) L.Cb[size_t(s) * L.nn + v] = 0.0;
    }
  fix_A(L, dim);
  fix_S(L, dim);

  // load: constant traction per facet, |facet|/dim to each of its vertices
  P.F.assign(size_t(m.nn) * (dim + 1), 0.0);
  for (int f = 0; f < ld.n_facets; ++f) {
    const int32_t* fv = ld.facet_nodes + size_t(f) * dim;
    double p0[3], p1[3], p2[3] = {0, 0, 0};
    for (int a = 0; a < dim; ++a)
      if (fv[a] < 0 || fv[a] >= m.nn) return "facet node out of range";
    for (int c = 0; c < dim; ++c) {
      p0[c] = m.xyz[size_t(fv[0]) * dim + c];
      p1[c] = m.xyz[size_t(fv[1]) * dim + c];
      if (dim == 3) p2[c] = m.xyz[size_t(fv[2]) * dim + c];
    }
    double meas;
    if (dim == 2) {
      meas = std::hypot(p1[0] - p0[0], p1[1] - p0[1]);
    } else {
      double u[3] = {p1[0] - p0[0], p1[1] - p0[1], p1[2] - p0[2]};
      double w[3] = {p2[0] - p0[0], p2[1] - p0[1], p2[2] - p0[2]};
      double cx = u[1] * w[2] - u[2] * w[1], cy = u[2] * w[0] - u[0] * w[2], cz = u[0] * w[1] - u[1] * w[0];
      meas = 0.5 * std::sqrt(cx * cx + cy * cy + cz * cz);
    }
    for (int a = 0; a < dim; ++a)
      for (int c = 0; c < dim; ++c)
        P.F[size_t(fv[a]) * (dim + 1) + c] += ld.traction[size_t(f) * dim + c] * meas / dim;
  }
  for (int v = 0; v < m.nn; ++v)
    for (int c = 0; c < dim; ++c)
      if ((L.fixed[v] >> c) & 1) P.F[size_t(v) * (dim + 1) + c] = 0.0;
  // internal load terms: the traction first (kept in registers by the
  // residual kernel), then the caller's terms, then the lifting terms
  {
    std::vector<std::vector<double>> all_v, all_c;
    if (ld.n_facets > 0) {
      all_v.push_back(P.F);
      all_c.emplace_back(ld.coef, ld.coef + ns);
    }
    for (int j = 0; j < ld.n_terms; ++j) {
      all_v.push_back(masked(ld.terms + nd * j, false));
      std::vector<double> c(ns);
      for (size_t n = 0; n < ns; ++n) c[n] = ld.term_coef[n * ld.n_terms + j];
      all_c.push_back(std::move(c));
    }
    for (size_t j = 0; j < tv.size(); ++j) {
      all_v.push_back(std::move(tv[j]));
      all_c.push_back(std::move(tc[j]));
    }
    P.nterms = int(all_v.size());
    P.terms.assign(nd * P.nterms, 0.0);
    P.tcoef.assign(ns * P.nterms, 0.0);
    for (int j = 0; j < P.nterms; ++j) {
      std::copy(all_v[j].begin(), all_v[j].end(), P.terms.begin() + nd * j);
      for (size_t n = 0; n < ns; ++n) P.tcoef[n * P.nterms + j] = all_c[j][n];
    }
  }

  // multigrid hierarchy: halve while even and at least min_cells remain
  std::vector<Grid> grids{g0};
  while (grids.back().n % 2 == 0 && grids.back().n / 2 >= opt.min_cells) {
    int nc = grids.back().n / 2;
    grids.push_back(Grid{dim, nc, nc + 1});
  }
  for (size_t l = 1; l < grids.size(); ++l) {
    P.levels.emplace_back();
    std::string err = coarsen(P.levels[l - 1], grids[l - 1], P.levels[l], grids[l], dim);
    if (!err.empty()) return err;
  }
  for (auto& Lv : P.levels) {
    block_inverses(Lv, dim);
  }
  for (size_t l = 0; l + 1 < P.levels.size(); ++l) {
    P.levels[l].lmaxA = opt.lmax_safety * power_A(P.levels[l], dim, opt.power_iters);
    P.levels[l].lmaxS = opt.lmax_safety * power_S(P.levels[l], opt.power_iters);
  }
  // coarsest level: dense inverses
  HostLevel& Lc = P.levels.back();
  {
    int n = Lc.nn * dim;
    std::vector<double> M(size_t(n) * n, 0.0);
    for (int v = 0; v < Lc.nn; ++v)
      for (int s = 0; s < Lc.W; ++s) {
        int w = Lc.nbr[size_t(s) * Lc.nn + v];
        if (s != 0 && w == v) continue;
        for (int a = 0; a < dim; ++a)
          for (int b = 0; b < dim; ++b)
            M[size_t(v * dim + a) * n + w * dim + b] += Lc.A[(size_t(s) * dim * dim + a * dim + b) * Lc.nn + v];
      }
    if (!invert(M, n)) return "coarsest displacement operator is singular";
    P.coarseAinv.swap(M);
    int ns = Lc.nn;
    std::vector<double> Ms(size_t(ns) * ns, 0.0);
    for (int v = 0; v < Lc.nn; ++v)
      for (int s = 0; s < Lc.W; ++s) {
        int w = Lc.nbr[size_t(s) * Lc.nn + v];
        if (s != 0 && w == v) continue;
        Ms[size_t(v) * ns + w] += Lc.S[size_t(s) * Lc.nn + v];
      }
    if (!invert(Ms, ns)) return "coarsest pressure operator is singular";
    P.coarseSinv.swap(Ms);
  }
  P.sample_of = {0};
  P.csteps = {n_steps};
  P.clast = {int(P.levels.size()) - 1};
  P.cAoff = {0};
  P.cSoff = {0};
  return "";
}

std::string concat_problems(const std::vector<HostProblem>& parts, int pad, HostProblem& P) {
  if (parts.empty()) return "no samples";
  const HostProblem& p0 = parts[0];
  const int S = int(parts.size()), dim = p0.dim, D1 = dim + 1;
  for (const HostProblem& q : parts) {
    if (q.dim != dim || q.levels.empty() || q.levels[0].copies != 1)
      return "samples of a batch must be single problems of the same dimension";
    if (q.nterms != p0.nterms || q.npres != p0.npres || q.x0.empty() != p0.x0.empty())
      return "samples of a batch must have the same load, prescribed-value and initial-state structure";
    const size_t nmin = std::min(q.tcoef.size(), p0.tcoef.size());
    for (size_t n = 0; n < nmin; ++n)
      if (q.tcoef[n] != p0.tcoef[n]) return "load multipliers of a batch must agree step by step";
    const size_t pmin = std::min(q.pcoef.size(), p0.pcoef.size());
    for (size_t n = 0; n < pmin; ++n)
      if (q.pcoef[n] != p0.pcoef[n])
        return "prescribed-value multipliers of a batch must agree step by step";
  }
  // copies: largest grids first (stable); a deeper hierarchy must not belong
  // to a smaller grid, so that the copies of every level form a prefix
  std::vector<int> order(S);
  for (int i = 0; i < S; ++i) order[i] = i;
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
    return parts[a].levels[0].n_cells > parts[b].levels[0].n_cells;
  });
  for (int c = 1; c < S; ++c)
    if (parts[order[c]].levels.size() > parts[order[c - 1]].levels.size())
      return "samples of a batch: a smaller grid has a deeper multigrid hierarchy";
  P = HostProblem{};
  P.dim = dim;
  P.alpha = p0.alpha;
  P.dt = p0.dt;
  P.nterms = p0.nterms;
  P.npres = p0.npres;
  int nmax = 0;
  for (const HostProblem& q : parts) {
    nmax = std::max(nmax, q.n_steps);
    if (q.tcoef.size() > P.tcoef.size()) P.tcoef = q.tcoef;
    if (q.pcoef.size() > P.pcoef.size()) P.pcoef = q.pcoef;
  }
  P.n_steps = nmax;
  const size_t dd = size_t(dim) * dim;
  const size_t nlev = parts[order[0]].levels.size();
  for (size_t l = 0; l < nlev; ++l) {
    int k = 0;  // copies with a level l
    while (k < S && parts[order[k]].levels.size() > l) ++k;
    const HostLevel& a0 = parts[order[0]].levels[l];
    HostLevel L;
    L.W = a0.W;
    L.copies = k;
    L.cbase.assign(size_t(k) + 1, 0);
    L.ccells.assign(size_t(k), 0);
    for (int c = 0; c < k; ++c) {
      const HostLevel& q = parts[order[c]].levels[l];
      L.ccells[c] = q.n_cells;
      L.cbase[c + 1] = L.cbase[c] + (q.nn + pad - 1) / pad * pad;
    }
    L.nn = L.cbase[k];
    L.n_cells = a0.n_cells;
    L.nreal = a0.nn;
    L.nn1 = L.cbase[1];
    L.bcopy.assign(size_t((L.nn + 255) / 256), 0);
    for (int c = 0; c < k; ++c)
      for (int b = L.cbase[c] / 256; b < L.cbase[c + 1] / 256; ++b) L.bcopy[b] = c;
    const int W = L.W, nn = L.nn;
    L.nbr.assign(size_t(W) * nn, 0);
    L.A.assign(size_t(W) * dd * nn, 0.0);
    L.S.assign(size_t(W) * nn, 0.0);
    L.Ainv.assign(dd * nn, 0.0);
    L.Sinv.assign(size_t(nn), 0.0);
    L.fixed.assign(size_t(nn), uint8_t((1u << D1) - 1));
    const bool fine = l == 0;
    if (fine) {
      L.B.assign(size_t(W) * dim * nn, 0.0);
      L.Bt.assign(size_t(W) * dim * nn, 0.0);
      L.Cb.assign(size_t(W) * nn, 0.0);
    }
    for (int c = 0; c < k; ++c) {
      const HostLevel& q = parts[order[c]].levels[l];
      const int base = L.cbase[c], n1 = q.nn;
      for (int v = 0; v < L.cbase[c + 1] - base; ++v) {
        const int g = base + v;
        const bool real = v < n1;
        for (int s2 = 0; s2 < W; ++s2) {
          L.nbr[size_t(s2) * nn + g] = real ? base + q.nbr[size_t(s2) * n1 + v] : g;
          for (size_t e = 0; e < dd; ++e)
            L.A[(s2 * dd + e) * nn + g] = real ? q.A[(s2 * dd + e) * n1 + v] : 0.0;
          L.S[size_t(s2) * nn + g] = real ? q.S[size_t(s2) * n1 + v] : 0.0;
          if (fine)
            for (int kk = 0; kk < dim; ++kk) {
              L.B[(size_t(s2) * dim + kk) * nn + g] = real ? q.B[(size_t(s2) * dim + kk) * n1 + v] : 0.0;
              L.Bt[(size_t(s2) * dim + kk) * nn + g] = real ? q.Bt[(size_t(s2) * dim + kk) * n1 + v] : 0.0;
            }
          if (fine) L.Cb[size_t(s2) * nn + g] = real ? q.Cb[size_t(s2) * n1 + v] : 0.0;
        }
        for (size_t e = 0; e < dd; ++e)
          L.Ainv[e * nn + g] = real ? q.Ainv[e * n1 + v] : (e % (dim + 1) == 0 ? 1.0 : 0.0);
        L.Sinv[g] = real ? q.Sinv[v] : 1.0;
        if (real) {
          L.fixed[g] = q.fixed[v];
        } else {
          for (int kk = 0; kk < dim; ++kk) L.A[(kk * dim + kk) * size_t(nn) + g] = 1.0;  // slot 0
          L.S[g] = 1.0;
        }
      }
      // spectral bounds of the levels that smooth (not a copy's coarsest)
      if (l + 1 < parts[order[c]].levels.size()) {
        L.lmaxA = std::max(L.lmaxA, q.lmaxA);
        L.lmaxS = std::max(L.lmaxS, q.lmaxS);
      }
    }
    P.levels.push_back(std::move(L));
  }
  const HostLevel& L0 = P.levels[0];
  P.nn = L0.nn;
  P.ne = 0;
  // per-copy node-major vectors of every term, side by side (padding nodes zero)
  auto join = [&](int count, std::vector<double> HostProblem::*field, std::vector<double>& out) {
    const size_t nd = size_t(L0.nn) * D1;
    out.assign(nd * count, 0.0);
    for (int j = 0; j < count; ++j)
      for (int c = 0; c < S; ++c) {
        const HostProblem& q = parts[order[c]];
        const std::vector<double>& src = q.*field;
        const size_t nd1 = size_t(q.nn) * D1;
        std::copy(src.begin() + nd1 * j, src.begin() + nd1 * (j + 1),
                  out.begin() + nd * j + size_t(L0.cbase[c]) * D1);
      }
  };
  join(1, &HostProblem::F, P.F);
  join(P.nterms, &HostProblem::terms, P.terms);
  join(P.npres, &HostProblem::pres, P.pres);
  if (!p0.x0.empty()) join(1, &HostProblem::x0, P.x0);
  for (int c = 0; c < S; ++c) {
    const HostProblem& q = parts[order[c]];
    P.sample_of.push_back(order[c]);
    P.csteps.push_back(q.n_steps);
    P.clast.push_back(int(q.levels.size()) - 1);
    P.cAoff.push_back(int64_t(P.coarseAinv.size()));
    P.cSoff.push_back(int64_t(P.coarseSinv.size()));
    P.coarseAinv.insert(P.coarseAinv.end(), q.coarseAinv.begin(), q.coarseAinv.end());
    P.coarseSinv.insert(P.coarseSinv.end(), q.coarseSinv.begin(), q.coarseSinv.end());
  }
  return "";
}

void fold_first_step(HostProblem& p) {
  const int dim = p.dim, dd = dim * dim;
  for (HostLevel& L : p.levels) {
    const size_t nn = size_t(L.nn);
    L.AD.assign(size_t(L.W) * dd * nn, 0.0);
    L.SD.assign(size_t(L.W) * nn, 0.0);
    for (int k = 0; k < L.W; ++k)
      for (size_t i = 0; i < nn; ++i) {
        const size_t w = size_t(L.nbr[k * nn + i]);
        for (int a = 0; a < dim; ++a)
          for (int c = 0; c < dim; ++c) {
            double acc = 0.0;
            for (int j = 0; j < dim; ++j)
              acc += L.A[(size_t(k) * dd + a * dim + j) * nn + i] * L.Ainv[size_t(j * dim + c) * nn + w];
            L.AD[(size_t(k) * dd + a * dim + c) * nn + i] = acc;
          }
        L.SD[k * nn + i] = L.S[k * nn + i] * L.Sinv[w];
      }
  }
}

}  // namespace biot
