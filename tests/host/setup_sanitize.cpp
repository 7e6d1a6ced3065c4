// Host-only driver of the library's set-up code (setup.cpp), built with the
// address and undefined-behaviour sanitizers by tests/test_setup_sanitized.py.
// It runs the assembly, the boundary-condition elimination, the lifting of
// prescribed values, the multigrid hierarchy, the batch concatenation and the
// folded operators on structured 2D and 3D meshes, plus the argument checks,
// and checks a few invariants; any sanitizer report fails the run.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <string>
#include <vector>

#include "../../paper_2310_10430_amd/csrc/setup.hpp"

using namespace biot;

namespace {

int failures = 0;
void check(bool ok, const std::string& what) {
  if (!ok) {
    std::fprintf(stderr, "FAILED: %s\n", what.c_str());
    ++failures;
  }
}

struct Mesh {
  int dim, n, nn, ne;
  std::vector<double> xyz;
  std::vector<int32_t> conn;
  std::vector<uint8_t> flags;
  std::vector<int32_t> top;      // facets on the loaded face
  std::vector<double> traction;
};

// structured unit square / cube; consolidation-column flags and top facets
Mesh make_mesh(int dim, int n) {
  Mesh m;
  m.dim = dim;
  m.n = n;
  const int p = n + 1;
  m.nn = dim == 2 ? p * p : p * p * p;
  for (int v = 0; v < m.nn; ++v) {
    const int i = v % p, j = (v / p) % p, k = v / (p * p);
    m.xyz.push_back(double(i) / n);
    m.xyz.push_back(double(j) / n);
    if (dim == 3) m.xyz.push_back(double(k) / n);
    const int up = dim == 2 ? j : k;
    uint8_t f = 0;
    if (up == 0) f |= (1u << dim) - 1;                 // fixed base
    if (i == 0 || i == n) f |= 1u;                      // rollers
    if (dim == 3 && (j == 0 || j == n)) f |= 2u;
    if (up == n) f |= 1u << dim;                        // drained top
    m.flags.push_back(f);
  }
  auto id2 = [&](int i, int j) { return j * p + i; };
  auto id3 = [&](int i, int j, int k) { return (k * p + j) * p + i; };
  if (dim == 2) {
    for (int j = 0; j < n; ++j)
      for (int i = 0; i < n; ++i) {
        const int a = id2(i, j), b = id2(i + 1, j), c = id2(i + 1, j + 1), d = id2(i, j + 1);
        m.conn.insert(m.conn.end(), {a, b, c, a, c, d});
      }
    for (int i = 0; i < n; ++i) {
      m.top.insert(m.top.end(), {id2(i, n), id2(i + 1, n)});
      m.traction.insert(m.traction.end(), {0.0, -1.0});
    }
  } else {
    const int perms[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2}, {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};
    for (int k = 0; k < n; ++k)
      for (int j = 0; j < n; ++j)
        for (int i = 0; i < n; ++i)
          for (const auto& pr : perms) {
            int c[3] = {i, j, k};
            int tet[4];
            tet[0] = id3(c[0], c[1], c[2]);
            for (int s = 0; s < 3; ++s) {
              ++c[pr[s]];
              tet[s + 1] = id3(c[0], c[1], c[2]);
            }
            // orient positively
            double x[4][3];
            for (int a = 0; a < 4; ++a)
              for (int d = 0; d < 3; ++d) x[a][d] = m.xyz[size_t(tet[a]) * 3 + d];
            double e1[3], e2[3], e3[3];
            for (int d = 0; d < 3; ++d) {
              e1[d] = x[1][d] - x[0][d];
              e2[d] = x[2][d] - x[0][d];
              e3[d] = x[3][d] - x[0][d];
            }
            const double det = e1[0] * (e2[1] * e3[2] - e2[2] * e3[1]) -
                               e1[1] * (e2[0] * e3[2] - e2[2] * e3[0]) +
                               e1[2] * (e2[0] * e3[1] - e2[1] * e3[0]);
            if (det < 0) std::swap(tet[2], tet[3]);
            m.conn.insert(m.conn.end(), tet, tet + 4);
          }
    for (int j = 0; j < n; ++j)
      for (int i = 0; i < n; ++i) {
        m.top.insert(m.top.end(), {id3(i, j, n), id3(i + 1, j, n), id3(i + 1, j + 1, n)});
        m.top.insert(m.top.end(), {id3(i, j, n), id3(i + 1, j + 1, n), id3(i, j + 1, n)});
        m.traction.insert(m.traction.end(), {0.0, 0.0, -1.0, 0.0, 0.0, -1.0});
      }
  }
  m.ne = int(m.conn.size()) / (dim + 1);
  return m;
}

std::string build(const Mesh& m, int steps, bool general, bool beta, HostProblem& P,
                  double young_scale = 1.0) {
  std::vector<double> E(m.ne), nu(m.ne, 0.3), K(m.ne), b(m.ne);
  for (int e = 0; e < m.ne; ++e) {
    E[e] = young_scale * (5e3 + 1.5e4 * ((e * 37) % 101) / 100.0);
    K[e] = 1e-2 * std::exp(std::sin(0.1 * e));
    b[e] = 1e-8;
  }
  std::vector<double> coef(steps + 1, 1.0);
  coef[0] = 0.0;
  const int D1 = m.dim + 1;
  const size_t nd = size_t(m.nn) * D1;
  std::vector<double> terms(2 * nd), tcoef((steps + 1) * 2), pres(nd), pcoef(steps + 1), x0(nd);
  for (size_t i = 0; i < terms.size(); ++i) terms[i] = std::sin(0.37 * double(i)) * 1e-3;
  for (int n = 0; n <= steps; ++n) {
    tcoef[n * 2] = std::cos(0.3 * n);
    tcoef[n * 2 + 1] = std::sin(0.2 * n);
    pcoef[n] = 1.0 + 0.1 * n;
  }
  for (size_t i = 0; i < nd; ++i) {
    pres[i] = 1e-4 * std::cos(0.11 * double(i));
    x0[i] = 1e-4 * std::sin(0.07 * double(i));
  }
  MeshIn mi{m.dim, m.nn, m.ne, m.n, m.xyz.data(), m.conn.data(), m.flags.data()};
  MaterialsIn mt{E.data(), nu.data(), K.data(), beta ? b.data() : nullptr, 1.0, 1.0 / m.n,
                 nullptr, nullptr};
  LoadIn ld{int(m.top.size()) / m.dim, m.top.data(), m.traction.data(), coef.data(),
            general ? 2 : 0, general ? terms.data() : nullptr, general ? tcoef.data() : nullptr,
            general ? 1 : 0, general ? pres.data() : nullptr, general ? pcoef.data() : nullptr,
            general ? x0.data() : nullptr};
  HostOptions opt;
  return build_problem(mi, mt, ld, 1.0 / steps, steps, opt, P);
}

double sum_abs(const std::vector<double>& v) {
  double s = 0;
  for (double x : v) s += std::fabs(x);
  return s;
}

}  // namespace

int main() {
  for (int dim : {2, 3}) {
    for (int n : dim == 2 ? std::vector<int>{16, 12, 7} : std::vector<int>{4, 3}) {
      const Mesh m = make_mesh(dim, n);
      for (int general = 0; general < 2; ++general) {
        HostProblem P;
        const std::string e = build(m, 6, general != 0, general == 0 && n == 12, P);
        check(e.empty(), "build dim " + std::to_string(dim) + " n " + std::to_string(n) + ": " + e);
        if (!e.empty()) continue;
        fold_first_step(P);
        check(P.levels[0].nn == m.nn, "level 0 nodes");
        check(P.nterms == (general ? 1 + 2 + 2 + 1 : 1), "internal load terms");
        check(std::isfinite(sum_abs(P.terms)) && std::isfinite(sum_abs(P.levels[0].AD)),
              "finite terms and folded operators");
        for (size_t l = 0; l + 1 < P.levels.size(); ++l)
          check(P.levels[l].lmaxA > 0 && P.levels[l].lmaxS > 0, "spectral bounds");
        // terms vanish at prescribed dofs
        bool zero = true;
        for (int j = 0; j < P.nterms; ++j)
          for (int v = 0; v < m.nn; ++v)
            for (int c = 0; c <= dim; ++c)
              if (((P.levels[0].fixed[v] >> c) & 1) &&
                  P.terms[(size_t(j) * m.nn + v) * (dim + 1) + c] != 0.0)
                zero = false;
        check(zero, "load terms zero at prescribed dofs");
      }
      // a batch of three samples (one with stiffer moduli)
      std::vector<HostProblem> parts(3);
      for (int s = 0; s < 3; ++s) check(build(m, 4 + s, false, false, parts[s], 1.0 + s).empty(), "part");
      HostProblem B;
      const std::string e = concat_problems(parts, 256, B);
      check(e.empty(), "concat: " + e);
      if (e.empty()) {
        fold_first_step(B);
        check(B.levels[0].copies == 3 && B.levels[0].nn % 256 == 0, "batch padding");
        check(B.n_steps == 6, "batch steps");
      }
      // inconsistent batch structure is refused
      std::vector<HostProblem> mixed(2);
      check(build(m, 4, false, false, mixed[0]).empty() && build(m, 4, true, false, mixed[1]).empty(),
            "mixed parts");
      HostProblem Bm;
      check(!concat_problems(mixed, 256, Bm).empty(), "mixed batch refused");
    }
  }
  // argument checks
  {
    const Mesh m = make_mesh(2, 4);
    HostProblem P;
    Mesh bad = m;
    bad.xyz[3] += 0.1;
    check(!build(bad, 3, false, false, P).empty(), "non-grid node refused");
    bad = m;
    bad.conn[2] = m.nn + 5;
    check(!build(bad, 3, false, false, P).empty(), "connectivity out of range refused");
    MeshIn mi{2, m.nn, m.ne, m.n, m.xyz.data(), m.conn.data(), m.flags.data()};
    std::vector<double> E(m.ne, 1e4), nu(m.ne, 0.3), K(m.ne, 1e-2), coef(4, 1.0);
    MaterialsIn mt{E.data(), nu.data(), K.data(), nullptr, 1.0, 0.25, nullptr, nullptr};
    LoadIn ld{int(m.top.size()) / 2, m.top.data(), m.traction.data(), coef.data(), 9, nullptr,
              nullptr, 0, nullptr, nullptr, nullptr};
    HostOptions opt;
    check(!build_problem(mi, mt, ld, 0.25, 3, opt, P).empty(), "n_terms out of range refused");
    ld.n_terms = 0;
    nu[1] = 0.5;
    check(!build_problem(mi, mt, ld, 0.25, 3, opt, P).empty(), "nu = 0.5 refused");
  }
  if (failures) {
    std::fprintf(stderr, "%d check(s) failed\n", failures);
    return 1;
  }
  std::printf("setup sanitizer driver: all checks passed\n");
  return 0;
}
