// Host code of the library (grid hierarchy, geometry, assembly of the
// factorised and per-(T, k) coefficients, vertical advection, colouring,
// prolongation weights) run under AddressSanitizer and
// UndefinedBehaviorSanitizer by tests/test_host_sanitizers.py. Besides
// running every path, it checks invariants that do not depend on the
// oracle: the cells of a grid tile the unit sphere (total area 4 pi), the
// neighbour relation is symmetric, children tile their parent, coarse
// coefficients are area-weighted means, colourings are proper, every
// coefficient is positive and finite; and that invalid inputs throw.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <random>
#include <stdexcept>
#include <vector>

#include "../../paper_1408_2981_amd/csrc/host.h"

namespace {

int failures = 0;

void expect(bool ok, const char* what, int a = -1, int b = -1) {
  if (!ok) {
    std::printf("FAILED: %s (%d, %d)\n", what, a, b);
    ++failures;
  }
}

std::vector<double> faces(int nz, double thickness) {
  std::vector<double> r(nz + 1);
  for (int k = 0; k <= nz; ++k) {
    const double z = static_cast<double>(k) / nz;
    r[k] = 1.0 + thickness * z * z;   // quadratic grading
  }
  return r;
}

void check_grid(const tpmg::Grid& g) {
  const double pi = std::acos(-1.0);
  for (int r = 0; r <= g.refinement; ++r) {
    const tpmg::MeshLevel& L = g.levels[r];
    double total = 0.0;
    for (int t = 0; t < L.n; ++t) {
      total += L.area[t];
      expect(L.area[t] > 0.0, "positive area", r, t);
      for (int j = 0; j < 3; ++j) {
        const int o = L.nbr[3 * t + j];
        expect(o >= 0 && o < L.n && o != t, "neighbour index", r, t);
        int back = 0;
        for (int i = 0; i < 3; ++i) back += L.nbr[3 * o + i] == t;
        expect(back == 1, "symmetric neighbours", r, t);
        expect(L.g[3 * t + j] > 0.0 && std::isfinite(L.g[3 * t + j]), "flux factor", r, t);
      }
    }
    expect(std::fabs(total - 4.0 * pi) < 1e-12, "areas tile the sphere", r);
    if (r > 0) {
      const tpmg::MeshLevel& C = g.levels[r - 1];
      for (int p = 0; p < C.n; ++p) {
        double s = 0.0;
        for (int i = 0; i < 4; ++i) s += L.area[4 * p + i];
        expect(std::fabs(s - C.area[p]) < 1e-13 * C.area[p] + 1e-15, "children tile the parent", r, p);
      }
    }
  }
}

void check_operator(const tpmg::Operator& op, const tpmg::Grid& g) {
  const int nl = static_cast<int>(op.levels.size());
  for (int l = 0; l < nl; ++l) {
    const tpmg::LevelCoeffs& C = op.levels[l];
    for (int t = 0; t < C.n; ++t) {
      expect(C.beta_h[t] > 0.0 && C.ar_h[t] > 0.0, "positive horizontal factors", l, t);
      for (int j = 0; j < 3; ++j) expect(C.as_h[3 * t + j] > 0.0, "positive edge factor", l, t);
    }
    if (l > 0) expect(C.pw.size() == 3 * static_cast<size_t>(C.n), "prolongation weights", l);
    if (op.full) {
      for (double v : C.fb) expect(v > 0.0 && std::isfinite(v), "per-(T, k) mass", l);
      for (double v : C.fas) expect(v > 0.0 && std::isfinite(v), "per-(T, k) horizontal coupling", l);
    }
  }
  for (int k = 1; k < op.nz; ++k) expect(op.ar_v[k] > 0.0, "vertical coupling", k);
  (void)g;
}

void check_colouring(const tpmg::Grid& g) {
  for (int r = 0; r <= g.refinement; ++r) {
    const tpmg::MeshLevel& L = g.levels[r];
    const std::vector<int8_t> c = tpmg::greedy_colouring(L.nbr, L.n);
    for (int t = 0; t < L.n; ++t) {
      expect(c[t] >= 0 && c[t] < 4, "colour range", r, t);
      for (int j = 0; j < 3; ++j) expect(c[t] != c[L.nbr[3 * t + j]], "proper colouring", r, t);
    }
  }
}

}  // namespace

int main() {
  std::mt19937_64 rng(7);
  std::uniform_real_distribution<double> U(0.5, 2.0);
  for (int ref : {0, 1, 3, 5}) {
    for (int nz : {1, 3, 16}) {
      const std::vector<double> r = faces(nz, 1.5e-3);
      tpmg::Grid g;
      tpmg::build_grid(g, ref, nz, r.data());
      check_grid(g);
      check_colouring(g);
      const int nl = ref + 1 < 6 ? ref + 1 : 6;
      const size_t nf = g.levels[ref].n;
      std::vector<double> arv(nz + 1), asv(nz), bv(nz), arh(nf), ash(nf), bh(nf);
      for (auto* v : {&arv, &asv, &bv, &arh, &ash, &bh})
        for (double& x : *v) x = U(rng);
      tpmg::Operator op;
      tpmg::build_operator(op, g, nl, 3.0, arv.data(), asv.data(), bv.data(), arh.data(), ash.data(), bh.data());
      check_operator(op, g);
      // coarse horizontal factors: area-weighted means of the children
      for (int l = 1; l < nl; ++l) {
        const tpmg::LevelCoeffs& F = op.levels[l];
        const tpmg::LevelCoeffs& C = op.levels[l - 1];
        const tpmg::MeshLevel& MF = g.levels[F.refinement];
        const tpmg::MeshLevel& MC = g.levels[C.refinement];
        for (int p = 0; p < C.n; ++p) {
          double s = 0.0;
          for (int i = 0; i < 4; ++i) s += F.beta_h[4 * p + i];   // |T| beta: a cell integral
          expect(std::fabs(s - C.beta_h[p]) < 1e-12 * C.beta_h[p], "coarse mass conserves", l, p);
          (void)MF;
          (void)MC;
        }
      }
      // caller samples on every grid
      std::vector<std::vector<double>> samples(ref + 1);
      std::vector<const double*> table(ref + 1, nullptr);
      for (int rr = 0; rr <= ref; ++rr) {
        samples[rr].resize(g.levels[rr].n);
        for (double& x : samples[rr]) x = U(rng);
        if (rr % 2 == 0) table[rr] = samples[rr].data();
      }
      tpmg::Operator op2;
      tpmg::build_operator(op2, g, nl, 3.0, arv.data(), asv.data(), bv.data(), nullptr, nullptr, nullptr,
                           table.data(), nullptr, table.data());
      check_operator(op2, g);
      // profiles that do not factorise, with and without advection
      std::vector<double> ar(nf * (nz + 1)), as(nf * nz), b(nf * nz), xi(nf * (nz + 1));
      for (auto* v : {&ar, &as, &b}) for (double& x : *v) x = U(rng);
      for (double& x : xi) x = 1e-3 * (U(rng) - 1.25);
      tpmg::build_full(op, g, ar.data(), as.data(), b.data(), nullptr);
      check_operator(op, g);
      tpmg::build_full(op, g, ar.data(), as.data(), b.data(), xi.data());
      check_operator(op, g);
      // an advection stronger than the diffusion is refused
      if (nz > 2) {
        std::vector<double> big(xi.size(), 1e12);
        bool threw = false;
        try {
          tpmg::build_full(op, g, ar.data(), as.data(), b.data(), big.data());
        } catch (const std::runtime_error&) {
          threw = true;
        }
        expect(threw, "advection beyond diffusion refused", ref, nz);
      }
    }
  }
  // an operator on another grid is refused
  {
    const std::vector<double> r = faces(4, 1e-3);
    tpmg::Grid g2, g3;
    tpmg::build_grid(g2, 2, 4, r.data());
    tpmg::build_grid(g3, 3, 4, r.data());
    std::vector<double> v5(5, 1.0), v4(4, 1.0);
    tpmg::Operator op;
    tpmg::build_operator(op, g2, 3, 1.0, v5.data(), v4.data(), v4.data(), nullptr, nullptr, nullptr);
    std::vector<double> ar(1280 * 5, 1.0), as(1280 * 4, 1.0), b(1280 * 4, 1.0);
    bool threw = false;
    try {
      tpmg::build_full(op, g3, ar.data(), as.data(), b.data(), nullptr);
    } catch (const std::runtime_error&) {
      threw = true;
    }
    expect(threw, "operator and grid differ");
  }
  if (failures) {
    std::printf("%d checks failed\n", failures);
    return 1;
  }
  std::printf("host checks passed\n");
  return 0;
}
