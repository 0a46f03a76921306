// Factorised tensor-stencil coefficients and grid-transfer weights.
//
// Paper, Appendix A (eq. hatFunctionsFac) with the vertical advection term
// dropped (Section 3.2.1):
//   beta^S_T     = |T| beta^S_T               beta^r_k   = v_k beta^r_k
//   alphaS^S_TT' = omega^2 g_TT' alpha_S^S    alphaS^r_k = (r_{k+1}-r_k) alpha_S^r_k
//   alphar^S_T   = omega^2 |T| alpha_r^S_T    alphar^r_k = sigma_k 2 r_k^2/(r_{k+1}-r_{k-1}) alpha_r^r_k
// (the omega^2 of the horizontal coupling is applied once). sigma_0 =
// sigma_nz = 0 imposes the homogeneous Neumann condition. The horizontal
// profile factor on an edge is the mean of its two cells; on coarse grids
// the horizontal factors are area-weighted means of the four children and
// the stencil is rediscretised on the coarse geometry (the matrix-free
// counterpart of the Galerkin coarse operator of Section 3.2.1).
//
// Prolongation (Section 5, "linear interpolation"): a fine cell c with
// parent P takes e_P + G . delta_c, where G is the least-squares gradient
// in the tangent plane at r_P fitted to the parent's three neighbours and
// delta_c the tangent-plane offset of c's centre.
#include <cmath>
#include <stdexcept>
#include <utility>

#include "host.h"

namespace tpmg {
namespace {

struct V3 {
  double x, y, z;
};
inline V3 at(const std::vector<double>& v, int i) { return {v[3 * i], v[3 * i + 1], v[3 * i + 2]}; }
inline V3 sub(V3 a, V3 b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
inline double dot(V3 a, V3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
inline V3 tangent(V3 v, V3 n) {
  double s = dot(v, n);
  return {v.x - s * n.x, v.y - s * n.y, v.z - s * n.z};
}

// weights w[3c + j] for the fine cells of `fine` from parents on `coarse`
std::vector<double> prolongation(const MeshLevel& coarse, const MeshLevel& fine) {
  std::vector<double> w(3 * static_cast<size_t>(fine.n), 0.0);
  for (int P = 0; P < coarse.n; ++P) {
    V3 rp = at(coarse.centre, P);
    V3 d[3];
    double m[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
    double scale = 0.0;
    for (int j = 0; j < 3; ++j) {
      d[j] = tangent(sub(at(coarse.centre, coarse.nbr[3 * P + j]), rp), rp);
      scale += dot(d[j], d[j]);
      const double dv[3] = {d[j].x, d[j].y, d[j].z};
      for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) m[a][b] += dv[a] * dv[b];
    }
    // the normal direction is outside the span of the offsets; adding
    // s n n^T (s ~ |d|^2) makes the normal matrix invertible without changing
    // its action on tangent vectors
    scale /= 3.0;
    const double nv[3] = {rp.x, rp.y, rp.z};
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b) m[a][b] += scale * nv[a] * nv[b];
    double c00 = m[1][1] * m[2][2] - m[1][2] * m[2][1];
    double c01 = m[1][2] * m[2][0] - m[1][0] * m[2][2];
    double c02 = m[1][0] * m[2][1] - m[1][1] * m[2][0];
    double det = m[0][0] * c00 + m[0][1] * c01 + m[0][2] * c02;
    if (!(std::fabs(det) > 0.0)) throw std::runtime_error("degenerate prolongation stencil");
    double inv[3][3] = {
        {c00 / det, (m[0][2] * m[2][1] - m[0][1] * m[2][2]) / det, (m[0][1] * m[1][2] - m[0][2] * m[1][1]) / det},
        {c01 / det, (m[0][0] * m[2][2] - m[0][2] * m[2][0]) / det, (m[0][2] * m[1][0] - m[0][0] * m[1][2]) / det},
        {c02 / det, (m[0][1] * m[2][0] - m[0][0] * m[2][1]) / det, (m[0][0] * m[1][1] - m[0][1] * m[1][0]) / det}};
    for (int i = 0; i < 4; ++i) {
      int c = 4 * P + i;
      V3 dl = tangent(sub(at(fine.centre, c), rp), rp);
      const double dv[3] = {dl.x, dl.y, dl.z};
      double y[3];   // y = M^-1 delta (M symmetric)
      for (int a = 0; a < 3; ++a) y[a] = inv[a][0] * dv[0] + inv[a][1] * dv[1] + inv[a][2] * dv[2];
      for (int j = 0; j < 3; ++j) w[3 * static_cast<size_t>(c) + j] = y[0] * d[j].x + y[1] * d[j].y + y[2] * d[j].z;
    }
  }
  return w;
}

}  // namespace

void build_operator(Operator& op, const Grid& g, int n_levels, double omega2, const double* alpha_r_v,
                    const double* alpha_s_v, const double* beta_v, const double* alpha_r_h,
                    const double* alpha_s_h, const double* beta_h, const double* const* level_alpha_r_h,
                    const double* const* level_alpha_s_h, const double* const* level_beta_h) {
  const int nz = g.nz;
  op.nz = nz;
  op.refinement = g.refinement;
  op.omega2 = omega2;
  op.beta_v.resize(nz);
  op.as_v.resize(nz);
  op.ar_v.assign(nz + 1, 0.0);
  for (int k = 0; k < nz; ++k) {
    op.beta_v[k] = g.vk[k] * beta_v[k];
    op.as_v[k] = (g.r[k + 1] - g.r[k]) * alpha_s_v[k];
  }
  for (int k = 1; k < nz; ++k) op.ar_v[k] = 2.0 * g.r[k] * g.r[k] / (g.r[k + 1] - g.r[k - 1]) * alpha_r_v[k];

  // horizontal profile factors on every grid, finest first
  const int fine_ref = g.refinement;
  const int coarse_ref = fine_ref - n_levels + 1;
  std::vector<std::vector<double>> hr(fine_ref + 1), hs(fine_ref + 1), hb(fine_ref + 1);
  const int nf = g.levels[fine_ref].n;
  auto init = [nf](std::vector<double>& dst, const double* src) {
    dst.assign(nf, 1.0);
    if (src)
      for (int i = 0; i < nf; ++i) dst[i] = src[i];
  };
  auto given = [](const double* const* lv, int r) -> const double* { return lv ? lv[r] : nullptr; };
  init(hr[fine_ref], given(level_alpha_r_h, fine_ref) ? given(level_alpha_r_h, fine_ref) : alpha_r_h);
  init(hs[fine_ref], given(level_alpha_s_h, fine_ref) ? given(level_alpha_s_h, fine_ref) : alpha_s_h);
  init(hb[fine_ref], given(level_beta_h, fine_ref) ? given(level_beta_h, fine_ref) : beta_h);
  for (int r = fine_ref; r > coarse_ref; --r) {
    const MeshLevel& F = g.levels[r];
    const int nc = g.levels[r - 1].n;
    const std::pair<std::vector<std::vector<double>>*, const double* const*> planes[3] = {
        {&hr, level_alpha_r_h}, {&hs, level_alpha_s_h}, {&hb, level_beta_h}};
    for (const auto& plane : planes) {
      std::vector<double>& src = (*plane.first)[r];
      std::vector<double>& dst = (*plane.first)[r - 1];
      if (const double* v = given(plane.second, r - 1)) {   // the caller's samples on this grid
        dst.assign(v, v + nc);
        continue;
      }
      dst.assign(nc, 0.0);
      for (int P = 0; P < nc; ++P) {
        double num = 0.0, den = 0.0;
        for (int i = 0; i < 4; ++i) {
          num += src[4 * P + i] * F.area[4 * P + i];
          den += F.area[4 * P + i];
        }
        dst[P] = num / den;
      }
    }
  }

  op.levels.clear();
  op.levels.resize(n_levels);
  for (int l = 0; l < n_levels; ++l) {
    const int r = coarse_ref + l;
    const MeshLevel& M = g.levels[r];
    LevelCoeffs& C = op.levels[l];
    C.refinement = r;
    C.n = M.n;
    C.nbr = M.nbr;
    C.beta_h.resize(M.n);
    C.ar_h.resize(M.n);
    C.as_h.resize(3 * static_cast<size_t>(M.n));
    for (int t = 0; t < M.n; ++t) {
      C.beta_h[t] = M.area[t] * hb[r][t];
      C.ar_h[t] = omega2 * M.area[t] * hr[r][t];
      for (int j = 0; j < 3; ++j) {
        int o = M.nbr[3 * t + j];
        C.as_h[3 * t + j] = omega2 * M.g[3 * t + j] * (0.5 * (hs[r][t] + hs[r][o]));
      }
    }
    if (l > 0) C.pw = prolongation(g.levels[r - 1], M);
  }
}

std::vector<int8_t> greedy_colouring(const std::vector<int32_t>& nbr, int n) {
  std::vector<int8_t> col(static_cast<size_t>(n), -1);
  for (int t = 0; t < n; ++t) {
    bool used[4] = {false, false, false, false};
    for (int j = 0; j < 3; ++j) {
      const int8_t c = col[nbr[3 * static_cast<size_t>(t) + j]];
      if (c >= 0) used[c] = true;
    }
    int8_t c = 0;
    while (used[c]) ++c;
    col[t] = c;
  }
  return col;
}

void build_full(Operator& op, const Grid& g, const double* alpha_r, const double* alpha_s, const double* beta,
                const double* xi_r) {
  const int nz = op.nz;
  if (g.nz != nz || g.refinement != op.refinement) throw std::runtime_error("grid and operator differ");
  const int fine_ref = g.refinement;
  const int nl = static_cast<int>(op.levels.size());
  const int coarse_ref = fine_ref - nl + 1;
  // per-level profiles [n][m], finest first; coarse = area-weighted means
  struct Prof {
    std::vector<double> ar, as, b, xi;
  };
  std::vector<Prof> pf(fine_ref + 1);
  const size_t nf = g.levels[fine_ref].n;
  pf[fine_ref].ar.assign(alpha_r, alpha_r + nf * (nz + 1));
  pf[fine_ref].as.assign(alpha_s, alpha_s + nf * nz);
  pf[fine_ref].b.assign(beta, beta + nf * nz);
  if (xi_r) pf[fine_ref].xi.assign(xi_r, xi_r + nf * (nz + 1));
  for (int r = fine_ref; r > coarse_ref; --r) {
    const MeshLevel& F = g.levels[r];
    const int nc = g.levels[r - 1].n;
    auto restrict_rows = [&](const std::vector<double>& src, std::vector<double>& dst, int m) {
      dst.assign(static_cast<size_t>(nc) * m, 0.0);
      for (int P = 0; P < nc; ++P) {
        double den = 0.0;
        for (int i = 0; i < 4; ++i) den += F.area[4 * P + i];
        for (int k = 0; k < m; ++k) {
          double num = 0.0;
          for (int i = 0; i < 4; ++i) num += src[static_cast<size_t>(4 * P + i) * m + k] * F.area[4 * P + i];
          dst[static_cast<size_t>(P) * m + k] = num / den;
        }
      }
    };
    restrict_rows(pf[r].ar, pf[r - 1].ar, nz + 1);
    restrict_rows(pf[r].as, pf[r - 1].as, nz);
    restrict_rows(pf[r].b, pf[r - 1].b, nz);
    if (xi_r) restrict_rows(pf[r].xi, pf[r - 1].xi, nz + 1);
  }
  const double omega2 = op.omega2;
  std::vector<double> face(nz + 1, 0.0);
  for (int k = 1; k < nz; ++k) face[k] = 2.0 * g.r[k] * g.r[k] / (g.r[k + 1] - g.r[k - 1]);
  // advection through cell k's lower and upper face: sigma_k r_k^2
  // (r_{k+1}-r_k)/(r_{k+1}-r_{k-1}) and sigma_{k+1} r_{k+1}^2
  // (r_{k+1}-r_k)/(r_{k+2}-r_k)
  std::vector<double> adv_lo(nz, 0.0), adv_up(nz, 0.0);
  for (int k = 0; k < nz; ++k) {
    if (k > 0) adv_lo[k] = g.r[k] * g.r[k] * (g.r[k + 1] - g.r[k]) / (g.r[k + 1] - g.r[k - 1]);
    if (k + 1 < nz) adv_up[k] = g.r[k + 1] * g.r[k + 1] * (g.r[k + 1] - g.r[k]) / (g.r[k + 2] - g.r[k]);
  }
  for (int l = 0; l < nl; ++l) {
    const int r = coarse_ref + l;
    const MeshLevel& M = g.levels[r];
    LevelCoeffs& C = op.levels[l];
    const Prof& P = pf[r];
    const size_t n = M.n;
    C.fb.resize(n * nz);
    C.far.resize(n * (nz + 1));
    C.fas.resize(3 * n * nz);

    for (size_t t = 0; t < n; ++t) {
      for (int k = 0; k < nz; ++k) C.fb[t * nz + k] = M.area[t] * g.vk[k] * P.b[t * nz + k];
      for (int k = 0; k <= nz; ++k)
        C.far[t * (nz + 1) + k] = omega2 * face[k] * M.area[t] * P.ar[t * (nz + 1) + k];
      for (int j = 0; j < 3; ++j) {
        const size_t o = M.nbr[3 * t + j];
        for (int k = 0; k < nz; ++k)
          C.fas[(3 * t + j) * nz + k] = omega2 * (g.r[k + 1] - g.r[k]) * M.g[3 * t + j] *
                                        (0.5 * (P.as[t * nz + k] + P.as[o * nz + k]));
      }
    }
    // (after the diffusion coefficients, which the advection is checked against)
    if (xi_r) {
      C.fxl.resize(n * nz);
      C.fxu.resize(n * nz);
      for (size_t t = 0; t < n; ++t)
        for (int k = 0; k < nz; ++k) {
          C.fxl[t * nz + k] = omega2 * M.area[t] * adv_lo[k] * P.xi[t * (nz + 1) + k];
          C.fxu[t * nz + k] = omega2 * M.area[t] * adv_up[k] * P.xi[t * (nz + 1) + k + 1];
          // the column stays an M-matrix: both radial couplings positive
          if ((k > 0 && !(C.far[t * (nz + 1) + k] - C.fxl[t * nz + k] > 0.0)) ||
              (k + 1 < nz && !(C.far[t * (nz + 1) + k + 1] + C.fxu[t * nz + k] > 0.0)))
            throw std::runtime_error("the vertical advection exceeds the vertical diffusion");
        }
    } else {
      C.fxl.clear();
      C.fxu.clear();
    }
  }
  op.full = true;
  op.adv = xi_r != nullptr;
}

}  // namespace tpmg
