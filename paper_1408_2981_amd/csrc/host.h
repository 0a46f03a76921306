// Host-side data structures of the TPMG library: the icosahedral grid
// hierarchy with its geometry, and the factorised operator coefficients.
// Nothing here touches the GPU; the C ABI's host-only entry points use it
// directly, and the device setup uploads from it.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

namespace tpmg {

// One refinement level of the icosahedral grid (Section 4.2). Arrays are
// cell-major: [T] or [T][j] with j the edge / neighbour index.
struct MeshLevel {
  int refinement = 0;
  int n = 0;
  std::vector<int32_t> faces;   // 3n vertex ids, counter-clockwise from outside
  std::vector<int32_t> nbr;     // 3n: cell across edge j = (v_j, v_{j+1})
  std::vector<double> centre;   // 3n: spherical circumcentre
  std::vector<double> area;     // n : spherical area |T|
  std::vector<double> arc;      // 3n: great-circle edge length |S_TT'|
  std::vector<double> g;        // 3n: |S_TT'| n.(r_T' - r_T) / |r_T' - r_T|^2
};

struct Grid {
  int refinement = 0;
  int nz = 0;
  std::vector<double> r;        // nz+1 radial faces
  std::vector<double> vk;       // nz radial volume factors
  std::vector<double> verts;    // 3 * n_vertices, all levels
  std::vector<MeshLevel> levels;  // index = refinement
};

// Builds the hierarchy for refinements 0..refinement. Throws std::runtime_error.
void build_grid(Grid& g, int refinement, int nz, const double* r_faces);

// Factorised coefficients of one multigrid level (Appendix A,
// eq. hatFunctionsFac). The full coefficients are products:
//   beta^_{T,k} = beta_h[T] * beta_v[k]
//   alphaS^_{TT',k} = as_h[3T+j] * as_v[k]
//   alphar^_{T,k} = ar_h[T] * ar_v[k]      (face k below cell k)
struct LevelCoeffs {
  int refinement = 0;
  int n = 0;
  std::vector<int32_t> nbr;     // 3n
  std::vector<double> beta_h;   // n
  std::vector<double> ar_h;     // n
  std::vector<double> as_h;     // 3n
  std::vector<double> pw;       // 3n prolongation weights from the next coarser level (empty on level 0)
  // profiles that do not factorise (Operator::full; Appendix A, eq.
  // hatFunctionsNonFac): the coefficients per (T, k), cell-major
  std::vector<double> fb;       // n (nz):        beta^_{T,k}
  std::vector<double> far;      // n (nz + 1):    alphar^_{T,k} on radial face k
  std::vector<double> fas;      // n (3) (nz):    alphaS^_{TT'_j,k}
  // vertical advection (Operator::adv): omega^2 times the coefficients of
  // cell k's lower and upper face (Appendix A, "Vertical advection")
  std::vector<double> fxl;      // n (nz)
  std::vector<double> fxu;      // n (nz)
};

struct Operator {
  int nz = 0;
  int refinement = 0;
  double omega2 = 0;
  std::vector<double> beta_v;   // nz
  std::vector<double> as_v;     // nz
  std::vector<double> ar_v;     // nz+1
  std::vector<LevelCoeffs> levels;  // 0 = coarsest
  bool full = false;            // the levels also hold coefficients of profiles that do not factorise
  bool adv = false;             // ... and of the vertical advection
};

// Assembles the operator on the n_levels finest grids of g. level_*: NULL
// or refinement + 1 pointers, indexed by refinement level, to caller samples
// of that grid's horizontal factors (n values); where a pointer is NULL the
// finest grid takes alpha_r_h / alpha_s_h / beta_h (NULL: 1) and a coarse
// grid the area-weighted means of its four children's factors.
void build_operator(Operator& op, const Grid& g, int n_levels, double omega2, const double* alpha_r_v,
                    const double* alpha_s_v, const double* beta_v, const double* alpha_r_h,
                    const double* alpha_s_h, const double* beta_h,
                    const double* const* level_alpha_r_h = nullptr, const double* const* level_alpha_s_h = nullptr,
                    const double* const* level_beta_h = nullptr);

// Adds the coefficients of profiles that do not factorise, point samples on
// the finest grid (cell-major: alpha_r [n][nz+1] at the radial faces,
// alpha_s and beta [n][nz] at the layer midpoints), to every level of op
// (coarse grids: area-weighted means of the four children, level by level;
// on an edge the mean of its two cells). xi_r (nullable) [n][nz+1] at the
// radial faces adds the vertical advection. Throws std::runtime_error.
void build_full(Operator& op, const Grid& g, const double* alpha_r, const double* alpha_s, const double* beta,
                const double* xi_r = nullptr);

// Colours of the cells of a grid level (nbr: 3n, cell-major) with no two
// neighbours alike: cells in index order, each taking the smallest colour
// none of its already coloured neighbours has (at most 4 on degree 3).
std::vector<int8_t> greedy_colouring(const std::vector<int32_t>& nbr, int n);

}  // namespace tpmg
