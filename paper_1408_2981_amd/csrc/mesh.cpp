// Icosahedral grid hierarchy and spherical finite-volume geometry.
//
// Paper: the horizontal grid is an icosahedral grid projected onto the
// sphere whose coarse triangles each consist of four finer ones (Section
// 4.1, Section 4.2); the geometric factors are those of the finite-volume
// scheme of Appendix A: cell areas |T|, centres r_T, edge lengths |S_TT'|,
// outward edge normals n_TT' and the two-point flux factor
// |S_TT'| n_TT'.(r_T' - r_T) / |r_T' - r_T|^2.
//
// Conventions fixed by the library (the paper leaves them open):
//  * base icosahedron: poles plus rings of five vertices at latitude
//    +-atan(1/2), longitudes 72 i (north) and 36 + 72 i (south); faces in
//    the order north cap, upper band, lower band, south cap, each
//    counter-clockwise seen from outside;
//  * face (a, b, c) splits into (a, m_ab, m_ca), (m_ab, b, m_bc),
//    (m_ca, m_bc, c), (m_ab, m_bc, m_ca), m = normalise((p + q) / 2); child i
//    of P is 4P + i, so every coarse cell's children are contiguous;
//  * centre = spherical circumcentre, area = spherical excess, edge length =
//    great-circle arc; the flux factor is evaluated once per edge and
//    shared by its two cells, so the operator is exactly symmetric.
#include <cmath>
#include <stdexcept>
#include <unordered_map>

#include "host.h"

namespace tpmg {
namespace {

struct V3 {
  double x, y, z;
};
inline V3 sub(V3 a, V3 b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
inline V3 add(V3 a, V3 b) { return {a.x + b.x, a.y + b.y, a.z + b.z}; }
inline V3 scale(V3 a, double s) { return {a.x * s, a.y * s, a.z * s}; }
inline double dot(V3 a, V3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
inline V3 cross(V3 a, V3 b) { return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x}; }
inline double norm(V3 a) { return std::sqrt(dot(a, a)); }
inline V3 unit(V3 a) {
  const double s = norm(a);
  return {a.x / s, a.y / s, a.z / s};
}

inline V3 vert(const std::vector<double>& v, int32_t i) { return {v[3 * i], v[3 * i + 1], v[3 * i + 2]}; }

inline uint64_t edge_key(int32_t a, int32_t b) {
  uint32_t lo = static_cast<uint32_t>(a < b ? a : b), hi = static_cast<uint32_t>(a < b ? b : a);
  return (static_cast<uint64_t>(lo) << 32) | hi;
}

void base_icosahedron(std::vector<double>& verts, std::vector<int32_t>& faces) {
  const double pi = std::acos(-1.0);
  const double lat = std::atan(0.5);
  verts.assign(36, 0.0);
  auto put = [&](int i, double x, double y, double z) {
    verts[3 * i] = x;
    verts[3 * i + 1] = y;
    verts[3 * i + 2] = z;
  };
  put(0, 0.0, 0.0, 1.0);
  put(11, 0.0, 0.0, -1.0);
  for (int i = 0; i < 5; ++i) {
    double ln = 2.0 * pi * i / 5.0, ls = ln + pi / 5.0;
    put(1 + i, std::cos(lat) * std::cos(ln), std::cos(lat) * std::sin(ln), std::sin(lat));
    put(6 + i, std::cos(lat) * std::cos(ls), std::cos(lat) * std::sin(ls), -std::sin(lat));
  }
  faces.clear();
  auto tri = [&](int a, int b, int c) {
    faces.push_back(a);
    faces.push_back(b);
    faces.push_back(c);
  };
  for (int i = 0; i < 5; ++i) tri(0, 1 + i, 1 + (i + 1) % 5);
  for (int i = 0; i < 5; ++i) tri(1 + i, 6 + i, 1 + (i + 1) % 5);
  for (int i = 0; i < 5; ++i) tri(1 + (i + 1) % 5, 6 + i, 6 + (i + 1) % 5);
  for (int i = 0; i < 5; ++i) tri(11, 6 + (i + 1) % 5, 6 + i);
}

// faces of the next finer grid; new edge midpoints are appended to verts
std::vector<int32_t> split(std::vector<double>& verts, const std::vector<int32_t>& faces) {
  const size_t n = faces.size() / 3;
  std::unordered_map<uint64_t, int32_t> mid;
  mid.reserve(n * 2);
  auto midpoint = [&](int32_t a, int32_t b) -> int32_t {
    uint64_t k = edge_key(a, b);
    auto it = mid.find(k);
    if (it != mid.end()) return it->second;
    V3 m = unit(scale(add(vert(verts, a), vert(verts, b)), 0.5));
    int32_t id = static_cast<int32_t>(verts.size() / 3);
    verts.push_back(m.x);
    verts.push_back(m.y);
    verts.push_back(m.z);
    mid.emplace(k, id);
    return id;
  };
  std::vector<int32_t> out(n * 12);
  for (size_t t = 0; t < n; ++t) {
    int32_t a = faces[3 * t], b = faces[3 * t + 1], c = faces[3 * t + 2];
    int32_t ab = midpoint(a, b), bc = midpoint(b, c), ca = midpoint(c, a);
    const int32_t kids[12] = {a, ab, ca, ab, b, bc, ca, bc, c, ab, bc, ca};
    for (int i = 0; i < 12; ++i) out[12 * t + i] = kids[i];
  }
  return out;
}

void fill_level(MeshLevel& L, const std::vector<double>& verts) {
  const int n = L.n;
  L.nbr.assign(3 * n, -1);
  L.centre.assign(3 * n, 0.0);
  L.area.assign(n, 0.0);
  L.arc.assign(3 * n, 0.0);
  L.g.assign(3 * n, 0.0);
  std::unordered_map<uint64_t, int32_t> first;   // edge -> 3T + j of its first cell
  first.reserve(static_cast<size_t>(n) * 2);
  for (int t = 0; t < n; ++t) {
    for (int j = 0; j < 3; ++j) {
      int32_t a = L.faces[3 * t + j], b = L.faces[3 * t + (j + 1) % 3];
      uint64_t k = edge_key(a, b);
      auto it = first.find(k);
      if (it == first.end()) {
        first.emplace(k, 3 * t + j);
      } else {
        int32_t o = it->second;
        if (L.nbr[o] != -1) throw std::runtime_error("edge shared by more than two cells");
        L.nbr[o] = t;
        L.nbr[3 * t + j] = o / 3;
      }
    }
  }
  for (int i = 0; i < 3 * n; ++i)
    if (L.nbr[i] < 0) throw std::runtime_error("open edge in icosahedral grid");
  for (int t = 0; t < n; ++t) {
    V3 a = vert(verts, L.faces[3 * t]), b = vert(verts, L.faces[3 * t + 1]), c = vert(verts, L.faces[3 * t + 2]);
    V3 cc = unit(cross(sub(b, a), sub(c, a)));
    L.centre[3 * t] = cc.x;
    L.centre[3 * t + 1] = cc.y;
    L.centre[3 * t + 2] = cc.z;
    double num = std::fabs(dot(a, cross(b, c)));
    double den = 1.0 + dot(a, b) + dot(b, c) + dot(c, a);
    L.area[t] = 2.0 * std::atan2(num, den);
  }
  // edge quantities: computed once from the first cell's side, shared
  for (int t = 0; t < n; ++t) {
    for (int j = 0; j < 3; ++j) {
      int32_t o = L.nbr[3 * t + j];
      if (o < t) continue;
      V3 p = vert(verts, L.faces[3 * t + j]), q = vert(verts, L.faces[3 * t + (j + 1) % 3]);
      V3 pq = cross(p, q);
      double len = std::atan2(norm(pq), dot(p, q));
      V3 nout = unit(cross(q, p));   // interior lies on the side of p x q
      V3 rt = {L.centre[3 * t], L.centre[3 * t + 1], L.centre[3 * t + 2]};
      V3 ro = {L.centre[3 * o], L.centre[3 * o + 1], L.centre[3 * o + 2]};
      V3 d = sub(ro, rt);
      double gf = len * dot(nout, d) / dot(d, d);
      if (!(gf > 0.0)) throw std::runtime_error("non-positive two-point flux factor");
      int jb = -1;
      for (int i = 0; i < 3; ++i)
        if (L.nbr[3 * o + i] == t) jb = i;
      L.arc[3 * t + j] = len;
      L.arc[3 * o + jb] = len;
      L.g[3 * t + j] = gf;
      L.g[3 * o + jb] = gf;
    }
  }
}

}  // namespace

void build_grid(Grid& g, int refinement, int nz, const double* r_faces) {
  g.refinement = refinement;
  g.nz = nz;
  g.r.assign(r_faces, r_faces + nz + 1);
  g.vk.resize(nz);
  for (int k = 0; k < nz; ++k) {
    double lo = g.r[k], hi = g.r[k + 1];
    // (hi^3 - lo^3)/3 without cancelling the cubes
    g.vk[k] = (hi - lo) * (hi * hi + hi * lo + lo * lo) / 3.0;
  }
  std::vector<int32_t> faces;
  base_icosahedron(g.verts, faces);
  g.levels.clear();
  g.levels.resize(refinement + 1);
  for (int r = 0; r <= refinement; ++r) {
    if (r > 0) faces = split(g.verts, faces);
    MeshLevel& L = g.levels[r];
    L.refinement = r;
    L.n = static_cast<int>(faces.size() / 3);
    L.faces = faces;
    fill_level(L, g.verts);
  }
}

}  // namespace tpmg
