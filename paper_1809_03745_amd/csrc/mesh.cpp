// Host side of signed distance fields from surface tessellations (the
// geometry-generation section of the paper): a half-edge (doubly-connected
// edge list) view of a watertight two-manifold triangle mesh, the
// angle-weighted pseudonormals of its faces, edges and vertices that fix the
// sign of the distance to the closest feature, and a bounding-volume
// hierarchy (a k-d tree of axis-aligned boxes over the triangles) for the
// nearest-first closest-feature search the device kernel runs.
//
// Sign: the angle-weighted pseudonormal of the feature (face, edge or
// vertex) that holds the closest surface point c of a query point p gives
// sign((p - c) . n) = the side of the surface p lies on (Baerentzen and
// Aanaes, "Signed distance computation using the angle weighted
// pseudonormal", 2005): face normal for a face, the sum of the two adjacent
// face normals for an edge, the incident face normals weighted by their
// angles at a vertex.

#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>
#include <unordered_map>

#include "internal.hpp"

namespace ebmg {

namespace {

struct V3 {
  double x, y, z;
};
inline V3 sub(V3 a, V3 b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
inline V3 add(V3 a, V3 b) { return {a.x + b.x, a.y + b.y, a.z + b.z}; }
inline V3 scl(V3 a, double s) { return {a.x * s, a.y * s, a.z * s}; }
inline double dot(V3 a, V3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
inline V3 cross(V3 a, V3 b) { return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x}; }
inline double norm(V3 a) { return std::sqrt(dot(a, a)); }
inline V3 unit(V3 a) {
  const double n = norm(a);
  return n > 0 ? scl(a, 1.0 / n) : V3{0, 0, 0};
}

struct Builder {
  const MeshInput& in;
  std::vector<int32_t> order;   // triangle permutation built by the tree
  std::vector<MeshNode> nodes;
  std::vector<double> cen;      // triangle centroids (3 per triangle)
  std::vector<double> lo, hi;   // triangle bounds (3 per triangle)
  explicit Builder(const MeshInput& m) : in(m) {}

  void bounds(int32_t b, int32_t e, double* bl, double* bh) const {
    for (int d = 0; d < 3; ++d) {
      bl[d] = 1e300;
      bh[d] = -1e300;
    }
    for (int32_t k = b; k < e; ++k) {
      const int32_t t = order[k];
      for (int d = 0; d < 3; ++d) {
        bl[d] = std::min(bl[d], lo[3 * t + d]);
        bh[d] = std::max(bh[d], hi[3 * t + d]);
      }
    }
  }

  // node over order[b, e): a leaf of at most kMeshLeaf triangles, or a split
  // at the median centroid along the axis where the centroids spread most
  int32_t build(int32_t b, int32_t e) {
    const int32_t id = (int32_t)nodes.size();
    nodes.emplace_back();
    double bl[3], bh[3];
    bounds(b, e, bl, bh);
    for (int d = 0; d < 3; ++d) {
      nodes[id].lo[d] = bl[d];
      nodes[id].hi[d] = bh[d];
    }
    if (e - b <= kMeshLeaf) {
      nodes[id].first = b;
      nodes[id].count = e - b;
      return id;
    }
    double cl[3] = {1e300, 1e300, 1e300}, ch[3] = {-1e300, -1e300, -1e300};
    for (int32_t k = b; k < e; ++k)
      for (int d = 0; d < 3; ++d) {
        cl[d] = std::min(cl[d], cen[3 * order[k] + d]);
        ch[d] = std::max(ch[d], cen[3 * order[k] + d]);
      }
    int ax = 0;
    for (int d = 1; d < 3; ++d)
      if (ch[d] - cl[d] > ch[ax] - cl[ax]) ax = d;
    const int32_t mid = b + (e - b) / 2;
    std::nth_element(order.begin() + b, order.begin() + mid, order.begin() + e, [&](int32_t p, int32_t q) {
      const double a = cen[3 * p + ax], c = cen[3 * q + ax];
      return a < c || (a == c && p < q);
    });
    const int32_t l = build(b, mid);
    const int32_t r = build(mid, e);
    nodes[id].first = l;
    nodes[id].count = -r;   // internal node: children l and r
    return id;
  }
};

}  // namespace

void build_mesh(const MeshInput& m, MeshHost& out) {
  const int32_t nv = m.nvert, nt = m.ntri;
  if (nv < 4 || nt < 4) throw ArgError("a closed surface needs at least 4 vertices and 4 triangles");
  auto P = [&](int32_t v) { return V3{m.verts[3 * v], m.verts[3 * v + 1], m.verts[3 * v + 2]}; };
  for (int64_t k = 0; k < 3 * (int64_t)nv; ++k)
    if (!std::isfinite(m.verts[k])) throw ArgError("non-finite vertex coordinate");
  // half-edges: directed edge (a, b) of triangle t; its twin is (b, a)
  std::unordered_map<uint64_t, int64_t> half;   // key (a, b) -> half-edge id 3 t + j
  half.reserve((size_t)nt * 3 * 2);
  auto key = [](int32_t a, int32_t b) { return ((uint64_t)(uint32_t)a << 32) | (uint32_t)b; };
  for (int32_t t = 0; t < nt; ++t)
    for (int j = 0; j < 3; ++j) {
      const int32_t a = m.tris[3 * t + j], b = m.tris[3 * t + (j + 1) % 3];
      if (a < 0 || a >= nv || b < 0 || b >= nv || a == b) throw GeomError("triangle with a bad vertex index");
      if (!half.emplace(key(a, b), 3 * (int64_t)t + j).second)
        throw GeomError("edge used twice in one direction: the surface is not an oriented two-manifold");
    }
  std::vector<int64_t> twin((size_t)nt * 3);
  for (int32_t t = 0; t < nt; ++t)
    for (int j = 0; j < 3; ++j) {
      const int32_t a = m.tris[3 * t + j], b = m.tris[3 * t + (j + 1) % 3];
      const auto it = half.find(key(b, a));
      if (it == half.end()) throw GeomError("edge without an opposite half-edge: the surface is not watertight");
      twin[3 * (size_t)t + j] = it->second;
    }
  // face normals (the winding gives the outward side) and areas
  std::vector<V3> fn(nt);
  for (int32_t t = 0; t < nt; ++t) {
    const V3 a = P(m.tris[3 * t]), b = P(m.tris[3 * t + 1]), c = P(m.tris[3 * t + 2]);
    const V3 n = cross(sub(b, a), sub(c, a));
    if (!(norm(n) > 0)) throw GeomError("degenerate triangle (zero area)");
    fn[t] = unit(n);
  }
  // vertex pseudonormals: incident face normals weighted by the face angle
  std::vector<V3> vn(nv, V3{0, 0, 0});
  for (int32_t t = 0; t < nt; ++t)
    for (int j = 0; j < 3; ++j) {
      const int32_t v = m.tris[3 * t + j];
      const V3 e1 = unit(sub(P(m.tris[3 * t + (j + 1) % 3]), P(v)));
      const V3 e2 = unit(sub(P(m.tris[3 * t + (j + 2) % 3]), P(v)));
      const double ang = std::acos(std::max(-1.0, std::min(1.0, dot(e1, e2))));
      vn[v] = add(vn[v], scl(fn[t], ang));
    }
  // per triangle: vertices, face normal, edge and vertex pseudonormals
  out.ntri = nt;
  out.tri.assign((size_t)nt * kMeshTriDoubles, 0.0);
  for (int32_t t = 0; t < nt; ++t) {
    double* r = &out.tri[(size_t)t * kMeshTriDoubles];
    for (int j = 0; j < 3; ++j) {
      const V3 p = P(m.tris[3 * t + j]);
      r[3 * j] = p.x;
      r[3 * j + 1] = p.y;
      r[3 * j + 2] = p.z;
    }
    r[9] = fn[t].x;
    r[10] = fn[t].y;
    r[11] = fn[t].z;
    for (int j = 0; j < 3; ++j) {   // edge j joins vertex j and vertex j+1
      const int64_t o = twin[3 * (size_t)t + j];
      const V3 en = unit(add(fn[t], fn[o / 3]));
      r[12 + 3 * j] = en.x;
      r[13 + 3 * j] = en.y;
      r[14 + 3 * j] = en.z;
    }
    for (int j = 0; j < 3; ++j) {
      const V3 n = unit(vn[m.tris[3 * t + j]]);
      r[21 + 3 * j] = n.x;
      r[22 + 3 * j] = n.y;
      r[23 + 3 * j] = n.z;
    }
  }
  // the tree over the triangles; the triangle records follow the leaf order
  Builder B(m);
  B.order.resize(nt);
  std::iota(B.order.begin(), B.order.end(), 0);
  B.cen.resize(3 * (size_t)nt);
  B.lo.resize(3 * (size_t)nt);
  B.hi.resize(3 * (size_t)nt);
  for (int32_t t = 0; t < nt; ++t) {
    const double* r = &out.tri[(size_t)t * kMeshTriDoubles];
    for (int d = 0; d < 3; ++d) {
      B.cen[3 * t + d] = (r[d] + r[3 + d] + r[6 + d]) / 3.0;
      B.lo[3 * t + d] = std::min(r[d], std::min(r[3 + d], r[6 + d]));
      B.hi[3 * t + d] = std::max(r[d], std::max(r[3 + d], r[6 + d]));
    }
  }
  B.nodes.reserve(2 * (size_t)nt / kMeshLeaf + 2);
  B.build(0, nt);
  std::vector<double> sorted((size_t)nt * kMeshTriDoubles);
  for (int32_t k = 0; k < nt; ++k)
    std::memcpy(&sorted[(size_t)k * kMeshTriDoubles], &out.tri[(size_t)B.order[k] * kMeshTriDoubles],
                sizeof(double) * kMeshTriDoubles);
  out.tri.swap(sorted);
  out.nodes.swap(B.nodes);
  int depth = 0;
  // depth of the tree (for the device traversal stack)
  std::vector<std::pair<int32_t, int>> st{{0, 1}};
  while (!st.empty()) {
    auto [n, d] = st.back();
    st.pop_back();
    depth = std::max(depth, d);
    if (out.nodes[n].count < 0) {
      st.push_back({out.nodes[n].first, d + 1});
      st.push_back({-out.nodes[n].count, d + 1});
    }
  }
  out.depth = depth;
}

}  // namespace ebmg
