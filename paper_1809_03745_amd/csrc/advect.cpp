// Host preparation of the advection step on the gas phase of a cut-cell
// grid (Convection-Diffusion-Reaction equations: Advective discretization
// and Hybrid divergence). Everything the step needs that depends on the
// geometry alone is built here once per problem:
//  * a cell class per cell: no gas (0), full cell (1: kappa = 1, every face
//    full, face-centred fluxes are the centroid fluxes), cut cell (2), full
//    cell in the 3^D block of a cut cell (3: its conservative divergence is
//    kept for the cut cell's non-conservative one);
//  * per cut cell, its conservative divergence as a linear form over the
//    face-centred fluxes: sum over its faces of +-alpha_f / (kappa h) times
//    the centroid interpolation weights of that face (the same rule as the
//    Helmholtz fluxes: linear in 2D, bilinear in 3D over the open parallel
//    faces whose two cells carry gas, falling back to linear along the
//    available axis with the larger offset, then face-centred);
//  * per cut cell, the gas cells of its 3^D block with the weights
//    kappa_j / sum kappa of the non-conservative divergence, and the sum S
//    of kappa over the block without the cell (the redistribution weights);
//  * per cell that receives redistributed mass, the cut cells it receives
//    from.
// Face arrays are stored direction by direction (faces normal to x, then y,
// then z), each x fastest with the face axis extended by one.

#include <algorithm>
#include <cmath>

#include "internal.hpp"

namespace ebmg {

namespace {

struct FaceIx {
  const Grid& g;
  int64_t base[3] = {0, 0, 0};
  explicit FaceIx(const Grid& gr) : g(gr) {
    int64_t o = 0;
    for (int d = 0; d < g.dim; ++d) {
      base[d] = o;
      o += (int64_t)(g.n[0] + (d == 0)) * (g.n[1] + (d == 1)) * (g.dim == 3 ? g.n[2] + (d == 2) : 1);
    }
    total = o;
  }
  int64_t total = 0;
  // face d at node plane c[d] (cell-like index c)
  int64_t at(int d, const int* c) const {
    const int64_t m0 = g.n[0] + (d == 0), m1 = g.n[1] + (d == 1);
    return base[d] + c[0] + m0 * (c[1] + m1 * (int64_t)c[2]);
  }
};

}  // namespace

void build_advection(const Geometry& G, AdvHost& A) {
  const Grid& g = G.g;
  const int D = g.dim;
  const double h = g.h;
  const FaceIx fx(g);
  A.nfaces = fx.total;
  for (int d = 0; d < 3; ++d) A.face_base[d] = fx.base[d];
  const int64_t N = G.N;
  A.cls.assign(N, 0);
  A.kappa.assign(N, 0.0);
  for (int64_t c = 0; c < N; ++c) {
    if (!G.has(0, c)) continue;
    const double k = G.kappa(0, c);
    A.kappa[c] = k;
    A.cls[c] = k < 1.0 ? 2 : 1;
  }
  auto gas = [&](const int* c) {
    for (int d = 0; d < D; ++d)
      if (c[d] < 0 || c[d] >= g.n[d]) return false;
    return A.cls[g.cell(c[0], c[1], D == 3 ? c[2] : 0)] != 0;
  };
  // face (d, c) open with both its (in-box) cells carrying gas
  auto face_ok = [&](int d, const int* c) {
    for (int e = 0; e < D; ++e)
      if (c[e] < 0 || c[e] > g.n[e] - (e == d ? 0 : 1)) return false;
    if (!(G.alpha(0, d, c) > 0.0)) return false;
    int lo[3] = {c[0], c[1], c[2]};
    lo[d] -= 1;
    if (lo[d] >= 0 && !gas(lo)) return false;
    if (c[d] < g.n[d] && !gas(c)) return false;
    return true;
  };
  // centroid-interpolated flux of face (d, c) as weights over face fluxes
  auto centroid = [&](int d, const int* c, std::vector<std::pair<int64_t, double>>& w) {
    w.clear();
    double off[2];
    G.face_off(0, d, c, off);
    int tr[2], nt = 0;
    for (int e = 0; e < D; ++e)
      if (e != d) tr[nt++] = e;
    int ax[2];
    double sv[2];
    int na = 0;
    for (int q = 0; q < D - 1; ++q)
      if (std::fabs(off[q]) >= kTiny) {
        ax[na] = tr[q];
        sv[na] = off[q];
        ++na;
      }
    const int64_t f0 = fx.at(d, c);
    auto shifted = [&](int e1, int s1, int e2, int s2, int64_t& f) {
      int q[3] = {c[0], c[1], c[2]};
      if (e1 >= 0) q[e1] += s1;
      if (e2 >= 0) q[e2] += s2;
      if (!face_ok(d, q)) return false;
      f = fx.at(d, q);
      return true;
    };
    if (na == 0) {
      w.emplace_back(f0, 1.0);
      return;
    }
    if (na == 1) {
      int64_t f1;
      const double u = std::fabs(sv[0]);
      if (shifted(ax[0], sv[0] > 0 ? 1 : -1, -1, 0, f1)) {
        w.emplace_back(f0, 1.0 - u);
        w.emplace_back(f1, u);
      } else {
        w.emplace_back(f0, 1.0);
      }
      return;
    }
    const int d1 = sv[0] > 0 ? 1 : -1, d2 = sv[1] > 0 ? 1 : -1;
    const double u1 = std::fabs(sv[0]), u2 = std::fabs(sv[1]);
    int64_t f1 = 0, f2 = 0, f12 = 0;
    const bool h1 = shifted(ax[0], d1, -1, 0, f1), h2 = shifted(ax[1], d2, -1, 0, f2);
    const bool h12 = shifted(ax[0], d1, ax[1], d2, f12);
    if (h1 && h2 && h12) {
      w.emplace_back(f0, (1 - u1) * (1 - u2));
      w.emplace_back(f1, u1 * (1 - u2));
      w.emplace_back(f2, (1 - u1) * u2);
      w.emplace_back(f12, u1 * u2);
      return;
    }
    // linear along the available axis with the larger offset (ties: lower axis)
    int pick = -1;
    if (h1 && h2)
      pick = u2 > u1 ? 1 : 0;
    else if (h1)
      pick = 0;
    else if (h2)
      pick = 1;
    if (pick < 0) {
      w.emplace_back(f0, 1.0);
      return;
    }
    const double u = pick == 0 ? u1 : u2;
    w.emplace_back(f0, 1.0 - u);
    w.emplace_back(pick == 0 ? f1 : f2, u);
  };
  A.cut_cell.clear();
  A.dc_ptr.assign(1, 0);
  A.dc_face.clear();
  A.dc_coef.clear();
  A.nb_ptr.assign(1, 0);
  A.nb_cell.clear();
  A.nb_w.clear();
  A.cut_S.clear();
  std::vector<std::pair<int64_t, double>> w;
  std::vector<int32_t> cut_id(N, -1);
  const int nz = D == 3 ? g.n[2] : 1;
  for (int k = 0; k < nz; ++k)
    for (int j = 0; j < g.n[1]; ++j)
      for (int i = 0; i < g.n[0]; ++i) {
        const int64_t c = g.cell(i, j, k);
        if (A.cls[c] != 2) continue;
        cut_id[c] = (int32_t)A.cut_cell.size();
        A.cut_cell.push_back(c);
        const double kap = A.kappa[c];
        const int ijk[3] = {i, j, k};
        for (int d = 0; d < D; ++d)
          for (int side = 0; side < 2; ++side) {
            int fcell[3] = {i, j, k};
            fcell[d] += side;
            const double a = G.alpha(0, d, fcell);
            if (!(a > 0.0)) continue;
            centroid(d, fcell, w);
            const double sg = side ? 1.0 : -1.0;
            for (auto& e : w) {
              A.dc_face.push_back(e.first);
              A.dc_coef.push_back(sg * a * e.second / (kap * h));
            }
          }
        A.dc_ptr.push_back((int64_t)A.dc_face.size());
        // the gas cells of the 3^D block, in z, y, x order
        double ks = 0, S = 0;
        const int64_t nb0 = (int64_t)A.nb_cell.size();
        for (int dz = (D == 3 ? -1 : 0); dz <= (D == 3 ? 1 : 0); ++dz)
          for (int dy = -1; dy <= 1; ++dy)
            for (int dx = -1; dx <= 1; ++dx) {
              const int q[3] = {ijk[0] + dx, ijk[1] + dy, ijk[2] + dz};
              if (!gas(q)) continue;
              const int64_t qc = g.cell(q[0], q[1], q[2]);
              A.nb_cell.push_back(qc);
              if (A.cls[qc] == 1) A.cls[qc] = 3;   // a full cell whose D^c the block needs
              A.nb_w.push_back(A.kappa[qc]);
              ks += A.kappa[qc];
              if (qc != c) S += A.kappa[qc];
            }
        for (int64_t e = nb0; e < (int64_t)A.nb_cell.size(); ++e) A.nb_w[e] /= ks;
        A.nb_ptr.push_back((int64_t)A.nb_cell.size());
        A.cut_S.push_back(S);
      }
  // receivers: gas cells in the block of a cut cell with S > 0, other than
  // that cell; each with its donors (cut ids, in cut order)
  std::vector<std::vector<int32_t>> don(N);
  std::vector<int64_t> order;
  for (size_t q = 0; q < A.cut_cell.size(); ++q) {
    if (!(A.cut_S[q] > 0)) continue;
    for (int64_t e = A.nb_ptr[q]; e < A.nb_ptr[q + 1]; ++e) {
      const int64_t r = A.nb_cell[e];
      if (r == A.cut_cell[q]) continue;
      if (don[r].empty()) order.push_back(r);
      don[r].push_back((int32_t)q);
    }
  }
  // the cells whose final rate is not their conservative divergence: every
  // cut cell and every receiver, each once, in cell order
  for (int64_t c : A.cut_cell)
    if (don[c].empty()) order.push_back(c);
  std::sort(order.begin(), order.end());
  A.sp_cell = order;
  A.sp_cut.assign(order.size(), -1);
  A.sp_ptr.assign(1, 0);
  A.sp_donor.clear();
  for (size_t s = 0; s < order.size(); ++s) {
    const int64_t c = order[s];
    A.sp_cut[s] = cut_id[c];
    for (int32_t q : don[c]) A.sp_donor.push_back(q);
    A.sp_ptr.push_back((int64_t)A.sp_donor.size());
  }
}

}  // namespace ebmg
