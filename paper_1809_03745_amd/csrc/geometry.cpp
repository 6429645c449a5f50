// Cut-cell geometry from node-sampled signed distances (host side).
//
// Spatial-discretisation section of arXiv:1809.03745: the boundary is the
// zero set of a level set, linearised inside each cut cell (segments in 2D,
// planar facets in 3D), and each cut cell keeps its volume fraction, face
// apertures and centroids, and an EB facet (area fraction, centroid, outward
// normal). Formulas (the paper defers them to the EBChombo documentation):
//   * a phase occupies s > 0; along an edge whose ends differ in sign the
//     crossing is at t = s_a/(s_a - s_b) from the lower node a;
//   * a face (2D: edge, 3D: square) keeps the area and centroid of its wet
//     part, the square's wet part being the polygon of inside corners and
//     crossings (four crossings = saddle, rejected);
//   * 2D cell: exact polygon area/centroid; EB = segment between crossings;
//   * 3D cell: EB = triangle fan from the mean of the crossing loop (one loop
//     only), volume and centroid of the closed polyhedron from cones over its
//     faces with apex at the cell centre;
//   * EB area vector from closure: sum_d (alpha_lo - alpha_hi) e_d;
//   * kappa < 1e-12 is covered, alpha < 1e-12 closed;
//   * a cell cut by two objects is rejected; a gas/dielectric interface cell
//     carries one unknown per phase sharing the gas facet.
#include <algorithm>
#include <cmath>
#include <cstring>

#include "internal.hpp"

namespace ebmg {

namespace {

inline double cross_t(double sa, double sb) { return sa / (sa - sb); }

struct Poly {
  double v[8][2];
  int nv = 0;
  double x[4][2];
  int nx = 0;
};

// Wet polygon of the unit square (corners (0,0),(1,0),(1,1),(0,1)), walked
// counter-clockwise. Throws on a saddle.
void square_walk(double c00, double c10, double c11, double c01, Poly& P) {
  bool i0 = c00 > 0, i1 = c10 > 0, i2 = c11 > 0, i3 = c01 > 0;
  P.nv = P.nx = 0;
  auto push = [&](double u, double v, bool cr) {
    P.v[P.nv][0] = u;
    P.v[P.nv][1] = v;
    ++P.nv;
    if (cr) {
      P.x[P.nx][0] = u;
      P.x[P.nx][1] = v;
      ++P.nx;
    }
  };
  if (i0) push(0.0, 0.0, false);
  if (i0 != i1) push(cross_t(c00, c10), 0.0, true);
  if (i1) push(1.0, 0.0, false);
  if (i1 != i2) push(1.0, cross_t(c10, c11), true);
  if (i2) push(1.0, 1.0, false);
  if (i2 != i3) push(cross_t(c01, c11), 1.0, true);
  if (i3) push(0.0, 1.0, false);
  if (i3 != i0) push(0.0, cross_t(c00, c01), true);
  if (P.nx == 4) throw GeomError("saddle square in the level set");
}

// shoelace area and centroid
void poly_moments(const Poly& P, double& area, double& cu, double& cv) {
  if (P.nv < 3) {
    area = 0.0;
    cu = cv = 0.5;
    return;
  }
  double a = 0, sx = 0, sy = 0;
  for (int k = 0; k < P.nv; ++k) {
    const double* p = P.v[k];
    const double* q = P.v[(k + 1) % P.nv];
    double cr = p[0] * q[1] - q[0] * p[1];
    a += cr;
    sx += (p[0] + q[0]) * cr;
    sy += (p[1] + q[1]) * cr;
  }
  a *= 0.5;
  if (a <= 0.0) {
    area = 0.0;
    cu = cv = 0.5;
    return;
  }
  area = a;
  cu = sx / (6.0 * a);
  cv = sy / (6.0 * a);
}

void edge_wet(double sa, double sb, double& len, double& cen) {
  bool ia = sa > 0, ib = sb > 0;
  if (ia && ib) {
    len = 1.0;
    cen = 0.5;
  } else if (!ia && !ib) {
    len = 0.0;
    cen = 0.5;
  } else {
    double t = cross_t(sa, sb);
    if (ia) {
      len = t;
      cen = 0.5 * t;
    } else {
      len = 1.0 - t;
      cen = 0.5 * (1.0 + t);
    }
  }
}

// transverse axes of d in increasing order
inline void transverse(int dim, int d, int* tr) {
  int m = 0;
  for (int e = 0; e < dim; ++e)
    if (e != d) tr[m++] = e;
}

struct PhaseBuilder {
  const Grid& g;
  Phase& P;
  PhaseBuilder(const Grid& g_, Phase& P_) : g(g_), P(P_) {}

  double sv(int i, int j, int k) const { return P.s[g.node(i, j, k)]; }

  // corner values of face (d, c) in (u, v) order
  void face_corners(int d, const int* c, double* out) const {
    int i = c[0], j = c[1], k = c[2];
    if (g.dim == 2) {
      if (d == 0) {
        out[0] = sv(i, j, 0);
        out[1] = sv(i, j + 1, 0);
      } else {
        out[0] = sv(i, j, 0);
        out[1] = sv(i + 1, j, 0);
      }
      return;
    }
    if (d == 0) {
      out[0] = sv(i, j, k); out[1] = sv(i, j + 1, k); out[2] = sv(i, j + 1, k + 1); out[3] = sv(i, j, k + 1);
    } else if (d == 1) {
      out[0] = sv(i, j, k); out[1] = sv(i + 1, j, k); out[2] = sv(i + 1, j, k + 1); out[3] = sv(i, j, k + 1);
    } else {
      out[0] = sv(i, j, k); out[1] = sv(i + 1, j, k); out[2] = sv(i + 1, j + 1, k); out[3] = sv(i, j + 1, k);
    }
  }

  // record face (d, c) if it is cut; returns its aperture
  double face(int d, const int* c) {
    int64_t key = g.face(d, c[0], c[1], c[2]);
    auto it = P.fcut[d].find(key);
    if (it != P.fcut[d].end()) return it->second.alpha;
    double cv[4];
    face_corners(d, c, cv);
    int nc = g.dim == 2 ? 2 : 4;
    int nin = 0;
    for (int q = 0; q < nc; ++q) nin += cv[q] > 0;
    if (nin == nc) return 1.0;
    if (nin == 0) return 0.0;
    FaceCut fc;
    if (g.dim == 2) {
      double len, cen;
      edge_wet(cv[0], cv[1], len, cen);
      fc.alpha = len;
      fc.off[0] = cen - 0.5;
      fc.off[1] = 0.0;
    } else {
      Poly Q;
      square_walk(cv[0], cv[1], cv[2], cv[3], Q);
      double a, cu, cw;
      if (nin == 4) {
        a = 1.0; cu = cw = 0.5;
      } else {
        poly_moments(Q, a, cu, cw);
      }
      fc.alpha = a;
      fc.off[0] = cu - 0.5;
      fc.off[1] = cw - 0.5;
    }
    if (fc.alpha < kTiny) fc.alpha = 0.0;
    P.fcut[d].emplace(key, fc);
    return fc.alpha;
  }

  void cell2(int i, int j, CellCut& cc) {
    Poly Q;
    square_walk(sv(i, j, 0), sv(i + 1, j, 0), sv(i + 1, j + 1, 0), sv(i, j + 1, 0), Q);
    double a, cu, cv;
    poly_moments(Q, a, cu, cv);
    double h = g.h;
    double x0 = g.lo[0] + i * h, y0 = g.lo[1] + j * h;
    cc.kappa = a;
    cc.vc[0] = x0 + cu * h;
    cc.vc[1] = y0 + cv * h;
    cc.vc[2] = 0;
    cc.eb_area = 0;
    cc.eb_c[0] = cc.eb_c[1] = cc.eb_c[2] = 0;
    cc.eb_n[0] = cc.eb_n[1] = cc.eb_n[2] = 0;
    if (Q.nx == 2) {
      cc.eb_c[0] = x0 + 0.5 * (Q.x[0][0] + Q.x[1][0]) * h;
      cc.eb_c[1] = y0 + 0.5 * (Q.x[0][1] + Q.x[1][1]) * h;
      int c0[3] = {i, j, 0}, c1[3] = {i + 1, j, 0}, c2[3] = {i, j + 1, 0};
      double vx = face(0, c0) - face(0, c1);
      double vy = face(1, c0) - face(1, c2);
      double nrm = std::hypot(vx, vy);
      cc.eb_area = nrm;
      if (nrm > 0) {
        cc.eb_n[0] = vx / nrm;
        cc.eb_n[1] = vy / nrm;
      }
    }
  }

  void cell3(int i, int j, int k, CellCut& cc) {
    const double h = g.h;
    const double x0[3] = {g.lo[0] + i * h, g.lo[1] + j * h, g.lo[2] + k * h};
    const double xc[3] = {x0[0] + 0.5 * h, x0[1] + 0.5 * h, x0[2] + 0.5 * h};
    const int base[3] = {i, j, k};
    // edge crossings: id = ax*4 + a + 2*b, (a, b) offsets of the transverse axes
    bool has[12] = {};
    double pt[12][3];
    int nx = 0;
    for (int ax = 0; ax < 3; ++ax) {
      int tr[2];
      transverse(3, ax, tr);
      for (int b = 0; b < 2; ++b)
        for (int a = 0; a < 2; ++a) {
          int o[3] = {0, 0, 0};
          o[tr[0]] = a;
          o[tr[1]] = b;
          int o2[3] = {o[0], o[1], o[2]};
          o2[ax] = 1;
          double sa = sv(i + o[0], j + o[1], k + o[2]);
          double sb = sv(i + o2[0], j + o2[1], k + o2[2]);
          if ((sa > 0) != (sb > 0)) {
            int id = ax * 4 + a + 2 * b;
            has[id] = true;
            for (int e = 0; e < 3; ++e) pt[id][e] = x0[e] + o[e] * h;
            pt[id][ax] += cross_t(sa, sb) * h;
            ++nx;
          }
        }
    }
    double vol = 0, mom[3] = {0, 0, 0};
    double alo[3], ahi[3];
    int adj[12][2];
    int nadj[12] = {};
    for (int d = 0; d < 3; ++d) {
      int tr[2];
      transverse(3, d, tr);
      for (int side = 0; side < 2; ++side) {
        int c[3] = {i, j, k};
        c[d] += side;
        double a = face(d, c);
        (side ? ahi : alo)[d] = a;
        if (a > 0) {
          double off[2] = {0, 0};
          auto it = P.fcut[d].find(g.face(d, c[0], c[1], c[2]));
          if (it != P.fcut[d].end()) {
            off[0] = it->second.off[0];
            off[1] = it->second.off[1];
          }
          double fc[3] = {x0[0], x0[1], x0[2]};
          fc[d] += side * h;
          fc[tr[0]] += (0.5 + off[0]) * h;
          fc[tr[1]] += (0.5 + off[1]) * h;
          double cone = a * h * h * (0.5 * h) / 3.0;
          vol += cone;
          for (int e = 0; e < 3; ++e) mom[e] += cone * (xc[e] + 0.75 * (fc[e] - xc[e]));
        }
        // crossings on this face's four edges -> one facet segment
        int ends[4], ne = 0;
        for (int id = 0; id < 12; ++id) {
          if (!has[id]) continue;
          int ax = id / 4;
          if (ax == d) continue;
          int t2[2];
          transverse(3, ax, t2);
          int a_ = id % 2, b_ = (id / 2) % 2;
          int od = (t2[0] == d) ? a_ : b_;
          if (od == side) ends[ne++] = id;
        }
        if (ne == 4) throw GeomError("saddle face in a cut cell");
        if (ne == 2) {
          adj[ends[0]][nadj[ends[0]]++] = ends[1];
          adj[ends[1]][nadj[ends[1]]++] = ends[0];
        }
      }
    }
    cc.eb_area = 0;
    for (int e = 0; e < 3; ++e) cc.eb_c[e] = cc.eb_n[e] = 0;
    if (nx > 0) {
      int start = -1;
      for (int id = 0; id < 12; ++id)
        if (has[id]) {
          start = id;
          break;
        }
      int loop[12], nl = 0;
      int prev = -1, cur = start;
      while (true) {
        if (nadj[cur] != 2) throw GeomError("open crossing loop in a cut cell");
        loop[nl++] = cur;
        int nxt = adj[cur][0] != prev ? adj[cur][0] : adj[cur][1];
        prev = cur;
        cur = nxt;
        if (cur == start) break;
        if (nl >= 12) throw GeomError("bad crossing loop in a cut cell");
      }
      if (nl != nx) throw GeomError("multi-valued cut cell");
      double cl[3] = {alo[0] - ahi[0], alo[1] - ahi[1], alo[2] - ahi[2]};
      double m[3] = {0, 0, 0};
      for (int q = 0; q < nl; ++q)
        for (int e = 0; e < 3; ++e) m[e] += pt[loop[q]][e];
      for (int e = 0; e < 3; ++e) m[e] /= nl;
      double tri_a[12][3], tri_c[12][3], tot[3] = {0, 0, 0};
      for (int q = 0; q < nl; ++q) {
        const double* a = pt[loop[q]];
        const double* b = pt[loop[(q + 1) % nl]];
        double u[3] = {a[0] - m[0], a[1] - m[1], a[2] - m[2]};
        double v[3] = {b[0] - m[0], b[1] - m[1], b[2] - m[2]};
        tri_a[q][0] = 0.5 * (u[1] * v[2] - u[2] * v[1]);
        tri_a[q][1] = 0.5 * (u[2] * v[0] - u[0] * v[2]);
        tri_a[q][2] = 0.5 * (u[0] * v[1] - u[1] * v[0]);
        for (int e = 0; e < 3; ++e) {
          tri_c[q][e] = (m[e] + a[e] + b[e]) / 3.0;
          tot[e] += tri_a[q][e];
        }
      }
      double sgn = (tot[0] * cl[0] + tot[1] * cl[1] + tot[2] * cl[2]) >= 0.0 ? 1.0 : -1.0;
      double nrm = std::sqrt(cl[0] * cl[0] + cl[1] * cl[1] + cl[2] * cl[2]);
      cc.eb_area = nrm;
      if (nrm > 0)
        for (int e = 0; e < 3; ++e) cc.eb_n[e] = cl[e] / nrm;
      double wsum = 0, cen[3] = {0, 0, 0};
      for (int q = 0; q < nl; ++q) {
        double av[3] = {sgn * tri_a[q][0], sgn * tri_a[q][1], sgn * tri_a[q][2]};
        double w = std::sqrt(av[0] * av[0] + av[1] * av[1] + av[2] * av[2]);
        wsum += w;
        double cone = 0;
        for (int e = 0; e < 3; ++e) {
          cen[e] += w * tri_c[q][e];
          cone += (tri_c[q][e] - xc[e]) * av[e];
        }
        cone /= 3.0;
        vol += cone;
        for (int e = 0; e < 3; ++e) mom[e] += cone * (xc[e] + 0.75 * (tri_c[q][e] - xc[e]));
      }
      for (int e = 0; e < 3; ++e) cc.eb_c[e] = wsum > 0 ? cen[e] / wsum : m[e];
    }
    cc.kappa = vol / (h * h * h);
    for (int e = 0; e < 3; ++e) cc.vc[e] = vol > 0 ? mom[e] / vol : xc[e];
  }

  void build() {
    const int64_t N = g.ncell();
    P.cls.assign(N, 0);
    const int nk = g.dim == 3 ? g.n[2] : 1;
    const int ncorner = g.dim == 3 ? 8 : 4;
    for (int k = 0; k < nk; ++k)
      for (int j = 0; j < g.n[1]; ++j)
        for (int i = 0; i < g.n[0]; ++i) {
          int nin = 0;
          for (int q = 0; q < ncorner; ++q)
            nin += sv(i + (q & 1), j + ((q >> 1) & 1), k + ((q >> 2) & 1)) > 0;
          int64_t c = g.cell(i, j, k);
          if (nin == ncorner) {
            P.cls[c] = 1;
          } else if (nin > 0) {
            // record all faces of the cell, then the cell
            for (int d = 0; d < g.dim; ++d)
              for (int side = 0; side < 2; ++side) {
                int cc[3] = {i, j, k};
                cc[d] += side;
                face(d, cc);
              }
            CellCut cut;
            cut.cutter = -1;
            if (g.dim == 2)
              cell2(i, j, cut);
            else
              cell3(i, j, k, cut);
            if (cut.kappa >= kTiny) {
              P.cls[c] = 2;
              P.ccut.emplace(c, cut);
            }
          }
        }
  }
};

}  // namespace

double Geometry::alpha(int p, int d, const int* c) const {
  const Phase& P = ph[p];
  auto it = P.fcut[d].find(g.face(d, c[0], c[1], c[2]));
  if (it != P.fcut[d].end()) return it->second.alpha;
  // uncut face: all corners share a side
  int i = c[0], j = c[1], k = c[2];
  double v = P.s[g.node(i, j, k)];
  return v > 0 ? 1.0 : 0.0;
}

void Geometry::face_off(int p, int d, const int* c, double* off) const {
  const Phase& P = ph[p];
  auto it = P.fcut[d].find(g.face(d, c[0], c[1], c[2]));
  if (it != P.fcut[d].end()) {
    off[0] = it->second.off[0];
    off[1] = it->second.off[1];
  } else {
    off[0] = off[1] = 0.0;
  }
}

double Geometry::kappa(int p, int64_t cell) const {
  if (p >= nphase) return 0.0;
  uint8_t c = ph[p].cls[cell];
  if (c == 1) return 1.0;
  if (c == 0) return 0.0;
  return ph[p].ccut.at(cell).kappa;
}

int64_t Geometry::dof(const int* c, int p) const {
  if (!g.inbox(c)) return -1;
  int64_t cell = g.cell(c[0], c[1], g.dim == 3 ? c[2] : 0);
  if (!has(p, cell)) return -1;
  if (primary[cell] == p) return cell;
  return N + sec_of[cell];
}

void build_geometry(Geometry& geo, const ebmg_box& box, int nobj, const ebmg_object* objs) {
  Grid& g = geo.g;
  g.dim = box.dim;
  if (g.dim != 2 && g.dim != 3) throw ArgError("dim must be 2 or 3");
  for (int d = 0; d < 3; ++d) {
    g.n[d] = d < g.dim ? box.n[d] : 1;
    g.lo[d] = d < g.dim ? box.lo[d] : 0.0;
    if (g.n[d] < 1) throw ArgError("box size must be positive");
  }
  g.h = box.h;
  if (!(g.h > 0)) throw ArgError("h must be positive");
  const int64_t NN = g.nnode();
  int ndiel = 0;
  geo.obj_kind.clear();
  geo.obj_value.clear();
  for (int k = 0; k < nobj; ++k) {
    if (objs[k].kind < 0 || objs[k].kind > 2) throw ArgError("bad object kind");
    if (!objs[k].sdf) throw ArgError("object without level set");
    for (int64_t q = 0; q < NN; ++q)
      if (!std::isfinite(objs[k].sdf[q])) throw ArgError("non-finite level-set value");
    geo.obj_kind.push_back(objs[k].kind);
    geo.obj_value.push_back(objs[k].value);
    if (objs[k].kind == EBMG_OBJ_DIELECTRIC) {
      ++ndiel;
      geo.diel_obj = k;
    }
  }
  if (ndiel > 1) throw ArgError("at most one dielectric object");
  geo.nphase = ndiel ? 2 : 1;
  // phase level sets
  Phase& Pg = geo.ph[0];
  Pg.s.assign(NN, 1.0);
  for (int k = 0; k < nobj; ++k)
    for (int64_t q = 0; q < NN; ++q) Pg.s[q] = k == 0 ? objs[k].sdf[q] : std::min(Pg.s[q], objs[k].sdf[q]);
  if (ndiel) {
    Phase& Pd = geo.ph[1];
    Pd.s.resize(NN);
    const double* dd = objs[geo.diel_obj].sdf;
    for (int64_t q = 0; q < NN; ++q) Pd.s[q] = -dd[q];
    for (int k = 0; k < nobj; ++k) {
      if (k == geo.diel_obj) continue;
      for (int64_t q = 0; q < NN; ++q) Pd.s[q] = std::min(Pd.s[q], objs[k].sdf[q]);
    }
  }
  for (int p = 0; p < geo.nphase; ++p) {
    PhaseBuilder B(g, geo.ph[p]);
    B.build();
  }
  // cutter object of each cut cell (exactly one object may change sign)
  const int ncorner = g.dim == 3 ? 8 : 4;
  for (int p = 0; p < geo.nphase; ++p) {
    for (auto& kv : geo.ph[p].ccut) {
      int64_t c = kv.first;
      int i = (int)(c % g.n[0]);
      int j = (int)((c / g.n[0]) % g.n[1]);
      int k = (int)(c / ((int64_t)g.n[0] * g.n[1]));
      int found = -1, count = 0;
      for (int o = 0; o < nobj; ++o) {
        // cut unless the level set has one strict sign at every corner (a
        // node exactly on the surface belongs to neither side)
        int npos = 0, nneg = 0;
        for (int q = 0; q < ncorner; ++q) {
          const double v = objs[o].sdf[g.node(i + (q & 1), j + ((q >> 1) & 1), k + ((q >> 2) & 1))];
          npos += v > 0;
          nneg += v < 0;
        }
        if (npos < ncorner && nneg < ncorner) {
          found = o;
          ++count;
        }
      }
      if (count != 1) throw GeomError("cell cut by " + std::to_string(count) + " objects");
      kv.second.cutter = found;
    }
  }
  if (geo.nphase == 2) {
    for (auto& kv : geo.ph[1].ccut) {
      CellCut& cd = kv.second;
      auto it = geo.ph[0].ccut.find(kv.first);
      if (it == geo.ph[0].ccut.end()) continue;
      const CellCut& cg = it->second;
      if (cd.cutter == geo.diel_obj && cg.cutter == geo.diel_obj) {
        cd.eb_area = cg.eb_area;
        for (int e = 0; e < 3; ++e) {
          cd.eb_c[e] = cg.eb_c[e];
          cd.eb_n[e] = -cg.eb_n[e];
        }
      }
    }
  }
  // unknowns
  const int64_t N = g.ncell();
  geo.N = N;
  geo.primary.assign(N, -1);
  geo.sec_of.assign(N, -1);
  geo.sec_cell.clear();
  for (int64_t c = 0; c < N; ++c) {
    bool h0 = geo.ph[0].cls[c] != 0;
    bool h1 = geo.nphase == 2 && geo.ph[1].cls[c] != 0;
    geo.primary[c] = h0 ? 0 : (h1 ? 1 : -1);
    if (h0 && h1) {
      geo.sec_of[c] = (int32_t)geo.sec_cell.size();
      geo.sec_cell.push_back(c);
    }
  }
  geo.N2 = (int64_t)geo.sec_cell.size();
}

}  // namespace ebmg
