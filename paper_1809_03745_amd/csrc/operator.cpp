// Finest-level operator of the embedded-boundary finite-volume system.
//
// Helmholtz-equations section of arXiv:1809.03745. Row of unknown (cell i,
// phase p) in the volume-weighted integral form
//   L_i = kappa_i alpha a_p phi_i + (beta/h)[sum_f alpha_f Fbar_f + alpha_EB F_EB],
// every flux outward; b_i = kappa_i rho_i - L_i(0). Face-centred fluxes
// b_p (phi_R - phi_L)/h are interpolated to face centroids (linear in 2D,
// bilinear in 3D with linear / face-centred fallbacks when a neighbour face is
// missing). Domain faces: Neumann, Dirichlet (linear two-point by default,
// quadratic one-sided as an option), Robin (linear extrapolation, Taylor
// option). EB Dirichlet: normal derivative from ray casting to the planes of
// cell centres one and two cells away along the dominant normal axis with
// quadratic transverse interpolation (order 2, the cut cell never used), or
// one plane and linear interpolation (order 1); least squares over the
// unknowns (and Dirichlet domain-face centres) in front of the facet when a
// ray stencil is not available, and for slivers against Dirichlet box faces
// a one-sided difference toward the face. Multifluid facets: one stencil per side and
// elimination of the boundary state from
//   eps_g dphi/dm_g + eps_s dphi/dm_s = -sigma   (m_q into phase q).
// Cells whose row is the plain (2D+1)-point template (full cell of its primary
// phase, every in-box neighbour of the same primary phase, a two-point domain
// closure) are tagged regular and computed on the fly by the kernels; every
// other unknown gets an explicit sparse row.
#include <algorithm>
#include <array>
#include <cmath>

#include "internal.hpp"

namespace ebmg {

void Data::axpy(double w, const Data& o) {
  for (int f = 0; f < 6; ++f) face[f] += w * o.face[f];
  if (o.obj >= 0) {
    if (obj >= 0 && obj != o.obj) throw GeomError("row references two objects");
    obj = o.obj;
    cobj += w * o.cobj;
  }
  csig += w * o.csig;
}

void Form::add(int64_t col, double v) {
  for (auto& e : c)
    if (e.first == col) {
      e.second += v;
      return;
    }
  c.emplace_back(col, v);
}

void Form::axpy(double w, const Form& o) {
  if (w == 0.0) return;
  for (auto& e : o.c) add(e.first, w * e.second);
  d.axpy(w, o.d);
}

namespace {

struct Builder {
  const Problem& pb;
  const Geometry& geo;
  const Grid& g;
  explicit Builder(const Problem& p) : pb(p), geo(p.geo), g(p.geo.g) {}

  int64_t dof(const int* c, int p) const {
    int cc[3] = {c[0], c[1], g.dim == 3 ? c[2] : 0};
    return geo.dof(cc, p);
  }

  // face-centred outward flux of face (d, side) of cell c
  bool centred_out(const int* c, int p, int d, int side, Form& f) const {
    const double b = pb.bph[p], h = g.h;
    int64_t me = dof(c, p);
    if (me < 0) return false;
    int nb[3] = {c[0], c[1], c[2]};
    nb[d] += side ? 1 : -1;
    f.c.clear();
    f.d = Data();
    if (nb[d] >= 0 && nb[d] < g.n[d]) {
      int64_t j = dof(nb, p);
      if (j < 0) return false;
      f.add(j, b / h);
      f.add(me, -b / h);
      return true;
    }
    const int fid = 2 * d + side;
    const int kind = pb.bc.kind[fid];
    int nn[3] = {c[0], c[1], c[2]};
    nn[d] += side ? -1 : 1;
    int64_t jn = (nn[d] >= 0 && nn[d] < g.n[d]) ? dof(nn, p) : -1;
    if (kind == EBMG_BC_NEUMANN) {
      f.d.face[fid] = b;
    } else if (kind == EBMG_BC_DIRICHLET) {
      if (pb.opt.dirichlet_closure == 1 && jn >= 0) {
        f.add(me, -3.0 * b / h);
        f.add(jn, (1.0 / 3.0) * b / h);
        f.d.face[fid] = (8.0 / 3.0) * b / h;
      } else {
        f.add(me, -2.0 * b / h);
        f.d.face[fid] = 2.0 * b / h;
      }
    } else {
      const double a1 = pb.bc.robin_a1[fid], a2 = pb.bc.robin_a2[fid];
      if (pb.opt.robin_closure == 1 && jn >= 0) {
        f.add(me, -(b / a2) * a1 * 1.5);
        f.add(jn, (b / a2) * a1 * 0.5);
        f.d.face[fid] = b / a2;
      } else {
        const double cc = 1.0 / (1.0 + 0.5 * h * a1 / a2);
        f.add(me, -(b * a1 / a2) * cc);
        f.d.face[fid] = (b / a2) * (1.0 - a1 * cc * 0.5 * h / a2);
      }
    }
    return true;
  }

  double aperture(int p, int d, const int* c, int side) const {
    int fi[3] = {c[0], c[1], g.dim == 3 ? c[2] : 0};
    fi[d] += side;
    return geo.alpha(p, d, fi);
  }

  bool shifted(const int* c, int p, int d, int side, int e1, int s1, int e2, int s2, Form& f) const {
    int sc[3] = {c[0], c[1], c[2]};
    if (e1 >= 0) sc[e1] += s1;
    if (e2 >= 0) sc[e2] += s2;
    if (!g.inbox(sc)) return false;
    if (aperture(p, d, sc, side) <= 0.0) return false;
    return centred_out(sc, p, d, side, f);
  }

  // centroid-interpolated outward flux; returns the aperture (0 if closed)
  double face_out(const int* c, int p, int d, int side, Form& out) const {
    double a = aperture(p, d, c, side);
    if (a <= 0.0) return 0.0;
    Form base;
    if (!centred_out(c, p, d, side, base)) return 0.0;
    int fi[3] = {c[0], c[1], g.dim == 3 ? c[2] : 0};
    fi[d] += side;
    double off[2];
    geo.face_off(p, d, fi, off);
    int tr[2], m = 0;
    for (int e = 0; e < g.dim; ++e)
      if (e != d) tr[m++] = e;
    int ax[2];
    double sv[2];
    int na = 0;
    for (int q = 0; q < g.dim - 1; ++q)
      if (std::fabs(off[q]) >= kTiny) {
        ax[na] = tr[q];
        sv[na] = off[q];
        ++na;
      }
    out = Form();
    if (na == 0) {
      out = base;
      return a;
    }
    if (na == 1) {
      Form f1;
      if (!shifted(c, p, d, side, ax[0], sv[0] > 0 ? 1 : -1, -1, 0, f1)) {
        out = base;
        return a;
      }
      double u = std::fabs(sv[0]);
      out.axpy(1.0 - u, base);
      out.axpy(u, f1);
      return a;
    }
    const int d1 = sv[0] > 0 ? 1 : -1, d2 = sv[1] > 0 ? 1 : -1;
    Form f1, f2, f12;
    bool h1 = shifted(c, p, d, side, ax[0], d1, -1, 0, f1);
    bool h2 = shifted(c, p, d, side, ax[1], d2, -1, 0, f2);
    bool h12 = shifted(c, p, d, side, ax[0], d1, ax[1], d2, f12);
    const double u1 = std::fabs(sv[0]), u2 = std::fabs(sv[1]);
    if (h1 && h2 && h12) {
      out.axpy((1 - u1) * (1 - u2), base);
      out.axpy(u1 * (1 - u2), f1);
      out.axpy((1 - u1) * u2, f2);
      out.axpy(u1 * u2, f12);
      return a;
    }
    // linear along the available axis with the larger |s| (ties: lower axis)
    bool use1 = h1, use2 = h2;
    if (use1 && use2) {
      if (u2 > u1) use1 = false;
      else use2 = false;
    }
    if (use1) {
      out.axpy(1.0 - u1, base);
      out.axpy(u1, f1);
    } else if (use2) {
      out.axpy(1.0 - u2, base);
      out.axpy(u2, f2);
    } else {
      out = base;
    }
    return a;
  }

  // ray stencil for dphi/dm at xb; false if unavailable
  bool ray(const int* c, int p, const double* xb, const double* m, int order, double& wB, Form& S) const {
    const int dim = g.dim;
    const double h = g.h;
    double mx = 0;
    for (int d = 0; d < dim; ++d) mx = std::max(mx, std::fabs(m[d]));
    int ds = 0;
    for (int d = 0; d < dim; ++d)
      if (std::fabs(m[d]) >= mx - 1e-12) {
        ds = d;
        break;
      }
    const int sr = m[ds] > 0 ? 1 : -1;
    const int nk = order == 2 ? 2 : 1;
    double t[2];
    Form val[2];
    for (int kk = 0; kk < nk; ++kk) {
      const int plane = c[ds] + (kk + 1) * sr;
      if (plane < 0 || plane >= g.n[ds]) return false;
      const double xp = g.lo[ds] + (plane + 0.5) * h;
      t[kk] = (xp - xb[ds]) / m[ds];
      double pt[3];
      for (int d = 0; d < dim; ++d) pt[d] = xb[d] + t[kk] * m[d];
      // transverse interpolation cells and weights
      int te[2], nte = 0;
      int cs[2][3];
      double ws[2][3];
      int nw = order == 2 ? 3 : 2;
      for (int e = 0; e < dim; ++e) {
        if (e == ds) continue;
        const double q = (pt[e] - g.lo[e]) / h;
        if (order == 2) {
          const int cc = (int)std::floor(q);
          const double xi = q - (cc + 0.5);
          cs[nte][0] = cc - 1; ws[nte][0] = 0.5 * xi * (xi - 1.0);
          cs[nte][1] = cc;     ws[nte][1] = 1.0 - xi * xi;
          cs[nte][2] = cc + 1; ws[nte][2] = 0.5 * xi * (xi + 1.0);
        } else {
          const int cc = (int)std::floor(q - 0.5);
          const double th = q - (cc + 0.5);
          cs[nte][0] = cc;     ws[nte][0] = 1.0 - th;
          cs[nte][1] = cc + 1; ws[nte][1] = th;
        }
        te[nte++] = e;
      }
      Form& F = val[kk];
      F = Form();
      const int n2 = nte == 2 ? nw : 1;
      for (int a = 0; a < nw; ++a)
        for (int b = 0; b < n2; ++b) {
          int cell[3] = {c[0], c[1], c[2]};
          cell[ds] = plane;
          cell[te[0]] = cs[0][a];
          double w = ws[0][a];
          if (nte == 2) {
            cell[te[1]] = cs[1][b];
            w *= ws[1][b];
          }
          int64_t j = dof(cell, p);
          if (j < 0) return false;
          F.add(j, w);
        }
    }
    S = Form();
    if (order == 2) {
      const double w1 = t[1] / (t[0] * (t[1] - t[0]));
      const double w2 = -t[0] / (t[1] * (t[1] - t[0]));
      S.axpy(w1, val[0]);
      S.axpy(w2, val[1]);
      wB = -(w1 + w2);
    } else {
      S.axpy(1.0 / t[0], val[0]);
      wB = -1.0 / t[0];
    }
    return true;
  }

  // least squares over unknowns in front of the facet ((x_j - xb).m > 0),
  // radius 2 then 3; accepted with full rank and a negative boundary weight
  void lsq(const int* c, int p, const double* xb, const double* m, double& wB, Form& S) const {
    const int dim = g.dim;
    const double h = g.h;
    for (int R = 2; R <= 3; ++R) {
      std::vector<std::pair<int64_t, std::array<double, 4>>> rows;
      const int rz = dim == 3 ? R : 0;
      for (int oz = -rz; oz <= rz; ++oz)
        for (int oy = -R; oy <= R; ++oy)
          for (int ox = -R; ox <= R; ++ox) {
            const bool own = std::max(std::abs(ox), std::max(std::abs(oy), std::abs(oz))) < 1;
            int cell[3] = {c[0] + ox, c[1] + oy, c[2] + oz};
            int64_t j = dof(cell, p);
            if (j < 0) continue;
            std::array<double, 4> r4{};
            double n2 = 0, proj = 0;
            for (int d = 0; d < dim; ++d) {
              r4[d] = g.centre(d, cell[d]) - xb[d];
              n2 += r4[d] * r4[d];
              proj += r4[d] * m[d];
            }
            if (!own && proj > 1e-9 * h) {
              r4[3] = 1.0 / n2;
              rows.emplace_back(j, r4);
            }
            // centres of Dirichlet domain faces of this cell (known values),
            // keyed -1 - face
            for (int d = 0; d < dim; ++d)
              for (int side = 0; side < 2; ++side) {
                if (cell[d] != (side ? g.n[d] - 1 : 0)) continue;
                const int f = 2 * d + side;
                if (pb.bc.kind[f] != EBMG_BC_DIRICHLET) continue;
                std::array<double, 4> w4{};
                double wn2 = 0, wproj = 0;
                for (int e = 0; e < dim; ++e) {
                  w4[e] = g.centre(e, cell[e]) - xb[e];
                  if (e == d) w4[e] += side ? 0.5 * h : -0.5 * h;
                  wn2 += w4[e] * w4[e];
                  wproj += w4[e] * m[e];
                }
                if (wproj > 1e-9 * h) {
                  w4[3] = 1.0 / wn2;
                  rows.emplace_back(-1 - f, w4);
                }
              }
          }
      if ((int)rows.size() < dim) continue;
      double M[3][3] = {};
      for (auto& rw : rows)
        for (int a = 0; a < dim; ++a)
          for (int b = 0; b < dim; ++b) M[a][b] += rw.second[3] * rw.second[a] * rw.second[b];
      double det, tr = 0;
      double Mi[3][3];
      for (int a = 0; a < dim; ++a) tr += M[a][a];
      if (dim == 2) {
        det = M[0][0] * M[1][1] - M[0][1] * M[1][0];
        Mi[0][0] = M[1][1] / det; Mi[0][1] = -M[0][1] / det;
        Mi[1][0] = -M[1][0] / det; Mi[1][1] = M[0][0] / det;
      } else {
        double c00 = M[1][1] * M[2][2] - M[1][2] * M[2][1];
        double c01 = M[1][2] * M[2][0] - M[1][0] * M[2][2];
        double c02 = M[1][0] * M[2][1] - M[1][1] * M[2][0];
        det = M[0][0] * c00 + M[0][1] * c01 + M[0][2] * c02;
        Mi[0][0] = c00 / det;
        Mi[1][0] = c01 / det;
        Mi[2][0] = c02 / det;
        Mi[0][1] = (M[0][2] * M[2][1] - M[0][1] * M[2][2]) / det;
        Mi[1][1] = (M[0][0] * M[2][2] - M[0][2] * M[2][0]) / det;
        Mi[2][1] = (M[0][1] * M[2][0] - M[0][0] * M[2][1]) / det;
        Mi[0][2] = (M[0][1] * M[1][2] - M[0][2] * M[1][1]) / det;
        Mi[1][2] = (M[0][2] * M[1][0] - M[0][0] * M[1][2]) / det;
        Mi[2][2] = (M[0][0] * M[1][1] - M[0][1] * M[1][0]) / det;
      }
      if (det <= 1e-10 * std::pow(tr / dim, dim)) continue;
      Form T;
      double wsum = 0;
      for (auto& rw : rows) {
        double v = 0;
        for (int a = 0; a < dim; ++a) {
          double q = 0;
          for (int b = 0; b < dim; ++b) q += Mi[a][b] * rw.second[b];
          v += q * m[a];
        }
        const double cj = rw.second[3] * v;
        if (rw.first >= 0)
          T.add(rw.first, cj);
        else
          T.d.face[-1 - rw.first] += cj;
        wsum += cj;
      }
      if (wsum <= 0.0) continue;
      S = T;
      wB = -wsum;
      return;
    }
    throw GeomError("no least-squares stencil for an embedded-boundary cell");
  }

  // last resort for slivers against Dirichlet box faces: derivative toward the
  // face that m faces most, (m.n_w)(phi_wall - phiB)/d_w, d_w >= h/20
  void wall(const int* c, int p, const double* xb, const double* m, double& wB, Form& S) const {
    const double h = g.h;
    int bd = -1, bs = 0, bf = -1;
    double bmn = 0;
    for (int d = 0; d < g.dim; ++d)
      for (int side = 0; side < 2; ++side) {
        if (c[d] != (side ? g.n[d] - 1 : 0)) continue;
        const int f = 2 * d + side;
        if (pb.bc.kind[f] != EBMG_BC_DIRICHLET) continue;
        const double mn = side ? m[d] : -m[d];
        if (mn > 1e-12 && (bf < 0 || mn > bmn + 1e-12)) {
          bmn = mn;
          bd = d;
          bs = side;
          bf = f;
        }
      }
    (void)p;
    if (bf < 0) throw GeomError("no boundary stencil for an embedded-boundary cell");
    const double wallx = g.lo[bd] + (bs ? g.n[bd] : 0) * h;
    const double dw = std::max(std::fabs(wallx - xb[bd]), 0.05 * h);
    S = Form();
    S.d.face[bf] = bmn / dw;
    wB = -bmn / dw;
  }

  void dphi_dm(const int* c, int p, const double* xb, const double* m, int order, double& wB, Form& S) const {
    if (ray(c, p, xb, m, order, wB, S)) return;
    try {
      lsq(c, p, xb, m, wB, S);
    } catch (const GeomError&) {
      wall(c, p, xb, m, wB, S);
    }
  }

  // outward EB flux; returns the EB area fraction (0 if none)
  double eb_flux(const int* c, int p, Form& f) const {
    int64_t cell = g.cell(c[0], c[1], g.dim == 3 ? c[2] : 0);
    const CellCut* cc = geo.cut(p, cell);
    if (!cc || cc->eb_area <= 0.0) return 0.0;
    const double b = pb.bph[p];
    const int kind = geo.obj_kind[cc->cutter];
    f = Form();
    if (kind == EBMG_OBJ_WALL) {
      f.d.obj = cc->cutter;
      f.d.cobj = b;
      return cc->eb_area;
    }
    if (kind == EBMG_OBJ_ELECTRODE) {
      double m[3] = {-cc->eb_n[0], -cc->eb_n[1], -cc->eb_n[2]};
      double wB;
      Form S;
      dphi_dm(c, p, cc->eb_c, m, pb.opt.eb_order, wB, S);
      f.axpy(-b, S);
      f.d.obj = cc->cutter;
      f.d.cobj = -b * wB;
      return cc->eb_area;
    }
    if (geo.nphase < 2) throw GeomError("interface without a dielectric phase");
    double ng[3], mg[3], ms[3];
    for (int e = 0; e < 3; ++e) {
      ng[e] = p == 0 ? cc->eb_n[e] : -cc->eb_n[e];
      mg[e] = -ng[e];
      ms[e] = ng[e];
    }
    const double eg = pb.bph[0], es = pb.bph[1];
    double wg, ws;
    Form Sg, Ss;
    dphi_dm(c, 0, cc->eb_c, mg, 2, wg, Sg);
    dphi_dm(c, 1, cc->eb_c, ms, 2, ws, Ss);
    const double den = eg * wg + es * ws;
    Form phiB;
    phiB.d.csig = -1.0 / den;
    phiB.axpy(-eg / den, Sg);
    phiB.axpy(-es / den, Ss);
    Form dm;
    if (p == 0) {
      dm.axpy(wg, phiB);
      dm.axpy(1.0, Sg);
    } else {
      dm.axpy(ws, phiB);
      dm.axpy(1.0, Ss);
    }
    f.axpy(-pb.bph[p], dm);
    return cc->eb_area;
  }

  void row(const int* c, int p, double& mass, Form& flux) const {
    const double h = g.h, beta = pb.opt.beta;
    int64_t cell = g.cell(c[0], c[1], g.dim == 3 ? c[2] : 0);
    mass = geo.kappa(p, cell) * pb.opt.alpha * pb.aph[p];
    flux = Form();
    Form f;
    for (int d = 0; d < g.dim; ++d)
      for (int side = 0; side < 2; ++side) {
        double a = face_out(c, p, d, side, f);
        if (a > 0) flux.axpy(beta * a / h, f);
      }
    double a = eb_flux(c, p, f);
    if (a > 0) flux.axpy(beta * a / h, f);
  }

  // cell-centred E of unknown (c, p): E_d = sum_j coef phi_j + data
  void efield(const int* c, int p, Form* E) const {
    const double b = pb.bph[p];
    int64_t cell = g.cell(c[0], c[1], g.dim == 3 ? c[2] : 0);
    for (int d = 0; d < g.dim; ++d) {
      E[d] = Form();
      Form f;
      int cnt = 0;
      Form sum;
      for (int side = 0; side < 2; ++side) {
        double a = face_out(c, p, d, side, f);
        if (a <= 0) continue;
        sum.axpy((side ? 1.0 : -1.0) / b, f);
        ++cnt;
      }
      if (cnt) {
        E[d].axpy(-1.0 / cnt, sum);
      } else {
        double a = eb_flux(c, p, f);
        if (a > 0) {
          const CellCut* cc = geo.cut(p, cell);
          E[d].axpy(-(1.0 / b) * cc->eb_n[d], f);
        }
      }
    }
  }
};

}  // namespace

// --- finest level -----------------------------------------------------------

// Template constants of the finest level (off-diagonal, diagonal and the
// per-face boundary corrections for each phase) and the per-face data of the
// right-hand side and of E at domain faces: the parts of the fine operator
// that depend only on the coefficients and the boundary data.
void fine_template(Problem& pb) {
  Level& L = pb.levels[0];
  FineData& F = pb.fine;
  const Grid& g = L.g;
  const Options& o = pb.opt;
  const double h = g.h, beta = o.beta;
  for (int p = 0; p < 2; ++p) {
    const double b = pb.bph[p];
    L.coff[p] = beta * b / (h * h);
    L.mass[p] = o.alpha * pb.aph[p];
    L.d0[p] = L.mass[p] - 2.0 * g.dim * L.coff[p];
    for (int f = 0; f < 2 * g.dim; ++f) {
      const int kind = pb.bc.kind[f];
      double dme, dat, ga, gb;
      if (kind == EBMG_BC_NEUMANN) {
        dme = 0; dat = b; ga = 0; gb = 1;
      } else if (kind == EBMG_BC_DIRICHLET) {
        dme = -2.0 * b / h; dat = 2.0 * b / h; ga = -2.0 / h; gb = 2.0 / h;
      } else {
        const double a1 = pb.bc.robin_a1[f], a2 = pb.bc.robin_a2[f];
        const double cc = 1.0 / (1.0 + 0.5 * h * a1 / a2);
        dme = -(b * a1 / a2) * cc;
        dat = (b / a2) * (1.0 - a1 * cc * 0.5 * h / a2);
        ga = -a1 * cc / a2;
        gb = (1.0 - a1 * cc * 0.5 * h / a2) / a2;
      }
      L.cb[f][p] = (beta / h) * dme + L.coff[p];
      F.dat[f][p] = (beta / h) * dat;
      F.ega[f][p] = ga;
      F.egb[f][p] = gb;
    }
  }
}

void build_fine_level(Problem& pb) {
  const Geometry& geo = pb.geo;
  const Grid& g = geo.g;
  const Options& o = pb.opt;
  Builder B(pb);
  pb.levels.clear();
  pb.levels.emplace_back();
  Level& L = pb.levels[0];
  FineData& F = pb.fine;
  F = FineData();
  L.g = g;
  L.N = geo.N;
  L.N2 = geo.N2;
  L.primary = geo.primary;
  L.sec_of = geo.sec_of;
  L.sec_cell.assign(geo.sec_cell.begin(), geo.sec_cell.end());
  const double h = g.h, beta = o.beta;
  fine_template(pb);
  // regular mask
  const int64_t N = geo.N;
  L.tag.assign(N, TAG_IRR);
  const int nk = g.dim == 3 ? g.n[2] : 1;
  for (int k = 0; k < nk; ++k)
    for (int j = 0; j < g.n[1]; ++j)
      for (int i = 0; i < g.n[0]; ++i) {
        const int64_t cell = g.cell(i, j, k);
        const int p = geo.primary[cell];
        if (p < 0) {
          L.tag[cell] = TAG_COV;
          continue;
        }
        if (geo.ph[p].cls[cell] != 1) continue;
        bool ok = true;
        int c[3] = {i, j, k};
        for (int d = 0; d < g.dim && ok; ++d)
          for (int side = 0; side < 2 && ok; ++side) {
            int nb[3] = {i, j, k};
            nb[d] += side ? 1 : -1;
            if (nb[d] >= 0 && nb[d] < g.n[d]) {
              if (geo.primary[g.cell(nb[0], nb[1], nb[2])] != p) ok = false;
            } else {
              const int kind = pb.bc.kind[2 * d + side];
              if ((kind == EBMG_BC_DIRICHLET && o.dirichlet_closure == 1) ||
                  (kind == EBMG_BC_ROBIN && o.robin_closure == 1))
                ok = false;
            }
          }
        (void)c;
        if (ok) L.tag[cell] = (uint8_t)p;
      }
  // irregular rows: primary unknowns of irregular cells, then secondaries
  std::vector<std::pair<int64_t, int>> todo;
  for (int64_t c = 0; c < N; ++c)
    if (L.tag[c] == TAG_IRR) todo.emplace_back(c, geo.primary[c]);
  for (int64_t s = 0; s < geo.N2; ++s) todo.emplace_back(geo.sec_cell[s], 1);
  L.rp.assign(1, 0);
  for (auto& t : todo) {
    const int64_t cell = t.first;
    const int p = t.second;
    int c[3] = {(int)(cell % g.n[0]), (int)((cell / g.n[0]) % g.n[1]), (int)(cell / ((int64_t)g.n[0] * g.n[1]))};
    const int64_t me = geo.dof(c, p);
    double mass;
    Form fl;
    B.row(c, p, mass, fl);
    double dg = mass;
    for (auto& e : fl.c) {
      if (e.first == me)
        dg += e.second;
      else {
        L.col.push_back((int32_t)e.first);
        L.val.push_back(e.second);
      }
    }
    L.irow_dof.push_back(me);
    L.idiag.push_back(dg);
    L.imass.push_back(mass);
    L.rp.push_back((int64_t)L.col.size());
    F.idata.push_back(fl.d);
    F.isrc.push_back(p == geo.primary[cell] ? geo.kappa(p, cell) : 0.0);
  }
  // E rows of irregular primary cells
  F.erp.assign(1, 0);
  for (int64_t c = 0; c < N; ++c) {
    if (L.tag[c] != TAG_IRR) continue;
    const int p = geo.primary[c];
    int cc[3] = {(int)(c % g.n[0]), (int)((c / g.n[0]) % g.n[1]), (int)(c / ((int64_t)g.n[0] * g.n[1]))};
    Form E[3];
    B.efield(cc, p, E);
    F.ecell.push_back(c);
    for (int d = 0; d < 3; ++d) {
      if (d < g.dim)
        for (auto& e : E[d].c) {
          F.ecol.push_back((int32_t)e.first);
          F.eval.push_back(e.second);
        }
      F.erp.push_back((int64_t)F.ecol.size());
      F.edata.push_back(d < g.dim ? E[d].d : Data());
    }
  }
}

void host_rhs(const Problem& pb, const double* rho, const double* sigma, const double* bcv, const double* objv,
              double* b) {
  const Level& L = pb.levels[0];
  const Grid& g = L.g;
  const FineData& F = pb.fine;
  double bv[6], ov[64];
  for (int f = 0; f < 6; ++f) bv[f] = bcv ? bcv[f] : pb.bc.value[f];
  for (size_t k = 0; k < pb.geo.obj_value.size() && k < 64; ++k) ov[k] = objv ? objv[k] : pb.geo.obj_value[k];
  const int nk = g.dim == 3 ? g.n[2] : 1;
  for (int64_t q = 0; q < L.N + L.N2; ++q) b[q] = 0.0;
  for (int k = 0; k < nk; ++k)
    for (int j = 0; j < g.n[1]; ++j)
      for (int i = 0; i < g.n[0]; ++i) {
        const int64_t c = g.cell(i, j, k);
        const uint8_t t = L.tag[c];
        if (t > 1) continue;
        double v = rho[c];
        int ci[3] = {i, j, k};
        for (int d = 0; d < g.dim; ++d) {
          if (ci[d] == 0) v -= F.dat[2 * d][t] * bv[2 * d];
          if (ci[d] == g.n[d] - 1) v -= F.dat[2 * d + 1][t] * bv[2 * d + 1];
        }
        b[c] = v;
      }
  for (size_t r = 0; r < L.irow_dof.size(); ++r) {
    const int64_t q = L.irow_dof[r];
    const int64_t cell = q < L.N ? q : L.sec_cell[q - L.N];
    const Data& D = F.idata[r];
    double v = F.isrc[r] * rho[cell];
    for (int f = 0; f < 6; ++f) v -= D.face[f] * bv[f];
    if (D.obj >= 0) v -= D.cobj * ov[D.obj];
    if (sigma) v -= D.csig * sigma[cell];
    b[q] = v;
  }
}

}  // namespace ebmg
