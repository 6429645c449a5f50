// Host preparation of the composite operator of a nested AMR hierarchy
// (Numerical methods: patch-based refinement; Helmholtz equations: the
// refluxing of coarse-fine faces). The hierarchy is a tree of boxes,
// refinement ratio 2, level 0 the whole domain, every other box inside one
// box of the next coarser level (its parent); a patch's faces inside the
// domain are coarse-fine faces, set up as homogeneous Dirichlet faces
// (linear closure) of the patch's own problem. Per parent-child pair this
// builds the sparse corrections that turn the boxes' own operators into the
// composite one:
//  * fine rows next to a coarse-fine face gain (beta b / h_f^2)(phi_G + phi_F)
//    with the ghost phi_G = 8/15 phi_C + 2/3 phi_F - 1/5 phi_Fn (quadratic
//    along the normal through the coarse value at -1 fine cell and the two
//    fine cells inside, taken at -1/2), phi_C the coarse level's quadratic
//    Taylor interpolant about the coarse cell holding the ghost at the
//    ghost's tangential offsets (+-1/4 coarse cell): first and second
//    differences per tangential axis, centred where both neighbours are
//    valid regular gas cells, else one-sided on the side where two are, and
//    in 3D the mixed difference, centred or one-sided in the first sign
//    pair (+,+), (+,-), (-,+), (-,-) that is available;
//  * coarse rows next to the finer box: the face flux into a covered cell,
//    b (phi_Cv - phi_C) / h_c, is replaced by the mean over the 2^(D-1) fine
//    faces on it of b (phi_F - phi_G) / h_f (refluxing);
//  * the covered coarse unknowns (identity rows of the composite system),
//    the restriction of fine residuals onto them (mean of the children's
//    unknowns of the same phase) and the piecewise-constant prolongation of
//    coarse corrections onto the fine unknowns, for the preconditioner.
// Every cell the ghosts and the reflux use must be a regular gas cell that
// no finer box covers; anything else is rejected (GeomError).

#include <cmath>
#include <map>

#include "internal.hpp"

namespace ebmg {

namespace {

struct Lev {
  const Problem& P;
  const AmrBox& box;
  const std::vector<const AmrBox*>& kids;   // the boxes refining this one
  int dim() const { return P.geo.g.dim; }
};

bool in_box(const AmrBox& b, int dim, const int* g) {
  for (int d = 0; d < dim; ++d)
    if (g[d] < b.lo[d] || g[d] >= b.lo[d] + b.n[d]) return false;
  return true;
}

// coarse global cell gc under the box fb of the next finer level
bool under(const AmrBox& fb, int dim, const int* gc) {
  for (int d = 0; d < dim; ++d)
    if (2 * gc[d] < fb.lo[d] || 2 * gc[d] + 1 >= fb.lo[d] + fb.n[d]) return false;
  return true;
}

int64_t local_cell(const Lev& L, const int* g) {
  int c[3] = {0, 0, 0};
  for (int d = 0; d < L.dim(); ++d) c[d] = g[d] - L.box.lo[d];
  return L.P.geo.g.cell(c[0], c[1], c[2]);
}

int64_t slot(const Lev& L, const int* g, int p) {
  int c[3] = {0, 0, 0};
  for (int d = 0; d < L.dim(); ++d) c[d] = g[d] - L.box.lo[d];
  return L.P.geo.dof(c, p);
}

bool regular_gas(const Lev& L, const int* g) {
  const int D = L.dim();
  if (!in_box(L.box, D, g)) return false;
  for (const AmrBox* k : L.kids)
    if (under(*k, D, g)) return false;
  const Geometry& G = L.P.geo;
  const int64_t c = local_cell(L, g);
  if (G.primary[c] != 0 || G.sec_of[c] >= 0) return false;
  return std::fabs(G.kappa(0, c) - 1.0) < 1e-14;
}

using Stencil = std::map<std::vector<int>, double>;

void add(Stencil& w, const Stencil& s, double f) {
  for (const auto& e : s) w[e.first] += f * e.second;
}

std::vector<int> shifted(const std::vector<int>& c, int e, int k) {
  std::vector<int> o = c;
  o[e] += k;
  return o;
}

// the coarse interpolant about C at ghost G's tangential position (normal d)
Stencil coarse_interp(const Lev& Cl, const std::vector<int>& C, const std::vector<int>& G, int d) {
  const int D = Cl.dim();
  auto ok = [&](const std::vector<int>& c) { return regular_gas(Cl, c.data()); };
  if (!ok(C)) throw GeomError("a coarse-fine ghost's coarse cell is not a regular gas cell of the coarser level");
  Stencil w;
  w[C] = 1.0;
  int tang[2], nt = 0;
  for (int e = 0; e < D; ++e)
    if (e != d) tang[nt++] = e;
  double delta[3] = {0, 0, 0};
  for (int q = 0; q < nt; ++q) {
    const int e = tang[q];
    delta[e] = (G[e] + 0.5) / 2.0 - (C[e] + 0.5);
    const auto p1 = shifted(C, e, 1), m1 = shifted(C, e, -1), p2 = shifted(C, e, 2), m2 = shifted(C, e, -2);
    Stencil d1, d2;
    if (ok(p1) && ok(m1)) {
      d1 = {{p1, 0.5}, {m1, -0.5}};
      d2 = {{p1, 1.0}, {C, -2.0}, {m1, 1.0}};
    } else if (ok(p1) && ok(p2)) {
      d1 = {{C, -1.5}, {p1, 2.0}, {p2, -0.5}};
      d2 = {{C, 1.0}, {p1, -2.0}, {p2, 1.0}};
    } else if (ok(m1) && ok(m2)) {
      d1 = {{C, 1.5}, {m1, -2.0}, {m2, 0.5}};
      d2 = {{C, 1.0}, {m1, -2.0}, {m2, 1.0}};
    } else {
      throw GeomError("no tangential stencil for a coarse-fine ghost");
    }
    add(w, d1, delta[e]);
    add(w, d2, 0.5 * delta[e] * delta[e]);
  }
  if (D == 3) {
    const int e1 = tang[0], e2 = tang[1];
    auto corner = [&](int s1, int s2) { return shifted(shifted(C, e1, s1), e2, s2); };
    Stencil d12;
    if (ok(corner(1, 1)) && ok(corner(1, -1)) && ok(corner(-1, 1)) && ok(corner(-1, -1))) {
      d12 = {{corner(1, 1), 0.25}, {corner(1, -1), -0.25}, {corner(-1, 1), -0.25}, {corner(-1, -1), 0.25}};
    } else {
      const int sg[4][2] = {{1, 1}, {1, -1}, {-1, 1}, {-1, -1}};
      bool found = false;
      for (const auto& s : sg) {
        const auto a = shifted(C, e1, s[0]), b = shifted(C, e2, s[1]), c = corner(s[0], s[1]);
        if (ok(a) && ok(b) && ok(c)) {
          const double ss = s[0] * s[1];
          d12[c] += ss;
          d12[a] -= ss;
          d12[b] -= ss;
          d12[C] += ss;
          found = true;
          break;
        }
      }
      if (!found) throw GeomError("no mixed stencil for a coarse-fine ghost");
    }
    add(w, d12, delta[e1] * delta[e2]);
  }
  return w;
}

// ghost of fine cell F across face (d, side): coarse slots and fine slots
void ghost(const Lev& Cl, const Lev& Fl, const std::vector<int>& F, int d, int side,
           std::map<int64_t, double>& wc, std::map<int64_t, double>& wf) {
  const int D = Fl.dim();
  const int sg = side ? 1 : -1;
  const auto G = shifted(F, d, sg), Fn = shifted(F, d, -sg);
  if (!regular_gas(Fl, F.data()) || !regular_gas(Fl, Fn.data()))
    throw GeomError("a fine cell next to a coarse-fine face is not a regular gas cell");
  std::vector<int> C(D);
  for (int q = 0; q < D; ++q) C[q] = (int)std::floor(G[q] / 2.0);
  wc.clear();
  wf.clear();
  for (const auto& e : coarse_interp(Cl, C, G, d)) wc[slot(Cl, e.first.data(), 0)] += (8.0 / 15.0) * e.second;
  wf[slot(Fl, F.data(), 0)] += 2.0 / 3.0;
  wf[slot(Fl, Fn.data(), 0)] += -1.0 / 5.0;
}

void flush_row(int64_t row, const std::map<int64_t, double>& m, std::vector<int64_t>& rows,
               std::vector<int64_t>& ptr, std::vector<int64_t>& col, std::vector<double>& w) {
  rows.push_back(row);
  for (const auto& e : m) {
    col.push_back(e.first);
    w.push_back(e.second);
  }
  ptr.push_back((int64_t)col.size());
}

}  // namespace

void build_amr_link(const Problem& C, const AmrBox& cb, const std::vector<const AmrBox*>& ckids, const Problem& F,
                    const AmrBox& fb, const std::vector<const AmrBox*>& fkids, AmrLink& out) {
  const int D = C.geo.g.dim;
  const Lev Cl{C, cb, ckids};
  const Lev Fl{F, fb, fkids};
  out = AmrLink();
  // proper nesting: the box lies inside the coarser one on coarse cells
  for (int d = 0; d < D; ++d) {
    if (fb.lo[d] % 2 || fb.n[d] % 2 || fb.n[d] < 4) throw ArgError("AMR boxes need even corners and sizes >= 4");
    if (fb.lo[d] < 2 * cb.lo[d] || fb.lo[d] + fb.n[d] > 2 * (cb.lo[d] + cb.n[d]))
      throw ArgError("an AMR box must lie inside the next coarser box");
  }
  const double hf = F.geo.g.h, hc = C.geo.g.h;
  const double kf = F.opt.beta * F.bph[0] / (hf * hf);
  const double kc = C.opt.beta * C.bph[0] / (hc * hc);
  const double kr = C.opt.beta * C.bph[0] / (hc * hf * (D == 3 ? 4.0 : 2.0));
  std::map<int64_t, double> wc, wf;
  // fine rows: cells of the box with a coarse-fine face
  const int nz = D == 3 ? fb.n[2] : 1;
  for (int k = 0; k < nz; ++k)
    for (int j = 0; j < fb.n[1]; ++j)
      for (int i = 0; i < fb.n[0]; ++i) {
        const int loc[3] = {i, j, k};
        bool edge = false;
        for (int d = 0; d < D; ++d)
          edge |= (loc[d] == 0 && fb.cf[2 * d]) || (loc[d] == fb.n[d] - 1 && fb.cf[2 * d + 1]);
        if (!edge) continue;
        std::vector<int> Fg(D);
        for (int d = 0; d < D; ++d) Fg[d] = fb.lo[d] + loc[d];
        std::map<int64_t, double> row;   // >= 0: fine slot; < 0: -(coarse slot) - 1
        for (int d = 0; d < D; ++d)
          for (int side = 0; side < 2; ++side) {
            const bool at = side ? loc[d] == fb.n[d] - 1 : loc[d] == 0;
            if (!at || !fb.cf[2 * d + side]) continue;
            ghost(Cl, Fl, Fg, d, side, wc, wf);
            for (const auto& e : wc) row[-e.first - 1] += kf * e.second;
            for (const auto& e : wf) row[e.first] += kf * e.second;
            row[slot(Fl, Fg.data(), 0)] += kf;
          }
        flush_row(slot(Fl, Fg.data(), 0), row, out.frow, out.fptr, out.fcol, out.fw);
      }
  // coarse rows: valid cells of the coarse box sharing a face with the box
  const int cz = D == 3 ? cb.n[2] : 1;
  for (int k = 0; k < cz; ++k)
    for (int j = 0; j < cb.n[1]; ++j)
      for (int i = 0; i < cb.n[0]; ++i) {
        std::vector<int> Cg = {cb.lo[0] + i, cb.lo[1] + j};
        if (D == 3) Cg.push_back(cb.lo[2] + k);
        if (under(fb, D, Cg.data())) continue;
        std::map<int64_t, double> row;   // >= 0: coarse slot; < 0: -(fine slot) - 1
        bool any = false;
        for (int d = 0; d < D; ++d)
          for (int sg = 1; sg >= -1; sg -= 2) {
            const auto Cv = shifted(Cg, d, sg);
            if (!in_box(cb, D, Cv.data()) || !under(fb, D, Cv.data())) continue;
            if (!regular_gas(Cl, Cg.data()))
              throw GeomError("a coarse cell next to a finer box is not a regular gas cell");
            any = true;
            const int64_t me = slot(Cl, Cg.data(), 0);
            // the covered neighbour's gas unknown (its face with a regular
            // gas cell is a full gas face)
            const int64_t cv = slot(Cl, Cv.data(), 0);
            if (cv < 0) throw GeomError("a coarse cell next to a finer box faces a cell without gas");
            row[cv] += -kc;
            row[me] += kc;
            int tang[2], nt = 0;
            for (int e = 0; e < D; ++e)
              if (e != d) tang[nt++] = e;
            for (int o = 0; o < (1 << (D - 1)); ++o) {
              std::vector<int> Fc(D);
              Fc[d] = 2 * Cv[d] + (sg > 0 ? 0 : 1);
              for (int q = 0; q < nt; ++q) Fc[tang[q]] = 2 * Cv[tang[q]] + ((o >> q) & 1);
              ghost(Cl, Fl, Fc, d, sg > 0 ? 0 : 1, wc, wf);
              row[-slot(Fl, Fc.data(), 0) - 1] += kr;
              for (const auto& e : wc) row[e.first] += -kr * e.second;
              for (const auto& e : wf) row[-e.first - 1] += -kr * e.second;
            }
          }
        if (any) flush_row(slot(Cl, Cg.data(), 0), row, out.crow, out.cptr, out.ccol, out.cw);
      }
  // covered coarse slots, and the restriction of fine unknowns onto them
  const Geometry& Gc = C.geo;
  const Geometry& Gf = F.geo;
  const double rw = 1.0 / (D == 3 ? 8.0 : 4.0);
  for (int k = 0; k < cz; ++k)
    for (int j = 0; j < cb.n[1]; ++j)
      for (int i = 0; i < cb.n[0]; ++i) {
        int Cg[3] = {cb.lo[0] + i, cb.lo[1] + j, D == 3 ? cb.lo[2] + k : 0};
        if (!under(fb, D, Cg)) continue;
        const int64_t cell = Gc.g.cell(i, j, k);
        out.cov.push_back(cell);
        if (Gc.sec_of[cell] >= 0) out.cov.push_back(Gc.N + Gc.sec_of[cell]);
        for (int p = 0; p < 2; ++p) {
          const int cl[3] = {i, j, k};
          const int64_t cs = Gc.dof(cl, p);
          if (cs < 0) continue;
          std::map<int64_t, double> row;
          for (int o = 0; o < (1 << D); ++o) {
            int fc[3] = {0, 0, 0};
            for (int d = 0; d < D; ++d) fc[d] = 2 * Cg[d] + ((o >> d) & 1) - fb.lo[d];
            const int64_t fs = Gf.dof(fc, p);
            if (fs >= 0) row[fs] += rw;
          }
          const double cnt = (double)row.size();
          flush_row(cs, row, out.rrow, out.rptr, out.rcol, out.rw);
          for (size_t e = 0; e < row.size(); ++e) out.aw.push_back(1.0 / cnt);
        }
      }
  // prolongation: each fine slot from its parent's unknown of the same phase
  // (else the parent's primary unknown)
  out.pcol.assign(Gf.N + Gf.N2, -1);
  for (int k = 0; k < nz; ++k)
    for (int j = 0; j < fb.n[1]; ++j)
      for (int i = 0; i < fb.n[0]; ++i) {
        const int64_t cell = Gf.g.cell(i, j, k);
        const int loc[3] = {i, j, k};
        int pc[3] = {0, 0, 0};
        for (int d = 0; d < D; ++d) pc[d] = (fb.lo[d] + loc[d]) / 2 - cb.lo[d];
        const int64_t pcell = Gc.g.cell(pc[0], pc[1], pc[2]);
        auto parent = [&](int p) -> int64_t {
          int64_t s = Gc.dof(pc, p);
          if (s < 0 && Gc.primary[pcell] >= 0) s = Gc.dof(pc, Gc.primary[pcell]);
          return s;
        };
        if (Gf.primary[cell] >= 0) out.pcol[cell] = parent(Gf.primary[cell]);
        if (Gf.sec_of[cell] >= 0) out.pcol[Gf.N + Gf.sec_of[cell]] = parent(1);
      }
}

}  // namespace ebmg
