// Multigrid hierarchy: coarse levels, transfer lists, colouring, bottom inverse.
//
// The paper's solver is the residual-correction geometric multigrid of its
// multigrid-solver subsection; the coarse operators are not specified there
// (EBChombo coarsens the EB graph). Here each coarse cell aggregates 2^D fine
// cells and carries one unknown per phase present among its children. Rows of
// coarse cells whose children are all regular cells of one phase (and whose
// neighbours share that primary phase) are the rediscretised (2D+1)-point
// template at spacing 2h; every other coarse row is the Galerkin product of the
// fine rows with piecewise-constant prolongation, its flux part scaled by
// 2^-(D+1) and its mass part by 2^-D, which equals the rediscretised template
// wherever both apply. Restriction averages the 2^D children (covered children
// count as zero residual), prolongation injects. Only the convergence rate
// depends on these choices; the fixed point is the finest-level system.
#include <algorithm>
#include <cmath>
#include <unordered_map>

#include "internal.hpp"

namespace ebmg {

namespace {

inline void cell_ijk(const Grid& g, int64_t c, int* ijk) {
  ijk[0] = (int)(c % g.n[0]);
  ijk[1] = (int)((c / g.n[0]) % g.n[1]);
  ijk[2] = (int)(c / ((int64_t)g.n[0] * g.n[1]));
}

std::vector<int32_t> irow_index(const Level& L) {
  std::vector<int32_t> m(L.N + L.N2, -1);
  for (size_t r = 0; r < L.irow_dof.size(); ++r) m[L.irow_dof[r]] = (int32_t)r;
  return m;
}

}  // namespace

// Rediscretised template constants of a coarse level at its own spacing.
void coarse_template(Level& C, const Problem& pb) {
  const double h = C.g.h, beta = pb.opt.beta;
  for (int p = 0; p < 2; ++p) {
    const double b = pb.bph[p];
    C.coff[p] = beta * b / (h * h);
    C.mass[p] = pb.opt.alpha * pb.aph[p];
    C.d0[p] = C.mass[p] - 2.0 * C.g.dim * C.coff[p];
    for (int f = 0; f < 2 * C.g.dim; ++f) {
      const int kind = pb.bc.kind[f];
      double dme;
      if (kind == EBMG_BC_NEUMANN)
        dme = 0;
      else if (kind == EBMG_BC_DIRICHLET)
        dme = -2.0 * b / h;
      else {
        const double a1 = pb.bc.robin_a1[f], a2 = pb.bc.robin_a2[f];
        dme = -(b * a1 / a2) / (1.0 + 0.5 * h * a1 / a2);
      }
      C.cb[f][p] = (beta / h) * dme + C.coff[p];
    }
  }
}


void Level::row(int64_t q, double& mass_out, std::vector<std::pair<int64_t, double>>& out) const {
  out.clear();
  mass_out = 0;
  int64_t cell = q < N ? q : sec_cell[q - N];
  uint8_t t = tag[cell] & 3;
  if (q < N && t <= 1) {
    int c[3];
    cell_ijk(g, cell, c);
    double dg = d0[t];
    for (int d = 0; d < g.dim; ++d)
      for (int side = 0; side < 2; ++side) {
        int nb[3] = {c[0], c[1], c[2]};
        nb[d] += side ? 1 : -1;
        if (nb[d] >= 0 && nb[d] < g.n[d])
          out.emplace_back(g.cell(nb[0], nb[1], nb[2]), coff[t]);
        else
          dg += cb[2 * d + side][t];
      }
    mass_out = mass[t];
    out.emplace_back(q, dg - mass[t]);
    return;
  }
  if (t == TAG_COV && q < N) return;
  // irregular: linear search is avoided by the caller's index when available
  auto it = std::lower_bound(irow_dof.begin(), irow_dof.end(), q);
  if (it == irow_dof.end() || *it != q) throw std::logic_error("missing irregular row");
  size_t r = it - irow_dof.begin();
  mass_out = imass[r];
  out.emplace_back(q, idiag[r] - imass[r]);
  for (int64_t e = rp[r]; e < rp[r + 1]; ++e) out.emplace_back(col[e], val[e]);
}

// Explicit rows grouped by the red/black colour of their cell (group 0: red,
// i+j+k even), in row order within a group.
void colour_irregular(Level& L) {
  const size_t R = L.irow_dof.size();
  L.cls_ptr.assign(3, 0);
  L.cls_rows.clear();
  L.cls_rows.reserve(R);
  for (int grp = 0; grp < 2; ++grp) {
    for (size_t r = 0; r < R; ++r) {
      const int64_t q = L.irow_dof[r];
      const int64_t cell = q < L.N ? q : L.sec_cell[q - L.N];
      int ijk[3];
      cell_ijk(L.g, cell, ijk);
      if (((ijk[0] + ijk[1] + ijk[2]) & 1) == grp) L.cls_rows.push_back((int32_t)r);
    }
    L.cls_ptr[grp + 1] = (int32_t)L.cls_rows.size();
  }
}

static bool coarsen(Problem& pb, size_t lf) {
  Level& L = pb.levels[lf];
  const Grid& gf = L.g;
  for (int d = 0; d < gf.dim; ++d)
    if (gf.n[d] % 2 || gf.n[d] < 4) return false;
  Level C;
  C.g = gf;
  for (int d = 0; d < gf.dim; ++d) C.g.n[d] = gf.n[d] / 2;
  C.g.h = 2 * gf.h;
  const Grid& gc = C.g;
  const int D = gf.dim;
  const int nch = 1 << D;
  C.N = gc.ncell();
  std::vector<uint8_t> has(C.N, 0);
  auto parent = [&](int64_t c) {
    int ijk[3];
    cell_ijk(gf, c, ijk);
    return gc.cell(ijk[0] / 2, ijk[1] / 2, D == 3 ? ijk[2] / 2 : 0);
  };
  auto child = [&](int64_t P, int q) {
    int ijk[3];
    cell_ijk(gc, P, ijk);
    return gf.cell(2 * ijk[0] + (q & 1), 2 * ijk[1] + ((q >> 1) & 1), D == 3 ? 2 * ijk[2] + ((q >> 2) & 1) : 0);
  };
  for (int64_t c = 0; c < L.N; ++c) {
    int64_t P = parent(c);
    if (L.primary[c] == 0) has[P] |= 1;
    if (L.primary[c] == 1) has[P] |= 2;
    if (L.sec_of[c] >= 0) has[P] |= 2;
  }
  C.primary.assign(C.N, -1);
  C.sec_of.assign(C.N, -1);
  for (int64_t P = 0; P < C.N; ++P) {
    C.primary[P] = (has[P] & 1) ? 0 : ((has[P] & 2) ? 1 : -1);
    if (has[P] == 3) {
      C.sec_of[P] = (int32_t)C.sec_cell.size();
      C.sec_cell.push_back((int32_t)P);
    }
  }
  C.N2 = (int64_t)C.sec_cell.size();
  auto cdof = [&](int64_t P, int p) -> int64_t {
    if (C.primary[P] == p) return P;
    return C.N + C.sec_of[P];
  };
  auto fine_phase = [&](int64_t q) -> int { return q < L.N ? L.primary[q] : 1; };
  auto fine_cell = [&](int64_t q) -> int64_t { return q < L.N ? q : L.sec_cell[q - L.N]; };
  auto agg = [&](int64_t q) { return cdof(parent(fine_cell(q)), fine_phase(q)); };
  // tags
  C.tag.assign(C.N, TAG_IRR);
  std::vector<uint8_t> simple(C.N, 1);
  for (int64_t P = 0; P < C.N; ++P) {
    int pc = C.primary[P];
    if (pc < 0) {
      C.tag[P] = TAG_COV;
      continue;
    }
    bool allreg = true;
    for (int q = 0; q < nch; ++q) {
      int64_t c = child(P, q);
      if (L.sec_of[c] >= 0 || (L.primary[c] >= 0 && L.primary[c] != pc)) simple[P] = 0;
      if ((L.tag[c] & 3) != pc) allreg = false;
    }
    if (allreg) {
      int ijk[3];
      cell_ijk(gc, P, ijk);
      for (int d = 0; d < D && allreg; ++d)
        for (int side = 0; side < 2; ++side) {
          int nb[3] = {ijk[0], ijk[1], ijk[2]};
          nb[d] += side ? 1 : -1;
          if (nb[d] >= 0 && nb[d] < gc.n[d] && C.primary[gc.cell(nb[0], nb[1], nb[2])] != pc) allreg = false;
        }
    }
    C.tag[P] = allreg ? (uint8_t)pc : (uint8_t)TAG_IRR;
    if (!simple[P]) C.tag[P] |= TAG_NONSIMPLE;
  }
  coarse_template(C, pb);
  // children of each coarse unknown
  std::vector<int64_t> kids;
  std::vector<std::pair<int64_t, double>> rowbuf;
  std::unordered_map<int64_t, double> acc;
  const double sflux = 1.0 / (double)(2 * nch), smass = 1.0 / (double)nch;
  // irregular coarse rows: primaries of irregular cells (cell order), then secondaries
  std::vector<int64_t> todo;
  for (int64_t P = 0; P < C.N; ++P)
    if ((C.tag[P] & 3) == TAG_IRR) todo.push_back(P);
  for (int64_t s = 0; s < C.N2; ++s) todo.push_back(C.N + s);
  C.rp.assign(1, 0);
  for (int64_t J : todo) {
    const int64_t P = J < C.N ? J : C.sec_cell[J - C.N];
    const int pj = J < C.N ? C.primary[P] : 1;
    acc.clear();
    double mass = 0;
    for (int q = 0; q < nch; ++q) {
      int64_t c = child(P, q);
      int64_t fd[2];
      int nf = 0;
      if (L.primary[c] == pj) fd[nf++] = c;
      if (pj == 1 && L.sec_of[c] >= 0) fd[nf++] = L.N + L.sec_of[c];
      for (int t = 0; t < nf; ++t) {
        double m;
        L.row(fd[t], m, rowbuf);
        mass += smass * m;
        for (auto& e : rowbuf) acc[agg(e.first)] += sflux * e.second;
      }
    }
    double dg = mass;
    std::vector<std::pair<int64_t, double>> ent;
    for (auto& kv : acc) {
      if (kv.first == J)
        dg += kv.second;
      else
        ent.emplace_back(kv.first, kv.second);
    }
    std::sort(ent.begin(), ent.end());
    for (auto& e : ent) {
      C.col.push_back((int32_t)e.first);
      C.val.push_back(e.second);
    }
    C.irow_dof.push_back(J);
    C.idiag.push_back(dg);
    C.imass.push_back(mass);
    C.rp.push_back((int64_t)C.col.size());
  }
  // transfer lists for non-simple coarse cells
  L.ns_cdof.clear();
  L.ns_ptr.assign(1, 0);
  L.ns_child.clear();
  L.np_fdof.clear();
  L.np_cdof.clear();
  for (int64_t P = 0; P < C.N; ++P) {
    if (simple[P] || C.primary[P] < 0) continue;
    for (int ph = 0; ph < 2; ++ph) {
      if (!((has[P] >> ph) & 1)) continue;
      const int64_t J = cdof(P, ph);
      L.ns_cdof.push_back(J);
      for (int q = 0; q < nch; ++q) {
        int64_t c = child(P, q);
        if (L.primary[c] == ph) L.ns_child.push_back(c);
        if (ph == 1 && L.sec_of[c] >= 0) L.ns_child.push_back(L.N + L.sec_of[c]);
      }
      L.ns_ptr.push_back((int32_t)L.ns_child.size());
    }
  }
  for (int64_t q = 0; q < L.N + L.N2; ++q) {
    int64_t c = fine_cell(q);
    if (q < L.N && L.primary[c] < 0) continue;
    int64_t P = parent(c);
    if (simple[P]) continue;
    L.np_fdof.push_back(q);
    L.np_cdof.push_back(agg(q));
  }
  colour_irregular(C);
  pb.levels.push_back(std::move(C));
  return true;
}

static void dense_inverse(std::vector<double>& A, int64_t n) {
  std::vector<double> I(n * n, 0.0);
  for (int64_t i = 0; i < n; ++i) I[i * n + i] = 1.0;
  for (int64_t c = 0; c < n; ++c) {
    int64_t piv = c;
    double best = std::fabs(A[c * n + c]);
    for (int64_t r = c + 1; r < n; ++r)
      if (std::fabs(A[r * n + c]) > best) {
        best = std::fabs(A[r * n + c]);
        piv = r;
      }
    if (best == 0.0) throw GeomError("singular bottom-level operator");
    if (piv != c)
      for (int64_t k = 0; k < n; ++k) {
        std::swap(A[c * n + k], A[piv * n + k]);
        std::swap(I[c * n + k], I[piv * n + k]);
      }
    const double inv = 1.0 / A[c * n + c];
    for (int64_t k = 0; k < n; ++k) {
      A[c * n + k] *= inv;
      I[c * n + k] *= inv;
    }
    for (int64_t r = 0; r < n; ++r) {
      if (r == c) continue;
      const double f = A[r * n + c];
      if (f == 0.0) continue;
      for (int64_t k = 0; k < n; ++k) {
        A[r * n + k] -= f * A[c * n + k];
        I[r * n + k] -= f * I[c * n + k];
      }
    }
  }
  A.swap(I);
}

void build_hierarchy(Problem& pb) {
  colour_irregular(pb.levels[0]);
  while (pb.levels.size() < 16 && pb.levels.back().ndof() > pb.opt.bottom_max) {
    if (!coarsen(pb, pb.levels.size() - 1)) break;
  }
  build_bottom(pb);
}

// Dense FP64 inverse of the coarsest level (left empty above 4096 unknowns,
// where the bottom is relaxed instead).
void build_bottom(Problem& pb) {
  const Level& B = pb.levels.back();
  const int64_t n = B.ndof();
  pb.bottom_n = n;
  pb.bottom_inv.clear();
  if (n > 4096) return;  // bottom solved by relaxation sweeps instead
  std::vector<double> A(n * n, 0.0);
  std::vector<std::pair<int64_t, double>> rowbuf;
  for (int64_t q = 0; q < n; ++q) {
    int64_t cell = q < B.N ? q : B.sec_cell[q - B.N];
    if (q < B.N && B.primary[cell] < 0) {
      A[q * n + q] = 1.0;
      continue;
    }
    double m;
    B.row(q, m, rowbuf);
    A[q * n + q] += m;
    for (auto& e : rowbuf) A[q * n + e.first] += e.second;
  }
  dense_inverse(A, n);
  pb.bottom_inv.swap(A);
}

}  // namespace ebmg
