// Internal data structures of the ebmg library (host side).
#pragma once

#include <cstdint>
#include <stdexcept>
#include <string>
#include <unordered_map>
#include <utility>
#include <vector>

#include "../../include/ebmg.h"

namespace ebmg {

struct GeomError : std::runtime_error {
  using std::runtime_error::runtime_error;
};
struct ArgError : std::runtime_error {
  using std::runtime_error::runtime_error;
};

constexpr double kTiny = 1e-12;

// Uniform box of cells; 2D boxes use n[2] = 1 and k = 0.
struct Grid {
  int dim = 2;
  int n[3] = {1, 1, 1};
  double h = 1.0;
  double lo[3] = {0, 0, 0};
  int64_t ncell() const { return (int64_t)n[0] * n[1] * n[2]; }
  int64_t cell(int i, int j, int k) const { return i + (int64_t)n[0] * (j + (int64_t)n[1] * k); }
  int64_t node(int i, int j, int k) const {
    return i + (int64_t)(n[0] + 1) * (j + (int64_t)(n[1] + 1) * k);
  }
  int64_t nnode() const { return (int64_t)(n[0] + 1) * (n[1] + 1) * (dim == 3 ? n[2] + 1 : 1); }
  // face normal to d at node-plane index along d
  int64_t face(int d, int i, int j, int k) const {
    int64_t m0 = n[0] + (d == 0), m1 = n[1] + (d == 1);
    return i + m0 * (j + m1 * k);
  }
  bool inbox(const int* c) const {
    for (int d = 0; d < dim; ++d)
      if (c[d] < 0 || c[d] >= n[d]) return false;
    return true;
  }
  double centre(int d, int c) const { return lo[d] + (c + 0.5) * h; }
};

struct FaceCut {
  double alpha;
  double off[2];
};

struct CellCut {
  double kappa;
  double vc[3];
  double eb_area;
  double eb_c[3];
  double eb_n[3];
  int cutter;
};

// One phase: node level set, per-cell class, and the cut faces and cells.
struct Phase {
  std::vector<double> s;
  std::vector<uint8_t> cls;  // 0 covered, 1 full, 2 cut
  std::unordered_map<int64_t, FaceCut> fcut[3];
  std::unordered_map<int64_t, CellCut> ccut;
};

struct Geometry {
  Grid g;
  int nphase = 1;
  int diel_obj = -1;
  std::vector<int> obj_kind;
  std::vector<double> obj_value;
  Phase ph[2];
  std::vector<int8_t> primary;    // per cell: 0, 1, -1
  std::vector<int32_t> sec_of;    // per cell: secondary index or -1
  std::vector<int64_t> sec_cell;  // secondary -> cell
  int64_t N = 0, N2 = 0;

  // aperture of face (d, node-plane c) for phase p; c is a cell-like index
  // with c[d] the node plane
  double alpha(int p, int d, const int* c) const;
  void face_off(int p, int d, const int* c, double* off) const;
  double kappa(int p, int64_t cell) const;
  const CellCut* cut(int p, int64_t cell) const {
    auto it = ph[p].ccut.find(cell);
    return it == ph[p].ccut.end() ? nullptr : &it->second;
  }
  bool has(int p, int64_t cell) const { return p < nphase && ph[p].cls[cell] != 0; }
  // unknown index of phase p in cell c (-1 if none / outside)
  int64_t dof(const int* c, int p) const;
};

void build_geometry(Geometry& geo, const ebmg_box& box, int nobj, const ebmg_object* objs);

// ---------------------------------------------------------------------------
// linear forms
// ---------------------------------------------------------------------------
struct Data {
  double face[6] = {0, 0, 0, 0, 0, 0};
  int obj = -1;
  double cobj = 0;
  double csig = 0;
  void axpy(double w, const Data& o);
};

struct Form {
  std::vector<std::pair<int64_t, double>> c;
  Data d;
  void add(int64_t col, double v);
  void axpy(double w, const Form& o);
};

struct Problem;

// ---------------------------------------------------------------------------
// one multigrid level
// ---------------------------------------------------------------------------
enum : uint8_t { TAG_GAS = 0, TAG_DIEL = 1, TAG_IRR = 2, TAG_COV = 3, TAG_NONSIMPLE = 4 };

struct Level {
  Grid g;
  int64_t N = 0, N2 = 0;
  std::vector<uint8_t> tag;
  std::vector<int8_t> primary;
  std::vector<int32_t> sec_of;
  std::vector<int32_t> sec_cell;
  // regular template: A phi_i = diag_i phi_i + coff[p] * sum_nb phi_nb,
  // diag_i = d0[p] + sum over touched domain faces f of cb[f][p]
  double coff[2] = {0, 0};
  double d0[2] = {0, 0};
  double cb[6][2] = {};
  double mass[2] = {0, 0};
  // irregular rows
  std::vector<int64_t> irow_dof;
  std::vector<int64_t> rp;
  std::vector<int32_t> col;
  std::vector<double> val;
  std::vector<double> idiag;
  std::vector<double> imass;
  std::vector<int32_t> cls_ptr;   // colour classes of irregular rows
  std::vector<int32_t> cls_rows;
  // transfer to the next coarser level (filled when that level exists)
  std::vector<int64_t> ns_cdof;   // non-simple coarse unknowns
  std::vector<int32_t> ns_ptr;
  std::vector<int64_t> ns_child;  // their fine children (unknown indices)
  std::vector<int64_t> np_fdof;   // fine unknowns whose parent is non-simple
  std::vector<int64_t> np_cdof;
  int64_t ndof() const { return N + N2; }
  void row(int64_t dof, double& mass_out, std::vector<std::pair<int64_t, double>>& out) const;
};

// finest-level extras: right-hand-side data and field rows
struct FineData {
  std::vector<Data> idata;        // per irregular row
  std::vector<double> isrc;       // kappa for the rho term (0 on secondary rows)
  double dat[6][2] = {};          // regular rows: b -= dat[f][p] * value_f
  // E rows of irregular primary cells: rows e = 3*q + d for cell ecell[q]
  std::vector<int64_t> ecell;
  std::vector<int64_t> erp;
  std::vector<int32_t> ecol;
  std::vector<double> eval;
  std::vector<Data> edata;
  // regular E at domain faces: dphi/dn_out = ga*phi_n + gb*value
  double ega[6][2] = {}, egb[6][2] = {};
};

struct Options {
  double alpha = 0, beta = -1, a_gas = 0, a_diel = 0, b_gas = 1;
  int dirichlet_closure = 0, robin_closure = 0, eb_order = 2;
  int precision = 0, nu1 = 2, nu2 = 2, bottom_max = 600, krylov = 1, smoother = 0, tail = 0, batch = 0, graphs = 0;
};

struct Problem {
  Options opt;
  ebmg_domain_bc bc;
  Geometry geo;
  double bph[2] = {1, 1};
  double aph[2] = {0, 0};
  std::vector<Level> levels;
  FineData fine;
  std::vector<double> bottom_inv;  // dense inverse of the coarsest level
  int64_t bottom_n = 0;
};

void build_fine_level(Problem& pb);
void build_hierarchy(Problem& pb);
void fine_template(Problem& pb);
void coarse_template(Level& C, const Problem& pb);
void build_bottom(Problem& pb);
void colour_irregular(Level& L);
void host_rhs(const Problem& pb, const double* rho, const double* sigma, const double* bcv,
              const double* objv, double* b);

// ---------------------------------------------------------------------------
// signed distance from a triangle mesh (host preparation; mesh.cpp)
// ---------------------------------------------------------------------------
struct MeshInput {
  int32_t nvert = 0, ntri = 0;
  const double* verts = nullptr;   // 3 per vertex
  const int32_t* tris = nullptr;   // 3 vertex indices per triangle, counter-clockwise seen from outside
};

// tree node: box; a leaf holds triangles [first, first + count) of the
// sorted records, an internal node (count < 0) has children first and -count
struct MeshNode {
  double lo[3], hi[3];
  int32_t first, count;
};

constexpr int kMeshLeaf = 4;
// per triangle: 3 vertices (9), face normal (3), pseudonormals of edges
// 01, 12, 20 (9), pseudonormals of vertices 0, 1, 2 (9)
constexpr int kMeshTriDoubles = 30;

struct MeshHost {
  int32_t ntri = 0;
  int depth = 0;
  std::vector<double> tri;         // kMeshTriDoubles per triangle, in leaf order
  std::vector<MeshNode> nodes;     // node 0 is the root
};

void build_mesh(const MeshInput& m, MeshHost& out);

// ---------------------------------------------------------------------------
// advection on the gas phase (host preparation; advect.cpp)
// ---------------------------------------------------------------------------
struct AdvHost {
  int64_t nfaces = 0;
  int64_t face_base[3] = {0, 0, 0};     // first face of each direction
  std::vector<uint8_t> cls;             // per cell: 0 no gas, 1 full, 2 cut, 3 full in a cut cell's block
  std::vector<double> kappa;            // per cell (gas volume fraction)
  std::vector<int64_t> cut_cell;        // cut cells in cell order
  std::vector<int64_t> dc_ptr, dc_face; // per cut cell: conservative divergence
  std::vector<double> dc_coef;          //   = sum coef * face flux
  std::vector<int64_t> nb_ptr, nb_cell; // per cut cell: gas cells of its block
  std::vector<double> nb_w;             //   with weights kappa_j / sum kappa
  std::vector<double> cut_S;            // per cut cell: sum kappa of the block without it
  std::vector<int64_t> sp_cell;         // cells whose rate is not D^c: cut cells and receivers
  std::vector<int32_t> sp_cut;          //   their cut id (-1: a full cell that receives)
  std::vector<int64_t> sp_ptr;          //   their donors (cut ids)
  std::vector<int32_t> sp_donor;
};

void build_advection(const Geometry& G, AdvHost& A);

// ---------------------------------------------------------------------------
// nested AMR hierarchies (amr.cpp)
// ---------------------------------------------------------------------------
struct AmrBox {
  int lo[3] = {0, 0, 0};   // first cell in the level's global index space
  int n[3] = {1, 1, 1};
  bool cf[6] = {false, false, false, false, false, false};   // coarse-fine faces
  int level = 0;
  int parent = -1;         // the box of the next coarser level holding it
};

// Coupling of a box (fine) with its parent (coarse), as sparse rows over
// unknown slots (cells, then second-phase unknowns, of each box).
struct AmrLink {
  // added to the fine level's A x: column >= 0 a fine slot, < 0 the coarse
  // slot -column - 1
  std::vector<int64_t> frow, fptr{0}, fcol;
  std::vector<double> fw;
  // added to the coarse level's A x: column >= 0 a coarse slot, < 0 the fine
  // slot -column - 1
  std::vector<int64_t> crow, cptr{0}, ccol;
  std::vector<double> cw;
  std::vector<int64_t> cov;                     // coarse slots under the fine box
  std::vector<int64_t> rrow, rptr{0}, rcol;     // covered coarse unknown <- its
  std::vector<double> rw, aw;                   // children's (rw: 1/2^D, aw: mean)
  std::vector<int64_t> pcol;                    // fine slot <- coarse slot (-1: none)
};

// C, cb: the parent box; ckids: every box refining it (fb among them);
// F, fb: the child; fkids: the boxes refining the child
void build_amr_link(const Problem& C, const AmrBox& cb, const std::vector<const AmrBox*>& ckids, const Problem& F,
                    const AmrBox& fb, const std::vector<const AmrBox*>& fkids, AmrLink& out);

}  // namespace ebmg
