// Solver driver and C ABI (see include/ebmg.h).
//
// Multigrid-solver subsection of arXiv:1809.03745: residual-correction
// geometric multigrid, Gauss-Seidel relaxation (red-black here, plus the
// irregular rows class by class), a direct bottom solve, and the stopping rule
// ||r|| < rtol ||r0|| with r0 the residual at phi = 0 (= ||b||).
// Mixed precision: the V-cycle (smoothing, restriction, prolongation) runs in
// FP32 on the correction equation A e = r, with r = b - A phi formed in FP64,
// the bottom level solved in FP64, and phi += e applied in FP64.
#include <hip/hip_runtime.h>
#include <hip/hip_ext.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <mutex>
#include <unordered_map>
#include <thread>
#include <type_traits>
#include <cmath>
#include <cstring>
#include <memory>
#include <string>
#include <vector>

#include "internal.hpp"
#include "block_engine.hpp"
#include "batch_wide.hpp"
#include "kernels.hpp"
#include "zq_kernels.hpp"
#include "sdf_kernels.hpp"
#include "adv_kernels.hpp"
#include "amr_kernels.hpp"

namespace ebmg {

struct DeviceError : std::runtime_error {
  using std::runtime_error::runtime_error;
};

#define HIPCHECK(expr)                                                                    \
  do {                                                                                    \
    hipError_t e_ = (expr);                                                               \
    if (e_ != hipSuccess)                                                                 \
      throw DeviceError(std::string(#expr) + ": " + hipGetErrorString(e_));               \
  } while (0)

static inline unsigned nblk(int64_t n) { return (unsigned)((n + kBlock - 1) / kBlock); }

// 3D launch shape over an (nx, ny, nz) index box: blocks of bx*by = 256
// threads (bx = 64 unless the rows are shorter), one grid z per plane
struct Shape {
  dim3 g, b;
};
static inline Shape shape3(int nx, int ny, int nz) {
  int bx = 64;
  while (bx > 8 && bx / 2 >= nx) bx /= 2;
  int by = kBlock / bx;
  while (by > 1 && by / 2 >= ny) by /= 2;
  Shape s;
  s.b = dim3(bx, by, 1);
  s.g = dim3((nx + bx - 1) / bx, (ny + by - 1) / by, nz);
  return s;
}

template <typename T>
struct DevBuf {
  T* p = nullptr;
  int64_t n = 0;
  bool own = true;   // false: an alias of another problem's buffer (a family member's shared structure)
  void alloc(int64_t count, int64_t& bytes) {
    n = count;
    own = true;
    if (count > 0) {
      HIPCHECK(hipMalloc((void**)&p, sizeof(T) * count));
      bytes += sizeof(T) * count;
    }
  }
  void upload(const T* host, int64_t count, hipStream_t s, int64_t& bytes) {
    alloc(count, bytes);
    if (count > 0) HIPCHECK(hipMemcpyAsync(p, host, sizeof(T) * count, hipMemcpyHostToDevice, s));
  }
  // use o's memory without owning it; returns the bytes not allocated
  int64_t share(const DevBuf& o) {
    p = o.p;
    n = o.n;
    own = false;
    return (int64_t)sizeof(T) * n;
  }
  void release() {
    if (p && own) (void)hipFree(p);
    p = nullptr;
    n = 0;
    own = true;
  }
};

// Event pairs stamped with the start and end of one level's kernel launches
// during solves (measurement hook; the launches go through KLAUNCH), read
// after the solve's final synchronisation.
struct KTiming {
  std::vector<hipEvent_t> ev;
  size_t used = 0;   // events handed out since the last harvest (pairs)
  int64_t n = 0;     // launches timed
  double ms = 0;     // their total duration
  std::pair<hipEvent_t, hipEvent_t> pair() {
    while (used + 2 > ev.size()) {
      hipEvent_t e = nullptr;
      HIPCHECK(hipEventCreate(&e));
      ev.push_back(e);
    }
    used += 2;
    return {ev[used - 2], ev[used - 1]};
  }
  void harvest() {
    for (size_t i = 0; i + 1 < used; i += 2) {
      float t = 0;
      HIPCHECK(hipEventElapsedTime(&t, ev[i], ev[i + 1]));
      ms += t;
      ++n;
    }
    used = 0;
  }
  ~KTiming() {
    for (hipEvent_t e : ev) (void)hipEventDestroy(e);
  }
};

// A kernel launch; with a timing record kt (non-null) the kernel's own start
// and end are stamped into a fresh event pair of kt by the dispatch itself.
#define KLAUNCH(kt, kernel, grid, block, shmem, stream, ...)                                            \
  do {                                                                                                \
    if (kt) {                                                                                         \
      const auto ev_ = (kt)->pair();                                                                  \
      hipExtLaunchKernelGGL(kernel, grid, block, shmem, stream, ev_.first, ev_.second, 0, __VA_ARGS__); \
    } else {                                                                                          \
      hipLaunchKernelGGL(kernel, grid, block, shmem, stream, __VA_ARGS__);                            \
    }                                                                                                 \
  } while (0)

struct DevLevel {
  int dim = 2;
  int n[3] = {1, 1, 1};
  int64_t N = 0, N2 = 0, R = 0;
  DevBuf<uint8_t> tag;
  DevBuf<int64_t> irow_dof, rp, ns_cdof, ns_child, np_fdof, np_cdof;
  DevBuf<int32_t> col, cls_rows, ns_ptr;
  DevBuf<double> val64, diag64;
  DevBuf<float> val32, diag32;
  std::vector<int32_t> cls_ptr;
  // sliced copy of the explicit rows (engine and batched kernels)
  DevBuf<int64_t> sl_ptr;
  DevBuf<int32_t> sl_col;
  DevBuf<int32_t> sl_colj;   // group 1's columns with explicit-row unknowns renamed (see k_irr_jac_sl2x)
  DevBuf<double> sl_val64;
  DevBuf<float> sl_val32;
  int sl_grp[3] = {0, 0, 0};
  int64_t n_ns = 0, n_np = 0;
  bool fused = false;              // smoother variant chosen for this level
  bool oop = false;                // non-fused: one-launch colour phases (else split in place)
  int fvar = 0;                    // fused variant: 0 3D/2D tile, 1 z-marching (3D)
  int zmcfg = 0;                   // z-marching tile configuration
  KTiming* kt = nullptr;           // sweep launches timed during solves (or none)
  KTiming* ktr = nullptr;          // FP64 residual launches timed during solves (or none)
  double tune_split_ms = 0, tune_fused_ms = 0, tune_zm_ms = 0, tune_oop_ms = 0;
  std::vector<double> tune_zm_cfg_ms;   // sweep ms of each z-marching configuration (0: not timed)
  Tmpl<double> t64;
  Tmpl<float> t32;
  // vectors
  DevBuf<double> x64, b64, r64, w64, xa64;
  DevBuf<float> x32, b32, r32, w32, xa32;
  void release() {
    tag.release(); irow_dof.release(); rp.release(); ns_cdof.release(); ns_child.release();
    np_fdof.release(); np_cdof.release(); col.release(); cls_rows.release(); ns_ptr.release();
    val64.release(); diag64.release(); val32.release(); diag32.release();
    sl_ptr.release(); sl_col.release(); sl_colj.release(); sl_val64.release(); sl_val32.release();
    x64.release(); b64.release(); r64.release(); x32.release(); b32.release(); r32.release();
    w64.release(); w32.release(); xa64.release(); xa32.release();
  }
};

struct DevProblem {
  std::vector<DevLevel> lv;
  DevBuf<double> bottom;
  int64_t bottom_n = 0;
  // rhs data of irregular rows
  DevBuf<int64_t> icell;
  DevBuf<double> isrc, iface, icobj, icsig;
  DevBuf<int32_t> iobj;
  // E rows
  DevBuf<int64_t> ecell, erp;
  DevBuf<int32_t> ecol, eobj;
  DevBuf<double> eval, eface, ecobj, ecsig;
  DevBuf<double> objv;
  DevBuf<double> part, scal;
  double* host_scal = nullptr;
  // BiCGStab work vectors: r, rh, p, v, ph, s, sh, t; for mixed precision the
  // preconditioner outputs stay FP32 (ph32, sh32) and are widened on use
  DevBuf<double> kv[8];
  DevBuf<float> ph32, sh32;
  bool krylov = false;
  // coarse tail run by one workgroup: levels tail_l0 .. end (-1: none)
  int tail_l0 = -1;
  std::vector<int> tail_cand;     // candidate first tail levels timed at setup
  std::vector<double> tail_ms;    // V-cycle ms for each candidate
  DevBuf<uint8_t> tail_lv;
  // Krylov bottom solve (no dense inverse): work vectors and its device view
  DevBuf<double> bk_vec;
  DevBuf<uint8_t> bk_dev;
  // replayed iteration graphs (captured at the first solve that needs them)
  hipGraphExec_t g_krylov = nullptr, g_plain = nullptr;
  // measurement hook: sweep launches of one level timed during solves, which
  // then launch their kernels directly instead of replaying graphs
  std::unique_ptr<KTiming> kt[2];   // [0] sweeps, [1] FP64 residuals
  int kt_level[2] = {-1, -1};
  bool timing() const { return kt[0] || kt[1]; }
  int64_t bytes = 0;
  int64_t shared_bytes = 0;   // structure taken from another family member (not allocated here)
  // advection on the gas phase (built at the first ebmg_advect call)
  struct Adv {
    bool ready = false;
    int64_t nfaces = 0, fbase[3] = {0, 0, 0};
    int ncut = 0, nsp = 0;
    DevBuf<uint8_t> cls;
    DevBuf<double> kappa, dc_coef, nb_w, cut_S, F, Dc, Dcut, give;
    DevBuf<int64_t> cut_cell, dc_ptr, dc_face, nb_ptr, nb_cell, sp_cell, sp_ptr;
    DevBuf<int32_t> sp_cut, sp_donor;
    void release() {
      cls.release(); kappa.release(); dc_coef.release(); nb_w.release(); cut_S.release(); F.release();
      Dc.release(); Dcut.release(); give.release(); cut_cell.release(); dc_ptr.release(); dc_face.release();
      nb_ptr.release(); nb_cell.release(); sp_cell.release(); sp_ptr.release(); sp_cut.release(); sp_donor.release();
      ready = false;
    }
  } adv;
  void drop_graphs() {
    if (g_krylov) (void)hipGraphExecDestroy(g_krylov);
    if (g_plain) (void)hipGraphExecDestroy(g_plain);
    g_krylov = g_plain = nullptr;
  }
  void release() {
    drop_graphs();
    kt[0].reset();
    kt[1].reset();
    for (auto& l : lv) l.release();
    lv.clear();
    bottom.release(); icell.release(); isrc.release(); iface.release(); icobj.release(); icsig.release();
    iobj.release(); ecell.release(); erp.release(); ecol.release(); eobj.release(); eval.release();
    eface.release(); ecobj.release(); ecsig.release(); objv.release(); part.release(); scal.release();
    for (auto& k : kv) k.release();
    ph32.release();
    sh32.release();
    tail_lv.release();
    bk_vec.release();
    bk_dev.release();
    adv.release();
    if (host_scal) (void)hipHostFree(host_scal);
    host_scal = nullptr;
  }
};

}  // namespace ebmg

// A queued solve: device pointers as given, boundary values copied at submit.
struct AsyncJob {
  uint64_t ticket = 0;
  ebmg_problem pb = nullptr;
  const double* rho = nullptr;
  const double* sigma = nullptr;
  std::vector<double> bcv, objv;  // empty: the setup values
  double rtol = 0;
  int max_cycles = 0;
  double* phi = nullptr;
  double* phi2 = nullptr;
  double* E = nullptr;
};

struct AsyncResult {
  bool done = false;
  ebmg_status status = EBMG_OK;
  ebmg_solve_info info{};
  std::string err;
};

struct ebmg_ctx_s {
  int device = -1;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  std::string err;
  // submitted solves: one worker thread per context runs them in order
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<AsyncJob> queue;
  std::unordered_map<uint64_t, AsyncResult> results;
  uint64_t next_ticket = 1;
  bool stop = false;
  std::thread worker;
  // the handle plus each live problem and batch: the stream and the worker
  // outlive ebmg_destroy until the last problem set up on the context is gone
  std::atomic<int> refs{1};
};

struct ebmg_problem_s {
  ebmg_ctx ctx = nullptr;
  std::unique_ptr<ebmg::Problem> host;
  ebmg::DevProblem dev;
  bool on_device = false;
  int pending = 0;  // submitted solves not yet finished (guarded by ctx->mu)
};

// A triangle mesh resident on the device for signed-distance queries.
struct ebmg_mesh_s {
  ebmg_ctx ctx = nullptr;
  ebmg::DevBuf<double> tri;
  ebmg::DevBuf<uint8_t> nodes;
  ebmg::DevBuf<unsigned long long> visits;   // search counter of the last query
  int32_t ntri = 0, nnode = 0, depth = 0;
  int64_t bytes = 0;
};

// Operators on one geometry (a family): member 0 owns the device structure,
// the others take it and hold their own values and vectors; each member has
// a private context (its own stream), so members solve concurrently.
struct ebmg_family_s {
  ebmg_ctx ctx = nullptr;                    // the caller's context
  std::vector<ebmg_ctx> mctx;                // one private context per member
  std::vector<ebmg_problem_s*> mem;
  bool warm = false;                         // every member has solved once (graphs captured)
};

// A nested AMR hierarchy: one problem per box (its own operator and
// multigrid hierarchy), the coupling rows of every parent-child pair on the
// device, and the composite vectors (every box's unknowns in one contiguous
// array, each box's slice starting on a 64-entry boundary).
struct ebmg_amr_s {
  ebmg_ctx ctx = nullptr;
  std::vector<ebmg_problem_s*> lev;
  std::vector<ebmg::AmrBox> box;
  struct Link {
    ebmg::DevBuf<int64_t> frow, fptr, fcol, crow, cptr, ccol, cov, rrow, rptr, rcol, pcol;
    ebmg::DevBuf<double> fw, cw, rw, aw;
    int64_t nf = 0, nc = 0, ncov = 0, nr = 0, np = 0;
    void release() {
      frow.release(); fptr.release(); fcol.release(); crow.release(); cptr.release(); ccol.release();
      cov.release(); rrow.release(); rptr.release(); rcol.release(); pcol.release();
      fw.release(); cw.release(); rw.release(); aw.release();
    }
  };
  std::vector<Link> link;          // link[i] couples box i with its parent (i >= 1)
  std::vector<int64_t> off, nd;    // per box: slice offset and unknowns (N + N2)
  std::vector<int> order;          // boxes by level, deepest first
  int64_t ntot = 0;
  ebmg::DevBuf<double> x, b, r, rh, p, v, sv, t, ph, sh, rt, y, e, part, scal;
  int64_t bytes = 0;
};

// Many independent boxes solved by one persistent launch.
struct ebmg_batch_s {
  ebmg_ctx ctx = nullptr;
  std::vector<std::unique_ptr<ebmg_problem_s>> boxes;
  std::vector<ebmg::DevBuf<uint8_t>> lvbuf;   // per-box device level views
  ebmg::DevBuf<uint8_t> bbox;                 // BBox<T> per box
  ebmg::DevBuf<uint8_t> bio;                  // BIO per box
  ebmg::DevBuf<uint8_t> bres;                 // BRes per box
  ebmg::DevBuf<int32_t> order;                // boxes, largest first
  bool mixed = false;
  int dim = 3;
  int nu1 = 2, nu2 = 2;
  int64_t cells = 0, cells2 = 0, bytes = 0;
  // level-synchronous mode (mode 2)
  int mode = 2;
  struct Table {
    ebmg::DevBuf<uint8_t> d;   // WEnt entries, padded to a multiple of 8
    int n = 0;                 // padded count (0: nothing to launch)
  };
  struct WideLevel {
    Table rb, jac[2], scat[2], cell, res, pro;
  };
  std::vector<ebmg::DevBuf<uint8_t>> wl;      // BLev per box for levels >= 1 (index = level)
  ebmg::DevBuf<uint8_t> wl0[2];               // level 0 with the cycle vectors of application 0 / 1
  std::vector<WideLevel> wide;                // levels run by grid-wide launches
  Table op64, vec;
  Table bot;                                  // grid-wide bottom solves
  ebmg::DevBuf<int32_t> ebeg_op, ebeg_vec, lt;
  ebmg::DevBuf<int32_t> tail_list;            // boxes whose coarse part runs in one workgroup
  int n_tail = 0;
  ebmg::DevBuf<double> part0, part1;
  ebmg::DevBuf<uint8_t> state, wio;
  ebmg::DevBuf<int32_t> count;
  int* host_count = nullptr;
  int tail_cells = 0;
  int tail_opt = 0;   // options.tail of the boxes: 0 timed, 1 bottom only, 2 from kTailMax unknowns
  std::vector<int> cand_cells;
  std::vector<double> cand_ms;
  // replayed iteration graph and the stopping parameters baked into it
  bool graphs = true;
  hipGraphExec_t g_iter = nullptr;
  double g_rtol = 0;
  int g_max_cycles = -1;
};

namespace ebmg {

// ---------------------------------------------------------------------------
// upload
// ---------------------------------------------------------------------------
template <typename T>
static Tmpl<T> make_tmpl(const Level& L) {
  Tmpl<T> t;
  for (int p = 0; p < 2; ++p) {
    t.coff[p] = (T)L.coff[p];
    t.d0[p] = (T)L.d0[p];
    t.mass[p] = (T)L.mass[p];
    for (int f = 0; f < 6; ++f) {
      t.cb[f][p] = (T)L.cb[f][p];
      t.cbm[f][p] = (T)(L.cb[f][p] - L.coff[p]);
    }
  }
  for (int d = 0; d < 3; ++d) t.n[d] = L.g.n[d];
  return t;
}

template <typename T>
struct Vec;
template <>
struct Vec<double> {
  static double* x(DevLevel& l) { return l.x64.p; }
  static double* b(DevLevel& l) { return l.b64.p; }
  static double* r(DevLevel& l) { return l.r64.p; }
  static const double* val(DevLevel& l) { return l.val64.p; }
  static const double* diag(DevLevel& l) { return l.diag64.p; }
  static const double* sval(DevLevel& l) { return l.sl_val64.p; }
  static const Tmpl<double>& t(DevLevel& l) { return l.t64; }
  static double* tmp(DevLevel& l) { return l.w64.p; }
  static double* xa(DevLevel& l) { return l.xa64.p; }
};
template <>
struct Vec<float> {
  static float* x(DevLevel& l) { return l.x32.p; }
  static float* b(DevLevel& l) { return l.b32.p; }
  static float* r(DevLevel& l) { return l.r32.p; }
  static const float* val(DevLevel& l) { return l.val32.p; }
  static const float* diag(DevLevel& l) { return l.diag32.p; }
  static const float* sval(DevLevel& l) { return l.sl_val32.p; }
  static const Tmpl<float>& t(DevLevel& l) { return l.t32; }
  static float* tmp(DevLevel& l) { return l.w32.p; }
  static float* xa(DevLevel& l) { return l.xa32.p; }
};

template <typename T>
static void fill(T* x, int64_t n, T v, hipStream_t s) {
  if (n > 0) hipLaunchKernelGGL((k_fill<T>), dim3(nblk(n)), dim3(kBlock), 0, s, x, n, v);
}

// levels large enough for the fused out-of-place red/black sweep
// 3D levels of at least this many cells take the z-marching residual kernel
constexpr int64_t kResidZMMin = 1 << 18;

// tiles of the z-marching residual (a 1D grid)
static int64_t zm_resid_blocks(const DevLevel& l) {
  return (int64_t)((l.n[0] + kRZX - 1) / kRZX) * ((l.n[1] + kRZY - 1) / kRZY) * ((l.n[2] + kRZ - 1) / kRZ);
}

// blocks of one matrix-vector product on a level (the partials it leaves)
// FP64 residuals of 3D levels with an even x extent use the paired-cell
// kernel (2-element accesses need that, and aligned arrays, which device
// allocations are)
static bool pair_ok(const DevLevel& l) { return l.dim == 3 && l.N >= kResidZMMin && l.n[0] % 2 == 0; }
static int64_t zp_resid_blocks(const DevLevel& l) {
  return (int64_t)((l.n[0] + kRPX - 1) / kRPX) * ((l.n[1] + kRPY - 1) / kRPY) * ((l.n[2] + kRPZ - 1) / kRPZ);
}
template <typename A>
static bool al2(const A* p) {
  return ((uintptr_t)p % (2 * sizeof(A))) == 0;
}
// partials one matrix-vector product on a level may leave (for sizing): the
// template-cell blocks of whichever residual kernel runs, plus the explicit
// rows' blocks of whichever row kernel runs (the sliced one takes a block per
// 64-row slice of each colour group, the CSR one a block per 32 rows)
static int64_t matvec_blocks(const DevLevel& l) {
  const int64_t csr = (int64_t)nblk(l.R * kSub);
  if (l.dim == 3 && l.N >= kResidZMMin) {
    int64_t sl = 0;
    if (l.cls_ptr.size() == 3)
      sl = (l.cls_ptr[1] - l.cls_ptr[0] + kSplitRows - 1) / kSplitRows +
           (l.cls_ptr[2] - l.cls_ptr[1] + kSplitRows - 1) / kSplitRows;
    else
      sl = (l.R + kSplitRows - 1) / kSplitRows;
    return std::max(zm_resid_blocks(l), zp_resid_blocks(l)) + std::max(csr, sl);
  }
  return (int64_t)nblk(l.N) + csr;
}

static bool fused_ok(const DevLevel& l) {
  return l.dim == 3 ? (l.N >= 32768 && l.n[0] >= 32) : (l.N >= 65536 && l.n[0] >= 64);
}

// z-marching sweep configurations (tile width x height x planes per block);
// the setup autotuner picks one per level
constexpr int kZMConfigs = 14;   // 7..9: wide-fetch versions of 1, 4, 6 (x extent a multiple of 4);
                                  // 10: 64x16 over 8 planes (enough blocks on mid-size levels);
                                  // 11..13: quad form (k_rb_zq3) 64x16, 128x16 and 128x8 over 32
                                  // (x extent a multiple of 4)
static bool zm_cfg_ok(const DevLevel& l, int c) { return (c < 7 || c == 10) || l.n[0] % 4 == 0; }

// zin: x is zero on entry, so the sweep need not read it (not timed by the
// in-solve hook: it moves fewer bytes than a full sweep)
template <typename T, int TX, int TY, int KZ, bool WIDE = false>
static void launch_zm_cfg(DevLevel& l, const T* xin, T* xout, const T* b, const Tmpl<T>& tp, hipStream_t s,
                          bool zin) {
  if (WIDE && l.n[0] % 4 != 0) throw ArgError("the wide-fetch sweep needs an x extent that is a multiple of 4");
  const int64_t nb = (int64_t)((l.n[0] + TX - 1) / TX) * ((l.n[1] + TY - 1) / TY) * ((l.n[2] + KZ - 1) / KZ);
  if (zin)
    hipLaunchKernelGGL((k_rb_zm3<T, TX, TY, KZ, WIDE, true>), dim3((unsigned)nb), dim3(TX * TY / 2), 0, s, l.tag.p,
                       xin, xout, b, tp, l.N2);
  else
    KLAUNCH(l.kt, (k_rb_zm3<T, TX, TY, KZ, WIDE>), dim3((unsigned)nb), dim3(TX * TY / 2), 0, s, l.tag.p, xin, xout,
            b, tp, l.N2);
}

template <typename T, int TX, int TY, int KZ, int OCC>
static void launch_zq_cfg(DevLevel& l, const T* xin, T* xout, const T* b, const Tmpl<T>& tp, hipStream_t s,
                          bool zin) {
  if (l.n[0] % 4 != 0) throw ArgError("the quad sweep needs an x extent that is a multiple of 4");
  auto al4 = [](const void* p, size_t es) { return (uintptr_t)p % (4 * es) == 0; };
  if (!al4(xout, sizeof(T)) || !al4(b, sizeof(T)) || !al4(l.tag.p, 1) || (!zin && !al4(xin, sizeof(T))) ||
      (l.N + l.N2) * (int64_t)sizeof(T) >= ((int64_t)1 << 31)) {
    // vectors not aligned to whole quads, or too large for the kernel's
    // 32-bit byte offsets: the same sweep by the pair form
    launch_zm_cfg<T, 64, 16, 32>(l, xin, xout, b, tp, s, zin);
    return;
  }
  const int64_t nb = (int64_t)((l.n[0] + TX - 1) / TX) * ((l.n[1] + TY - 1) / TY) * ((l.n[2] + KZ - 1) / KZ);
  if (zin)
    hipLaunchKernelGGL((k_rb_zq3<T, TX, TY, KZ, OCC, true>), dim3((unsigned)nb), dim3(TX * TY / 4), 0, s, l.tag.p, xin,
                       xout, b, tp, l.N2);
  else
    KLAUNCH(l.kt, (k_rb_zq3<T, TX, TY, KZ, OCC>), dim3((unsigned)nb), dim3(TX * TY / 4), 0, s, l.tag.p, xin, xout, b,
            tp, l.N2);
}

template <typename T>
static void launch_zm(DevLevel& l, const T* xin, T* xout, const T* b, const Tmpl<T>& tp, hipStream_t s,
                      bool zin = false) {
  switch (l.zmcfg) {
    case 11: launch_zq_cfg<T, 64, 16, 32, 2>(l, xin, xout, b, tp, s, zin); break;
    case 12: launch_zq_cfg<T, 128, 16, 32, 2>(l, xin, xout, b, tp, s, zin); break;
    case 13: launch_zq_cfg<T, 128, 8, 32, 2>(l, xin, xout, b, tp, s, zin); break;
    case 1: launch_zm_cfg<T, 64, 16, 32>(l, xin, xout, b, tp, s, zin); break;
    case 2: launch_zm_cfg<T, 32, 16, 32>(l, xin, xout, b, tp, s, zin); break;
    case 3: launch_zm_cfg<T, 64, 8, 16>(l, xin, xout, b, tp, s, zin); break;
    case 4: launch_zm_cfg<T, 128, 8, 32>(l, xin, xout, b, tp, s, zin); break;
    case 5: launch_zm_cfg<T, 32, 8, 32>(l, xin, xout, b, tp, s, zin); break;
    case 6: launch_zm_cfg<T, 32, 32, 32>(l, xin, xout, b, tp, s, zin); break;
    case 7: launch_zm_cfg<T, 64, 16, 32, true>(l, xin, xout, b, tp, s, zin); break;
    case 8: launch_zm_cfg<T, 128, 8, 32, true>(l, xin, xout, b, tp, s, zin); break;
    case 9: launch_zm_cfg<T, 32, 32, 32, true>(l, xin, xout, b, tp, s, zin); break;
    case 10: launch_zm_cfg<T, 64, 16, 8>(l, xin, xout, b, tp, s, zin); break;
    default: launch_zm_cfg<T, 64, 8, 32>(l, xin, xout, b, tp, s, zin); break;
  }
}

// zin (z-marching form only): x is zero on entry
template <typename T>
static void launch_fused(DevLevel& l, const T* xin, T* xout, const T* b, const Tmpl<T>& tp, hipStream_t s,
                         bool zin = false) {
  if (l.dim == 3 && l.fvar == 1) {
    launch_zm<T>(l, xin, xout, b, tp, s, zin);
  } else if (l.dim == 3) {
    const int64_t nb = (int64_t)((l.n[0] + kTX - 1) / kTX) * ((l.n[1] + kTY - 1) / kTY) * ((l.n[2] + kTZ - 1) / kTZ);
    KLAUNCH(l.kt, (k_rb_tile3<T>), dim3((unsigned)nb), dim3(kTileThreads), 0, s, l.tag.p, xin, xout, b, tp, l.N2);
  } else {
    const int64_t nb = (int64_t)((l.n[0] + kTX2 - 1) / kTX2) * ((l.n[1] + kTY2 - 1) / kTY2);
    KLAUNCH(l.kt, (k_rb_tile2<T>), dim3((unsigned)nb), dim3(kTileThreads), 0, s, l.tag.p, xin, xout, b, tp, l.N2);
  }
}

// Levels with at most this many unknowns may be run by the one-workgroup
// engine; the setup autotuner picks the first such level (or none).
constexpr int64_t kTailMax = 32768;

template <typename T>
static BLev<T> make_blev(DevLevel& l) {
  BLev<T> v;
  std::memset(&v, 0, sizeof(v));
  v.dim = l.dim;
  for (int d = 0; d < 3; ++d) v.n[d] = l.n[d];
  v.N = (int)l.N;
  v.N2 = (int)l.N2;
  v.R = (int)l.R;
  v.tag = l.tag.p;
  v.irow_dof = l.irow_dof.p;
  v.rp = l.rp.p;
  v.col = l.col.p;
  v.val = Vec<T>::val(l);
  v.diag = Vec<T>::diag(l);
  v.grp_rows = l.cls_rows.p;
  for (int g = 0; g < 3; ++g) v.grp_ptr[g] = g < (int)l.cls_ptr.size() ? l.cls_ptr[g] : (g == 0 ? 0 : (int)l.R);
  v.sl_ptr = l.sl_ptr.p;
  v.sl_col = l.sl_col.p;
  v.sl_val = Vec<T>::sval(l);
  for (int g = 0; g < 3; ++g) v.sl_grp[g] = l.sl_grp[g];
  v.tp = Vec<T>::t(l);
  v.x = Vec<T>::x(l);
  v.b = Vec<T>::b(l);
  v.r = Vec<T>::r(l);
  v.w = Vec<T>::tmp(l);
  v.n_ns = (int)l.n_ns;
  v.ns_cdof = l.ns_cdof.p;
  v.ns_ptr = l.ns_ptr.p;
  v.ns_child = l.ns_child.p;
  v.n_np = (int)l.n_np;
  v.np_fdof = l.np_fdof.p;
  v.np_cdof = l.np_cdof.p;
  return v;
}

template <typename T>
static void vcycle(DevProblem& D, const Options& o, size_t l, hipStream_t s, T* x, const T* b, bool xz = false);

// Tail autotuner: time a whole V-cycle (on zero vectors) with the one-
// workgroup engine starting at each level of at most kTailMax unknowns, and
// with no tail at all; keep the fastest.
// Sweep timings alone rank the z-marching configurations of the finest level
// only to within a few per cent; where the finest level uses one, the
// fastest few are timed again inside whole V-cycles (the solve's own cache
// state) and the fastest V-cycle decides.
template <typename T>
static void refine_finest_zm(DevProblem& D, const Options& o, hipStream_t s) {
  DevLevel& L0 = D.lv[0];
  if (o.smoother != 0 || !L0.fused || L0.fvar != 1 || L0.tune_zm_cfg_ms.empty() || D.lv.size() < 2) return;
  std::vector<int> cfg;
  for (int c = 0; c < (int)L0.tune_zm_cfg_ms.size(); ++c)
    if (L0.tune_zm_cfg_ms[c] > 0) cfg.push_back(c);
  std::sort(cfg.begin(), cfg.end(), [&](int a, int b) { return L0.tune_zm_cfg_ms[a] < L0.tune_zm_cfg_ms[b]; });
  if (cfg.size() > 3) cfg.resize(3);
  if (cfg.size() < 2) return;
  T* x = Vec<T>::x(L0);
  T* b = Vec<T>::b(L0);
  fill<T>(x, L0.N + L0.N2, T(0), s);
  fill<T>(b, L0.N + L0.N2, T(0), s);
  const int tail0 = D.tail_l0;
  D.tail_l0 = -1;
  hipEvent_t e0, e1;
  HIPCHECK(hipEventCreate(&e0));
  HIPCHECK(hipEventCreate(&e1));
  double best = 1e30;
  int pick = L0.zmcfg;
  for (int c : cfg) {
    L0.zmcfg = c;
    for (int r = 0; r < 2; ++r) vcycle<T>(D, o, 0, s, x, b);
    const int reps = 5;
    HIPCHECK(hipEventRecord(e0, s));
    for (int r = 0; r < reps; ++r) vcycle<T>(D, o, 0, s, x, b);
    HIPCHECK(hipEventRecord(e1, s));
    HIPCHECK(hipEventSynchronize(e1));
    float ms = 0;
    HIPCHECK(hipEventElapsedTime(&ms, e0, e1));
    if (ms < best) {
      best = ms;
      pick = c;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  L0.zmcfg = pick;
  D.tail_l0 = tail0;
}

template <typename T>
static void tune_tail(DevProblem& D, const Options& o, hipStream_t s) {
  const int nl = (int)D.lv.size();
  std::vector<int> cand;
  if (o.tail != 2) cand.push_back(-1);
  if (o.tail != 1)
    for (int l = nl - 1; l >= 0 && D.lv[l].N + D.lv[l].N2 <= kTailMax; --l) cand.push_back(l);
  if (o.tail == 2 && cand.size() > 1) cand.erase(cand.begin(), cand.end() - 1);
  if (cand.size() == 1) {
    D.tail_cand = cand;
    D.tail_ms.assign(1, 0.0);
    D.tail_l0 = cand[0];
    return;
  }
  DevLevel& L0 = D.lv[0];
  T* x = Vec<T>::x(L0);
  T* b = Vec<T>::b(L0);
  fill<T>(x, L0.N + L0.N2, T(0), s);
  fill<T>(b, L0.N + L0.N2, T(0), s);
  hipEvent_t e0, e1;
  HIPCHECK(hipEventCreate(&e0));
  HIPCHECK(hipEventCreate(&e1));
  double best = 1e30;
  int pick = -1;
  D.tail_ms.assign(cand.size(), 0.0);
  for (size_t k = 0; k < cand.size(); ++k) {
    D.tail_l0 = cand[k];
    for (int r = 0; r < 2; ++r) vcycle<T>(D, o, 0, s, x, b);
    const int reps = 5;
    HIPCHECK(hipEventRecord(e0, s));
    for (int r = 0; r < reps; ++r) vcycle<T>(D, o, 0, s, x, b);
    HIPCHECK(hipEventRecord(e1, s));
    HIPCHECK(hipEventSynchronize(e1));
    float ms = 0;
    HIPCHECK(hipEventElapsedTime(&ms, e0, e1));
    D.tail_ms[k] = ms / reps;
    if (ms / reps < best) {
      best = ms / reps;
      pick = cand[k];
    }
  }
  D.tail_cand = cand;
  D.tail_l0 = pick;
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
}

template <typename T>
static void upload_tail(DevProblem& D, hipStream_t s) {
  const int nl = (int)D.lv.size();
  D.tail_l0 = -1;
  std::vector<BLev<T>> v;
  for (int l = 0; l < nl; ++l) v.push_back(make_blev<T>(D.lv[l]));
  int64_t by = 0;
  D.tail_lv.upload((const uint8_t*)v.data(), (int64_t)(v.size() * sizeof(BLev<T>)), s, by);
  D.bytes += by;
  HIPCHECK(hipStreamSynchronize(s));
}

template <typename T>
static void smooth(DevLevel& l, T* x, const T* b, int sweeps, hipStream_t s, bool xz = false);

// Smoother autotuner: time a complete sweep (template cells and explicit
// rows) of each variant with HIP events on zeroed vectors and keep the
// fastest. On levels whose vectors could stay in the last-level cache
// between back-to-back sweeps while a solve would have evicted them, a
// scratch buffer larger than that cache is written between the timed pairs
// of sweeps, so the sweeps are timed from memory as in a solve. Variants:
// split half-sweeps in place with grouped explicit rows, one-launch
// colour phases out of place, and where they apply the fused tile sweep and
// the z-marching sweep in each tile configuration. Forced modes: 1 split,
// 2 fused tile, 3 z-marching (tile in 2D) where the fused sweeps apply;
// 4 a fixed rule with no timing (z-marching 64x16 tiles / tile sweep where
// the fused sweeps apply, one-launch colour phases elsewhere).
template <typename T>
static double time_smooth(DevLevel& l, T* x, const T* b, hipStream_t s, float* flush, int64_t nflush) {
  hipEvent_t e0, e1;
  HIPCHECK(hipEventCreate(&e0));
  HIPCHECK(hipEventCreate(&e1));
  smooth<T>(l, x, b, 2, s);
  double tot = 0;
  const int pairs = flush ? 2 : 1;
  for (int r = 0; r < pairs; ++r) {
    if (flush) fill<float>(flush, nflush, (float)r, s);
    HIPCHECK(hipEventRecord(e0, s));
    smooth<T>(l, x, b, flush ? 2 : 4, s);
    HIPCHECK(hipEventRecord(e1, s));
    HIPCHECK(hipEventSynchronize(e1));
    HIPCHECK(hipGetLastError());
    float ms = 0;
    HIPCHECK(hipEventElapsedTime(&ms, e0, e1));
    tot += ms;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return tot / 4.0;
}

template <typename T>
static void tune_level(DevLevel& l, T* x, T* xa, T* b, int mode, hipStream_t s, float* flush, int64_t nflush) {
  const int64_t nd = l.N + l.N2;
  fill<T>(x, nd, T(0), s);
  fill<T>(xa, nd, T(0), s);
  fill<T>(b, nd, T(0), s);
  const bool fok = fused_ok(l);
  l.fused = false;
  l.oop = false;
  l.fvar = 0;
  if (mode == 1) return;
  if (mode == 2 || mode == 3) {
    l.fused = fok;
    l.fvar = (mode == 3 && l.dim == 3) ? 1 : 0;
    return;
  }
  if (mode == 4) {
    // fixed rule (no timing, so the choice never depends on what else runs):
    // 3D levels of at least 2^23 cells take the z-marching sweep (quad form
    // where the x extent allows), smaller ones the one-launch colour phases,
    // which on those sizes beat a z-march with too few blocks; 2D levels take
    // the fused tile sweep where it applies
    const bool big3 = l.dim == 3 && l.N >= ((int64_t)1 << 23);
    l.fused = l.dim == 3 ? (fok && big3) : fok;
    l.fvar = l.dim == 3 ? 1 : 0;
    l.zmcfg = l.n[0] % 4 == 0 ? 13 : 1;
    l.oop = !l.fused;
    return;
  }
  struct Cand {
    bool fused, oop;
    int fvar, zmcfg;
    double ms;
  };
  std::vector<Cand> cands = {{false, false, 0, 0, 0}, {false, true, 0, 0, 0}};
  if (fok) {
    cands.push_back({true, false, 0, 0, 0});
    if (l.dim == 3)
      for (int c = 0; c < kZMConfigs; ++c)
        if (zm_cfg_ok(l, c)) cands.push_back({true, false, 1, c, 0});
  }
  size_t best = 0;
  double zbest = 1e30;
  for (size_t q = 0; q < cands.size(); ++q) {
    l.fused = cands[q].fused;
    l.oop = cands[q].oop;
    l.fvar = cands[q].fvar;
    l.zmcfg = cands[q].zmcfg;
    cands[q].ms = time_smooth<T>(l, x, b, s, flush, nflush);
    if (cands[q].ms < cands[best].ms) best = q;
    if (!cands[q].fused && !cands[q].oop) l.tune_split_ms = cands[q].ms;
    if (cands[q].oop) l.tune_oop_ms = cands[q].ms;
    if (cands[q].fused && cands[q].fvar == 0) l.tune_fused_ms = cands[q].ms;
    if (cands[q].fused && cands[q].fvar == 1) {
      l.tune_zm_cfg_ms.resize(kZMConfigs, 0.0);
      l.tune_zm_cfg_ms[cands[q].zmcfg] = cands[q].ms;
    }
    if (cands[q].fused && cands[q].fvar == 1 && cands[q].ms < zbest) {
      zbest = cands[q].ms;
      l.tune_zm_ms = zbest;
    }
  }
  l.fused = cands[best].fused;
  l.oop = cands[best].oop;
  l.fvar = cands[best].fvar;
  l.zmcfg = cands[best].zmcfg;
  fill<T>(x, nd, T(0), s);
  fill<T>(xa, nd, T(0), s);
}

// Last-level cache of the device (256 MB on MI355X) and the scratch written
// between timed sweeps: sweeps whose vectors and tags exceed a quarter of it
// are timed from memory.
constexpr int64_t kLLCBytes = (int64_t)256 << 20;
constexpr int64_t kFlushBytes = (int64_t)512 << 20;

static void tune_smoother(DevLevel& l, bool mixed, int mode, hipStream_t s) {
  l.fused = false;
  l.oop = false;
  const int64_t es = mixed ? 4 : 8;
  float* flush = nullptr;
  if (mode == 0 && (l.N + l.N2) * (3 * es + 1) > kLLCBytes / 4) {
    // best effort: without the scratch the sweeps are timed back to back
    if (hipMalloc((void**)&flush, kFlushBytes) != hipSuccess) {
      flush = nullptr;
      (void)hipGetLastError();
    }
  }
  const int64_t nflush = kFlushBytes / (int64_t)sizeof(float);
  try {
    if (mixed) {
      if (l.xa32.p) tune_level<float>(l, l.x32.p, l.xa32.p, l.b32.p, mode, s, flush, nflush);
    } else {
      if (l.xa64.p) tune_level<double>(l, l.x64.p, l.xa64.p, l.b64.p, mode, s, flush, nflush);
    }
  } catch (...) {
    if (flush) {
      (void)hipStreamSynchronize(s);
      (void)hipFree(flush);
    }
    throw;
  }
  if (flush) {
    HIPCHECK(hipStreamSynchronize(s));
    HIPCHECK(hipFree(flush));
  }
}

// Device view of the Krylov bottom solve (hierarchies whose bottom level has
// no dense inverse); rebuilt when the level's template constants change.
static void upload_bottom_krylov(DevProblem& D, hipStream_t s) {
  DevLevel& B = D.lv.back();
  const int64_t n = B.N + B.N2;
  if (!D.bk_vec.p) D.bk_vec.alloc(8 * n, D.bytes);
  BBot k;
  std::memset(&k, 0, sizeof(k));
  k.L = make_blev<double>(B);
  for (int q = 0; q < 8; ++q) k.w[q] = D.bk_vec.p + q * n;
  k.maxit = (int)std::min<int64_t>(4000, std::max<int64_t>(200, 2 * n));
  k.tol = 1e-10;
  D.bytes -= D.bk_dev.n;
  D.bk_dev.release();
  D.bk_dev.upload((const uint8_t*)&k, (int64_t)sizeof(BBot), s, D.bytes);
  HIPCHECK(hipStreamSynchronize(s));
}

// Device order of a level's explicit rows: by colour group, and within
// windows of kSortWindow rows of a group by decreasing number of stored
// entries (host order among equals), so the 64-row slices of the sliced
// layout need little padding while a slice's rows stay near each other.
constexpr int64_t kSortWindow = 512;
static std::vector<int32_t> row_order(const Level& L) {
  const int64_t R = (int64_t)L.irow_dof.size();
  std::vector<int32_t> id;
  std::vector<int32_t> ptr;
  if ((int64_t)L.cls_rows.size() == R && L.cls_ptr.size() == 3) {
    id = L.cls_rows;
    ptr = L.cls_ptr;
  } else {
    id.resize(R);
    for (int64_t k = 0; k < R; ++k) id[k] = (int32_t)k;
    ptr = {0, (int32_t)R, (int32_t)R};
  }
  auto len = [&](int32_t r) { return L.rp[r + 1] - L.rp[r]; };
  for (int g = 0; g < 2; ++g)
    for (int64_t w0 = ptr[g]; w0 < ptr[g + 1]; w0 += kSortWindow)
      std::stable_sort(id.begin() + w0, id.begin() + std::min<int64_t>(ptr[g + 1], w0 + kSortWindow),
                       [&](int32_t a, int32_t b) { return len(a) > len(b); });
  return id;
}

// Sliced layout of the (device-ordered) explicit rows: each colour group is
// cut into slices of kSlice rows; entry j of the slice's rows is stored at
// sl_ptr[slice] + j * kSlice + (row within the slice), padded to the slice's
// longest row with column 0 and value 0. grp[g] is group g's first slice.
static void build_sliced(const std::vector<int64_t>& rp, const std::vector<int32_t>& col,
                         const std::vector<double>& val, const std::vector<int32_t>& gptr,
                         std::vector<int64_t>& sptr, std::vector<int32_t>& scol, std::vector<double>& sval,
                         int grp[3]) {
  sptr.assign(1, 0);
  scol.clear();
  sval.clear();
  for (int g = 0; g < 2; ++g) {
    grp[g] = (int)sptr.size() - 1;
    for (int64_t r0 = gptr[g]; r0 < gptr[g + 1]; r0 += kSlice) {
      const int64_t r1 = std::min<int64_t>(gptr[g + 1], r0 + kSlice);
      int64_t len = 0;
      for (int64_t r = r0; r < r1; ++r) len = std::max(len, rp[r + 1] - rp[r]);
      const int64_t base = sptr.back();
      scol.resize(base + len * kSlice, 0);
      sval.resize(base + len * kSlice, 0.0);
      for (int64_t r = r0; r < r1; ++r)
        for (int64_t j = 0; j < rp[r + 1] - rp[r]; ++j) {
          scol[base + j * kSlice + (r - r0)] = col[rp[r] + j];
          sval[base + j * kSlice + (r - r0)] = val[rp[r] + j];
        }
      sptr.push_back(base + len * kSlice);
    }
  }
  grp[2] = (int)sptr.size() - 1;
}

// Whether two levels (of family members on one geometry) have the same
// structure: cell tags, explicit rows and their columns, colour groups and
// transfer lists. Their device copies are then the same arrays.
static bool same_structure(const Level& a, const Level& b) {
  return a.g.dim == b.g.dim && a.g.n[0] == b.g.n[0] && a.g.n[1] == b.g.n[1] && a.g.n[2] == b.g.n[2] &&
         a.N == b.N && a.N2 == b.N2 && a.tag == b.tag && a.sec_cell == b.sec_cell && a.irow_dof == b.irow_dof &&
         a.rp == b.rp && a.col == b.col && a.cls_ptr == b.cls_ptr && a.cls_rows == b.cls_rows &&
         a.ns_cdof == b.ns_cdof && a.ns_ptr == b.ns_ptr && a.ns_child == b.ns_child && a.np_fdof == b.np_fdof &&
         a.np_cdof == b.np_cdof;
}

// Upload a problem's hierarchy. With `share` (a family member set up on the
// same geometry as `share`), every level whose structure equals share's
// takes share's device structure arrays instead of its own copies (the
// values, template constants, bottom inverse and vectors stay per problem),
// and the smoother and coarse-tail choices are share's (no timing).
static void upload(ebmg_problem_s* P, bool batch_box = false, const ebmg_problem_s* share = nullptr) {
  Problem& H = *P->host;
  DevProblem& D = P->dev;
  hipStream_t s = P->ctx->stream;
  int64_t& by = D.bytes;
  const bool mixed = H.opt.precision == EBMG_MIXED;
  D.lv.resize(H.levels.size());
  for (size_t l = 0; l < H.levels.size(); ++l) {
    const Level& L = H.levels[l];
    DevLevel& d = D.lv[l];
    d.dim = L.g.dim;
    for (int e = 0; e < 3; ++e) d.n[e] = L.g.n[e];
    d.N = L.N;
    d.N2 = L.N2;
    d.R = (int64_t)L.irow_dof.size();
    const DevLevel* sd = nullptr;   // the level whose structure arrays this one takes
    if (share && l < share->host->levels.size() && same_structure(L, share->host->levels[l]))
      sd = &share->dev.lv[l];
    if (sd)
      D.shared_bytes += d.tag.share(sd->tag);
    else
      d.tag.upload(L.tag.data(), L.N, s, by);
    // explicit rows are stored on the device group by group (red rows, then
    // black rows), so a colour group is a contiguous row range
    const std::vector<int32_t> perm = row_order(L);
    std::vector<int64_t> idof(d.R), rp(d.R + 1, 0);
    std::vector<int32_t> col, ident(d.R);
    std::vector<double> val, dg(d.R);
    col.reserve(L.col.size());
    val.reserve(L.val.size());
    // each row's entries in column order: neighbouring rows of a slice then
    // gather x at neighbouring addresses for the same entry position
    std::vector<std::pair<int32_t, double>> ent;
    for (int64_t k = 0; k < d.R; ++k) {
      const int32_t r = perm[k];
      idof[k] = L.irow_dof[r];
      dg[k] = L.idiag[r];
      ent.clear();
      for (int64_t e = L.rp[r]; e < L.rp[r + 1]; ++e) ent.emplace_back((int32_t)L.col[e], L.val[e]);
      std::stable_sort(ent.begin(), ent.end(),
                       [](const std::pair<int32_t, double>& a, const std::pair<int32_t, double>& b) {
                         return a.first < b.first;
                       });
      for (const auto& pe : ent) {
        col.push_back(pe.first);
        val.push_back(pe.second);
      }
      rp[k + 1] = (int64_t)col.size();
      ident[k] = (int32_t)k;
    }
    if (sd) {
      D.shared_bytes += d.irow_dof.share(sd->irow_dof) + d.rp.share(sd->rp) + d.col.share(sd->col) +
                        d.cls_rows.share(sd->cls_rows);
    } else {
      d.irow_dof.upload(idof.data(), d.R, s, by);
      d.rp.upload(rp.data(), d.R + 1, s, by);
      d.col.upload(col.data(), (int64_t)col.size(), s, by);
      d.cls_rows.upload(ident.data(), d.R, s, by);
    }
    d.cls_ptr = L.cls_ptr;
    d.val64.upload(val.data(), (int64_t)val.size(), s, by);
    d.diag64.upload(dg.data(), d.R, s, by);
    if (mixed) {
      std::vector<float> v(val.begin(), val.end()), g(dg.begin(), dg.end());
      d.val32.upload(v.data(), (int64_t)v.size(), s, by);
      d.diag32.upload(g.data(), (int64_t)g.size(), s, by);
    }
    {
      std::vector<int32_t> gptr = L.cls_ptr.size() == 3 ? L.cls_ptr : std::vector<int32_t>{0, (int32_t)d.R, (int32_t)d.R};
      std::vector<int64_t> sptr;
      std::vector<int32_t> scol;
      std::vector<double> sval;
      build_sliced(rp, col, val, gptr, sptr, scol, sval, d.sl_grp);
      if (sd) {
        D.shared_bytes += d.sl_ptr.share(sd->sl_ptr) + d.sl_col.share(sd->sl_col) + d.sl_colj.share(sd->sl_colj);
      } else {
        d.sl_ptr.upload(sptr.data(), (int64_t)sptr.size(), s, by);
        d.sl_col.upload(scol.data(), (int64_t)scol.size(), s, by);
      }
      // group 1's columns with every explicit-row unknown renamed into the
      // work array w that follows x: a group-0 unknown to N + N2 + (its
      // position in group 0), whose new value is in w[0, n0); a group-1
      // unknown to N + N2 + n0 + n1 + (its position in group 1), whose value
      // before the pass k_irr_jac_sl0c copies there. The pass over group 1
      // (k_irr_jac_sl2x) then reads no explicit-row unknown from x and can
      // write its results, and group 0's, straight into x.
      const int64_t nxv = L.N + L.N2;
      const int64_t n0g = gptr[1] - gptr[0], n1g = gptr[2] - gptr[1];
      if (!sd && L.cls_ptr.size() == 3 && n0g > 0 && n1g > 0 && nxv + n0g + 2 * n1g < (int64_t)INT32_MAX) {
        std::unordered_map<int64_t, int32_t> pos;
        pos.reserve((size_t)(n0g + n1g) * 2);
        for (int32_t k = gptr[0]; k < gptr[1]; ++k) pos.emplace(idof[k], (int32_t)(k - gptr[0]));
        for (int32_t k = gptr[1]; k < gptr[2]; ++k) pos.emplace(idof[k], (int32_t)(n0g + n1g + (k - gptr[1])));
        std::vector<int32_t> scolj(scol);
        for (int64_t e = sptr[d.sl_grp[1]]; e < sptr[d.sl_grp[2]]; ++e) {
          const auto it = pos.find(scolj[e]);
          if (it != pos.end()) scolj[e] = (int32_t)(nxv + it->second);
        }
        d.sl_colj.upload(scolj.data(), (int64_t)scolj.size(), s, by);
      }
      d.sl_val64.upload(sval.data(), (int64_t)sval.size(), s, by);
      if (mixed) {
        std::vector<float> v(sval.begin(), sval.end());
        d.sl_val32.upload(v.data(), (int64_t)v.size(), s, by);
      }
      HIPCHECK(hipStreamSynchronize(s));
    }
    HIPCHECK(hipStreamSynchronize(s));
    d.n_ns = (int64_t)L.ns_cdof.size();
    d.n_np = (int64_t)L.np_fdof.size();
    if (sd) {
      D.shared_bytes += d.ns_cdof.share(sd->ns_cdof) + d.ns_ptr.share(sd->ns_ptr) + d.ns_child.share(sd->ns_child) +
                        d.np_fdof.share(sd->np_fdof) + d.np_cdof.share(sd->np_cdof);
    } else {
      d.ns_cdof.upload(L.ns_cdof.data(), d.n_ns, s, by);
      d.ns_ptr.upload(L.ns_ptr.data(), (int64_t)L.ns_ptr.size(), s, by);
      d.ns_child.upload(L.ns_child.data(), (int64_t)L.ns_child.size(), s, by);
      d.np_fdof.upload(L.np_fdof.data(), d.n_np, s, by);
      d.np_cdof.upload(L.np_cdof.data(), d.n_np, s, by);
    }
    d.t64 = make_tmpl<double>(L);
    d.t32 = make_tmpl<float>(L);
    const int64_t nd = L.N + L.N2;
    // the work array holds the explicit rows' Jacobi values and, after them,
    // group 1's values before its pass (k_irr_jac_sl0c)
    const int64_t grp1_rows = L.cls_ptr.size() == 3 ? L.cls_ptr[2] - L.cls_ptr[1] : 0;
    if (!mixed || l == 0) {
      d.x64.alloc(nd, by);
      d.b64.alloc(nd, by);
      d.r64.alloc(nd, by);
      d.w64.alloc(std::max<int64_t>(1, d.R + grp1_rows), by);
      if (!batch_box) d.xa64.alloc(nd, by);
    }
    if (mixed) {
      d.x32.alloc(nd, by);
      d.b32.alloc(nd, by);
      d.r32.alloc(nd, by);
      d.w32.alloc(std::max<int64_t>(1, d.R + grp1_rows), by);
      if (!batch_box) d.xa32.alloc(nd, by);
    }
  }
  D.bottom_n = H.bottom_n;
  D.bottom.upload(H.bottom_inv.data(), (int64_t)H.bottom_inv.size(), s, by);
  if (D.bottom.n == 0) upload_bottom_krylov(D, s);
  // rhs data
  const FineData& F = H.fine;
  const Level& L0 = H.levels[0];
  const int64_t R = (int64_t)L0.irow_dof.size();
  const std::vector<int32_t> perm0 = row_order(L0);
  std::vector<int64_t> icell(R);
  std::vector<double> iface(6 * R), icobj(R), icsig(R), isrc(R);
  std::vector<int32_t> iobj(R);
  for (int64_t k = 0; k < R; ++k) {
    const int32_t r = perm0[k];
    const int64_t q = L0.irow_dof[r];
    icell[k] = q < L0.N ? q : L0.sec_cell[q - L0.N];
    for (int f = 0; f < 6; ++f) iface[6 * k + f] = F.idata[r].face[f];
    iobj[k] = F.idata[r].obj;
    icobj[k] = F.idata[r].cobj;
    icsig[k] = F.idata[r].csig;
    isrc[k] = F.isrc[r];
  }
  D.icell.upload(icell.data(), R, s, by);
  D.isrc.upload(isrc.data(), R, s, by);
  D.iface.upload(iface.data(), 6 * R, s, by);
  D.iobj.upload(iobj.data(), R, s, by);
  D.icobj.upload(icobj.data(), R, s, by);
  D.icsig.upload(icsig.data(), R, s, by);
  const int64_t NE = (int64_t)F.edata.size();
  std::vector<double> eface(6 * NE), ecobj(NE), ecsig(NE);
  std::vector<int32_t> eobj(NE);
  for (int64_t e = 0; e < NE; ++e) {
    for (int f = 0; f < 6; ++f) eface[6 * e + f] = F.edata[e].face[f];
    eobj[e] = F.edata[e].obj;
    ecobj[e] = F.edata[e].cobj;
    ecsig[e] = F.edata[e].csig;
  }
  D.ecell.upload(F.ecell.data(), (int64_t)F.ecell.size(), s, by);
  D.erp.upload(F.erp.data(), (int64_t)F.erp.size(), s, by);
  D.ecol.upload(F.ecol.data(), (int64_t)F.ecol.size(), s, by);
  D.eval.upload(F.eval.data(), (int64_t)F.eval.size(), s, by);
  D.eface.upload(eface.data(), 6 * NE, s, by);
  D.eobj.upload(eobj.data(), NE, s, by);
  D.ecobj.upload(ecobj.data(), NE, s, by);
  D.ecsig.upload(ecsig.data(), NE, s, by);
  D.objv.alloc(std::max<int64_t>(1, (int64_t)H.geo.obj_value.size()), by);
  D.part.alloc(std::max<int64_t>(2 * kNormBlocks, 2 * matvec_blocks(D.lv[0])), by);
  D.scal.alloc(SC_NUM, by);
  HIPCHECK(hipHostMalloc((void**)&D.host_scal, SC_NUM * sizeof(double), hipHostMallocDefault));
  D.krylov = H.opt.krylov == 2;
  if (batch_box) {
    // the in-group solver keeps its Krylov / correction vectors here
    for (auto& k : D.kv) k.alloc(L0.N + L0.N2, by);
    HIPCHECK(hipStreamSynchronize(s));
    return;
  }
  HIPCHECK(hipStreamSynchronize(s));
  if (share && share->dev.lv.size() == D.lv.size()) {
    // a family member: the kernel choices of the member it shares with
    for (size_t l = 0; l < D.lv.size(); ++l) {
      const DevLevel& o = share->dev.lv[l];
      DevLevel& d = D.lv[l];
      d.fused = o.fused;
      d.oop = o.oop;
      d.fvar = o.fvar;
      d.zmcfg = o.zmcfg;
      d.tune_split_ms = o.tune_split_ms;
      d.tune_fused_ms = o.tune_fused_ms;
      d.tune_zm_ms = o.tune_zm_ms;
      d.tune_oop_ms = o.tune_oop_ms;
      d.tune_zm_cfg_ms = o.tune_zm_cfg_ms;
    }
    if (mixed)
      upload_tail<float>(D, s);
    else
      upload_tail<double>(D, s);
    D.tail_l0 = share->dev.tail_l0;
    D.tail_cand = share->dev.tail_cand;
    D.tail_ms = share->dev.tail_ms;
  } else {
    for (auto& l : D.lv) tune_smoother(l, mixed, H.opt.smoother, s);
    if (mixed) {
      upload_tail<float>(D, s);
      refine_finest_zm<float>(D, H.opt, s);
      tune_tail<float>(D, H.opt, s);
    } else {
      upload_tail<double>(D, s);
      refine_finest_zm<double>(D, H.opt, s);
      tune_tail<double>(D, H.opt, s);
    }
  }
  if (D.krylov) {
    // FP64 ph and sh (slots 4 and 6) only without mixed precision
    for (int k = 0; k < 8; ++k)
      if (!(mixed && (k == 4 || k == 6))) D.kv[k].alloc(L0.N + L0.N2, by);
    if (mixed) {
      D.ph32.alloc(L0.N + L0.N2, by);
      D.sh32.alloc(L0.N + L0.N2, by);
    }
  }
  HIPCHECK(hipStreamSynchronize(s));
}

// ---------------------------------------------------------------------------
// cycle pieces
// ---------------------------------------------------------------------------
static inline unsigned nblk_sub(int64_t rows) { return nblk(rows * kSub); }

// One colour phase of the out-of-place sweep; with rows = false the explicit
// rows are only copied (template-cell sweeps).
template <typename T>
static void launch_oop(DevLevel& l, int colour, bool rows, const T* xin, T* xout, const T* b, hipStream_t s) {
  const Tmpl<T>& tp = Vec<T>::t(l);
  const size_t qa = 4 * sizeof(T);
  const bool quad = tp.n[0] % 4 == 0 && l.N < ((int64_t)1 << 31) && (uintptr_t)xin % qa == 0 &&
                    (uintptr_t)xout % qa == 0 && (uintptr_t)b % qa == 0 && (uintptr_t)l.tag.p % 4 == 0;
  const bool pair = !quad && tp.n[0] % 2 == 0;
  const unsigned nbc = nblk(quad ? l.N / 4 : pair ? l.N / 2 : l.N);
  int n0 = 0, n1 = 0;
  const int32_t* g0 = l.cls_rows.p;
  const int32_t* g1 = l.cls_rows.p;
  if (l.cls_ptr.size() >= 3) {
    n0 = l.cls_ptr[1] - l.cls_ptr[0];
    n1 = l.cls_ptr[2] - l.cls_ptr[1];
    g0 = l.cls_rows.p + l.cls_ptr[0];
    g1 = l.cls_rows.p + l.cls_ptr[1];
  }
  const int32_t* up = colour == 0 ? g0 : g1;
  const int32_t* cp = colour == 0 ? g1 : g0;
  int nup = colour == 0 ? n0 : n1;
  int ncp = colour == 0 ? n1 : n0;
  if (!rows) {
    // template cells only: copy every explicit row, update none
    const int32_t* all = l.cls_rows.p;
    cp = all;
    ncp = n0 + n1;
    up = all;
    nup = 0;
  }
  const unsigned nbu = nblk_sub(nup);
  const unsigned nbr = nbu + nblk(ncp);
#define OOP_LAUNCH(D, W)                                                                                     \
  KLAUNCH(l.kt, (k_rb_oop<T, D, W>), dim3(nbc + nbr), dim3(kBlock), 0, s, l.tag.p, xin, xout, b, tp, colour, nbc, \
          nbu, nbr, up, nup, cp, ncp, l.irow_dof.p, l.rp.p, l.col.p, Vec<T>::val(l), Vec<T>::diag(l))
  if (l.dim == 3) {
    if (quad) OOP_LAUNCH(3, 4); else if (pair) OOP_LAUNCH(3, 2); else OOP_LAUNCH(3, 1);
  } else {
    if (quad) OOP_LAUNCH(2, 4); else if (pair) OOP_LAUNCH(2, 2); else OOP_LAUNCH(2, 1);
  }
#undef OOP_LAUNCH
}

template <typename T>
static void irr_group(DevLevel& l, int grp, T* x, const T* b, hipStream_t s) {
  if (l.cls_ptr.size() < 3) return;
  const int nr = l.cls_ptr[grp + 1] - l.cls_ptr[grp];
  if (nr <= 0) return;
  const int32_t* rows = l.cls_rows.p + l.cls_ptr[grp];
  T* tmp = Vec<T>::tmp(l);
  if (l.sl_ptr.p && Vec<T>::sval(l))
    hipLaunchKernelGGL((k_irr_jac_sl<T>), dim3((unsigned)((nr + kSplitRows - 1) / kSplitRows)), dim3(kRowBlock), 0, s,
                       make_blev<T>(l), grp, x, b);
  else
    hipLaunchKernelGGL((k_irr_jacobi<T>), dim3(nblk_sub(nr)), dim3(kBlock), 0, s, rows, nr, l.irow_dof.p, l.rp.p,
                       l.col.p, Vec<T>::val(l), Vec<T>::diag(l), x, b, tmp);
  hipLaunchKernelGGL((k_irr_scatter<T>), dim3(nblk(nr)), dim3(kBlock), 0, s, rows, nr, l.irow_dof.p, tmp, x);
}

// xz: x is zero on entry (a V-cycle level's correction); used by the
// z-marching sweep, whose first sweep then does not read x
// Both groups' Jacobi passes with one scatter: group 0 into w[0, n0), group 1
// into w[n0, R) reading group 0's values from w, then every row into x
// (the same values as irr_group(0) then irr_group(1)).
template <typename T>
static void irr_groups(DevLevel& l, T* x, const T* b, hipStream_t s) {
  const int n0 = l.cls_ptr.size() == 3 ? l.cls_ptr[1] - l.cls_ptr[0] : 0;
  const int n1 = l.cls_ptr.size() == 3 ? l.cls_ptr[2] - l.cls_ptr[1] : 0;
  if (!l.sl_colj.p || !Vec<T>::sval(l) || n0 <= 0 || n1 <= 0) {
    irr_group<T>(l, 0, x, b, s);
    irr_group<T>(l, 1, x, b, s);
    return;
  }
  T* w = Vec<T>::tmp(l);
  const BLev<T> L0 = make_blev<T>(l);
  // group 0 into w[0, n0), with group 1's values copied to w[n0 + n1, ...);
  // then group 1 straight into x (its columns renamed into w) and group 0
  // copied from w into x: the same values as the two passes and a scatter
  const unsigned nb0 = (unsigned)((n0 + kSplitRows - 1) / kSplitRows);
  const unsigned nb1 = (unsigned)((n1 + kSplitRows - 1) / kSplitRows);
  hipLaunchKernelGGL((k_irr_jac_sl0c<T>), dim3(nb0 + (unsigned)((n1 + kRowBlock - 1) / kRowBlock)), dim3(kRowBlock),
                     0, s, L0, nb0, x, b, w + n0 + n1);
  BLev<T> L1 = L0;
  L1.sl_col = l.sl_colj.p;
  hipLaunchKernelGGL((k_irr_jac_sl2x<T>), dim3(nb1 + (unsigned)((n0 + kRowBlock - 1) / kRowBlock)), dim3(kRowBlock),
                     0, s, L1, nb1, x, b, (const T*)w, (int)(l.N + l.N2));
}

template <typename T>
static void smooth(DevLevel& l, T* x, const T* b, int sweeps, hipStream_t s, bool xz) {
  const Tmpl<T>& tp = Vec<T>::t(l);
  if (l.fused && Vec<T>::xa(l)) {
    // out-of-place fused red+black sweeps, then the explicit rows of red and
    // of black cells
    T* cur = x;
    T* alt = Vec<T>::xa(l);
    for (int it = 0; it < sweeps; ++it) {
      launch_fused<T>(l, cur, alt, b, tp, s, xz && it == 0);
      std::swap(cur, alt);
      irr_groups<T>(l, cur, b, s);
    }
    if (cur != x)
      hipLaunchKernelGGL((k_convert<T, T>), dim3(nblk(l.N + l.N2)), dim3(kBlock), 0, s, cur, x, l.N + l.N2);
    HIPCHECK(hipGetLastError());
    return;
  }
  if (l.oop && Vec<T>::xa(l)) {
    // one launch per colour phase, out of place (two per sweep)
    T* cur = x;
    T* alt = Vec<T>::xa(l);
    for (int it = 0; it < sweeps; ++it)
      for (int colour = 0; colour < 2; ++colour) {
        launch_oop<T>(l, colour, true, cur, alt, b, s);
        std::swap(cur, alt);
      }
    HIPCHECK(hipGetLastError());
    return;
  }
  const Shape sh = shape3((l.n[0] + 1) / 2, l.n[1], l.dim == 3 ? l.n[2] : 1);
  for (int it = 0; it < sweeps; ++it) {
    for (int colour = 0; colour < 2; ++colour) {
      if (l.dim == 3)
        KLAUNCH(l.kt, (k_rb<T, 3>), sh.g, sh.b, 0, s, l.tag.p, x, b, tp, colour);
      else
        KLAUNCH(l.kt, (k_rb<T, 2>), sh.g, sh.b, 0, s, l.tag.p, x, b, tp, colour);
      irr_group<T>(l, colour, x, b, s);
    }
  }
  HIPCHECK(hipGetLastError());
}

// Explicit rows of r = b - A x (MODE 0) or A x (MODE 1) on a large level.
template <typename T, int MODE>
static void residual_rows(DevLevel& l, const T* x, const T* b, T* r, hipStream_t s) {
  if (l.R > 0 && l.sl_ptr.p && Vec<T>::sval(l)) {
    const BLev<T> L = make_blev<T>(l);
    const int nb0 = (L.grp_ptr[1] - L.grp_ptr[0] + kSplitRows - 1) / kSplitRows;
    const int nb1 = (L.grp_ptr[2] - L.grp_ptr[1] + kSplitRows - 1) / kSplitRows;
    hipLaunchKernelGGL((k_resid_irr_sl<T, MODE>), dim3((unsigned)(nb0 + nb1)), dim3(kRowBlock), 0, s, L, nb0, x, b, r);
  } else if (l.R > 0) {
    hipLaunchKernelGGL((k_resid_irr<T, MODE>), dim3(nblk_sub(l.R)), dim3(kBlock), 0, s, (int)l.R, l.irow_dof.p,
                       l.rp.p, l.col.p, Vec<T>::val(l), Vec<T>::diag(l), x, b, r);
  }
}

template <typename T, int MODE>
static void residual(DevLevel& l, const T* x, const T* b, T* r, hipStream_t s) {
  const Tmpl<T>& tp = Vec<T>::t(l);
  if (l.dim == 3 && l.N >= kResidZMMin) {
    KTiming* kr = (sizeof(T) == 8 && MODE == 0) ? l.ktr : nullptr;
    if (sizeof(T) == 8 && pair_ok(l) && al2(x) && al2(b) && al2(r))
      KLAUNCH(kr, (k_resid_zp3<T, MODE>), dim3((unsigned)zp_resid_blocks(l)), dim3(64, kRPY), 0, s, l.tag.p, x, b, r,
              tp, (const T*)nullptr, (double*)nullptr, (int64_t)0);
    else
      KLAUNCH(kr, (k_resid_zm3<T, MODE>), dim3((unsigned)zm_resid_blocks(l)), dim3(kRZX, kRZY), 0, s, l.tag.p, x, b,
              r, tp, (const T*)nullptr, (double*)nullptr, (int64_t)0);
    residual_rows<T, MODE>(l, x, b, r, s);
  } else {
    // small levels: template cells and explicit rows in one launch
    const unsigned nbc = nblk(l.N);
    const dim3 g(nbc + nblk_sub(l.R));
    if (l.dim == 3)
      hipLaunchKernelGGL((k_resid_all<T, 3, MODE>), g, dim3(kBlock), 0, s, l.tag.p, x, b, r, tp, nbc, (int)l.R,
                         l.irow_dof.p, l.rp.p, l.col.p, Vec<T>::val(l), Vec<T>::diag(l));
    else
      hipLaunchKernelGGL((k_resid_all<T, 2, MODE>), g, dim3(kBlock), 0, s, l.tag.p, x, b, r, tp, nbc, (int)l.R,
                         l.irow_dof.p, l.rp.p, l.col.p, Vec<T>::val(l), Vec<T>::diag(l));
  }
  HIPCHECK(hipGetLastError());
}

// restriction of rf into the coarse right-hand side bc, clearing the coarse
// correction xc, in one launch
template <typename T>
static void restrict_to(DevLevel& f, DevLevel& c, const T* rf, T* bc, T* xc, hipStream_t s) {
  const unsigned nbc = nblk(c.N), nbn = nblk(f.n_ns);
  const int64_t ncd = c.N + c.N2;
  const dim3 g(nbc + nbn + nblk(ncd));
  if (f.dim == 3)
    hipLaunchKernelGGL((k_restrict_all<T, 3>), g, dim3(kBlock), 0, s, c.tag.p, rf, bc, xc, c.n[0], c.n[1], c.n[2],
                       nbc, nbn, (int)f.n_ns, f.ns_cdof.p, f.ns_ptr.p, f.ns_child.p, ncd);
  else
    hipLaunchKernelGGL((k_restrict_all<T, 2>), g, dim3(kBlock), 0, s, c.tag.p, rf, bc, xc, c.n[0], c.n[1], 1, nbc,
                       nbn, (int)f.n_ns, f.ns_cdof.p, f.ns_ptr.p, f.ns_child.p, ncd);
  HIPCHECK(hipGetLastError());
}

// The V-cycle's residual of level f restricted into level c's b, clearing c's
// x: on large 3D levels one kernel restricts the residual straight into the
// simple coarse cells (r is kept only for the children of the non-simple
// coarse unknowns, whose lists are restricted next, with the clear);
// elsewhere r is formed and restricted as separate steps. The same values
// either way.
// form (measurement hook only): 0 the solver's choice, 1 the fused pair
// kernel, 2 separate residual and restriction kernels (ArgError where a
// form does not apply)
template <typename T>
static void residual_restrict(DevLevel& f, DevLevel& c, const T* x, const T* b, hipStream_t s, int form = 0) {
  T* r = Vec<T>::r(f);
  const bool fuse = f.dim == 3 && f.N >= kResidZMMin && f.n[0] % 2 == 0 && f.n[1] % 2 == 0 && f.n[2] % 2 == 0 &&
                    c.n[0] * 2 == f.n[0] && c.n[1] * 2 == f.n[1] && c.n[2] * 2 == f.n[2];
  if (form == 1 && !fuse) throw ArgError("this level has no fused residual restriction");
  if (!fuse || form == 2) {
    residual<T, 0>(f, x, b, r, s);
    restrict_to<T>(f, c, r, Vec<T>::b(c), Vec<T>::x(c), s);
    return;
  }
  residual_rows<T, 0>(f, x, b, r, s);   // the explicit rows' r, read by the fused kernel
  // quad form where x extents and alignment allow (the same values)
  auto al4 = [](const void* p, size_t es) { return (uintptr_t)p % (4 * es) == 0; };
  const bool quad = form == 0 && f.n[0] % 4 == 0 && al4(x, sizeof(T)) && al4(b, sizeof(T)) && al4(r, sizeof(T)) &&
                    al4(f.tag.p, 1) && ((uintptr_t)c.tag.p % 2) == 0;
  // planes per thread: kRRZ, halved (staying even) until the grid has 2048
  // workgroups, eight per CU
  const int64_t ncol =
      (int64_t)((f.n[0] + (quad ? kRQX : kRRX) - 1) / (quad ? kRQX : kRRX)) * ((f.n[1] + 2 * kRRW - 1) / (2 * kRRW));
  int zc = kRRZ;
  while (zc > 2 && ncol * ((f.n[2] + zc - 1) / zc) < 2048) zc /= 2;
  const int64_t nb = ncol * ((f.n[2] + zc - 1) / zc);
  if (quad)
    hipLaunchKernelGGL((k_resid_restrict3q<T>), dim3((unsigned)nb), dim3(64, kRRW), 0, s, f.tag.p, x, b, r, c.tag.p,
                       Vec<T>::b(c), Vec<T>::t(f), zc);
  else
    hipLaunchKernelGGL((k_resid_restrict3<T>), dim3((unsigned)nb), dim3(64, kRRW), 0, s, f.tag.p, x, b, r, c.tag.p,
                       Vec<T>::b(c), Vec<T>::t(f), zc);
  const unsigned nbn = nblk(f.n_ns);
  const int64_t ncd = c.N + c.N2;
  hipLaunchKernelGGL((k_restrict_all<T, 3>), dim3(nbn + nblk(ncd)), dim3(kBlock), 0, s, c.tag.p, r, Vec<T>::b(c),
                     Vec<T>::x(c), c.n[0], c.n[1], c.n[2], 0u, nbn, (int)f.n_ns, f.ns_cdof.p, f.ns_ptr.p, f.ns_child.p,
                     ncd);
  HIPCHECK(hipGetLastError());
}

template <typename T>
static void prolong_from(DevLevel& f, DevLevel& c, const T* ec, T* xf, hipStream_t s) {
  const int64_t rows = (int64_t)f.n[1] * (f.dim == 3 ? f.n[2] : 1);
  if (f.n[0] % 4 == 0 && (uintptr_t)xf % (4 * sizeof(T)) == 0 && al2(ec) && (uintptr_t)f.tag.p % 4 == 0 &&
      (uintptr_t)c.tag.p % 2 == 0) {
    // four fine cells per lane: (bx, by) blocks, bx lanes along x, by rows
    const int q = f.n[0] / 4;
    int bx = 64;
    while (bx > 16 && bx / 2 >= q) bx /= 2;
    const int by = kBlock / bx;
    const unsigned nrb = (unsigned)((rows + by - 1) / by);
    const dim3 g(nrb + nblk(f.n_np), (unsigned)((q + bx - 1) / bx));
    if (f.dim == 3)
      hipLaunchKernelGGL((k_prolong_q<T, 3>), g, dim3(bx, by), 0, s, f.tag.p, c.tag.p, ec, xf, f.n[0], f.n[1],
                         f.n[2], nrb, (int)f.n_np, f.np_fdof.p, f.np_cdof.p);
    else
      hipLaunchKernelGGL((k_prolong_q<T, 2>), g, dim3(bx, by), 0, s, f.tag.p, c.tag.p, ec, xf, f.n[0], f.n[1], 1,
                         nrb, (int)f.n_np, f.np_fdof.p, f.np_cdof.p);
    HIPCHECK(hipGetLastError());
    return;
  }
  // (bx, by) blocks: bx cells along x (a power of two up to kBlock), by rows
  int bx = kBlock;
  while (bx > 16 && bx / 2 >= f.n[0]) bx /= 2;
  const int by = kBlock / bx;
  const unsigned nrb = (unsigned)((rows + by - 1) / by);
  const dim3 g(nrb + nblk(f.n_np), (unsigned)((f.n[0] + bx - 1) / bx));
  if (f.dim == 3)
    hipLaunchKernelGGL((k_prolong_all<T, 3>), g, dim3(bx, by), 0, s, f.tag.p, c.tag.p, ec, xf, f.n[0], f.n[1],
                       f.n[2], nrb, (int)f.n_np, f.np_fdof.p, f.np_cdof.p);
  else
    hipLaunchKernelGGL((k_prolong_all<T, 2>), g, dim3(bx, by), 0, s, f.tag.p, c.tag.p, ec, xf, f.n[0], f.n[1], 1,
                       nrb, (int)f.n_np, f.np_fdof.p, f.np_cdof.p);
  HIPCHECK(hipGetLastError());
}


template <typename T>
// xz: x holds zeros on entry (lets the first z-marching sweep skip reading it)
static void vcycle(DevProblem& D, const Options& o, size_t l, hipStream_t s, T* x, const T* b, bool xz) {
  DevLevel& L = D.lv[l];
  if ((int)l == D.tail_l0) {
    const BLev<T>* lv = (const BLev<T>*)D.tail_lv.p;
    if (L.dim == 3)
      hipLaunchKernelGGL((k_tail_vcycle<T, 3>), dim3(1), dim3(kBE), 0, s, lv, (int)l, (int)D.lv.size(),
                         D.bottom.n > 0 ? D.bottom.p : nullptr, (int)D.bottom_n, (const BBot*)D.bk_dev.p, o.nu1,
                         o.nu2, x, b);
    else
      hipLaunchKernelGGL((k_tail_vcycle<T, 2>), dim3(1), dim3(kBE), 0, s, lv, (int)l, (int)D.lv.size(),
                         D.bottom.n > 0 ? D.bottom.p : nullptr, (int)D.bottom_n, (const BBot*)D.bk_dev.p, o.nu1,
                         o.nu2, x, b);
    HIPCHECK(hipGetLastError());
    return;
  }
  if (l + 1 == D.lv.size()) {
    if (D.bottom.n > 0) {
      hipLaunchKernelGGL((k_bottom<T>), dim3((unsigned)D.bottom_n), dim3(64), 0, s, D.bottom.p, b, x,
                         (int)D.bottom_n);
      HIPCHECK(hipGetLastError());
    } else if (L.dim == 3) {
      hipLaunchKernelGGL((k_bottom_krylov<T, 3>), dim3(1), dim3(kBE), 0, s, (const BBot*)D.bk_dev.p, b, x);
      HIPCHECK(hipGetLastError());
    } else {
      hipLaunchKernelGGL((k_bottom_krylov<T, 2>), dim3(1), dim3(kBE), 0, s, (const BBot*)D.bk_dev.p, b, x);
      HIPCHECK(hipGetLastError());
    }
    return;
  }
  DevLevel& C = D.lv[l + 1];
  smooth<T>(L, x, b, o.nu1, s, xz);
  residual_restrict<T>(L, C, x, b, s);   // also clears the coarse x
  vcycle<T>(D, o, l + 1, s, Vec<T>::x(C), Vec<T>::b(C), true);
  prolong_from<T>(L, C, Vec<T>::x(C), x, s);
  smooth<T>(L, x, b, o.nu2, s);
}

// preconditioner z = M r: one V-cycle from zero (FP64, or FP32 with the
// input rounded to FP32 and the output widened to FP64)
static void precond(DevProblem& D, const Options& o, const double* r, double* z, hipStream_t s) {
  DevLevel& L = D.lv[0];
  const int64_t nd = L.N + L.N2;
  if (o.precision == EBMG_MIXED) {
    hipLaunchKernelGGL((k_convert<double, float>), dim3(nblk(nd)), dim3(kBlock), 0, s, r, L.b32.p, nd);
    fill<float>(L.x32.p, nd, 0.0f, s);
    vcycle<float>(D, o, 0, s, L.x32.p, L.b32.p);
    hipLaunchKernelGGL((k_convert<float, double>), dim3(nblk(nd)), dim3(kBlock), 0, s, L.x32.p, z, nd);
  } else {
    fill<double>(z, nd, 0.0, s);
    vcycle<double>(D, o, 0, s, z, r);
  }
  HIPCHECK(hipGetLastError());
}

// Algorithmic device-memory bytes (each kernel's minimum reads and writes)
// of the solve's steps, for ebmg_solve_info.est_bytes. Per unknown of a
// level with values of vsz bytes: a template sweep reads x, b and the tag
// and writes x; explicit rows read per stored entry a column index and a
// value and per row its unknown index, b and diagonal, and write x; the
// V-cycle residual restricted into the coarse b reads x, b and the tag and
// writes the coarse b; prolongation reads the coarse correction, x and the
// tag and writes x; the dense bottom inverse is read once per application.
static double rows_bytes(const DevLevel& l, int vsz) {
  return (double)l.R * (8.0 + 3.0 * vsz) + (double)l.col.n * (4.0 + vsz);
}

static double vcycle_bytes(const DevProblem& D, const Options& o, int vsz) {
  double by = 0;
  for (size_t l = 0; l < D.lv.size(); ++l) {
    const DevLevel& L = D.lv[l];
    const double n = (double)(L.N + L.N2);
    if (l + 1 == D.lv.size()) {
      by += D.bottom_n > 0 ? (double)D.bottom_n * D.bottom_n * 8.0 + 2.0 * D.bottom_n * vsz : 3.0 * n * vsz;
      break;
    }
    const DevLevel& C = D.lv[l + 1];
    const double sweeps = o.nu1 + o.nu2;
    by += sweeps * ((double)L.N * (3.0 * vsz + 1.0) + rows_bytes(L, vsz));
    by += (double)L.N * (2.0 * vsz + 1.0) + rows_bytes(L, vsz) + (double)(C.N + C.N2) * vsz;   // residual, restriction
    by += (double)(C.N + C.N2) * vsz + n * 2.0 * vsz + (double)L.N;                                // prolongation
  }
  return by;
}

// per outer iteration, besides its V-cycles: BiCGStab's vector steps and its
// two FP64 matrix-vector products (with their dot products), or a refinement
// cycle's conversions, correction and FP64 residual with its norm
static double iteration_bytes(const DevProblem& D, const Options& o) {
  const DevLevel& L = D.lv[0];
  const double n = (double)(L.N + L.N2);
  const bool mixed = o.precision == EBMG_MIXED;
  const double zs = mixed ? 4.0 : 8.0;
  const double mv = (double)L.N * 1.0 + n * (zs + 16.0) + rows_bytes(L, 8);
  if (D.krylov)
    return n * (32.0 + 24.0 + 56.0 + 2.0 * zs + (mixed ? 8.0 : 0.0)) + 2.0 * mv;
  return n * (mixed ? 12.0 + 4.0 + 20.0 : 0.0) + (double)L.N * 25.0 + rows_bytes(L, 8) + n * 8.0;
}

// estimated bytes of one box of a batched solve: its cycles and outer
// iterations as for a single solve, plus its right-hand side and residuals
static int64_t box_bytes(ebmg_problem_s* P, int cycles, int iters) {
  const DevProblem& D = P->dev;
  const DevLevel& L = D.lv[0];
  const Options& o = P->host->opt;
  const double n = (double)(L.N + L.N2);
  double by = (double)L.N * 17.0 + rows_bytes(L, 8) + 2.0 * ((double)L.N * 25.0 + rows_bytes(L, 8) + n * 8.0);
  by += cycles * vcycle_bytes(D, o, o.precision == EBMG_MIXED ? 4 : 8);
  by += (D.krylov ? iters : cycles) * iteration_bytes(D, o);
  return (int64_t)by;
}

// deterministic dot product into device scalar slot `slot`
template <typename T>
static void dot_dev(DevProblem& D, const T* a, const T* b, int64_t n, int slot, hipStream_t s) {
  hipLaunchKernelGGL((k_dot_partial<T>), dim3(kNormBlocks), dim3(kBlock), 0, s, a, b, n, D.part.p);
  hipLaunchKernelGGL(k_dot_final, dim3(1), dim3(kBlock), 0, s, D.part.p, kNormBlocks, 1, D.scal.p + slot);
  HIPCHECK(hipGetLastError());
}

// Run body(stream) as a HIP graph on s: captured once on a private stream
// (default priority) into exec, then replayed. The captured work holds only
// kernel launches (no memset or copy nodes).
template <typename F>
static void graph_run(hipGraphExec_t& exec, hipStream_t s, F&& body) {
  if (!exec) {
    hipStream_t cs = nullptr;
    HIPCHECK(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
    hipGraph_t g = nullptr;
    try {
      HIPCHECK(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
      body(cs);
      HIPCHECK(hipStreamEndCapture(cs, &g));
      HIPCHECK(hipGraphInstantiate(&exec, g, nullptr, nullptr, 0));
    } catch (...) {
      hipGraph_t junk = nullptr;
      hipStreamCaptureStatus cst = hipStreamCaptureStatusNone;
      if (hipStreamIsCapturing(cs, &cst) == hipSuccess && cst != hipStreamCaptureStatusNone)
        (void)hipStreamEndCapture(cs, &junk);
      if (junk) (void)hipGraphDestroy(junk);
      if (g) (void)hipGraphDestroy(g);
      (void)hipStreamDestroy(cs);
      exec = nullptr;
      throw;
    }
    (void)hipGraphDestroy(g);
    (void)hipStreamDestroy(cs);
  }
  HIPCHECK(hipGraphLaunch(exec, s));
}

static void fetch_scalars(DevProblem& D, hipStream_t s) {
  HIPCHECK(hipMemcpyAsync(D.host_scal, D.scal.p, SC_NUM * sizeof(double), hipMemcpyDeviceToHost, s));
  HIPCHECK(hipStreamSynchronize(s));
}

template <typename T>
static double norm2(DevProblem& D, const T* r, int64_t n, hipStream_t s) {
  dot_dev<T>(D, r, r, n, SC_RR, s);
  fetch_scalars(D, s);
  return std::sqrt(D.host_scal[SC_RR]);
}

static void rhs(ebmg_problem_s* P, const double* rho, const double* sigma, const double* bcv, const double* objv) {
  Problem& H = *P->host;
  DevProblem& D = P->dev;
  DevLevel& L = D.lv[0];
  hipStream_t s = P->ctx->stream;
  FaceVals fv;
  for (int f = 0; f < 6; ++f) fv.v[f] = bcv ? bcv[f] : H.bc.value[f];
  const size_t no = H.geo.obj_value.size();
  std::vector<double> ov(std::max<size_t>(1, no), 0.0);
  for (size_t k = 0; k < no; ++k) ov[k] = objv ? objv[k] : H.geo.obj_value[k];
  HIPCHECK(hipMemcpyAsync(D.objv.p, ov.data(), sizeof(double) * ov.size(), hipMemcpyHostToDevice, s));
  Tmpl<double> dat;
  for (int d = 0; d < 3; ++d) dat.n[d] = L.n[d];
  for (int f = 0; f < 6; ++f)
    for (int p = 0; p < 2; ++p) dat.cb[f][p] = H.fine.dat[f][p] * fv.v[f];
  const Shape sh = shape3(L.n[0], L.n[1], L.dim == 3 ? L.n[2] : 1);
  if (L.dim == 3)
    hipLaunchKernelGGL((k_rhs_reg<3>), sh.g, sh.b, 0, s, L.tag.p, rho, L.b64.p, dat, 0);
  else
    hipLaunchKernelGGL((k_rhs_reg<2>), sh.g, sh.b, 0, s, L.tag.p, rho, L.b64.p, dat, 0);
  if (L.R > 0)
    hipLaunchKernelGGL(k_rhs_irr, dim3(nblk(L.R)), dim3(kBlock), 0, s, (int)L.R, L.irow_dof.p, D.icell.p, D.isrc.p,
                       D.iface.p, D.iobj.p, D.icobj.p, D.icsig.p, rho, sigma, D.objv.p, fv, L.b64.p);
  HIPCHECK(hipGetLastError());
  // the host copy of ov must outlive the async copy
  HIPCHECK(hipStreamSynchronize(s));
}

static void efield(ebmg_problem_s* P, const double* x, const double* sigma, const double* bcv, double* E) {
  Problem& H = *P->host;
  DevProblem& D = P->dev;
  DevLevel& L = D.lv[0];
  hipStream_t s = P->ctx->stream;
  FaceVals fv;
  for (int f = 0; f < 6; ++f) fv.v[f] = bcv ? bcv[f] : H.bc.value[f];
  Tmpl<double> ga, gb;
  for (int d = 0; d < 3; ++d) ga.n[d] = gb.n[d] = L.n[d];
  for (int f = 0; f < 6; ++f)
    for (int p = 0; p < 2; ++p) {
      ga.cb[f][p] = H.fine.ega[f][p];
      gb.cb[f][p] = H.fine.egb[f][p] * fv.v[f];
    }
  const double ih = 1.0 / H.levels[0].g.h;
  const Shape sh = shape3(L.n[0], L.n[1], L.dim == 3 ? L.n[2] : 1);
  if (L.dim == 3 && L.N >= kResidZMMin)
    hipLaunchKernelGGL(k_efield_zm3,
                       dim3((unsigned)((L.n[0] + kEZX - 1) / kEZX), (unsigned)((L.n[1] + kEZY - 1) / kEZY),
                            (unsigned)((L.n[2] + kEZ - 1) / kEZ)),
                       dim3(kEZX, kEZY), 0, s, L.tag.p, x, E, ga, gb, ih);
  else if (L.dim == 3)
    hipLaunchKernelGGL((k_efield_reg<3>), sh.g, sh.b, 0, s, L.tag.p, x, E, ga, gb, ih);
  else
    hipLaunchKernelGGL((k_efield_reg<2>), sh.g, sh.b, 0, s, L.tag.p, x, E, ga, gb, ih);
  const int nc = (int)H.fine.ecell.size();
  if (nc > 0)
    hipLaunchKernelGGL(k_efield_irr, dim3(nblk((int64_t)nc * L.dim)), dim3(kBlock), 0, s, nc, L.dim, L.N, D.ecell.p,
                       D.erp.p, D.ecol.p, D.eval.p, D.eface.p, D.eobj.p, D.ecobj.p, D.ecsig.p, x, sigma, D.objv.p,
                       fv, E);
  HIPCHECK(hipGetLastError());
}

// Right-preconditioned BiCGStab with the V-cycle as preconditioner; all
// scalars stay on the device, one host synchronisation per iteration for the
// convergence test. On entry L.x64 holds phi, L.r64 the residual b - A phi.
// out = A x on level 0 (x of type Z, widened exactly), with the dot products
// (da, out) and, for ndot = 2, (out, out) into device slots slot, slot + 1,
// from per-block partials of the same launches
template <typename Z>
static void matvec_dots(DevProblem& D, const Z* x, double* out, const double* da, int ndot, int slot, hipStream_t s) {
  DevLevel& l = D.lv[0];
  const Tmpl<double>& tp = l.t64;
  int64_t pt = matvec_blocks(l);
  if (l.dim == 3 && l.N >= kResidZMMin) {
    const bool pair = pair_ok(l) && al2(x) && al2(out) && al2(da);
    const dim3 g((unsigned)(pair ? zp_resid_blocks(l) : zm_resid_blocks(l)));
    const int64_t G = (int64_t)g.x;
    // explicit rows: the sliced copy (one thread per row) where there is one
    const bool sl = l.R > 0 && l.sl_ptr.p;
    int nb0 = 0, nb1 = 0;
    if (sl) {
      nb0 = (l.cls_ptr.size() == 3 ? l.cls_ptr[1] - l.cls_ptr[0] : (int)l.R);
      nb1 = (l.cls_ptr.size() == 3 ? l.cls_ptr[2] - l.cls_ptr[1] : 0);
      nb0 = (nb0 + kSplitRows - 1) / kSplitRows;
      nb1 = (nb1 + kSplitRows - 1) / kSplitRows;
    }
    pt = G + (sl ? (int64_t)(nb0 + nb1) : (int64_t)nblk(l.R * kSub));
    if ((int64_t)ndot * pt > D.part.n) throw DeviceError("matrix-vector partials exceed their buffer");
    if (pair) {
      if (ndot == 1)
        hipLaunchKernelGGL((k_resid_zp3<double, 1, Z, 1>), g, dim3(64, kRPY), 0, s, l.tag.p, x, nullptr, out, tp, da,
                           D.part.p, pt);
      else
        hipLaunchKernelGGL((k_resid_zp3<double, 1, Z, 2>), g, dim3(64, kRPY), 0, s, l.tag.p, x, nullptr, out, tp, da,
                           D.part.p, pt);
    } else if (ndot == 1) {
      hipLaunchKernelGGL((k_resid_zm3<double, 1, Z, 1>), g, dim3(kRZX, kRZY), 0, s, l.tag.p, x, nullptr, out, tp, da,
                         D.part.p, pt);
    } else {
      hipLaunchKernelGGL((k_resid_zm3<double, 1, Z, 2>), g, dim3(kRZX, kRZY), 0, s, l.tag.p, x, nullptr, out, tp, da,
                         D.part.p, pt);
    }
    if (sl) {
      const BLev<double> L = make_blev<double>(l);
      if (ndot == 1)
        hipLaunchKernelGGL((k_resid_irr_sl<double, 1, Z, 1>), dim3((unsigned)(nb0 + nb1)), dim3(kRowBlock), 0, s, L, nb0,
                           x, nullptr, out, da, D.part.p, pt, G);
      else
        hipLaunchKernelGGL((k_resid_irr_sl<double, 1, Z, 2>), dim3((unsigned)(nb0 + nb1)), dim3(kRowBlock), 0, s, L, nb0,
                           x, nullptr, out, da, D.part.p, pt, G);
    } else if (l.R > 0) {
      if (ndot == 1)
        hipLaunchKernelGGL((k_resid_irr<double, 1, Z, 1>), dim3(nblk_sub(l.R)), dim3(kBlock), 0, s, (int)l.R,
                           l.irow_dof.p, l.rp.p, l.col.p, l.val64.p, l.diag64.p, x, nullptr, out, da, D.part.p, pt,
                           G);
      else
        hipLaunchKernelGGL((k_resid_irr<double, 1, Z, 2>), dim3(nblk_sub(l.R)), dim3(kBlock), 0, s, (int)l.R,
                           l.irow_dof.p, l.rp.p, l.col.p, l.val64.p, l.diag64.p, x, nullptr, out, da, D.part.p, pt,
                           G);
    }
  } else {
    const unsigned nbc = nblk(l.N);
    const dim3 g(nbc + nblk_sub(l.R));
#define MV_ALL(DIM, ND)                                                                                           \
  hipLaunchKernelGGL((k_resid_all<double, DIM, 1, Z, ND>), g, dim3(kBlock), 0, s, l.tag.p, x, nullptr, out, tp,   \
                     nbc, (int)l.R, l.irow_dof.p, l.rp.p, l.col.p, l.val64.p, l.diag64.p, da, D.part.p, pt)
    if (l.dim == 3) {
      if (ndot == 1) MV_ALL(3, 1); else MV_ALL(3, 2);
    } else {
      if (ndot == 1) MV_ALL(2, 1); else MV_ALL(2, 2);
    }
#undef MV_ALL
  }
  hipLaunchKernelGGL(k_dot_final, dim3(1), dim3(kBlock), 0, s, D.part.p, (int)pt, ndot, D.scal.p + slot);
  HIPCHECK(hipGetLastError());
}

// V-cycle-preconditioned BiCGStab (right preconditioning) with the vector
// steps fused: each iteration is p-update, V-cycle, A ph with (rh, v),
// s-update, V-cycle, A sh with (s, t) and (t, t), then the x/r update with
// (rh, r) and (r, r) for the next iteration; one host sync per iteration.
// Z is the preconditioner output type (FP32 for mixed precision).
template <typename Z>
static ebmg_status bicgstab_t(DevProblem& D, const Options& o, double bn, double rtol, int max_cycles, double& rel,
                              int& cyc, ebmg_solve_info& info, Z* ph, Z* sh, hipStream_t s, const double* r0) {
  DevLevel& L = D.lv[0];
  const int64_t nd = L.N + L.N2;
  const bool mixed = o.precision == EBMG_MIXED;
  double *r = D.kv[0].p, *rh = D.kv[1].p, *p = D.kv[2].p, *v = D.kv[3].p;
  double *sv = D.kv[5].p, *t = D.kv[7].p;
  double* x = L.x64.p;
  float* bf = mixed ? L.b32.p : nullptr;
  const unsigned nb = nblk(nd);
  // r0: the initial residual (the solve's r, or b for a zero guess); a
  // restart after a breakdown starts from the true residual in r64
  // (rh, r) = (b, b) when the start is from b: the solve has just formed
  // that sum in SC_RR with the same reduction, so it is copied
  auto restart = [&](const double* r0src, bool rr_is_r0r0) {
    hipLaunchKernelGGL(k_bicg_restart, dim3(nb), dim3(kBlock), 0, s, r0src, r, rh, nd);
    hipLaunchKernelGGL(k_sc_reset, dim3(1), dim3(1), 0, s, D.scal.p);
    if (rr_is_r0r0)
      hipLaunchKernelGGL(k_sc_copy, dim3(1), dim3(1), 0, s, D.scal.p, (int)SC_RHO, (int)SC_RR);
    else
      dot_dev<double>(D, rh, r, nd, SC_RHO, s);
  };
  // the preconditioner output starts from zero: cleared by the p- and
  // s-updates, unless the finest level's first sweep is the z-marching one,
  // which then takes x = 0 without reading it
  const bool zin = L.dim == 3 && L.fused && L.fvar == 1 && Vec<Z>::xa(L) && D.tail_l0 != 0 && o.nu1 > 0;
  auto vcyc = [&](Z* z, const double* in, hipStream_t q) {
    if constexpr (std::is_same<Z, float>::value) {
      (void)in;
      vcycle<float>(D, o, 0, q, z, L.b32.p, zin);
    } else {
      vcycle<double>(D, o, 0, q, z, in, zin);
    }
  };
  // one iteration: p-update, V-cycle, A ph, s-update, V-cycle, A sh, x/r update
  auto iteration = [&](hipStream_t q) {
    hipLaunchKernelGGL((k_bicg_p2<Z>), dim3(nb), dim3(kBlock), 0, q, p, r, v, D.scal.p, nd, bf, zin ? nullptr : ph);
    vcyc(ph, p, q);
    matvec_dots<Z>(D, ph, v, rh, 1, SC_RV, q);
    hipLaunchKernelGGL(k_sc_alpha, dim3(1), dim3(1), 0, q, D.scal.p);
    hipLaunchKernelGGL((k_bicg_s2<Z>), dim3(nb), dim3(kBlock), 0, q, sv, r, v, D.scal.p, nd, bf, zin ? nullptr : sh);
    vcyc(sh, sv, q);
    matvec_dots<Z>(D, sh, t, sv, 2, SC_TS, q);
    hipLaunchKernelGGL(k_sc_omega, dim3(1), dim3(1), 0, q, D.scal.p);
    hipLaunchKernelGGL((k_bicg_xr2<Z>), dim3(kNormBlocks), dim3(kBlock), 0, q, x, r, ph, sh, sv, t, rh, D.scal.p, nd,
                       D.part.p);
    hipLaunchKernelGGL(k_dot_final, dim3(1), dim3(kBlock), 0, q, D.part.p, kNormBlocks, 2, D.scal.p + SC_RHO);
    HIPCHECK(hipGetLastError());
  };
  restart(r0, r0 == L.b64.p);
  int restarts = 0;
  while (rel > rtol) {
    if (cyc + 2 > max_cycles) return EBMG_ERR_NOCONV;
    if (o.graphs == 0 && !D.timing())
      graph_run(D.g_krylov, s, iteration);
    else
      iteration(s);
    fetch_scalars(D, s);
    cyc += 2;
    ++info.outer_iters;
    const double* h = D.host_scal;
    double nrel = std::sqrt(h[SC_RR]) / bn;
    const bool broke = !std::isfinite(nrel) || !std::isfinite(h[SC_ALPHA]) || h[SC_OMEGA] == 0.0 ||
                       !std::isfinite(h[SC_OMEGA]);
    if (info.n_hist < 64) info.hist[info.n_hist++] = nrel;
    if (broke || nrel <= rtol) {
      // confirm with the true residual (and restart from it if needed)
      residual<double, 0>(L, x, L.b64.p, L.r64.p, s);
      nrel = norm2<double>(D, L.r64.p, nd, s) / bn;
      if (!std::isfinite(nrel) || nrel > 1e6) {
        rel = nrel;
        return EBMG_ERR_NUMERIC;
      }
      if (nrel > rtol) {
        if (++restarts > 8) {
          rel = nrel;
          return EBMG_ERR_NOCONV;
        }
        restart(L.r64.p, false);
      }
    } else if (nrel > 1e6) {
      rel = nrel;
      return EBMG_ERR_NUMERIC;
    }
    rel = nrel;
  }
  return EBMG_OK;
}

static ebmg_status bicgstab(DevProblem& D, const Options& o, double bn, double rtol, int max_cycles, double& rel,
                            int& cyc, ebmg_solve_info& info, hipStream_t s, const double* r0) {
  if (o.precision == EBMG_MIXED)
    return bicgstab_t<float>(D, o, bn, rtol, max_cycles, rel, cyc, info, D.ph32.p, D.sh32.p, s, r0);
  return bicgstab_t<double>(D, o, bn, rtol, max_cycles, rel, cyc, info, D.kv[4].p, D.kv[6].p, s, r0);
}

static ebmg_status solve(ebmg_problem_s* P, const double* rho, const double* sigma, const double* bcv,
                         const double* objv, double rtol, int max_cycles, double* phi, double* phi2, double* E,
                         ebmg_solve_info* info) {
  auto t0 = std::chrono::steady_clock::now();
  Problem& H = *P->host;
  DevProblem& D = P->dev;
  hipStream_t s = P->ctx->stream;
  DevLevel& L = D.lv[0];
  const int64_t nd = L.N + L.N2;
  const bool mixed = H.opt.precision == EBMG_MIXED;
  ebmg_solve_info loc;
  std::memset(&loc, 0, sizeof(loc));
  loc.levels = (int)D.lv.size();
  rhs(P, rho, sigma, bcv, objv);
  double* guess_nz = D.scal.p + SC_GUESS;
  fill<double>(guess_nz, 1, 0.0, s);
  hipLaunchKernelGGL(k_guess_in, dim3(nblk(L.N)), dim3(kBlock), 0, s, L.tag.p, phi, L.x64.p, L.N, guess_nz);
  if (L.N2 > 0) {
    if (phi2)
      hipLaunchKernelGGL(k_guess_in, dim3(nblk(L.N2)), dim3(kBlock), 0, s, (const uint8_t*)nullptr, phi2,
                         L.x64.p + L.N, L.N2, guess_nz);
    else
      fill<double>(L.x64.p + L.N, L.N2, 0.0, s);
  }
  const double bn = norm2<double>(D, L.b64.p, nd, s);
  // a zero initial guess: r0 = b exactly (A 0 = 0, and b is 0 on covered
  // cells, as the residual kernels write there), so A x and its norm are not
  // formed; the relative residual is then exactly 1
  const bool zero_guess = D.host_scal[SC_GUESS] == 0.0;
  loc.r0_norm = bn;
  ebmg_status st = EBMG_OK;
  if (!std::isfinite(bn)) {
    st = EBMG_ERR_NUMERIC;
  } else if (bn == 0.0) {
    fill<double>(L.x64.p, nd, 0.0, s);
    loc.rel_residual = 0.0;
  } else {
    double rel = 1.0;
    if (!zero_guess) {
      residual<double, 0>(L, L.x64.p, L.b64.p, L.r64.p, s);
      rel = norm2<double>(D, L.r64.p, nd, s) / bn;
    } else if (!D.krylov) {
      HIPCHECK(hipMemcpyAsync(L.r64.p, L.b64.p, sizeof(double) * nd, hipMemcpyDeviceToDevice, s));
    }
    int cyc = 0;
    if (D.krylov) {
      st = bicgstab(D, H.opt, bn, rtol, max_cycles, rel, cyc, loc, s, zero_guess ? L.b64.p : L.r64.p);
    } else {
      // one refinement cycle and its residual norm
      auto cycle = [&](hipStream_t q) {
        if (mixed) {
          hipLaunchKernelGGL((k_convert<double, float>), dim3(nblk(nd)), dim3(kBlock), 0, q, L.r64.p, L.b32.p, nd);
          fill<float>(L.x32.p, nd, 0.0f, q);
          vcycle<float>(D, H.opt, 0, q, L.x32.p, L.b32.p);
          hipLaunchKernelGGL(k_add_f32, dim3(nblk(nd)), dim3(kBlock), 0, q, L.x64.p, L.x32.p, nd);
        } else {
          vcycle<double>(D, H.opt, 0, q, L.x64.p, L.b64.p);
        }
        residual<double, 0>(L, L.x64.p, L.b64.p, L.r64.p, q);
        dot_dev<double>(D, L.r64.p, L.r64.p, nd, SC_RR, q);
      };
      while (rel > rtol) {
        if (cyc >= max_cycles) {
          st = EBMG_ERR_NOCONV;
          break;
        }
        if (H.opt.graphs == 0 && !D.timing())
          graph_run(D.g_plain, s, cycle);
        else
          cycle(s);
        if (mixed) ++loc.outer_iters;
        ++cyc;
        fetch_scalars(D, s);
        double nrel = std::sqrt(D.host_scal[SC_RR]) / bn;
        if (loc.n_hist < 64) loc.hist[loc.n_hist++] = nrel;
        if (!std::isfinite(nrel) || nrel > 1e6) {
          rel = nrel;
          st = EBMG_ERR_NUMERIC;
          break;
        }
        rel = nrel;
      }
    }
    loc.cycles = cyc;
    loc.rel_residual = rel;
  }
  HIPCHECK(hipMemcpyAsync(phi, L.x64.p, sizeof(double) * L.N, hipMemcpyDeviceToDevice, s));
  if (phi2 && L.N2 > 0)
    HIPCHECK(hipMemcpyAsync(phi2, L.x64.p + L.N, sizeof(double) * L.N2, hipMemcpyDeviceToDevice, s));
  if (E) efield(P, L.x64.p, sigma, bcv, E);
  HIPCHECK(hipStreamSynchronize(s));
  for (auto& k : D.kt)
    if (k) k->harvest();
  loc.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  {
    // right-hand side, guess intake, ||b||, first residual and its norm,
    // the solution copy-out and E; then the cycles and outer iterations
    const double n = (double)nd;
    double by = (double)L.N * (8.0 + 1.0 + 8.0) + rows_bytes(L, 8) + (double)L.N * 17.0 + n * 8.0 +
                (double)L.N * 25.0 + rows_bytes(L, 8) + n * 8.0 + n * 16.0;
    if (E) by += (double)L.N * (9.0 + 8.0 * L.dim);
    const int vsz = mixed ? 4 : 8;
    by += loc.cycles * vcycle_bytes(D, H.opt, vsz);
    by += (D.krylov ? loc.outer_iters : loc.cycles) * iteration_bytes(D, H.opt);
    loc.est_bytes = (int64_t)by;
  }
  if (info) *info = loc;
  return st;
}


// ---------------------------------------------------------------------------
// batched boxes
// ---------------------------------------------------------------------------
template <typename T>
static BBox<T> make_bbox(ebmg_problem_s* P, const BLev<T>* lv_dev) {
  Problem& H = *P->host;
  DevProblem& D = P->dev;
  DevLevel& L0 = D.lv[0];
  BBox<T> B;
  std::memset(&B, 0, sizeof(B));
  B.dim = L0.dim;
  B.nlev = (int)D.lv.size();
  B.N = (int)L0.N;
  B.N2 = (int)L0.N2;
  B.lv = lv_dev;
  B.f64 = make_blev<double>(L0);
  B.Ainv = D.bottom.n > 0 ? D.bottom.p : nullptr;
  B.nbot = (int)D.bottom_n;
  B.bk = (const BBot*)D.bk_dev.p;
  B.icell = D.icell.p;
  B.isrc = D.isrc.p;
  B.iface = D.iface.p;
  B.iobj = D.iobj.p;
  B.icobj = D.icobj.p;
  B.icsig = D.icsig.p;
  for (int d = 0; d < 3; ++d) B.dat.n[d] = L0.n[d];
  for (int f = 0; f < 6; ++f) {
    B.fv[f] = H.bc.value[f];
    for (int p = 0; p < 2; ++p) B.dat.cb[f][p] = H.fine.dat[f][p] * H.bc.value[f];
  }
  B.objv = D.objv.p;
  for (int k = 0; k < 8; ++k) B.kv[k] = D.kv[k].p;
  B.krylov = H.opt.krylov;
  if constexpr (sizeof(T) == sizeof(double)) {
    B.zx[0] = (T*)D.kv[4].p;
    B.zx[1] = (T*)D.kv[6].p;
    B.zb[0] = (T*)D.kv[2].p;
    B.zb[1] = (T*)D.kv[5].p;
  } else {
    // FP32 cycle outputs live in the (otherwise unused) FP64 ph / sh slots
    B.zx[0] = (T*)(void*)D.kv[4].p;
    B.zx[1] = (T*)(void*)D.kv[6].p;
    B.zb[0] = B.zb[1] = (T*)L0.b32.p;
  }
  return B;
}

template <typename T>
static void upload_batch_views(ebmg_batch_s* Bt, hipStream_t s) {
  std::vector<BBox<T>> hb;
  Bt->lvbuf.resize(Bt->boxes.size());
  for (size_t i = 0; i < Bt->boxes.size(); ++i) {
    ebmg_problem_s* P = Bt->boxes[i].get();
    std::vector<BLev<T>> v;
    for (auto& l : P->dev.lv) v.push_back(make_blev<T>(l));
    int64_t by = 0;
    Bt->lvbuf[i].upload((const uint8_t*)v.data(), (int64_t)(v.size() * sizeof(BLev<T>)), s, by);
    Bt->bytes += by;
    HIPCHECK(hipStreamSynchronize(s));
    hb.push_back(make_bbox<T>(P, (const BLev<T>*)Bt->lvbuf[i].p));
  }
  int64_t by = 0;
  Bt->bbox.upload((const uint8_t*)hb.data(), (int64_t)(hb.size() * sizeof(BBox<T>)), s, by);
  Bt->bytes += by;
  HIPCHECK(hipStreamSynchronize(s));
}
// ---------------------------------------------------------------------------
// level-synchronous batched solver (host side)
// ---------------------------------------------------------------------------
static inline int cdiv(int64_t a, int64_t b) { return (int)((a + b - 1) / b); }

// Explicit rows of colour group g of a level (as the device views count them).
static int group_rows(const DevLevel& l, int g) {
  if (l.cls_ptr.size() == 3) return l.cls_ptr[g + 1] - l.cls_ptr[g];
  return g == 0 ? (int)l.R : 0;
}

// Append chunks [0, nch) of segment seg of box b.
static inline void add_chunks(std::vector<WEnt>& t, int b, int seg, int nch) {
  for (int c = 0; c < nch; ++c) t.push_back(WEnt{b, seg, c, 0});
}

static void upload_table(ebmg_batch_s::Table& T, std::vector<WEnt>& e, hipStream_t s, int64_t& by) {
  T.d.release();
  T.n = 0;
  if (e.empty()) return;
  while (e.size() % kXCD) e.push_back(WEnt{-1, 0, 0, 0});
  T.n = (int)e.size();
  T.d.upload((const uint8_t*)e.data(), (int64_t)(e.size() * sizeof(WEnt)), s, by);
}

// First level of box P that runs in one workgroup: the first with at most
// `cells` unknowns, the bottom level at the latest.
static int first_tail_level(ebmg_problem_s* P, int cells) {
  const auto& lv = P->dev.lv;
  const int nl = (int)lv.size();
  for (int l = 0; l < nl - 1; ++l)
    if (lv[l].N + lv[l].N2 <= cells) return l;
  return nl - 1;
}

// Work tables of the grid-wide levels for a coarse-part threshold.
template <typename T>
static void build_wide_tables(ebmg_batch_s* Bt, int cells, hipStream_t s) {
  if (Bt->g_iter) (void)hipGraphExecDestroy(Bt->g_iter);   // its tables are about to go
  Bt->g_iter = nullptr;
  const int nbox = (int)Bt->boxes.size();
  std::vector<int32_t> lt(nbox);
  int lw = 0;
  for (int i = 0; i < nbox; ++i) {
    lt[i] = first_tail_level(Bt->boxes[i].get(), cells);
    lw = std::max(lw, lt[i]);
  }
  int64_t by = 0;
  for (auto& w : Bt->wide) {
    for (auto* t : {&w.rb, &w.jac[0], &w.jac[1], &w.scat[0], &w.scat[1], &w.cell, &w.res, &w.pro}) {
      t->d.release();
      t->n = 0;
    }
  }
  Bt->wide.clear();
  Bt->wide.resize(lw);
  const int CH = WCh<T>::v;
  for (int l = 0; l < lw; ++l) {
    std::vector<WEnt> rb, jac[2], scat[2], cell, res, pro;
    for (int i = 0; i < nbox; ++i) {
      if (lt[i] <= l) continue;
      const auto& lv = Bt->boxes[i]->dev.lv;
      const DevLevel& F = lv[l];
      const DevLevel& C = lv[l + 1];
      const int64_t half = (int64_t)((F.n[0] + 1) / 2) * F.n[1] * (F.dim == 3 ? F.n[2] : 1);
      add_chunks(rb, i, 0, cdiv(half, CH));
      for (int g = 0; g < 2; ++g) {
        const int rows = group_rows(F, g);
        add_chunks(jac[g], i, 0, cdiv(rows, kSlice));   // one slice per entry (kw_irr_jac)
        add_chunks(scat[g], i, 0, cdiv(rows, kWList));
      }
      add_chunks(cell, i, 0, cdiv(F.N, CH));
      add_chunks(cell, i, 1, cdiv(group_rows(F, 0), kWRows));
      add_chunks(cell, i, 2, cdiv(group_rows(F, 1), kWRows));
      add_chunks(res, i, 0, cdiv(C.N, CH));
      add_chunks(res, i, 1, cdiv(F.n_ns, kWList));
      add_chunks(res, i, 2, cdiv(C.N2, kWList));
      add_chunks(pro, i, 0, cdiv(F.N, CH));
      add_chunks(pro, i, 1, cdiv(F.n_np, kWList));
    }
    auto& W = Bt->wide[l];
    upload_table(W.rb, rb, s, by);
    for (int g = 0; g < 2; ++g) {
      upload_table(W.jac[g], jac[g], s, by);
      upload_table(W.scat[g], scat[g], s, by);
    }
    upload_table(W.cell, cell, s, by);
    upload_table(W.res, res, s, by);
    upload_table(W.pro, pro, s, by);
  }
  // coarse parts that are a bottom level with an inverse go to the grid-wide
  // bottom kernel, the others to one workgroup each
  std::vector<WEnt> bot;
  std::vector<int32_t> tl;
  for (int i = 0; i < nbox; ++i) {
    DevProblem& D = Bt->boxes[i]->dev;
    if (lt[i] == (int)D.lv.size() - 1 && D.bottom.n > 0)
      add_chunks(bot, i, 0, cdiv(D.bottom_n, kWBotRows));
    else
      tl.push_back(i);
  }
  upload_table(Bt->bot, bot, s, by);
  Bt->tail_list.release();
  Bt->n_tail = (int)tl.size();
  if (!tl.empty()) Bt->tail_list.upload(tl.data(), (int64_t)tl.size(), s, by);
  Bt->lt.release();
  Bt->lt.upload(lt.data(), nbox, s, by);
  Bt->tail_cells = cells;
  HIPCHECK(hipStreamSynchronize(s));
}

// Everything of the level-synchronous mode that does not depend on the
// coarse-part threshold: level views, finest-level tables, partial sums,
// per-box state.
template <typename T>
static void setup_wide_common(ebmg_batch_s* Bt, hipStream_t s) {
  const int nbox = (int)Bt->boxes.size();
  int64_t by = 0;
  int nl = 0;
  for (auto& P : Bt->boxes) nl = std::max(nl, (int)P->dev.lv.size());
  Bt->wl.resize(nl);
  BLev<T> zero;
  std::memset(&zero, 0, sizeof(zero));
  for (int l = 1; l < nl; ++l) {
    std::vector<BLev<T>> v(nbox, zero);
    for (int i = 0; i < nbox; ++i) {
      auto& lv = Bt->boxes[i]->dev.lv;
      if (l < (int)lv.size()) v[i] = make_blev<T>(lv[l]);
    }
    Bt->wl[l].upload((const uint8_t*)v.data(), (int64_t)(v.size() * sizeof(BLev<T>)), s, by);
    HIPCHECK(hipStreamSynchronize(s));
  }
  std::vector<BBox<T>> hb(nbox);
  HIPCHECK(hipMemcpy(hb.data(), Bt->bbox.p, sizeof(BBox<T>) * nbox, hipMemcpyDeviceToHost));
  for (int w = 0; w < 2; ++w) {
    std::vector<BLev<T>> v(nbox);
    for (int i = 0; i < nbox; ++i) {
      v[i] = make_blev<T>(Bt->boxes[i]->dev.lv[0]);
      v[i].x = hb[i].zx[w];
      v[i].b = hb[i].zb[w];
    }
    Bt->wl0[w].upload((const uint8_t*)v.data(), (int64_t)(v.size() * sizeof(BLev<T>)), s, by);
    HIPCHECK(hipStreamSynchronize(s));
  }
  std::vector<WEnt> op, vec;
  std::vector<int32_t> eop(nbox + 1), evec(nbox + 1);
  for (int i = 0; i < nbox; ++i) {
    const DevLevel& L0 = Bt->boxes[i]->dev.lv[0];
    eop[i] = (int32_t)op.size();
    add_chunks(op, i, 0, cdiv(L0.N, WCh<double>::v));
    add_chunks(op, i, 1, cdiv(group_rows(L0, 0), kWRows));
    add_chunks(op, i, 2, cdiv(group_rows(L0, 1), kWRows));
    evec[i] = (int32_t)vec.size();
    add_chunks(vec, i, 0, cdiv(L0.N + L0.N2, kWVec));
  }
  eop[nbox] = (int32_t)op.size();
  evec[nbox] = (int32_t)vec.size();
  upload_table(Bt->op64, op, s, by);
  upload_table(Bt->vec, vec, s, by);
  Bt->ebeg_op.upload(eop.data(), nbox + 1, s, by);
  Bt->ebeg_vec.upload(evec.data(), nbox + 1, s, by);
  const int np = std::max(Bt->op64.n, Bt->vec.n);
  Bt->part0.alloc(np, by);
  Bt->part1.alloc(np, by);
  Bt->state.alloc((int64_t)(nbox * sizeof(WState)), by);
  Bt->wio.alloc((int64_t)(nbox * sizeof(WIO)), by);
  Bt->count.alloc(1, by);
  HIPCHECK(hipHostMalloc((void**)&Bt->host_count, sizeof(int), hipHostMallocDefault));
  Bt->bytes += by;
  HIPCHECK(hipStreamSynchronize(s));
}

template <typename T, int DIM>
static void wide_smooth(ebmg_batch_s* Bt, int l, const BLev<T>* W, int sweeps, hipStream_t s) {
  auto& L = Bt->wide[l];
  const WState* st = (const WState*)Bt->state.p;
  for (int it = 0; it < sweeps; ++it)
    for (int colour = 0; colour < 2; ++colour) {
      hipLaunchKernelGGL((kw_rb<T, DIM>), dim3(L.rb.n), dim3(kWB), 0, s, W, (const WEnt*)L.rb.d.p, st, colour);
      if (L.jac[colour].n) {
        hipLaunchKernelGGL((kw_irr_jac<T>), dim3(L.jac[colour].n), dim3(kWB), 0, s, W,
                           (const WEnt*)L.jac[colour].d.p, st, colour);
        hipLaunchKernelGGL((kw_irr_scat<T>), dim3(L.scat[colour].n), dim3(kWB), 0, s, W,
                           (const WEnt*)L.scat[colour].d.p, st, colour);
      }
    }
}

// One V-cycle of every active box on (zb[which], zx[which]) from zx = 0.
template <typename T, int DIM>
static void wide_vcycle(ebmg_batch_s* Bt, int which, hipStream_t s) {
  const int lw = (int)Bt->wide.size();
  const WState* st = (const WState*)Bt->state.p;
  auto view = [&](int l) -> const BLev<T>* {
    return (const BLev<T>*)(l == 0 ? Bt->wl0[which].p : Bt->wl[l].p);
  };
  for (int l = 0; l < lw; ++l) {
    auto& L = Bt->wide[l];
    wide_smooth<T, DIM>(Bt, l, view(l), Bt->nu1, s);
    hipLaunchKernelGGL((kw_resid<T, DIM>), dim3(L.cell.n), dim3(kWB), 0, s, view(l), (const WEnt*)L.cell.d.p, st);
    hipLaunchKernelGGL((kw_restrict<T, DIM>), dim3(L.res.n), dim3(kWB), 0, s, view(l), view(l + 1),
                       (const WEnt*)L.res.d.p, st);
  }
  if (Bt->bot.n)
    hipLaunchKernelGGL((kw_bottom<T>), dim3(Bt->bot.n), dim3(kWB), 0, s, (const BBox<T>*)Bt->bbox.p, Bt->lt.p,
                       (const WEnt*)Bt->bot.d.p, st, which);
  if (Bt->n_tail)
    hipLaunchKernelGGL((kw_tail<T, DIM>), dim3(Bt->n_tail), dim3(kBE), 0, s, (const BBox<T>*)Bt->bbox.p, Bt->lt.p,
                       Bt->tail_list.p, st, which, Bt->nu1, Bt->nu2);
  for (int l = lw - 1; l >= 0; --l) {
    auto& L = Bt->wide[l];
    hipLaunchKernelGGL((kw_prolong<T, DIM>), dim3(L.pro.n), dim3(kWB), 0, s, view(l), view(l + 1),
                       (const WEnt*)L.pro.d.p, st);
    wide_smooth<T, DIM>(Bt, l, view(l), Bt->nu2, s);
  }
}

// The finest level's template half-sweeps (which 0) or explicit-row Jacobi
// passes (which 1) of every box, both colours, as inside a V-cycle (for the
// measurement hook).
template <typename T, int DIM>
static void wide_level0_kernels(ebmg_batch_s* Bt, int which, hipStream_t s) {
  auto& L = Bt->wide[0];
  const WState* st = (const WState*)Bt->state.p;
  const BLev<T>* W = (const BLev<T>*)Bt->wl0[0].p;
  for (int colour = 0; colour < 2; ++colour) {
    if (which == 0)
      hipLaunchKernelGGL((kw_rb<T, DIM>), dim3(L.rb.n), dim3(kWB), 0, s, W, (const WEnt*)L.rb.d.p, st, colour);
    else if (L.jac[colour].n)
      hipLaunchKernelGGL((kw_irr_jac<T>), dim3(L.jac[colour].n), dim3(kWB), 0, s, W, (const WEnt*)L.jac[colour].d.p,
                         st, colour);
  }
  HIPCHECK(hipGetLastError());
}

template <typename T, int OP>
static void wide_vec(ebmg_batch_s* Bt, int filt, hipStream_t s) {
  hipLaunchKernelGGL((kw_vec<T, OP>), dim3(Bt->vec.n), dim3(kWB), 0, s, (const BBox<T>*)Bt->bbox.p,
                     (const WEnt*)Bt->vec.d.p, (const WState*)Bt->state.p, (const WIO*)Bt->wio.p, filt,
                     Bt->part0.p, Bt->part1.p);
}

template <typename T, typename TX, int DIM, int MODE, int NDOT>
static void wide_op(ebmg_batch_s* Bt, int filt, int which, int out, int da, hipStream_t s) {
  hipLaunchKernelGGL((kw_op64<T, TX, DIM, MODE, NDOT>), dim3(Bt->op64.n), dim3(kWB), 0, s,
                     (const BBox<T>*)Bt->bbox.p, (const WEnt*)Bt->op64.d.p, (const WState*)Bt->state.p, filt, which,
                     out, da, Bt->part0.p, Bt->part1.p);
}

template <int STAGE>
static void wide_fin(ebmg_batch_s* Bt, bool vec, double rtol, int max_cycles, hipStream_t s) {
  const int nbox = (int)Bt->boxes.size();
  const int per = kWB / 64;
  hipLaunchKernelGGL((kw_fin<STAGE>), dim3((nbox + per - 1) / per), dim3(kWB), 0, s,
                     vec ? Bt->ebeg_vec.p : Bt->ebeg_op.p, Bt->part0.p, Bt->part1.p, (WState*)Bt->state.p, nbox,
                     rtol, max_cycles);
}

static std::vector<WState> initial_state(ebmg_batch_s* Bt) {
  std::vector<WState> st(Bt->boxes.size());
  for (size_t i = 0; i < st.size(); ++i) {
    std::memset(&st[i], 0, sizeof(WState));
    st[i].active = 1;
    st[i].mode = Bt->boxes[i]->host->opt.krylov == 2 ? 2 : 1;
    st[i].rho_old = st[i].alpha = st[i].omega = 1.0;
  }
  return st;
}

// One BiCGStab iteration (or two refinement cycles) of every active box.
template <typename T, int DIM>
static void wide_iteration(ebmg_batch_s* Bt, double rtol, int max_cycles, hipStream_t s) {
  wide_vec<T, WV_P>(Bt, WF_ACTIVE, s);
  wide_vcycle<T, DIM>(Bt, 0, s);
  wide_op<T, T, DIM, 1, 1>(Bt, WF_ACTIVE, 0, 3, 1, s);            // v = A ph, (rh, v)
  wide_fin<WS_A>(Bt, false, rtol, max_cycles, s);
  wide_vec<T, WV_S>(Bt, WF_ACTIVE, s);
  wide_vcycle<T, DIM>(Bt, 1, s);
  wide_op<T, T, DIM, 1, 2>(Bt, WF_ACTIVE, 1, 7, 5, s);            // t = A sh, (s, t), (t, t)
  wide_fin<WS_B>(Bt, false, rtol, max_cycles, s);
  wide_vec<T, WV_XR>(Bt, WF_ACTIVE, s);
  wide_fin<WS_C>(Bt, true, rtol, max_cycles, s);
  wide_op<T, double, DIM, 0, 2>(Bt, WF_VERIFY, 0, 0, 0, s);       // true r = b - A x where tested
  wide_fin<WS_D>(Bt, false, rtol, max_cycles, s);
  wide_vec<T, WV_RESTART>(Bt, WF_RESTART, s);
}

template <typename T, int DIM>
static void wide_solve(ebmg_batch_s* Bt, const std::vector<WIO>& io, double rtol, int max_cycles,
                       std::vector<WState>& out, hipStream_t s) {
  const int nbox = (int)Bt->boxes.size();
  std::vector<WState> st = initial_state(Bt);
  HIPCHECK(hipMemcpyAsync(Bt->state.p, st.data(), sizeof(WState) * nbox, hipMemcpyHostToDevice, s));
  HIPCHECK(hipMemcpyAsync(Bt->wio.p, io.data(), sizeof(WIO) * nbox, hipMemcpyHostToDevice, s));
  hipLaunchKernelGGL((kw_rhs<T, DIM>), dim3(Bt->op64.n), dim3(kWB), 0, s, (const BBox<T>*)Bt->bbox.p,
                     (const WEnt*)Bt->op64.d.p, (const WIO*)Bt->wio.p);
  wide_vec<T, WV_INIT>(Bt, WF_ACTIVE, s);                         // x = guess, (b, b)
  wide_fin<WS_BB>(Bt, true, rtol, max_cycles, s);
  wide_op<T, double, DIM, 0, 2>(Bt, WF_ACTIVE, 0, 0, 0, s);       // r = b - A x, (r, r)
  wide_fin<WS_R0>(Bt, false, rtol, max_cycles, s);
  wide_vec<T, WV_RESTART>(Bt, WF_RESTART, s);
  HIPCHECK(hipGetLastError());
  // every iteration adds two cycles to each active box, so max_cycles / 2
  // iterations stop every box
  const int limit = max_cycles / 2 + 2;
  for (int it = 0;; ++it) {
    hipLaunchKernelGGL(kw_count, dim3(1), dim3(kWB), 0, s, (const WState*)Bt->state.p, nbox, Bt->count.p);
    HIPCHECK(hipMemcpyAsync(Bt->host_count, Bt->count.p, sizeof(int), hipMemcpyDeviceToHost, s));
    HIPCHECK(hipStreamSynchronize(s));
    if (*Bt->host_count == 0) break;
    if (it >= limit) throw DeviceError("batched solve did not stop");
    if (Bt->graphs) {
      if (Bt->g_iter && (Bt->g_rtol != rtol || Bt->g_max_cycles != max_cycles)) {
        (void)hipGraphExecDestroy(Bt->g_iter);
        Bt->g_iter = nullptr;
      }
      Bt->g_rtol = rtol;
      Bt->g_max_cycles = max_cycles;
      graph_run(Bt->g_iter, s, [&](hipStream_t q) { wide_iteration<T, DIM>(Bt, rtol, max_cycles, q); });
    } else {
      wide_iteration<T, DIM>(Bt, rtol, max_cycles, s);
    }
    HIPCHECK(hipGetLastError());
  }
  wide_vec<T, WV_OUT>(Bt, WF_ACTIVE, s);
  out.resize(nbox);
  HIPCHECK(hipMemcpyAsync(out.data(), Bt->state.p, sizeof(WState) * nbox, hipMemcpyDeviceToHost, s));
  HIPCHECK(hipStreamSynchronize(s));
}

// Coarse-part autotuner: time one V-cycle of all boxes (on zero vectors)
// for each candidate threshold; keep the fastest.
template <typename T, int DIM>
static void tune_wide(ebmg_batch_s* Bt, hipStream_t s) {
  if (Bt->tail_opt == 1 || Bt->tail_opt == 2) {
    // a fixed threshold (no timing, so the choice never depends on what
    // else runs on the device): only the bottom level, or every level of at
    // most kTailMax unknowns, in each box's one-workgroup coarse part
    const int c = Bt->tail_opt == 1 ? 0 : (int)kTailMax;
    Bt->cand_cells.assign(1, c);
    Bt->cand_ms.assign(1, 0.0);
    build_wide_tables<T>(Bt, c, s);
    return;
  }
  const int nbox = (int)Bt->boxes.size();
  std::vector<WState> st = initial_state(Bt);
  HIPCHECK(hipMemcpyAsync(Bt->state.p, st.data(), sizeof(WState) * nbox, hipMemcpyHostToDevice, s));
  for (auto& P : Bt->boxes) {
    DevProblem& D = P->dev;
    const int64_t nd = D.lv[0].N + D.lv[0].N2;
    for (int k : {2, 4, 5, 6}) HIPCHECK(hipMemsetAsync(D.kv[k].p, 0, sizeof(double) * nd, s));
    if (Bt->mixed) HIPCHECK(hipMemsetAsync(D.lv[0].b32.p, 0, sizeof(float) * nd, s));
  }
  const int cand[] = {0, 512, 4096, 32768};
  Bt->cand_cells.clear();
  Bt->cand_ms.clear();
  hipEvent_t e0, e1;
  HIPCHECK(hipEventCreate(&e0));
  HIPCHECK(hipEventCreate(&e1));
  double best = 1e30;
  int pick = 0;
  std::vector<int> seen;
  for (int c : cand) {
    // skip thresholds that give the same split as one already timed
    std::vector<int> lt(nbox);
    for (int i = 0; i < nbox; ++i) lt[i] = first_tail_level(Bt->boxes[i].get(), c);
    bool dup = false;
    for (int q : seen) {
      bool same = true;
      for (int i = 0; i < nbox && same; ++i) same = first_tail_level(Bt->boxes[i].get(), q) == lt[i];
      dup = dup || same;
    }
    if (dup) continue;
    seen.push_back(c);
    build_wide_tables<T>(Bt, c, s);
    for (int r = 0; r < 2; ++r) wide_vcycle<T, DIM>(Bt, 0, s);
    const int reps = 3;
    HIPCHECK(hipEventRecord(e0, s));
    for (int r = 0; r < reps; ++r) wide_vcycle<T, DIM>(Bt, 0, s);
    HIPCHECK(hipEventRecord(e1, s));
    HIPCHECK(hipEventSynchronize(e1));
    float ms = 0;
    HIPCHECK(hipEventElapsedTime(&ms, e0, e1));
    Bt->cand_cells.push_back(c);
    Bt->cand_ms.push_back(ms / reps);
    if (ms / reps < best) {
      best = ms / reps;
      pick = c;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  build_wide_tables<T>(Bt, pick, s);
}

template <typename T>
static void setup_wide(ebmg_batch_s* Bt, hipStream_t s) {
  setup_wide_common<T>(Bt, s);
  if (Bt->dim == 3)
    tune_wide<T, 3>(Bt, s);
  else
    tune_wide<T, 2>(Bt, s);
}

static void release_wide(ebmg_batch_s* Bt) {
  if (Bt->g_iter) (void)hipGraphExecDestroy(Bt->g_iter);
  Bt->g_iter = nullptr;
  for (auto& w : Bt->wide)
    for (auto* t : {&w.rb, &w.jac[0], &w.jac[1], &w.scat[0], &w.scat[1], &w.cell, &w.res, &w.pro}) t->d.release();
  Bt->wide.clear();
  for (auto& b : Bt->wl) b.release();
  Bt->wl.clear();
  Bt->wl0[0].release();
  Bt->wl0[1].release();
  Bt->op64.d.release();
  Bt->vec.d.release();
  Bt->bot.d.release();
  Bt->tail_list.release();
  Bt->ebeg_op.release();
  Bt->ebeg_vec.release();
  Bt->lt.release();
  Bt->part0.release();
  Bt->part1.release();
  Bt->state.release();
  Bt->wio.release();
  Bt->count.release();
  if (Bt->host_count) (void)hipHostFree(Bt->host_count);
  Bt->host_count = nullptr;
}

// Template-cell sweeps only (no explicit rows), for ebmg_smooth.
template <typename T>
static void template_sweeps(DevLevel& l, int variant, int sweeps, T* x, const T* b, hipStream_t s) {
  const Tmpl<T>& tp = Vec<T>::t(l);
  if (variant == 5 + kZMConfigs) {
    // fused sweeps with the explicit rows' Jacobi passes after each, as
    // smooth() runs them
    if (!fused_ok(l)) throw ArgError("this level has no fused sweep");
    const bool f0 = l.fused;
    const int v0 = l.fvar, c0 = l.zmcfg;
    if (!l.fused) {
      l.fvar = l.dim == 3 ? 1 : 0;
      l.zmcfg = 1;
    }
    l.fused = true;
    T* cur = x;
    T* alt = Vec<T>::xa(l);
    for (int it = 0; it < sweeps; ++it) {
      launch_fused<T>(l, cur, alt, b, tp, s);
      std::swap(cur, alt);
      irr_groups<T>(l, cur, b, s);
    }
    l.fused = f0;
    l.fvar = v0;
    l.zmcfg = c0;
    if (cur != x) HIPCHECK(hipMemcpyAsync(x, cur, sizeof(T) * (l.N + l.N2), hipMemcpyDeviceToDevice, s));
    HIPCHECK(hipGetLastError());
    return;
  }
  if (variant == 3 + kZMConfigs || variant == 4 + kZMConfigs) {
    // one-launch colour phases; the second form also relaxes each phase's
    // explicit rows (from the values before the phase), as smooth() does on
    // levels that use these phases
    const bool rows = variant == 4 + kZMConfigs;
    T* cur = x;
    T* alt = Vec<T>::xa(l);
    for (int it = 0; it < sweeps; ++it)
      for (int colour = 0; colour < 2; ++colour) {
        launch_oop<T>(l, colour, rows, cur, alt, b, s);
        std::swap(cur, alt);
      }
    HIPCHECK(hipGetLastError());
    return;
  }
  if (variant > 1) {
    const bool f0 = l.fused;
    const int v0 = l.fvar, c0 = l.zmcfg;
    l.fused = true;
    l.fvar = variant >= 3 ? 1 : 0;
    if (variant >= 3) l.zmcfg = variant - 3;
    T* cur = x;
    T* alt = Vec<T>::xa(l);
    for (int it = 0; it < sweeps; ++it) {
      launch_fused<T>(l, cur, alt, b, tp, s);
      std::swap(cur, alt);
    }
    l.fused = f0;
    l.fvar = v0;
    l.zmcfg = c0;
    if (cur != x) HIPCHECK(hipMemcpyAsync(x, cur, sizeof(T) * (l.N + l.N2), hipMemcpyDeviceToDevice, s));
  } else {
    const Shape sh = shape3((l.n[0] + 1) / 2, l.n[1], l.dim == 3 ? l.n[2] : 1);
    for (int it = 0; it < sweeps; ++it)
      for (int colour = 0; colour < 2; ++colour) {
        if (l.dim == 3)
          hipLaunchKernelGGL((k_rb<T, 3>), sh.g, sh.b, 0, s, l.tag.p, x, b, tp, colour);
        else
          hipLaunchKernelGGL((k_rb<T, 2>), sh.g, sh.b, 0, s, l.tag.p, x, b, tp, colour);
      }
  }
  HIPCHECK(hipGetLastError());
}

}  // namespace ebmg

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
using namespace ebmg;

template <typename F>
static ebmg_status guard_msg(std::string* err, F&& f) {
  try {
    return f();
  } catch (const ArgError& e) {
    if (err) *err = e.what();
    return EBMG_ERR_ARG;
  } catch (const GeomError& e) {
    if (err) *err = e.what();
    return EBMG_ERR_GEOMETRY;
  } catch (const DeviceError& e) {
    if (err) *err = e.what();
    return std::string(e.what()).find("out of memory") != std::string::npos ? EBMG_ERR_OOM : EBMG_ERR_DEVICE;
  } catch (const std::bad_alloc&) {
    if (err) *err = "host allocation failed";
    return EBMG_ERR_OOM;
  } catch (const std::exception& e) {
    if (err) *err = e.what();
    return EBMG_ERR_ARG;
  }
}

template <typename F>
static ebmg_status guard(ebmg_ctx ctx, F&& f) {
  return guard_msg(ctx ? &ctx->err : nullptr, std::forward<F>(f));
}

// Worker of a context: runs submitted solves in submission order on the
// context's stream, records each outcome under its ticket.
static void async_worker(ebmg_ctx c) {
  for (;;) {
    AsyncJob j;
    {
      std::unique_lock<std::mutex> lk(c->mu);
      c->cv_work.wait(lk, [&] { return c->stop || !c->queue.empty(); });
      if (c->queue.empty()) return;  // stopping and drained
      j = std::move(c->queue.front());
      c->queue.pop_front();
    }
    AsyncResult r;
    r.status = guard_msg(&r.err, [&]() -> ebmg_status {
      HIPCHECK(hipSetDevice(c->device));
      return solve(j.pb, j.rho, j.sigma, j.bcv.empty() ? nullptr : j.bcv.data(),
                   j.objv.empty() ? nullptr : j.objv.data(), j.rtol, j.max_cycles, j.phi, j.phi2, j.E, &r.info);
    });
    r.done = true;
    {
      std::lock_guard<std::mutex> lk(c->mu);
      c->results[j.ticket] = std::move(r);
      --j.pb->pending;
    }
    c->cv_done.notify_all();
  }
}

// Block until no submitted solve of P is queued or running.
static void drain(ebmg_problem_s* P) {
  ebmg_ctx c = P->ctx;
  std::unique_lock<std::mutex> lk(c->mu);
  c->cv_done.wait(lk, [&] { return P->pending == 0; });
}

static void stop_worker(ebmg_ctx c) {
  {
    std::lock_guard<std::mutex> lk(c->mu);
    c->stop = true;
  }
  c->cv_work.notify_all();
  if (c->worker.joinable()) c->worker.join();
  std::lock_guard<std::mutex> lk(c->mu);
  c->stop = false;  // a later submit (on a problem that outlived the handle) starts a new worker
}

static void ctx_unref(ebmg_ctx c) {
  if (--c->refs > 0) return;
  stop_worker(c);
  if (c->own_stream) {
    (void)hipSetDevice(c->device);
    (void)hipStreamDestroy(c->stream);
  }
  delete c;
}

namespace ebmg {

static void amr_free(ebmg_amr_s* A) {
  if (A->ctx && A->ctx->device >= 0) {
    (void)hipSetDevice(A->ctx->device);
    (void)hipStreamSynchronize(A->ctx->stream);
  }
  for (auto& k : A->link) k.release();
  A->link.clear();
  for (auto* b : {&A->x, &A->b, &A->r, &A->rh, &A->p, &A->v, &A->sv, &A->t, &A->ph, &A->sh, &A->rt, &A->y, &A->e,
                  &A->part, &A->scal})
    b->release();
  for (ebmg_problem_s* P : A->lev) {
    if (!P) continue;
    if (P->on_device) P->dev.release();
    delete P;
  }
  A->lev.clear();
}

// y = A_comp x: every level's operator, the coupling rows of each interface
// (fine rows with their ghosts, refluxed coarse rows) and identity rows for
// the covered coarse unknowns
static void amr_apply(ebmg_amr_s* A, const double* x, double* y, hipStream_t s) {
  const int L = (int)A->lev.size();
  for (int l = 0; l < L; ++l) residual<double, 1>(A->lev[l]->dev.lv[0], x + A->off[l], nullptr, y + A->off[l], s);
  for (int l = 1; l < L; ++l) {
    auto& K = A->link[l];
    const int64_t of = A->off[l], oc = A->off[A->box[l].parent];
    if (K.nf)
      hipLaunchKernelGGL(k_amr_rows, dim3(nblk(K.nf)), dim3(256), 0, s, K.nf, K.frow.p, K.fptr.p, K.fcol.p, K.fw.p,
                         x + of, x + oc, y + of);
    if (K.nc)
      hipLaunchKernelGGL(k_amr_rows, dim3(nblk(K.nc)), dim3(256), 0, s, K.nc, K.crow.p, K.cptr.p, K.ccol.p, K.cw.p,
                         x + oc, x + of, y + oc);
    if (K.ncov)
      hipLaunchKernelGGL(k_amr_set, dim3(nblk(K.ncov)), dim3(256), 0, s, K.ncov, K.cov.p, x + oc, y + oc);
  }
  HIPCHECK(hipGetLastError());
}

// z = M r: one V-cycle over the levels of the hierarchy. Down from the
// finest box: a V-cycle of the level on its residual (homogeneous
// coarse-fine faces), then the coarser level's residual updated by that
// correction (the level's residual after it restricted onto the covered
// unknowns, the refluxed rows next to the box reduced by its effect); one
// V-cycle of level 0 over the domain; then up again: the coarse correction
// prolonged (piecewise constant), the level's residual with the ghosts of
// the coarse correction, and a second V-cycle of the level. Covered unknowns
// end at 0. A fixed linear map (every V-cycle starts from zero), so it serves
// as the right preconditioner of BiCGStab.
static void amr_precond(ebmg_amr_s* A, const double* r, double* z, hipStream_t s) {
  const int L = (int)A->lev.size();
  const int64_t n = A->ntot;
  double* rt = A->rt.p;
  double* y = A->y.p;
  double* e = A->e.p;
  hipLaunchKernelGGL(k_amr_lin, dim3(nblk(n)), dim3(256), 0, s, n, 1.0, r, 0.0, r, rt);
  fill<double>(z, n, 0.0, s);
  // down: every box before its parent (deepest level first)
  for (int q = 0; q < L; ++q) {
    const int l = A->order[q];
    if (l == 0) continue;
    auto& K = A->link[l];
    const int pa = A->box[l].parent;
    const int64_t of = A->off[l], oc = A->off[pa], m = A->nd[l], mc = A->nd[pa];
    precond(A->lev[l]->dev, A->lev[l]->host->opt, rt + of, z + of, s);
    residual<double, 1>(A->lev[l]->dev.lv[0], z + of, nullptr, y + of, s);
    if (K.nf)
      hipLaunchKernelGGL(k_amr_rows, dim3(nblk(K.nf)), dim3(256), 0, s, K.nf, K.frow.p, K.fptr.p, K.fcol.p, K.fw.p,
                         z + of, z + oc, y + of);
    hipLaunchKernelGGL(k_amr_lin, dim3(nblk(m)), dim3(256), 0, s, m, 1.0, rt + of, -1.0, y + of, y + of);
    if (K.nr)
      hipLaunchKernelGGL(k_amr_gather, dim3(nblk(K.nr)), dim3(256), 0, s, K.nr, K.rrow.p, K.rptr.p, K.rcol.p, K.rw.p,
                         y + of, rt + oc);
    if (K.nc) {
      fill<double>(y + oc, mc, 0.0, s);
      hipLaunchKernelGGL(k_amr_rows, dim3(nblk(K.nc)), dim3(256), 0, s, K.nc, K.crow.p, K.cptr.p, K.ccol.p, K.cw.p,
                         z + oc, z + of, y + oc);
      hipLaunchKernelGGL(k_amr_lin, dim3(nblk(mc)), dim3(256), 0, s, mc, 1.0, rt + oc, -1.0, y + oc, rt + oc);
    }
  }
  precond(A->lev[0]->dev, A->lev[0]->host->opt, rt + A->off[0], z + A->off[0], s);
  // up: every box after its parent (coarsest level first)
  for (int q = L - 1; q >= 0; --q) {
    const int l = A->order[q];
    if (l == 0) continue;
    auto& K = A->link[l];
    const int64_t of = A->off[l], oc = A->off[A->box[l].parent], m = A->nd[l];
    hipLaunchKernelGGL(k_amr_prolong, dim3(nblk(m)), dim3(256), 0, s, m, K.pcol.p, z + oc, e + of);
    hipLaunchKernelGGL(k_amr_lin, dim3(nblk(m)), dim3(256), 0, s, m, 1.0, z + of, 1.0, e + of, z + of);
    residual<double, 1>(A->lev[l]->dev.lv[0], z + of, nullptr, y + of, s);
    if (K.nf)
      hipLaunchKernelGGL(k_amr_rows, dim3(nblk(K.nf)), dim3(256), 0, s, K.nf, K.frow.p, K.fptr.p, K.fcol.p, K.fw.p,
                         z + of, z + oc, y + of);
    hipLaunchKernelGGL(k_amr_lin, dim3(nblk(m)), dim3(256), 0, s, m, 1.0, rt + of, -1.0, y + of, y + of);
    precond(A->lev[l]->dev, A->lev[l]->host->opt, y + of, e + of, s);
    hipLaunchKernelGGL(k_amr_lin, dim3(nblk(m)), dim3(256), 0, s, m, 1.0, z + of, 1.0, e + of, z + of);
  }
  for (int l = 1; l < L; ++l) {
    auto& K = A->link[l];
    if (K.ncov)
      hipLaunchKernelGGL(k_amr_set, dim3(nblk(K.ncov)), dim3(256), 0, s, K.ncov, K.cov.p, (const double*)nullptr,
                         z + A->off[A->box[l].parent]);
  }
  HIPCHECK(hipGetLastError());
}

static double amr_dot(ebmg_amr_s* A, const double* a, const double* b, hipStream_t s) {
  hipLaunchKernelGGL((k_dot_partial<double>), dim3(kNormBlocks), dim3(kBlock), 0, s, a, b, A->ntot, A->part.p);
  hipLaunchKernelGGL(k_dot_final, dim3(1), dim3(kBlock), 0, s, A->part.p, kNormBlocks, 1, A->scal.p);
  HIPCHECK(hipGetLastError());
  double h = 0;
  HIPCHECK(hipMemcpyAsync(&h, A->scal.p, sizeof(double), hipMemcpyDeviceToHost, s));
  HIPCHECK(hipStreamSynchronize(s));
  return h;
}

// right-preconditioned BiCGStab over the composite vector, FP64, from the
// guess in A->x; one host round trip per dot product
static ebmg_status amr_bicgstab(ebmg_amr_s* A, double rtol, int maxit, double& bn, double& rel, int& iters,
                                hipStream_t s) {
  const int64_t n = A->ntot;
  const dim3 g(nblk(n)), blk(256);
  double *x = A->x.p, *b = A->b.p, *r = A->r.p, *rh = A->rh.p, *p = A->p.p, *v = A->v.p, *sv = A->sv.p,
         *t = A->t.p, *ph = A->ph.p, *sh = A->sh.p, *y = A->y.p;
  iters = 0;
  bn = std::sqrt(amr_dot(A, b, b, s));
  if (!(bn > 0)) {
    fill<double>(x, n, 0.0, s);
    rel = 0;
    return EBMG_OK;
  }
  amr_apply(A, x, y, s);
  hipLaunchKernelGGL(k_amr_lin, g, blk, 0, s, n, 1.0, b, -1.0, y, r);
  rel = std::sqrt(amr_dot(A, r, r, s)) / bn;
  if (rel <= rtol) return EBMG_OK;
  hipLaunchKernelGGL(k_amr_lin, g, blk, 0, s, n, 1.0, r, 0.0, r, rh);
  fill<double>(p, n, 0.0, s);
  fill<double>(v, n, 0.0, s);
  double rho_old = 1, alpha = 1, omega = 1;
  while (iters < maxit) {
    ++iters;
    const double rho = amr_dot(A, rh, r, s);
    if (!std::isfinite(rho)) return EBMG_ERR_NUMERIC;
    if (rho == 0.0) return EBMG_ERR_NOCONV;
    const double beta = (rho / rho_old) * (alpha / omega);
    hipLaunchKernelGGL(k_amr_p, g, blk, 0, s, n, r, beta, omega, v, p);
    amr_precond(A, p, ph, s);
    amr_apply(A, ph, v, s);
    alpha = rho / amr_dot(A, rh, v, s);
    hipLaunchKernelGGL(k_amr_lin, g, blk, 0, s, n, 1.0, r, -alpha, v, sv);
    const double sn = std::sqrt(amr_dot(A, sv, sv, s)) / bn;
    if (!std::isfinite(sn)) return EBMG_ERR_NUMERIC;
    if (sn <= rtol) {
      hipLaunchKernelGGL(k_amr_lin, g, blk, 0, s, n, 1.0, x, alpha, ph, x);
      hipLaunchKernelGGL(k_amr_lin, g, blk, 0, s, n, 1.0, sv, 0.0, sv, r);
      rel = sn;
      return EBMG_OK;
    }
    amr_precond(A, sv, sh, s);
    amr_apply(A, sh, t, s);
    const double tt = amr_dot(A, t, t, s);
    omega = tt > 0 ? amr_dot(A, t, sv, s) / tt : 0.0;
    hipLaunchKernelGGL(k_amr_xr, g, blk, 0, s, n, alpha, ph, omega, sh, sv, t, x, r);
    rel = std::sqrt(amr_dot(A, r, r, s)) / bn;
    if (!std::isfinite(rel)) return EBMG_ERR_NUMERIC;
    if (rel <= rtol) return EBMG_OK;
    if (omega == 0.0) return EBMG_ERR_NOCONV;
    rho_old = rho;
  }
  return EBMG_ERR_NOCONV;
}

}  // namespace ebmg

extern "C" {

void ebmg_default_options(ebmg_options* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->alpha = 0.0;
  o->beta = -1.0;
  o->b_gas = 1.0;
  o->eb_order = 2;
  o->precision = EBMG_FP64;
  o->nu1 = 2;
  o->nu2 = 2;
  o->bottom_max_dof = 600;
}

int ebmg_abi_version(void) { return EBMG_ABI_VERSION; }

static thread_local std::string g_create_error;

// Device scratch of ebmg_apply_noalloc: a file-scope array that every GPU the
// library runs on holds until the process ends (2 x kNoAllocMax doubles,
// 18 MiB: the staged input [phi; phi2] and the staged output). In host code
// the array's name is only a stand-in for the symbol: its device address is
// looked up once per device with that device current and kept in
// g_scratch, which is what host code passes to kernels.
constexpr int64_t kNoAllocMax = ((int64_t)1 << 20) + ((int64_t)1 << 17);   // unknowns (N + N2) at most
constexpr int kMaxDevices = 64;
static __device__ __align__(256) double scratch[2 * kNoAllocMax];
static std::mutex g_scratch_mu;
static double* g_scratch[kMaxDevices] = {};

// the current device's scratch address (looked up on first use per device)
static hipError_t scratch_ptr(int device, double** out) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  if (!g_scratch[device]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch[device] = (double*)p;
  }
  *out = g_scratch[device];
  return hipSuccess;
}

ebmg_status ebmg_create(int32_t device, void* stream, ebmg_ctx* out) {
  if (!out) return EBMG_ERR_ARG;
  *out = nullptr;
  auto* c = new (std::nothrow) ebmg_ctx_s;
  if (!c) return EBMG_ERR_OOM;
  c->device = device;
  if (device >= 0) {
    int n = 0;
    hipError_t e = hipGetDeviceCount(&n);
    if (e == hipSuccess && device >= n) e = hipErrorInvalidDevice;
    if (e == hipSuccess) e = hipSetDevice(device);
    if (e == hipSuccess) {
      if (stream) {
        c->stream = (hipStream_t)stream;
      } else {
        e = hipStreamCreate(&c->stream);
        c->own_stream = e == hipSuccess;
      }
    }
    if (e == hipSuccess) {
      double* sp = nullptr;   // the no-allocation scratch of this device, set up at init
      e = scratch_ptr(device, &sp);
    }
    if (e != hipSuccess) {
      g_create_error = std::string("device ") + std::to_string(device) + " (" + std::to_string(n) +
                       " visible): " + hipGetErrorString(e);
      delete c;
      return EBMG_ERR_DEVICE;
    }
  }
  *out = c;
  return EBMG_OK;
}

ebmg_status ebmg_destroy(ebmg_ctx ctx) {
  if (!ctx) return EBMG_ERR_ARG;
  stop_worker(ctx);
  ctx_unref(ctx);
  return EBMG_OK;
}

const char* ebmg_last_error(ebmg_ctx ctx) { return ctx ? ctx->err.c_str() : g_create_error.c_str(); }

static ebmg_status parse_options(const ebmg_options* opt, int nobj, ebmg::Options& out) {
  ebmg_options o;
  if (opt)
    o = *opt;
  else
    ebmg_default_options(&o);
  out.alpha = o.alpha;
  out.beta = o.beta;
  out.a_gas = o.a_gas;
  out.a_diel = o.a_diel;
  out.b_gas = o.b_gas;
  out.dirichlet_closure = o.dirichlet_closure;
  out.robin_closure = o.robin_closure;
  out.eb_order = o.eb_order == 1 ? 1 : 2;
  out.precision = o.precision;
  out.nu1 = o.nu1 > 0 ? o.nu1 : 2;
  out.nu2 = o.nu2 > 0 ? o.nu2 : 2;
  out.bottom_max = o.bottom_max_dof > 0 ? o.bottom_max_dof : 600;
  if (o.precision != EBMG_FP64 && o.precision != EBMG_MIXED) return EBMG_ERR_ARG;
  if (!(o.beta != 0.0) || !std::isfinite(o.beta)) return EBMG_ERR_ARG;
  if (o.krylov < 0 || o.krylov > 2 || o.smoother < 0 || o.smoother > 4 || o.tail < 0 || o.tail > 2 ||
      o.batch < 0 || o.batch > 2 || o.graphs < 0 || o.graphs > 1)
    return EBMG_ERR_ARG;
  for (int k = 0; k < 3; ++k)
    if (o.reserved[k] != 0) return EBMG_ERR_ARG;
  out.graphs = o.graphs;
  out.tail = o.tail;
  out.batch = o.batch == 1 ? 1 : 2;
  out.krylov = o.krylov == 0 ? (nobj > 0 ? 2 : 1) : o.krylov;
  out.smoother = o.smoother;
  return EBMG_OK;
}

// host part of a problem setup (no device work)
static void build_host_problem(ebmg::Problem& H, const ebmg_box* box, int nobj, const ebmg_object* objs,
                               const ebmg_domain_bc* bc) {
  using namespace ebmg;
  H.bc = *bc;
  for (int f = 0; f < 2 * box->dim && f < 6; ++f) {
    if (bc->kind[f] < 0 || bc->kind[f] > 2) throw ArgError("bad boundary kind");
    if (bc->kind[f] == EBMG_BC_ROBIN && !(bc->robin_a2[f] != 0.0)) throw ArgError("Robin a2 must be nonzero");
  }
  build_geometry(H.geo, *box, nobj, objs);
  H.bph[0] = H.opt.b_gas;
  H.aph[0] = H.opt.a_gas;
  if (H.geo.nphase == 2) {
    H.bph[1] = H.geo.obj_value[H.geo.diel_obj];
    H.aph[1] = H.opt.a_diel;
  } else {
    H.bph[1] = H.opt.b_gas;
    H.aph[1] = H.opt.a_diel;
  }
  if (!(H.bph[0] > 0) || !(H.bph[1] > 0)) throw ArgError("b must be positive");
  bool anchored = H.opt.alpha != 0.0;
  for (int f = 0; f < 2 * box->dim; ++f) anchored |= bc->kind[f] != EBMG_BC_NEUMANN;
  for (int k = 0; k < nobj; ++k) anchored |= objs[k].kind == EBMG_OBJ_ELECTRODE;
  if (!anchored) throw ArgError("pure Neumann problem is singular");
  build_fine_level(H);
  build_hierarchy(H);
}

ebmg_status ebmg_setup(ebmg_ctx ctx, const ebmg_box* box, int32_t nobj, const ebmg_object* objs,
                       const ebmg_domain_bc* bc, const ebmg_options* opt, ebmg_problem* out) {
  if (!ctx || !box || !bc || !out || (nobj > 0 && !objs) || nobj < 0 || nobj > 64) {
    if (ctx) ctx->err = "invalid argument to ebmg_setup";
    return EBMG_ERR_ARG;
  }
  *out = nullptr;
  return guard(ctx, [&]() -> ebmg_status {
    auto P = std::make_unique<ebmg_problem_s>();
    P->ctx = ctx;
    P->host = std::make_unique<Problem>();
    Problem& H = *P->host;
    if (parse_options(opt, nobj, H.opt) != EBMG_OK) throw ArgError("bad options");
    build_host_problem(H, box, nobj, objs, bc);
    if (ctx->device >= 0) {
      HIPCHECK(hipSetDevice(ctx->device));
      try {
        upload(P.get());
      } catch (...) {
        P->dev.release();
        throw;
      }
      P->on_device = true;
    }
    *out = P.release();
    ++ctx->refs;
    return EBMG_OK;
  });
}

ebmg_status ebmg_query(ebmg_problem pb, int64_t* n_cells, int64_t* n_phase2, int32_t* n_levels,
                       int64_t* device_bytes) {
  if (!pb) return EBMG_ERR_ARG;
  if (n_cells) *n_cells = pb->host->geo.N;
  if (n_phase2) *n_phase2 = pb->host->geo.N2;
  if (n_levels) *n_levels = (int32_t)pb->host->levels.size();
  if (device_bytes) *device_bytes = pb->dev.bytes;
  return EBMG_OK;
}

ebmg_status ebmg_query_level(ebmg_problem pb, int32_t level, int64_t* n_cells, int64_t* n_phase2) {
  if (!pb || level < 0 || level >= (int32_t)pb->host->levels.size()) return EBMG_ERR_ARG;
  if (n_cells) *n_cells = pb->host->levels[level].N;
  if (n_phase2) *n_phase2 = pb->host->levels[level].N2;
  return EBMG_OK;
}

ebmg_status ebmg_query_tuning(ebmg_problem pb, int32_t level, int32_t* fused, double* split_ms, double* fused_ms) {
  if (!pb || level < -1 || level >= (int32_t)pb->host->levels.size()) return EBMG_ERR_ARG;
  if (!pb->on_device) return EBMG_ERR_DEVICE;
  if (level == -1) {
    const DevProblem& D = pb->dev;
    if (fused) *fused = D.tail_l0;
    double tno = 0, tpick = 0;
    for (size_t k = 0; k < D.tail_cand.size(); ++k) {
      if (D.tail_cand[k] == -1) tno = D.tail_ms[k];
      if (D.tail_cand[k] == D.tail_l0) tpick = D.tail_ms[k];
    }
    if (split_ms) *split_ms = tno;
    if (fused_ms) *fused_ms = tpick;
    return EBMG_OK;
  }
  const DevLevel& l = pb->dev.lv[level];
  if (fused) *fused = l.fused ? (l.fvar ? 2 + l.zmcfg : 1) : (l.oop ? 2 + kZMConfigs : 0);
  if (split_ms) *split_ms = l.tune_split_ms;
  if (fused_ms) *fused_ms = l.fvar == 1 ? l.tune_zm_ms : l.tune_fused_ms;
  return EBMG_OK;
}

ebmg_status ebmg_export_level(ebmg_problem pb, int32_t level, uint8_t* tag, int8_t* primary, int64_t* sec_cell) {
  if (!pb || level < 0 || level >= (int32_t)pb->host->levels.size()) return EBMG_ERR_ARG;
  const Level& L = pb->host->levels[level];
  for (int64_t c = 0; c < L.N; ++c) {
    if (tag) tag[c] = L.tag[c];
    if (primary) primary[c] = L.primary[c];
  }
  if (sec_cell)
    for (int64_t s = 0; s < L.N2; ++s) sec_cell[s] = L.sec_cell[s];
  return EBMG_OK;
}

ebmg_status ebmg_export_geometry(ebmg_problem pb, double* kg, double* kd, int8_t* primary, int64_t* sec_cell) {
  if (!pb) return EBMG_ERR_ARG;
  const Geometry& G = pb->host->geo;
  for (int64_t c = 0; c < G.N; ++c) {
    if (kg) kg[c] = G.kappa(0, c);
    if (kd) kd[c] = G.kappa(1, c);
    if (primary) primary[c] = G.primary[c];
  }
  if (sec_cell)
    for (int64_t s = 0; s < G.N2; ++s) sec_cell[s] = G.sec_cell[s];
  return EBMG_OK;
}

ebmg_status ebmg_export_moments(ebmg_problem pb, int32_t phase, double* vcent, double* apert, double* foff,
                                double* eb_area, double* eb_cent, double* eb_normal) {
  if (!pb || phase < 0 || phase >= pb->host->geo.nphase) return EBMG_ERR_ARG;
  return guard(pb->ctx, [&]() -> ebmg_status {
    const Geometry& G = pb->host->geo;
    const Grid& g = G.g;
    const int dim = g.dim;
    const int nz = dim == 3 ? g.n[2] : 1;
    for (int k = 0; k < nz; ++k)
      for (int j = 0; j < g.n[1]; ++j)
        for (int i = 0; i < g.n[0]; ++i) {
          const int64_t c = g.cell(i, j, k);
          const int ijk[3] = {i, j, k};
          const CellCut* cc = G.cut(phase, c);
          const bool has = G.has(phase, c);
          for (int d = 0; d < dim; ++d) {
            if (vcent) vcent[d * G.N + c] = !has ? 0.0 : (cc ? cc->vc[d] : g.centre(d, ijk[d]));
            if (eb_cent) eb_cent[d * G.N + c] = cc && cc->eb_area > 0 ? cc->eb_c[d] : 0.0;
            if (eb_normal) eb_normal[d * G.N + c] = cc && cc->eb_area > 0 ? cc->eb_n[d] : 0.0;
          }
          if (eb_area) eb_area[c] = cc ? cc->eb_area : 0.0;
        }
    int64_t base = 0;
    for (int d = 0; d < dim; ++d) {
      const int m0 = g.n[0] + (d == 0), m1 = g.n[1] + (d == 1), m2 = dim == 3 ? g.n[2] + (d == 2) : 1;
      for (int k = 0; k < m2; ++k)
        for (int j = 0; j < m1; ++j)
          for (int i = 0; i < m0; ++i) {
            const int c[3] = {i, j, k};
            const int64_t f = base + i + (int64_t)m0 * (j + (int64_t)m1 * k);
            if (apert) apert[f] = G.alpha(phase, d, c);
            if (foff) {
              double off[2];
              G.face_off(phase, d, c, off);
              for (int q = 0; q < dim - 1; ++q) foff[(dim - 1) * f + q] = off[q];
            }
          }
      base += (int64_t)m0 * m1 * m2;
    }
    return EBMG_OK;
  });
}

ebmg_status ebmg_export_operator(ebmg_problem pb, int32_t level, int64_t* nnz, int64_t* row_ptr, int64_t* cols,
                                 double* vals) {
  if (!pb || !nnz || level < 0 || level >= (int32_t)pb->host->levels.size()) return EBMG_ERR_ARG;
  return guard(pb->ctx, [&]() -> ebmg_status {
    const Level& L = pb->host->levels[level];
    const int64_t n = L.N + L.N2;
    std::vector<std::pair<int64_t, double>> buf;
    int64_t cnt = 0;
    if (row_ptr) row_ptr[0] = 0;
    for (int64_t q = 0; q < n; ++q) {
      const int64_t cell = q < L.N ? q : L.sec_cell[q - L.N];
      if (q < L.N && L.primary[cell] < 0) {
        buf.assign(1, {q, 1.0});
      } else {
        double m;
        L.row(q, m, buf);
        bool found = false;
        for (auto& e : buf)
          if (e.first == q) {
            e.second += m;
            found = true;
          }
        if (!found) buf.emplace_back(q, m);
      }
      if (row_ptr) {
        for (auto& e : buf) {
          cols[cnt] = e.first;
          vals[cnt] = e.second;
          ++cnt;
        }
        row_ptr[q + 1] = cnt;
      } else {
        cnt += (int64_t)buf.size();
      }
    }
    *nnz = cnt;
    return EBMG_OK;
  });
}

ebmg_status ebmg_export_rhs(ebmg_problem pb, const double* rho, const double* sigma, const double* bcv,
                            const double* objv, double* b) {
  if (!pb || !rho || !b) return EBMG_ERR_ARG;
  return guard(pb->ctx, [&]() -> ebmg_status {
    host_rhs(*pb->host, rho, sigma, bcv, objv, b);
    return EBMG_OK;
  });
}

ebmg_status ebmg_solve(ebmg_problem pb, const double* rho, const double* sigma, const double* bcv, const double* objv,
                       double rtol, int32_t max_cycles, double* phi, double* phi2, double* E, ebmg_solve_info* info) {
  if (!pb) return EBMG_ERR_ARG;
  ebmg_ctx ctx = pb->ctx;
  if (!rho || !phi || !(rtol > 0) || max_cycles < 0) {
    ctx->err = "invalid argument to ebmg_solve";
    return EBMG_ERR_ARG;
  }
  if (!pb->on_device) {
    ctx->err = "problem is not on a device (host-only context)";
    return EBMG_ERR_DEVICE;
  }
  return guard(ctx, [&]() -> ebmg_status {
    drain(pb);
    HIPCHECK(hipSetDevice(ctx->device));
    return solve(pb, rho, sigma, bcv, objv, rtol, max_cycles, phi, phi2, E, info);
  });
}

ebmg_status ebmg_submit(ebmg_problem pb, const double* rho, const double* sigma, const double* bcv,
                        const double* objv, double rtol, int32_t max_cycles, double* phi, double* phi2, double* E,
                        uint64_t* ticket) {
  if (!pb) return EBMG_ERR_ARG;
  ebmg_ctx ctx = pb->ctx;
  if (!rho || !phi || !ticket || !(rtol > 0) || max_cycles < 0) {
    ctx->err = "invalid argument to ebmg_submit";
    return EBMG_ERR_ARG;
  }
  if (!pb->on_device) {
    ctx->err = "problem is not on a device (host-only context)";
    return EBMG_ERR_DEVICE;
  }
  return guard(ctx, [&]() -> ebmg_status {
    AsyncJob j;
    j.pb = pb;
    j.rho = rho;
    j.sigma = sigma;
    if (bcv) j.bcv.assign(bcv, bcv + 6);
    const size_t no = pb->host->geo.obj_value.size();
    if (objv && no) j.objv.assign(objv, objv + no);
    j.rtol = rtol;
    j.max_cycles = max_cycles;
    j.phi = phi;
    j.phi2 = phi2;
    j.E = E;
    {
      std::lock_guard<std::mutex> lk(ctx->mu);
      if (!ctx->worker.joinable()) ctx->worker = std::thread(async_worker, ctx);
      j.ticket = ctx->next_ticket++;
      ctx->results.emplace(j.ticket, AsyncResult{});
      ++pb->pending;
      *ticket = j.ticket;
      ctx->queue.push_back(std::move(j));
    }
    ctx->cv_work.notify_one();
    return EBMG_OK;
  });
}

// Shared by poll and wait: hand over a finished ticket's outcome and forget it.
static ebmg_status take_result(ebmg_ctx ctx, uint64_t ticket, bool block, int32_t* done, ebmg_status* result,
                               ebmg_solve_info* info) {
  std::unique_lock<std::mutex> lk(ctx->mu);
  // looked up again after every wake: a submit in between may rehash the map
  auto it = ctx->results.find(ticket);
  if (block)
    ctx->cv_done.wait(lk, [&] {
      it = ctx->results.find(ticket);
      return it == ctx->results.end() || it->second.done;
    });
  if (it == ctx->results.end()) {
    ctx->err = "unknown or already collected ticket " + std::to_string(ticket);
    return EBMG_ERR_ARG;
  }
  if (done) *done = it->second.done ? 1 : 0;
  if (!it->second.done) return EBMG_OK;
  *result = it->second.status;
  if (info) *info = it->second.info;
  if (it->second.status != EBMG_OK) ctx->err = it->second.err;
  ctx->results.erase(it);
  return EBMG_OK;
}

ebmg_status ebmg_poll(ebmg_ctx ctx, uint64_t ticket, int32_t* done, ebmg_status* result, ebmg_solve_info* info) {
  if (!ctx || !done || !result) return EBMG_ERR_ARG;
  return take_result(ctx, ticket, false, done, result, info);
}

ebmg_status ebmg_wait(ebmg_ctx ctx, uint64_t ticket, ebmg_status* result, ebmg_solve_info* info) {
  if (!ctx || !result) return EBMG_ERR_ARG;
  return take_result(ctx, ticket, true, nullptr, result, info);
}

ebmg_status ebmg_apply(ebmg_problem pb, const double* phi, const double* phi2, double* out, double* out2) {
  if (!pb || !phi || !out) return EBMG_ERR_ARG;
  if (!pb->on_device) return EBMG_ERR_DEVICE;
  return guard(pb->ctx, [&]() -> ebmg_status {
    drain(pb);
    HIPCHECK(hipSetDevice(pb->ctx->device));
    DevLevel& L = pb->dev.lv[0];
    hipStream_t s = pb->ctx->stream;
    HIPCHECK(hipMemcpyAsync(L.x64.p, phi, sizeof(double) * L.N, hipMemcpyDeviceToDevice, s));
    if (L.N2 > 0) {
      if (!phi2 || !out2) throw ArgError("second-phase arrays required");
      HIPCHECK(hipMemcpyAsync(L.x64.p + L.N, phi2, sizeof(double) * L.N2, hipMemcpyDeviceToDevice, s));
    }
    residual<double, 1>(L, L.x64.p, nullptr, L.r64.p, s);
    HIPCHECK(hipMemcpyAsync(out, L.r64.p, sizeof(double) * L.N, hipMemcpyDeviceToDevice, s));
    if (L.N2 > 0) HIPCHECK(hipMemcpyAsync(out2, L.r64.p + L.N, sizeof(double) * L.N2, hipMemcpyDeviceToDevice, s));
    HIPCHECK(hipStreamSynchronize(s));
    return EBMG_OK;
  });
}

ebmg_status ebmg_apply_noalloc(ebmg_problem pb, const double* phi, const double* phi2, double* out,
                               double* out2) {
  if (!pb || !phi || !out) return EBMG_ERR_ARG;
  if (!pb->on_device) return EBMG_ERR_DEVICE;
  return guard(pb->ctx, [&]() -> ebmg_status {
    DevLevel& L = pb->dev.lv[0];
    const int64_t nd = L.N + L.N2;
    if (nd > kNoAllocMax) throw ArgError("ebmg_apply_noalloc: N + N2 exceeds its scratch of 1179648 unknowns");
    if (L.N2 > 0 && (!phi2 || !out2)) throw ArgError("second-phase arrays required");
    drain(pb);
    HIPCHECK(hipSetDevice(pb->ctx->device));
    double* sp = nullptr;
    HIPCHECK(scratch_ptr(pb->ctx->device, &sp));
    double* xs = sp;                  // staged [phi; phi2]
    double* rs = sp + kNoAllocMax;    // staged [out; out2]
    hipStream_t s = pb->ctx->stream;
    hipLaunchKernelGGL((k_convert<double, double>), dim3(nblk(L.N)), dim3(kBlock), 0, s, phi, xs, L.N);
    if (L.N2 > 0)
      hipLaunchKernelGGL((k_convert<double, double>), dim3(nblk(L.N2)), dim3(kBlock), 0, s, phi2, xs + L.N, L.N2);
    // every entry of rs is written: covered cells, template cells, explicit rows
    residual<double, 1>(L, xs, nullptr, rs, s);
    hipLaunchKernelGGL((k_convert<double, double>), dim3(nblk(L.N)), dim3(kBlock), 0, s, rs, out, L.N);
    if (L.N2 > 0)
      hipLaunchKernelGGL((k_convert<double, double>), dim3(nblk(L.N2)), dim3(kBlock), 0, s, rs + L.N, out2, L.N2);
    HIPCHECK(hipGetLastError());
    return EBMG_OK;
  });
}

ebmg_status ebmg_efield(ebmg_problem pb, const double* phi, const double* phi2, const double* sigma,
                        const double* bcv, const double* objv, double* E) {
  if (!pb || !phi || !E) return EBMG_ERR_ARG;
  if (!pb->on_device) return EBMG_ERR_DEVICE;
  return guard(pb->ctx, [&]() -> ebmg_status {
    drain(pb);
    HIPCHECK(hipSetDevice(pb->ctx->device));
    DevProblem& D = pb->dev;
    DevLevel& L = D.lv[0];
    hipStream_t s = pb->ctx->stream;
    const Problem& H = *pb->host;
    const size_t no = H.geo.obj_value.size();
    std::vector<double> ov(std::max<size_t>(1, no), 0.0);
    for (size_t k = 0; k < no; ++k) ov[k] = objv ? objv[k] : H.geo.obj_value[k];
    HIPCHECK(hipMemcpyAsync(D.objv.p, ov.data(), sizeof(double) * ov.size(), hipMemcpyHostToDevice, s));
    HIPCHECK(hipMemcpyAsync(L.x64.p, phi, sizeof(double) * L.N, hipMemcpyDeviceToDevice, s));
    if (L.N2 > 0) {
      if (!phi2) throw ArgError("second-phase array required");
      HIPCHECK(hipMemcpyAsync(L.x64.p + L.N, phi2, sizeof(double) * L.N2, hipMemcpyDeviceToDevice, s));
    }
    efield(pb, L.x64.p, sigma, bcv, E);
    HIPCHECK(hipStreamSynchronize(s));
    return EBMG_OK;
  });
}

ebmg_status ebmg_smooth(ebmg_problem pb, int32_t level, int32_t variant, int32_t sweeps, double* x,
                        const double* b) {
  if (!pb || !x || !b || sweeps < 0 || variant < 1 || variant > 5 + kZMConfigs) return EBMG_ERR_ARG;
  if (!pb->on_device) return EBMG_ERR_DEVICE;
  if (level < 0 || level >= (int32_t)pb->dev.lv.size()) return EBMG_ERR_ARG;
  return guard(pb->ctx, [&]() -> ebmg_status {
    drain(pb);
    HIPCHECK(hipSetDevice(pb->ctx->device));
    DevLevel& L = pb->dev.lv[level];
    hipStream_t s = pb->ctx->stream;
    const bool mixed = pb->host->opt.precision == EBMG_MIXED;
    if (variant > 1 && (mixed ? !L.xa32.p : !L.xa64.p)) throw ArgError("this level has no second vector");
    if (variant > 1 && variant < 3 + kZMConfigs && !fused_ok(L)) throw ArgError("this level has no fused sweep");
    if (variant >= 3 && variant < 3 + kZMConfigs && L.dim != 3) throw ArgError("the z-marching sweep is 3D only");
    if (variant >= 3 && variant < 3 + kZMConfigs && !zm_cfg_ok(L, variant - 3))
      throw ArgError("the wide-fetch sweep needs an x extent that is a multiple of 4");
    const int64_t nd = L.N + L.N2;
    if (mixed) {
      hipLaunchKernelGGL((k_convert<double, float>), dim3(nblk(nd)), dim3(kBlock), 0, s, x, L.x32.p, nd);
      hipLaunchKernelGGL((k_convert<double, float>), dim3(nblk(nd)), dim3(kBlock), 0, s, b, L.b32.p, nd);
      template_sweeps<float>(L, variant, sweeps, L.x32.p, L.b32.p, s);
      hipLaunchKernelGGL((k_convert<float, double>), dim3(nblk(nd)), dim3(kBlock), 0, s, L.x32.p, x, nd);
    } else {
      template_sweeps<double>(L, variant, sweeps, x, b, s);
    }
    HIPCHECK(hipGetLastError());
    HIPCHECK(hipStreamSynchronize(s));
    return EBMG_OK;
  });
}

ebmg_status ebmg_restrict_residual(ebmg_problem pb, int32_t level, int32_t form, const double* x, const double* b,
                                   double* bc) {
  if (!pb || !x || !b || !bc || form < 0 || form > 2) return EBMG_ERR_ARG;
  if (!pb->on_device) return EBMG_ERR_DEVICE;
  if (level < 0 || level + 1 >= (int32_t)pb->dev.lv.size()) return EBMG_ERR_ARG;
  return guard(pb->ctx, [&]() -> ebmg_status {
    drain(pb);
    HIPCHECK(hipSetDevice(pb->ctx->device));
    DevLevel& F = pb->dev.lv[level];
    DevLevel& C = pb->dev.lv[level + 1];
    hipStream_t s = pb->ctx->stream;
    const bool mixed = pb->host->opt.precision == EBMG_MIXED;
    const int64_t nf = F.N + F.N2, nc = C.N + C.N2;
    if (mixed) {
      if (!F.x32.p || !F.b32.p || !C.b32.p || !C.x32.p || !F.r32.p) throw ArgError("no FP32 vectors on these levels");
      hipLaunchKernelGGL((k_convert<double, float>), dim3(nblk(nf)), dim3(kBlock), 0, s, x, F.x32.p, nf);
      hipLaunchKernelGGL((k_convert<double, float>), dim3(nblk(nf)), dim3(kBlock), 0, s, b, F.b32.p, nf);
      residual_restrict<float>(F, C, F.x32.p, F.b32.p, s, form);
      hipLaunchKernelGGL((k_convert<float, double>), dim3(nblk(nc)), dim3(kBlock), 0, s, C.b32.p, bc, nc);
    } else {
      if (!F.x64.p || !F.b64.p || !C.b64.p || !C.x64.p || !F.r64.p) throw ArgError("no FP64 vectors on these levels");
      HIPCHECK(hipMemcpyAsync(F.x64.p, x, sizeof(double) * nf, hipMemcpyDeviceToDevice, s));
      HIPCHECK(hipMemcpyAsync(F.b64.p, b, sizeof(double) * nf, hipMemcpyDeviceToDevice, s));
      residual_restrict<double>(F, C, F.x64.p, F.b64.p, s, form);
      HIPCHECK(hipMemcpyAsync(bc, C.b64.p, sizeof(double) * nc, hipMemcpyDeviceToDevice, s));
    }
    HIPCHECK(hipGetLastError());
    HIPCHECK(hipStreamSynchronize(s));
    return EBMG_OK;
  });
}

ebmg_status ebmg_time_kernel(ebmg_problem pb, int32_t which, int32_t level, int32_t reps, double* avg_ms,
                             double* alg_bytes) {
  if (!pb || !avg_ms || reps <= 0) return EBMG_ERR_ARG;
  if (!pb->on_device) return EBMG_ERR_DEVICE;
  if (level < 0 || level >= (int32_t)pb->dev.lv.size()) return EBMG_ERR_ARG;
  return guard(pb->ctx, [&]() -> ebmg_status {
    drain(pb);
    HIPCHECK(hipSetDevice(pb->ctx->device));
    DevProblem& D = pb->dev;
    DevLevel& L = D.lv[level];
    hipStream_t s = pb->ctx->stream;
    const bool mixed = pb->host->opt.precision == EBMG_MIXED;
    const int64_t nd = L.N + L.N2;
    const int64_t nreg_half = (L.N + 1) / 2;
    hipEvent_t e0, e1;
    HIPCHECK(hipEventCreate(&e0));
    HIPCHECK(hipEventCreate(&e1));
    double bytes = 0;
    const Shape shh = shape3((L.n[0] + 1) / 2, L.n[1], L.dim == 3 ? L.n[2] : 1);
    const Shape shf = shape3(L.n[0], L.n[1], L.dim == 3 ? L.n[2] : 1);
    if (which < 0 || which > 5) throw ArgError("unknown kernel id");
    if (which == 5) {
      // reference stream with the fused sweep's bytes per cell over the
      // level's arrays
      auto al = [](const void* p, size_t es) { return (uintptr_t)p % (4 * es) == 0; };
      const bool ok = mixed ? (L.xa32.p && al(L.x32.p, 4) && al(L.xa32.p, 4) && al(L.b32.p, 4))
                            : (L.xa64.p && al(L.x64.p, 8) && al(L.xa64.p, 8) && al(L.b64.p, 8));
      if (!ok || L.N % 4 != 0 || !al(L.tag.p, 1)) throw ArgError("the reference stream needs N a multiple of 4");
      const unsigned g = (unsigned)std::min<int64_t>(8192, (L.N / 4 + 255) / 256);
      auto go = [&](int r) {
        if (mixed)
          hipLaunchKernelGGL((k_stream_ref<float>), dim3(g), dim3(256), 0, s, L.tag.p, (r & 1) ? L.xa32.p : L.x32.p,
                             L.b32.p, (r & 1) ? L.x32.p : L.xa32.p, L.N);
        else
          hipLaunchKernelGGL((k_stream_ref<double>), dim3(g), dim3(256), 0, s, L.tag.p, (r & 1) ? L.xa64.p : L.x64.p,
                             L.b64.p, (r & 1) ? L.x64.p : L.xa64.p, L.N);
      };
      go(0);
      go(1);
      HIPCHECK(hipEventRecord(e0, s));
      for (int r = 0; r < reps; ++r) go(r);
      HIPCHECK(hipEventRecord(e1, s));
      HIPCHECK(hipEventSynchronize(e1));
      HIPCHECK(hipGetLastError());
      float ms = 0;
      HIPCHECK(hipEventElapsedTime(&ms, e0, e1));
      (void)hipEventDestroy(e0);
      (void)hipEventDestroy(e1);
      *avg_ms = ms / reps;
      if (alg_bytes) *alg_bytes = (double)L.N * (3.0 * (mixed ? 4 : 8) + 1.0);
      return EBMG_OK;
    }
    if (which >= 3 && (mixed ? !L.xa32.p : !L.xa64.p)) throw ArgError("this level has no fused sweep");
    if (which == 4 && L.dim != 3) throw ArgError("the z-marching sweep is 3D only");
    const bool fz = (which == 0 && L.fused) || which == 3 || which == 4;
    auto launch = [&](int colour) {
      if (fz) {
        if (mixed) {
          float* xi = (colour & 1) ? L.xa32.p : L.x32.p;
          float* xo = (colour & 1) ? L.x32.p : L.xa32.p;
          if (which == 4)
            launch_zm<float>(L, xi, xo, L.b32.p, L.t32, s);
          else
            launch_fused<float>(L, xi, xo, L.b32.p, L.t32, s);
        } else {
          double* xi = (colour & 1) ? L.xa64.p : L.x64.p;
          double* xo = (colour & 1) ? L.x64.p : L.xa64.p;
          if (which == 4)
            launch_zm<double>(L, xi, xo, L.b64.p, L.t64, s);
          else
            launch_fused<double>(L, xi, xo, L.b64.p, L.t64, s);
        }
        return;
      }
      if (which != 1) {
        if (mixed) {
          if (L.dim == 3)
            hipLaunchKernelGGL((k_rb<float, 3>), shh.g, shh.b, 0, s, L.tag.p, L.x32.p, L.b32.p, L.t32, colour);
          else
            hipLaunchKernelGGL((k_rb<float, 2>), shh.g, shh.b, 0, s, L.tag.p, L.x32.p, L.b32.p, L.t32, colour);
        } else {
          if (L.dim == 3)
            hipLaunchKernelGGL((k_rb<double, 3>), shh.g, shh.b, 0, s, L.tag.p, L.x64.p, L.b64.p, L.t64, colour);
          else
            hipLaunchKernelGGL((k_rb<double, 2>), shh.g, shh.b, 0, s, L.tag.p, L.x64.p, L.b64.p, L.t64, colour);
        }
      } else {
        if (pair_ok(L)) {
          hipLaunchKernelGGL((k_resid_zp3<double, 0>), dim3((unsigned)zp_resid_blocks(L)), dim3(64, kRPY), 0, s,
                             L.tag.p, L.x64.p, L.b64.p, L.r64.p, L.t64);
        } else if (L.dim == 3 && L.N >= kResidZMMin) {
          const dim3 g((unsigned)zm_resid_blocks(L));
          hipLaunchKernelGGL((k_resid_zm3<double, 0>), g, dim3(kRZX, kRZY), 0, s, L.tag.p, L.x64.p, L.b64.p,
                             L.r64.p, L.t64);
        } else if (L.dim == 3) {
          hipLaunchKernelGGL((k_resid_reg<double, 3, 0>), shf.g, shf.b, 0, s, L.tag.p, L.x64.p, L.b64.p, L.r64.p, L.t64);
        } else {
          hipLaunchKernelGGL((k_resid_reg<double, 2, 0>), shf.g, shf.b, 0, s, L.tag.p, L.x64.p, L.b64.p, L.r64.p, L.t64);
        }
      }
    };
    if (which == 1 && !L.x64.p) throw ArgError("no FP64 vectors on this level");
    if (which != 1) {
      // algorithmic bytes of one half-sweep: each updated cell reads x and b,
      // writes x, reads its tag
      const int es = mixed ? 4 : 8;
      // half-sweep: the cells of one colour; fused sweep: every cell
      bytes = (fz ? (double)L.N : (double)nreg_half) * (3.0 * es + 1.0);
      if (mixed) {
        fill<float>(L.x32.p, nd, 0.0f, s);
        fill<float>(L.b32.p, nd, 0.0f, s);
        if (L.xa32.p) fill<float>(L.xa32.p, nd, 0.0f, s);
      } else {
        if (L.xa64.p) fill<double>(L.xa64.p, nd, 0.0, s);
        fill<double>(L.x64.p, nd, 0.0, s);
        fill<double>(L.b64.p, nd, 0.0, s);
      }
    } else {
      bytes = (double)L.N * (3.0 * 8 + 1.0);
      fill<double>(L.x64.p, nd, 0.0, s);
      fill<double>(L.b64.p, nd, 0.0, s);
    }
    launch(0);
    launch(1);
    HIPCHECK(hipEventRecord(e0, s));
    for (int r = 0; r < reps; ++r) launch(r & 1);
    HIPCHECK(hipEventRecord(e1, s));
    HIPCHECK(hipEventSynchronize(e1));
    HIPCHECK(hipGetLastError());
    float ms = 0;
    HIPCHECK(hipEventElapsedTime(&ms, e0, e1));
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    *avg_ms = ms / reps;
    if (alg_bytes) *alg_bytes = bytes;
    return EBMG_OK;
  });
}

ebmg_status ebmg_kernel_timing(ebmg_problem pb, int32_t which, int32_t level, int32_t enable, int64_t* launches,
                               double* mean_ms, double* alg_bytes) {
  if (!pb || (enable != 0 && enable != 1) || (which != 0 && which != 1)) return EBMG_ERR_ARG;
  if (!pb->on_device) return EBMG_ERR_DEVICE;
  if (level < 0 || level >= (int32_t)pb->dev.lv.size()) return EBMG_ERR_ARG;
  return guard(pb->ctx, [&]() -> ebmg_status {
    drain(pb);
    DevProblem& D = pb->dev;
    DevLevel& L = D.lv[level];
    std::unique_ptr<KTiming>& K = D.kt[which];
    auto slot = [&](DevLevel& l) -> KTiming*& { return which == 0 ? l.kt : l.ktr; };
    if (enable) {
      if (K && D.kt_level[which] >= 0) slot(D.lv[D.kt_level[which]]) = nullptr;
      K.reset(new KTiming());
      D.kt_level[which] = level;
      slot(L) = K.get();
      return EBMG_OK;
    }
    if (!K || D.kt_level[which] != level) throw ArgError("kernel timing is not enabled on this level");
    HIPCHECK(hipSetDevice(pb->ctx->device));
    HIPCHECK(hipStreamSynchronize(pb->ctx->stream));
    K->harvest();
    const int es = which == 1 ? 8 : (pb->host->opt.precision == EBMG_MIXED ? 4 : 8);
    const double cells = (which == 1 || L.fused) ? (double)L.N : (double)((L.N + 1) / 2);
    if (launches) *launches = K->n;
    if (mean_ms) *mean_ms = K->n > 0 ? K->ms / (double)K->n : 0.0;
    if (alg_bytes) *alg_bytes = cells * (3.0 * es + 1.0);
    slot(L) = nullptr;
    K.reset();
    D.kt_level[which] = -1;
    return EBMG_OK;
  });
}

ebmg_status ebmg_setup_batch(ebmg_ctx ctx, int32_t nbox, const ebmg_box* boxes, const int32_t* nobj,
                             const ebmg_object* const* objs, const ebmg_domain_bc* bcs, const ebmg_options* opts,
                             ebmg_batch* out) {
  if (!ctx || nbox <= 0 || !boxes || !nobj || !objs || !bcs || !out) {
    if (ctx) ctx->err = "invalid argument to ebmg_setup_batch";
    return EBMG_ERR_ARG;
  }
  *out = nullptr;
  if (ctx->device < 0) {
    ctx->err = "batched solves need a device context";
    return EBMG_ERR_DEVICE;
  }
  return guard(ctx, [&]() -> ebmg_status {
    auto Bt = std::make_unique<ebmg_batch_s>();
    Bt->ctx = ctx;
    Bt->dim = boxes[0].dim;
    Bt->boxes.resize(nbox);
    int prec = -1;
    for (int i = 0; i < nbox; ++i) {
      if (boxes[i].dim != Bt->dim) throw ArgError("all boxes of a batch must have the same dimension");
      if (nobj[i] < 0 || nobj[i] > 64 || (nobj[i] > 0 && !objs[i])) throw ArgError("bad object list");
      auto P = std::make_unique<ebmg_problem_s>();
      P->ctx = ctx;
      P->host = std::make_unique<Problem>();
      if (parse_options(opts ? &opts[i] : nullptr, nobj[i], P->host->opt) != EBMG_OK)
        throw ArgError("bad options for a batch box");
      if (prec < 0) prec = P->host->opt.precision;
      if (P->host->opt.precision != prec) throw ArgError("all boxes of a batch must use one precision");
      if (i == 0) {
        Bt->mode = P->host->opt.batch;
        Bt->graphs = P->host->opt.graphs == 0;
      }
      if (P->host->opt.batch != Bt->mode) throw ArgError("all boxes of a batch must use one batch mode");
      Bt->boxes[i] = std::move(P);
    }
    Bt->mixed = prec == EBMG_MIXED;
    Bt->nu1 = Bt->boxes[0]->host->opt.nu1;
    Bt->nu2 = Bt->boxes[0]->host->opt.nu2;
    Bt->tail_opt = Bt->boxes[0]->host->opt.tail;
    // host setup of the boxes in parallel (independent problems)
    unsigned nw = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
    std::vector<std::string> errs(nbox);
    std::vector<int> kinds(nbox, 0);
    std::atomic<int> next(0);
    auto work = [&]() {
      for (int i = next++; i < nbox; i = next++) {
        try {
          build_host_problem(*Bt->boxes[i]->host, &boxes[i], nobj[i], objs[i], &bcs[i]);
        } catch (const ArgError& e) {
          errs[i] = e.what();
          kinds[i] = 1;
        } catch (const GeomError& e) {
          errs[i] = e.what();
          kinds[i] = 2;
        } catch (const std::exception& e) {
          errs[i] = e.what();
          kinds[i] = 1;
        }
      }
    };
    std::vector<std::thread> th;
    for (unsigned w = 0; w < nw; ++w) th.emplace_back(work);
    for (auto& t : th) t.join();
    for (int i = 0; i < nbox; ++i) {
      if (kinds[i] == 1) throw ArgError("box " + std::to_string(i) + ": " + errs[i]);
      if (kinds[i] == 2) throw GeomError("box " + std::to_string(i) + ": " + errs[i]);
    }
    HIPCHECK(hipSetDevice(ctx->device));
    hipStream_t s = ctx->stream;
    try {
      for (int i = 0; i < nbox; ++i) {
        ebmg_problem_s* P = Bt->boxes[i].get();
        upload(P, true);
        P->on_device = true;
        // object values for the right-hand side
        const auto& ov = P->host->geo.obj_value;
        if (!ov.empty()) {
          HIPCHECK(hipMemcpyAsync(P->dev.objv.p, ov.data(), sizeof(double) * ov.size(), hipMemcpyHostToDevice, s));
          HIPCHECK(hipStreamSynchronize(s));
        }
        Bt->cells += P->host->geo.N;
        Bt->cells2 += P->host->geo.N2;
        Bt->bytes += P->dev.bytes;
      }
      if (Bt->mixed)
        upload_batch_views<float>(Bt.get(), s);
      else
        upload_batch_views<double>(Bt.get(), s);
      if (Bt->mode == 2) {
        if (Bt->mixed)
          setup_wide<float>(Bt.get(), s);
        else
          setup_wide<double>(Bt.get(), s);
      }
      std::vector<int32_t> order(nbox);
      for (int i = 0; i < nbox; ++i) order[i] = i;
      std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
        return Bt->boxes[a]->host->geo.N + Bt->boxes[a]->host->geo.N2 >
               Bt->boxes[b]->host->geo.N + Bt->boxes[b]->host->geo.N2;
      });
      int64_t by = 0;
      Bt->order.upload(order.data(), nbox, s, by);
      Bt->bio.alloc((int64_t)(nbox * sizeof(BIO)), by);
      Bt->bres.alloc((int64_t)(nbox * sizeof(BRes)), by);
      Bt->bytes += by;
      HIPCHECK(hipStreamSynchronize(s));
    } catch (...) {
      for (auto& P : Bt->boxes)
        if (P) P->dev.release();
      for (auto& b : Bt->lvbuf) b.release();
      Bt->bbox.release();
      Bt->order.release();
      Bt->bio.release();
      Bt->bres.release();
      release_wide(Bt.get());
      throw;
    }
    *out = Bt.release();
    ++ctx->refs;
    return EBMG_OK;
  });
}

ebmg_status ebmg_query_batch(ebmg_batch bt, int64_t* cells, int64_t* cells2, int64_t* device_bytes) {
  if (!bt) return EBMG_ERR_ARG;
  if (cells) *cells = bt->cells;
  if (cells2) *cells2 = bt->cells2;
  if (device_bytes) *device_bytes = bt->bytes;
  return EBMG_OK;
}

ebmg_status ebmg_query_batch_box(ebmg_batch bt, int32_t box, int64_t* n_cells, int64_t* n_phase2) {
  if (!bt || box < 0 || box >= (int32_t)bt->boxes.size()) return EBMG_ERR_ARG;
  const ebmg::Geometry& G = bt->boxes[box]->host->geo;
  if (n_cells) *n_cells = G.N;
  if (n_phase2) *n_phase2 = G.N2;
  return EBMG_OK;
}

ebmg_status ebmg_query_batch_tuning(ebmg_batch bt, int32_t* mode, int32_t* tail_cells, int32_t* wide_levels,
                                    int32_t* ncand, int32_t* cand_cells, double* cand_ms) {
  if (!bt) return EBMG_ERR_ARG;
  if (mode) *mode = bt->mode;
  if (tail_cells) *tail_cells = bt->tail_cells;
  if (wide_levels) *wide_levels = (int32_t)bt->wide.size();
  const int nc = std::min<int>(8, (int)bt->cand_cells.size());
  if (ncand) *ncand = nc;
  for (int k = 0; k < nc; ++k) {
    if (cand_cells) cand_cells[k] = bt->cand_cells[k];
    if (cand_ms) cand_ms[k] = bt->cand_ms[k];
  }
  return EBMG_OK;
}

ebmg_status ebmg_solve_batch(ebmg_batch bt, const double* const* rho, const double* const* sigma, double rtol,
                             int32_t max_cycles, double* const* phi, double* const* phi2, ebmg_solve_info* infos) {
  if (!bt || !rho || !phi || !(rtol > 0) || max_cycles < 0) {
    if (bt) bt->ctx->err = "invalid argument to ebmg_solve_batch";
    return EBMG_ERR_ARG;
  }
  const int nbox = (int)bt->boxes.size();
  for (int i = 0; i < nbox; ++i)
    if (!rho[i] || !phi[i] || (bt->boxes[i]->host->geo.N2 > 0 && phi2 && !phi2[i])) {
      bt->ctx->err = "missing array in ebmg_solve_batch";
      return EBMG_ERR_ARG;
    }
  return guard(bt->ctx, [&]() -> ebmg_status {
    auto t0 = std::chrono::steady_clock::now();
    HIPCHECK(hipSetDevice(bt->ctx->device));
    hipStream_t s = bt->ctx->stream;
    std::vector<BIO> io(nbox);
    for (int i = 0; i < nbox; ++i) {
      io[i].rho = rho[i];
      io[i].sigma = sigma ? sigma[i] : nullptr;
      io[i].phi = phi[i];
      io[i].phi2 = phi2 ? phi2[i] : nullptr;
    }
    if (bt->mode == 2) {
      std::vector<WIO> wio(nbox);
      for (int i = 0; i < nbox; ++i) wio[i] = WIO{io[i].rho, io[i].sigma, io[i].phi, io[i].phi2};
      std::vector<WState> st;
      if (bt->mixed) {
        if (bt->dim == 3)
          wide_solve<float, 3>(bt, wio, rtol, max_cycles, st, s);
        else
          wide_solve<float, 2>(bt, wio, rtol, max_cycles, st, s);
      } else {
        if (bt->dim == 3)
          wide_solve<double, 3>(bt, wio, rtol, max_cycles, st, s);
        else
          wide_solve<double, 2>(bt, wio, rtol, max_cycles, st, s);
      }
      const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
      ebmg_status worst = EBMG_OK;
      for (int i = 0; i < nbox; ++i) {
        if (infos) {
          std::memset(&infos[i], 0, sizeof(ebmg_solve_info));
          infos[i].cycles = st[i].cycles;
          infos[i].outer_iters = st[i].iters;
          infos[i].levels = (int)bt->boxes[i]->dev.lv.size();
          infos[i].r0_norm = st[i].bn;
          infos[i].rel_residual = st[i].rel;
          infos[i].seconds = secs;
          infos[i].est_bytes = box_bytes(bt->boxes[i].get(), st[i].cycles, st[i].iters);
        }
        if (st[i].status != EBMG_OK && worst == EBMG_OK) worst = (ebmg_status)st[i].status;
      }
      return worst;
    }
    HIPCHECK(hipMemcpyAsync(bt->bio.p, io.data(), sizeof(BIO) * nbox, hipMemcpyHostToDevice, s));
    int ncu = 256;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, bt->ctx->device) == hipSuccess && prop.multiProcessorCount > 0)
      ncu = prop.multiProcessorCount;
    const int grid = std::min(nbox, 2 * ncu);
    if (bt->mixed) {
      if (bt->dim == 3)
        hipLaunchKernelGGL((k_batch_solve<float, 3>), dim3(grid), dim3(kBE), 0, s, (const BBox<float>*)bt->bbox.p,
                           (const BIO*)bt->bio.p, (BRes*)bt->bres.p, bt->order.p, nbox, rtol, max_cycles, bt->nu1,
                           bt->nu2);
      else
        hipLaunchKernelGGL((k_batch_solve<float, 2>), dim3(grid), dim3(kBE), 0, s, (const BBox<float>*)bt->bbox.p,
                           (const BIO*)bt->bio.p, (BRes*)bt->bres.p, bt->order.p, nbox, rtol, max_cycles, bt->nu1,
                           bt->nu2);
    } else {
      if (bt->dim == 3)
        hipLaunchKernelGGL((k_batch_solve<double, 3>), dim3(grid), dim3(kBE), 0, s, (const BBox<double>*)bt->bbox.p,
                           (const BIO*)bt->bio.p, (BRes*)bt->bres.p, bt->order.p, nbox, rtol, max_cycles, bt->nu1,
                           bt->nu2);
      else
        hipLaunchKernelGGL((k_batch_solve<double, 2>), dim3(grid), dim3(kBE), 0, s, (const BBox<double>*)bt->bbox.p,
                           (const BIO*)bt->bio.p, (BRes*)bt->bres.p, bt->order.p, nbox, rtol, max_cycles, bt->nu1,
                           bt->nu2);
    }
    HIPCHECK(hipGetLastError());
    std::vector<BRes> res(nbox);
    HIPCHECK(hipMemcpyAsync(res.data(), bt->bres.p, sizeof(BRes) * nbox, hipMemcpyDeviceToHost, s));
    HIPCHECK(hipStreamSynchronize(s));
    const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    ebmg_status worst = EBMG_OK;
    for (int i = 0; i < nbox; ++i) {
      if (infos) {
        std::memset(&infos[i], 0, sizeof(ebmg_solve_info));
        infos[i].cycles = res[i].cycles;
        infos[i].outer_iters = res[i].iters;
        infos[i].levels = (int)bt->boxes[i]->dev.lv.size();
        infos[i].r0_norm = res[i].r0;
        infos[i].rel_residual = res[i].rel;
        infos[i].seconds = secs;
        infos[i].est_bytes = box_bytes(bt->boxes[i].get(), res[i].cycles, res[i].iters);
      }
      if (res[i].status != EBMG_OK && worst == EBMG_OK) worst = (ebmg_status)res[i].status;
    }
    return worst;
  });
}

ebmg_status ebmg_release_batch(ebmg_batch bt) {
  if (!bt) return EBMG_ERR_ARG;
  (void)hipSetDevice(bt->ctx->device);
  (void)hipStreamSynchronize(bt->ctx->stream);
  for (auto& P : bt->boxes)
    if (P) P->dev.release();
  for (auto& b : bt->lvbuf) b.release();
  bt->bbox.release();
  bt->order.release();
  bt->bio.release();
  bt->bres.release();
  ebmg::release_wide(bt);
  ebmg_ctx ctx = bt->ctx;
  delete bt;
  ctx_unref(ctx);
  return EBMG_OK;
}

ebmg_status ebmg_set_coefficients(ebmg_problem pb, const ebmg_options* opt, const ebmg_domain_bc* bc) {
  if (!pb || !opt || !bc) return EBMG_ERR_ARG;
  return guard(pb->ctx, [&]() -> ebmg_status {
    drain(pb);
    Problem& H = *pb->host;
    if (!H.geo.obj_value.empty() || H.geo.N2 > 0) throw ArgError("problem has embedded objects");
    for (const Level& L : H.levels)
      if (!L.irow_dof.empty()) throw ArgError("problem has explicit rows");
    Options o2;
    if (parse_options(opt, 0, o2) != EBMG_OK) throw ArgError("bad options");
    const Options& o = H.opt;
    if (o2.precision != o.precision || o2.nu1 != o.nu1 || o2.nu2 != o.nu2 || o2.bottom_max != o.bottom_max ||
        o2.krylov != o.krylov || o2.smoother != o.smoother || o2.tail != o.tail ||
        o2.dirichlet_closure != o.dirichlet_closure || o2.robin_closure != o.robin_closure ||
        o2.eb_order != o.eb_order || o2.graphs != o.graphs)
      throw ArgError("only alpha, beta, a and b may change");
    const int nf = 2 * H.geo.g.dim;
    for (int f = 0; f < nf; ++f) {
      if (bc->kind[f] != H.bc.kind[f]) throw ArgError("boundary kinds are fixed at setup");
      if (bc->kind[f] == EBMG_BC_ROBIN && !(bc->robin_a2[f] != 0.0)) throw ArgError("Robin a2 must be nonzero");
    }
    if (!(o2.b_gas > 0)) throw ArgError("b must be positive");
    // host: new template constants on every level and a new bottom inverse
    H.opt.alpha = o2.alpha;
    H.opt.beta = o2.beta;
    H.opt.a_gas = o2.a_gas;
    H.opt.a_diel = o2.a_diel;
    H.opt.b_gas = o2.b_gas;
    H.bc = *bc;
    H.bph[0] = H.bph[1] = o2.b_gas;
    H.aph[0] = o2.a_gas;
    H.aph[1] = o2.a_diel;
    fine_template(H);
    for (size_t l = 1; l < H.levels.size(); ++l) coarse_template(H.levels[l], H);
    build_bottom(H);
    if (!pb->on_device) return EBMG_OK;
    HIPCHECK(hipSetDevice(pb->ctx->device));
    hipStream_t s = pb->ctx->stream;
    DevProblem& D = pb->dev;
    HIPCHECK(hipStreamSynchronize(s));
    // the template constants are kernel arguments, so replay graphs hold the
    // old ones: drop them (the next solve captures again)
    D.drop_graphs();
    for (size_t l = 0; l < H.levels.size(); ++l) {
      D.lv[l].t64 = make_tmpl<double>(H.levels[l]);
      D.lv[l].t32 = make_tmpl<float>(H.levels[l]);
    }
    if (!H.bottom_inv.empty()) {
      if ((int64_t)H.bottom_inv.size() != D.bottom.n) throw ArgError("bottom size changed");
      HIPCHECK(hipMemcpyAsync(D.bottom.p, H.bottom_inv.data(), sizeof(double) * H.bottom_inv.size(),
                              hipMemcpyHostToDevice, s));
    } else {
      upload_bottom_krylov(D, s);   // its view holds the bottom level's template constants
    }
    // the one-workgroup engine keeps copies of the templates in its level views
    const int keep = D.tail_l0;
    D.bytes -= D.tail_lv.n;
    D.tail_lv.release();
    if (H.opt.precision == EBMG_MIXED)
      upload_tail<float>(D, s);
    else
      upload_tail<double>(D, s);
    D.tail_l0 = keep;
    HIPCHECK(hipStreamSynchronize(s));
    return EBMG_OK;
  });
}

// host part of a family member: member 0's geometry, the member's own
// coefficients and boundary data, its operator and hierarchy
static void build_member(ebmg::Problem& H, const ebmg::Problem& H0, const ebmg_box* box, int nobj,
                         const ebmg_object* objs, const ebmg_domain_bc* bc) {
  using namespace ebmg;
  H.bc = *bc;
  for (int f = 0; f < 2 * box->dim && f < 6; ++f) {
    if (bc->kind[f] != H0.bc.kind[f]) throw ArgError("family members must share the boundary kinds");
    if (bc->kind[f] == EBMG_BC_ROBIN && !(bc->robin_a2[f] != 0.0)) throw ArgError("Robin a2 must be nonzero");
  }
  H.geo = H0.geo;
  H.bph[0] = H.opt.b_gas;
  H.aph[0] = H.opt.a_gas;
  H.bph[1] = H.geo.nphase == 2 ? H.geo.obj_value[H.geo.diel_obj] : H.opt.b_gas;
  H.aph[1] = H.opt.a_diel;
  if (!(H.bph[0] > 0) || !(H.bph[1] > 0)) throw ArgError("b must be positive");
  bool anchored = H.opt.alpha != 0.0;
  for (int f = 0; f < 2 * box->dim; ++f) anchored |= bc->kind[f] != EBMG_BC_NEUMANN;
  for (int k = 0; k < nobj; ++k) anchored |= objs[k].kind == EBMG_OBJ_ELECTRODE;
  if (!anchored) throw ArgError("pure Neumann problem is singular");
  build_fine_level(H);
  build_hierarchy(H);
}

static void family_free(ebmg_family_s* F) {
  // members that take member 0's structure go first
  for (size_t k = F->mem.size(); k-- > 0;) {
    ebmg_problem_s* P = F->mem[k];
    if (!P) continue;
    if (P->on_device) {
      (void)hipSetDevice(P->ctx->device);
      (void)hipStreamSynchronize(P->ctx->stream);
      P->dev.release();
    }
    delete P;
  }
  F->mem.clear();
  for (ebmg_ctx c : F->mctx) ctx_unref(c);
  F->mctx.clear();
}

ebmg_status ebmg_setup_family(ebmg_ctx ctx, const ebmg_box* box, int32_t nobj, const ebmg_object* objs,
                              int32_t nmem, const ebmg_domain_bc* bcs, const ebmg_options* opts, ebmg_family* out) {
  if (!ctx || !box || !bcs || !opts || !out || (nobj > 0 && !objs) || nobj < 0 || nobj > 64 || nmem < 1 ||
      nmem > 64) {
    if (ctx) ctx->err = "invalid argument to ebmg_setup_family";
    return EBMG_ERR_ARG;
  }
  *out = nullptr;
  auto F = std::make_unique<ebmg_family_s>();
  F->ctx = ctx;
  const ebmg_status st = guard(ctx, [&]() -> ebmg_status {
    for (int k = 0; k < nmem; ++k) {
      // every option but the coefficients must be member 0's
      ebmg_options a = opts[k], b = opts[0];
      a.alpha = b.alpha;
      a.beta = b.beta;
      a.a_gas = b.a_gas;
      a.a_diel = b.a_diel;
      a.b_gas = b.b_gas;
      if (std::memcmp(&a, &b, sizeof(a)) != 0) throw ArgError("family members differ in an option other than the coefficients");
    }
    for (int k = 0; k < nmem; ++k) {
      ebmg_ctx mc = ctx;
      if (ctx->device >= 0) {
        if (ebmg_create(ctx->device, nullptr, &mc) != EBMG_OK) throw DeviceError("member stream: " + g_create_error);
      } else {
        ++ctx->refs;
      }
      F->mctx.push_back(mc);
      auto P = std::make_unique<ebmg_problem_s>();
      P->ctx = mc;
      P->host = std::make_unique<Problem>();
      Problem& H = *P->host;
      if (parse_options(&opts[k], nobj, H.opt) != EBMG_OK) throw ArgError("bad options");
      if (k == 0)
        build_host_problem(H, box, nobj, objs, &bcs[0]);
      else
        build_member(H, *F->mem[0]->host, box, nobj, objs, &bcs[k]);
      F->mem.push_back(P.release());
      ebmg_problem_s* M = F->mem.back();
      if (ctx->device >= 0) {
        HIPCHECK(hipSetDevice(ctx->device));
        upload(M, false, k == 0 ? nullptr : F->mem[0]);
        M->on_device = true;
      }
    }
    return EBMG_OK;
  });
  if (st != EBMG_OK) {
    family_free(F.get());
    return st;
  }
  *out = F.release();
  ++ctx->refs;
  return EBMG_OK;
}

ebmg_status ebmg_query_family(ebmg_family fam, int32_t* nmem, int64_t* n_cells, int64_t* n_phase2,
                              int64_t* device_bytes, int64_t* shared_bytes) {
  if (!fam || fam->mem.empty()) return EBMG_ERR_ARG;
  const ebmg::Geometry& G = fam->mem[0]->host->geo;
  int64_t by = 0, sh = 0;
  for (auto* P : fam->mem) {
    by += P->dev.bytes;
    sh += P->dev.shared_bytes;
  }
  if (nmem) *nmem = (int32_t)fam->mem.size();
  if (n_cells) *n_cells = G.N;
  if (n_phase2) *n_phase2 = G.N2;
  if (device_bytes) *device_bytes = by;
  if (shared_bytes) *shared_bytes = sh;
  return EBMG_OK;
}

ebmg_status ebmg_solve_family(ebmg_family fam, const double* const* rho, const double* const* sigma, double rtol,
                              int32_t max_cycles, double* const* phi, double* const* phi2, ebmg_solve_info* infos,
                              ebmg_status* statuses) {
  if (!fam || !rho || !phi || !(rtol > 0) || max_cycles < 0) {
    if (fam) fam->ctx->err = "invalid argument to ebmg_solve_family";
    return EBMG_ERR_ARG;
  }
  ebmg_ctx ctx = fam->ctx;
  const int K = (int)fam->mem.size();
  for (int k = 0; k < K; ++k) {
    if (rho[k] && !phi[k]) {
      ctx->err = "member " + std::to_string(k) + ": rho without phi";
      return EBMG_ERR_ARG;
    }
    if (rho[k] && fam->mem[k]->host->geo.N2 > 0 && phi2 && !phi2[k]) {
      ctx->err = "member " + std::to_string(k) + ": second-phase array required";
      return EBMG_ERR_ARG;
    }
  }
  if (!fam->mem[0]->on_device) {
    ctx->err = "family is not on a device (host-only context)";
    return EBMG_ERR_DEVICE;
  }
  std::vector<ebmg_status> st(K, EBMG_OK);
  std::vector<std::string> err(K);
  std::vector<ebmg_solve_info> inf(K);
  const ebmg_status pre = guard(ctx, [&]() -> ebmg_status {
    HIPCHECK(hipSetDevice(ctx->device));
    // the members' streams start after the work queued on the caller's stream
    hipEvent_t ev = nullptr;
    HIPCHECK(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
    HIPCHECK(hipEventRecord(ev, ctx->stream));
    for (int k = 0; k < K; ++k) HIPCHECK(hipStreamWaitEvent(fam->mctx[k]->stream, ev, 0));
    HIPCHECK(hipEventDestroy(ev));
    return EBMG_OK;
  });
  if (pre != EBMG_OK) return pre;
  auto run = [&](int k) {
    ebmg_problem_s* P = fam->mem[k];
    std::memset(&inf[k], 0, sizeof(ebmg_solve_info));
    st[k] = guard_msg(&err[k], [&]() -> ebmg_status {
      HIPCHECK(hipSetDevice(ctx->device));
      return ebmg::solve(P, rho[k], sigma ? sigma[k] : nullptr, nullptr, nullptr, rtol, max_cycles, phi[k],
                         phi2 ? phi2[k] : nullptr, nullptr, &inf[k]);
    });
  };
  if (fam->warm && K > 1) {
    // members on their own streams, each driven by its own host thread
    std::vector<std::thread> th;
    for (int k = 0; k < K; ++k)
      if (rho[k]) th.emplace_back(run, k);
    for (auto& t : th) t.join();
  } else {
    // first solve: one member after another (each captures its graphs)
    for (int k = 0; k < K; ++k)
      if (rho[k]) run(k);
    bool all = true;
    for (int k = 0; k < K; ++k) all = all && rho[k] && st[k] == EBMG_OK;
    fam->warm = fam->warm || all;
  }
  ebmg_status worst = EBMG_OK;
  for (int k = 0; k < K; ++k) {
    if (infos) infos[k] = inf[k];
    if (statuses) statuses[k] = rho[k] ? st[k] : EBMG_OK;
    if (rho[k] && st[k] != EBMG_OK && worst == EBMG_OK) {
      worst = st[k];
      ctx->err = "member " + std::to_string(k) + ": " + err[k];
    }
  }
  return worst;
}

ebmg_status ebmg_release_family(ebmg_family fam) {
  if (!fam) return EBMG_ERR_ARG;
  ebmg_ctx ctx = fam->ctx;
  family_free(fam);
  delete fam;
  ctx_unref(ctx);
  return EBMG_OK;
}

ebmg_status ebmg_advect(ebmg_problem pb, const double* n_in, const double* u_x, const double* u_y,
                        const double* u_z, double dt, const double* inflow, double* n_out) {
  if (!pb) return EBMG_ERR_ARG;
  ebmg_ctx ctx = pb->ctx;
  if (!n_in || !n_out || !u_x || !u_y || !(dt >= 0) || !std::isfinite(dt)) {
    ctx->err = "invalid argument to ebmg_advect";
    return EBMG_ERR_ARG;
  }
  if (!pb->on_device) {
    ctx->err = "problem is not on a device (host-only context)";
    return EBMG_ERR_DEVICE;
  }
  return guard(ctx, [&]() -> ebmg_status {
    const Geometry& G = pb->host->geo;
    const int D = G.g.dim;
    if (D == 3 && !u_z) throw ArgError("3D advection needs the z face velocities");
    if (n_in == n_out) throw ArgError("n_in and n_out must be different arrays");
    drain(pb);
    HIPCHECK(hipSetDevice(ctx->device));
    hipStream_t s = ctx->stream;
    auto& A = pb->dev.adv;
    if (!A.ready) {
      AdvHost H;
      build_advection(G, H);
      int64_t by = 0;
      A.nfaces = H.nfaces;
      for (int d = 0; d < 3; ++d) A.fbase[d] = H.face_base[d];
      A.ncut = (int)H.cut_cell.size();
      A.nsp = (int)H.sp_cell.size();
      A.cls.upload(H.cls.data(), (int64_t)H.cls.size(), s, by);
      A.kappa.upload(H.kappa.data(), (int64_t)H.kappa.size(), s, by);
      A.cut_cell.upload(H.cut_cell.data(), (int64_t)H.cut_cell.size(), s, by);
      A.dc_ptr.upload(H.dc_ptr.data(), (int64_t)H.dc_ptr.size(), s, by);
      A.dc_face.upload(H.dc_face.data(), (int64_t)H.dc_face.size(), s, by);
      A.dc_coef.upload(H.dc_coef.data(), (int64_t)H.dc_coef.size(), s, by);
      A.nb_ptr.upload(H.nb_ptr.data(), (int64_t)H.nb_ptr.size(), s, by);
      A.nb_cell.upload(H.nb_cell.data(), (int64_t)H.nb_cell.size(), s, by);
      A.nb_w.upload(H.nb_w.data(), (int64_t)H.nb_w.size(), s, by);
      A.cut_S.upload(H.cut_S.data(), (int64_t)H.cut_S.size(), s, by);
      A.sp_cell.upload(H.sp_cell.data(), (int64_t)H.sp_cell.size(), s, by);
      A.sp_cut.upload(H.sp_cut.data(), (int64_t)H.sp_cut.size(), s, by);
      A.sp_ptr.upload(H.sp_ptr.data(), (int64_t)H.sp_ptr.size(), s, by);
      A.sp_donor.upload(H.sp_donor.data(), (int64_t)H.sp_donor.size(), s, by);
      A.F.alloc(std::max<int64_t>(1, A.nfaces), by);
      A.Dc.alloc(std::max<int64_t>(1, G.N), by);
      A.Dcut.alloc(std::max<int64_t>(1, A.ncut), by);
      A.give.alloc(std::max<int64_t>(1, A.ncut), by);
      HIPCHECK(hipStreamSynchronize(s));
      pb->dev.bytes += by;
      A.ready = true;
    }
    AdvGrid g;
    g.dim = D;
    for (int d = 0; d < 3; ++d) {
      g.n[d] = d < D ? G.g.n[d] : 1;
      g.fbase[d] = A.fbase[d];
    }
    g.h = G.g.h;
    g.dt = dt;
    for (int f = 0; f < 6; ++f) g.inflow[f] = inflow ? inflow[f] : 0.0;
    AdvVel vel;
    vel.u[0] = u_x;
    vel.u[1] = u_y;
    vel.u[2] = D == 3 ? u_z : u_x;
    auto flux_grid = [&](int d) { return dim3(nblk((int64_t)(g.n[0] + (d == 0)) * (g.n[1] + (d == 1)))); };
    const dim3 cell_grid(nblk((int64_t)g.n[0] * g.n[1]));
    const bool off32 = (int64_t)(g.n[0] + 1) * (g.n[1] + 1) * (g.n[2] + 1) < ((int64_t)1 << 31);
    if (D == 3 && off32) {
      // one z-marching pass (its offsets are 32-bit)
      constexpr int TX = 16, TY = 16, ZC = 32;
      const int tiles_x = (g.n[0] + TX - 1) / TX, tiles_y = (g.n[1] + TY - 1) / TY;
      const int64_t blocks = (int64_t)tiles_x * tiles_y * ((g.n[2] + ZC - 1) / ZC);
      hipLaunchKernelGGL((k_adv_zm<TX, TY, ZC>), dim3((unsigned)blocks), dim3(TX * TY), 0, s, n_in, A.cls.p, vel, g,
                         tiles_x, tiles_y, A.F.p, A.Dc.p, n_out);
    } else if (D == 3) {
      // boxes of 2^31 faces or more: face fluxes, then the full cells
      for (int d = 0; d < 3; ++d) {
        const dim3 grid(nblk((int64_t)(g.n[0] + (d == 0)) * (g.n[1] + (d == 1))), (unsigned)(g.n[2] + (d == 2)));
        auto k = d == 0 ? k_adv_flux<3, 0> : (d == 1 ? k_adv_flux<3, 1> : k_adv_flux<3, 2>);
        hipLaunchKernelGGL(k, grid, dim3(256), 0, s, n_in, A.cls.p, vel, g, A.F.p + A.fbase[d]);
      }
      hipLaunchKernelGGL(k_adv_full<3>, dim3(nblk((int64_t)g.n[0] * g.n[1]), (unsigned)g.n[2]), dim3(256), 0, s,
                         A.cls.p, g, A.F.p, n_in, A.Dc.p, n_out);
    } else {
      hipLaunchKernelGGL((k_adv_flux<2, 0>), flux_grid(0), dim3(256), 0, s, n_in, A.cls.p, vel, g, A.F.p + A.fbase[0]);
      hipLaunchKernelGGL((k_adv_flux<2, 1>), flux_grid(1), dim3(256), 0, s, n_in, A.cls.p, vel, g, A.F.p + A.fbase[1]);
      hipLaunchKernelGGL(k_adv_full<2>, cell_grid, dim3(256), 0, s, A.cls.p, g, A.F.p, n_in, A.Dc.p, n_out);
    }
    if (A.ncut > 0) {
      hipLaunchKernelGGL(k_adv_dc_cut, dim3(nblk(A.ncut)), dim3(256), 0, s, A.ncut, A.cut_cell.p, A.dc_ptr.p,
                         A.dc_face.p, A.dc_coef.p, A.F.p, A.Dc.p);
      hipLaunchKernelGGL(k_adv_cut, dim3(nblk(A.ncut)), dim3(256), 0, s, A.ncut, A.cut_cell.p, A.kappa.p, A.nb_ptr.p,
                         A.nb_cell.p, A.nb_w.p, A.cut_S.p, A.Dc.p, A.Dcut.p, A.give.p);
    }
    if (A.nsp > 0)
      hipLaunchKernelGGL(k_adv_special, dim3(nblk(A.nsp)), dim3(256), 0, s, A.nsp, A.sp_cell.p, A.sp_cut.p, A.sp_ptr.p,
                         A.sp_donor.p, dt, n_in, A.Dc.p, A.Dcut.p, A.give.p, n_out);
    HIPCHECK(hipGetLastError());
    HIPCHECK(hipStreamSynchronize(s));
    return EBMG_OK;
  });
}

ebmg_status ebmg_time_batch_kernel(ebmg_batch bt, int32_t which, int32_t reps, double* avg_ms, double* alg_bytes) {
  if (!bt || which < 0 || which > 1 || reps < 1) return EBMG_ERR_ARG;
  return guard(bt->ctx, [&]() -> ebmg_status {
    if (bt->mode != 2 || bt->wide.empty())
      throw ArgError("the finest-level timing needs the level-synchronous batch mode");
    HIPCHECK(hipSetDevice(bt->ctx->device));
    hipStream_t s = bt->ctx->stream;
    const int nbox = (int)bt->boxes.size();
    // every box active, as at the start of a solve; the cycle vectors hold
    // the last solve's values and are overwritten by the next one
    std::vector<WState> st = initial_state(bt);
    HIPCHECK(hipMemcpyAsync(bt->state.p, st.data(), sizeof(WState) * nbox, hipMemcpyHostToDevice, s));
    auto run = [&]() {
      if (bt->mixed) {
        if (bt->dim == 3) wide_level0_kernels<float, 3>(bt, which, s); else wide_level0_kernels<float, 2>(bt, which, s);
      } else {
        if (bt->dim == 3) wide_level0_kernels<double, 3>(bt, which, s); else wide_level0_kernels<double, 2>(bt, which, s);
      }
    };
    run();
    hipEvent_t e0, e1;
    HIPCHECK(hipEventCreate(&e0));
    HIPCHECK(hipEventCreate(&e1));
    HIPCHECK(hipEventRecord(e0, s));
    for (int k = 0; k < reps; ++k) run();
    HIPCHECK(hipEventRecord(e1, s));
    HIPCHECK(hipEventSynchronize(e1));
    float ms = 0;
    HIPCHECK(hipEventElapsedTime(&ms, e0, e1));
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    const int vsz = bt->mixed ? 4 : 8;
    double by = 0;
    for (auto& P : bt->boxes) {
      const DevLevel& l = P->dev.lv[0];
      by += which == 0 ? (double)l.N * (3.0 * vsz + 1.0) : rows_bytes(l, vsz);
    }
    if (avg_ms) *avg_ms = ms / reps;
    if (alg_bytes) *alg_bytes = by;
    return EBMG_OK;
  });
}

ebmg_status ebmg_setup_amr(ebmg_ctx ctx, int32_t nbox, const ebmg_box* boxes, const int32_t* levels,
                           const int32_t* nobj, const ebmg_object* const* objs, const ebmg_domain_bc* bc,
                           const ebmg_options* opts, ebmg_amr* out) {
  if (!ctx || nbox < 1 || nbox > 256 || !boxes || !levels || !nobj || !objs || !bc || !out) {
    if (ctx) ctx->err = "invalid argument to ebmg_setup_amr";
    return EBMG_ERR_ARG;
  }
  *out = nullptr;
  auto A = std::make_unique<ebmg_amr_s>();
  A->ctx = ctx;
  const ebmg_status st = guard(ctx, [&]() -> ebmg_status {
    const int D = boxes[0].dim;
    const int nlev = nbox;   // boxes, in the loops below
    if (D != 2 && D != 3) throw ArgError("dim must be 2 or 3");
    ebmg::Options o0;
    if (parse_options(opts, nobj[0], o0) != EBMG_OK) throw ArgError("bad options");
    if (o0.dirichlet_closure != 0)
      throw ArgError("AMR hierarchies use the linear Dirichlet closure on their coarse-fine faces");
    if (levels[0] != 0) throw ArgError("box 0 is the domain (level 0)");
    // boxes: level l has cells of size h0 / 2^l, corners on the level's lattice
    A->box.resize(nlev);
    for (int l = 0; l < nlev; ++l) {
      const ebmg_box& B = boxes[l];
      const int lev = levels[l];
      if (B.dim != D) throw ArgError("every box has the base box's dimension");
      if (lev < 0 || lev > 12 || (l > 0 && lev == 0)) throw ArgError("bad level of an AMR box");
      if (nobj[l] < 0 || nobj[l] > 64 || (nobj[l] > 0 && !objs[l])) throw ArgError("bad objects of a box");
      const double h = boxes[0].h / (double)(1 << lev);
      if (std::fabs(B.h - h) > 1e-12 * h) throw ArgError("a box of level l needs cells of size h0 / 2^l");
      ebmg::AmrBox& X = A->box[l];
      X.level = lev;
      for (int d = 0; d < D; ++d) {
        const double q = (B.lo[d] - boxes[0].lo[d]) / h;
        X.lo[d] = (int)std::lround(q);
        X.n[d] = B.n[d];
        if (std::fabs(q - X.lo[d]) > 1e-6) throw ArgError("an AMR box corner is off its level's lattice");
        const int full = boxes[0].n[d] << lev;
        if (X.lo[d] < 0 || X.n[d] < 1 || X.lo[d] + X.n[d] > full) throw ArgError("an AMR box leaves the domain");
        X.cf[2 * d] = lev > 0 && X.lo[d] > 0;
        X.cf[2 * d + 1] = lev > 0 && X.lo[d] + X.n[d] < full;
      }
      if (l == 0)
        for (int d = 0; d < D; ++d)
          if (X.lo[d] != 0 || X.n[d] != boxes[0].n[d]) throw ArgError("box 0 is the domain");
    }
    // proper nesting: each box on even corners, its coarse cells inside one
    // box of the next coarser level (its parent) and at least two cells from
    // that box's coarse-fine faces; boxes of one level do not overlap
    for (int l = 1; l < nlev; ++l) {
      ebmg::AmrBox& F = A->box[l];
      for (int d = 0; d < D; ++d)
        if (F.lo[d] % 2 || F.n[d] % 2 || F.n[d] < 4) throw ArgError("AMR boxes need even corners and sizes >= 4");
      for (int q = 0; q < nlev && F.parent < 0; ++q) {
        const ebmg::AmrBox& Cb = A->box[q];
        if (Cb.level != F.level - 1) continue;
        bool in = true;
        for (int d = 0; d < D; ++d) {
          const int clo = F.lo[d] / 2, chi = (F.lo[d] + F.n[d]) / 2;
          const int mlo = Cb.cf[2 * d] ? 2 : 0, mhi = Cb.cf[2 * d + 1] ? 2 : 0;
          in = in && clo >= Cb.lo[d] + mlo && chi <= Cb.lo[d] + Cb.n[d] - mhi;
        }
        if (in) F.parent = q;
      }
      if (F.parent < 0)
        throw ArgError("an AMR box must lie inside a box of the next coarser level, two cells from its coarse-fine faces");
      for (int q = 1; q < l; ++q) {
        const ebmg::AmrBox& G = A->box[q];
        if (G.level != F.level) continue;
        bool overlap = true;
        for (int d = 0; d < D; ++d)
          overlap = overlap && F.lo[d] < G.lo[d] + G.n[d] && G.lo[d] < F.lo[d] + F.n[d];
        if (overlap) throw ArgError("boxes of one AMR level overlap");
      }
    }
    // one problem per level: the domain's conditions on domain faces,
    // homogeneous Dirichlet on coarse-fine faces
    for (int l = 0; l < nlev; ++l) {
      auto P = std::make_unique<ebmg_problem_s>();
      P->ctx = ctx;
      P->host = std::make_unique<Problem>();
      Problem& H = *P->host;
      if (parse_options(opts, nobj[l], H.opt) != EBMG_OK) throw ArgError("bad options");
      ebmg_domain_bc lb = *bc;
      for (int f = 0; f < 2 * D; ++f)
        if (A->box[l].cf[f]) {
          lb.kind[f] = EBMG_BC_DIRICHLET;
          lb.value[f] = 0.0;
        }
      build_host_problem(H, &boxes[l], nobj[l], objs[l], &lb);
      A->lev.push_back(P.release());
    }
    std::vector<std::vector<const ebmg::AmrBox*>> kids(nlev);
    for (int l = 1; l < nlev; ++l) kids[A->box[l].parent].push_back(&A->box[l]);
    std::vector<AmrLink> host_links(nlev);
    for (int l = 1; l < nlev; ++l) {
      const int pa = A->box[l].parent;
      build_amr_link(*A->lev[pa]->host, A->box[pa], kids[pa], *A->lev[l]->host, A->box[l], kids[l], host_links[l]);
    }
    // boxes deepest level first (the preconditioner's downward order)
    A->order.resize(nlev);
    for (int l = 0; l < nlev; ++l) A->order[l] = l;
    std::stable_sort(A->order.begin(), A->order.end(),
                     [&](int x, int y) { return A->box[x].level > A->box[y].level; });
    // the host part is checked on any context; the solve needs a device
    if (ctx->device < 0) throw DeviceError("an AMR hierarchy needs a device context");
    HIPCHECK(hipSetDevice(ctx->device));
    hipStream_t s = ctx->stream;
    for (ebmg_problem_s* P : A->lev) {
      upload(P);
      P->on_device = true;
      A->bytes += P->dev.bytes;
    }
    A->off.assign(nlev, 0);
    A->nd.assign(nlev, 0);
    int64_t o = 0;
    for (int l = 0; l < nlev; ++l) {
      A->off[l] = o;
      A->nd[l] = A->lev[l]->host->geo.N + A->lev[l]->host->geo.N2;
      o += (A->nd[l] + 63) / 64 * 64;
    }
    A->ntot = o;
    int64_t by = 0;
    A->link.resize(nlev);
    for (int l = 1; l < nlev; ++l) {
      AmrLink& H = host_links[l];
      auto& K = A->link[l];
      K.nf = (int64_t)H.frow.size();
      K.nc = (int64_t)H.crow.size();
      K.ncov = (int64_t)H.cov.size();
      K.nr = (int64_t)H.rrow.size();
      K.np = (int64_t)H.pcol.size();
      K.frow.upload(H.frow.data(), (int64_t)H.frow.size(), s, by);
      K.fptr.upload(H.fptr.data(), (int64_t)H.fptr.size(), s, by);
      K.fcol.upload(H.fcol.data(), (int64_t)H.fcol.size(), s, by);
      K.fw.upload(H.fw.data(), (int64_t)H.fw.size(), s, by);
      K.crow.upload(H.crow.data(), (int64_t)H.crow.size(), s, by);
      K.cptr.upload(H.cptr.data(), (int64_t)H.cptr.size(), s, by);
      K.ccol.upload(H.ccol.data(), (int64_t)H.ccol.size(), s, by);
      K.cw.upload(H.cw.data(), (int64_t)H.cw.size(), s, by);
      K.cov.upload(H.cov.data(), (int64_t)H.cov.size(), s, by);
      K.rrow.upload(H.rrow.data(), (int64_t)H.rrow.size(), s, by);
      K.rptr.upload(H.rptr.data(), (int64_t)H.rptr.size(), s, by);
      K.rcol.upload(H.rcol.data(), (int64_t)H.rcol.size(), s, by);
      K.rw.upload(H.rw.data(), (int64_t)H.rw.size(), s, by);
      K.aw.upload(H.aw.data(), (int64_t)H.aw.size(), s, by);
      K.pcol.upload(H.pcol.data(), (int64_t)H.pcol.size(), s, by);
    }
    for (auto* b : {&A->x, &A->b, &A->r, &A->rh, &A->p, &A->v, &A->sv, &A->t, &A->ph, &A->sh, &A->rt, &A->y, &A->e})
      b->alloc(A->ntot, by);
    A->part.alloc(kNormBlocks, by);
    A->scal.alloc(8, by);
    for (auto* b : {&A->x, &A->b, &A->r, &A->rh, &A->p, &A->v, &A->sv, &A->t, &A->ph, &A->sh, &A->rt, &A->y, &A->e})
      fill<double>(b->p, A->ntot, 0.0, s);
    HIPCHECK(hipStreamSynchronize(s));
    A->bytes += by;
    return EBMG_OK;
  });
  if (st != EBMG_OK) {
    amr_free(A.get());
    return st;
  }
  *out = A.release();
  ++ctx->refs;
  return EBMG_OK;
}

ebmg_status ebmg_query_amr(ebmg_amr a, int32_t level, int64_t* n_cells, int64_t* n_phase2, int64_t* n_covered,
                           int64_t* device_bytes) {
  if (!a || level < 0 || level >= (int32_t)a->lev.size()) return EBMG_ERR_ARG;
  if (n_cells) *n_cells = a->lev[level]->host->geo.N;
  if (n_phase2) *n_phase2 = a->lev[level]->host->geo.N2;
  if (n_covered) {
    int64_t c = 0;
    for (size_t l = 1; l < a->lev.size(); ++l)
      if (a->box[l].parent == level) c += a->link[l].ncov;
    *n_covered = c;
  }
  if (device_bytes) *device_bytes = a->bytes;
  return EBMG_OK;
}

// phi (and phi2) per level <- / -> the composite vector slices
static void amr_copy(ebmg_amr_s* A, double* const* phi, double* const* phi2, bool in, hipStream_t s) {
  for (size_t l = 0; l < A->lev.size(); ++l) {
    const int64_t N = A->lev[l]->host->geo.N, N2 = A->lev[l]->host->geo.N2;
    double* slice = A->x.p + A->off[l];
    if (in) {
      HIPCHECK(hipMemcpyAsync(slice, phi[l], sizeof(double) * N, hipMemcpyDeviceToDevice, s));
      if (N2 > 0) HIPCHECK(hipMemcpyAsync(slice + N, phi2[l], sizeof(double) * N2, hipMemcpyDeviceToDevice, s));
    } else {
      HIPCHECK(hipMemcpyAsync(phi[l], slice, sizeof(double) * N, hipMemcpyDeviceToDevice, s));
      if (N2 > 0) HIPCHECK(hipMemcpyAsync(phi2[l], slice + N, sizeof(double) * N2, hipMemcpyDeviceToDevice, s));
    }
  }
}

// per level a non-null array, and where need2 a second one for levels with
// second-phase unknowns
static void amr_check_args(ebmg_amr_s* A, const void* const* a, const void* const* a2, bool need2, const char* what) {
  for (size_t l = 0; l < A->lev.size(); ++l) {
    if (!a[l]) throw ArgError(std::string(what) + ": a level's array is null");
    if (need2 && A->lev[l]->host->geo.N2 > 0 && (!a2 || !a2[l]))
      throw ArgError(std::string(what) + ": a level with second-phase unknowns needs its second array");
  }
}

ebmg_status ebmg_solve_amr(ebmg_amr a, const double* const* rho, double rtol, int32_t max_iters, double* const* phi,
                           double* const* phi2, ebmg_solve_info* info) {
  if (!a || !rho || !phi || !(rtol > 0) || max_iters < 1) {
    if (a) a->ctx->err = "invalid argument to ebmg_solve_amr";
    return EBMG_ERR_ARG;
  }
  ebmg_solve_info loc{};
  const ebmg_status st = guard(a->ctx, [&]() -> ebmg_status {
    auto t0 = std::chrono::steady_clock::now();
    amr_check_args(a, (const void* const*)rho, nullptr, false, "rho");
    amr_check_args(a, (const void* const*)phi, (const void* const*)phi2, true, "phi");
    HIPCHECK(hipSetDevice(a->ctx->device));
    hipStream_t s = a->ctx->stream;
    const int L = (int)a->lev.size();
    // right-hand side per level (its boundary data; 0 on coarse-fine faces),
    // 0 on covered unknowns
    for (int l = 0; l < L; ++l) {
      ebmg_problem_s* P = a->lev[l];
      rhs(P, rho[l], nullptr, nullptr, nullptr);
      HIPCHECK(hipMemcpyAsync(a->b.p + a->off[l], P->dev.lv[0].b64.p, sizeof(double) * a->nd[l],
                              hipMemcpyDeviceToDevice, s));
    }
    amr_copy(a, phi, phi2, true, s);
    for (int l = 1; l < L; ++l) {
      auto& K = a->link[l];
      const int64_t oc = a->off[a->box[l].parent];
      if (K.ncov) {
        hipLaunchKernelGGL(k_amr_set, dim3(nblk(K.ncov)), dim3(256), 0, s, K.ncov, K.cov.p, (const double*)nullptr,
                           a->b.p + oc);
        hipLaunchKernelGGL(k_amr_set, dim3(nblk(K.ncov)), dim3(256), 0, s, K.ncov, K.cov.p, (const double*)nullptr,
                           a->x.p + oc);
      }
    }
    HIPCHECK(hipGetLastError());
    double bn = 0, rel = 0;
    int iters = 0;
    ebmg_status res = amr_bicgstab(a, rtol, max_iters, bn, rel, iters, s);
    // the true residual of the result
    if (res == EBMG_OK || res == EBMG_ERR_NOCONV) {
      amr_apply(a, a->x.p, a->y.p, s);
      hipLaunchKernelGGL(k_amr_lin, dim3(nblk(a->ntot)), dim3(256), 0, s, a->ntot, 1.0, a->b.p, -1.0, a->y.p,
                         a->r.p);
      rel = bn > 0 ? std::sqrt(amr_dot(a, a->r.p, a->r.p, s)) / bn : 0.0;
      if (!std::isfinite(rel)) res = EBMG_ERR_NUMERIC;
    }
    // covered cells take the mean of their children, deepest boxes first
    for (int q = 0; q < L; ++q) {
      const int l = a->order[q];
      if (l == 0) continue;
      auto& K = a->link[l];
      if (K.nr)
        hipLaunchKernelGGL(k_amr_gather, dim3(nblk(K.nr)), dim3(256), 0, s, K.nr, K.rrow.p, K.rptr.p, K.rcol.p,
                           K.aw.p, a->x.p + a->off[l], a->x.p + a->off[a->box[l].parent]);
    }
    amr_copy(a, phi, phi2, false, s);
    HIPCHECK(hipStreamSynchronize(s));
    loc.cycles = 2 * iters;
    loc.outer_iters = iters;
    loc.levels = L;
    loc.r0_norm = bn;
    loc.rel_residual = rel;
    loc.est_bytes = 0;
    loc.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    if (res == EBMG_ERR_NOCONV) a->ctx->err = "AMR solve did not reach the tolerance";
    if (res == EBMG_ERR_NUMERIC) a->ctx->err = "AMR solve produced a non-finite residual";
    return res;
  });
  if (info) *info = loc;
  return st;
}

ebmg_status ebmg_apply_amr(ebmg_amr a, const double* const* phi, const double* const* phi2, double* const* out,
                           double* const* out2) {
  if (!a || !phi || !out) return EBMG_ERR_ARG;
  return guard(a->ctx, [&]() -> ebmg_status {
    amr_check_args(a, (const void* const*)phi, (const void* const*)phi2, true, "phi");
    amr_check_args(a, (const void* const*)out, (const void* const*)out2, true, "out");
    HIPCHECK(hipSetDevice(a->ctx->device));
    hipStream_t s = a->ctx->stream;
    amr_copy(a, const_cast<double* const*>(phi), const_cast<double* const*>(phi2), true, s);
    amr_apply(a, a->x.p, a->y.p, s);
    // the result leaves through the x slices
    HIPCHECK(hipMemcpyAsync(a->x.p, a->y.p, sizeof(double) * a->ntot, hipMemcpyDeviceToDevice, s));
    amr_copy(a, out, out2, false, s);
    HIPCHECK(hipStreamSynchronize(s));
    return EBMG_OK;
  });
}

ebmg_status ebmg_release_amr(ebmg_amr a) {
  if (!a) return EBMG_OK;
  ebmg_ctx ctx = a->ctx;
  amr_free(a);
  delete a;
  ctx_unref(ctx);
  return EBMG_OK;
}

ebmg_status ebmg_mesh_create(ebmg_ctx ctx, int32_t nvert, const double* verts, int32_t ntri, const int32_t* tris,
                             ebmg_mesh* out) {
  if (!ctx || !verts || !tris || !out || nvert <= 0 || ntri <= 0) {
    if (ctx) ctx->err = "invalid argument to ebmg_mesh_create";
    return EBMG_ERR_ARG;
  }
  *out = nullptr;
  if (ctx->device < 0) {
    ctx->err = "a mesh needs a device context";
    return EBMG_ERR_DEVICE;
  }
  auto M = std::make_unique<ebmg_mesh_s>();
  M->ctx = ctx;
  const ebmg_status st = guard(ctx, [&]() -> ebmg_status {
    MeshInput in;
    in.nvert = nvert;
    in.ntri = ntri;
    in.verts = verts;
    in.tris = tris;
    MeshHost H;
    build_mesh(in, H);
    if (H.depth >= kSdfStack) throw ArgError("mesh tree deeper than the search stack");
    static_assert(sizeof(MeshNode) == sizeof(DevMeshNode), "node layouts differ");
    HIPCHECK(hipSetDevice(ctx->device));
    hipStream_t s = ctx->stream;
    M->tri.upload(H.tri.data(), (int64_t)H.tri.size(), s, M->bytes);
    M->nodes.upload((const uint8_t*)H.nodes.data(), (int64_t)(H.nodes.size() * sizeof(MeshNode)), s, M->bytes);
    M->visits.alloc(1, M->bytes);
    HIPCHECK(hipStreamSynchronize(s));
    M->ntri = H.ntri;
    M->nnode = (int32_t)H.nodes.size();
    M->depth = H.depth;
    return EBMG_OK;
  });
  if (st != EBMG_OK) {
    M->tri.release();
    M->nodes.release();
    M->visits.release();
    return st;
  }
  *out = M.release();
  ++ctx->refs;
  return EBMG_OK;
}

ebmg_status ebmg_mesh_query(ebmg_mesh m, int32_t* ntri, int32_t* nnode, int32_t* depth, int64_t* device_bytes) {
  if (!m) return EBMG_ERR_ARG;
  if (ntri) *ntri = m->ntri;
  if (nnode) *nnode = m->nnode;
  if (depth) *depth = m->depth;
  if (device_bytes) *device_bytes = m->bytes;
  return EBMG_OK;
}

ebmg_status ebmg_mesh_sdf(ebmg_mesh m, const ebmg_box* box, double* sdf, int64_t* visits) {
  if (!m || !box || !sdf) return EBMG_ERR_ARG;
  ebmg_ctx ctx = m->ctx;
  return guard(ctx, [&]() -> ebmg_status {
    if (box->dim != 3) throw ArgError("mesh distances are 3D");
    for (int d = 0; d < 3; ++d)
      if (box->n[d] < 1) throw ArgError("bad box size");
    if (!(box->h > 0) || !std::isfinite(box->h)) throw ArgError("bad cell size");
    const int m0 = box->n[0] + 1, m1 = box->n[1] + 1, m2 = box->n[2] + 1;
    const int64_t total = (int64_t)m0 * m1 * m2;
    HIPCHECK(hipSetDevice(ctx->device));
    hipStream_t s = ctx->stream;
    unsigned long long* vis = visits ? m->visits.p : nullptr;
    if (vis) HIPCHECK(hipMemsetAsync(vis, 0, sizeof(unsigned long long), s));
    const unsigned nb = (unsigned)((total + kSdfBlock - 1) / kSdfBlock);
    hipLaunchKernelGGL(k_sdf_mesh, dim3(nb), dim3(kSdfBlock), 0, s, (const DevMeshNode*)m->nodes.p, m->tri.p, m0, m1, m2,
                       box->h, box->lo[0], box->lo[1], box->lo[2], sdf, vis);
    HIPCHECK(hipGetLastError());
    if (visits) {
      unsigned long long v = 0;
      HIPCHECK(hipMemcpyAsync(&v, vis, sizeof(v), hipMemcpyDeviceToHost, s));
      HIPCHECK(hipStreamSynchronize(s));
      *visits = (int64_t)v;
    }
    HIPCHECK(hipStreamSynchronize(s));
    return EBMG_OK;
  });
}

ebmg_status ebmg_mesh_release(ebmg_mesh m) {
  if (!m) return EBMG_ERR_ARG;
  ebmg_ctx ctx = m->ctx;
  (void)hipSetDevice(ctx->device);
  (void)hipStreamSynchronize(ctx->stream);
  m->tri.release();
  m->nodes.release();
  m->visits.release();
  delete m;
  ctx_unref(ctx);
  return EBMG_OK;
}

ebmg_status ebmg_release(ebmg_problem pb) {
  if (!pb) return EBMG_ERR_ARG;
  drain(pb);
  if (pb->on_device) {
    (void)hipSetDevice(pb->ctx->device);
    (void)hipStreamSynchronize(pb->ctx->stream);
    pb->dev.release();
  }
  ebmg_ctx ctx = pb->ctx;
  delete pb;
  ctx_unref(ctx);
  return EBMG_OK;
}

}  // extern "C"
