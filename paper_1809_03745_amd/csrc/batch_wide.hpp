// Level-synchronous batched solver (gfx950).
//
// The persistent engine gives each box one workgroup for its whole solve, so
// a large box runs at one CU's share of the memory system and the chip idles
// while the last large boxes finish. Here each phase of the V-cycle is ONE
// launch over every box at once: the work of a box on a level (half-sweep
// items, cells, explicit rows, transfer-list entries, vector entries) is cut
// into fixed chunks, listed box by box in a table of work entries, one
// workgroup per entry. The chunking of a box does not depend on the other
// boxes and every chunk computes exactly what the engine's loop computes for
// those items, so a box's result is independent of the batch.
//
// Each box's coarse levels (from a setup-tuned size down) run as the
// engine's one-workgroup sub-V-cycle, all boxes in a single launch. The
// BiCGStab scalars, convergence tests, restarts and stopping rule are kept
// per box in device memory and updated by one wavefront per box; a box that
// has stopped leaves its entries idle. Dot products are per-entry partial
// sums (fixed order inside a workgroup) added up per box in a fixed order.
#pragma once

#include "block_engine.hpp"

namespace ebmg {

constexpr int kWB = 256;               // threads of a level-synchronous workgroup
constexpr int kWRows = kWB;            // explicit rows per entry (one slice per wavefront)
constexpr int kWList = kWB;            // list entries (one per thread) per entry
constexpr int kWVec = 4 * kWB;         // vector entries per entry

template <typename T>
struct WCh {
  static constexpr int v = kWB * BeU<T>::U;   // cells (or half-sweep items) per entry
};

// One workgroup's work: box, segment (cells / rows / lists) and chunk.
// box < 0 pads a table to a multiple of the XCD count.
struct WEnt {
  int box, seg, chunk, pad;
};

// Per-box solver state.
struct WState {
  double bn, rel, rho, rho_old, alpha, omega, rv, ts, tt, rr;
  int cycles, iters, restarts, status;
  int active;    // still iterating
  int verify;    // true residual to be formed and tested this iteration
  int restart;   // Krylov vectors to be reset (rh = r, p = v = 0)
  int mode;      // 2: BiCGStab; else plain V-cycle refinement (beta = 0, alpha = omega = 1)
};

enum WFilt { WF_ACTIVE = 0, WF_VERIFY = 1, WF_RESTART = 2 };

__device__ __forceinline__ bool w_pass(const WState& s, int filt) {
  return filt == WF_ACTIVE ? s.active != 0 : (filt == WF_VERIFY ? s.verify != 0 : s.restart != 0 && s.active != 0);
}

// Entry of this workgroup; consecutive table entries (neighbouring chunks of
// one box) go to one XCD so their halos meet in its L2.
__device__ __forceinline__ int w_entry() { return (int)xcd_block(blockIdx.x, gridDim.x); }

// Sum over the workgroup in a fixed order; the result is valid in thread 0.
__device__ __forceinline__ double w_block_sum(double v, double* red) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  double s = 0;
  if (threadIdx.x == 0)
    for (int w = 0; w < kWB / 64; ++w) s += red[w];
  return s;
}

// ---------------------------------------------------------------------------
// cycle phases over all boxes of one level
// ---------------------------------------------------------------------------
template <typename T, int DIM>
__global__ void __launch_bounds__(kWB) kw_rb(const BLev<T>* __restrict__ WL, const WEnt* __restrict__ tab,
                                            const WState* __restrict__ st, int colour) {
  const WEnt e = tab[w_entry()];
  if (e.box < 0 || !st[e.box].active) return;
  const BLev<T>& L = WL[e.box];
  be_rb_part<T, DIM>(L, L.x, L.b, colour, e.chunk * WCh<T>::v, WCh<T>::v);
}

// Jacobi values of one 64-row slice of a box's colour group into its w: the
// slice's entries are split over the four wavefronts (as in k_irr_jac_sl),
// which cuts the chain of dependent loads each row waits on to a quarter
// (512-box batch: 0.288 -> 0.266 ms for both groups' passes, 52.0 -> 49.7 ms
// per mixed batch; the same split in the residual and operator rows, which
// run once per level and cycle, changed nothing).
static_assert(kWB == kRowBlock, "one slice per workgroup of the split row form");
template <typename T>
__global__ void __launch_bounds__(kWB) kw_irr_jac(const BLev<T>* __restrict__ WL, const WEnt* __restrict__ tab,
                                                 const WState* __restrict__ st, int grp) {
  FP_EXACT_ORDER
  const WEnt e = tab[w_entry()];
  if (e.box < 0 || !st[e.box].active) return;
  const BLev<T>& L = WL[e.box];
  if (L.grp_ptr[grp + 1] <= L.grp_ptr[grp]) return;
  const int r0 = L.grp_ptr[grp];
  const GPtr<const int64_t> dof = gview(L.irow_dof);
  const GPtr<const T> dgv = gview(L.diag), bg = gview((const T*)L.b);
  const GPtr<T> wg = gview(L.w);
  split_rows<T, T, false>(
      L, grp, L.x, e.chunk,
      [&](int g) {
        const int64_t q = dof[g];
        return RowOwn<T>{q, dgv[g], bg[q]};
      },
      [&](int g, const RowOwn<T>& o, T sm) { wg[g - r0] = (o.v - sm) / o.d; });
}

template <typename T>
__global__ void __launch_bounds__(kWB) kw_irr_scat(const BLev<T>* __restrict__ WL, const WEnt* __restrict__ tab,
                                                  const WState* __restrict__ st, int grp) {
  const WEnt e = tab[w_entry()];
  if (e.box < 0 || !st[e.box].active) return;
  const BLev<T>& L = WL[e.box];
  be_irr_scat_part<T>(L, grp, L.x, e.chunk * kWList, kWList);
}

// r = b - A x on a level: segment 0 cells, segments 1 and 2 explicit rows of
// colour group 0 and 1
template <typename T, int DIM>
__global__ void __launch_bounds__(kWB) kw_resid(const BLev<T>* __restrict__ WL, const WEnt* __restrict__ tab,
                                               const WState* __restrict__ st) {
  const WEnt e = tab[w_entry()];
  if (e.box < 0 || !st[e.box].active) return;
  const BLev<T>& L = WL[e.box];
  double a0 = 0, a1 = 0;
  if (e.seg == 0)
    be_resid_cells_part<T, T, DIM, 0, 0>(L, L.x, L.b, L.r, e.chunk * WCh<T>::v, WCh<T>::v, nullptr, a0, a1);
  else
    be_resid_rows_part<T, T, 0, 0>(L, e.seg - 1, L.x, L.b, L.r, e.chunk * kWRows, kWRows, nullptr, a0, a1);
}

// restriction of the fine residual into the coarse b, coarse x cleared:
// segment 0 coarse cells, 1 non-simple coarse unknowns, 2 coarse second-phase x
template <typename T, int DIM>
__global__ void __launch_bounds__(kWB) kw_restrict(const BLev<T>* __restrict__ WF, const BLev<T>* __restrict__ WC,
                                                  const WEnt* __restrict__ tab, const WState* __restrict__ st) {
  const WEnt e = tab[w_entry()];
  if (e.box < 0 || !st[e.box].active) return;
  const BLev<T>& F = WF[e.box];
  const BLev<T>& C = WC[e.box];
  if (e.seg == 0) {
    be_restrict_cells_part<T, DIM>(F, C, F.r, C.b, C.x, e.chunk * WCh<T>::v, WCh<T>::v);
  } else if (e.seg == 1) {
    be_restrict_ns_part<T, DIM>(F, F.r, C.b, e.chunk * kWList, kWList);
  } else {
    const int q = C.N + e.chunk * kWList + (int)threadIdx.x;
    if (q < C.N + C.N2) C.x[q] = T(0);
  }
}

// prolongation of the coarse x into the fine x: segment 0 fine cells, 1 list
template <typename T, int DIM>
__global__ void __launch_bounds__(kWB) kw_prolong(const BLev<T>* __restrict__ WF, const BLev<T>* __restrict__ WC,
                                                 const WEnt* __restrict__ tab, const WState* __restrict__ st) {
  const WEnt e = tab[w_entry()];
  if (e.box < 0 || !st[e.box].active) return;
  const BLev<T>& F = WF[e.box];
  const BLev<T>& C = WC[e.box];
  if (e.seg == 0)
    be_prolong_cells_part<T, DIM>(F, C, C.x, F.x, e.chunk * WCh<T>::v, WCh<T>::v);
  else
    be_prolong_np_part<T>(F, C.x, F.x, e.chunk * kWList, kWList);
}

// Coarse part of the cycle: workgroup k runs box list[k]'s V-cycle from its
// level lt down (the bottom solve included) and back up to lt.
template <typename T, int DIM>
__global__ void __launch_bounds__(kBE) kw_tail(const BBox<T>* __restrict__ boxes, const int32_t* __restrict__ lt,
                                              const int32_t* __restrict__ list, const WState* __restrict__ st,
                                              int which, int nu1, int nu2) {
  const int bi = list[blockIdx.x];
  if (!st[bi].active) return;
  const BBox<T>& B = boxes[bi];
  const int l0 = lt[bi];
  T* x0 = l0 == 0 ? B.zx[which] : B.lv[l0].x;
  const T* b0 = l0 == 0 ? B.zb[which] : B.lv[l0].b;
  be_vcycle<T, DIM>(B.lv, l0, B.nlev, B.Ainv, B.nbot, B.bk, nu1, nu2, x0, b0);
}

// Bottom solves x = Ainv b of boxes whose coarse part is the bottom level
// alone, kWBotRows rows of one box per entry (one wavefront per row, as the
// engine), so the inverses stream through the whole chip.
constexpr int kWBotRows = 4 * (kWB / 64);

template <typename T>
__global__ void __launch_bounds__(kWB) kw_bottom(const BBox<T>* __restrict__ boxes, const int32_t* __restrict__ lt,
                                                const WEnt* __restrict__ tab, const WState* __restrict__ st,
                                                int which) {
  const WEnt e = tab[w_entry()];
  if (e.box < 0 || !st[e.box].active) return;
  const BBox<T>& B = boxes[e.box];
  const int l0 = lt[e.box];
  T* x = l0 == 0 ? B.zx[which] : B.lv[l0].x;
  const T* b = l0 == 0 ? B.zb[which] : B.lv[l0].b;
  const int n = B.nbot;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int r1 = min(n, (e.chunk + 1) * kWBotRows);
  for (int row = e.chunk * kWBotRows + wave; row < r1; row += kWB / 64) {
    const double s = bottom_row<T>(B.Ainv + (int64_t)row * n, n, b, lane);
    if (lane == 0) x[row] = (T)s;
  }
}

// ---------------------------------------------------------------------------
// finest level in FP64: operator, right-hand side, Krylov vectors
// ---------------------------------------------------------------------------
// MODE 1: kv[out] = A x with x = zx[which] (precision TX); MODE 0: kv[out] =
// b - A x for the solution x. Per-entry partials of (kv[da], out) to part0
// and, for NDOT 2, (out, out) to part1.
template <typename T, typename TX, int DIM, int MODE, int NDOT>
__global__ void __launch_bounds__(kWB) kw_op64(const BBox<T>* __restrict__ boxes, const WEnt* __restrict__ tab,
                                              const WState* __restrict__ st, int filt, int which, int out, int da,
                                              double* __restrict__ part0, double* __restrict__ part1) {
  __shared__ double red[2][kWB / 64];
  const int idx = w_entry();
  const WEnt e = tab[idx];
  if (e.box < 0 || !w_pass(st[e.box], filt)) return;
  const BBox<T>& B = boxes[e.box];
  const BLev<double>& F = B.f64;
  const TX* x = MODE == 0 ? (const TX*)F.x : (const TX*)B.zx[which];
  double* r = B.kv[out];
  const double* dv = NDOT >= 1 ? B.kv[da] : nullptr;
  double a0 = 0, a1 = 0;
  if (e.seg == 0)
    be_resid_cells_part<double, TX, DIM, MODE, NDOT>(F, x, F.b, r, e.chunk * WCh<double>::v, WCh<double>::v, dv,
                                                     a0, a1);
  else
    be_resid_rows_part<double, TX, MODE, NDOT>(F, e.seg - 1, x, F.b, r, e.chunk * kWRows, kWRows, dv, a0, a1);
  if (NDOT >= 1) {
    const double s0 = w_block_sum(a0, red[0]);
    if (threadIdx.x == 0) part0[idx] = s0;
  }
  if (NDOT == 2) {
    const double s1 = w_block_sum(a1, red[1]);
    if (threadIdx.x == 0) part1[idx] = s1;
  }
}

struct WIO {
  const double* rho;
  const double* sigma;
  double* phi;
  double* phi2;
};

// right-hand side of every box: segment 0 cells, 1 and 2 explicit rows of
// colour group 0 and 1
template <typename T, int DIM>
__global__ void __launch_bounds__(kWB) kw_rhs(const BBox<T>* __restrict__ boxes, const WEnt* __restrict__ tab,
                                             const WIO* __restrict__ io) {
  const WEnt e = tab[w_entry()];
  if (e.box < 0) return;
  const BBox<T>& B = boxes[e.box];
  const BLev<double>& F = B.f64;
  const WIO o = io[e.box];
  if (e.seg == 0)
    be_rhs_cells_part<DIM>(F, B.dat, o.rho, F.b, e.chunk * WCh<double>::v, WCh<double>::v);
  else
    be_rhs_rows_part(F, B.fv, B.icell, B.isrc, B.iface, B.iobj, B.icobj, B.icsig, B.objv, o.rho, o.sigma, F.b,
                     F.grp_ptr[e.seg - 1] + e.chunk * kWRows,
                     min(kWRows, F.grp_ptr[e.seg] - F.grp_ptr[e.seg - 1] - e.chunk * kWRows));
}

enum WVecOp { WV_INIT = 0, WV_P, WV_S, WV_XR, WV_RESTART, WV_OUT };

// Vector steps over the finest-level unknowns (N + N2 per box):
//   INIT    x = guess (0 on covered cells); partial (b, b)
//   P       p = r + beta (p - omega v) (plain refinement: p = r); cycle input
//           zb[0] = p, cycle output zx[0] = 0
//   S       s = r - alpha v; zb[1] = s, zx[1] = 0
//   XR      x += alpha ph + omega sh; r = s - omega t; partials (rh, r), (r, r)
//   RESTART rh = r, p = v = 0
//   OUT     guess arrays = x (0 when b = 0)
// The FP64 streams of P, S and XR carry non-temporal hints, as in the
// single-box Krylov steps (a V-cycle lies between two uses of a vector).
template <typename T, int OP>
__global__ void __launch_bounds__(kWB) kw_vec(const BBox<T>* __restrict__ boxes, const WEnt* __restrict__ tab,
                                             const WState* __restrict__ st, const WIO* __restrict__ io, int filt,
                                             double* __restrict__ part0, double* __restrict__ part1) {
  __shared__ double red[2][kWB / 64];
  const int idx = w_entry();
  const WEnt e = tab[idx];
  if (e.box < 0) return;
  const WState& S = st[e.box];
  if (OP != WV_OUT && OP != WV_INIT && !w_pass(S, filt)) return;
  const BBox<T>& B = boxes[e.box];
  const int N = B.N, nd = B.N + B.N2;
  const int beg = e.chunk * kWVec + (int)threadIdx.x;
  double* __restrict__ x = B.f64.x;
  double* __restrict__ r = B.kv[0];
  double* __restrict__ rh = B.kv[1];
  double* __restrict__ p = B.kv[2];
  double* __restrict__ v = B.kv[3];
  double* __restrict__ sv = B.kv[5];
  double* __restrict__ tv = B.kv[7];
  double a0 = 0, a1 = 0;
  if (OP == WV_INIT) {
    const WIO o = io[e.box];
    const double* __restrict__ b = B.f64.b;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int i = beg + u * kWB;
      if (i < nd) {
        // covered cells (identity rows, b = 0, never updated) start at 0
        x[i] = i < N ? (tclass(B.f64.tag[i]) == 3 ? 0.0 : o.phi[i]) : (o.phi2 ? o.phi2[i - N] : 0.0);
        a0 += b[i] * b[i];
      }
    }
  } else if (OP == WV_P) {
    const bool kry = S.mode == 2;
    const double beta = kry ? (S.rho / S.rho_old) * (S.alpha / S.omega) : 0.0;
    const double om = S.omega;
    T* __restrict__ zb = B.zb[0];
    T* __restrict__ zx = B.zx[0];
    const bool sep = (void*)zb != (void*)p;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int i = beg + u * kWB;
      if (i < nd) {
        const double ri = ld_stream<true>(r + i);
        const double pv = kry ? ri + beta * (ld_stream<true>(p + i) - om * ld_stream<true>(v + i)) : ri;
        st_stream<true>(pv, p + i);
        if (sep) zb[i] = (T)pv;
        zx[i] = T(0);
      }
    }
  } else if (OP == WV_S) {
    const double al = S.alpha;
    T* __restrict__ zb = B.zb[1];
    T* __restrict__ zx = B.zx[1];
    const bool sep = (void*)zb != (void*)sv;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int i = beg + u * kWB;
      if (i < nd) {
        const double s = ld_stream<true>(r + i) - al * ld_stream<true>(v + i);
        st_stream<true>(s, sv + i);
        if (sep) zb[i] = (T)s;
        zx[i] = T(0);
      }
    }
  } else if (OP == WV_XR) {
    const double al = S.alpha, om = S.omega;
    const T* __restrict__ ph = B.zx[0];
    const T* __restrict__ sh = B.zx[1];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int i = beg + u * kWB;
      if (i < nd) {
        const double xi = ld_stream<true>(x + i);
        st_stream<true>(xi + (al * (double)ld_stream<true>(ph + i) + om * (double)ld_stream<true>(sh + i)), x + i);
        const double rn = ld_stream<true>(sv + i) - om * ld_stream<true>(tv + i);
        r[i] = rn;
        a0 += ld_stream<true>(rh + i) * rn;
        a1 += rn * rn;
      }
    }
  } else if (OP == WV_RESTART) {
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int i = beg + u * kWB;
      if (i < nd) {
        rh[i] = r[i];
        p[i] = 0.0;
        v[i] = 0.0;
      }
    }
  } else {
    const WIO o = io[e.box];
    const bool zero = S.bn == 0.0;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int i = beg + u * kWB;
      if (i < nd) {
        const double xv = zero ? 0.0 : x[i];
        if (i < N)
          o.phi[i] = xv;
        else if (o.phi2)
          o.phi2[i - N] = xv;
      }
    }
  }
  if (OP == WV_INIT || OP == WV_XR) {
    const double s0 = w_block_sum(a0, red[0]);
    if (threadIdx.x == 0) part0[idx] = s0;
  }
  if (OP == WV_XR) {
    const double s1 = w_block_sum(a1, red[1]);
    if (threadIdx.x == 0) part1[idx] = s1;
  }
}

// ---------------------------------------------------------------------------
// per-box scalars and decisions: one wavefront per box
// ---------------------------------------------------------------------------
enum WStage {
  WS_BB = 0,   // (b, b) -> ||b||; zero or non-finite right-hand sides stop here
  WS_R0,       // (r, r) of the initial residual -> start or done
  WS_A,        // (rh, v) -> alpha
  WS_B,        // (t, s), (t, t) -> omega
  WS_C,        // (rh, r), (r, r) after the update -> iterate, verify or stop
  WS_D         // (r, r) of the true residual -> converged, restart or stop
};

template <int STAGE>
__global__ void __launch_bounds__(kWB) kw_fin(const int32_t* __restrict__ ebeg, const double* __restrict__ part0,
                                             const double* __restrict__ part1, WState* __restrict__ st, int nbox,
                                             double rtol, int max_cycles) {
  const int box = blockIdx.x * (kWB / 64) + (int)(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (box >= nbox) return;
  WState& S = st[box];
  const int filt = STAGE == WS_D ? WF_VERIFY : WF_ACTIVE;
  if (!w_pass(S, filt)) return;
  const int e0 = ebeg[box], e1 = ebeg[box + 1];
  double s0 = 0, s1 = 0;
  for (int q = e0 + lane; q < e1; q += 64) {
    s0 += part0[q];
    if (STAGE == WS_R0 || STAGE == WS_B || STAGE == WS_C || STAGE == WS_D) s1 += part1[q];
  }
  for (int off = 32; off > 0; off >>= 1) {
    s0 += __shfl_down(s0, off, 64);
    s1 += __shfl_down(s1, off, 64);
  }
  if (lane != 0) return;
  const bool kry = S.mode == 2;
  if (STAGE == WS_BB) {
    const double bn = sqrt(s0);
    S.bn = bn;
    S.rel = 0;
    if (!(bn == bn) || bn > 1e300) {
      S.status = EBMG_ERR_NUMERIC;
      S.active = 0;
    } else if (bn == 0.0) {
      S.active = 0;
    }
  } else if (STAGE == WS_R0) {
    const double rel = sqrt(s1) / S.bn;
    S.rel = rel;
    if (rel <= rtol) {
      S.active = 0;
    } else {
      S.rho = s1;        // rh = r
      S.rho_old = S.alpha = S.omega = 1.0;
      S.restart = 1;
      if (S.cycles + 2 > max_cycles) {
        S.status = EBMG_ERR_NOCONV;
        S.active = 0;
      }
    }
  } else if (STAGE == WS_A) {
    S.restart = 0;
    S.rv = s0;
    S.alpha = kry ? S.rho / s0 : 1.0;
  } else if (STAGE == WS_B) {
    S.ts = s0;
    S.tt = s1;
    S.omega = kry ? (s1 > 0 ? s0 / s1 : 0.0) : 1.0;
  } else if (STAGE == WS_C) {
    S.rho_old = S.rho;
    S.rho = s0;
    S.rr = s1;
    S.cycles += 2;
    S.iters += 1;
    const double nrel = sqrt(s1) / S.bn;
    const bool broke = kry && (!(nrel == nrel) || !(S.alpha == S.alpha) || S.omega == 0.0 || !(S.omega == S.omega));
    if (broke || !(nrel == nrel) || nrel <= rtol) {
      S.verify = 1;
    } else if (nrel > 1e6) {
      S.status = EBMG_ERR_NUMERIC;
      S.active = 0;
    } else if (S.cycles + 2 > max_cycles) {
      S.status = EBMG_ERR_NOCONV;
      S.active = 0;
    }
    S.rel = nrel;
  } else {
    S.verify = 0;
    const double nrel = sqrt(s1) / S.bn;
    S.rel = nrel;
    if (!(nrel == nrel) || nrel > 1e6) {
      S.status = EBMG_ERR_NUMERIC;
      S.active = 0;
    } else if (nrel <= rtol) {
      S.active = 0;
    } else if (kry && ++S.restarts > 8) {
      S.status = EBMG_ERR_NOCONV;
      S.active = 0;
    } else {
      S.rho = s1;        // rh = r after the restart
      S.rho_old = S.alpha = S.omega = 1.0;
      S.restart = 1;
      if (S.cycles + 2 > max_cycles) {
        S.status = EBMG_ERR_NOCONV;
        S.active = 0;
      }
    }
  }
}

// number of boxes still iterating (one workgroup)
__global__ void __launch_bounds__(kWB) kw_count(const WState* __restrict__ st, int nbox, int* __restrict__ out) {
  __shared__ int red[kWB];
  int c = 0;
  for (int b = threadIdx.x; b < nbox; b += kWB) c += st[b].active != 0;
  red[threadIdx.x] = c;
  __syncthreads();
  for (int w = kWB / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = red[0];
}

}  // namespace ebmg
