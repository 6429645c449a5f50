// Single-workgroup multigrid engine (gfx950).
//
// Small levels are latency-bound: a V-cycle over them as separate grid-wide
// launches pays a launch and a drain per phase. Here one workgroup of
// kBE threads runs a whole (sub-)V-cycle -- red/black sweeps, explicit-row
// groups, residual, restriction, prolongation and the dense bottom solve --
// with workgroup barriers between phases and the level data in global memory
// (L2-resident at these sizes). It serves two uses: the coarse tail of a
// large hierarchy (one launch per V-cycle instead of ~30 per level), and the
// batched solver, where each workgroup of a persistent grid solves whole
// boxes on a fixed round-robin over a largest-first order.
//
// Phases follow the grid-wide kernels exactly (same update formulas, same
// summation orders); the explicit rows use one thread per row here.
#pragma once

#include "kernels.hpp"

namespace ebmg {

constexpr int kBE = 512;        // threads of an engine workgroup (two per CU)
constexpr int kSlice = 64;      // rows per slice of the sliced explicit-row layout (one wavefront)
constexpr int kMaxLev = 16;

// Device view of one multigrid level (all pointers device memory).
template <typename T>
struct BLev {
  int dim;
  int n[3];
  int N, N2, R;
  const uint8_t* tag;
  const int64_t* irow_dof;
  const int64_t* rp;
  const int32_t* col;
  const T* val;
  const T* diag;
  const int32_t* grp_rows;
  int grp_ptr[3];
  // sliced copy of the explicit rows: kSlice rows per slice, entry j of a
  // slice's rows contiguous; slices sl_grp[g] .. sl_grp[g + 1] - 1 hold group g
  const int64_t* sl_ptr;
  const int32_t* sl_col;
  const T* sl_val;
  int sl_grp[3];
  Tmpl<T> tp;
  T* x;
  T* b;
  T* r;
  T* w;
  // transfer to the next coarser level
  int n_ns;
  const int64_t* ns_cdof;
  const int32_t* ns_ptr;
  const int64_t* ns_child;
  int n_np;
  const int64_t* np_fdof;
  const int64_t* np_cdof;
};

template <typename T>
__device__ void be_fill(T* x, int n, T v) {
  _Pragma("unroll 4") for (int t = threadIdx.x; t < n; t += blockDim.x) x[t] = v;
  __syncthreads();
}

// deterministic workgroup dot product (fixed-order tree in LDS)
__device__ inline double be_dot(const double* __restrict__ a, const double* __restrict__ b, int n, double* red) {
  double s = 0;
  _Pragma("unroll 4") for (int t = threadIdx.x; t < n; t += blockDim.x) s += a[t] * b[t];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = blockDim.x / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  const double v = red[0];
  __syncthreads();
  return v;
}

// Loops below handle U cells per thread per iteration and issue all their
// loads before the first use (neighbours at clamped, always valid
// addresses), so a thread has U dependent load chains in flight instead of
// one; a workgroup walks a whole box alone, so that parallelism is its only
// way to cover memory latency.
template <typename T>
struct BeU {
  static constexpr int U = sizeof(T) == 4 ? 4 : 2;
};

// Every phase below comes as a "part" over the work items [beg, beg + cnt)
// of a level (cells, rows or list entries; cnt may run past the end), with
// no barrier, so that the persistent engine (one workgroup, the whole range)
// and the level-synchronous batched kernels (one chunk per workgroup) run
// the same code.
__device__ __forceinline__ int be_end(int n, int beg, int cnt) {
  return (int)min((int64_t)n, (int64_t)beg + cnt);
}
constexpr int kAll = 0x7fffffff;
// The engine's phases run inlined into different kernels (the persistent
// solver, the coarse-tail kernel and the level-synchronous kernels); with
// contraction left to the backend, a product-plus-sum could become an FMA in
// one inlining and not in another. Every product is rounded on its own
// instead, so a phase gives the same bits wherever it runs.
#define FP_EXACT_ORDER _Pragma("clang fp contract(off)")

// Global-memory views of the level's arrays: pointers read from a level
// struct are generic to the compiler, whose generic (flat) loads also count
// as LDS operations, so every use waits for all of them; through these views
// the loads are global ones, waited for one by one.
template <typename T>
using GPtr = T __attribute__((address_space(1)))*;
template <typename T>
__device__ __forceinline__ GPtr<T> gview(T* p) { return (GPtr<T>)p; }

template <typename T, int DIM>
__device__ void be_rb_part(const BLev<T>& L, T* __restrict__ xp, const T* __restrict__ bp, int colour, int beg,
                           int cnt) {
  FP_EXACT_ORDER
  const GPtr<T> x = gview(xp);
  const GPtr<const T> b = gview(bp);
  constexpr int U = BeU<T>::U;
  const int nx = L.n[0], ny = L.n[1], nz = DIM == 3 ? L.n[2] : 1;
  const int nxh = (nx + 1) >> 1;
  const int nthr = nxh * ny * nz;
  const int64_t sxy = (int64_t)nx * ny;
  const int64_t last = (int64_t)nx * ny * nz - 1;
  const Tmpl<T> tp = L.tp;
  const GPtr<const uint8_t> tag = gview(L.tag);
  const int end = be_end(nthr, beg, cnt);
  for (int t0 = beg + (int)threadIdx.x; t0 < end; t0 += blockDim.x * U) {
    int64_t cc[U];
    int ii[U], jj[U], kk[U];
    bool act[U];
    uint8_t tg[U];
    T v[U][6], bv[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int t = t0 + u * (int)blockDim.x;
      const int tt = t < nthr ? t : 0;
      const int ih = tt % nxh;
      const int jk = tt / nxh;
      const int j = jk % ny;
      const int k = DIM == 3 ? jk / ny : 0;
      const int i0 = 2 * ih + ((j + k + colour) & 1);
      act[u] = t < nthr && i0 < nx;
      // inactive lanes take cell 0 with all coordinates 0, so every address
      // below stays inside the level (neighbours only towards higher
      // indices, clamped to the last cell)
      const int i = act[u] ? i0 : 0;
      const int jj0 = act[u] ? j : 0;
      const int kk0 = act[u] ? k : 0;
      const int64_t c = act[u] ? i + (int64_t)nx * jk : 0;
      cc[u] = c;
      ii[u] = i;
      jj[u] = jj0;
      kk[u] = kk0;
      tg[u] = tag[c];
      bv[u] = b[c];
      v[u][0] = x[i > 0 ? c - 1 : c];
      v[u][1] = x[min(i < nx - 1 ? c + 1 : c, last)];
      v[u][2] = x[jj0 > 0 ? c - nx : c];
      v[u][3] = x[min(jj0 < ny - 1 ? c + nx : c, last)];
      if (DIM == 3) {
        v[u][4] = x[kk0 > 0 ? c - sxy : c];
        v[u][5] = x[min(kk0 < nz - 1 ? c + sxy : c, last)];
      }
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int p = tclass(tg[u]);
      if (!act[u] || p > 1) continue;
      T s = 0, dg = tp.D0(p);
      if (ii[u] > 0) s += v[u][0]; else dg += tp.CB(0, p);
      if (ii[u] < nx - 1) s += v[u][1]; else dg += tp.CB(1, p);
      if (jj[u] > 0) s += v[u][2]; else dg += tp.CB(2, p);
      if (jj[u] < ny - 1) s += v[u][3]; else dg += tp.CB(3, p);
      if (DIM == 3) {
        if (kk[u] > 0) s += v[u][4]; else dg += tp.CB(4, p);
        if (kk[u] < nz - 1) s += v[u][5]; else dg += tp.CB(5, p);
      }
      x[cc[u]] = (bv[u] - tp.CO(p) * s) * (T(1) / dg);
    }
  }
}

template <typename T, int DIM>
__device__ void be_rb(const BLev<T>& L, T* __restrict__ x, const T* __restrict__ b, int colour) {
  be_rb_part<T, DIM>(L, x, b, colour, 0, kAll);
  __syncthreads();
}

// Explicit rows, sliced layout: one thread per row, a wavefront per slice of
// kSlice rows of one colour group, so every column and value load is one
// contiguous wavefront access. Entries are fetched kRowJ at a time (columns
// and values, then the x values, then summed in entry order): a thread keeps
// kRowJ load chains in flight. Padding entries add 0 * x[0].
constexpr int kRowJ = 8;

// TWO: columns c >= nx name entries x2[c - nx] of a second source.
template <typename T, typename TX, bool TWO = false>
__device__ __forceinline__ T sliced_row(const int32_t* __restrict__ col, const T* __restrict__ val,
                                        const TX* __restrict__ x, int64_t p, int len,
                                        const TX* __restrict__ x2 = nullptr, int nx = 0) {
  FP_EXACT_ORDER
  const GPtr<const int32_t> cg = gview(col);
  const GPtr<const T> vg = gview(val);
  const GPtr<const TX> xg = gview(x), x2g = gview(x2);
  auto ld = [&](int c) -> T { return TWO ? (T)(c < nx ? xg[c] : x2g[c - nx]) : (T)xg[c]; };
  T s = T(0);
  int j = 0;
  for (; j + kRowJ <= len; j += kRowJ) {
    int c[kRowJ];
    T v[kRowJ], xv[kRowJ];
#pragma unroll
    for (int k = 0; k < kRowJ; ++k) {
      c[k] = cg[p + (int64_t)(j + k) * kSlice];
      v[k] = vg[p + (int64_t)(j + k) * kSlice];
    }
#pragma unroll
    for (int k = 0; k < kRowJ; ++k) xv[k] = ld(c[k]);
#pragma unroll
    for (int k = 0; k < kRowJ; ++k) s = s + v[k] * xv[k];
  }
  for (; j < len; ++j) s = s + vg[p + (int64_t)j * kSlice] * ld(cg[p + (int64_t)j * kSlice]);
  return s;
}

// Visit the rows [beg, beg + cnt) of colour group grp (relative to the
// group; beg a multiple of kSlice) one slice per wavefront. pre(g) issues the
// row's own loads (unknown index, diagonal, b) before the entry loop and
// returns them; f(g, pre, s) finishes the row, s its off-diagonal sum.
template <typename T, typename TX, bool TWO = false, typename Pre, typename F>
__device__ __forceinline__ void sliced_rows(const BLev<T>& L, int grp, const TX* __restrict__ x, int beg, int cnt,
                                            Pre&& pre, F&& f, const TX* __restrict__ x2 = nullptr, int nx = 0) {
  const int r0 = L.grp_ptr[grp];
  const int n = L.grp_ptr[grp + 1] - r0;
  const int end = be_end(n, beg, cnt);
  const int lane = threadIdx.x & (kSlice - 1), wave = threadIdx.x / kSlice, nw = blockDim.x / kSlice;
  for (int s0 = beg + wave * kSlice; s0 < end; s0 += nw * kSlice) {
    const int sl = L.sl_grp[grp] + s0 / kSlice;
    const int64_t p0 = L.sl_ptr[sl];
    const int len = (int)((L.sl_ptr[sl + 1] - p0) / kSlice);
    const int g = s0 + lane;
    const bool in = g < end;
    const auto own = pre(r0 + (in ? g : 0));
    const T sm = sliced_row<T, TX, TWO>(L.sl_col, L.sl_val, x, p0 + lane, len, x2, nx);
    if (in) f(r0 + g, own, sm);
  }
}

template <typename T>
struct RowOwn {
  int64_t q;
  T d, v;
};

// Jacobi values (b - offdiag . x) / diag of group grp's rows [beg, beg + cnt)
// (relative to the group) into w.
template <typename T, bool TWO = false>
__device__ void be_irr_jac_part(const BLev<T>& L, int grp, const T* __restrict__ x, const T* __restrict__ b,
                                int beg, int cnt, const T* __restrict__ x2 = nullptr, int nx = 0) {
  FP_EXACT_ORDER
  const int r0 = L.grp_ptr[grp];
  if (L.grp_ptr[grp + 1] <= r0) return;
  sliced_rows<T, T, TWO>(
      L, grp, x, beg, cnt,
      [&](int g) {
        const int64_t q = L.irow_dof[g];
        return RowOwn<T>{q, L.diag[g], b[q]};
      },
      [&](int g, const RowOwn<T>& o, T sm) { L.w[g - r0] = (o.v - sm) / o.d; }, x2, nx);
}

template <typename T>
__device__ void be_irr_scat_part(const BLev<T>& L, int grp, T* __restrict__ x, int beg, int cnt) {
  const int r0 = L.grp_ptr[grp];
  const int end = r0 + be_end(L.grp_ptr[grp + 1] - r0, beg, cnt);
  for (int g = r0 + beg + (int)threadIdx.x; g < end; g += blockDim.x) x[L.irow_dof[g]] = L.w[g - r0];
}

template <typename T>
__device__ void be_irr_group(const BLev<T>& L, int grp, T* __restrict__ x, const T* __restrict__ b) {
  if (L.grp_ptr[grp + 1] <= L.grp_ptr[grp]) return;
  be_irr_jac_part<T>(L, grp, x, b, 0, kAll);
  __syncthreads();
  be_irr_scat_part<T>(L, grp, x, 0, kAll);
  __syncthreads();
}

template <typename T, int DIM>
__device__ void be_smooth(const BLev<T>& L, T* x, const T* b, int sweeps) {
  for (int it = 0; it < sweeps; ++it)
    for (int colour = 0; colour < 2; ++colour) {
      be_rb<T, DIM>(L, x, b, colour);
      be_irr_group<T>(L, colour, x, b);
    }
}

// MODE 0: r = b - A x; MODE 1: r = A x. x may be narrower than T (FP32
// input widened on load). NDOT >= 1 adds da[q] * r[q] over the unknowns this
// part writes to acc0, NDOT == 2 also r[q]^2 to acc1.
template <typename T, typename TX, int DIM, int MODE, int NDOT>
__device__ void be_resid_cells_part(const BLev<T>& L, const TX* __restrict__ xp, const T* __restrict__ bp,
                                    T* __restrict__ rp, int beg, int cnt, const double* __restrict__ dap,
                                    double& acc0, double& acc1) {
  FP_EXACT_ORDER
  const GPtr<const TX> x = gview(xp);
  const GPtr<const T> b = gview(bp);
  const GPtr<T> r = gview(rp);
  const GPtr<const double> da = gview(dap);
  constexpr int U = BeU<T>::U;
  const int nx = L.n[0], ny = L.n[1], nz = DIM == 3 ? L.n[2] : 1;
  const int64_t sxy = (int64_t)nx * ny;
  const Tmpl<T> tp = L.tp;
  const GPtr<const uint8_t> tag = gview(L.tag);
  const int N = L.N;
  const int end = be_end(N, beg, cnt);
  for (int c0 = beg + (int)threadIdx.x; c0 < end; c0 += blockDim.x * U) {
    int ii[U], jj[U], kk[U], cc[U];
    uint8_t tg[U];
    T v[U][7], bv[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int c1 = c0 + u * (int)blockDim.x;
      const int c = c1 < N ? c1 : 0;
      const int i = c % nx;
      const int jk = c / nx;
      const int j = jk % ny;
      const int k = DIM == 3 ? jk / ny : 0;
      cc[u] = c1;
      ii[u] = i;
      jj[u] = j;
      kk[u] = k;
      tg[u] = tag[c];
      bv[u] = MODE == 0 ? b[c] : T(0);
      v[u][6] = (T)x[c];
      v[u][0] = (T)x[i > 0 ? c - 1 : c];
      v[u][1] = (T)x[min(i < nx - 1 ? c + 1 : c, N - 1)];
      v[u][2] = (T)x[j > 0 ? c - nx : c];
      v[u][3] = (T)x[min(j < ny - 1 ? c + nx : c, N - 1)];
      if (DIM == 3) {
        v[u][4] = (T)x[k > 0 ? c - (int)sxy : c];
        v[u][5] = (T)x[min(k < nz - 1 ? c + (int)sxy : c, N - 1)];
      }
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      if (cc[u] >= N) continue;
      const int p = tclass(tg[u]);
      if (p == 2) continue;
      T o;
      if (p == 3) {
        o = MODE == 0 ? T(0) : v[u][6];
      } else {
        const T xv = v[u][6];
        T s = 0, dg = tp.M(p);
        if (ii[u] > 0) s += v[u][0] - xv; else dg += tp.CBM(0, p);
        if (ii[u] < nx - 1) s += v[u][1] - xv; else dg += tp.CBM(1, p);
        if (jj[u] > 0) s += v[u][2] - xv; else dg += tp.CBM(2, p);
        if (jj[u] < ny - 1) s += v[u][3] - xv; else dg += tp.CBM(3, p);
        if (DIM == 3) {
          if (kk[u] > 0) s += v[u][4] - xv; else dg += tp.CBM(4, p);
          if (kk[u] < nz - 1) s += v[u][5] - xv; else dg += tp.CBM(5, p);
        }
        const T ax = dg * xv + tp.CO(p) * s;
        o = MODE == 0 ? bv[u] - ax : ax;
      }
      r[cc[u]] = o;
      if (NDOT >= 1) acc0 += da[cc[u]] * (double)o;
      if (NDOT == 2) acc1 += (double)o * (double)o;
    }
  }
}

// Explicit rows of colour group grp, [beg, beg + cnt) relative to the group.
template <typename T, typename TX, int MODE, int NDOT>
__device__ void be_resid_rows_part(const BLev<T>& L, int grp, const TX* __restrict__ xp, const T* __restrict__ bp,
                                   T* __restrict__ rp, int beg, int cnt, const double* __restrict__ dap,
                                   double& acc0, double& acc1) {
  FP_EXACT_ORDER
  if (L.grp_ptr[grp + 1] <= L.grp_ptr[grp]) return;
  const GPtr<const TX> x = gview(xp);
  const GPtr<const T> b = gview(bp);
  const GPtr<T> r = gview(rp);
  const GPtr<const double> da = gview(dap);
  const GPtr<const int64_t> dof = gview(L.irow_dof);
  const GPtr<const T> dgv = gview(L.diag);
  sliced_rows<T, TX>(
      L, grp, xp, beg, cnt,
      [&](int g) {
        const int64_t q = dof[g];
        return RowOwn<T>{q, dgv[g], (T)x[q]};
      },
      [&](int g, const RowOwn<T>& w, T sm) {
        const T ax = w.d * w.v + sm;
        const T o = MODE == 0 ? b[w.q] - ax : ax;
        r[w.q] = o;
        if (NDOT >= 1) acc0 += da[w.q] * (double)o;
        if (NDOT == 2) acc1 += (double)o * (double)o;
      });
}

template <typename T, int DIM, int MODE>
__device__ void be_resid(const BLev<T>& L, const T* __restrict__ x, const T* __restrict__ b, T* __restrict__ r) {
  double a0 = 0, a1 = 0;
  be_resid_cells_part<T, T, DIM, MODE, 0>(L, x, b, r, 0, kAll, nullptr, a0, a1);
  be_resid_rows_part<T, T, MODE, 0>(L, 0, x, b, r, 0, kAll, nullptr, a0, a1);
  be_resid_rows_part<T, T, MODE, 0>(L, 1, x, b, r, 0, kAll, nullptr, a0, a1);
  __syncthreads();
}

// Grid-wide forms of the explicit-row phases over the sliced copy, for one
// level passed by value. A launch has few rows per CU, so each 64-row slice
// is split over kRowSplit wavefronts along its entries (cutting the chain of
// dependent loads a row waits on; 4 beat 2 by 3 % and 8 by 4 % of a 256^3
// solve): block blk takes slice blk of the group, wavefront q sums the q-th
// run of entries (whole batches of kRowJ) and hands its partial sums over
// LDS, and the first finishes the rows with f(g, pre, s0 + s1 + s2 + s3).
// The sums therefore differ in rounding from the one-wavefront parts of the
// engine, and the grid-wide kernels agree only with each other.
constexpr int kRowSplit = 4;                    // wavefronts per slice
constexpr int kRowBlock = kSlice * kRowSplit;   // threads per block: one slice per block
constexpr int kSplitRows = kSlice;              // rows per block

template <typename T, typename TX, bool TWO, typename Pre, typename F>
__device__ __forceinline__ void split_rows(const BLev<T>& L, int grp, const TX* __restrict__ x, int blk, Pre&& pre,
                                           F&& f, const TX* __restrict__ x2 = nullptr, int nx = 0) {
  constexpr int S = kRowSplit, SPB = kRowBlock / kSlice / S;   // slices per block
  __shared__ T part[SPB][S][kSlice];
  const int r0 = L.grp_ptr[grp];
  const int n = L.grp_ptr[grp + 1] - r0;
  const int lane = threadIdx.x & (kSlice - 1), wave = threadIdx.x / kSlice;
  const int q = wave % S, slot = wave / S;
  const int s0 = (SPB * blk + slot) * kSlice;   // the slice's first row (group-relative)
  const bool have = s0 < n;
  const int g = s0 + lane;
  const bool in = have && g < n;
  T sm = T(0);
  auto own = pre(r0 + (in ? g : 0));
  if (have) {
    const int sl = L.sl_grp[grp] + s0 / kSlice;
    const int64_t p0 = L.sl_ptr[sl];
    const int len = (int)((L.sl_ptr[sl + 1] - p0) / kSlice);
    const int chunk = ((len + S - 1) / S + kRowJ - 1) / kRowJ * kRowJ;
    const int j0 = min(len, q * chunk), j1 = min(len, (q + 1) * chunk);
    sm = sliced_row<T, TX, TWO>(L.sl_col, L.sl_val, x, p0 + lane + (int64_t)j0 * kSlice, j1 - j0, x2, nx);
    if (q > 0) part[slot][q][lane] = sm;
  }
  __syncthreads();
  if (in && q == 0) {
#pragma unroll
    for (int k = 1; k < S; ++k) sm = sm + part[slot][k][lane];
    f(r0 + g, own, sm);
  }
}

// Jacobi values of group grp's rows into L.w (rows relative to the group).
template <typename T>
__global__ void __launch_bounds__(kRowBlock) k_irr_jac_sl(BLev<T> L, int grp, const T* __restrict__ x,
                                                       const T* __restrict__ b) {
  FP_EXACT_ORDER
  const int r0 = L.grp_ptr[grp];
  split_rows<T, T, false>(
      L, grp, x, (int)blockIdx.x,
      [&](int g) {
        const int64_t q = L.irow_dof[g];
        return RowOwn<T>{q, L.diag[g], b[q]};
      },
      [&](int g, const RowOwn<T>& o, T sm) { L.w[g - r0] = (o.v - sm) / o.d; });
}

// k_irr_jac_sl on group 0 (blocks [0, nb0)) with, in the remaining blocks,
// group 1's current values copied to w1old (one thread per row), for the
// pass below.
template <typename T>
__global__ void __launch_bounds__(kRowBlock) k_irr_jac_sl0c(BLev<T> L, int nb0, const T* __restrict__ x,
                                                         const T* __restrict__ b, T* __restrict__ w1old) {
  FP_EXACT_ORDER
  if ((int)blockIdx.x >= nb0) {
    const int g = ((int)blockIdx.x - nb0) * kRowBlock + (int)threadIdx.x;
    if (g < L.grp_ptr[2] - L.grp_ptr[1]) w1old[g] = x[L.irow_dof[L.grp_ptr[1] + g]];
    return;
  }
  const int r0 = L.grp_ptr[0];
  split_rows<T, T, false>(
      L, 0, x, (int)blockIdx.x,
      [&](int g) {
        const int64_t q = L.irow_dof[g];
        return RowOwn<T>{q, L.diag[g], b[q]};
      },
      [&](int g, const RowOwn<T>& o, T sm) { L.w[g - r0] = (o.v - sm) / o.d; });
}

// Group 1's Jacobi values written straight into x (blocks [0, nb1)) while
// the remaining blocks copy group 0's new values from L.w into x (one thread
// per row). L carries group 1's columns with every explicit-row unknown
// renamed nx + (its place in L.w): group 0's new values at [0, n0), group
// 1's values before the pass at [n0 + n1, n0 + 2 n1), so no block reads an
// entry of x that another block writes. The same values as a pass over
// group 1 reading group 0's new values after a scatter of group 0, and a
// scatter of group 1 after the pass.
template <typename T>
__global__ void __launch_bounds__(kRowBlock) k_irr_jac_sl2x(BLev<T> L, int nb1, T* __restrict__ x,
                                                         const T* __restrict__ b, const T* __restrict__ w, int nx) {
  FP_EXACT_ORDER
  if ((int)blockIdx.x >= nb1) {
    const int g = ((int)blockIdx.x - nb1) * kRowBlock + (int)threadIdx.x;
    if (g < L.grp_ptr[1] - L.grp_ptr[0]) x[L.irow_dof[L.grp_ptr[0] + g]] = w[g];
    return;
  }
  split_rows<T, T, true>(
      L, 1, (const T*)x, (int)blockIdx.x,
      [&](int g) {
        const int64_t q = L.irow_dof[g];
        return RowOwn<T>{q, L.diag[g], b[q]};
      },
      [&](int g, const RowOwn<T>& o, T sm) { x[o.q] = (o.v - sm) / o.d; }, w, nx);
}

// r = b - A x (MODE 0) or A x (MODE 1) on the explicit rows: blocks [0, nb0)
// take group 0, the rest group 1 (kSplitRows rows per block). x may be
// narrower than T; NDOT >= 1 adds da[q] * r[q] and NDOT == 2 also r[q]^2 over
// the rows, one partial per block at part[d * pt + boff + block].
template <typename T, int MODE, typename TX = T, int NDOT = 0>
__global__ void __launch_bounds__(kRowBlock) k_resid_irr_sl(BLev<T> L, int nb0, const TX* __restrict__ x,
                                                         const T* __restrict__ b, T* __restrict__ r,
                                                         const double* __restrict__ da = nullptr,
                                                         double* __restrict__ part = nullptr, int64_t pt = 0,
                                                         int64_t boff = 0) {
  FP_EXACT_ORDER
  double a0 = 0, a1 = 0;
  const int grp = (int)blockIdx.x < nb0 ? 0 : 1;
  const int blk = grp == 0 ? (int)blockIdx.x : (int)blockIdx.x - nb0;
  split_rows<T, TX, false>(
      L, grp, x, blk,
      [&](int g) {
        const int64_t q = L.irow_dof[g];
        return RowOwn<T>{q, L.diag[g], (T)x[q]};
      },
      [&](int g, const RowOwn<T>& w, T sm) {
        const T ax = w.d * w.v + sm;
        const T o = MODE == 0 ? b[w.q] - ax : ax;
        r[w.q] = o;
        if (NDOT >= 1) a0 += da[w.q] * (double)o;
        if (NDOT == 2) a1 += (double)o * (double)o;
      });
  if (NDOT > 0) block_partials<kRowBlock>(a0, a1, NDOT, part, pt, boff + blockIdx.x, threadIdx.x);
}

// Restriction of rf into the coarse b over coarse cells [beg, beg + cnt);
// xc (may be null) is cleared over the same cells.
template <typename T, int DIM>
__device__ void be_restrict_cells_part(const BLev<T>& F, const BLev<T>& Cl, const T* __restrict__ rf,
                                       T* __restrict__ bc, T* __restrict__ xc, int beg, int cnt) {
  FP_EXACT_ORDER
  constexpr int U = BeU<T>::U;
  const int cnx = Cl.n[0], cny = Cl.n[1];
  const int fnx = 2 * cnx;
  const int64_t fsxy = (int64_t)fnx * 2 * cny;
  const int CN = Cl.N;
  const T w = DIM == 3 ? T(0.125) : T(0.25);
  const int end = be_end(CN, beg, cnt);
  for (int P0 = beg + (int)threadIdx.x; P0 < end; P0 += blockDim.x * U) {
    T v[U][8];
    uint8_t tg[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int P1 = P0 + u * (int)blockDim.x;
      const int P = P1 < CN ? P1 : 0;
      const int I = P % cnx;
      const int JK = P / cnx;
      const int J = JK % cny;
      const int K = DIM == 3 ? JK / cny : 0;
      const int64_t c0 = 2 * I + (int64_t)fnx * (2 * J) + (DIM == 3 ? fsxy * (2 * K) : 0);
      tg[u] = Cl.tag[P];
      v[u][0] = rf[c0];
      v[u][1] = rf[c0 + 1];
      v[u][2] = rf[c0 + fnx];
      v[u][3] = rf[c0 + fnx + 1];
      if (DIM == 3) {
        v[u][4] = rf[c0 + fsxy];
        v[u][5] = rf[c0 + fsxy + 1];
        v[u][6] = rf[c0 + fsxy + fnx];
        v[u][7] = rf[c0 + fsxy + fnx + 1];
      }
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int P = P0 + u * (int)blockDim.x;
      if (P >= CN) continue;
      if (xc) xc[P] = T(0);
      if (tclass(tg[u]) == 3) {
        bc[P] = 0;
        continue;
      }
      if (tg[u] & 4) continue;
      T s = v[u][0] + v[u][1] + v[u][2] + v[u][3];
      if (DIM == 3) s += v[u][4] + v[u][5] + v[u][6] + v[u][7];
      bc[P] = s * w;
    }
  }
}

// Coarse unknowns of non-simple coarse cells: sums over their listed children.
template <typename T, int DIM>
__device__ void be_restrict_ns_part(const BLev<T>& F, const T* __restrict__ rf, T* __restrict__ bc, int beg,
                                    int cnt) {
  FP_EXACT_ORDER
  const T w = DIM == 3 ? T(0.125) : T(0.25);
  const int end = be_end(F.n_ns, beg, cnt);
  for (int t = beg + (int)threadIdx.x; t < end; t += blockDim.x) {
    T s = 0;
    for (int e = F.ns_ptr[t]; e < F.ns_ptr[t + 1]; ++e) s += rf[F.ns_child[e]];
    bc[F.ns_cdof[t]] = s * w;
  }
}

template <typename T, int DIM>
__device__ void be_restrict(const BLev<T>& F, const BLev<T>& Cl, const T* __restrict__ rf, T* __restrict__ bc) {
  be_restrict_cells_part<T, DIM>(F, Cl, rf, bc, nullptr, 0, kAll);
  be_restrict_ns_part<T, DIM>(F, rf, bc, 0, kAll);
  __syncthreads();
}

// Prolongation (piecewise constant) of the coarse correction ec into xf over
// fine cells [beg, beg + cnt) whose parent is simple; the listed fine
// unknowns of non-simple parents take their coarse unknown's value.
template <typename T, int DIM>
__device__ void be_prolong_cells_part(const BLev<T>& F, const BLev<T>& Cl, const T* __restrict__ ec,
                                      T* __restrict__ xf, int beg, int cnt) {
  FP_EXACT_ORDER
  constexpr int U = BeU<T>::U;
  const int fnx = F.n[0], fny = F.n[1];
  const int cnx = fnx >> 1, cny = fny >> 1;
  const int FN = F.N;
  const int end = be_end(FN, beg, cnt);
  for (int c0 = beg + (int)threadIdx.x; c0 < end; c0 += blockDim.x * U) {
    T e[U], xv[U];
    uint8_t ft[U], ct[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int c1 = c0 + u * (int)blockDim.x;
      const int c = c1 < FN ? c1 : 0;
      const int i = c % fnx;
      const int jk = c / fnx;
      const int j = jk % fny;
      const int k = DIM == 3 ? jk / fny : 0;
      const int P = (i >> 1) + cnx * ((j >> 1) + cny * (k >> 1));
      ft[u] = F.tag[c];
      ct[u] = Cl.tag[P];
      e[u] = ec[P];
      xv[u] = xf[c];
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int c = c0 + u * (int)blockDim.x;
      if (c >= FN || tclass(ft[u]) == 3 || (ct[u] & 4)) continue;
      xf[c] = xv[u] + e[u];
    }
  }
}

template <typename T>
__device__ void be_prolong_np_part(const BLev<T>& F, const T* __restrict__ ec, T* __restrict__ xf, int beg,
                                   int cnt) {
  const int end = be_end(F.n_np, beg, cnt);
  for (int t = beg + (int)threadIdx.x; t < end; t += blockDim.x) xf[F.np_fdof[t]] += ec[F.np_cdof[t]];
}

template <typename T, int DIM>
__device__ void be_prolong(const BLev<T>& F, const BLev<T>& Cl, const T* __restrict__ ec, T* __restrict__ xf) {
  be_prolong_cells_part<T, DIM>(F, Cl, ec, xf, 0, kAll);
  be_prolong_np_part<T>(F, ec, xf, 0, kAll);
  __syncthreads();
}

// One row of x = Ainv b on the bottom level (FP64 accumulation): lanes over
// columns (coalesced), fixed-order shuffle reduction; valid in lane 0.
template <typename T>
__device__ __forceinline__ double bottom_row(const double* __restrict__ arow, int n, const T* __restrict__ b,
                                             int lane) {
  FP_EXACT_ORDER
  double s = 0;
#pragma unroll 4
  for (int c = lane; c < n; c += 64) s += arow[c] * (double)b[c];
  for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
  return s;
}

// x = Ainv b, one wavefront per row
template <typename T>
__device__ void be_bottom(const double* __restrict__ Ainv, int n, const T* __restrict__ b, T* __restrict__ x) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nwaves = blockDim.x >> 6;
  for (int row = wave; row < n; row += nwaves) {
    const double s = bottom_row<T>(Ainv + (int64_t)row * n, n, b, lane);
    if (lane == 0) x[row] = (T)s;
  }
  __syncthreads();
}

// Bottom level without a dense inverse (coarsening stopped on a level too
// large to invert): BiCGStab in FP64 on it, by the whole workgroup, until
// ||r|| <= tol ||b|| (or breakdown, or maxit iterations), from x = 0. The
// operator is the level's FP64 one; the vectors are the eight work arrays.
struct BBot {
  BLev<double> L;
  double* w[8];   // x, b, r, rh, p, v, s, t (N + N2 each)
  int maxit;
  double tol;
};

template <typename T, int DIM>
__device__ void be_bottom_krylov(const BBot& K, const T* __restrict__ bin, T* __restrict__ xout) {
  __shared__ double red[kBE];
  const int n = K.L.N + K.L.N2;
  double *x = K.w[0], *b = K.w[1], *r = K.w[2], *rh = K.w[3], *p = K.w[4], *v = K.w[5], *s = K.w[6], *t = K.w[7];
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    const double bi = (double)bin[i];
    b[i] = bi;
    x[i] = 0.0;
    r[i] = bi;
    rh[i] = bi;
    p[i] = 0.0;
    v[i] = 0.0;
  }
  __syncthreads();
  const double bb = be_dot(b, b, n, red);
  if (bb > 0) {
    const double stop = K.tol * K.tol * bb;
    double rho_old = 1.0, alpha = 1.0, omega = 1.0;
    for (int it = 0; it < K.maxit; ++it) {
      const double rho = be_dot(rh, r, n, red);
      const double beta = (rho / rho_old) * (alpha / omega);
      for (int i = threadIdx.x; i < n; i += blockDim.x) p[i] = r[i] + beta * (p[i] - omega * v[i]);
      __syncthreads();
      be_resid<double, DIM, 1>(K.L, p, nullptr, v);
      alpha = rho / be_dot(rh, v, n, red);
      for (int i = threadIdx.x; i < n; i += blockDim.x) s[i] = r[i] - alpha * v[i];
      __syncthreads();
      be_resid<double, DIM, 1>(K.L, s, nullptr, t);
      const double tt = be_dot(t, t, n, red);
      omega = tt > 0 ? be_dot(t, s, n, red) / tt : 0.0;
      for (int i = threadIdx.x; i < n; i += blockDim.x) {
        x[i] += alpha * p[i] + omega * s[i];
        r[i] = s[i] - omega * t[i];
      }
      __syncthreads();
      rho_old = rho;
      const double rr = be_dot(r, r, n, red);
      if (!(rr > stop) || omega == 0.0) break;   // converged, broken down or not finite
    }
  }
  for (int i = threadIdx.x; i < n; i += blockDim.x) xout[i] = (T)x[i];
  __syncthreads();
}

// Bottom solve: dense inverse where there is one, else the Krylov solve.
template <typename T, int DIM>
__device__ void be_bottom_any(const BLev<T>& L, const double* Ainv, int nbot, const BBot* bk, const T* b, T* x) {
  if (Ainv)
    be_bottom<T>(Ainv, nbot, b, x);
  else if (bk)
    be_bottom_krylov<T, DIM>(*bk, b, x);
  else
    be_smooth<T, DIM>(L, x, b, 40);
}

// V-cycle over levels l0 .. nlev-1; level l0 uses (x0, b0), deeper levels
// their own vectors.
template <typename T, int DIM>
__device__ void be_vcycle(const BLev<T>* lv, int l0, int nlev, const double* Ainv, int nbot, const BBot* bk,
                          int nu1, int nu2, T* x0, const T* b0) {
  for (int l = l0; l < nlev - 1; ++l) {
    T* x = l == l0 ? x0 : lv[l].x;
    const T* b = l == l0 ? b0 : lv[l].b;
    be_smooth<T, DIM>(lv[l], x, b, nu1);
    be_resid<T, DIM, 0>(lv[l], x, b, lv[l].r);
    be_restrict<T, DIM>(lv[l], lv[l + 1], lv[l].r, lv[l + 1].b);
    be_fill<T>(lv[l + 1].x, lv[l + 1].N + lv[l + 1].N2, T(0));
  }
  {
    const int l = nlev - 1;
    T* x = l == l0 ? x0 : lv[l].x;
    const T* b = l == l0 ? b0 : lv[l].b;
    be_bottom_any<T, DIM>(lv[l], Ainv, nbot, bk, b, x);
  }
  for (int l = nlev - 2; l >= l0; --l) {
    T* x = l == l0 ? x0 : lv[l].x;
    const T* b = l == l0 ? b0 : lv[l].b;
    be_prolong<T, DIM>(lv[l], lv[l + 1], lv[l + 1].x, x);
    be_smooth<T, DIM>(lv[l], x, b, nu2);
  }
}

// Coarse tail of a large hierarchy: one workgroup runs the V-cycle from
// level l0 down, on (x0, b0) at level l0 (x0 holds the initial guess).
template <typename T, int DIM>
__global__ void __launch_bounds__(kBE) k_tail_vcycle(const BLev<T>* lv, int l0, int nlev, const double* Ainv,
                                                     int nbot, const BBot* bk, int nu1, int nu2, T* x0,
                                                     const T* b0) {
  be_vcycle<T, DIM>(lv, l0, nlev, Ainv, nbot, bk, nu1, nu2, x0, b0);
}

// Krylov bottom solve of a hierarchy without a dense bottom inverse, one
// workgroup of kBE threads.
template <typename T, int DIM>
__global__ void __launch_bounds__(kBE) k_bottom_krylov(const BBot* bk, const T* b, T* x) {
  be_bottom_krylov<T, DIM>(*bk, b, x);
}

}  // namespace ebmg

namespace ebmg {

// ---------------------------------------------------------------------------
// batched solver: one workgroup per box at a time
// ---------------------------------------------------------------------------
template <typename T>
struct BBox {
  int dim;
  int nlev;
  int N, N2;
  const BLev<T>* lv;     // cycle levels (precision T)
  BLev<double> f64;      // finest level in FP64 (residual, matvec, refinement)
  const double* Ainv;
  int nbot;
  const BBot* bk;        // Krylov bottom solve when there is no inverse
  // right-hand-side data
  const int64_t* icell;
  const double* isrc;
  const double* iface;
  const int32_t* iobj;
  const double* icobj;
  const double* icsig;
  Tmpl<double> dat;      // regular cells: b -= dat.CB(f, p) on touched faces
  double fv[6];
  const double* objv;
  // BiCGStab work vectors (FP64, N + N2 each): r, rh, p, v, ph, s, sh, t
  double* kv[8];
  int krylov;            // 2: BiCGStab, else plain V-cycles with refinement
  // level-synchronous solver: finest-level cycle output (ph, sh) and input
  // (p, s) of the two preconditioner applications of an iteration
  T* zx[2];
  T* zb[2];
};

struct BIO {
  const double* rho;
  const double* sigma;
  double* phi;
  double* phi2;
};

struct BRes {
  int cycles;
  int iters;
  int status;
  int pad;
  double r0;
  double rel;
};

template <int DIM>
__device__ void be_rhs_cells_part(const BLev<double>& F, const Tmpl<double>& dat, const double* rho, double* b,
                                  int beg, int cnt) {
  const int nx = F.n[0], ny = F.n[1];
  const int end = be_end(F.N, beg, cnt);
  for (int c = beg + (int)threadIdx.x; c < end; c += blockDim.x) {
    const uint8_t p = tclass(F.tag[c]);
    if (p == 3) {
      b[c] = 0;
      continue;
    }
    if (p == 2) continue;
    const int i = c % nx;
    const int jk = c / nx;
    const int j = jk % ny;
    const int k = DIM == 3 ? jk / ny : 0;
    double v = rho[c];
    if (i == 0) v -= dat.CB(0, p);
    if (i == nx - 1) v -= dat.CB(1, p);
    if (j == 0) v -= dat.CB(2, p);
    if (j == ny - 1) v -= dat.CB(3, p);
    if (DIM == 3) {
      if (k == 0) v -= dat.CB(4, p);
      if (k == F.n[2] - 1) v -= dat.CB(5, p);
    }
    b[c] = v;
  }
}

__device__ inline void be_rhs_rows_part(const BLev<double>& F, const double* fv, const int64_t* icell,
                                        const double* isrc, const double* iface, const int32_t* iobj,
                                        const double* icobj, const double* icsig, const double* objv,
                                        const double* rho, const double* sigma, double* b, int beg, int cnt) {
  const int end = be_end(F.R, beg, cnt);
  for (int t = beg + (int)threadIdx.x; t < end; t += blockDim.x) {
    const int64_t c = icell[t];
    double v = isrc[t] * rho[c];
    for (int f = 0; f < 6; ++f) v -= iface[6 * t + f] * fv[f];
    if (iobj[t] >= 0) v -= icobj[t] * objv[iobj[t]];
    if (sigma) v -= icsig[t] * sigma[c];
    b[F.irow_dof[t]] = v;
  }
}

template <int DIM>
__device__ void be_rhs(const BLev<double>& F, const Tmpl<double>& dat, const double* fv, const int64_t* icell,
                       const double* isrc, const double* iface, const int32_t* iobj, const double* icobj,
                       const double* icsig, const double* objv, const double* rho, const double* sigma, double* b) {
  be_rhs_cells_part<DIM>(F, dat, rho, b, 0, kAll);
  be_rhs_rows_part(F, fv, icell, isrc, iface, iobj, icobj, icsig, objv, rho, sigma, b, 0, kAll);
  __syncthreads();
}

// z = M r: one V-cycle from zero in precision T (FP64 in, FP64 out)
template <typename T, int DIM>
__device__ void be_precond(const BBox<T>& B, const BLev<T>* lv, int nu1, int nu2, const double* r, double* z) {
  const int nd = B.N + B.N2;
  if (sizeof(T) == sizeof(double)) {
    _Pragma("unroll 4") for (int t = threadIdx.x; t < nd; t += blockDim.x) z[t] = 0.0;
    __syncthreads();
    be_vcycle<T, DIM>(lv, 0, B.nlev, B.Ainv, B.nbot, B.bk, nu1, nu2, (T*)z, (const T*)r);
  } else {
    T* x0 = lv[0].x;
    T* b0 = lv[0].b;
    _Pragma("unroll 4") for (int t = threadIdx.x; t < nd; t += blockDim.x) {
      b0[t] = (T)r[t];
      x0[t] = T(0);
    }
    __syncthreads();
    be_vcycle<T, DIM>(lv, 0, B.nlev, B.Ainv, B.nbot, B.bk, nu1, nu2, x0, b0);
    _Pragma("unroll 4") for (int t = threadIdx.x; t < nd; t += blockDim.x) z[t] = (double)x0[t];
    __syncthreads();
  }
}

template <typename T, int DIM>
__device__ void be_solve_box(const BBox<T>& B, const BIO& io, BRes& out, double rtol, int max_cycles, int nu1,
                             int nu2, double* red) {
  const BLev<double>& F = B.f64;
  const BLev<T>* lv = B.lv;
  const int N = B.N, nd = B.N + B.N2;
  double* x = F.x;
  double* b = F.b;
  be_rhs<DIM>(F, B.dat, B.fv, B.icell, B.isrc, B.iface, B.iobj, B.icobj, B.icsig, B.objv, io.rho, io.sigma,
              b);
  // the guess; covered cells (identity rows, b = 0, never updated) start at 0
  _Pragma("unroll 4") for (int t = threadIdx.x; t < nd; t += blockDim.x) x[t] =
      t < N ? (tclass(F.tag[t]) == 3 ? 0.0 : io.phi[t]) : (io.phi2 ? io.phi2[t - N] : 0.0);
  __syncthreads();
  const double bn = sqrt(be_dot(b, b, nd, red));
  int status = 0, cycles = 0, iters = 0;
  double rel = 0;
  if (!(bn == bn) || bn > 1e300) {
    status = EBMG_ERR_NUMERIC;
  } else if (bn > 0) {
    double* r = B.kv[0];
    be_resid<double, DIM, 0>(F, x, b, r);
    rel = sqrt(be_dot(r, r, nd, red)) / bn;
    if (B.krylov != 2) {
      double* e = B.kv[4];
      while (rel > rtol) {
        if (cycles >= max_cycles) {
          status = EBMG_ERR_NOCONV;
          break;
        }
        be_precond<T, DIM>(B, lv, nu1, nu2, r, e);
        _Pragma("unroll 4") for (int t = threadIdx.x; t < nd; t += blockDim.x) x[t] += e[t];
        __syncthreads();
        ++cycles;
        ++iters;
        be_resid<double, DIM, 0>(F, x, b, r);
        rel = sqrt(be_dot(r, r, nd, red)) / bn;
        if (!(rel == rel) || rel > 1e6) {
          status = EBMG_ERR_NUMERIC;
          break;
        }
      }
    } else {
      double *rh = B.kv[1], *p = B.kv[2], *v = B.kv[3], *ph = B.kv[4], *sv = B.kv[5], *sh = B.kv[6],
             *tv = B.kv[7];
      int restarts = 0;
      double rho_old = 1, alpha = 1, omega = 1;
      _Pragma("unroll 4") for (int t = threadIdx.x; t < nd; t += blockDim.x) {
        rh[t] = r[t];
        p[t] = 0;
        v[t] = 0;
      }
      __syncthreads();
      while (rel > rtol) {
        if (cycles + 2 > max_cycles) {
          status = EBMG_ERR_NOCONV;
          break;
        }
        const double rho = be_dot(rh, r, nd, red);
        const double beta = (rho / rho_old) * (alpha / omega);
        _Pragma("unroll 4") for (int t = threadIdx.x; t < nd; t += blockDim.x) p[t] = r[t] + beta * (p[t] - omega * v[t]);
        __syncthreads();
        be_precond<T, DIM>(B, lv, nu1, nu2, p, ph);
        be_resid<double, DIM, 1>(F, ph, nullptr, v);
        alpha = rho / be_dot(rh, v, nd, red);
        _Pragma("unroll 4") for (int t = threadIdx.x; t < nd; t += blockDim.x) sv[t] = r[t] - alpha * v[t];
        __syncthreads();
        be_precond<T, DIM>(B, lv, nu1, nu2, sv, sh);
        be_resid<double, DIM, 1>(F, sh, nullptr, tv);
        const double ts = be_dot(tv, sv, nd, red);
        const double tt = be_dot(tv, tv, nd, red);
        omega = tt > 0 ? ts / tt : 0.0;
        rho_old = rho;
        _Pragma("unroll 4") for (int t = threadIdx.x; t < nd; t += blockDim.x) {
          x[t] += alpha * ph[t] + omega * sh[t];
          r[t] = sv[t] - omega * tv[t];
        }
        __syncthreads();
        cycles += 2;
        ++iters;
        double nrel = sqrt(be_dot(r, r, nd, red)) / bn;
        const bool broke = !(nrel == nrel) || !(alpha == alpha) || omega == 0.0 || !(omega == omega);
        if (broke || nrel <= rtol) {
          be_resid<double, DIM, 0>(F, x, b, r);
          nrel = sqrt(be_dot(r, r, nd, red)) / bn;
          if (!(nrel == nrel) || nrel > 1e6) {
            rel = nrel;
            status = EBMG_ERR_NUMERIC;
            break;
          }
          if (nrel > rtol) {
            if (++restarts > 8) {
              rel = nrel;
              status = EBMG_ERR_NOCONV;
              break;
            }
            _Pragma("unroll 4") for (int t = threadIdx.x; t < nd; t += blockDim.x) {
              rh[t] = r[t];
              p[t] = 0;
              v[t] = 0;
            }
            __syncthreads();
            rho_old = alpha = omega = 1;
          }
        } else if (nrel > 1e6) {
          rel = nrel;
          status = EBMG_ERR_NUMERIC;
          break;
        }
        rel = nrel;
      }
    }
  } else {
    _Pragma("unroll 4") for (int t = threadIdx.x; t < nd; t += blockDim.x) x[t] = 0;
    __syncthreads();
  }
  _Pragma("unroll 4") for (int t = threadIdx.x; t < nd; t += blockDim.x) {
    if (t < N)
      io.phi[t] = x[t];
    else if (io.phi2)
      io.phi2[t - N] = x[t];
  }
  if (threadIdx.x == 0) {
    out.cycles = cycles;
    out.iters = iters;
    out.status = status;
    out.r0 = bn;
    out.rel = rel;
  }
  __syncthreads();
}

// Persistent batched solve: workgroup g solves boxes order[g], order[g+G], ...
// (order lists the boxes largest first), so the assignment is fixed and the
// result of a box does not depend on the others.
template <typename T, int DIM>
__global__ void __launch_bounds__(kBE) k_batch_solve(const BBox<T>* boxes, const BIO* io, BRes* res,
                                                     const int32_t* order, int nbox, double rtol, int max_cycles,
                                                     int nu1, int nu2) {
  __shared__ double red[kBE];
  for (int q = blockIdx.x; q < nbox; q += gridDim.x) {
    const int bi = order[q];
    be_solve_box<T, DIM>(boxes[bi], io[bi], res[bi], rtol, max_cycles, nu1, nu2, red);
  }
}

}  // namespace ebmg
