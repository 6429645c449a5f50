// HIP kernels of the multigrid cycle (gfx950, wave64).
//
// Regular cells (tag 0/1) evaluate the (2D+1)-point template on the fly:
//   (A x)_i = diag_i x_i + coff[p] * sum_{in-box nb} x_nb,
//   diag_i  = d0[p] + sum_{domain faces touched} cb[f][p];
// irregular unknowns (tag 2 cells and all second-phase unknowns) use explicit
// sparse rows. A smoothing sweep updates the red regular cells (they read
// only black cells), then the explicit rows of red cells, then the black
// regular cells, then the explicit rows of black cells. Explicit rows of one
// colour may reference each other (ray stencils reach two cells), so each
// group is updated Jacobi-style through a temporary buffer; every launch is
// race-free and every sweep bitwise deterministic.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ebmg {

template <typename T>
struct Tmpl {
  T coff[2];
  T d0[2];
  T cb[6][2];
  // the residual's difference form: A x_i = (mass + sum over touched domain
  // faces of cbm) x_i + coff * sum over neighbours of (x_j - x_i), with
  // cbm = cb - coff; the same operator, without the cancellation of the
  // large diagonal against the neighbour sum that limits the attainable
  // relative residual on fine grids
  T mass[2];
  T cbm[6][2];
  int n[3];
  // phase-selected constants: a select between the two values keeps them in
  // registers (indexing by a runtime phase would read the argument block
  // from memory inside the loops and stall on every outstanding load)
  __device__ __forceinline__ T CO(int p) const { return p ? coff[1] : coff[0]; }
  __device__ __forceinline__ T D0(int p) const { return p ? d0[1] : d0[0]; }
  __device__ __forceinline__ T CB(int f, int p) const { return p ? cb[f][1] : cb[f][0]; }
  __device__ __forceinline__ T M(int p) const { return p ? mass[1] : mass[0]; }
  __device__ __forceinline__ T CBM(int f, int p) const { return p ? cbm[f][1] : cbm[f][0]; }
};

constexpr int kBlock = 256;
constexpr int kNormBlocks = 1024;

// Streams that a launch reads or writes exactly once (right-hand sides,
// tags, outputs) carry non-temporal hints when HINT is set, so they do not
// displace the x planes that neighbouring tiles re-read from the caches. On
// gfx950 this pays for the FP64 residual (8-byte streams, ~11 % at 256^3)
// and costs the FP32 kernels, which therefore load plainly.
template <bool HINT, typename T>
__device__ __forceinline__ T ld_stream(const T* p) {
  if (HINT) return __builtin_nontemporal_load(p);
  return *p;
}
template <bool HINT, typename T>
__device__ __forceinline__ void st_stream(T v, T* p) {
  if (HINT)
    __builtin_nontemporal_store(v, p);
  else
    *p = v;
}

__device__ __forceinline__ uint8_t tclass(uint8_t t) { return t & 3; }

template <typename T, int DIM>
__device__ __forceinline__ T template_apply(const T* __restrict__ x, const Tmpl<T>& tp, int i, int j, int k,
                                            int64_t c, int p, T& diag) {
  const int nx = tp.n[0], ny = tp.n[1];
  T s = 0;
  T dg = tp.D0(p);
  if (i > 0) s += x[c - 1]; else dg += tp.CB(0, p);
  if (i < nx - 1) s += x[c + 1]; else dg += tp.CB(1, p);
  if (j > 0) s += x[c - nx]; else dg += tp.CB(2, p);
  if (j < ny - 1) s += x[c + nx]; else dg += tp.CB(3, p);
  if (DIM == 3) {
    const int64_t sxy = (int64_t)nx * ny;
    if (k > 0) s += x[c - sxy]; else dg += tp.CB(4, p);
    if (k < tp.n[2] - 1) s += x[c + sxy]; else dg += tp.CB(5, p);
  }
  diag = dg;
  return tp.CO(p) * s;
}

// Gauss-Seidel update of a template cell: (b - coff * sum) times the
// reciprocal of the diagonal. Every smoother kernel computes it this way, so
// all sweep variants agree bitwise.
template <typename T>
__device__ __forceinline__ T tmpl_update_r(const Tmpl<T>& tp, int p, T bc, T s, T rdg) {
  return (bc - tp.CO(p) * s) * rdg;
}

template <typename T>
__device__ __forceinline__ T tmpl_update(const Tmpl<T>& tp, int p, T bc, T s, T dg) {
  return tmpl_update_r<T>(tp, p, bc, s, T(1) / dg);
}

// Red/black Gauss-Seidel half-sweep over regular cells on a 3D launch grid:
// x threads take the cells of one colour along a row (i = 2*ih + parity),
// grid y/z give the row and plane, so no index division is needed.
template <typename T, int DIM>
__global__ void __launch_bounds__(kBlock) k_rb(const uint8_t* __restrict__ tag, T* __restrict__ x,
                                               const T* __restrict__ b, Tmpl<T> tp, int colour) {
  const int ih = blockIdx.x * blockDim.x + threadIdx.x;
  const int j = blockIdx.y * blockDim.y + threadIdx.y;
  const int k = DIM == 3 ? (int)blockIdx.z : 0;
  if (j >= tp.n[1]) return;
  const int i = 2 * ih + ((j + k + colour) & 1);
  if (i >= tp.n[0]) return;
  const int64_t c = i + (int64_t)tp.n[0] * (j + (int64_t)tp.n[1] * k);
  const uint8_t p = tclass(tag[c]);
  if (p > 1) return;
  T dg;
  const T off = template_apply<T, DIM>(x, tp, i, j, k, c, p, dg);
  x[c] = (b[c] - off) * (T(1) / dg);
}

// Fused red+black sweep over regular cells, out of place (xin -> xout).
// A block owns a tile of cells: it loads the tile with a halo ring of two
// cells into LDS in one phase, applies the red update to the tile and a ring
// of one cell (old values only), then the black update to the tile (red-
// updated values only) -- exactly a red half-sweep followed by a black
// half-sweep. Ring cells are recomputed redundantly by neighbouring blocks
// from the same old values, so blocks never exchange data. Explicit-row,
// covered and second-phase values are copied through unchanged. Blocks are
// numbered so that consecutive tiles of a slab fall on the same XCD (the
// hardware deals workgroups round-robin over the 8 XCDs), keeping halo
// re-reads in that XCD's L2.
constexpr int kTX = 32, kTY = 8, kTZ = 8;     // 3D tile
constexpr int kTX2 = 64, kTY2 = 32;           // 2D tile
constexpr int kXCD = 8;

__device__ __forceinline__ int64_t xcd_block(int64_t bid, int64_t nblocks) {
  if (nblocks % kXCD) return bid;
  return (bid % kXCD) * (nblocks / kXCD) + bid / kXCD;
}

constexpr int kTileThreads = 512;

// All global loads of a block (halo tile, and the tag and b values of the
// cells this thread updates) are issued up front into registers, so one
// memory latency is exposed per block instead of one per phase.
template <typename T>
__global__ void __launch_bounds__(kTileThreads) k_rb_tile3(const uint8_t* __restrict__ tag,
                                                           const T* __restrict__ xin, T* __restrict__ xout,
                                                           const T* __restrict__ b, Tmpl<T> tp, int64_t nsec) {
  constexpr int OX = kTX + 4, OY = kTY + 4, OZ = kTZ + 4, NOq = OX * OY * OZ;
  constexpr int RX = kTX + 2, RY = kTY + 2, RZ = kTZ + 2, NRq = RX * RY * RZ;
  constexpr int NTq = kTX * kTY * kTZ;
  constexpr int NT = kTileThreads;
  constexpr int UO = (NOq + NT - 1) / NT, UR = (NRq + NT - 1) / NT, UT = (NTq + NT - 1) / NT;
  __shared__ T O[NOq];
  __shared__ T R[NRq];
  const int nx = tp.n[0], ny = tp.n[1], nz = tp.n[2];
  const int bx = (nx + kTX - 1) / kTX, by = (ny + kTY - 1) / kTY;
  const int64_t nblocks = (int64_t)gridDim.x;
  const int64_t t = xcd_block(blockIdx.x, nblocks);
  const int x0 = (int)(t % bx) * kTX, y0 = (int)((t / bx) % by) * kTY, z0 = (int)(t / ((int64_t)bx * by)) * kTZ;
  const int tid = threadIdx.x;
  const int64_t sxy = (int64_t)nx * ny;
  T ov[UO];
  uint8_t rt[UR], bt[UT];
  T rb[UR], bb[UT];
#pragma unroll
  for (int u = 0; u < UO; ++u) {
    const int q = tid + u * NT;
    ov[u] = T(0);
    if (q < NOq) {
      const int gx = x0 + q % OX - 2, gy = y0 + (q / OX) % OY - 2, gz = z0 + q / (OX * OY) - 2;
      if (gx >= 0 && gx < nx && gy >= 0 && gy < ny && gz >= 0 && gz < nz) ov[u] = xin[gx + (int64_t)nx * gy + sxy * gz];
    }
  }
#pragma unroll
  for (int u = 0; u < UR; ++u) {
    const int q = tid + u * NT;
    rt[u] = 3;
    rb[u] = T(0);
    if (q < NRq) {
      const int gx = x0 + q % RX - 1, gy = y0 + (q / RX) % RY - 1, gz = z0 + q / (RX * RY) - 1;
      if (gx >= 0 && gx < nx && gy >= 0 && gy < ny && gz >= 0 && gz < nz && ((gx + gy + gz) & 1) == 0) {
        const int64_t c = gx + (int64_t)nx * gy + sxy * gz;
        rt[u] = tclass(tag[c]);
        rb[u] = b[c];
      }
    }
  }
#pragma unroll
  for (int u = 0; u < UT; ++u) {
    const int q = tid + u * NT;
    bt[u] = 3;
    bb[u] = T(0);
    if (q < NTq) {
      const int gx = x0 + q % kTX, gy = y0 + (q / kTX) % kTY, gz = z0 + q / (kTX * kTY);
      if (gx < nx && gy < ny && gz < nz && ((gx + gy + gz) & 1) == 1) {
        const int64_t c = gx + (int64_t)nx * gy + sxy * gz;
        bt[u] = tclass(tag[c]);
        bb[u] = b[c];
      }
    }
  }
#pragma unroll
  for (int u = 0; u < UO; ++u) {
    const int q = tid + u * NT;
    if (q < NOq) O[q] = ov[u];
  }
  __syncthreads();
#pragma unroll
  for (int u = 0; u < UR; ++u) {
    const int q = tid + u * NT;
    if (q >= NRq) continue;
    const int lx = q % RX, ly = (q / RX) % RY, lz = q / (RX * RY);
    const int gx = x0 + lx - 1, gy = y0 + ly - 1, gz = z0 + lz - 1;
    const int oq = (lx + 1) + OX * ((ly + 1) + OY * (lz + 1));
    T v = O[oq];
    const int p = rt[u];
    if (p <= 1) {
      T sum = 0, dg = tp.D0(p);
      if (gx > 0) sum += O[oq - 1]; else dg += tp.CB(0, p);
      if (gx < nx - 1) sum += O[oq + 1]; else dg += tp.CB(1, p);
      if (gy > 0) sum += O[oq - OX]; else dg += tp.CB(2, p);
      if (gy < ny - 1) sum += O[oq + OX]; else dg += tp.CB(3, p);
      if (gz > 0) sum += O[oq - OX * OY]; else dg += tp.CB(4, p);
      if (gz < nz - 1) sum += O[oq + OX * OY]; else dg += tp.CB(5, p);
      v = tmpl_update<T>(tp, p, rb[u], sum, dg);
    }
    R[q] = v;
  }
  __syncthreads();
#pragma unroll
  for (int u = 0; u < UT; ++u) {
    const int q = tid + u * NT;
    if (q >= NTq) continue;
    const int lx = q % kTX, ly = (q / kTX) % kTY, lz = q / (kTX * kTY);
    const int gx = x0 + lx, gy = y0 + ly, gz = z0 + lz;
    if (gx >= nx || gy >= ny || gz >= nz) continue;
    const int rq = (lx + 1) + RX * ((ly + 1) + RY * (lz + 1));
    T v = R[rq];
    const int p = bt[u];
    if (p <= 1) {
      T sum = 0, dg = tp.D0(p);
      if (gx > 0) sum += R[rq - 1]; else dg += tp.CB(0, p);
      if (gx < nx - 1) sum += R[rq + 1]; else dg += tp.CB(1, p);
      if (gy > 0) sum += R[rq - RX]; else dg += tp.CB(2, p);
      if (gy < ny - 1) sum += R[rq + RX]; else dg += tp.CB(3, p);
      if (gz > 0) sum += R[rq - RX * RY]; else dg += tp.CB(4, p);
      if (gz < nz - 1) sum += R[rq + RX * RY]; else dg += tp.CB(5, p);
      v = tmpl_update<T>(tp, p, bb[u], sum, dg);
    }
    xout[gx + (int64_t)nx * gy + sxy * gz] = v;
  }
  // second-phase unknowns are not touched by this sweep: copy them through
  const int64_t N = sxy * nz;
  for (int64_t q = (int64_t)blockIdx.x * NT + tid; q < nsec; q += nblocks * NT) xout[N + q] = xin[N + q];
}

template <typename T>
__global__ void __launch_bounds__(kTileThreads) k_rb_tile2(const uint8_t* __restrict__ tag,
                                                           const T* __restrict__ xin, T* __restrict__ xout,
                                                           const T* __restrict__ b, Tmpl<T> tp, int64_t nsec) {
  constexpr int OX = kTX2 + 4, OY = kTY2 + 4, NOq = OX * OY;
  constexpr int RX = kTX2 + 2, RY = kTY2 + 2, NRq = RX * RY;
  constexpr int NTq = kTX2 * kTY2;
  constexpr int NT = kTileThreads;
  constexpr int UO = (NOq + NT - 1) / NT, UR = (NRq + NT - 1) / NT, UT = (NTq + NT - 1) / NT;
  __shared__ T O[NOq];
  __shared__ T R[NRq];
  const int nx = tp.n[0], ny = tp.n[1];
  const int bx = (nx + kTX2 - 1) / kTX2;
  const int64_t nblocks = (int64_t)gridDim.x;
  const int64_t t = xcd_block(blockIdx.x, nblocks);
  const int x0 = (int)(t % bx) * kTX2, y0 = (int)(t / bx) * kTY2;
  const int tid = threadIdx.x;
  T ov[UO];
  uint8_t rt[UR], bt[UT];
  T rb[UR], bb[UT];
#pragma unroll
  for (int u = 0; u < UO; ++u) {
    const int q = tid + u * NT;
    ov[u] = T(0);
    if (q < NOq) {
      const int gx = x0 + q % OX - 2, gy = y0 + q / OX - 2;
      if (gx >= 0 && gx < nx && gy >= 0 && gy < ny) ov[u] = xin[gx + (int64_t)nx * gy];
    }
  }
#pragma unroll
  for (int u = 0; u < UR; ++u) {
    const int q = tid + u * NT;
    rt[u] = 3;
    rb[u] = T(0);
    if (q < NRq) {
      const int gx = x0 + q % RX - 1, gy = y0 + q / RX - 1;
      if (gx >= 0 && gx < nx && gy >= 0 && gy < ny && ((gx + gy) & 1) == 0) {
        const int64_t c = gx + (int64_t)nx * gy;
        rt[u] = tclass(tag[c]);
        rb[u] = b[c];
      }
    }
  }
#pragma unroll
  for (int u = 0; u < UT; ++u) {
    const int q = tid + u * NT;
    bt[u] = 3;
    bb[u] = T(0);
    if (q < NTq) {
      const int gx = x0 + q % kTX2, gy = y0 + q / kTX2;
      if (gx < nx && gy < ny && ((gx + gy) & 1) == 1) {
        const int64_t c = gx + (int64_t)nx * gy;
        bt[u] = tclass(tag[c]);
        bb[u] = b[c];
      }
    }
  }
#pragma unroll
  for (int u = 0; u < UO; ++u) {
    const int q = tid + u * NT;
    if (q < NOq) O[q] = ov[u];
  }
  __syncthreads();
#pragma unroll
  for (int u = 0; u < UR; ++u) {
    const int q = tid + u * NT;
    if (q >= NRq) continue;
    const int lx = q % RX, ly = q / RX;
    const int gx = x0 + lx - 1, gy = y0 + ly - 1;
    const int oq = (lx + 1) + OX * (ly + 1);
    T v = O[oq];
    const int p = rt[u];
    if (p <= 1) {
      T sum = 0, dg = tp.D0(p);
      if (gx > 0) sum += O[oq - 1]; else dg += tp.CB(0, p);
      if (gx < nx - 1) sum += O[oq + 1]; else dg += tp.CB(1, p);
      if (gy > 0) sum += O[oq - OX]; else dg += tp.CB(2, p);
      if (gy < ny - 1) sum += O[oq + OX]; else dg += tp.CB(3, p);
      v = tmpl_update<T>(tp, p, rb[u], sum, dg);
    }
    R[q] = v;
  }
  __syncthreads();
#pragma unroll
  for (int u = 0; u < UT; ++u) {
    const int q = tid + u * NT;
    if (q >= NTq) continue;
    const int lx = q % kTX2, ly = q / kTX2;
    const int gx = x0 + lx, gy = y0 + ly;
    if (gx >= nx || gy >= ny) continue;
    const int rq = (lx + 1) + RX * (ly + 1);
    T v = R[rq];
    const int p = bt[u];
    if (p <= 1) {
      T sum = 0, dg = tp.D0(p);
      if (gx > 0) sum += R[rq - 1]; else dg += tp.CB(0, p);
      if (gx < nx - 1) sum += R[rq + 1]; else dg += tp.CB(1, p);
      if (gy > 0) sum += R[rq - RX]; else dg += tp.CB(2, p);
      if (gy < ny - 1) sum += R[rq + RX]; else dg += tp.CB(3, p);
      v = tmpl_update<T>(tp, p, bb[u], sum, dg);
    }
    xout[gx + (int64_t)nx * gy] = v;
  }
  const int64_t N = (int64_t)nx * ny;
  for (int64_t q = (int64_t)blockIdx.x * NT + tid; q < nsec; q += nblocks * NT) xout[N + q] = xin[N + q];
}

// Fused red+black sweep in 3D, out of place (xin -> xout), marching along z.
// A block owns a TX x TY column of cells over KZ planes. It keeps five planes
// of the (TX+4) x (TY+4) halo region in LDS (a ring of planes k-2 .. k+2).
// Step k applies the red update to plane k over the tile plus a one-cell ring
// (old black values only), then the black update to the tile of plane k-1
// (red-updated values only) and writes plane k-1: exactly a red half-sweep
// followed by a black half-sweep, with the same arithmetic as the split
// kernels. Each step first moves plane k+2 from registers to LDS (into the
// ring slots of planes k-3 and k-2, which no phase of step k reads) and
// requests plane k+4 from memory, so each load has two steps to arrive; two
// barriers per step. The staging runs every step (the last requests repeat
// the final plane) so that the compiler's wait counts stay exact across
// the loop, and staging slots go to lanes in reverse order, so the partial
// last slot falls on the waves without a second red cell. Ring cells and the two extra planes at each
// end of the z range are recomputed by the neighbouring blocks from the same
// old values, so blocks never exchange data. Threads take cells of one colour
// at a time (no idle lanes): each of the TX*TY/2 threads owns one black tile
// cell and its red partner. Out-of-box halo entries hold 0, so the neighbour
// sums need no masks; the in-plane boundary terms of the diagonal are folded
// into per-thread reciprocal diagonals once, and only planes at the z faces
// take the general path. (Written without lambdas so that every per-thread
// table stays in registers.)
// The update of one template cell from its six neighbour values. Inner form
// (cell not on a z face): the neighbours summed in the order x-, x+, y-, y+,
// z-, z+ (out-of-box neighbours hold 0) and scaled by the reciprocal in-plane
// diagonal rdg; general form: boundary faces skipped in the sum and folded
// into the diagonal.
template <typename T>
__device__ __forceinline__ T zv_general(T w, T e, T so, T no, T dn, T up, int gx, int gy, int z, int nx, int ny,
                                        int nz, const T* tc, T bc) {
  T s = 0, dg = tc[1];
  s += gx > 0 ? w : T(0);
  dg += gx > 0 ? T(0) : tc[2];
  s += gx < nx - 1 ? e : T(0);
  dg += gx < nx - 1 ? T(0) : tc[3];
  s += gy > 0 ? so : T(0);
  dg += gy > 0 ? T(0) : tc[4];
  s += gy < ny - 1 ? no : T(0);
  dg += gy < ny - 1 ? T(0) : tc[5];
  s += z > 0 ? dn : T(0);
  dg += z > 0 ? T(0) : tc[6];
  s += z < nz - 1 ? up : T(0);
  dg += z < nz - 1 ? T(0) : tc[7];
  return (bc - tc[0] * s) * (T(1) / dg);
}

template <typename T>
__device__ __forceinline__ T zv_inner(T w, T e, T so, T no, T dn, T up, T co, T bc, T rdg) {
  T s = w;
  s += e;
  s += so;
  s += no;
  s += dn;
  s += up;
  return (bc - co * s) * rdg;
}

template <typename T>
__device__ __forceinline__ T zm_update_general(const T* vm, const T* vc, const T* vp, int oq, int OX, int gx,
                                               int gy, int z, int nx, int ny, int nz, const T* tc, T bc) {
  return zv_general<T>(vc[oq - 1], vc[oq + 1], vc[oq - OX], vc[oq + OX], vm[oq], vp[oq], gx, gy, z, nx, ny, nz, tc,
                       bc);
}

template <typename T>
__device__ __forceinline__ T zm_update_inner(const T* vm, const T* vc, const T* vp, int oq, int OX, T co, T bc,
                                             T rdg) {
  return zv_inner<T>(vc[oq - 1], vc[oq + 1], vc[oq - OX], vc[oq + OX], vm[oq], vp[oq], co, bc, rdg);
}

template <typename T>
__device__ __forceinline__ T zm_inplane_rdg(int gx, int gy, int nx, int ny, const T* tc) {
  T dg = tc[1];
  dg += gx > 0 ? T(0) : tc[2];
  dg += gx < nx - 1 ? T(0) : tc[3];
  dg += gy > 0 ? T(0) : tc[4];
  dg += gy < ny - 1 ? T(0) : tc[5];
  return T(1) / dg;
}

// WIDE: the halo and ring regions are fetched as aligned 16-byte chunks of x
// and b and 4-byte words of tags (the chunk rows extend past the regions to
// alignment) and scattered into the same LDS layout; needs nx % 4 == 0.
// ZIN: x is zero on entry (the first sweep of a V-cycle level from a zero
// correction): xin is not read, every x value staged is 0 and the
// second-phase unknowns are written as 0; the result is the same.
template <typename T, int TX, int TY, int KZ, bool WIDE = false, bool ZIN = false>
__global__ void __launch_bounds__(TX * TY / 2) k_rb_zm3(const uint8_t* __restrict__ tag,
                                                      const T* __restrict__ xin, T* __restrict__ xout,
                                                      const T* __restrict__ b, Tmpl<T> tp, int64_t nsec) {
  constexpr int NT = TX * TY / 2;
  constexpr int OX = TX + 4, OY = TY + 4, NO = OX * OY;      // old-value halo region
  constexpr int RX = TX + 2, RY = TY + 2, NR = RX * RY;      // red ring region
  constexpr int NRED = (RX / 2) * RY;                        // red cells of the ring region
  constexpr int UO = (NO + NT - 1) / NT, UR = (NR + NT - 1) / NT;
  // wide fetch: VW values per x / b chunk, 4 tags per word, chunks per row
  constexpr int VW = 16 / (int)sizeof(T);
  constexpr int CPO = TX / VW + 2, CPR = TX / VW + 2, CPT = TX / 4 + 2;
  constexpr int NOW = CPO * OY, NRW = CPR * RY, NTW = CPT * RY;
  constexpr int UOW = (NOW + NT - 1) / NT, URW = (NRW + NT - 1) / NT, UTW = (NTW + NT - 1) / NT;
  typedef T VT __attribute__((ext_vector_type(16 / sizeof(T))));
  static_assert(TX % 4 == 0, "wide fetch needs a tile width that is a multiple of 4");
  static_assert(TX % 2 == 0, "tile width must be even");
  static_assert(NRED <= 2 * NT, "two red cells per thread at most");
  static_assert(NRED >= NT, "every thread has a first red cell");
  // planes padded to whole staging rounds, so every staging store of a
  // round lands in the array (the slots past NO / NR are never read)
  constexpr int NOP = UO * NT > NO ? UO * NT : NO, NRP = UR * NT > NR ? UR * NT : NR;
  __shared__ T V[5][NOP];
  __shared__ T Bs[4][NRP];
  __shared__ uint8_t Ts[4][NRP];
  // the template constants per phase (coff, d0, cb[0..5]): a phase chosen per
  // cell then reads LDS instead of the argument block in memory
  __shared__ T TC[2][8];
  const int nx = tp.n[0], ny = tp.n[1], nz = tp.n[2];
  const int bx = (nx + TX - 1) / TX, by = (ny + TY - 1) / TY;
  const int64_t nblocks = (int64_t)gridDim.x;
  const int64_t t = xcd_block(blockIdx.x, nblocks);
  const int x0 = (int)(t % bx) * TX, y0 = (int)((t / bx) % by) * TY;
  const int z0 = (int)(t / ((int64_t)bx * by)) * KZ;
  const int z1 = min(z0 + KZ, nz);
  const int tid = threadIdx.x;
  const int stid = NT - 1 - tid;   // staging lane (reversed)
  const int64_t sxy = (int64_t)nx * ny;
  if (tid < 16) {
    const int p = tid >> 3, j = tid & 7;
    TC[p][j] = j == 0 ? tp.coff[p] : (j == 1 ? tp.d0[p] : tp.cb[j - 2][p]);
  }
  __syncthreads();

  // per-thread tables, fixed over the march: in-plane offsets of the loaded
  // halo cells and whether they lie in the box
  int offo[UO], offr[UR];
  uint32_t ino = 0, inr = 0;
#pragma unroll
  for (int u = 0; u < UO; ++u) {
    const int q = stid + u * NT;
    const int gx = x0 - 2 + q % OX, gy = y0 - 2 + q / OX;
    const bool ok = q < NO && gx >= 0 && gx < nx && gy >= 0 && gy < ny;
    offo[u] = ok ? gx + nx * gy : 0;
    ino |= (uint32_t)ok << u;
  }
#pragma unroll
  for (int u = 0; u < UR; ++u) {
    const int q = stid + u * NT;
    const int gx = x0 - 1 + q % RX, gy = y0 - 1 + q / RX;
    const bool ok = q < NR && gx >= 0 && gx < nx && gy >= 0 && gy < ny;
    offr[u] = ok ? gx + nx * gy : 0;
    inr |= (uint32_t)ok << u;
  }
  // the (up to two) red cells of this thread: (gx0 + par, gy) with
  // par = (cpar + k) & 1, and their reciprocal in-plane diagonals
  int rgx0[2], rgy[2], roq0[2], rrq0[2], rcp[2];
  T r00[2], r01[2], r10[2], r11[2];                  // [parity][phase]
  bool ract[2];
#pragma unroll
  for (int u = 0; u < 2; ++u) {
    const int q = tid + u * NT;
    const int ry = q / (RX / 2), m = q % (RX / 2);
    ract[u] = q < NRED;
    rgy[u] = y0 - 1 + ry;
    rgx0[u] = x0 - 1 + 2 * m;
    roq0[u] = (2 * m + 1) + OX * (ry + 1);
    rrq0[u] = (2 * m) + RX * ry;
    rcp[u] = (x0 - 1 + rgy[u]) & 1;
    r00[u] = zm_inplane_rdg<T>(rgx0[u], rgy[u], nx, ny, TC[0]);
    r01[u] = zm_inplane_rdg<T>(rgx0[u], rgy[u], nx, ny, TC[1]);
    r10[u] = zm_inplane_rdg<T>(rgx0[u] + 1, rgy[u], nx, ny, TC[0]);
    r11[u] = zm_inplane_rdg<T>(rgx0[u] + 1, rgy[u], nx, ny, TC[1]);
  }
  // the black cell and its red partner: the pair (gxa, gxa + 1)
  const int bry = tid / (TX / 2), bm = tid % (TX / 2);
  const int bgy = y0 + bry, bgxa = x0 + 2 * bm;
  const int boq0 = (2 * bm + 2) + OX * (bry + 2), brq0 = (2 * bm + 1) + RX * (bry + 1);
  const int bcp = (bgxa + bgy) & 1;
  const T b00 = zm_inplane_rdg<T>(bgxa + 1, bgy, nx, ny, TC[0]);   // parity 0: black at gxa + 1
  const T b01 = zm_inplane_rdg<T>(bgxa + 1, bgy, nx, ny, TC[1]);
  const T b10 = zm_inplane_rdg<T>(bgxa, bgy, nx, ny, TC[0]);       // parity 1: black at gxa
  const T b11 = zm_inplane_rdg<T>(bgxa, bgy, nx, ny, TC[1]);

  // wide fetch tables: chunk offsets (chunk starts x0 - VW + VW ch, resp.
  // x0 - 4 + 4 ch for tags) and whether the chunk lies in the box
  int offow[WIDE ? UOW : 1], offbw[WIDE ? URW : 1], offtw[WIDE ? UTW : 1];
  uint32_t inow = 0, inbw = 0, intw = 0;
  if (WIDE) {
#pragma unroll
    for (int u = 0; u < UOW; ++u) {
      const int q = tid + u * NT;
      const int gx = x0 - VW + VW * (q % CPO), gy = y0 - 2 + q / CPO;
      const bool ok = q < NOW && gx >= 0 && gx < nx && gy >= 0 && gy < ny;
      offow[u] = ok ? gx + nx * gy : 0;
      inow |= (uint32_t)ok << u;
    }
#pragma unroll
    for (int u = 0; u < URW; ++u) {
      const int q = tid + u * NT;
      const int gx = x0 - VW + VW * (q % CPR), gy = y0 - 1 + q / CPR;
      const bool ok = q < NRW && gx >= 0 && gx < nx && gy >= 0 && gy < ny;
      offbw[u] = ok ? gx + nx * gy : 0;
      inbw |= (uint32_t)ok << u;
    }
#pragma unroll
    for (int u = 0; u < UTW; ++u) {
      const int q = tid + u * NT;
      const int gx = x0 - 4 + 4 * (q % CPT), gy = y0 - 1 + q / CPT;
      const bool ok = q < NTW && gx >= 0 && gx < nx && gy >= 0 && gy < ny;
      offtw[u] = ok ? gx + nx * gy : 0;
      intw |= (uint32_t)ok << u;
    }
  }

  // planes in flight: raw loaded values (lanes outside the box read a valid
  // address; the value is discarded when stored, so no load is waited for
  // before the step that stores it)
  T Aov[WIDE ? 1 : UO], Abv[WIDE ? 1 : UR], Bov[WIDE ? 1 : UO], Bbv[WIDE ? 1 : UR];
  uint8_t Atv[WIDE ? 1 : UR], Btv[WIDE ? 1 : UR];
  VT Aow[WIDE ? UOW : 1], Abw[WIDE ? URW : 1], Bow[WIDE ? UOW : 1], Bbw[WIDE ? URW : 1];
  uint32_t Atw[WIDE ? UTW : 1], Btw[WIDE ? UTW : 1];

#define ZM_LOAD_Q(P, z, Q)                                                   \
  {                                                                          \
    const int zz_ = (z);                                                     \
    const int64_t zoff_ = sxy * (zz_ >= 0 && zz_ < nz ? zz_ : 0);            \
    if constexpr (WIDE) {                                                    \
      if constexpr (!ZIN) {                                                  \
        _Pragma("unroll") for (int u = 0; u < UOW; ++u) P##ow[u] = *(Q const VT*)(xin + zoff_ + offow[u]); \
      }                                                                      \
      _Pragma("unroll") for (int u = 0; u < URW; ++u) P##bw[u] = *(Q const VT*)(b + zoff_ + offbw[u]); \
      _Pragma("unroll") for (int u = 0; u < UTW; ++u) P##tw[u] = *(Q const uint32_t*)(tag + zoff_ + offtw[u]); \
    } else {                                                                 \
      if constexpr (!ZIN) {                                                  \
        _Pragma("unroll") for (int u = 0; u < UO; ++u) P##ov[u] = ((Q const T*)xin)[zoff_ + offo[u]]; \
      }                                                                      \
      _Pragma("unroll") for (int u = 0; u < UR; ++u) {                       \
        P##bv[u] = ((Q const T*)b)[zoff_ + offr[u]];                         \
        P##tv[u] = ((Q const uint8_t*)tag)[zoff_ + offr[u]];                 \
      }                                                                      \
    }                                                                        \
  }
#define ZM_LOAD(P, z) ZM_LOAD_Q(P, z, )
#define ZM_STORE(P, z, VS, BSL)                                              \
  {                                                                          \
    const int zz_ = (z);                                                     \
    const bool zin_ = zz_ >= 0 && zz_ < nz;                                  \
    T* v_ = V[VS];                                                           \
    T* bs_ = Bs[BSL];                                                        \
    uint8_t* ts_ = Ts[BSL];                                                  \
    if constexpr (WIDE) {                                                    \
      _Pragma("unroll") for (int u = 0; u < UOW; ++u) {                      \
        const int q = tid + u * NT;                                          \
        if (q < NOW) {                                                       \
          const int row_ = q / CPO, c0_ = VW * (q % CPO) - (VW - 2);         \
          const bool ok_ = zin_ && ((inow >> u) & 1);                        \
          _Pragma("unroll") for (int e = 0; e < VW; ++e) {                   \
            const int col_ = c0_ + e;                                        \
            if (col_ >= 0 && col_ < OX) v_[col_ + OX * row_] = (ok_ && !ZIN) ? P##ow[u][e] : T(0); \
          }                                                                  \
        }                                                                    \
      }                                                                      \
      _Pragma("unroll") for (int u = 0; u < URW; ++u) {                      \
        const int q = tid + u * NT;                                          \
        if (q < NRW) {                                                       \
          const int row_ = q / CPR, c0_ = VW * (q % CPR) - (VW - 1);         \
          const bool ok_ = zin_ && ((inbw >> u) & 1);                        \
          _Pragma("unroll") for (int e = 0; e < VW; ++e) {                   \
            const int col_ = c0_ + e;                                        \
            if (col_ >= 0 && col_ < RX) bs_[col_ + RX * row_] = ok_ ? P##bw[u][e] : T(0); \
          }                                                                  \
        }                                                                    \
      }                                                                      \
      _Pragma("unroll") for (int u = 0; u < UTW; ++u) {                      \
        const int q = tid + u * NT;                                          \
        if (q < NTW) {                                                       \
          const int row_ = q / CPT, c0_ = 4 * (q % CPT) - 3;                 \
          const bool ok_ = zin_ && ((intw >> u) & 1);                        \
          _Pragma("unroll") for (int e = 0; e < 4; ++e) {                    \
            const int col_ = c0_ + e;                                        \
            if (col_ >= 0 && col_ < RX)                                      \
              ts_[col_ + RX * row_] = ok_ ? (uint8_t)(P##tw[u] >> (8 * e)) : (uint8_t)3; \
          }                                                                  \
        }                                                                    \
      }                                                                      \
    } else {                                                                 \
      _Pragma("unroll") for (int u = 0; u < UO; ++u) {                       \
        const int q = stid + u * NT;                                         \
        v_[q] = (!ZIN && zin_ && ((ino >> u) & 1)) ? P##ov[u] : T(0);        \
      }                                                                      \
      _Pragma("unroll") for (int u = 0; u < UR; ++u) {                       \
        const int q = stid + u * NT;                                         \
        const bool ok_ = zin_ && ((inr >> u) & 1);                           \
        bs_[q] = ok_ ? P##bv[u] : T(0);                                      \
        ts_[q] = ok_ ? P##tv[u] : (uint8_t)3;                                \
      }                                                                      \
    }                                                                        \
  }
#define ZM_STEP(P, kk)                                                       \
  {                                                                          \
    const int k = (kk);                                                      \
    ZM_STORE(P, k + 2, sVp2, sBp2);                                            \
    ZM_LOAD(P, min(k + 4, z1 + 1));                                          \
    if (k >= 0 && k < nz) { /* red update of plane k over the ring region */ \
      const bool zint = k > 0 && k < nz - 1;                                 \
      const T* vm = V[sVm1];                                                  \
      T* vc = V[sV0];                                                        \
      const T* vp = V[sVp1];                                                  \
      const T* bs = Bs[sB0];                                                 \
      const uint8_t* ts = Ts[sB0];                                           \
      _Pragma("unroll") for (int u = 0; u < 2; ++u) {                        \
        if (u == 0 || ract[u]) { /* every thread has a first red cell */     \
          const int par = (rcp[u] + k) & 1;                                  \
          const int gx = rgx0[u] + par, oq = roq0[u] + par, rq = rrq0[u] + par; \
          const int pc = tclass(ts[rq]);                                     \
          const int p = pc & 1;                                              \
          T v;                                                               \
          if (zint) {                                                        \
            const T r = par ? (p ? r11[u] : r10[u]) : (p ? r01[u] : r00[u]); \
            v = zm_update_inner<T>(vm, vc, vp, oq, OX, TC[p][0], bs[rq], r); \
          } else {                                                           \
            v = zm_update_general<T>(vm, vc, vp, oq, OX, gx, rgy[u], k, nx, ny, nz, TC[p], bs[rq]); \
          }                                                                  \
          if (pc <= 1) vc[oq] = v;                                           \
        }                                                                    \
      }                                                                      \
    }                                                                        \
    __syncthreads();                                                         \
    const int kb = k - 1;                                                    \
    if (kb >= z0 && kb < z1) { /* black update of plane k-1, and its write */ \
      const T* vm = V[sVm2];                                                  \
      const T* vc = V[sVm1];                                                  \
      const T* vp = V[sV0];                                                  \
      const T* bs = Bs[sBm1];                                                 \
      const uint8_t* ts = Ts[sBm1];                                           \
      const int par = (bcp + kb) & 1; /* 1: gxa is black */                  \
      const int sh = par ? 0 : 1;                                            \
      const int gx = bgxa + sh, oq = boq0 + sh, rq = brq0 + sh;              \
      const int pc = tclass(ts[rq]);                                         \
      const int p = pc & 1;                                                  \
      T vu;                                                                  \
      if (kb > 0 && kb < nz - 1) {                                           \
        const T r = par ? (p ? b11 : b10) : (p ? b01 : b00);                 \
        vu = zm_update_inner<T>(vm, vc, vp, oq, OX, TC[p][0], bs[rq], r);    \
      } else {                                                               \
        vu = zm_update_general<T>(vm, vc, vp, oq, OX, gx, bgy, kb, nx, ny, nz, TC[p], bs[rq]); \
      }                                                                      \
      const T vb = pc <= 1 ? vu : vc[oq];                                    \
      const T vr = vc[oq + (par ? 1 : -1)]; /* the red partner, updated */   \
      T* out = xout + (int64_t)nx * bgy + sxy * kb;                          \
      if (full) { /* the whole tile lies in the box: no per-lane test */     \
        out[bgxa] = par ? vb : vr;                                           \
        out[bgxa + 1] = par ? vr : vb;                                       \
      } else if (bgy < ny) {                                                 \
        if (bgxa < nx) out[bgxa] = par ? vb : vr;                            \
        if (bgxa + 1 < nx) out[bgxa + 1] = par ? vr : vb;                    \
      }                                                                      \
    }                                                                        \
    __syncthreads();                                                         \
    /* the ring slots of the planes around the next step */                  \
    {                                                                        \
      const int t5_ = sVm2;                                                  \
      sVm2 = sVm1;                                                           \
      sVm1 = sV0;                                                            \
      sV0 = sVp1;                                                            \
      sVp1 = sVp2;                                                           \
      sVp2 = t5_;                                                            \
      const int t4_ = sBm1;                                                  \
      sBm1 = sB0;                                                            \
      sB0 = sBp1;                                                            \
      sBp1 = sBp2;                                                           \
      sBp2 = t4_;                                                            \
    }                                                                        \
  }

  // LDS ring slots: plane p lives in V[(p + 10) % 5] and in Bs / Ts
  // [(p + 8) & 3]; the slots of the planes around the current step rotate
  // in scalars instead of being recomputed from p at every use
  const bool full = x0 + TX <= nx && y0 + TY <= ny;
  int sVm2 = (z0 - 3 + 10) % 5, sVm1 = (z0 - 2 + 10) % 5, sV0 = (z0 - 1 + 10) % 5, sVp1 = (z0 + 10) % 5,
      sVp2 = (z0 + 1 + 10) % 5;
  int sBm1 = (z0 - 2 + 8) & 3, sB0 = (z0 - 1 + 8) & 3, sBp1 = (z0 + 8) & 3, sBp2 = (z0 + 1 + 8) & 3;
  ZM_LOAD(A, z0 - 2);
  ZM_STORE(A, z0 - 2, (z0 - 2 + 10) % 5, (z0 - 2 + 8) & 3);
  ZM_LOAD(A, z0 - 1);
  ZM_STORE(A, z0 - 1, (z0 - 1 + 10) % 5, (z0 - 1 + 8) & 3);
  ZM_LOAD(A, z0);
  ZM_STORE(A, z0, (z0 + 10) % 5, (z0 + 8) & 3);
  // planes z0+1, z0+3, ... travel in A; z0+2, z0+4, ... in B. These two
  // planes are read through volatile pointers so that they are issued in
  // this order, every A load ahead of every B load, as in the loop: if the
  // compiler moved an A load after the B loads here, the wait counts at the
  // loop head would have to assume an A load was issued last and would drain
  // every load in flight at every other step.
  ZM_LOAD_Q(A, z0 + 1, volatile);
  ZM_LOAD_Q(B, z0 + 2, volatile);
  __syncthreads();
  // an odd step count ends with one extra step whose black plane lies
  // outside [z0, z1): it only stages and recomputes LDS values
  for (int k2 = z0 - 1; k2 <= z1; k2 += 2) {
    ZM_STEP(A, k2);
    ZM_STEP(B, k2 + 1);
  }
#undef ZM_STEP
#undef ZM_STORE
#undef ZM_LOAD
#undef ZM_LOAD_Q
  // second-phase unknowns are not touched by this sweep: copy them through
  const int64_t N = sxy * nz;
  for (int64_t q = (int64_t)blockIdx.x * NT + tid; q < nsec; q += nblocks * NT) xout[N + q] = ZIN ? T(0) : xin[N + q];
}


// Explicit (irregular) rows are processed by sub-wavefronts of kSub lanes:
// each lane takes every kSub-th entry of the row (coalesced column/value
// loads) and the partial sums are combined with xor-shuffles in a fixed
// pattern, so results are bitwise reproducible.
constexpr int kSub = 8;

template <typename T, typename TX = T>
__device__ __forceinline__ T row_dot(int64_t b, int64_t e, const int32_t* __restrict__ col,
                                     const T* __restrict__ val, const TX* __restrict__ x, int lane) {
#pragma clang fp contract(off)
  T s = 0;
  for (int64_t q = b + lane; q < e; q += kSub) s += val[q] * (T)x[col[q]];
  for (int off = kSub / 2; off > 0; off >>= 1) s += __shfl_xor(s, off, kSub);
  return s;
}

// Jacobi update of a group of explicit rows into tmp (the group's rows read
// only values the group does not write in this launch).
template <typename T>
__global__ void __launch_bounds__(kBlock) k_irr_jacobi(const int32_t* __restrict__ rows, int nrows,
                                                       const int64_t* __restrict__ dof,
                                                       const int64_t* __restrict__ rp,
                                                       const int32_t* __restrict__ col, const T* __restrict__ val,
                                                       const T* __restrict__ diag, const T* __restrict__ x,
                                                       const T* __restrict__ b, T* __restrict__ tmp) {
  const int64_t g = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kSub;
  const int lane = threadIdx.x % kSub;
  if (g >= nrows) return;
  const int r = rows[g];
  const T s = row_dot<T>(rp[r], rp[r + 1], col, val, x, lane);
  if (lane == 0) tmp[g] = (b[dof[r]] - s) / diag[r];
}

template <typename T>
__global__ void __launch_bounds__(kBlock) k_irr_scatter(const int32_t* __restrict__ rows, int nrows,
                                                        const int64_t* __restrict__ dof,
                                                        const T* __restrict__ tmp, T* __restrict__ x) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nrows) return;
  x[dof[rows[t]]] = tmp[t];
}

// One colour phase of an out-of-place red/black sweep in a single launch:
// template cells and explicit rows of colour `colour` are updated from xin,
// every other unknown is copied to xout. Blocks [0, nbu) update the rows
// rows_upd (kSub lanes per row), the next ones up to nbr copy the rows
// rows_cp (one thread per row), the last nbc take the template cells; the
// rows go first because each of them waits on a chain of dependent loads
// (row index, row extent, columns, values), which then overlaps with the
// cells instead of trailing them. Every update of the phase, template cell
// or explicit row, reads only the values before the phase: the explicit
// rows do not see this phase's template-cell updates (the grouped passes,
// which run after the phase's template cells, do), and rows of one colour
// see each other's previous values (Jacobi within a colour, as in the
// grouped passes). A sweep costs two launches, which is what matters on
// small levels.
// W cells per thread along x: W = 2 (nx even) takes an even-odd pair, of
// which exactly one cell has the phase's colour; W = 4 (nx a multiple of 4,
// fewer than 2^31 cells, arrays aligned to a quad) takes four cells, two of
// each colour, with every load and the store as one quad vector (tags as
// one 32-bit word) and 32-bit index arithmetic. Fewer threads wait on the
// same tag -> neighbours -> store chain; the arithmetic per cell is the
// same in every form.
template <typename T, int DIM>
__device__ __forceinline__ T oop_cell(const Tmpl<T>& tp, int p, T w, T e, T so, T no, T dn, T up, int i, int j,
                                      int k, T bc) {
  const int nx = tp.n[0], ny = tp.n[1];
  T s = 0;
  T dg = tp.D0(p);
  if (i > 0) s += w; else dg += tp.CB(0, p);
  if (i < nx - 1) s += e; else dg += tp.CB(1, p);
  if (j > 0) s += so; else dg += tp.CB(2, p);
  if (j < ny - 1) s += no; else dg += tp.CB(3, p);
  if (DIM == 3) {
    if (k > 0) s += dn; else dg += tp.CB(4, p);
    if (k < tp.n[2] - 1) s += up; else dg += tp.CB(5, p);
  }
  const T off = tp.CO(p) * s;
  return (bc - off) * (T(1) / dg);
}

template <typename T, int DIM, int W>
__global__ void __launch_bounds__(kBlock) k_rb_oop(const uint8_t* __restrict__ tag, const T* __restrict__ xin,
                                                   T* __restrict__ xout, const T* __restrict__ b, Tmpl<T> tp,
                                                   int colour, unsigned nbc, unsigned nbu, unsigned nbr,
                                                   const int32_t* __restrict__ rows_upd,
                                                   int nupd, const int32_t* __restrict__ rows_cp, int ncp,
                                                   const int64_t* __restrict__ dof, const int64_t* __restrict__ rp,
                                                   const int32_t* __restrict__ col, const T* __restrict__ val,
                                                   const T* __restrict__ diag) {
  if (blockIdx.x >= nbr) {
    const unsigned cb = blockIdx.x - nbr;
    const int nx = tp.n[0], ny = tp.n[1];
    if (W == 4) {
      typedef T Q __attribute__((ext_vector_type(4)));
      const uint32_t nq = (uint32_t)nx >> 2;
      const uint32_t q = cb * kBlock + threadIdx.x;
      const uint32_t row = q / nq;   // j + ny * k
      if (row >= (uint32_t)ny * (uint32_t)(DIM == 3 ? tp.n[2] : 1)) return;
      const int i = (int)(q - row * nq) * 4;
      const int j = (int)(row % (uint32_t)ny);
      const int k = DIM == 3 ? (int)(row / (uint32_t)ny) : 0;
      const uint32_t c = row * (uint32_t)nx + (uint32_t)i;
      // out-of-box neighbours read the quad itself (in bounds); the
      // update skips them
      const uint32_t cs = j > 0 ? c - nx : c, cn = j < ny - 1 ? c + nx : c;
      const int u = ((j + k) & 1) == colour ? 0 : 1;   // cells u and u + 2 have the phase's colour
      // the one x neighbour outside the quad: left of cell 0 (u = 0) or right of cell 3 (u = 1)
      const uint32_t co = u ? (i + 4 < nx ? c + 4 : c) : (i > 0 ? c - 1 : c);
      const uint32_t tw = *(const uint32_t*)(tag + c);
      const Q xc = *(const Q*)(xin + c);
      const T xo = xin[co];
      const Q xs = *(const Q*)(xin + cs);
      const Q xn = *(const Q*)(xin + cn);
      Q xd = xc, xu = xc;
      if (DIM == 3) {
        const uint32_t sxy = (uint32_t)nx * (uint32_t)ny;
        xd = *(const Q*)(xin + (k > 0 ? c - sxy : c));
        xu = *(const Q*)(xin + (k < tp.n[2] - 1 ? c + sxy : c));
      }
      const Q bq = *(const Q*)(b + c);
      const int pa = (int)((tw >> (8 * u)) & 3u), pb = (int)((tw >> (8 * (u + 2))) & 3u);
      T va = u ? xc.y : xc.x, vb = u ? xc.w : xc.z;
      if (pa <= 1)
        va = oop_cell<T, DIM>(tp, pa, u ? xc.x : xo, u ? xc.z : xc.y, u ? xs.y : xs.x, u ? xn.y : xn.x,
                              u ? xd.y : xd.x, u ? xu.y : xu.x, i + u, j, k, u ? bq.y : bq.x);
      if (pb <= 1)
        vb = oop_cell<T, DIM>(tp, pb, u ? xc.z : xc.y, u ? xo : xc.w, u ? xs.w : xs.z, u ? xn.w : xn.z,
                              u ? xd.w : xd.z, u ? xu.w : xu.z, i + u + 2, j, k, u ? bq.w : bq.z);
      Q o;
      o.x = u ? xc.x : va;
      o.y = u ? va : xc.y;
      o.z = u ? xc.z : vb;
      o.w = u ? vb : xc.w;
      // explicit-row cells (class 2) are written by the row blocks
      const bool e0 = (tw & 3u) == 2u, e1 = ((tw >> 8) & 3u) == 2u, e2 = ((tw >> 16) & 3u) == 2u,
                 e3 = ((tw >> 24) & 3u) == 2u;
      if (!(e0 | e1 | e2 | e3)) {
        *(Q*)(xout + c) = o;
      } else {
        if (!e0) xout[c] = o.x;
        if (!e1) xout[c + 1] = o.y;
        if (!e2) xout[c + 2] = o.z;
        if (!e3) xout[c + 3] = o.w;
      }
      return;
    }
    const int64_t N = (int64_t)nx * ny * (DIM == 3 ? tp.n[2] : 1);
    if (W == 2) {
      const int64_t c = 2 * ((int64_t)cb * kBlock + threadIdx.x);
      if (c >= N) return;
      const int i = (int)(c % nx);
      const int64_t jk = c / nx;
      const int j = (int)(jk % ny);
      const int k = DIM == 3 ? (int)(jk / ny) : 0;
      const int u = ((i + j + k) & 1) == colour ? 0 : 1;   // the pair's cell of this colour
      const uint8_t p0 = tclass(tag[c]), p1 = tclass(tag[c + 1]);
      const T x0 = xin[c], x1 = xin[c + 1];
      const uint8_t pu = u ? p1 : p0;
      T vu = u ? x1 : x0;
      if (pu <= 1) {
        T dg;
        const T off = template_apply<T, DIM>(xin, tp, i + u, j, k, c + u, pu, dg);
        vu = (b[c + u] - off) * (T(1) / dg);
      }
      if (p0 != 2) xout[c] = u ? x0 : vu;
      if (p1 != 2) xout[c + 1] = u ? vu : x1;
      return;
    }
    const int64_t c = (int64_t)cb * kBlock + threadIdx.x;
    if (c >= N) return;
    const uint8_t p = tclass(tag[c]);
    if (p == 2) return;
    const int i = (int)(c % nx);
    const int64_t jk = c / nx;
    const int j = (int)(jk % ny);
    const int k = DIM == 3 ? (int)(jk / ny) : 0;
    T v = xin[c];
    if (p <= 1 && ((i + j + k) & 1) == colour) {
      T dg;
      const T off = template_apply<T, DIM>(xin, tp, i, j, k, c, p, dg);
      v = (b[c] - off) * (T(1) / dg);
    }
    xout[c] = v;
    return;
  }
  if (blockIdx.x < nbu) {
    const int64_t g = ((int64_t)blockIdx.x * kBlock + threadIdx.x) / kSub;
    const int lane = threadIdx.x % kSub;
    if (g >= nupd) return;
    const int r = rows_upd[g];
    const T s = row_dot<T>(rp[r], rp[r + 1], col, val, xin, lane);
    const int64_t q = dof[r];
    if (lane == 0) xout[q] = (b[q] - s) / diag[r];
    return;
  }
  const int64_t g = (int64_t)(blockIdx.x - nbu) * kBlock + threadIdx.x;
  if (g >= ncp) return;
  const int64_t q = dof[rows_cp[g]];
  xout[q] = xin[q];
}

// MODE 0: r = b - A x ; MODE 1: r = A x. Regular cells and covered cells
// (3D launch grid over cells).
template <typename T, int DIM, int MODE>
__global__ void __launch_bounds__(kBlock) k_resid_reg(const uint8_t* __restrict__ tag, const T* __restrict__ x,
                                                      const T* __restrict__ b, T* __restrict__ r, Tmpl<T> tp) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int j = blockIdx.y * blockDim.y + threadIdx.y;
  const int k = DIM == 3 ? (int)blockIdx.z : 0;
  if (i >= tp.n[0] || j >= tp.n[1]) return;
  const int64_t c = i + (int64_t)tp.n[0] * (j + (int64_t)tp.n[1] * k);
  const uint8_t p = tclass(tag[c]);
  if (p == 3) {
    r[c] = MODE == 0 ? T(0) : x[c];
    return;
  }
  if (p == 2) return;
  const int nx = tp.n[0], ny = tp.n[1];
  const int64_t sxy = (int64_t)nx * ny;
  const T xv = x[c];
  T s = 0, dg = tp.M(p);
  if (i > 0) s += x[c - 1] - xv; else dg += tp.CBM(0, p);
  if (i < nx - 1) s += x[c + 1] - xv; else dg += tp.CBM(1, p);
  if (j > 0) s += x[c - nx] - xv; else dg += tp.CBM(2, p);
  if (j < ny - 1) s += x[c + nx] - xv; else dg += tp.CBM(3, p);
  if (DIM == 3) {
    if (k > 0) s += x[c - sxy] - xv; else dg += tp.CBM(4, p);
    if (k < tp.n[2] - 1) s += x[c + sxy] - xv; else dg += tp.CBM(5, p);
  }
  const T ax = dg * xv + tp.CO(p) * s;
  r[c] = MODE == 0 ? b[c] - ax : ax;
}

// Per-block partial sums of up to two dot products (fixed order: wave64
// shuffles, then the block's waves in order), stored at part[d * pt + bid].
// Every thread of the block must call it.
template <int NB>
__device__ __forceinline__ void block_partials(double s0, double s1, int ndot, double* __restrict__ part, int64_t pt,
                                               int64_t bid, int tid) {
  __shared__ double sh[2][NB / 64];
  for (int off = 32; off > 0; off >>= 1) {
    s0 += __shfl_down(s0, off, 64);
    s1 += __shfl_down(s1, off, 64);
  }
  if ((tid & 63) == 0) {
    sh[0][tid >> 6] = s0;
    sh[1][tid >> 6] = s1;
  }
  __syncthreads();
  if (tid == 0) {
    double t0 = 0, t1 = 0;
    for (int w = 0; w < NB / 64; ++w) {
      t0 += sh[0][w];
      t1 += sh[1][w];
    }
    part[bid] = t0;
    if (ndot > 1) part[pt + bid] = t1;
  }
}

// Template rows of a 3D level marching along z (r = b - A x, MODE 1: r = A x):
// each thread owns one (i, j) column of a block's 64 x 4 tile and walks KZ
// planes, keeping x of planes k-1, k, k+1 in registers (each x value leaves
// HBM once; the in-plane neighbours are cache hits) and requesting plane k+2,
// b and the tag one step ahead. Same arithmetic and order as the grid-wide
// kernel; explicit rows are left to k_resid_irr.
constexpr int kRZX = 64, kRZY = 4, kRZ = 16;

// TX: type of x (a FP32 preconditioner output is widened on load, exactly).
// NDOT > 0 (MODE 1): per-block partials of (da, r) and, if 2, (r, r) over the
// entries this block writes, at part[d * pt + block] (see block_partials).
template <typename T, int MODE, typename TX = T, int NDOT = 0>
__global__ void __launch_bounds__(kRZX * kRZY) k_resid_zm3(const uint8_t* __restrict__ tag,
                                                           const TX* __restrict__ x, const T* __restrict__ b,
                                                           T* __restrict__ r, Tmpl<T> tp,
                                                           const T* __restrict__ da = nullptr,
                                                           double* __restrict__ part = nullptr, int64_t pt = 0) {
  __shared__ T TC[2][8];
  const int tid = threadIdx.x + kRZX * threadIdx.y;
  if (tid < 16) {
    const int p = tid >> 3, j = tid & 7;
    TC[p][j] = j == 0 ? tp.coff[p] : (j == 1 ? tp.mass[p] : tp.cbm[j - 2][p]);
  }
  __syncthreads();
  const int nx = tp.n[0], ny = tp.n[1], nz = tp.n[2];
  // 1D grid of tiles, numbered so that each XCD takes a contiguous range
  // (neighbouring tiles then share that XCD's L2 for their halo rows)
  const int gbx = (nx + kRZX - 1) / kRZX, gby = (ny + kRZY - 1) / kRZY;
  const int64_t tt = xcd_block(blockIdx.x, gridDim.x);
  const int i = (int)(tt % gbx) * kRZX + threadIdx.x;
  const int j = (int)((tt / gbx) % gby) * kRZY + threadIdx.y;
  const int z0 = (int)(tt / ((int64_t)gbx * gby)) * kRZ, z1 = min(z0 + kRZ, nz);
  double d0 = 0, d1 = 0;
  if (i < nx && j < ny) {
    const int64_t sxy = (int64_t)nx * ny;
    const int64_t c0 = i + (int64_t)nx * j;
    // in-plane neighbour offsets (0 where the neighbour is outside the box:
    // the loaded value is then not used)
    const int64_t ow = i > 0 ? -1 : 0, oe = i < nx - 1 ? 1 : 0;
    const int64_t os = j > 0 ? -(int64_t)nx : 0, on = j < ny - 1 ? (int64_t)nx : 0;
    // everything a plane needs is requested one plane ahead, so the waits
    // of a step only cover loads issued in the previous step
    T xm = z0 > 0 ? (T)x[c0 + sxy * (z0 - 1)] : T(0);
    int64_t c = c0 + sxy * z0;
    T xc = (T)x[c];
    T xp = z0 + 1 < nz ? (T)x[c + sxy] : T(0);
    T w = (T)x[c + ow], e = (T)x[c + oe], so = (T)x[c + os], no = (T)x[c + on];
    constexpr bool H = sizeof(T) == 8;
    uint8_t tg = ld_stream<H>(tag + c);
    T bb = MODE == 0 ? ld_stream<H>(b + c) : T(0);
    T dc = NDOT > 0 ? ld_stream<H>(da + c) : T(0);
    for (int k = z0; k < z1; ++k, c += sxy) {
      // requests for plane k + 1 (its neighbours, b and tag) and x of k + 2
      const bool more = k + 1 < z1;
      const int64_t cn = more ? c + sxy : c;
      const T xpp = k + 2 < nz ? (T)x[c + 2 * sxy] : T(0);
      const T wn = (T)x[cn + ow], en = (T)x[cn + oe], son = (T)x[cn + os], non = (T)x[cn + on];
      const uint8_t tgn = more ? ld_stream<H>(tag + cn) : (uint8_t)3;
      const T bbn = (MODE == 0 && more) ? ld_stream<H>(b + cn) : T(0);
      const T dcn = (NDOT > 0 && more) ? ld_stream<H>(da + cn) : T(0);
      const int p = tclass(tg);
      if (p != 2) {
        T out;
        if (p == 3) {
          out = MODE == 0 ? T(0) : xc;
        } else {
          const T* tc = TC[p];
          T s = 0, dg = tc[1];
          if (i > 0) s += w - xc; else dg += tc[2];
          if (i < nx - 1) s += e - xc; else dg += tc[3];
          if (j > 0) s += so - xc; else dg += tc[4];
          if (j < ny - 1) s += no - xc; else dg += tc[5];
          if (k > 0) s += xm - xc; else dg += tc[6];
          if (k < nz - 1) s += xp - xc; else dg += tc[7];
          const T ax = dg * xc + tc[0] * s;
          out = MODE == 0 ? bb - ax : ax;
        }
        st_stream<H>(out, r + c);
        if (NDOT > 0) {
          d0 += (double)dc * (double)out;
          if (NDOT > 1) d1 += (double)out * (double)out;
        }
      }
      xm = xc;
      xc = xp;
      xp = xpp;
      dc = dcn;
      w = wn;
      e = en;
      so = son;
      no = non;
      tg = tgn;
      bb = bbn;
    }
  }
  if (NDOT > 0)
    block_partials<kRZX * kRZY>(d0, d1, NDOT, part, pt, blockIdx.x, tid);
}

// Residual r = b - A x of a 3D level restricted straight into the coarse
// right-hand side, for the simple coarse cells (the mean of the 8 children,
// summed in the order of k_restrict_all, with the residual of each template
// child computed as in k_resid_zm3): r itself is written only where a later
// step reads it, for the children of non-simple coarse unknowns (restricted
// from their child lists afterwards); the explicit-row children's r must be
// in place before (it is read here); covered coarse cells get 0. A wavefront
// holds a 32 x 2 patch of a plane (lanes 0-31 and 32-63 are neighbouring
// rows), so a 2 x 2 group of children is summed by lane shuffles and two
// consecutive planes by one thread; each thread walks zc planes (even, at
// most kRRZ; fewer on small levels so that the grid still fills the chip)
// with one plane requested ahead. Needs even extents (the coarse level is
// half the fine one in every direction).
constexpr int kRRX = 32, kRRW = 4, kRRZ = 16;   // tile: 32 x (2 kRRW) columns over zc planes

template <typename T>
__global__ void __launch_bounds__(64 * kRRW) k_resid_restrict3(const uint8_t* __restrict__ tag,
                                                               const T* __restrict__ x, const T* __restrict__ b,
                                                               T* __restrict__ r, const uint8_t* __restrict__ ctag,
                                                               T* __restrict__ bc, Tmpl<T> tp, int zc) {
  __shared__ T TC[2][8];
  const int tid = threadIdx.x + 64 * threadIdx.y;
  if (tid < 16) {
    const int p = tid >> 3, j = tid & 7;
    TC[p][j] = j == 0 ? tp.coff[p] : (j == 1 ? tp.mass[p] : tp.cbm[j - 2][p]);
  }
  __syncthreads();
  const int nx = tp.n[0], ny = tp.n[1], nz = tp.n[2];
  const int cnx = nx >> 1, cny = ny >> 1;
  const int gbx = (nx + kRRX - 1) / kRRX, gby = (ny + 2 * kRRW - 1) / (2 * kRRW);
  const int64_t tt = xcd_block(blockIdx.x, gridDim.x);
  const int lane = threadIdx.x;
  const int i = (int)(tt % gbx) * kRRX + (lane & 31);
  const int j = (int)((tt / gbx) % gby) * (2 * kRRW) + 2 * threadIdx.y + (lane >> 5);
  const int z0 = (int)(tt / ((int64_t)gbx * gby)) * zc, z1 = min(z0 + zc, nz);
  // lanes past the box edge load a valid cell, take part in the shuffles and
  // write nothing (extents are even, so a 2 x 2 group is all in or all out)
  const bool act = i < nx && j < ny;
  const int ic = act ? i : 0, jc = act ? j : 0;
  const bool lead = act && (lane & 1) == 0 && lane < 32;
  const int64_t sxy = (int64_t)nx * ny;
  const int64_t c0 = ic + (int64_t)nx * jc;
  const int64_t ow = ic > 0 ? -1 : 0, oe = ic < nx - 1 ? 1 : 0;
  const int64_t os = jc > 0 ? -(int64_t)nx : 0, on = jc < ny - 1 ? (int64_t)nx : 0;
  const int64_t P0 = (ic >> 1) + (int64_t)cnx * (jc >> 1);
  const int64_t csxy = (int64_t)cnx * cny;
  T xm = z0 > 0 ? x[c0 + sxy * (z0 - 1)] : T(0);
  int64_t c = c0 + sxy * z0;
  T xc = x[c];
  T xp = z0 + 1 < nz ? x[c + sxy] : T(0);
  T w = x[c + ow], e = x[c + oe], so = x[c + os], no = x[c + on];
  uint8_t tg = tag[c];
  T bb = b[c];
  uint8_t ct = ctag[P0 + csxy * (z0 >> 1)];
  T acc = 0;
  for (int k = z0; k < z1; ++k, c += sxy) {
    const bool more = k + 1 < z1;
    const int64_t cn = more ? c + sxy : c;
    const T xpp = k + 2 < nz ? x[c + 2 * sxy] : T(0);
    const T wn = x[cn + ow], en = x[cn + oe], son = x[cn + os], non = x[cn + on];
    const uint8_t tgn = more ? tag[cn] : (uint8_t)3;
    const T bbn = more ? b[cn] : T(0);
    const uint8_t ctn = more ? ctag[P0 + csxy * ((k + 1) >> 1)] : (uint8_t)3;
    const int p = tclass(tg);
    T out;
    if (p == 2) {
      out = r[c];   // an explicit row: its residual is already there
    } else if (p == 3) {
      out = T(0);
    } else {
      const T* tc = TC[p];
      T s = 0, dg = tc[1];
      if (ic > 0) s += w - xc; else dg += tc[2];
      if (ic < nx - 1) s += e - xc; else dg += tc[3];
      if (jc > 0) s += so - xc; else dg += tc[4];
      if (jc < ny - 1) s += no - xc; else dg += tc[5];
      if (k > 0) s += xm - xc; else dg += tc[6];
      if (k < nz - 1) s += xp - xc; else dg += tc[7];
      const T ax = dg * xc + tc[0] * s;
      out = bb - ax;
    }
    // the children of a non-simple coarse unknown keep their residual for
    // the list restriction that follows
    if (act && p != 2 && (ct & 4) && tclass(ct) != 3) r[c] = out;
    const T v10 = __shfl_xor(out, 1, 64), v01 = __shfl_xor(out, 32, 64), v11 = __shfl_xor(out, 33, 64);
    if (lead) {
      const T pk = ((out + v10) + v01) + v11;
      if ((k & 1) == 0) {
        acc = pk;
      } else {
        const int64_t P = P0 + csxy * (k >> 1);
        if (tclass(ct) == 3)
          bc[P] = T(0);
        else if (!(ct & 4))
          bc[P] = (acc + pk) * T(0.125);
      }
    }
    xm = xc;
    xc = xp;
    xp = xpp;
    w = wn;
    e = en;
    so = son;
    no = non;
    tg = tgn;
    bb = bbn;
    ct = (k & 1) ? ctn : ct;
  }
}

// The same residual / matrix-vector product with two neighbouring cells per
// lane (x even): x, b, r and the dot vector move as 2-element vectors and the
// tags as one 16-bit word, so a wavefront issues half the memory instructions
// at twice the width, and the once-read or once-written 8-byte streams carry
// non-temporal hints. Tiles of kRPX x kRPY columns over kRPZ planes, one
// plane requested ahead. Same arithmetic per cell as k_resid_zm3. Needs an
// even x extent and 2-element-aligned arrays.
constexpr int kRPX = 128, kRPY = 4, kRPZ = 32;

template <typename T, int MODE, typename TX = T, int NDOT = 0>
__global__ void __launch_bounds__(64 * kRPY) k_resid_zp3(const uint8_t* __restrict__ tag,
                                                        const TX* __restrict__ x, const T* __restrict__ b,
                                                        T* __restrict__ r, Tmpl<T> tp,
                                                        const T* __restrict__ da = nullptr,
                                                        double* __restrict__ part = nullptr, int64_t pt = 0) {
  typedef TX X2 __attribute__((ext_vector_type(2)));
  typedef T V2 __attribute__((ext_vector_type(2)));
  constexpr bool H = sizeof(T) == 8;
  __shared__ T TC[2][8];
  const int tid = threadIdx.x + 64 * threadIdx.y;
  if (tid < 16) {
    const int p = tid >> 3, j = tid & 7;
    TC[p][j] = j == 0 ? tp.coff[p] : (j == 1 ? tp.mass[p] : tp.cbm[j - 2][p]);
  }
  __syncthreads();
  const int nx = tp.n[0], ny = tp.n[1], nz = tp.n[2];
  const int gbx = (nx + kRPX - 1) / kRPX, gby = (ny + kRPY - 1) / kRPY;
  const int64_t tt = xcd_block(blockIdx.x, gridDim.x);
  const int i = (int)(tt % gbx) * kRPX + 2 * (int)threadIdx.x;
  const int j = (int)((tt / gbx) % gby) * kRPY + threadIdx.y;
  const int z0 = (int)(tt / ((int64_t)gbx * gby)) * kRPZ, z1 = min(z0 + kRPZ, nz);
  double d0 = 0, d1 = 0;
  if (i < nx && j < ny) {
    const int64_t sxy = (int64_t)nx * ny;
    const int64_t c0 = i + (int64_t)nx * j;
    const int64_t ow = i > 0 ? -1 : 0, oe = i + 2 < nx ? 2 : 1;
    const int64_t os = j > 0 ? -(int64_t)nx : 0, on = j < ny - 1 ? (int64_t)nx : 0;
    const X2 zx = {TX(0), TX(0)};
    const V2 zv = {T(0), T(0)};
    int64_t c = c0 + sxy * z0;
    X2 xm = z0 > 0 ? *(const X2*)(x + c - sxy) : zx;
    X2 xc = *(const X2*)(x + c);
    X2 xp = z0 + 1 < nz ? *(const X2*)(x + c + sxy) : zx;
    TX w = x[c + ow], e = x[c + oe];
    X2 so = *(const X2*)(x + c + os), no = *(const X2*)(x + c + on);
    uint16_t tg = ld_stream<H>((const uint16_t*)(tag + c));
    V2 bb = MODE == 0 ? ld_stream<H>((const V2*)(b + c)) : zv;
    V2 dc = NDOT > 0 ? ld_stream<H>((const V2*)(da + c)) : zv;
    for (int k = z0; k < z1; ++k, c += sxy) {
      // requests for plane k + 1 (its neighbours, b, tags, dot vector) and x of k + 2
      const bool more = k + 1 < z1;
      const int64_t cn = more ? c + sxy : c;
      const X2 xpp = k + 2 < nz ? *(const X2*)(x + c + 2 * sxy) : zx;
      const TX wn = x[cn + ow], en = x[cn + oe];
      const X2 son = *(const X2*)(x + cn + os), non = *(const X2*)(x + cn + on);
      const uint16_t tgn = more ? ld_stream<H>((const uint16_t*)(tag + cn)) : (uint16_t)0x0202;
      const V2 bbn = (MODE == 0 && more) ? ld_stream<H>((const V2*)(b + cn)) : zv;
      const V2 dcn = (NDOT > 0 && more) ? ld_stream<H>((const V2*)(da + cn)) : zv;
      T out[2];
      bool wr[2];
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        const int p = tclass((uint8_t)(tg >> (8 * u)));
        const T xv = (T)(u ? xc.y : xc.x);
        wr[u] = p != 2;
        if (p == 3) {
          out[u] = MODE == 0 ? T(0) : xv;
        } else {
          const T wv = (T)(u ? xc.x : w), ev = (T)(u ? e : xc.y);
          const T* tc = TC[p & 1];
          T s = 0, dg = tc[1];
          if (i + u > 0) s += wv - xv; else dg += tc[2];
          if (i + u < nx - 1) s += ev - xv; else dg += tc[3];
          if (j > 0) s += (T)(u ? so.y : so.x) - xv; else dg += tc[4];
          if (j < ny - 1) s += (T)(u ? no.y : no.x) - xv; else dg += tc[5];
          if (k > 0) s += (T)(u ? xm.y : xm.x) - xv; else dg += tc[6];
          if (k < nz - 1) s += (T)(u ? xp.y : xp.x) - xv; else dg += tc[7];
          const T ax = dg * xv + tc[0] * s;
          out[u] = MODE == 0 ? (u ? bb.y : bb.x) - ax : ax;
        }
        if (NDOT > 0 && wr[u]) {
          d0 += (double)(u ? dc.y : dc.x) * (double)out[u];
          if (NDOT > 1) d1 += (double)out[u] * (double)out[u];
        }
      }
      if (wr[0] && wr[1]) {
        const V2 o = {out[0], out[1]};
        st_stream<H>(o, (V2*)(r + c));
      } else {
        if (wr[0]) st_stream<H>(out[0], r + c);
        if (wr[1]) st_stream<H>(out[1], r + c + 1);
      }
      xm = xc;
      xc = xp;
      xp = xpp;
      w = wn;
      e = en;
      so = son;
      no = non;
      tg = tgn;
      bb = bbn;
      dc = dcn;
    }
  }
  if (NDOT > 0)
    block_partials<64 * kRPY>(d0, d1, NDOT, part, pt, blockIdx.x, tid);
}

template <typename T, int MODE, typename TX = T, int NDOT = 0>
__global__ void __launch_bounds__(kBlock) k_resid_irr(int nrows, const int64_t* __restrict__ dof,
                                                      const int64_t* __restrict__ rp, const int32_t* __restrict__ col,
                                                      const T* __restrict__ val, const T* __restrict__ diag,
                                                      const TX* __restrict__ x, const T* __restrict__ b,
                                                      T* __restrict__ r, const T* __restrict__ da = nullptr,
                                                      double* __restrict__ part = nullptr, int64_t pt = 0,
                                                      int64_t boff = 0) {
  const int64_t g = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kSub;
  const int lane = threadIdx.x % kSub;
  double d0 = 0, d1 = 0;
  if (g < nrows) {
    T s = 0;
    for (int64_t q = rp[g] + lane; q < rp[g + 1]; q += kSub) s += val[q] * (T)x[col[q]];
    for (int off = kSub / 2; off > 0; off >>= 1) s += __shfl_xor(s, off, kSub);
    if (lane == 0) {
      const int64_t q = dof[g];
      const T ax = diag[g] * (T)x[q] + s;
      const T out = MODE == 0 ? b[q] - ax : ax;
      r[q] = out;
      if (NDOT > 0) {
        d0 = (double)da[q] * (double)out;
        if (NDOT > 1) d1 = (double)out * (double)out;
      }
    }
  }
  if (NDOT > 0) block_partials<kBlock>(d0, d1, NDOT, part, pt, boff + blockIdx.x, threadIdx.x);
}

// Restriction in one launch: blocks [0, nbc) take simple coarse cells (mean
// of the 2^D children; covered coarse cells get 0), blocks [nbc, nbc + nbn)
// the non-simple coarse unknowns from their child lists, and the rest clear
// the coarse correction xc (cells and second-phase unknowns).
template <typename T, int DIM>
__global__ void __launch_bounds__(kBlock) k_restrict_all(const uint8_t* __restrict__ ctag, const T* __restrict__ rf,
                                                         T* __restrict__ bc, T* __restrict__ xc, int cnx, int cny,
                                                         int cnz, unsigned nbc, unsigned nbn, int nns,
                                                         const int64_t* __restrict__ cdof,
                                                         const int32_t* __restrict__ ptr,
                                                         const int64_t* __restrict__ child, int64_t ncd) {
  const unsigned bid = blockIdx.x;
  const T w = DIM == 3 ? T(0.125) : T(0.25);
  if (bid < nbc) {
    const int64_t P = (int64_t)bid * kBlock + threadIdx.x;
    const int64_t cN = (int64_t)cnx * cny * (DIM == 3 ? cnz : 1);
    if (P >= cN) return;
    const uint8_t t = ctag[P];
    if (tclass(t) == 3) {
      bc[P] = 0;
      return;
    }
    if (t & 4) return;
    const int I = (int)(P % cnx);
    const int64_t JK = P / cnx;
    const int J = (int)(JK % cny);
    const int K = DIM == 3 ? (int)(JK / cny) : 0;
    const int fnx = 2 * cnx;
    const int64_t fsxy = (int64_t)fnx * 2 * cny;
    const int64_t c0 = 2 * I + (int64_t)fnx * (2 * J) + (DIM == 3 ? fsxy * (2 * K) : 0);
    T s = rf[c0] + rf[c0 + 1] + rf[c0 + fnx] + rf[c0 + fnx + 1];
    if (DIM == 3) s += rf[c0 + fsxy] + rf[c0 + fsxy + 1] + rf[c0 + fsxy + fnx] + rf[c0 + fsxy + fnx + 1];
    bc[P] = s * w;
    return;
  }
  if (bid < nbc + nbn) {
    const int t = (int)((bid - nbc) * kBlock + threadIdx.x);
    if (t >= nns) return;
    T s = 0;
    for (int e = ptr[t]; e < ptr[t + 1]; ++e) s += rf[child[e]];
    bc[cdof[t]] = s * w;
    return;
  }
  const int64_t q = (int64_t)(bid - nbc - nbn) * kBlock + threadIdx.x;
  if (q < ncd) xc[q] = T(0);
}

// Prolongation in one launch. Blocks are (bx, by) threads: blocks x < nrb
// take by fine rows (j, k) each and bx cells of a row per block y, the fine
// cells of simple parents; blocks x >= nrb (y = 0) the fine unknowns of
// non-simple parents (disjoint sets). A cell's four loads (its tag and x, the
// parent's tag and correction) are issued before its test; no divisions of
// 64-bit indices.
template <typename T, int DIM>
__global__ void __launch_bounds__(kBlock) k_prolong_all(const uint8_t* __restrict__ ftag,
                                                        const uint8_t* __restrict__ ctag, const T* __restrict__ ec,
                                                        T* __restrict__ xf, int fnx, int fny, int fnz, unsigned nrb,
                                                        int nnp, const int64_t* __restrict__ fdof,
                                                        const int64_t* __restrict__ cdof) {
  const unsigned bid = blockIdx.x;
  if (bid < nrb) {
    const int row = (int)(bid * blockDim.y + threadIdx.y);        // j + fny * k
    const int i = (int)(blockIdx.y * blockDim.x + threadIdx.x);
    if (row >= fny * (DIM == 3 ? fnz : 1) || i >= fnx) return;
    const int j = row % fny, k = DIM == 3 ? row / fny : 0;
    const int cnx = fnx >> 1, cny = fny >> 1;
    const int64_t c = i + (int64_t)fnx * row;
    const int64_t P = (i >> 1) + (int64_t)cnx * ((j >> 1) + (int64_t)cny * (k >> 1));
    const uint8_t ft = ftag[c], ct = ctag[P];
    const T e = ec[P], xv = xf[c];
    if (tclass(ft) == 3 || (ct & 4)) return;
    xf[c] = xv + e;
    return;
  }
  if (blockIdx.y != 0) return;
  const int t = (int)((bid - nrb) * kBlock + threadIdx.y * blockDim.x + threadIdx.x);
  if (t >= nnp) return;
  xf[fdof[t]] += ec[cdof[t]];
}

// The same prolongation with four consecutive fine cells of a row per lane
// (x a multiple of 4, x-arrays 4-element aligned): the fine x and tags move
// as one 4-element vector and one 32-bit word, the two parents' values and
// tags as a 2-element vector and a 16-bit word. A fine cell is written only
// where the cell part updates it (the list part owns the others).
template <typename T, int DIM>
__global__ void __launch_bounds__(kBlock) k_prolong_q(const uint8_t* __restrict__ ftag,
                                                      const uint8_t* __restrict__ ctag, const T* __restrict__ ec,
                                                      T* __restrict__ xf, int fnx, int fny, int fnz, unsigned nrb,
                                                      int nnp, const int64_t* __restrict__ fdof,
                                                      const int64_t* __restrict__ cdof) {
  typedef T V4 __attribute__((ext_vector_type(4)));
  typedef T V2 __attribute__((ext_vector_type(2)));
  const unsigned bid = blockIdx.x;
  if (bid < nrb) {
    const int row = (int)(bid * blockDim.y + threadIdx.y);        // j + fny * k
    const int i = 4 * (int)(blockIdx.y * blockDim.x + threadIdx.x);
    if (row >= fny * (DIM == 3 ? fnz : 1) || i >= fnx) return;
    const int j = row % fny, k = DIM == 3 ? row / fny : 0;
    const int cnx = fnx >> 1, cny = fny >> 1;
    const int64_t c = i + (int64_t)fnx * row;
    const int64_t P = (i >> 1) + (int64_t)cnx * ((j >> 1) + (int64_t)cny * (k >> 1));
    const uint32_t ft = *(const uint32_t*)(ftag + c);
    const uint16_t ct = *(const uint16_t*)(ctag + P);
    const V2 e = *(const V2*)(ec + P);
    V4 xv = *(const V4*)(xf + c);
    bool up[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) up[u] = !(tclass((uint8_t)(ft >> (8 * u))) == 3 || ((ct >> (8 * (u >> 1))) & 4));
    xv.x = up[0] ? xv.x + e.x : xv.x;
    xv.y = up[1] ? xv.y + e.x : xv.y;
    xv.z = up[2] ? xv.z + e.y : xv.z;
    xv.w = up[3] ? xv.w + e.y : xv.w;
    if (up[0] && up[1] && up[2] && up[3]) {
      *(V4*)(xf + c) = xv;
    } else {
      if (up[0]) xf[c] = xv.x;
      if (up[1]) xf[c + 1] = xv.y;
      if (up[2]) xf[c + 2] = xv.z;
      if (up[3]) xf[c + 3] = xv.w;
    }
    return;
  }
  if (blockIdx.y != 0) return;
  const int t = (int)((bid - nrb) * kBlock + threadIdx.y * blockDim.x + threadIdx.x);
  if (t >= nnp) return;
  xf[fdof[t]] += ec[cdof[t]];
}

// Residual of a small level in one launch: blocks [0, nbc) take the template
// and covered cells (MODE as in k_resid_reg), the rest the explicit rows with
// kSub lanes each (as k_resid_irr); TX and NDOT as in k_resid_zm3, with one
// partial per block of this launch.
template <typename T, int DIM, int MODE, typename TX = T, int NDOT = 0>
__global__ void __launch_bounds__(kBlock) k_resid_all(const uint8_t* __restrict__ tag, const TX* __restrict__ x,
                                                      const T* __restrict__ b, T* __restrict__ r, Tmpl<T> tp,
                                                      unsigned nbc, int nrows, const int64_t* __restrict__ dof,
                                                      const int64_t* __restrict__ rp,
                                                      const int32_t* __restrict__ col, const T* __restrict__ val,
                                                      const T* __restrict__ diag, const T* __restrict__ da = nullptr,
                                                      double* __restrict__ part = nullptr, int64_t pt = 0) {
  double d0 = 0, d1 = 0;
  if (blockIdx.x < nbc) {
    const int nx = tp.n[0], ny = tp.n[1];
    const int64_t N = (int64_t)nx * ny * (DIM == 3 ? tp.n[2] : 1);
    const int64_t c = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (c < N) {
      const uint8_t p = tclass(tag[c]);
      if (p != 2) {
        T out;
        if (p == 3) {
          out = MODE == 0 ? T(0) : (T)x[c];
        } else {
          const int i = (int)(c % nx);
          const int64_t jk = c / nx;
          const int j = (int)(jk % ny);
          const int k = DIM == 3 ? (int)(jk / ny) : 0;
          const T xv = (T)x[c];
          T s = 0;
          T dg = tp.M(p);
          if (i > 0) s += (T)x[c - 1] - xv; else dg += tp.CBM(0, p);
          if (i < nx - 1) s += (T)x[c + 1] - xv; else dg += tp.CBM(1, p);
          if (j > 0) s += (T)x[c - nx] - xv; else dg += tp.CBM(2, p);
          if (j < ny - 1) s += (T)x[c + nx] - xv; else dg += tp.CBM(3, p);
          if (DIM == 3) {
            const int64_t sxy = (int64_t)nx * ny;
            if (k > 0) s += (T)x[c - sxy] - xv; else dg += tp.CBM(4, p);
            if (k < tp.n[2] - 1) s += (T)x[c + sxy] - xv; else dg += tp.CBM(5, p);
          }
          const T ax = dg * xv + tp.CO(p) * s;
          out = MODE == 0 ? b[c] - ax : ax;
        }
        r[c] = out;
        if (NDOT > 0) {
          d0 = (double)da[c] * (double)out;
          if (NDOT > 1) d1 = (double)out * (double)out;
        }
      }
    }
  } else {
    const int64_t g = ((int64_t)(blockIdx.x - nbc) * kBlock + threadIdx.x) / kSub;
    const int lane = threadIdx.x % kSub;
    if (g < nrows) {
      const int64_t q = dof[g];
      T s = 0;
      for (int64_t e = rp[g] + lane; e < rp[g + 1]; e += kSub) s += val[e] * (T)x[col[e]];
      for (int off = kSub / 2; off > 0; off >>= 1) s += __shfl_xor(s, off, kSub);
      if (lane == 0) {
        const T ax = diag[g] * (T)x[q] + s;
        const T out = MODE == 0 ? b[q] - ax : ax;
        r[q] = out;
        if (NDOT > 0) {
          d0 = (double)da[q] * (double)out;
          if (NDOT > 1) d1 = (double)out * (double)out;
        }
      }
    }
  }
  if (NDOT > 0) block_partials<kBlock>(d0, d1, NDOT, part, pt, blockIdx.x, threadIdx.x);
}

template <typename T>
__global__ void __launch_bounds__(kBlock) k_fill(T* __restrict__ x, int64_t n, T v) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < n) x[t] = v;
}

// Bottom solve x = Ainv b, one wavefront per row, FP64 accumulation.
template <typename T>
__global__ void __launch_bounds__(64) k_bottom(const double* __restrict__ Ainv, const T* __restrict__ b,
                                               T* __restrict__ x, int n) {
  const int row = blockIdx.x;
  const int lane = threadIdx.x;
  double s = 0;
  for (int c = lane; c < n; c += 64) s += Ainv[(int64_t)row * n + c] * (double)b[c];
  for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
  if (lane == 0) x[row] = (T)s;
}

// Deterministic dot products: a fixed grid of per-block partials (wave64
// shuffles, then a fixed-order sum of the block's waves), then one block sums
// the partials in a fixed order. No atomics, so results are bitwise
// reproducible for a given size.
template <typename T>
__global__ void __launch_bounds__(kBlock) k_dot_partial(const T* __restrict__ a, const T* __restrict__ b, int64_t n,
                                                        double* __restrict__ part) {
  __shared__ double sh[kBlock / 64];
  double s = 0;
  const int64_t st = (int64_t)gridDim.x * blockDim.x;
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  // four strided terms per step with their loads issued together, added in
  // the order of the plain strided loop
  for (; t + 3 * st < n; t += 4 * st) {
    const T a0 = a[t], a1 = a[t + st], a2 = a[t + 2 * st], a3 = a[t + 3 * st];
    const T b0 = b[t], b1 = b[t + st], b2 = b[t + 2 * st], b3 = b[t + 3 * st];
    s += (double)a0 * (double)b0;
    s += (double)a1 * (double)b1;
    s += (double)a2 * (double)b2;
    s += (double)a3 * (double)b3;
  }
  for (; t < n; t += st) s += (double)a[t] * (double)b[t];
  for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double tot = 0;
    for (int w = 0; w < kBlock / 64; ++w) tot += sh[w];
    part[blockIdx.x] = tot;
  }
}

// sums `nvec` consecutive partial arrays of length n into out[0..nvec)
__global__ void __launch_bounds__(kBlock) k_dot_final(const double* __restrict__ part, int n, int nvec,
                                                      double* __restrict__ out) {
  // nvec is 1 or 2; both sums are formed together, four strided terms per
  // step with their loads issued first, each sum taking its terms in the
  // order of the plain strided loop and then the fixed wave/block order
  __shared__ double sh[2][kBlock / 64];
  const double* __restrict__ p0 = part;
  const double* __restrict__ p1 = part + n;
  const bool two = nvec > 1;
  double s0 = 0, s1 = 0;
  int t = threadIdx.x;
  for (; t + 3 * kBlock < n; t += 4 * kBlock) {
    const double a0 = p0[t], a1 = p0[t + kBlock], a2 = p0[t + 2 * kBlock], a3 = p0[t + 3 * kBlock];
    double b0 = 0, b1 = 0, b2 = 0, b3 = 0;
    if (two) {
      b0 = p1[t];
      b1 = p1[t + kBlock];
      b2 = p1[t + 2 * kBlock];
      b3 = p1[t + 3 * kBlock];
    }
    s0 += a0;
    s0 += a1;
    s0 += a2;
    s0 += a3;
    s1 += b0;
    s1 += b1;
    s1 += b2;
    s1 += b3;
  }
  for (; t < n; t += kBlock) {
    s0 += p0[t];
    if (two) s1 += p1[t];
  }
  for (int off = 32; off > 0; off >>= 1) {
    s0 += __shfl_down(s0, off, 64);
    s1 += __shfl_down(s1, off, 64);
  }
  if ((threadIdx.x & 63) == 0) {
    sh[0][threadIdx.x >> 6] = s0;
    sh[1][threadIdx.x >> 6] = s1;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double tot0 = 0, tot1 = 0;
    for (int w = 0; w < kBlock / 64; ++w) {
      tot0 += sh[0][w];
      tot1 += sh[1][w];
    }
    out[0] = tot0;
    if (two) out[1] = tot1;
  }
}

// BiCGStab scalars live on the device: slots of `sc`
// SC_GUESS: 1 when the initial guess has a nonzero entry (set by k_guess_in);
// SC_FIRST: 1 from a (re)start until the first iteration's omega step
enum { SC_RHO = 0, SC_RR, SC_RHO_OLD, SC_ALPHA, SC_OMEGA, SC_RV, SC_TS, SC_TT, SC_GUESS, SC_FIRST, SC_NUM };

__global__ void k_sc_reset(double* sc) {
  sc[SC_RHO] = 1.0;
  sc[SC_RHO_OLD] = 1.0;
  sc[SC_ALPHA] = 1.0;
  sc[SC_OMEGA] = 1.0;
  sc[SC_FIRST] = 1.0;
}

__global__ void k_sc_copy(double* sc, int dst, int src) { sc[dst] = sc[src]; }

__global__ void k_sc_alpha(double* sc) { sc[SC_ALPHA] = sc[SC_RHO] / sc[SC_RV]; }

__global__ void k_sc_omega(double* sc) {
  sc[SC_OMEGA] = sc[SC_TT] > 0.0 ? sc[SC_TS] / sc[SC_TT] : 0.0;
  sc[SC_RHO_OLD] = sc[SC_RHO];
  sc[SC_FIRST] = 0.0;
}

// Fused BiCGStab vector steps. p = r + beta (p - omega v) (resp. s = r -
// alpha v) also clears the preconditioner output z and, for mixed precision,
// stores the preconditioner input bf = (float) p (resp. s), so no separate
// conversion or fill pass is needed.
// Every FP64 stream of the Krylov vector steps carries non-temporal hints:
// between two uses of a Krylov vector lies a V-cycle whose arrays fill the
// last-level cache, so caching these streams only displaces the V-cycle's
// data (the FP32 preconditioner input bf, read by the V-cycle's first
// kernel right after, is stored plainly). 18.3 -> 17.8 ms per 256^3 mixed
// solve; hinting the matrix-vector products' outputs, which the next vector
// step reads, is already the faster choice there.
template <typename Z>
__global__ void __launch_bounds__(kBlock) k_bicg_p2(double* __restrict__ p, const double* __restrict__ r,
                                                    const double* __restrict__ v, const double* __restrict__ sc,
                                                    int64_t n, float* __restrict__ bf, Z* __restrict__ z) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n) return;
  // the first iteration after a (re)start has p = v = 0, so p = r: the old
  // p and v are neither read nor need to be cleared by the restart
  double pv = ld_stream<true>(r + t);
  if (sc[SC_FIRST] == 0.0) {
    const double beta = (sc[SC_RHO] / sc[SC_RHO_OLD]) * (sc[SC_ALPHA] / sc[SC_OMEGA]);
    pv = pv + beta * (ld_stream<true>(p + t) - sc[SC_OMEGA] * ld_stream<true>(v + t));
  }
  st_stream<true>(pv, p + t);
  if (bf) bf[t] = (float)pv;
  if (z) z[t] = Z(0);
}

template <typename Z>
__global__ void __launch_bounds__(kBlock) k_bicg_s2(double* __restrict__ s, const double* __restrict__ r,
                                                    const double* __restrict__ v, const double* __restrict__ sc,
                                                    int64_t n, float* __restrict__ bf, Z* __restrict__ z) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n) return;
  const double sv = ld_stream<true>(r + t) - sc[SC_ALPHA] * ld_stream<true>(v + t);
  st_stream<true>(sv, s + t);
  if (bf) bf[t] = (float)sv;
  if (z) z[t] = Z(0);
}

// x += alpha ph + omega sh ; r = s - omega t, with the partials of (rh, r)
// and (r, r) for the next iteration (grid of kNormBlocks, the same
// partition as k_dot_partial). A breakdown (alpha or omega not finite, e.g.
// (rh, v) = 0) leaves x and r as they were, so that the host's restart from
// the true residual starts from the last good iterate; the partials are then
// zero and the host tests the true residual.
template <typename Z>
__global__ void __launch_bounds__(kBlock) k_bicg_xr2(double* __restrict__ x, double* __restrict__ r,
                                                     const Z* __restrict__ ph, const Z* __restrict__ sh,
                                                     const double* __restrict__ s, const double* __restrict__ tv,
                                                     const double* __restrict__ rh, const double* __restrict__ sc,
                                                     int64_t n, double* __restrict__ part) {
  const double a = sc[SC_ALPHA], w = sc[SC_OMEGA];
  double d0 = 0, d1 = 0;
  if (!isfinite(a) || !isfinite(w)) n = 0;
  const int64_t st = (int64_t)gridDim.x * blockDim.x;
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  // two strided entries per step with their loads issued together; the
  // partials take them in the order of the plain strided loop
  for (; t + st < n; t += 2 * st) {
    const int64_t u = t + st;
    const double x0 = ld_stream<true>(x + t), x1 = ld_stream<true>(x + u);
    const Z p0 = ld_stream<true>(ph + t), p1 = ld_stream<true>(ph + u), q0 = ld_stream<true>(sh + t),
            q1 = ld_stream<true>(sh + u);
    const double s0 = ld_stream<true>(s + t), s1 = ld_stream<true>(s + u), v0 = ld_stream<true>(tv + t),
                 v1 = ld_stream<true>(tv + u), h0 = ld_stream<true>(rh + t), h1 = ld_stream<true>(rh + u);
    st_stream<true>(x0 + (a * (double)p0 + w * (double)q0), x + t);
    st_stream<true>(x1 + (a * (double)p1 + w * (double)q1), x + u);
    const double r0 = s0 - w * v0, r1 = s1 - w * v1;
    r[t] = r0;
    r[u] = r1;
    d0 += h0 * r0;
    d1 += r0 * r0;
    d0 += h1 * r1;
    d1 += r1 * r1;
  }
  for (; t < n; t += st) {
    x[t] += a * (double)ph[t] + w * (double)sh[t];
    const double rv = s[t] - w * tv[t];
    r[t] = rv;
    d0 += rh[t] * rv;
    d1 += rv * rv;
  }
  block_partials<kBlock>(d0, d1, 2, part, gridDim.x, blockIdx.x, threadIdx.x);
}

template <typename S, typename D>
__global__ void __launch_bounds__(kBlock) k_convert(const S* __restrict__ s, D* __restrict__ d, int64_t n) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < n) d[t] = (D)s[t];
}

// The initial guess taken from the caller's array, in one pass with setting
// the covered entries to 0: covered cells are identity rows with b = 0 that
// no sweep, correction or Krylov update touches. tag null: every entry is
// taken as it is (second-phase unknowns). *nz (cleared before) is set to 1
// when an entry taken is nonzero: a zero guess lets the solve take r = b
// without forming A x (every lane that sees one writes the same value).
__global__ void __launch_bounds__(kBlock) k_guess_in(const uint8_t* __restrict__ tag, const double* __restrict__ phi,
                                                     double* __restrict__ x, int64_t n, double* __restrict__ nz) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  bool any = false;
  if (t < n) {
    const double v = (tag && tclass(tag[t]) == 3) ? 0.0 : phi[t];
    x[t] = v;
    any = v != 0.0;
  }
  if (__any(any) && (threadIdx.x & 63) == 0) *nz = 1.0;
}

// Krylov (re)start in one pass: r = rh = r0 (p and v are not read before
// the first iteration writes them, see k_bicg_p2).
__global__ void __launch_bounds__(kBlock) k_bicg_restart(const double* __restrict__ r0, double* __restrict__ r,
                                                         double* __restrict__ rh, int64_t n) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n) return;
  const double a = r0[t];
  r[t] = a;
  rh[t] = a;
}

__global__ void __launch_bounds__(kBlock) k_add_f32(double* __restrict__ x, const float* __restrict__ e, int64_t n) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < n) x[t] += (double)e[t];
}

// Right-hand side of regular and covered cells (3D launch grid).
template <int DIM>
__global__ void __launch_bounds__(kBlock) k_rhs_reg(const uint8_t* __restrict__ tag, const double* __restrict__ rho,
                                                    double* __restrict__ b, Tmpl<double> dat, int unused) {
  (void)unused;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int j = blockIdx.y * blockDim.y + threadIdx.y;
  const int k = DIM == 3 ? (int)blockIdx.z : 0;
  if (i >= dat.n[0] || j >= dat.n[1]) return;
  const int64_t c = i + (int64_t)dat.n[0] * (j + (int64_t)dat.n[1] * k);
  const uint8_t p = tclass(tag[c]);
  if (p == 3) {
    b[c] = 0;
    return;
  }
  if (p == 2) return;
  double v = rho[c];
  // dat.cb[f][p] holds dat[f][p] * value_f
  if (i == 0) v -= dat.CB(0, p);
  if (i == dat.n[0] - 1) v -= dat.CB(1, p);
  if (j == 0) v -= dat.CB(2, p);
  if (j == dat.n[1] - 1) v -= dat.CB(3, p);
  if (DIM == 3) {
    if (k == 0) v -= dat.CB(4, p);
    if (k == dat.n[2] - 1) v -= dat.CB(5, p);
  }
  b[c] = v;
}

struct FaceVals {
  double v[6];
};

__global__ void __launch_bounds__(kBlock) k_rhs_irr(int nrows, const int64_t* __restrict__ dof,
                                                    const int64_t* __restrict__ cell, const double* __restrict__ src,
                                                    const double* __restrict__ cface, const int32_t* __restrict__ obj,
                                                    const double* __restrict__ cobj, const double* __restrict__ csig,
                                                    const double* __restrict__ rho, const double* __restrict__ sigma,
                                                    const double* __restrict__ objv, FaceVals fv,
                                                    double* __restrict__ b) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nrows) return;
  const int64_t c = cell[t];
  double v = src[t] * rho[c];
  for (int f = 0; f < 6; ++f) v -= cface[6 * t + f] * fv.v[f];
  if (obj[t] >= 0) v -= cobj[t] * objv[obj[t]];
  if (sigma) v -= csig[t] * sigma[c];
  b[dof[t]] = v;
}

// Cell-centred E of regular cells (covered cells 0), 3D launch grid.
template <int DIM>
__global__ void __launch_bounds__(kBlock) k_efield_reg(const uint8_t* __restrict__ tag, const double* __restrict__ x,
                                                       double* __restrict__ E, Tmpl<double> ga, Tmpl<double> gbv,
                                                       double inv_h) {
  const int nx = ga.n[0], ny = ga.n[1];
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int j = blockIdx.y * blockDim.y + threadIdx.y;
  const int k = DIM == 3 ? (int)blockIdx.z : 0;
  if (i >= nx || j >= ny) return;
  const int64_t N = (int64_t)nx * ny * (DIM == 3 ? ga.n[2] : 1);
  const int64_t c = i + (int64_t)nx * (j + (int64_t)ny * k);
  const uint8_t p = tclass(tag[c]);
  if (p == 3) {
    for (int d = 0; d < DIM; ++d) E[d * N + c] = 0;
    return;
  }
  if (p == 2) return;
  const int idx[3] = {i, j, k};
  const int64_t stride[3] = {1, nx, (int64_t)nx * ny};
  const double xc = x[c];
  for (int d = 0; d < DIM; ++d) {
    double glo, ghi;
    // ga.CB(f, p) = closure coefficient on phi, gbv.CB(f, p) = coefficient * value
    if (idx[d] > 0)
      glo = (xc - x[c - stride[d]]) * inv_h;
    else
      glo = -(ga.CB(2 * d, p) * xc + gbv.CB(2 * d, p));
    if (idx[d] < ga.n[d] - 1)
      ghi = (x[c + stride[d]] - xc) * inv_h;
    else
      ghi = ga.CB(2 * d + 1, p) * xc + gbv.CB(2 * d + 1, p);
    E[d * N + c] = -0.5 * (glo + ghi);
  }
}

// The same field of a large 3D level marching along z: each thread owns one
// (i, j) column of a kEZX x kEZY tile and walks kEZ planes, keeping x of
// planes k - 1, k and k + 1 in registers, so x leaves HBM once (the in-plane
// neighbours are cache hits) where the plane-by-plane grid re-reads the
// planes above and below. The arithmetic per component is k_efield_reg's.
constexpr int kEZX = 64, kEZY = 4, kEZ = 32;
__global__ void __launch_bounds__(kEZX * kEZY) k_efield_zm3(const uint8_t* __restrict__ tag,
                                                          const double* __restrict__ x, double* __restrict__ E,
                                                          Tmpl<double> ga, Tmpl<double> gbv, double inv_h) {
  const int nx = ga.n[0], ny = ga.n[1], nz = ga.n[2];
  const int i = blockIdx.x * kEZX + threadIdx.x;
  const int j = blockIdx.y * kEZY + threadIdx.y;
  const int z0 = blockIdx.z * kEZ, z1 = min(z0 + kEZ, nz);
  if (i >= nx || j >= ny) return;
  const int64_t sxy = (int64_t)nx * ny, N = sxy * nz;
  int64_t c = i + (int64_t)nx * j + sxy * z0;
  double xm = z0 > 0 ? x[c - sxy] : 0.0;
  double xc = x[c];
  for (int k = z0; k < z1; ++k, c += sxy) {
    const double xp = k + 1 < nz ? x[c + sxy] : 0.0;
    const double xw = i > 0 ? x[c - 1] : 0.0, xe = i < nx - 1 ? x[c + 1] : 0.0;
    const double xs = j > 0 ? x[c - nx] : 0.0, xn = j < ny - 1 ? x[c + nx] : 0.0;
    const uint8_t p = tclass(tag[c]);
    if (p == 3) {
      E[c] = 0;
      E[N + c] = 0;
      E[2 * N + c] = 0;
    } else if (p != 2) {
      double glo, ghi;
      if (i > 0)
        glo = (xc - xw) * inv_h;
      else
        glo = -(ga.CB(0, p) * xc + gbv.CB(0, p));
      if (i < nx - 1)
        ghi = (xe - xc) * inv_h;
      else
        ghi = ga.CB(1, p) * xc + gbv.CB(1, p);
      E[c] = -0.5 * (glo + ghi);
      if (j > 0)
        glo = (xc - xs) * inv_h;
      else
        glo = -(ga.CB(2, p) * xc + gbv.CB(2, p));
      if (j < ny - 1)
        ghi = (xn - xc) * inv_h;
      else
        ghi = ga.CB(3, p) * xc + gbv.CB(3, p);
      E[N + c] = -0.5 * (glo + ghi);
      if (k > 0)
        glo = (xc - xm) * inv_h;
      else
        glo = -(ga.CB(4, p) * xc + gbv.CB(4, p));
      if (k < nz - 1)
        ghi = (xp - xc) * inv_h;
      else
        ghi = ga.CB(5, p) * xc + gbv.CB(5, p);
      E[2 * N + c] = -0.5 * (glo + ghi);
    }
    xm = xc;
    xc = xp;
  }
}

__global__ void __launch_bounds__(kBlock) k_efield_irr(int ncell, int dim, int64_t N, const int64_t* __restrict__ ecell,
                                                       const int64_t* __restrict__ rp, const int32_t* __restrict__ col,
                                                       const double* __restrict__ val, const double* __restrict__ cface,
                                                       const int32_t* __restrict__ obj, const double* __restrict__ cobj,
                                                       const double* __restrict__ csig, const double* __restrict__ x,
                                                       const double* __restrict__ sigma,
                                                       const double* __restrict__ objv, FaceVals fv,
                                                       double* __restrict__ E) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= ncell * dim) return;
  const int q = t / dim, d = t % dim;
  const int e = 3 * q + d;
  const int64_t c = ecell[q];
  double v = 0;
  for (int64_t z = rp[e]; z < rp[e + 1]; ++z) v += val[z] * x[col[z]];
  for (int f = 0; f < 6; ++f) v += cface[6 * e + f] * fv.v[f];
  if (obj[e] >= 0) v += cobj[e] * objv[obj[e]];
  if (sigma) v += csig[e] * sigma[c];
  E[d * N + c] = v;
}

}  // namespace ebmg
