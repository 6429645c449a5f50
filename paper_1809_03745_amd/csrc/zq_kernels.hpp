// Quad form of the z-marching red/black Gauss-Seidel sweep (Multigrid
// solver: red/black relaxation of the template cells), 3D, x extent a
// multiple of 4.
//
// The same sweep as k_rb_zm3 (a red half-sweep over the template cells
// followed by a black one, explicit rows, covered cells and second-phase
// unknowns left as they are) with the same arithmetic per cell, so the
// results agree bitwise; what changes is who does what:
//   * each thread owns four consecutive cells of a tile row (a "quad": two
//     cells of each colour in every plane), read from LDS and written to
//     memory as one 16-byte vector, with its tags as one 32-bit word and its
//     b values as one vector, kept in registers instead of LDS;
//   * the x halo of a plane is staged as aligned 4-cell chunks (one 16-byte
//     load and one 16-byte LDS store each);
//   * every wavefront takes tile rows of one parity, so which two cells of a
//     quad are red in a plane is the same for the whole wavefront and is
//     decided by a scalar branch instead of per-lane selects;
//   * the red cells of the one-cell ring around the tile (recomputed from
//     the same old values as the neighbouring blocks do, so blocks never
//     exchange data) are taken one per thread by the first TX + TY + 2
//     threads: the ring, walked around the tile, alternates colours, so
//     each of these threads owns two consecutive ring cells of which exactly
//     one is red in a plane (the same one for every thread).
// Per plane step k: stage the x chunks of plane k + 2 (loaded two steps
// earlier) and request those of plane k + 4 and the b / tag words of plane
// k + 2; red update of plane k (quads and ring); barrier; black update of
// plane k - 1 and its store; barrier. b / tag words live for four steps (two
// in flight, one for the red and one for the black update), so the march is
// unrolled by four steps with one register set per step.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kernels.hpp"

namespace ebmg {

// One plane step's red or black update of the two cells {H, H + 2} of a
// quad: c the quad, s / n its y- / y+ neighbours, d / u its z- / z+
// neighbours, lft / rgt the cells left of cell 0 and right of cell 3. zint:
// the plane is not a z face (inner form with the reciprocal in-plane
// diagonals rq[phase][cell]); otherwise the general form. Returns the quad
// with the two cells replaced where they are template cells (class <= 1).
template <typename T, int H>
__device__ __forceinline__ void zq_pair(T (&c)[4], const T (&s)[4], const T (&n)[4], const T (&d)[4],
                                        const T (&u)[4], T lft, T rgt, uint32_t tq, const T (&bq)[4],
                                        const T (&rq)[2][4], const T (*TC)[8], bool zint, int gx0, int gy, int z,
                                        int nx, int ny, int nz) {
  constexpr int A = H, B = H + 2;
  const T wa = H ? c[0] : lft, ea = c[A + 1];
  const T wb = c[B - 1], eb = H ? rgt : c[3];
  const int ca = (int)((tq >> (8 * A)) & 3u), cb = (int)((tq >> (8 * B)) & 3u);
  const int pa = ca & 1, pb = cb & 1;
  T va, vb;
  if (zint) {
    const T ra0 = rq[0][A], ra1 = rq[1][A], rb0 = rq[0][B], rb1 = rq[1][B];
    va = zv_inner<T>(wa, ea, s[A], n[A], d[A], u[A], TC[pa][0], bq[A], pa ? ra1 : ra0);
    vb = zv_inner<T>(wb, eb, s[B], n[B], d[B], u[B], TC[pb][0], bq[B], pb ? rb1 : rb0);
  } else {
    va = zv_general<T>(wa, ea, s[A], n[A], d[A], u[A], gx0 + A, gy, z, nx, ny, nz, TC[pa], bq[A]);
    vb = zv_general<T>(wb, eb, s[B], n[B], d[B], u[B], gx0 + B, gy, z, nx, ny, nz, TC[pb], bq[B]);
  }
  if (ca <= 1) c[A] = va;
  if (cb <= 1) c[B] = vb;
}

// (column, row) of cell i of the ring around a TX x TY tile, walked from
// (-1, -1) along row -1, up column TX, back along row TY and down column -1
template <int TX, int TY>
__device__ __forceinline__ void zq_ring_cell(int i, int& c, int& r) {
  if (i < TX + 2) {
    c = i - 1;
    r = -1;
  } else if (i < TX + TY + 3) {
    c = TX;
    r = i - (TX + 2);
  } else if (i < 2 * TX + TY + 4) {
    c = TX - 1 - (i - (TX + TY + 3));
    r = TY;
  } else {
    c = -1;
    r = TY - 1 - (i - (2 * TX + TY + 4));
  }
}

template <typename T, int TX, int TY, int KZ, int OCC, bool ZIN = false>
__global__ void __launch_bounds__(TX * TY / 4, OCC) k_rb_zq3(const uint8_t* __restrict__ tag,
                                                         const T* __restrict__ xin, T* __restrict__ xout,
                                                         const T* __restrict__ b, Tmpl<T> tp, int64_t nsec) {
  typedef T Q __attribute__((ext_vector_type(4)));
  constexpr int NT = TX * TY / 4, QX = TX / 4, RPW = 64 / QX;
  constexpr int PQ = QX + 2, PW = 4 * PQ, PH = TY + 4, NQ = PQ * PH;   // LDS plane: columns -4 .. TX+3, rows -2 .. TY+1
  constexpr int UC = (NQ + NT - 1) / NT;                               // staged chunks per thread
  constexpr int NRING = TX + TY + 2;                                   // red ring cells per plane
  static_assert(TX % 4 == 0 && 64 % QX == 0 && NT % 64 == 0, "the quads of a tile row fill whole wavefronts");
  static_assert(TY % (2 * RPW) == 0, "a wavefront takes tile rows of one parity");
  static_assert(NRING <= NT, "one ring cell pair per thread at most");
  __shared__ Q V[5][NQ];
  __shared__ T TC[2][8];
  const int nx = tp.n[0], ny = tp.n[1], nz = tp.n[2];
  const int bx = (nx + TX - 1) / TX, by = (ny + TY - 1) / TY;
  const int64_t nblocks = (int64_t)gridDim.x;
  const int64_t t = xcd_block(blockIdx.x, nblocks);
  const int x0 = (int)(t % bx) * TX, y0 = (int)((t / bx) % by) * TY;
  const int z0 = (int)(t / ((int64_t)bx * by)) * KZ;
  const int z1 = min(z0 + KZ, nz);
  const int tid = threadIdx.x;
  const int64_t sxy = (int64_t)nx * ny;
  if (tid < 16) {
    const int p = tid >> 3, j = tid & 7;
    TC[p][j] = j == 0 ? tp.coff[p] : (j == 1 ? tp.d0[p] : tp.cb[j - 2][p]);
  }
  __syncthreads();

  // this thread's quad: wavefront w takes rows base + 2 j (one parity)
  const int wv = tid >> 6, ln = tid & 63;
  const int ry = (wv >> 1) * (2 * RPW) + (wv & 1) + 2 * (ln / QX);
  const int m = ln % QX;
  const int gx0 = x0 + 4 * m, gy = y0 + ry;
  const bool qin = gx0 < nx && gy < ny;
  const int qoff = qin ? gx0 + nx * gy : 0;
  const int qi = (ry + 2) * PQ + m + 1;
  const int hrow = __builtin_amdgcn_readfirstlane((y0 + ry) & 1);
  T rq[2][4];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    rq[0][i] = zm_inplane_rdg<T>(gx0 + i, gy, nx, ny, TC[0]);
    rq[1][i] = zm_inplane_rdg<T>(gx0 + i, gy, nx, ny, TC[1]);
  }

  // staged chunks: LDS quad q of a plane holds the four cells of row
  // y0 - 2 + q / PQ from column x0 - 4 + 4 (q % PQ); a chunk lies wholly in
  // or out of the box (x0 and nx are multiples of 4)
  int coff[UC];
  uint32_t cin = 0;
#pragma unroll
  for (int u = 0; u < UC; ++u) {
    const int q = tid + u * NT;
    const int gx = x0 - 4 + 4 * (q % PQ), gyc = y0 - 2 + q / PQ;
    const bool ok = q < NQ && gx >= 0 && gx < nx && gyc >= 0 && gyc < ny;
    coff[u] = ok ? gx + nx * gyc : 0;
    cin |= (uint32_t)ok << u;
  }

  // ring cells 2 tid (a) and 2 tid + 1 (b); a is red in plane k iff
  // x0 + y0 + k is even, for every thread
  const bool rg = tid < NRING;
  int rca, rra, rcb, rrb;
  zq_ring_cell<TX, TY>(rg ? 2 * tid : 0, rca, rra);
  zq_ring_cell<TX, TY>(rg ? 2 * tid + 1 : 1, rcb, rrb);
  const int rgxa = x0 + rca, rgya = y0 + rra, rgxb = x0 + rcb, rgyb = y0 + rrb;
  const bool ina = rg && rgxa >= 0 && rgxa < nx && rgya >= 0 && rgya < ny;
  const bool inb = rg && rgxb >= 0 && rgxb < nx && rgyb >= 0 && rgyb < ny;
  const int rla = (rra + 2) * PW + rca + 4, rlb = (rrb + 2) * PW + rcb + 4;
  const int roffa = ina ? rgxa + nx * rgya : 0, roffb = inb ? rgxb + nx * rgyb : 0;
  const T ra0 = zm_inplane_rdg<T>(rgxa, rgya, nx, ny, TC[0]), ra1 = zm_inplane_rdg<T>(rgxa, rgya, nx, ny, TC[1]);
  const T rb0 = zm_inplane_rdg<T>(rgxb, rgyb, nx, ny, TC[0]), rb1 = zm_inplane_rdg<T>(rgxb, rgyb, nx, ny, TC[1]);
  const int rpar = (x0 + y0) & 1;

  // registers in flight: x chunks of two planes (A, B), and the b / tag
  // words of four planes (sets 0..3)
  Q XA[UC], XB[UC];
  Q BQ0, BQ1, BQ2, BQ3;
  uint32_t TQ0, TQ1, TQ2, TQ3;
  T RB0, RB1, RB2, RB3;
  uint8_t RT0, RT1, RT2, RT3;

#define ZQ_LOADX(P, z, QV)                                                              \
  if constexpr (!ZIN) {                                                                 \
    const int zz_ = (z);                                                                \
    const int64_t zoff_ = sxy * (zz_ >= 0 && zz_ < nz ? zz_ : 0);                      \
    _Pragma("unroll") for (int u = 0; u < UC; ++u) P[u] = *(QV const Q*)(xin + zoff_ + coff[u]); \
  }
#define ZQ_LOADBT(S, z, QV)                                                             \
  {                                                                                     \
    const int zz_ = (z);                                                                \
    const int64_t zoff_ = sxy * (zz_ >= 0 && zz_ < nz ? zz_ : 0);                      \
    BQ##S = *(QV const Q*)(b + zoff_ + qoff);                                           \
    TQ##S = *(QV const uint32_t*)(tag + zoff_ + qoff);                                  \
    const int ro_ = ((rpar + zz_) & 1) == 0 ? roffa : roffb;                            \
    RB##S = ((QV const T*)b)[zoff_ + ro_];                                              \
    RT##S = ((QV const uint8_t*)tag)[zoff_ + ro_];                                      \
  }
#define ZQ_STORE(P, z, VS)                                                              \
  {                                                                                     \
    const int zz_ = (z);                                                                \
    const bool zin_ = zz_ >= 0 && zz_ < nz;                                             \
    _Pragma("unroll") for (int u = 0; u < UC; ++u) {                                    \
      const int q = tid + u * NT;                                                       \
      if (UC * NT == NQ || q < NQ) {                                                    \
        Q v_ = Q(0);                                                                    \
        if constexpr (!ZIN) v_ = (zin_ && ((cin >> u) & 1)) ? P[u] : Q(0);              \
        V[VS][q] = v_;                                                                  \
      }                                                                                 \
    }                                                                                   \
  }
  // red update of plane k (quad cells and the ring's red cell) with the b /
  // tag words of set SR; black update of plane k - 1 with set SB and its
  // store; staging of plane k + 2 from P, loads of plane k + 4 into P and of
  // the b / tag words of plane k + 2 into set SL
#define ZQ_STEP(P, SR, SB, SL, kk)                                                      \
  {                                                                                     \
    const int k = (kk);                                                                 \
    ZQ_STORE(P, k + 2, sVp2);                                                           \
    ZQ_LOADX(P, min(k + 4, z1 + 1), );                                                  \
    ZQ_LOADBT(SL, min(k + 2, z1 + 1), );                                                \
    if (k >= 0 && k < nz) {                                                             \
      const bool zint = k > 0 && k < nz - 1;                                            \
      const Q* vm = V[sVm1];                                                            \
      Q* vc = V[sV0];                                                                   \
      const Q* vp = V[sVp1];                                                            \
      const int h = (hrow + k) & 1;                                                     \
      T c[4], s[4], n[4], d[4], u[4], bq[4];                                            \
      const Q cq = vc[qi], sq = vc[qi - PQ], nq = vc[qi + PQ], dq = vm[qi], uq = vp[qi]; \
      _Pragma("unroll") for (int i = 0; i < 4; ++i) {                                   \
        c[i] = cq[i]; s[i] = sq[i]; n[i] = nq[i]; d[i] = dq[i]; u[i] = uq[i];           \
        bq[i] = BQ##SR[i];                                                              \
      }                                                                                 \
      const T* vcs = (const T*)vc;                                                      \
      if (h == 0)                                                                       \
        zq_pair<T, 0>(c, s, n, d, u, vcs[4 * qi - 1], T(0), TQ##SR, bq, rq, TC, zint, gx0, gy, k, nx, ny, nz); \
      else                                                                              \
        zq_pair<T, 1>(c, s, n, d, u, T(0), vcs[4 * qi + 4], TQ##SR, bq, rq, TC, zint, gx0, gy, k, nx, ny, nz); \
      if (rg) { /* the ring's red cell */                                               \
        const bool sa = ((rpar + k) & 1) == 0;                                          \
        const int l = sa ? rla : rlb;                                                   \
        const int cls = (int)(RT##SR & 3);                                              \
        const int p = cls & 1;                                                          \
        T* vf = (T*)vc;                                                                 \
        const T* vmf = (const T*)vm;                                                    \
        const T* vpf = (const T*)vp;                                                    \
        T v;                                                                            \
        if (zint) {                                                                     \
          const T r = sa ? (p ? ra1 : ra0) : (p ? rb1 : rb0);                           \
          v = zv_inner<T>(vf[l - 1], vf[l + 1], vf[l - PW], vf[l + PW], vmf[l], vpf[l], TC[p][0], RB##SR, r); \
        } else {                                                                        \
          v = zv_general<T>(vf[l - 1], vf[l + 1], vf[l - PW], vf[l + PW], vmf[l], vpf[l], sa ? rgxa : rgxb, \
                            sa ? rgya : rgyb, k, nx, ny, nz, TC[p], RB##SR);            \
        }                                                                               \
        if ((sa ? ina : inb) && cls <= 1) vf[l] = v;                                    \
      }                                                                                 \
      if (qin) vc[qi] = Q{c[0], c[1], c[2], c[3]};                                      \
    }                                                                                   \
    __syncthreads();                                                                    \
    const int kb = k - 1;                                                               \
    if (kb >= z0 && kb < z1) { /* black update of plane k-1, and its store */          \
      const bool zint = kb > 0 && kb < nz - 1;                                          \
      const Q* vm = V[sVm2];                                                            \
      const Q* vc = V[sVm1];                                                            \
      const Q* vp = V[sV0];                                                             \
      const int h = (hrow + k) & 1;                                                     \
      T c[4], s[4], n[4], d[4], u[4], bq[4];                                            \
      const Q cq = vc[qi], sq = vc[qi - PQ], nq = vc[qi + PQ], dq = vm[qi], uq = vp[qi]; \
      _Pragma("unroll") for (int i = 0; i < 4; ++i) {                                   \
        c[i] = cq[i]; s[i] = sq[i]; n[i] = nq[i]; d[i] = dq[i]; u[i] = uq[i];           \
        bq[i] = BQ##SB[i];                                                              \
      }                                                                                 \
      const T* vcs = (const T*)vc;                                                      \
      if (h == 0)                                                                       \
        zq_pair<T, 0>(c, s, n, d, u, vcs[4 * qi - 1], T(0), TQ##SB, bq, rq, TC, zint, gx0, gy, kb, nx, ny, nz); \
      else                                                                              \
        zq_pair<T, 1>(c, s, n, d, u, T(0), vcs[4 * qi + 4], TQ##SB, bq, rq, TC, zint, gx0, gy, kb, nx, ny, nz); \
      if (qin) *(Q*)(xout + sxy * kb + qoff) = Q{c[0], c[1], c[2], c[3]};               \
    }                                                                                   \
    __syncthreads();                                                                    \
    {                                                                                   \
      const int t5_ = sVm2;                                                             \
      sVm2 = sVm1;                                                                      \
      sVm1 = sV0;                                                                       \
      sV0 = sVp1;                                                                       \
      sVp1 = sVp2;                                                                      \
      sVp2 = t5_;                                                                       \
    }                                                                                   \
  }

  // LDS ring slots: plane p lives in V[(p + 10) % 5]
  int sVm2 = (z0 - 3 + 10) % 5, sVm1 = (z0 - 2 + 10) % 5, sV0 = (z0 - 1 + 10) % 5, sVp1 = (z0 + 10) % 5,
      sVp2 = (z0 + 1 + 10) % 5;
  ZQ_LOADX(XA, z0 - 2, );
  ZQ_STORE(XA, z0 - 2, (z0 - 2 + 10) % 5);
  ZQ_LOADX(XA, z0 - 1, );
  ZQ_STORE(XA, z0 - 1, (z0 - 1 + 10) % 5);
  ZQ_LOADX(XA, z0, );
  ZQ_STORE(XA, z0, (z0 + 10) % 5);
  // the planes in flight at the loop head, requested in the loop's own
  // order (volatile reads keep it): x of z0+1 and b / tags of z0-1 as a
  // step of A, then x of z0+2 and b / tags of z0 as a step of B; otherwise
  // the wait counts at the loop head would drain every load in flight
  ZQ_LOADX(XA, z0 + 1, volatile);
  ZQ_LOADBT(0, z0 - 1, volatile);
  ZQ_LOADX(XB, z0 + 2, volatile);
  ZQ_LOADBT(1, z0, volatile);
  __syncthreads();
  // steps k = z0 - 1 .. z1 (the last one's black plane z1 - 1); step s =
  // k - z0 + 1 reads b / tags of set s % 4 (red), (s + 3) % 4 (black) and
  // loads set (s + 2) % 4; x chunks alternate A, B
  const int kend = z1;
  int kq = z0 - 1;
  for (; kq + 3 <= kend; kq += 4) {
    ZQ_STEP(XA, 0, 3, 2, kq);
    ZQ_STEP(XB, 1, 0, 3, kq + 1);
    ZQ_STEP(XA, 2, 1, 0, kq + 2);
    ZQ_STEP(XB, 3, 2, 1, kq + 3);
  }
  if (kq <= kend) ZQ_STEP(XA, 0, 3, 2, kq);
  if (kq + 1 <= kend) ZQ_STEP(XB, 1, 0, 3, kq + 1);
  if (kq + 2 <= kend) ZQ_STEP(XA, 2, 1, 0, kq + 2);
#undef ZQ_STEP
#undef ZQ_STORE
#undef ZQ_LOADBT
#undef ZQ_LOADX
  // second-phase unknowns are not touched by this sweep: copy them through
  const int64_t N = sxy * nz;
  for (int64_t q = (int64_t)blockIdx.x * NT + tid; q < nsec; q += nblocks * NT) xout[N + q] = ZIN ? T(0) : xin[N + q];
}

}  // namespace ebmg
