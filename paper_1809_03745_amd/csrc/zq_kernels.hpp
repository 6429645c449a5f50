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
// Per plane step k: stage the x chunks of plane k + 3 (loaded two steps
// earlier) and request those of plane k + 5; red update of plane k + 1
// (quads and ring) and black update of plane k - 1 with its store, in one
// phase (they touch disjoint planes of a six-plane LDS ring); request the
// b / tag words of plane k + 1 (its black update) and k + 3 (its red
// update); one barrier. Every register set in flight alternates between
// two copies (A, B), loaded two steps ahead of its use.
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
  __shared__ Q V[6][NQ];
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
  // reciprocal in-plane diagonals per phase and cell; cells 1 and 2 of a
  // quad are never on an x face, so they share one value
  T rq[2][4];
#pragma unroll
  for (int p = 0; p < 2; ++p) {
    rq[p][0] = zm_inplane_rdg<T>(gx0, gy, nx, ny, TC[p]);
    rq[p][1] = zm_inplane_rdg<T>(gx0 + 1, gy, nx, ny, TC[p]);
    rq[p][2] = rq[p][1];
    rq[p][3] = zm_inplane_rdg<T>(gx0 + 3, gy, nx, ny, TC[p]);
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
  // (on z faces the ring cell's position is recovered from its LDS index)
  const int rla = (rra + 2) * PW + rca + 4, rlb = (rrb + 2) * PW + rcb + 4;
  const int roffa = ina ? rgxa + nx * rgya : 0, roffb = inb ? rgxb + nx * rgyb : 0;
  const T ra0 = zm_inplane_rdg<T>(rgxa, rgya, nx, ny, TC[0]), ra1 = zm_inplane_rdg<T>(rgxa, rgya, nx, ny, TC[1]);
  const T rb0 = zm_inplane_rdg<T>(rgxb, rgyb, nx, ny, TC[0]), rb1 = zm_inplane_rdg<T>(rgxb, rgyb, nx, ny, TC[1]);
  const int rpar = (x0 + y0) & 1;

  // registers in flight, two sets each (A, B), all loaded two steps ahead
  // of their use: x chunks; b / tag words of the plane of a red update (R)
  // and of the plane of a black update (K: the same words again, read a
  // second time, from the cache, so that no register set is copied)
  Q XA[UC], XB[UC];
  Q BRA, BRB, BKA, BKB;
  uint32_t TRA, TRB, TKA, TKB;   // the quad's four tags (raw words: decoded where used, so
                                 // that no load is waited for before its step)
  T RBA, RBB;
  uint32_t RTA, RTB;             // the ring cell's tag

  // loads address the arrays by 32-bit offsets from their base (the
  // caller keeps every array below 2^31 bytes): plane offset (uniform) plus
  // in-plane offset (per lane)
#define ZQ_AT(ptr, TY2, QV, eoff) (*(QV const TY2*)((const char*)(ptr) + (uint32_t)(eoff)))
#define ZQ_LOADX(P, z, QV)                                                              \
  if constexpr (!ZIN) {                                                                 \
    const int zz_ = (z);                                                                \
    const uint32_t zo_ = (uint32_t)sxy * (uint32_t)(zz_ >= 0 && zz_ < nz ? zz_ : 0);   \
    _Pragma("unroll") for (int u = 0; u < UC; ++u)                                      \
      P[u] = ZQ_AT(xin, Q, QV, (zo_ + (uint32_t)coff[u]) * (uint32_t)sizeof(T));        \
  }
#define ZQ_LOADBT(S, z, QV)                                                             \
  {                                                                                     \
    const int zz_ = (z);                                                                \
    const uint32_t zo_ = (uint32_t)sxy * (uint32_t)(zz_ >= 0 && zz_ < nz ? zz_ : 0);   \
    BR##S = ZQ_AT(b, Q, QV, (zo_ + (uint32_t)qoff) * (uint32_t)sizeof(T));              \
    TR##S = ZQ_AT(tag, uint32_t, QV, zo_ + (uint32_t)qoff);                             \
    const uint32_t ro_ = zo_ + (uint32_t)(((rpar + zz_) & 1) == 0 ? roffa : roffb);     \
    RB##S = ZQ_AT(b, T, QV, ro_ * (uint32_t)sizeof(T));                                 \
    RT##S = ZQ_AT(tag, uint8_t, QV, ro_);                                               \
  }
#define ZQ_LOADK(S, z)                                                                  \
  {                                                                                     \
    const int zz_ = (z);                                                                \
    const uint32_t zo_ = (uint32_t)sxy * (uint32_t)(zz_ >= 0 && zz_ < nz ? zz_ : 0);   \
    BK##S = ZQ_AT(b, Q, , (zo_ + (uint32_t)qoff) * (uint32_t)sizeof(T));                \
    TK##S = ZQ_AT(tag, uint32_t, , zo_ + (uint32_t)qoff);                               \
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
  // Step k: stage plane k + 3 (x chunks of X##P, loaded two steps earlier)
  // into the slot of plane k - 3 and request plane k + 5; red update of
  // plane k + 1 (reads planes k .. k + 2, writes the red cells of plane
  // k + 1) and black update of plane k - 1 (reads planes k - 2 .. k, stores
  // plane k - 1) in the same phase: they touch disjoint planes, so one
  // barrier per step suffices. Both updates are computed every step; their
  // LDS write and store are skipped where the plane is not this block's.
#define ZQ_STEP(P, kk)                                                                  \
  {                                                                                     \
    const int k = (kk);                                                                 \
    ZQ_STORE(X##P, k + 3, sP3);                                                         \
    ZQ_LOADX(X##P, min(k + 5, z1 + 1), );                                               \
    const int kr = k + 1, kb = k - 1;                                                   \
    const bool zr = kr > 0 && kr < nz - 1, zb = kb > 0 && kb < nz - 1;                  \
    /* every LDS read of the step first (one latency for both updates) */               \
    Q* vr = V[sP1];                                                                     \
    const Q *vrm = V[sP0], *vrp = V[sP2], *vb = V[sM1], *vbm = V[sM2], *vbp = V[sP0];   \
    const Q rc = vr[qi], rs = vr[qi - PQ], rn = vr[qi + PQ], rd = vrm[qi], ru = vrp[qi]; \
    const Q bc = vb[qi], bs = vb[qi - PQ], bn = vb[qi + PQ], bd = vbm[qi], bu = vbp[qi]; \
    const T rl = ((const T*)vr)[4 * qi - 1], rr = ((const T*)vr)[4 * qi + 4];          \
    const T bl = ((const T*)vb)[4 * qi - 1], br = ((const T*)vb)[4 * qi + 4];          \
    /* the ring's red cell (computed by every thread, written by ring threads) */      \
    const bool sa = ((rpar + kr) & 1) == 0;                                             \
    const int l = rg ? (sa ? rla : rlb) : 4 * qi;                                       \
    T* vrf = (T*)vr;                                                                    \
    const T gw = vrf[l - 1], ge = vrf[l + 1], gs = vrf[l - PW], gn = vrf[l + PW];       \
    const T gd = ((const T*)vrm)[l], gu = ((const T*)vrp)[l];                           \
    T c[4], s[4], n[4], d[4], u[4], bq[4], e[4], f[4], g[4], m[4], o[4], bk[4];         \
    _Pragma("unroll") for (int i = 0; i < 4; ++i) {                                     \
      c[i] = rc[i]; s[i] = rs[i]; n[i] = rn[i]; d[i] = rd[i]; u[i] = ru[i];             \
      bq[i] = BR##P[i];                                                                 \
      e[i] = bc[i]; f[i] = bs[i]; g[i] = bn[i]; m[i] = bd[i]; o[i] = bu[i];             \
      bk[i] = BK##P[i];                                                                 \
    }                                                                                   \
    /* red cells of plane kr are h, h + 2; black cells of plane kb the others */        \
    if (((hrow + kr) & 1) == 0) {                                                       \
      zq_pair<T, 0>(c, s, n, d, u, rl, rr, TR##P, bq, rq, TC, zr, gx0, gy, kr, nx, ny, nz); \
      zq_pair<T, 1>(e, f, g, m, o, bl, br, TK##P, bk, rq, TC, zb, gx0, gy, kb, nx, ny, nz); \
    } else {                                                                            \
      zq_pair<T, 1>(c, s, n, d, u, rl, rr, TR##P, bq, rq, TC, zr, gx0, gy, kr, nx, ny, nz); \
      zq_pair<T, 0>(e, f, g, m, o, bl, br, TK##P, bk, rq, TC, zb, gx0, gy, kb, nx, ny, nz); \
    }                                                                                   \
    {                                                                                   \
      const int cls = (int)(RT##P & 3);                                                 \
      const int p = cls & 1;                                                            \
      T v;                                                                              \
      if (zr) {                                                                         \
        const T r = sa ? (p ? ra1 : ra0) : (p ? rb1 : rb0);                             \
        v = zv_inner<T>(gw, ge, gs, gn, gd, gu, TC[p][0], RB##P, r);                    \
      } else {                                                                          \
        v = zv_general<T>(gw, ge, gs, gn, gd, gu, x0 + l % PW - 4, y0 + l / PW - 2, kr, nx, ny, nz, TC[p], \
                          RB##P);                                                       \
      }                                                                                 \
      const bool dored = kr >= 0 && kr < nz && kr <= z1;                                \
      if (dored && (sa ? ina : inb) && cls <= 1) vrf[l] = v;                            \
      if (dored && qin) vr[qi] = Q{c[0], c[1], c[2], c[3]};                             \
    }                                                                                   \
    if (kb >= z0 && kb < z1 && qin)                                                     \
      *(Q*)((char*)xout + ((uint32_t)sxy * (uint32_t)kb + (uint32_t)qoff) * (uint32_t)sizeof(T)) = \
          Q{e[0], e[1], e[2], e[3]};                                                    \
    ZQ_LOADK(P, min(k + 1, z1 + 1));                                                    \
    ZQ_LOADBT(P, min(k + 3, z1 + 1), );                                                 \
    __syncthreads();                                                                    \
    {                                                                                   \
      const int t6_ = sM2;                                                              \
      sM2 = sM1;                                                                        \
      sM1 = sP0;                                                                        \
      sP0 = sP1;                                                                        \
      sP1 = sP2;                                                                        \
      sP2 = sP3;                                                                        \
      sP3 = t6_;                                                                        \
    }                                                                                   \
  }

  // LDS ring of six plane slots: plane p lives in V[(p + 12) % 6]; the
  // slots of the planes k - 2 .. k + 3 around step k rotate in scalars
  int sM2 = (z0 - 4 + 12) % 6, sM1 = (z0 - 3 + 12) % 6, sP0 = (z0 - 2 + 12) % 6, sP1 = (z0 - 1 + 12) % 6,
      sP2 = (z0 + 12) % 6, sP3 = (z0 + 1 + 12) % 6;
  ZQ_LOADX(XA, z0 - 2, );
  ZQ_STORE(XA, z0 - 2, (z0 - 2 + 12) % 6);
  ZQ_LOADX(XA, z0 - 1, );
  ZQ_STORE(XA, z0 - 1, (z0 - 1 + 12) % 6);
  ZQ_LOADX(XA, z0, );
  ZQ_STORE(XA, z0, (z0 + 12) % 6);
  // the planes in flight at the loop head, requested in the loop's own
  // order (volatile reads keep it): as a step of A, x of z0+1 and the red
  // words of z0-1; as a step of B, x of z0+2 and the red words of z0;
  // otherwise the wait counts at the loop head would drain every load in
  // flight
  ZQ_LOADX(XA, z0 + 1, volatile);
  ZQ_LOADBT(A, z0 - 1, volatile);
  ZQ_LOADX(XB, z0 + 2, volatile);
  ZQ_LOADBT(B, z0, volatile);
  BKA = Q(0);   // (black words of planes before z0: computed on, never stored)
  TKA = 0;
  BKB = Q(0);
  TKB = 0;
  __syncthreads();
  // steps k = z0 - 2 .. z1: red planes z0 - 1 .. z1, black planes z0 .. z1 - 1
  int kq = z0 - 2;
  for (; kq + 1 <= z1; kq += 2) {
    ZQ_STEP(A, kq);
    ZQ_STEP(B, kq + 1);
  }
  if (kq <= z1) ZQ_STEP(A, kq);
#undef ZQ_STEP
#undef ZQ_STORE
#undef ZQ_LOADK
#undef ZQ_LOADBT
#undef ZQ_LOADX
#undef ZQ_AT
  // second-phase unknowns are not touched by this sweep: copy them through
  const int64_t N = sxy * nz;
  for (int64_t q = (int64_t)blockIdx.x * NT + tid; q < nsec; q += nblocks * NT) xout[N + q] = ZIN ? T(0) : xin[N + q];
}

// Quad form of k_resid_restrict3 (x extent a multiple of 4, arrays aligned
// to four values): each lane takes four consecutive cells of a row (x, b and
// the row neighbours as 4-element vectors, the tags as one 32-bit word, the
// two coarse cells' tags as one 16-bit word), a wavefront 32 quads of two
// neighbouring rows (lanes 0-31 and 32-63), so the 2 x 2 groups of children
// are two coarse cells per lane pair, summed in-lane along x and by one
// shuffle along y, in the same order as k_resid_restrict3; the residual of
// each template child is formed with the same arithmetic. Tiles of kRQX x
// (2 kRRW) columns over zc planes, one plane requested ahead.
constexpr int kRQX = 128;

template <typename T>
__global__ void __launch_bounds__(64 * kRRW) k_resid_restrict3q(const uint8_t* __restrict__ tag,
                                                                const T* __restrict__ x, const T* __restrict__ b,
                                                                T* __restrict__ r, const uint8_t* __restrict__ ctag,
                                                                T* __restrict__ bc, Tmpl<T> tp, int zc) {
  typedef T Q __attribute__((ext_vector_type(4)));
  __shared__ T TC[2][8];
  const int tid = threadIdx.x + 64 * threadIdx.y;
  if (tid < 16) {
    const int p = tid >> 3, j = tid & 7;
    TC[p][j] = j == 0 ? tp.coff[p] : (j == 1 ? tp.mass[p] : tp.cbm[j - 2][p]);
  }
  __syncthreads();
  const int nx = tp.n[0], ny = tp.n[1], nz = tp.n[2];
  const int cnx = nx >> 1, cny = ny >> 1;
  const int gbx = (nx + kRQX - 1) / kRQX, gby = (ny + 2 * kRRW - 1) / (2 * kRRW);
  const int64_t tt = xcd_block(blockIdx.x, gridDim.x);
  const int lane = threadIdx.x;
  const int i = (int)(tt % gbx) * kRQX + 4 * (lane & 31);
  const int j = (int)((tt / gbx) % gby) * (2 * kRRW) + 2 * threadIdx.y + (lane >> 5);
  const int z0 = (int)(tt / ((int64_t)gbx * gby)) * zc, z1 = min(z0 + zc, nz);
  // lanes past the box edge load a valid cell, take part in the shuffles and
  // write nothing (a quad and its 2 x 2 groups are all in or all out)
  const bool act = i < nx && j < ny;
  const int ic = act ? i : 0, jc = act ? j : 0;
  const bool lead = act && lane < 32;
  const int64_t sxy = (int64_t)nx * ny;
  const int64_t c0 = ic + (int64_t)nx * jc;
  const int64_t ow = ic > 0 ? -1 : 0, oe = ic + 4 < nx ? 4 : 3;
  const int64_t os = jc > 0 ? -(int64_t)nx : 0, on = jc < ny - 1 ? (int64_t)nx : 0;
  const int64_t P0 = (ic >> 1) + (int64_t)cnx * (jc >> 1);
  const int64_t csxy = (int64_t)cnx * cny;
  const Q zq = {T(0), T(0), T(0), T(0)};
  Q xm = z0 > 0 ? *(const Q*)(x + c0 + sxy * (z0 - 1)) : zq;
  int64_t c = c0 + sxy * z0;
  Q xc = *(const Q*)(x + c);
  Q xp = z0 + 1 < nz ? *(const Q*)(x + c + sxy) : zq;
  T w = x[c + ow], e = x[c + oe];
  Q so = *(const Q*)(x + c + os), no = *(const Q*)(x + c + on);
  uint32_t tg = *(const uint32_t*)(tag + c);
  Q bb = *(const Q*)(b + c);
  uint32_t ct = *(const uint16_t*)(ctag + P0 + csxy * (z0 >> 1));
  T accA = 0, accB = 0;
  for (int k = z0; k < z1; ++k, c += sxy) {
    const bool more = k + 1 < z1;
    const int64_t cn = more ? c + sxy : c;
    const Q xpp = k + 2 < nz ? *(const Q*)(x + c + 2 * sxy) : zq;
    const T wn = x[cn + ow], en = x[cn + oe];
    const Q son = *(const Q*)(x + cn + os), non = *(const Q*)(x + cn + on);
    const uint32_t tgn = more ? *(const uint32_t*)(tag + cn) : 0x03030303u;
    const Q bbn = more ? *(const Q*)(b + cn) : zq;
    const uint32_t ctn = more ? (uint32_t)*(const uint16_t*)(ctag + P0 + csxy * ((k + 1) >> 1)) : 0x0303u;
    T out[4], up[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int p = tclass((uint8_t)(tg >> (8 * u)));
      const uint8_t cu = (uint8_t)(ct >> (8 * (u >> 1)));   // the coarse cell of child u
      if (p == 2) {
        out[u] = r[c + u];   // an explicit row: its residual is already there
      } else if (p == 3) {
        out[u] = T(0);
      } else {
        const T xv = xc[u];
        const T wv = u ? xc[u > 0 ? u - 1 : 0] : w, ev = u < 3 ? xc[u < 3 ? u + 1 : 3] : e;
        const T* tc = TC[p];
        T sm = 0, dg = tc[1];
        if (ic + u > 0) sm += wv - xv; else dg += tc[2];
        if (ic + u < nx - 1) sm += ev - xv; else dg += tc[3];
        if (jc > 0) sm += so[u] - xv; else dg += tc[4];
        if (jc < ny - 1) sm += no[u] - xv; else dg += tc[5];
        if (k > 0) sm += xm[u] - xv; else dg += tc[6];
        if (k < nz - 1) sm += xp[u] - xv; else dg += tc[7];
        const T ax = dg * xv + tc[0] * sm;
        out[u] = bb[u] - ax;
      }
      // the children of a non-simple coarse unknown keep their residual for
      // the list restriction that follows
      if (act && p != 2 && (cu & 4) && tclass(cu) != 3) r[c + u] = out[u];
      up[u] = __shfl_xor(out[u], 32, 64);
    }
    if (lead) {
      const T pkA = ((out[0] + out[1]) + up[0]) + up[1];
      const T pkB = ((out[2] + out[3]) + up[2]) + up[3];
      if ((k & 1) == 0) {
        accA = pkA;
        accB = pkB;
      } else {
        const int64_t P = P0 + csxy * (k >> 1);
        const uint8_t ca = (uint8_t)ct, cb = (uint8_t)(ct >> 8);
        if (tclass(ca) == 3)
          bc[P] = T(0);
        else if (!(ca & 4))
          bc[P] = (accA + pkA) * T(0.125);
        if (tclass(cb) == 3)
          bc[P + 1] = T(0);
        else if (!(cb & 4))
          bc[P + 1] = (accB + pkB) * T(0.125);
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

// Reference stream for the measurement hook: the fused sweep's bytes per
// cell with no stencil (reads x, b and the tag of every cell, writes one
// value per cell), four cells per thread in 16-byte accesses; n a multiple
// of 4 and the arrays aligned to 4 values (checked by the caller).
template <typename T>
__global__ void __launch_bounds__(256) k_stream_ref(const uint8_t* __restrict__ tag, const T* __restrict__ x,
                                                    const T* __restrict__ b, T* __restrict__ y, int64_t n) {
  typedef T Q __attribute__((ext_vector_type(4)));
  const int64_t n4 = n / 4;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n4; i += (int64_t)gridDim.x * 256) {
    const Q xv = ((const Q*)x)[i], bv = ((const Q*)b)[i];
    const uint32_t tv = ((const uint32_t*)tag)[i];
    Q r;
#pragma unroll
    for (int e = 0; e < 4; ++e) r[e] = xv[e] + bv[e] * (T)((tv >> (8 * e)) & 3u);
    ((Q*)y)[i] = r;
  }
}

}  // namespace ebmg
