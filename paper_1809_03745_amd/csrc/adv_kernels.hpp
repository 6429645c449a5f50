// One explicit advection step of a density on the gas phase of a cut-cell
// grid (Convection-Diffusion-Reaction equations: Advective discretization,
// Hybrid divergence), FP64:
//   k_adv_zm       (3D) the two launches below fused into one z-marching
//                  pass over the box;
//   k_adv_flux     face-centred fluxes u n_f of one direction, n_f the
//                  upwind state of an unsplit Godunov predictor with
//                  monotonised-central (van Leer) slopes, extrapolated to the
//                  face and to the half step including the transverse terms;
//                  inflow domain faces take the boundary density;
//   k_adv_full     full cells (every face full: the centroid fluxes are the
//                  face-centred ones): conservative divergence and
//                  n_out = n - dt D^c; 0 where there is no gas;
//   k_adv_dc_cut   conservative divergence of cut cells from their
//                  precomputed forms over the face fluxes (apertures,
//                  centroid interpolation, 1 / (kappa h));
//   k_adv_cut      per cut cell: the non-conservative divergence (kappa-
//                  weighted mean over its 3^D block), the hybrid
//                  kappa D^c + (1 - kappa) D^nc, and the rate change
//                  dM / S its mass defect dM = kappa (1 - kappa)(D^nc - D^c)
//                  gives every other gas cell of its block;
//   k_adv_special  cut cells and the cells receiving redistributed mass:
//                  n_out = n - dt (their hybrid or D^c, less what they
//                  receive), overwriting the previous launch's value.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kernels.hpp"

namespace ebmg {

struct AdvGrid {
  int n[3];
  int dim;
  int64_t fbase[3];
  double h, dt;
  double inflow[6];
};

__device__ __forceinline__ double adv_mc(double dl, double dr) {
  if (!(dl * dr > 0.0)) return 0.0;
  const double dc = 0.5 * (dl + dr);
  const double m = fmin(fmin(2.0 * fabs(dl), 2.0 * fabs(dr)), fabs(dc));
  return dc > 0.0 ? m : -m;
}

template <int DIM>
__device__ __forceinline__ bool adv_gas(const uint8_t* __restrict__ cls, const AdvGrid& G, int i, int j, int k) {
  if (i < 0 || i >= G.n[0] || j < 0 || j >= G.n[1]) return false;
  if (DIM == 3 && (k < 0 || k >= G.n[2])) return false;
  return cls[i + (int64_t)G.n[0] * (j + (int64_t)G.n[1] * k)] != 0;
}

// slope of cell (i, j, k) along e (0 without gas on both sides)
template <int DIM>
__device__ __forceinline__ double adv_slope(const double* __restrict__ n, const uint8_t* __restrict__ cls,
                                            const AdvGrid& G, int i, int j, int k, int e) {
  const int di = e == 0, dj = e == 1, dk = e == 2;
  if (!adv_gas<DIM>(cls, G, i - di, j - dj, k - dk) || !adv_gas<DIM>(cls, G, i + di, j + dj, k + dk)) return 0.0;
  const int64_t sx = 1, sy = G.n[0], sz = (int64_t)G.n[0] * G.n[1];
  const int64_t c = i + sy * j + sz * k;
  const int64_t st = e == 0 ? sx : (e == 1 ? sy : sz);
  const double nc = n[c];
  return adv_mc(nc - n[c - st], n[c + st] - nc);
}

// face velocity of direction e at face index (fi, fj, fk)
template <int DIM>
__device__ __forceinline__ double adv_u(const double* const* u, const AdvGrid& G, int e, int fi, int fj, int fk) {
  const int64_t m0 = G.n[0] + (e == 0), m1 = G.n[1] + (e == 1);
  return u[e][fi + m0 * (fj + m1 * (int64_t)fk)];
}

struct AdvVel {
  const double* u[3];
};

// flux u n_f through face (fi, fj, fk) of direction DIR (face index along
// DIR = the index of its high cell), read from global memory
template <int DIM, int DIR>
__device__ __forceinline__ double adv_face_flux(const double* __restrict__ n, const uint8_t* __restrict__ cls,
                                                const AdvVel& vel, const AdvGrid& G, int fi, int fj, int fk) {
  const int m0 = G.n[0] + (DIR == 0), m1 = G.n[1] + (DIR == 1);
  const int64_t fl = fi + (int64_t)m0 * (fj + (int64_t)m1 * fk);
  const int fc[3] = {fi, fj, fk};
  const double u = vel.u[DIR][fl];
  const double h = G.h, dt = G.dt;
  const bool up_lo = u >= 0.0;
  // the upwind cell: the low one (face on its high side) or the high one
  int c[3] = {fi, fj, fk};
  if (up_lo) c[DIR] -= 1;
  const bool outside = up_lo ? fc[DIR] == 0 : fc[DIR] == G.n[DIR];
  if (outside) return u * G.inflow[2 * DIR + (up_lo ? 0 : 1)];
  if (!adv_gas<DIM>(cls, G, c[0], c[1], c[2])) return 0.0;
  const int64_t cc = c[0] + (int64_t)G.n[0] * (c[1] + (int64_t)G.n[1] * c[2]);
  double trans = 0.0;
#pragma unroll
  for (int e = 0; e < DIM; ++e) {
    if (e == DIR) continue;
    int hi[3] = {c[0], c[1], c[2]};
    hi[e] += 1;
    const double ve = 0.5 * (adv_u<DIM>(vel.u, G, e, c[0], c[1], c[2]) + adv_u<DIM>(vel.u, G, e, hi[0], hi[1], hi[2]));
    trans += ve * adv_slope<DIM>(n, cls, G, c[0], c[1], c[2], e);
  }
  const double base = n[cc] - 0.5 * dt / h * trans;
  const double sd = adv_slope<DIM>(n, cls, G, c[0], c[1], c[2], DIR);
  return u * (base + ((up_lo ? 0.5 : -0.5) - u * dt / (2.0 * h)) * sd);
}

// one direction's face fluxes: thread = face of one z plane (x fastest),
// blockIdx.y = the face's z index; F is that direction's face array
template <int DIM, int DIR>
__global__ void __launch_bounds__(256) k_adv_flux(const double* __restrict__ n, const uint8_t* __restrict__ cls,
                                                  AdvVel vel, AdvGrid G, double* __restrict__ F) {
  const unsigned m0 = G.n[0] + (DIR == 0), m1 = G.n[1] + (DIR == 1);
  const unsigned f2 = blockIdx.x * 256u + threadIdx.x;
  if (f2 >= m0 * m1) return;
  const int fk = DIM == 3 ? (int)blockIdx.y : 0;
  F[f2 + (int64_t)m0 * m1 * fk] = adv_face_flux<DIM, DIR>(n, cls, vel, G, (int)(f2 % m0), (int)(f2 / m0), fk);
}

// cells with every face full (class 1, or 3 when a cut cell's block needs
// their D^c): n_out = n - dt D^c; cells without gas get 0; cut cells are
// left to the cut-cell launches. Thread = cell of one z plane.
template <int DIM>
__global__ void __launch_bounds__(256) k_adv_full(const uint8_t* __restrict__ cls, AdvGrid G,
                                                  const double* __restrict__ F, const double* __restrict__ n,
                                                  double* __restrict__ Dc, double* __restrict__ nout) {
  const unsigned nx = G.n[0], ny = G.n[1];
  const unsigned c2 = blockIdx.x * 256u + threadIdx.x;
  if (c2 >= nx * ny) return;
  const int k = DIM == 3 ? (int)blockIdx.y : 0;
  const int64_t c = c2 + (int64_t)nx * ny * k;
  const uint8_t t = cls[c];
  if (t == 2) return;
  if (t == 0) {
    nout[c] = 0.0;
    return;
  }
  const int i = (int)(c2 % nx), j = (int)(c2 / nx);
  double net = 0.0;
#pragma unroll
  for (int d = 0; d < DIM; ++d) {
    const int64_t m0 = nx + (d == 0), m1 = ny + (d == 1);
    const int64_t lo = G.fbase[d] + i + m0 * (j + m1 * (int64_t)k);
    const int64_t st = d == 0 ? 1 : (d == 1 ? m0 : m0 * m1);
    net += F[lo + st] - F[lo];
  }
  const double dc = net / G.h;
  if (t == 3) Dc[c] = dc;
  nout[c] = n[c] - G.dt * dc;
}

__global__ void __launch_bounds__(256) k_adv_dc_cut(int ncut, const int64_t* __restrict__ cell,
                                                    const int64_t* __restrict__ ptr, const int64_t* __restrict__ face,
                                                    const double* __restrict__ coef, const double* __restrict__ F,
                                                    double* __restrict__ Dc) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= ncut) return;
  double s = 0.0;
  for (int64_t e = ptr[q]; e < ptr[q + 1]; ++e) s += coef[e] * F[face[e]];
  Dc[cell[q]] = s;
}

__global__ void __launch_bounds__(256) k_adv_cut(int ncut, const int64_t* __restrict__ cell,
                                                 const double* __restrict__ kappa, const int64_t* __restrict__ ptr,
                                                 const int64_t* __restrict__ nbc, const double* __restrict__ nbw,
                                                 const double* __restrict__ S, const double* __restrict__ Dc,
                                                 double* __restrict__ Dcut, double* __restrict__ give) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= ncut) return;
  const int64_t c = cell[q];
  const double dc = Dc[c];
  if (!(S[q] > 0.0)) {   // no gas neighbour: the conservative divergence stays
    Dcut[q] = dc;
    give[q] = 0.0;
    return;
  }
  double dnc = 0.0;
  for (int64_t e = ptr[q]; e < ptr[q + 1]; ++e) dnc += nbw[e] * Dc[nbc[e]];
  const double k = kappa[c];
  Dcut[q] = k * dc + (1.0 - k) * dnc;
  give[q] = k * (1.0 - k) * (dnc - dc) / S[q];
}

__global__ void __launch_bounds__(256) k_adv_special(int nsp, const int64_t* __restrict__ cell,
                                                     const int32_t* __restrict__ cut, const int64_t* __restrict__ ptr,
                                                     const int32_t* __restrict__ donor, double dt,
                                                     const double* __restrict__ n, const double* __restrict__ Dc,
                                                     const double* __restrict__ Dcut, const double* __restrict__ give,
                                                     double* __restrict__ nout) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= nsp) return;
  const int64_t c = cell[s];
  double D = cut[s] >= 0 ? Dcut[cut[s]] : Dc[c];
  for (int64_t e = ptr[s]; e < ptr[s + 1]; ++e) D -= give[donor[e]];
  nout[c] = n[c] - dt * D;
}


// The whole full-cell step in one pass over the box (3D): a block owns a
// TX x TY column tile and marches up a chunk of ZC planes, keeping five planes
// of n and of the cell class (k - 1 .. k + 3, with a two-cell x/y halo) in an
// LDS ring. At plane k each thread takes its cell's slopes at k + 1 (carried
// to the next step), publishes the extrapolation bases and normal slopes of
// its cell at k for the x and y faces, the halo threads add those of the
// cells just outside the tile, and then every thread forms the six face
// fluxes of its cell (the z faces from its own column: the low one is the
// previous step's high one), its conservative divergence and n_out. The
// ring plane k + 4 and the own column's face velocities at k + 2 are loaded
// a step before they are needed, so their latency overlaps a step of
// arithmetic (the halo cells' few velocities are loaded in the step); the
// register budget is held to four waves per SIMD. Cut cells (class 2) only get their
// face fluxes stored (the cut-cell launches finish them); cells of class 2
// or 3 store all six fluxes into F for the cut-cell forms, class 3 also its
// D^c. Per face the arithmetic is that of adv_face_flux, up to contraction
// of the transverse sums.
template <int TX, int TY, int ZC>
__global__ void __launch_bounds__(TX * TY, 2) k_adv_zm(const double* __restrict__ n, const uint8_t* __restrict__ cls,
                                                    AdvVel vel, AdvGrid G, int tiles_x, int tiles_y,
                                                    double* __restrict__ F, double* __restrict__ Dc,
                                                    double* __restrict__ nout) {
  constexpr int RX = TX + 4, RY = TY + 4, RP = RX * RY, NT = TX * TY;
  constexpr int NR = (RP + NT - 1) / NT;   // ring elements per thread and plane
  constexpr int NH = 2 * TY + 2 * TX;      // halo cells
  static_assert(NH <= NT, "one halo cell per thread");
  __shared__ double rn[5][RP];
  __shared__ uint8_t rc[5][RP];
  // per step parity: columns i0 - 1 .. i0 + TX of the tile's rows (x faces),
  // rows j0 - 1 .. j0 + TY of its columns (y faces)
  __shared__ double bx[2][TY][TX + 2], sxs[2][TY][TX + 2];
  __shared__ double by[2][TY + 2][TX], sys[2][TY + 2][TX];
  // every array offset fits in 32 bits (checked by the host)
  const int nx = G.n[0], ny = G.n[1], nz = G.n[2];
  const unsigned sxy = (unsigned)nx * ny;              // plane stride of cells and z faces
  const unsigned sfx = (unsigned)(nx + 1) * ny;        // plane stride of x faces
  const unsigned sfy = (unsigned)nx * (ny + 1);        // plane stride of y faces
  const int64_t t = xcd_block(blockIdx.x, gridDim.x);
  const int tpc = tiles_x * tiles_y;
  const int zc = (int)(t / tpc), r = (int)(t % tpc);
  const int i0 = (r % tiles_x) * TX, j0 = (r / tiles_x) * TY;
  const int z0 = zc * ZC, z1 = min(nz, z0 + ZC);
  const int tx = threadIdx.x % TX, ty = threadIdx.x / TX;
  const int i = i0 + tx, j = j0 + ty;
  const bool own = i < nx && j < ny;
  const double h = G.h, dt = G.dt, c1 = 0.5 * dt / h, c2 = dt / (2.0 * h), rh = 1.0 / h;
  const double* __restrict__ ux = vel.u[0];
  const double* __restrict__ uy = vel.u[1];
  const double* __restrict__ uz = vel.u[2];
  // in-plane offsets: of the ring elements this thread fetches (-1: no cell),
  // of the own cell's low x, y and z faces and cell
  int roff[NR];
#pragma unroll
  for (int q = 0; q < NR; ++q) {
    const int e = threadIdx.x + q * NT;
    const int gi = i0 - 2 + e % RX, gj = j0 - 2 + e / RX;
    roff[q] = (e < RP && gi >= 0 && gi < nx && gj >= 0 && gj < ny) ? gi + nx * gj : -1;
  }
  const unsigned ofx = (unsigned)i + (unsigned)(nx + 1) * j, ofy = (unsigned)i + (unsigned)nx * j;
  const unsigned oc = ofy;   // cells and z faces share the in-plane layout
  // ring plane k: fetched into registers one step ahead, stored later. The
  // class and the density are requested together (a lane outside the box
  // reads cell 0 and discards it), and the rule "no gas: NaN" is applied
  // when the plane is stored, so no load waits for another.
  double pv[NR];
  uint8_t pc[NR];
  uint32_t pin = 0;   // bit q: element q lies in the box and in a plane of it
  auto fetch_plane = [&](int k) {
    const bool kin = k >= 0 && k < nz;
    const double* __restrict__ pn = n + (kin ? (int64_t)sxy * k : 0);
    const uint8_t* __restrict__ pcl = cls + (kin ? (int64_t)sxy * k : 0);
    pin = 0;
#pragma unroll
    for (int q = 0; q < NR; ++q) {
      const unsigned o = roff[q] >= 0 ? (unsigned)roff[q] : 0u;
      pc[q] = pcl[o];
      pv[q] = pn[o];
      pin |= (uint32_t)(kin && roff[q] >= 0) << q;
    }
  };
  auto slot = [](int k) { return (k + 5) % 5; };   // k >= -1
  auto store_plane = [&](int k) {
    const int sl = slot(k);
#pragma unroll
    for (int q = 0; q < NR; ++q) {
      const int e = threadIdx.x + q * NT;
      if (e < RP) {
        const uint8_t c = ((pin >> q) & 1) ? pc[q] : (uint8_t)0;
        rn[sl][e] = c ? pv[q] : __builtin_nan("");
        rc[sl][e] = c;
      }
    }
  };
  // monotonised-central slopes of ring cell e at plane k: the ring holds
  // NaN where there is no gas (or no cell), and adv_mc returns 0 for a NaN
  // difference, which is the rule of a slope without gas on both sides
  auto slopes = [&](int k, int e, double& sx, double& sy, double& sz) {
    const int sm = slot(k - 1), sc = slot(k), sp = slot(k + 1);
    const double c = rn[sc][e];
    sx = adv_mc(c - rn[sc][e - 1], rn[sc][e + 1] - c);
    sy = adv_mc(c - rn[sc][e - RX], rn[sc][e + RX] - c);
    sz = adv_mc(c - rn[sm][e], rn[sp][e] - c);
  };
  // this thread's halo cell (if any): columns i0 - 1 and i0 + TX of the
  // tile's rows (x faces), rows j0 - 1 and j0 + TY of its columns (y faces)
  const int hq = threadIdx.x;
  const bool has_halo = hq < NH;
  const bool isx = hq < 2 * TY;
  const int hx = isx ? ((hq & 1) ? TX : -1) : (hq - 2 * TY) % TX;
  const int hy = isx ? (hq >> 1) : (((hq - 2 * TY) / TX) ? TY : -1);
  const int hgi = i0 + hx, hgj = j0 + hy;
  const bool hin = has_halo && hgi >= 0 && hgi < nx && hgj >= 0 && hgj < ny;
  const int he = (hy + 2) * RX + (hx + 2);
  const unsigned hoz = hin ? (unsigned)hgi + (unsigned)nx * hgj : 0u;
  const unsigned hot = hin ? (isx ? hoz : (unsigned)hgi + (unsigned)(nx + 1) * hgj) : 0u;
  // halo velocities at a plane: the z faces, then the in-plane transverse faces
  // (requested unconditionally, a plane past the box clamped to the last
  // one and a lane without a halo cell reading face 0, so that the compiler
  // counts every load and never waits for more than the value it needs)
  auto fetch_halo = [&](int k, double& z0v, double& z1v, double& t0v, double& t1v) {
    const int kk = k < nz ? k : nz - 1;
    const double* __restrict__ pz = uz + (int64_t)sxy * kk;
    z0v = pz[hoz];
    z1v = pz[hoz + sxy];
    const double* __restrict__ pt = isx ? uy + (int64_t)sfy * kk : ux + (int64_t)sfx * kk;
    t0v = pt[hot];
    t1v = pt[hot + (isx ? (unsigned)nx : 1u)];
  };
  // own column: face velocities of the cell at a plane (requested the same way)
  const unsigned ofxo = own ? ofx : 0u, ofyo = own ? ofy : 0u, oco = own ? oc : 0u;
  auto fetch_own = [&](int k, double& xl, double& xh, double& yl, double& yh, double& zh) {
    const int kk = k < nz ? k : nz - 1;
    const double* __restrict__ px = ux + (int64_t)sfx * kk;
    const double* __restrict__ py = uy + (int64_t)sfy * kk;
    const double* __restrict__ pz = uz + (int64_t)sxy * (kk + 1);
    xl = px[ofxo];
    xh = px[ofxo + 1];
    yl = py[ofyo];
    yh = py[ofyo + nx];
    zh = pz[oco];
  };
  // inflow densities of the six domain faces, read once
  const double in0 = G.inflow[0], in1 = G.inflow[1], in2 = G.inflow[2], in3 = G.inflow[3], in5 = G.inflow[5];
  const int eo = (ty + 2) * RX + (tx + 2);
  double hz0 = 0, hz1 = 0, ht0 = 0, ht1 = 0;       // halo velocities of plane k
  double gz0 = 0, gz1 = 0, gt0 = 0, gt1 = 0;       // of plane k + 1 (requested a step ahead)
  double cuxl = 0, cuxh = 0, cuyl = 0, cuyh = 0, cuzl = 0, cuzh = 0;   // plane k
  double auxl = 0, auxh = 0, auyl = 0, auyh = 0, auzh = 0;             // plane k + 1
  fetch_plane(z0 - 1);
  store_plane(z0 - 1);
  fetch_plane(z0);
  store_plane(z0);
  fetch_plane(z0 + 1);
  store_plane(z0 + 1);
  fetch_plane(z0 + 2);
  store_plane(z0 + 2);
  fetch_plane(z0 + 3);
  fetch_own(z0, cuxl, cuxh, cuyl, cuyh, cuzh);
  fetch_own(z0 + 1, auxl, auxh, auyl, auyh, auzh);
  fetch_halo(z0, gz0, gz1, gt0, gt1);
  double fzl = 0.0;
  if (own) {
    cuzl = uz[(int64_t)sxy * z0 + oc];
    fzl = adv_face_flux<3, 2>(n, cls, vel, G, i, j, z0);
  }
  __syncthreads();
  double cn = 0, csx = 0, csy = 0, csz = 0;
  bool cg = false;
  if (own) {
    slopes(z0, eo, csx, csy, csz);
    cg = rc[slot(z0)][eo] != 0;
    cn = cg ? rn[slot(z0)][eo] : 0.0;
  }
  double* __restrict__ Fx = F + G.fbase[0];
  double* __restrict__ Fy = F + G.fbase[1];
  double* __restrict__ Fz = F + G.fbase[2];
  const int rrow = (ty + 2) * RX;
  // one barrier per plane: the ring runs three planes ahead (a plane is
  // stored a step before it is read) and the face bases alternate between
  // two buffers
  for (int k = z0; k < z1; ++k) {
    const int pb = k & 1;
    if (k + 3 <= z1 + 1) store_plane(k + 3);
    if (k + 4 <= z1 + 1) fetch_plane(k + 4);
    hz0 = gz0;
    hz1 = gz1;
    ht0 = gt0;
    ht1 = gt1;
    fetch_halo(k + 1, gz0, gz1, gt0, gt1);
    const int sk = slot(k);
    // the own cell at plane k + 1
    double nn = 0, nsx = 0, nsy = 0, nsz = 0;
    bool ng = false;
    if (own && k + 1 < nz) {
      slopes(k + 1, eo, nsx, nsy, nsz);
      ng = rc[slot(k + 1)][eo] != 0;
      nn = ng ? rn[slot(k + 1)][eo] : 0.0;
    }
    const double cvx = 0.5 * (cuxl + cuxh), cvy = 0.5 * (cuyl + cuyh), cvz = 0.5 * (cuzl + cuzh);
    if (own) {
      bx[pb][ty][tx + 1] = cn - c1 * (cvy * csy + cvz * csz);
      sxs[pb][ty][tx + 1] = csx;
      by[pb][ty + 1][tx] = cn - c1 * (cvx * csx + cvz * csz);
      sys[pb][ty + 1][tx] = csy;
    }
    if (has_halo) {
      double b = 0.0, sl = 0.0;
      if (hin) {
        double sx, sy, sz;
        slopes(k, he, sx, sy, sz);
        const double c = rn[sk][he];
        const double vz = 0.5 * (hz0 + hz1), vt = 0.5 * (ht0 + ht1);
        b = c - c1 * (vt * (isx ? sy : sx) + vz * sz);
        sl = isx ? sx : sy;
      }
      if (isx) {
        bx[pb][hy][hx + 1] = b;
        sxs[pb][hy][hx + 1] = sl;
      } else {
        by[pb][hy + 1][hx] = b;
        sys[pb][hy + 1][hx] = sl;
      }
    }
    __syncthreads();
    if (own) {
      // x faces i (low) and i + 1 (high); region column c <-> cell i0 - 1 + c
      auto xflux = [&](int f, double u) {
        const bool up = u >= 0.0;
        if (up ? f == 0 : f == nx) return u * (up ? in0 : in1);
        const int col = f - i0 + (up ? 0 : 1);
        if (!rc[sk][rrow + col + 1]) return 0.0;
        return u * (bx[pb][ty][col] + ((up ? 0.5 : -0.5) - u * c2) * sxs[pb][ty][col]);
      };
      auto yflux = [&](int f, double u) {
        const bool up = u >= 0.0;
        if (up ? f == 0 : f == ny) return u * (up ? in2 : in3);
        const int row = f - j0 + (up ? 0 : 1);
        if (!rc[sk][(row + 1) * RX + tx + 2]) return 0.0;
        return u * (by[pb][row][tx] + ((up ? 0.5 : -0.5) - u * c2) * sys[pb][row][tx]);
      };
      const double fxl = xflux(i, cuxl), fxh = xflux(i + 1, cuxh);
      const double fyl = yflux(j, cuyl), fyh = yflux(j + 1, cuyh);
      // z face k + 1: from the own cell at k (upwind from below) or at k + 1
      double fzh;
      {
        const double u = cuzh;
        const bool up = u >= 0.0;
        if (!up && k + 1 == nz) {
          fzh = u * in5;
        } else if (up) {
          fzh = cg ? u * ((cn - c1 * (cvx * csx + cvy * csy)) + (0.5 - u * c2) * csz) : 0.0;
        } else {
          const double nvx = 0.5 * (auxl + auxh), nvy = 0.5 * (auyl + auyh);
          fzh = ng ? u * ((nn - c1 * (nvx * nsx + nvy * nsy)) + (-0.5 - u * c2) * nsz) : 0.0;
        }
      }
      const unsigned q = oc + sxy * (unsigned)k;
      const uint8_t tc = rc[sk][eo];
      if (tc == 0) {
        nout[q] = 0.0;
      } else if (tc != 2) {
        const double dc = ((fxh - fxl) + (fyh - fyl) + (fzh - fzl)) * rh;
        if (tc == 3) Dc[q] = dc;
        nout[q] = cn - dt * dc;
      }
      if (tc >= 2) {
        const unsigned qx = ofx + sfx * (unsigned)k, qy = ofy + sfy * (unsigned)k;
        Fx[qx] = fxl;
        Fx[qx + 1] = fxh;
        Fy[qy] = fyl;
        Fy[qy + nx] = fyh;
        Fz[q] = fzl;
        Fz[q + sxy] = fzh;
      }
      fzl = fzh;
    }
    cn = nn; csx = nsx; csy = nsy; csz = nsz; cg = ng;
    cuxl = auxl; cuxh = auxh; cuyl = auyl; cuyh = auyh; cuzl = cuzh; cuzh = auzh;
    fetch_own(k + 2, auxl, auxh, auyl, auyh, auzh);
  }
}

}  // namespace ebmg
