// One explicit advection step of a density on the gas phase of a cut-cell
// grid (Convection-Diffusion-Reaction equations: Advective discretization,
// Hybrid divergence), FP64:
//   k_adv_faces    face-centred fluxes u n_f, n_f the upwind state of an
//                  unsplit Godunov predictor with monotonised-central (van
//                  Leer) slopes, extrapolated to the face and to the half
//                  step including the transverse terms; inflow domain faces
//                  take the boundary density;
//   k_adv_dc_full  conservative divergence of full cells (every face full:
//                  the centroid fluxes are the face-centred ones);
//   k_adv_dc_cut   conservative divergence of cut cells from their
//                  precomputed forms over the face fluxes (apertures,
//                  centroid interpolation, 1 / (kappa h));
//   k_adv_cut      per cut cell: the non-conservative divergence (kappa-
//                  weighted mean over its 3^D block), the hybrid
//                  kappa D^c + (1 - kappa) D^nc, and the rate change
//                  dM / S its mass defect dM = kappa (1 - kappa)(D^nc - D^c)
//                  gives every other gas cell of its block;
//   k_adv_update   n_out = n - dt D^c everywhere with gas (0 elsewhere);
//   k_adv_special  cut cells and the cells receiving redistributed mass:
//                  n_out = n - dt (their hybrid or D^c, less what they
//                  receive), overwriting the previous launch's value.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

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

template <int DIM>
__global__ void __launch_bounds__(256) k_adv_faces(const double* __restrict__ n, const uint8_t* __restrict__ cls,
                                                   AdvVel vel, AdvGrid G, int64_t nfaces, double* __restrict__ F) {
  const int64_t f = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= nfaces) return;
  const int d = (DIM == 3 && f >= G.fbase[2]) ? 2 : (f >= G.fbase[1] ? 1 : 0);
  const int64_t fl = f - G.fbase[d];
  const int64_t m0 = G.n[0] + (d == 0), m1 = G.n[1] + (d == 1);
  const int fi = (int)(fl % m0);
  const int64_t r = fl / m0;
  const int fj = (int)(r % m1), fk = DIM == 3 ? (int)(r / m1) : 0;
  const int fc[3] = {fi, fj, fk};
  const double u = vel.u[d][fl];
  const double h = G.h, dt = G.dt;
  double state;
  bool ok;
  const bool up_lo = u >= 0.0;
  // the upwind cell: the low one (face on its high side) or the high one
  int c[3] = {fi, fj, fk};
  if (up_lo) c[d] -= 1;
  const bool outside = up_lo ? fc[d] == 0 : fc[d] == G.n[d];
  if (outside) {
    state = G.inflow[2 * d + (up_lo ? 0 : 1)];
    ok = true;
  } else {
    ok = adv_gas<DIM>(cls, G, c[0], c[1], c[2]);
    state = 0.0;
    if (ok) {
      const int64_t cc = c[0] + (int64_t)G.n[0] * (c[1] + (int64_t)G.n[1] * c[2]);
      double trans = 0.0;
#pragma unroll
      for (int e = 0; e < DIM; ++e) {
        if (e == d) continue;
        const int lo[3] = {c[0], c[1], c[2]};
        int hi[3] = {c[0], c[1], c[2]};
        hi[e] += 1;
        const double ve = 0.5 * (adv_u<DIM>(vel.u, G, e, lo[0], lo[1], lo[2]) + adv_u<DIM>(vel.u, G, e, hi[0], hi[1], hi[2]));
        trans += ve * adv_slope<DIM>(n, cls, G, c[0], c[1], c[2], e);
      }
      const double base = n[cc] - 0.5 * dt / h * trans;
      const double sd = adv_slope<DIM>(n, cls, G, c[0], c[1], c[2], d);
      state = base + ((up_lo ? 0.5 : -0.5) - u * dt / (2.0 * h)) * sd;
    }
  }
  F[f] = ok ? u * state : 0.0;
}

template <int DIM>
__global__ void __launch_bounds__(256) k_adv_dc_full(const uint8_t* __restrict__ cls, AdvGrid G,
                                                     const double* __restrict__ F, double* __restrict__ Dc) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t N = (int64_t)G.n[0] * G.n[1] * (DIM == 3 ? G.n[2] : 1);
  if (c >= N) return;
  const uint8_t k = cls[c];
  if (k == 2) return;
  if (k == 0) {
    Dc[c] = 0.0;
    return;
  }
  const int i = (int)(c % G.n[0]);
  const int64_t r = c / G.n[0];
  const int j = (int)(r % G.n[1]), kz = DIM == 3 ? (int)(r / G.n[1]) : 0;
  double net = 0.0;
#pragma unroll
  for (int d = 0; d < DIM; ++d) {
    const int64_t m0 = G.n[0] + (d == 0), m1 = G.n[1] + (d == 1);
    const int64_t lo = G.fbase[d] + i + m0 * (j + m1 * (int64_t)kz);
    const int64_t st = d == 0 ? 1 : (d == 1 ? m0 : m0 * m1);
    net += F[lo + st] - F[lo];
  }
  Dc[c] = net / G.h;
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

__global__ void __launch_bounds__(256) k_adv_update(const uint8_t* __restrict__ cls, int64_t N, double dt,
                                                    const double* __restrict__ n, const double* __restrict__ Dc,
                                                    double* __restrict__ nout) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= N) return;
  nout[c] = cls[c] ? n[c] - dt * Dc[c] : 0.0;
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

}  // namespace ebmg
