// Kernels of the composite AMR solve (Numerical methods: patch-based
// refinement; Helmholtz equations: refluxing). The levels' own operators,
// smoothers and V-cycles are the single-box kernels; these add the sparse
// coarse-fine coupling rows, copy or clear lists of unknowns, restrict and
// prolong between a box and its coarser level, and run the FP64 vector
// steps of the composite BiCGStab over one contiguous vector holding every
// level.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ebmg {

// y[row[r]] += sum_e w[e] (col[e] >= 0 ? xs[col[e]] : xo[-col[e] - 1]):
// one thread per row (rows are distinct, so no two threads write one entry)
__global__ void __launch_bounds__(256) k_amr_rows(int64_t nrow, const int64_t* __restrict__ row,
                                                  const int64_t* __restrict__ ptr, const int64_t* __restrict__ col,
                                                  const double* __restrict__ w, const double* __restrict__ xs,
                                                  const double* __restrict__ xo, double* __restrict__ y) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= nrow) return;
  double s = 0.0;
  for (int64_t e = ptr[r]; e < ptr[r + 1]; ++e) {
    const int64_t c = col[e];
    s += w[e] * (c >= 0 ? xs[c] : xo[-c - 1]);
  }
  y[row[r]] += s;
}

// y[row[r]] = sum_e w[e] x[col[e]]
__global__ void __launch_bounds__(256) k_amr_gather(int64_t nrow, const int64_t* __restrict__ row,
                                                    const int64_t* __restrict__ ptr, const int64_t* __restrict__ col,
                                                    const double* __restrict__ w, const double* __restrict__ x,
                                                    double* __restrict__ y) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= nrow) return;
  double s = 0.0;
  for (int64_t e = ptr[r]; e < ptr[r + 1]; ++e) s += w[e] * x[col[e]];
  y[row[r]] = s;
}

// y[idx[i]] = x[idx[i]] (x null: 0)
__global__ void __launch_bounds__(256) k_amr_set(int64_t n, const int64_t* __restrict__ idx,
                                                 const double* __restrict__ x, double* __restrict__ y) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int64_t k = idx[i];
  y[k] = x ? x[k] : 0.0;
}

// xf[i] = xc[pcol[i]] (0 where there is no coarse unknown)
__global__ void __launch_bounds__(256) k_amr_prolong(int64_t n, const int64_t* __restrict__ pcol,
                                                     const double* __restrict__ xc, double* __restrict__ xf) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int64_t c = pcol[i];
  xf[i] = c >= 0 ? xc[c] : 0.0;
}

// z = a x + b y
__global__ void __launch_bounds__(256) k_amr_lin(int64_t n, double a, const double* __restrict__ x, double b,
                                                 const double* __restrict__ y, double* __restrict__ z) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) z[i] = a * x[i] + b * y[i];
}

// p = r + beta (p - omega v)
__global__ void __launch_bounds__(256) k_amr_p(int64_t n, const double* __restrict__ r, double beta, double omega,
                                               const double* __restrict__ v, double* __restrict__ p) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = r[i] + beta * (p[i] - omega * v[i]);
}

// x += alpha ph + omega sh; r = s - omega t
__global__ void __launch_bounds__(256) k_amr_xr(int64_t n, double alpha, const double* __restrict__ ph, double omega,
                                                const double* __restrict__ sh, const double* __restrict__ s,
                                                const double* __restrict__ t, double* __restrict__ x,
                                                double* __restrict__ r) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  x[i] += alpha * ph[i] + omega * sh[i];
  r[i] = s[i] - omega * t[i];
}

}  // namespace ebmg
