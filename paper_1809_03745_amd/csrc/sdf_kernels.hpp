// Signed distance from a triangle mesh at the nodes of a box (the
// geometry-generation section of the paper: the distance to the closest
// polygon, edge or vertex, found through a bounding-volume hierarchy by a
// nearest-first closest-feature search). One thread per node; the search
// keeps the best squared distance found so far and descends into the nearer
// child box first, pushing the farther one while its box could still hold a
// closer triangle. The sign is that of (p - c) . n, with c the closest point
// and n the angle-weighted pseudonormal of the feature c lies on (face, edge
// or vertex), prepared on the host (mesh.cpp). FP64 throughout.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ebmg {

constexpr int kSdfBlock = 256;
constexpr int kSdfStack = 48;   // pending subtrees per thread (at least the tree depth)

struct DevMeshNode {
  double lo[3], hi[3];
  int32_t first, count;
};

// Closest point of triangle (a, b, c) to p by the Voronoi regions of its
// vertices, edges and face (the method of Ericson, Real-Time Collision
// Detection, section 5.1.5): returns the squared distance and the point,
// and the feature: 0 the face, 1 + j the edge from vertex j to j + 1 (mod 3),
// 4 + j vertex j.
__device__ __forceinline__ double closest_on_triangle(const double* __restrict__ r, double px, double py, double pz,
                                                      double& cx, double& cy, double& cz, int& feat) {
  const double ax = r[0], ay = r[1], az = r[2];
  const double bx = r[3], by = r[4], bz = r[5];
  const double qx = r[6], qy = r[7], qz = r[8];
  const double abx = bx - ax, aby = by - ay, abz = bz - az;
  const double acx = qx - ax, acy = qy - ay, acz = qz - az;
  const double apx = px - ax, apy = py - ay, apz = pz - az;
  const double d1 = abx * apx + aby * apy + abz * apz;
  const double d2 = acx * apx + acy * apy + acz * apz;
  if (d1 <= 0.0 && d2 <= 0.0) {
    cx = ax; cy = ay; cz = az;
    feat = 4;
  } else {
    const double bpx = px - bx, bpy = py - by, bpz = pz - bz;
    const double d3 = abx * bpx + aby * bpy + abz * bpz;
    const double d4 = acx * bpx + acy * bpy + acz * bpz;
    const double cpx = px - qx, cpy = py - qy, cpz = pz - qz;
    const double d5 = abx * cpx + aby * cpy + abz * cpz;
    const double d6 = acx * cpx + acy * cpy + acz * cpz;
    const double vc = d1 * d4 - d3 * d2;
    const double vb = d5 * d2 - d1 * d6;
    const double va = d3 * d6 - d5 * d4;
    if (d3 >= 0.0 && d4 <= d3) {
      cx = bx; cy = by; cz = bz;
      feat = 5;
    } else if (d6 >= 0.0 && d5 <= d6) {
      cx = qx; cy = qy; cz = qz;
      feat = 6;
    } else if (vc <= 0.0 && d1 >= 0.0 && d3 <= 0.0) {
      const double v = d1 / (d1 - d3);
      cx = ax + v * abx; cy = ay + v * aby; cz = az + v * abz;
      feat = 1;
    } else if (vb <= 0.0 && d2 >= 0.0 && d6 <= 0.0) {
      const double w = d2 / (d2 - d6);
      cx = ax + w * acx; cy = ay + w * acy; cz = az + w * acz;
      feat = 3;
    } else if (va <= 0.0 && (d4 - d3) >= 0.0 && (d5 - d6) >= 0.0) {
      const double w = (d4 - d3) / ((d4 - d3) + (d5 - d6));
      cx = bx + w * (qx - bx); cy = by + w * (qy - by); cz = bz + w * (qz - bz);
      feat = 2;
    } else {
      const double den = 1.0 / (va + vb + vc);
      const double v = vb * den, w = vc * den;
      cx = ax + abx * v + acx * w; cy = ay + aby * v + acy * w; cz = az + abz * v + acz * w;
      feat = 0;
    }
  }
  const double dx = px - cx, dy = py - cy, dz = pz - cz;
  return dx * dx + dy * dy + dz * dz;
}

__device__ __forceinline__ double box_d2(const DevMeshNode& n, double px, double py, double pz) {
  const double ex = fmax(fmax(n.lo[0] - px, 0.0), px - n.hi[0]);
  const double ey = fmax(fmax(n.lo[1] - py, 0.0), py - n.hi[1]);
  const double ez = fmax(fmax(n.lo[2] - pz, 0.0), pz - n.hi[2]);
  return ex * ex + ey * ey + ez * ez;
}

// sdf[node] for the nodes lo + (i, j, k) h of an (n0+1) x (n1+1) x (n2+1)
// lattice (x fastest); visits (nullable) accumulates the boxes and
// triangles examined
__global__ void __launch_bounds__(kSdfBlock) k_sdf_mesh(const DevMeshNode* __restrict__ nodes,
                                                       const double* __restrict__ tri, int m0, int m1, int m2,
                                                       double h, double lox, double loy, double loz,
                                                       double* __restrict__ sdf,
                                                       unsigned long long* __restrict__ visits) {
  __shared__ int32_t stk[kSdfStack * kSdfBlock];
  __shared__ unsigned long long vsum[kSdfBlock / 64];
  const int64_t total = (int64_t)m0 * m1 * m2;
  const int64_t q = (int64_t)blockIdx.x * kSdfBlock + threadIdx.x;
  unsigned long long nvis = 0;
  if (q < total) {
    const int i = (int)(q % m0);
    const int64_t jk = q / m0;
    const int j = (int)(jk % m1), k = (int)(jk / m1);
    const double px = lox + i * h, py = loy + j * h, pz = loz + k * h;
    double best = 1e300, side = 1.0;
    int sp = 0;
    int32_t cur = 0;
    while (true) {
      const DevMeshNode nd = nodes[cur];
      ++nvis;
      if (nd.count >= 0) {
        for (int t = nd.first; t < nd.first + nd.count; ++t) {
          const double* r = tri + (int64_t)t * 30;
          double cx, cy, cz;
          int f;
          const double d2 = closest_on_triangle(r, px, py, pz, cx, cy, cz, f);
          ++nvis;
          if (d2 < best) {
            const double* nrm = f == 0 ? r + 9 : (f <= 3 ? r + 12 + 3 * (f - 1) : r + 21 + 3 * (f - 4));
            best = d2;
            side = (px - cx) * nrm[0] + (py - cy) * nrm[1] + (pz - cz) * nrm[2];
          }
        }
      } else {
        const int32_t l = nd.first, rr = -nd.count;
        const double dl = box_d2(nodes[l], px, py, pz), dr = box_d2(nodes[rr], px, py, pz);
        const int32_t nearer = dl <= dr ? l : rr, farther = dl <= dr ? rr : l;
        const double dn = fmin(dl, dr), df = fmax(dl, dr);
        if (dn < best) {
          if (df < best && sp < kSdfStack) stk[sp++ * kSdfBlock + threadIdx.x] = farther;
          cur = nearer;
          continue;
        }
      }
      // next pending subtree that may still hold a closer triangle
      bool found = false;
      while (sp > 0) {
        const int32_t c = stk[--sp * kSdfBlock + threadIdx.x];
        if (box_d2(nodes[c], px, py, pz) < best) {
          cur = c;
          found = true;
          break;
        }
      }
      if (!found) break;
    }
    sdf[q] = side >= 0.0 ? sqrt(best) : -sqrt(best);
  }
  if (visits) {
    // per-wavefront sums, then one atomic per block
    for (int o = 32; o > 0; o >>= 1) nvis += __shfl_xor(nvis, o);
    if ((threadIdx.x & 63) == 0) vsum[threadIdx.x >> 6] = nvis;
    __syncthreads();
    if (threadIdx.x == 0) {
      unsigned long long s = 0;
      for (int w = 0; w < kSdfBlock / 64; ++w) s += vsum[w];
      atomicAdd(visits, s);
    }
  }
}

}  // namespace ebmg
