// nh_tv.hpp -- the discrete total-variation regulariser of the inverse
// problem (eq. tv_discrete, App. D.1) and its gradient, fused in one pass.
//
//   R(a) = dx dy dz sum_p t_p,   t_p = sqrt((d_x a / dx)^2 + (d_y a / dy)^2 + (d_z a / dz)^2 + eps^2)
//
// with forward differences along the array axes, x and y wrapping around and
// d_z a = 0 on the last plane. t_p depends on a_p and its +x, +y, +z
// neighbours, so dR/da_p collects p's own term and the terms of its -x, -y,
// -z neighbours (a 13-point stencil of a). One thread per cell recomputes
// those four terms from global loads (adjacent threads share them in L1/L2),
// adds weight * dR/da_p to (or writes it into) the FP64 gradient, and the
// workgroup's partial sum of t goes to its own slot; tv_finish_kernel sums the
// slots in order, so the value is deterministic.
#pragma once

#include <hip/hip_runtime.h>

namespace nh {

constexpr int kTvBlock = 256;
constexpr int kTvMaxBlocks = 4096;

template <typename R>
struct TvArgs {
  const R* alpha;
  int nx, ny, nz;
  long long nxy, ng;
  R ix2, iy2, iz2;                          // 1 / h_d^2
  R eps2;
  double scale;                             // weight * dx dy dz
  double* grad;                             // [ng] FP64
  int accumulate;                           // 1: grad += scale dR/da; 0: grad = scale dR/da
  double* partial;                          // [gridDim.x] per-workgroup sums of t
};

// t of cell (i, j, k) and its three forward-difference weights d_d / (h_d^2 t).
template <typename R>
__device__ __forceinline__ R tv_term(const TvArgs<R>& A, int i, int j, int k, R& gx, R& gy, R& gz) {
  const long long p = (long long)i + (long long)A.nx * j + A.nxy * k;
  const R ap = A.alpha[p];
  const R dx = A.alpha[p + (i + 1 < A.nx ? 1 : 1 - A.nx)] - ap;
  const R dy = A.alpha[p + (j + 1 < A.ny ? (long long)A.nx : (long long)A.nx * (1 - A.ny))] - ap;
  const R dz = k + 1 < A.nz ? A.alpha[p + A.nxy] - ap : R(0);
  const R t = sqrt(dx * dx * A.ix2 + dy * dy * A.iy2 + dz * dz * A.iz2 + A.eps2);
  const R rt = R(1) / t;
  gx = dx * A.ix2 * rt;
  gy = dy * A.iy2 * rt;
  gz = dz * A.iz2 * rt;
  return t;
}

template <typename R>
__global__ void __launch_bounds__(kTvBlock) tv_kernel(TvArgs<R> A) {
  double tsum = 0.0;
  for (long long p = blockIdx.x * (long long)kTvBlock + threadIdx.x; p < A.ng;
       p += (long long)gridDim.x * kTvBlock) {
    const int k = (int)(p / A.nxy);
    const long long c = p - (long long)k * A.nxy;
    const int j = (int)(c / A.nx);
    const int i = (int)(c - (long long)j * A.nx);
    R gx, gy, gz, hx, hy, hz;
    const R t = tv_term(A, i, j, k, gx, gy, gz);
    R g = -((gx + gy) + gz);
    tv_term(A, i > 0 ? i - 1 : A.nx - 1, j, k, hx, hy, hz);
    g += hx;                                // p is the +x neighbour of the cell before it
    tv_term(A, i, j > 0 ? j - 1 : A.ny - 1, k, hx, hy, hz);
    g += hy;
    if (k > 0) {
      tv_term(A, i, j, k - 1, hx, hy, hz);
      g += hz;
    }
    const double v = A.scale * (double)g;
    A.grad[p] = A.accumulate ? A.grad[p] + v : v;
    tsum += (double)t;
  }
  // workgroup sum in a fixed order: wave butterfly, then the waves in order
  for (int o = 32; o > 0; o >>= 1) tsum += __shfl_xor(tsum, o, 64);
  __shared__ double red[kTvBlock / 64];
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = tsum;
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = 0.0;
    for (int w = 0; w < kTvBlock / 64; ++w) s += red[w];
    A.partial[blockIdx.x] = s;
  }
}

// value = scale * sum of the partials, in order (one workgroup).
__global__ void __launch_bounds__(kTvBlock) tv_finish_kernel(const double* partial, int n, double scale,
                                                               double* value) {
  __shared__ double red[kTvBlock];
  double s = 0.0;
  for (int b = threadIdx.x; b < n; b += kTvBlock) s += partial[b];
  red[threadIdx.x] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double tot = 0.0;
    for (int w = 0; w < kTvBlock; ++w) tot += red[w];
    *value = scale * tot;
  }
}

}  // namespace nh
