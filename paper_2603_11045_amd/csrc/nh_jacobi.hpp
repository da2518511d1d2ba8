// nh_jacobi.hpp -- the paper's fixed-K Jacobi inner solver (eq. jacobi_iter,
// App. D.2) with temporal blocking, for thin grids (nz <= NZ) in FP32.
//
// A team barrier costs ~6 us on this chip, several times a sweep of a small
// grid, so a step that barriers after every sweep is barrier-bound. Here each
// workgroup owns an interior tile of kJacIX x kJacIY columns and computes on
// the tile widened by kJacS columns on every lateral side (an extended tile
// of kJacEX x kJacEY = one column per thread, the whole column of nz cells in
// registers). A phase loads the extended tile's iterate, runs kJacS sweeps
// exchanging columns through LDS only, and stores the interior: after j
// sweeps the j outermost rings of the extended tile hold wrong values (they
// miss neighbours outside it), so after kJacS sweeps exactly the interior is
// right. One team barrier per phase instead of one per sweep; the halo
// columns are computed twice (by this workgroup and by their owner).
//
// The face conductances, 1/D and b = h1 + the top source are formed once per
// step and stay in registers. Columns outside the grid (zero-flux walls) have
// alpha = 0: every face toward them has conductance 0 and they stay at 0.
// With periodic lateral faces every extended column maps to a grid column.
#pragma once

#include "nh_kernels.hpp"

namespace nh {

constexpr int kJacBlock = 512;
constexpr int kJacEX = 32, kJacEY = 16;     // extended tile, columns
constexpr int kJacS = 4;                    // sweeps per phase = halo width
constexpr int kJacIX = kJacEX - 2 * kJacS;  // interior tile: 24 x 8 columns
constexpr int kJacIY = kJacEY - 2 * kJacS;
constexpr int kJacNZ = 16;                  // largest nz the kernel takes

template <int NZ>
__device__ StepResult jacobi_tb_step(const StepArgs<float>& S, const StepVar<float>& V, int rank, float* xs,
                                     Smem<float>& sh) {
  const Geom& g = S.g;
  const int tid = threadIdx.x;
  const int lx = tid % kJacEX, ly = tid / kJacEX;
  const int tx = rank % S.jtx, ty = rank / S.jtx;
  const int ux = tx * kJacIX - kJacS + lx, uy = ty * kJacIY - kJacS + ly;   // unwrapped grid column
  int gx = ux, gy = uy;
  bool valid;
  if (g.periodic) {
    gx = ((gx % g.nx) + g.nx) % g.nx;
    gy = ((gy % g.ny) + g.ny) % g.ny;
    valid = true;
  } else {
    valid = gx >= 0 && gx < g.nx && gy >= 0 && gy < g.ny;
  }
  const long long col = valid ? (long long)gx + (long long)g.nx * gy : 0;
  const bool inner = lx >= kJacS && lx < kJacS + kJacIX && ly >= kJacS && ly < kJacS + kJacIY && ux < g.nx &&
                     uy < g.ny;
  const bool hl = lx > 0, hr = lx < kJacEX - 1, hd = ly > 0, hu = ly < kJacEY - 1;
  const int nz = g.nz;
  const long long nxy = g.nxy;
  unsigned long long red = V.epoch_base;
  bool ok = true;

  // coefficients of the own column from the neighbours' alpha, exchanged through LDS
  float a[NZ];
#pragma unroll
  for (int k = 0; k < NZ; ++k) a[k] = (valid && k < nz) ? S.alpha[col + k * nxy] : 0.f;
#pragma unroll
  for (int k = 0; k < NZ; ++k) xs[k * kJacBlock + tid] = a[k];
  __syncthreads();
  float cxm[NZ], cxp[NZ], cym[NZ], cyp[NZ], cz[NZ], rd[NZ], b[NZ], x[NZ];
#pragma unroll
  for (int k = 0; k < NZ; ++k) {
    cxm[k] = cxp[k] = cym[k] = cyp[k] = cz[k] = 0.f;
    if (valid && k < nz) {                  // a[k] > 0: no face divides by zero
      if (hl) cxm[k] = face<float>(S.sx, a[k], xs[k * kJacBlock + tid - 1]);
      if (hr) cxp[k] = face<float>(S.sx, a[k], xs[k * kJacBlock + tid + 1]);
      if (hd) cym[k] = face<float>(S.sy, a[k], xs[k * kJacBlock + tid - kJacEX]);
      if (hu) cyp[k] = face<float>(S.sy, a[k], xs[k * kJacBlock + tid + kJacEX]);
      if (k + 1 < nz) cz[k] = face<float>(S.sz, a[k], a[k + 1]);
    }
  }
#pragma unroll
  for (int k = 0; k < NZ; ++k) {
    const float czm = k > 0 ? cz[k - 1] : 0.f;
    const float sk = k == nz - 1 ? S.sb : 0.f;
    const float D = 1.f + ((((cxm[k] + cxp[k]) + (cym[k] + cyp[k])) + (czm + cz[k])) + sk);
    rd[k] = (valid && k < nz) ? rcp<float>(D) : 1.f;
    float bk = 0.f;
    if (valid && k < nz) {
      if (V.xprev) bk = V.xprev[col + k * nxy];
      if (k == 0) bk += V.top_scale * V.top_src[col];
    }
    b[k] = bk;
  }
  __syncthreads();                          // alpha reads done before the first column exchange

  const int K = S.jacobi_k;
  const int phases = (K + kJacS - 1) / kJacS;
  const float* xin = V.xprev;
  double bb = 0.0, rr = 0.0;
  for (int ph = 0; ph < phases && ok; ++ph) {
    const int ns = min(kJacS, K - ph * kJacS);
    const bool last_phase = ph == phases - 1;
    float* xout = ((phases - 1 - ph) & 1) ? S.p0 : V.x;
#pragma unroll
    for (int k = 0; k < NZ; ++k) x[k] = (xin && valid && k < nz) ? xin[col + k * nxy] : 0.f;
    double vb = 0.0, vr = 0.0;
    for (int j = 0; j < ns; ++j) {
#pragma unroll
      for (int k = 0; k < NZ; ++k) xs[k * kJacBlock + tid] = x[k];
      __syncthreads();
      const bool acc = last_phase && j == ns - 1 && inner;
      float xn[NZ];
#pragma unroll
      for (int k = 0; k < NZ; ++k) {
        const float v = x[k];
        const float xl = hl ? xs[k * kJacBlock + tid - 1] : v;
        const float xr = hr ? xs[k * kJacBlock + tid + 1] : v;
        const float xd = hd ? xs[k * kJacBlock + tid - kJacEX] : v;
        const float xu = hu ? xs[k * kJacBlock + tid + kJacEX] : v;
        float s = cxm[k] * (v - xl);
        s += cxp[k] * (v - xr);
        s += cym[k] * (v - xd);
        s += cyp[k] * (v - xu);
        if (k > 0) s += cz[k - 1] * (v - x[k - 1]);
        if (k + 1 < NZ) s += cz[k] * (v - x[k + 1]);
        if (k == nz - 1) s += S.sb * v;
        const float r = b[k] - (v + s);
        xn[k] = v + r * rd[k];
        if (acc && k < nz) {
          vb += (double)b[k] * (double)b[k];
          vr += (double)r * (double)r;
        }
      }
      __syncthreads();                      // every read of this exchange done before the next
#pragma unroll
      for (int k = 0; k < NZ; ++k) x[k] = xn[k];
    }
    if (inner) {
#pragma unroll
      for (int k = 0; k < NZ; ++k)
        if (k < nz) st_out(xout + col + k * nxy, x[k]);
    }
    double v2[2] = {vb, vr};
    ok &= team_sum<float, 2, kJacBlock>(S, rank, red, v2, sh);
    if (last_phase) {
      bb = v2[0];
      rr = v2[1];
    }
    xin = xout;
  }
  return step_epilogue<float>(S, V, rank, ok, ok ? K : 0, kOk, bb, rr, sh);
}

template <int NZ>
__global__ void __launch_bounds__(kJacBlock, 1) jacobi_step_kernel(StepArgs<float> S) {
  __shared__ Smem<float> sh;
  __shared__ float xs[NZ * kJacBlock];
  jacobi_tb_step<NZ>(S, step_var(S), blockIdx.x, xs, sh);
}

}  // namespace nh
