// nh_proj.hpp -- initial guesses of the adjoint CG solves by projection onto
// the solutions of the preceding adjoint steps (P. F. Fischer, "Projection
// techniques for iterative solution of Ax = b with successive right-hand
// sides", Comput. Methods Appl. Mech. Engrg. 163, 1998), over a sliding window.
//
// The adjoint sweep solves A mu^n = c^n = mu^{n+1} + P^T g^n for n = N..1 with
// one operator A. With W = [w_0 .. w_{k-1}] the last k solutions (w_0 = mu^{n+1},
// newest first), the guess
//     x0 = W gamma,   (W^T A W) gamma = W^T c^n
// is the point of span(W) closest to the solution in the A-norm (it contains
// every extrapolation of the same states). The Gram matrix W^T A W is kept on
// the device and gains one row per step: after step n+1 the new solution v =
// mu^{n+1} enters the window and
//     A v                                  (proj_apply_kernel)
//     w_j . A v,  w_j . v,  w_j[k=0] . g^n  (proj_dots_kernel, block partials)
// give its row, and W^T c^n = W^T v + W^T P^T g^n. proj_solve_kernel sums the
// partials in a fixed order, updates the Gram matrix and solves for gamma by a
// Cholesky factorisation that takes the window newest first and drops a
// vector whose remaining A-norm is below a relative cut (a window of nearly
// parallel states is common); proj_combine_kernel forms x0. The CG solve
// that follows is unchanged, so the solution (its tolerance) is too: only
// where the iteration starts differs.
#pragma once

#include "nh_kernels.hpp"

namespace nh {

constexpr int kProjMax = 6;                 // window: solutions of the last kProjMax adjoint steps
constexpr int kProjRing = 8;                // adjoint state buffers: window + the step being solved
constexpr int kProjBlock = 256;
constexpr int kProjDotBlocks = 1024;        // fixed grid of the dot kernel (deterministic sums)
constexpr int kProjVals = 3 * kProjMax;     // per block: w_j.Av, w_j.v, w_j[top].g
constexpr double kProjCut = 1e-10;          // relative A-norm below which a window vector is dropped

template <typename R>
struct ProjWin {
  const R* w[kProjMax];                     // window, newest first (w[0] = v, the newest solution)
  int slot[kProjMax];                       // ring slot of each window vector (Gram matrix index)
  int k;                                    // window size, 1..kProjMax
};

// Device-resident state of the projection.
struct ProjState {
  double gram[kProjRing][kProjRing];        // w_a . A w_b by ring slot
  double coef[kProjMax];                    // gamma for the next solve, window order
  int kept;                                 // window vectors the last solve used
};

// y = A x for the projection (one thread per cell, neighbours through the
// caches): the same face terms and Robin sink as the step kernels, zero flux
// or lateral wrap-around at the walls.
template <typename R>
__global__ void __launch_bounds__(kProjBlock) proj_apply_kernel(Geom g, const R* __restrict__ alpha,
                                                                const R* __restrict__ x, R* __restrict__ y,
                                                                Coef<R> cf) {
  const long long i = (long long)blockIdx.x * kProjBlock + threadIdx.x;
  if (i >= g.ng) return;
  const int kz = (int)(i / g.nxy);
  const long long col = i - (long long)kz * g.nxy;
  const int iy = (int)(col / g.nx), ix = (int)(col - (long long)iy * g.nx);
  const R a = alpha[i], v = x[i];
  R s = R(0);
  auto add = [&](R sd, long long j) {
    const R c = face<R>(sd, a, alpha[j]);
    s += c * (v - x[j]);
  };
  const long long rowx = i - ix, base = i - col;
  if (ix > 0) add(cf.sx, i - 1);
  else if (g.periodic) add(cf.sx, rowx + g.nx - 1);
  if (ix + 1 < g.nx) add(cf.sx, i + 1);
  else if (g.periodic) add(cf.sx, rowx);
  if (iy > 0) add(cf.sy, i - g.nx);
  else if (g.periodic) add(cf.sy, base + (long long)(g.ny - 1) * g.nx + ix);
  if (iy + 1 < g.ny) add(cf.sy, i + g.nx);
  else if (g.periodic) add(cf.sy, base + ix);
  if (kz > 0) add(cf.sz, i - g.nxy);
  if (kz + 1 < g.nz) add(cf.sz, i + g.nxy);
  if (kz == cf.zb) s += cf.sb * v;
  y[i] = v + s;
}

// Block partials of w_j . Av, w_j . v (v = w_0) and, on the plane k = 0,
// w_j . g (g may be null): part[block][q * kProjMax + j].
template <typename R>
__global__ void __launch_bounds__(kProjBlock) proj_dots_kernel(ProjWin<R> W, const R* __restrict__ Av,
                                                               const R* __restrict__ gtop, long long n,
                                                               long long nxy, double* __restrict__ part) {
  double acc[kProjVals];
#pragma unroll
  for (int q = 0; q < kProjVals; ++q) acc[q] = 0.0;
  const long long stride = (long long)gridDim.x * kProjBlock;
  for (long long i = (long long)blockIdx.x * kProjBlock + threadIdx.x; i < n; i += stride) {
    const double av = Av[i], v = W.w[0][i];
    const double gv = (gtop && i < nxy) ? (double)gtop[i] : 0.0;
#pragma unroll
    for (int j = 0; j < kProjMax; ++j) {
      if (j < W.k) {
        const double wj = j == 0 ? v : (double)W.w[j][i];
        acc[j] += wj * av;
        acc[kProjMax + j] += wj * v;
        acc[2 * kProjMax + j] += wj * gv;
      }
    }
  }
  __shared__ double red[kProjBlock / 64][kProjVals];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int q = 0; q < kProjVals; ++q) {
    const double s = wave_sum(acc[q]);
    if (lane == 0) red[wave][q] = s;
  }
  __syncthreads();
  if (threadIdx.x < kProjVals) {
    double s = 0.0;
    for (int w = 0; w < kProjBlock / 64; ++w) s += red[w][threadIdx.x];
    part[(size_t)blockIdx.x * kProjVals + threadIdx.x] = s;
  }
}

// One workgroup: sums the partials of nblk blocks in a fixed order, stores the
// new Gram row and column (slot W.slot[0]) and solves for the coefficients.
template <typename R>
__global__ void __launch_bounds__(kProjBlock) proj_solve_kernel(ProjWin<R> W, const double* __restrict__ part,
                                                                int nblk, ProjState* st) {
  double acc[kProjVals];
#pragma unroll
  for (int q = 0; q < kProjVals; ++q) acc[q] = 0.0;
  for (int b = threadIdx.x; b < nblk; b += kProjBlock) {
#pragma unroll
    for (int q = 0; q < kProjVals; ++q) acc[q] += part[(size_t)b * kProjVals + q];
  }
  __shared__ double red[kProjBlock / 64][kProjVals];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int q = 0; q < kProjVals; ++q) {
    const double s = wave_sum(acc[q]);
    if (lane == 0) red[wave][q] = s;
  }
  __syncthreads();
  if (threadIdx.x != 0) return;
  double tot[kProjVals];
  for (int q = 0; q < kProjVals; ++q) {
    double s = 0.0;
    for (int w = 0; w < kProjBlock / 64; ++w) s += red[w][q];
    tot[q] = s;
  }
  const int k = W.k;
  const int s0 = W.slot[0];
  for (int j = 0; j < k; ++j) {
    st->gram[s0][W.slot[j]] = tot[j];
    st->gram[W.slot[j]][s0] = tot[j];
  }
  // right-hand side of the next solve: w_j . (v + P^T g)
  double rhs[kProjMax], L[kProjMax][kProjMax], y[kProjMax], gam[kProjMax];
  int keep[kProjMax], nk = 0;
  for (int j = 0; j < k; ++j) rhs[j] = tot[kProjMax + j] + tot[2 * kProjMax + j];
  // Cholesky of the Gram matrix over the kept vectors, newest first
  for (int j = 0; j < k; ++j) {
    const double gjj = st->gram[W.slot[j]][W.slot[j]];
    if (!(gjj > 0.0) || !(gjj < INFINITY)) continue;
    double row[kProjMax];
    double d = gjj;
    for (int a = 0; a < nk; ++a) {
      double s = st->gram[W.slot[j]][W.slot[keep[a]]];
      for (int b = 0; b < a; ++b) s -= row[b] * L[a][b];
      row[a] = s / L[a][a];
      d -= row[a] * row[a];
    }
    if (!(d > kProjCut * gjj)) continue;
    for (int a = 0; a < nk; ++a) L[nk][a] = row[a];
    L[nk][nk] = sqrt(d);
    keep[nk++] = j;
  }
  // L L^T gamma = rhs over the kept vectors
  for (int a = 0; a < nk; ++a) {
    double s = rhs[keep[a]];
    for (int b = 0; b < a; ++b) s -= L[a][b] * y[b];
    y[a] = s / L[a][a];
  }
  for (int a = nk - 1; a >= 0; --a) {
    double s = y[a];
    for (int b = a + 1; b < nk; ++b) s -= L[b][a] * gam[b];
    gam[a] = s / L[a][a];
  }
  for (int j = 0; j < kProjMax; ++j) st->coef[j] = 0.0;
  for (int a = 0; a < nk; ++a) st->coef[keep[a]] = gam[a];
  st->kept = nk;
}

// x0 = sum_j coef_j w_j (the window order of the solve).
template <typename R>
__global__ void __launch_bounds__(kProjBlock) proj_combine_kernel(ProjWin<R> W, const ProjState* __restrict__ st,
                                                                  R* __restrict__ x0, long long n) {
  const long long i = (long long)blockIdx.x * kProjBlock + threadIdx.x;
  if (i >= n) return;
  R s = R(0);
#pragma unroll
  for (int j = 0; j < kProjMax; ++j)
    if (j < W.k) s = fma((R)st->coef[j], W.w[j][i], s);
  x0[i] = s;
}

}  // namespace nh
