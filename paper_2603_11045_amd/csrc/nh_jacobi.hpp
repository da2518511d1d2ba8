// nh_jacobi.hpp -- the paper's fixed-K Jacobi inner solver (eq. jacobi_iter,
// App. D.2) with temporal blocking, for thin grids (nz <= 16) in FP32.
//
// A team barrier costs several microseconds on this chip, more than a sweep of
// a small grid, so a step that barriers after every sweep is barrier-bound.
// Here each workgroup owns an interior tile of kJacIX x kJacIY columns and
// computes on the tile widened by kJacS columns on every lateral side (an
// extended tile of kJacEX x kJacEY columns; two threads per column, each with
// half of the column's cells in registers). A phase loads the extended tile's
// iterate, runs kJacS sweeps exchanging the tile through LDS only, and stores
// the interior: after j sweeps the j outermost rings of the extended tile hold
// wrong values (they miss neighbours outside it), so after kJacS sweeps exactly
// the interior is right. One team barrier per phase instead of one per sweep;
// the halo columns are computed twice (by this workgroup and by their owner).
//
// The face conductances (in registers), 1/D and b = h1 + the top source (in
// LDS) are formed once per step. Columns outside the grid (zero-flux walls) have
// alpha = 0: every face toward them has conductance 0 and they stay at 0.
// With periodic lateral faces every extended column maps to a grid column.
//
// Between phases there is no team barrier: a phase stores its interior into
// a tagged buffer, one 64-bit word per cell holding the value and the phase's
// tag, stored and loaded device-coherent, and the next phase's loads spin on
// each word until its tag is the expected one. A workgroup can run at most one
// phase ahead of a neighbour (it needs the neighbour's previous phase), so the
// two alternating buffers are never overwritten while still being read. Tags
// grow from launch to launch (the host clears the buffers before they wrap),
// so a stale word never matches. The last phase stores plain values into x and
// ends with the all-gather reduction of the residual diagnostics, followed by
// an acquire fence, since the gradient pass reads x with ordinary loads.
#pragma once

#include "nh_kernels.hpp"
#include "nh_resident.hpp"

namespace nh {

constexpr int kJacBlock = 1024;
constexpr int kJacEX = 32, kJacEY = 16;     // extended tile, columns
constexpr int kJacCols = kJacEX * kJacEY;   // 512: two threads per column
constexpr int kJacS = 4;                    // sweeps per phase = halo width
constexpr int kJacIX = kJacEX - 2 * kJacS;  // interior tile: 24 x 8 columns
constexpr int kJacIY = kJacEY - 2 * kJacS;
constexpr int kJacNZ = 16;                  // largest nz the kernel takes
constexpr int kJacH = kJacNZ / 2;           // cells per thread

// LDS: xs the exchanged iterate, bs and rds the per-cell b and 1/D, each
// [2H planes][kJacCols columns].
template <int H>
__device__ StepResult jacobi_tb_step(const StepArgs<float>& S, const StepVar<float>& V, int rank, float* xs,
                                     float* bs, float* rds, Smem<float>& sh, ResRed* rs) {
  constexpr int C = kJacCols;
  const Geom& g = S.g;
  // a caller that loops over steps must not keep one step's per-thread
  // geometry live into the next: laundered, it is recomputed per step
  int tid = threadIdx.x, rank_l = rank;
  asm volatile("" : "+v"(tid));
  asm volatile("" : "+s"(rank_l));
  const int c = tid % C, k0 = (tid / C) * H;
  const int lx = c % kJacEX, ly = c / kJacEX;
  const int tx = rank_l % S.jtx, ty = rank_l / S.jtx;
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
  const bool hb = k0 > 0, ha = k0 + H < 2 * H;   // the other half of the column holds cell k0-1 / k0+H
  const int nz = g.nz;
  const long long nxy = g.nxy;
  unsigned long long red = V.epoch_base;
  bool ok = true;
  int ntr = 0;
  const bool tr = S.trace && rank == S.trace_rank && tid == 0;
  auto stamp = [&]() {
    if (tr && ntr < S.trace_cap) S.trace[ntr++] = wall_clock64();
  };
  stamp();

  // coefficients of the own cells from the neighbours' alpha, exchanged through LDS
  float a[H];
#pragma unroll
  for (int i = 0; i < H; ++i) a[i] = (valid && k0 + i < nz) ? S.alpha[col + (k0 + i) * nxy] : 0.f;
#pragma unroll
  for (int i = 0; i < H; ++i) xs[(k0 + i) * C + c] = a[i];
  __syncthreads();
  float cxm[H], cxp[H], cym[H], cyp[H], cz[H], x[H];
  float czb = 0.f;                          // the face below the first own cell
  if (hb && valid && k0 < nz) czb = face<float>(S.sz, xs[(k0 - 1) * C + c], a[0]);
#pragma unroll
  for (int i = 0; i < H; ++i) {
    const int k = k0 + i;
    cxm[i] = cxp[i] = cym[i] = cyp[i] = cz[i] = 0.f;
    if (valid && k < nz) {                  // a[i] > 0: no face divides by zero
      if (hl) cxm[i] = face<float>(S.sx, a[i], xs[k * C + c - 1]);
      if (hr) cxp[i] = face<float>(S.sx, a[i], xs[k * C + c + 1]);
      if (hd) cym[i] = face<float>(S.sy, a[i], xs[k * C + c - kJacEX]);
      if (hu) cyp[i] = face<float>(S.sy, a[i], xs[k * C + c + kJacEX]);
      if (k + 1 < nz) cz[i] = face<float>(S.sz, a[i], i + 1 < H ? a[i + 1] : xs[(k + 1) * C + c]);
    }
  }
#pragma unroll
  for (int i = 0; i < H; ++i) {
    const int k = k0 + i;
    const float czm = i > 0 ? cz[i - 1] : czb;
    const float sk = k == nz - 1 ? S.sb : 0.f;
    const float D = diag_of<float>(cxm[i], cxp[i], cym[i], cyp[i], czm, cz[i], sk);
    rds[k * C + c] = (valid && k < nz) ? rcp<float>(D) : 1.f;
    float bk = 0.f;
    if (valid && k < nz) {
      if (V.xprev) bk = V.xprev[col + k * nxy];
      if (k == 0) bk += V.top_scale * V.top_src[col];
    }
    bs[k * C + c] = bk;
  }
  __syncthreads();                          // alpha reads done before the first exchange of x
  stamp();

  const int K = S.jacobi_k;
  const int phases = (K + kJacS - 1) / kJacS;
  double bb = 0.0, rr = 0.0;
  for (int ph = 0; ph < phases; ++ph) {
    const int ns = min(kJacS, K - ph * kJacS);
    const bool last_phase = ph == phases - 1;
    // the column's first own cell; the others are uniform strides of nxy from
    // it (kept from being hoisted as one 64-bit offset per cell)
    long long base = col + (long long)k0 * nxy;
    asm volatile("" : "+v"(base));
    if (ph == 0) {
#pragma unroll
      for (int i = 0; i < H; ++i) x[i] = (V.xprev && valid && k0 + i < nz) ? V.xprev[base + i * nxy] : 0.f;
    } else {
      const unsigned tag = V.jtag + (unsigned)(ph - 1);
      unsigned long long* src = S.jt[(ph - 1) & 1];
#pragma unroll
      for (int i = 0; i < H; ++i) {
        x[i] = 0.f;
        if (valid && k0 + i < nz) {
          unsigned long long* w = src + base + i * nxy;
          unsigned long long v = __hip_atomic_load(w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          if ((unsigned)(v >> 32) != tag && ok) {   // after a time-out, wait no more
            const long long t0 = wall_clock64();
            do {
              __builtin_amdgcn_s_sleep(1);
              v = __hip_atomic_load(w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
              if (wall_clock64() - t0 > S.timeout_ticks) {
                ok = false;
                break;
              }
            } while ((unsigned)(v >> 32) != tag);
          }
          x[i] = __uint_as_float((unsigned)v);
        }
      }
    }
    if (tr) {                               // wait for the loads, for the stamp
      float t = 0.f;
#pragma unroll
      for (int i = 0; i < H; ++i) t += x[i];
      if (t == 12345.f) S.trace[S.trace_cap - 1] = 0;
    }
    stamp();
    double vb = 0.0, vr = 0.0;
    for (int j = 0; j < ns; ++j) {
      // one base address per sweep (kept from being hoisted into a register
      // per cell and neighbour): every access is a constant offset from it
      // neighbour reads without branches: a missing neighbour (edge of the
      // extended tile, end of the column) reads the cell itself, whose face
      // conductance is 0 or whose difference is 0
      int cb = k0 * C + c;
      asm volatile("" : "+v"(cb));
      float* xp = xs + cb;
      const float* bp = bs + cb;
      const float* rp = rds + cb;
      const float* pl = xp + (hl ? -1 : 0);
      const float* pr = xp + (hr ? 1 : 0);
      const float* pd = xp + (hd ? -kJacEX : 0);
      const float* pu = xp + (hu ? kJacEX : 0);
      const float* pb = xp + (hb ? -C : 0);
      const float* pa = xp + (ha ? H * C : (H - 1) * C);
#pragma unroll
      for (int i = 0; i < H; ++i) xp[i * C] = x[i];
      __syncthreads();
      const bool acc = last_phase && j == ns - 1 && inner;
      float xn[H];
#pragma unroll
      for (int i = 0; i < H; ++i) {
        const int k = k0 + i;
        const float v = x[i];
        const float xl = pl[i * C];
        const float xr = pr[i * C];
        const float xd = pd[i * C];
        const float xu = pu[i * C];
        const float xb = i > 0 ? x[i - 1] : pb[0];
        const float xa = i + 1 < H ? x[i + 1] : pa[0];
        float s = cxm[i] * (v - xl);
        s += cxp[i] * (v - xr);
        s += cym[i] * (v - xd);
        s += cyp[i] * (v - xu);
        s += (i > 0 ? cz[i - 1] : czb) * (v - xb);
        s += cz[i] * (v - xa);
        if (k == nz - 1) s += S.sb * v;
        const float bi = bp[i * C];
        const float r = bi - (v + s);
        xn[i] = v + r * rp[i * C];
        if (acc && k < nz) {
          vb += (double)bi * (double)bi;
          vr += (double)r * (double)r;
        }
      }
      __syncthreads();                      // every read of this exchange done before the next
#pragma unroll
      for (int i = 0; i < H; ++i) x[i] = xn[i];
    }
    stamp();
    if (last_phase) {
      if (inner) {
#pragma unroll
        for (int i = 0; i < H; ++i)
          if (k0 + i < nz) st_dev(V.x + base + i * nxy, x[i]);
      }
      double v2[2] = {vb, vr};
      ok &= team_sum_dev<2, kJacBlock>(S, rank, red, v2, rs);
      bb = v2[0];
      rr = v2[1];
    } else if (inner) {
      const unsigned long long tag = (unsigned long long)(V.jtag + (unsigned)ph) << 32;
      unsigned long long* dst = S.jt[ph & 1];
#pragma unroll
      for (int i = 0; i < H; ++i)
        if (k0 + i < nz)
          __hip_atomic_store(dst + base + i * nxy, tag | __float_as_uint(x[i]), __ATOMIC_RELAXED,
                             __HIP_MEMORY_SCOPE_AGENT);
    }
    stamp();
  }
  if (!ok && threadIdx.x == 0) atomicOr(S.err_flag, (int)kTimeout);
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");   // the gradient pass reads x with plain loads
  return step_epilogue<float>(S, V, rank, ok, ok ? K : 0, kOk, bb, rr, sh);
}

template <int H>
__global__ void __launch_bounds__(kJacBlock, 1) jacobi_step_kernel(StepArgs<float> S) {
  __shared__ Smem<float> sh;
  __shared__ ResRed rs;
  __shared__ float xs[2 * H * kJacCols];
  __shared__ float bs[2 * H * kJacCols];
  __shared__ float rds[2 * H * kJacCols];
  jacobi_tb_step<H>(S, step_var(S), blockIdx.x, xs, bs, rds, sh, &rs);
}

// Several consecutive steps of one sweep in one launch: step i takes its
// per-step fields from tab.v[i] (the rest of S is the same for all of them).
// Each step ends with a team reduction and an acquire fence, so the next
// step reads its predecessor's state complete; the host gives step i the
// epoch base B + i with B even, so consecutive steps' reductions alternate
// between the two slot banks and a workgroup one step ahead never
// overwrites a slot another still reads. This saves the ~25 us between two
// cooperative launches per step.
constexpr int kJacBatch = 12;               // steps per launch (their fields travel as kernel arguments)

struct JacSteps {
  StepVar<float> v[kJacBatch];
  int count;
};

template <int H>
__global__ void __launch_bounds__(kJacBlock, 1) jacobi_steps_kernel(StepArgs<float> S, JacSteps tab) {
  __shared__ Smem<float> sh;
  __shared__ ResRed rs;
  __shared__ float xs[2 * H * kJacCols];
  __shared__ float bs[2 * H * kJacCols];
  __shared__ float rds[2 * H * kJacCols];
  for (int i = 0; i < tab.count; ++i) jacobi_tb_step<H>(S, tab.v[i], blockIdx.x, xs, bs, rds, sh, &rs);
}

}  // namespace nh
