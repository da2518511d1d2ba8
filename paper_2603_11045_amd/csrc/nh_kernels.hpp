// nh_kernels.hpp -- gfx950 kernels of the implicit-Euler heat solver and its
// discrete adjoint (the paper's Sec. 4.2-4.3, App. D.2-D.3).
//
// One cooperative launch performs one time step of one problem: the residual
// set-up, every Jacobi-preconditioned CG iteration until convergence, and the
// step's epilogue (surface frame and checkpoint in the forward sweep, the
// gradient accumulation in the adjoint sweep). The workgroups of a launch form
// a "team" that synchronises only through FP64 reductions: every workgroup
// publishes its partial sums in a slot of its own, one master workgroup waits
// for all slots, sums them in a fixed order and publishes the result. No
// read-modify-write atomics are involved (no contention on one address, which
// grows linearly with the team), every workgroup receives the same bits, and a
// rerun is bit-identical.
//
// CG in the form used here (M = diag(A), the Jacobi preconditioner of
// App. D.2, as a preconditioner instead of as the solver):
//   set-up    r = b - A x,  z = r / D,  bb = |b|^2, rz = r.z, rr = |r|^2
//   phase A   p = z + beta p  (beta = 0 first),  w = A p,  pw = p.w
//   phase B   a = rz / pw,  x += a p,  z -= a (A p) / D,  rz = D z.z, rr = |D z|^2
// until rr <= rtol^2 bb. Only z is stored (r = D z); A p is recomputed in
// phase B instead of being stored, and D comes from alpha in-kernel, so an
// iteration moves 40 bytes per voxel in FP32. That is variant 0; the default
// is the single-reduction form of the same iteration (FusedOp below: one
// sweep and one team reduction per iteration).
//
// The stencil is evaluated by marching a 2-D tile of (x, y) columns along z:
// each z plane of the staged vectors and of 1/alpha, with its one-cell halo in
// x and y, goes through LDS with x-contiguous (coalesced) loads, while the
// +-z neighbours of a column stay in registers. Cells outside the grid read
// alpha = 0, staged as 1/alpha = +inf, which makes their harmonic-mean
// conductance 0: the zero-flux boundary needs no special case.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace nh {

// Threads per workgroup: 1024 (16 wave64, one workgroup per CU) for the
// FP32 path, 512 for the FP64 path, whose kernel needs more registers.
template <typename R> struct Cfg;
template <> struct Cfg<float> { static constexpr int kBlock = 1024; };
template <> struct Cfg<double> { static constexpr int kBlock = 512; };
constexpr int kMaxBlock = 1024;
constexpr int kMaxWaves = kMaxBlock / 64;
constexpr int kMaxPlane = 1188;             // max (TX+2)*(TY+2) with TX*TY <= 1024: 66*18
constexpr int kNumRed = 4;                  // doubles per workgroup partial slot
constexpr int kChebMax = 16;                // highest degree of the Chebyshev preconditioner

// Coefficients of Chebyshev step k = 1, 2, ... from rho_{k-1} (rho_0 = 1 / sigma):
// rho_k = 1 / (2 sigma - rho_{k-1}), c1 = rho_k rho_{k-1}, c2 = 2 rho_k / delta.
// The host and every workgroup evaluate the same FP64 recurrence.
__host__ __device__ __forceinline__ void cheb_coef(double sigma, double delta, double& rho, double& c1,
                                                   double& c2) {
  const double rn = 1.0 / (2.0 * sigma - rho);
  c1 = rn * rho;
  c2 = 2.0 * rn / delta;
  rho = rn;
}

enum StepMode : int { kForward = 0, kAdjoint = 1 };
enum StepStatus : int { kOk = 0, kNoConv = 1, kNonFinite = 2, kTimeout = 4 };

struct Geom {
  int nx, ny, nz;
  int TX, TY, TZ, txs;                      // tile extents, txs = log2(TX)
  int ntx, nty, ntz, ntiles;
  long long nxy, ng;
  int periodic;                             // 1: the lateral x and y faces wrap around (nx, ny >= 3)
};

template <typename R>
struct StepArgs {
  Geom g;
  R sx, sy, sz;                             // 2 dt / h_d^2 per axis
  R sb;                                     // dt beta: Robin sink of the back plane k = nz-1 (0: adiabatic)
  const R* alpha;
  R* x;                                     // the unknown, solved in place
  const R* xprev;                           // the previous state h1: T^{n-1} or mu^{n+1} (null = zero)
  const R* xprev2;                          // h2, h3: the two states before it, for the initial guess
  const R* xprev3;                          //   (guess_order)
  int gmode;                                // initial guess: extrapolation order 0, 1 or 2; or -1: the order
  const int* gi;                            //   whose probe step gi[gp[order]] took the fewest iterations
  int gp[3];                                //   (earlier steps of the same sweep)
  R* z;                                     // preconditioned residual
  R* p0;                                    // search direction, ping-pong pair
  R* p1;
  R* u1;                                    // single-reduction variant: second u buffer,
  R* w0;                                    //   A u / D and A p / D ping-pong pairs
  R* w1;
  R* s0;
  R* s1;
  R* xface;                                 // resident kernel: compact x-edge columns (nh_resident.hpp)
  int variant;                              // 0: two reductions per iteration, 1: one
  int jacobi_k;                             // > 0: K Jacobi sweeps from h1 instead of CG
  int jtx, jty;                             // temporally blocked fixed-K kernel: interior tiles per axis,
  unsigned long long* jt[2];                //   its tagged iterate buffers (value | tag << 32) and the
  unsigned jtag;                            //   tag of this launch's first phase
  const R* top_src;                         // [ny][nx] added on k = 0 (forward q_xy, adjoint g^n)
  R top_scale;                              // forward dt*q_t[n-1], adjoint 1
  R* surf_out;                              // frame of the solution on k = 0 (or null), times
  R surf_scale;                             //   surf_scale in the adjoint (dt: dL/dq^n = dt mu^n)
  R* ckpt_out;                              // forward: copy of T^n (or null)
  const R* T_grad;                          // adjoint: T^n for the gradient (or null)
  double* G;                                // adjoint: dL/dalpha accumulator
  void* slots;                              // [team + 1] Slot: per-workgroup partials, then the result
  unsigned long long epoch_base;            // unique per launch; each reduction uses epoch_base + k
  double rtol2;
  int max_iter;
  int mode;
  int team;
  int xcd_order;                            // 1: give each XCD a contiguous range of tiles
  int* out_iters;                           // per-step outputs written by rank 0
  double* out_relres;
  int* out_status;
  int* err_flag;                            // |= kTimeout by any workgroup whose wait timed out
  long long timeout_ticks;                  // barrier time limit in wall-clock ticks
  long long* trace;                         // optional: wall-clock stamps of phase ends
  int trace_rank;                           // workgroup whose thread 0 writes the stamps
  int trace_cap;                            // capacity of trace in entries
  int trace_detail;                         // resident kernel: extra stamps inside an iteration
  // Chebyshev polynomial preconditioner of the two-reduction form (cheb_m >= 2;
  // 1 = plain Jacobi): y_1 = cheb_s z, y_{k+1} = y_k + c1_k (y_k - y_{k-1})
  // + c2_k (z - A y_k / D) for k = 1..cheb_m-1, z = r / D, with c1_k, c2_k
  // from cheb_sigma and cheb_delta (cheb_coef). y_j lives in cheb_y0 (j even)
  // or cheb_y1 (j odd). (Scalars only: a kernel argument indexed at run time
  // would be copied to scratch memory.)
  int cheb_m;
  R cheb_s;
  double cheb_sigma, cheb_delta;
  R* cheb_y0;
  R* cheb_y1;
};

// ---------------------------------------------------------------------------
// arithmetic helpers

template <typename R> __device__ __forceinline__ R rcp(R v);
template <> __device__ __forceinline__ float rcp<float>(float v) { return __builtin_amdgcn_rcpf(v); }
template <> __device__ __forceinline__ double rcp<double>(double v) { return 1.0 / v; }

// Store of a sweep output: device-scope (write-through), so the team barrier's
// L2 write-back finds little dirty data. (Non-temporal stores were measured
// slower: they bypass the last-level cache that the next sweep reads from.)
template <typename T>
__device__ __forceinline__ void st_out(T* p, T v) {
  __hip_atomic_store((__attribute__((address_space(1))) T*)p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// A product and a sum rounded on their own, never fused into a multiply-add
// (where two kernels must produce the same bits, the contraction must not
// depend on how each compiles).
template <typename R>
__device__ __forceinline__ R mul_rn(R a, R b) {
#pragma clang fp contract(off)
  return a * b;
}
template <typename R>
__device__ __forceinline__ R add_rn(R a, R b) {
#pragma clang fp contract(off)
  return a + b;
}
// a * b + c with one rounding, in the precision of R
template <typename R> __device__ __forceinline__ R fma_r(R a, R b, R c);
template <> __device__ __forceinline__ float fma_r<float>(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
template <> __device__ __forceinline__ double fma_r<double>(double a, double b, double c) { return __builtin_fma(a, b, c); }

// dt * c_f = s * a*b/(a+b) with s = 2 dt / h^2 (Prop. 1); b = 0 outside the grid gives 0.
template <typename R>
__device__ __forceinline__ R face(R s, R a, R b) { return s * (a * b) * rcp<R>(a + b); }

// The step kernels stage 1/alpha instead of alpha (a cell outside the grid,
// read as 0, becomes +inf) and write the face term as s times the face
// weight 1/(1/a + 1/b) = a*b/(a+b): one addition and one reciprocal per face,
// and a face towards an absent cell weighs 1/inf = 0.
template <typename R>
__device__ __forceinline__ R inv_alpha(R a) { return rcp<R>(a); }
template <typename R>
__device__ __forceinline__ R face_w(R ia, R ib) { return rcp<R>(ia + ib); }

// D = 1 + sx (w0 + w1) + sy (w2 + w3) + sz (w4 + w5) and
// A v = v + sum over the axes of s_d (w_- (v - v_-) + w_+ (v - v_+)), from
// the face weights w (-x +x -y +y -z +z) and the neighbour values n, every
// rounding written out: kernels that stage the same values obtain the same
// bits however each compiles.
template <typename R>
__device__ __forceinline__ R diag_w(R sx, R sy, R sz, const R (&w)[6]) {
  R d = fma_r(sx, add_rn(w[0], w[1]), R(1));
  d = fma_r(sy, add_rn(w[2], w[3]), d);
  return fma_r(sz, add_rn(w[4], w[5]), d);
}
template <typename R>
__device__ __forceinline__ R apply_w(R sx, R sy, R sz, const R (&w)[6], R v, const R (&n)[6]) {
  const R gx = fma_r(w[1], v - n[1], mul_rn(w[0], v - n[0]));
  const R gy = fma_r(w[3], v - n[3], mul_rn(w[2], v - n[2]));
  const R gz = fma_r(w[5], v - n[5], mul_rn(w[4], v - n[4]));
  return fma_r(sz, gz, fma_r(sy, gy, fma_r(sx, gx, v)));
}

// The diagonal of A: 1 + the six face terms (+ the sink term), summed in this
// order (kernels that take the face terms one by one).
template <typename R>
__device__ __forceinline__ R diag_of(R c0, R c1, R c2, R c3, R c4, R c5) {
  return R(1) + (((c0 + c1) + (c2 + c3)) + (c4 + c5));
}
template <typename R>
__device__ __forceinline__ R diag_of(R c0, R c1, R c2, R c3, R c4, R c5, R sk) {
  return R(1) + ((((c0 + c1) + (c2 + c3)) + (c4 + c5)) + sk);
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// ---------------------------------------------------------------------------
// team reduction slots

struct alignas(64) Slot {
  double v[kNumRed];
  unsigned long long epoch;
  unsigned long long pad[3];
};

__device__ __forceinline__ unsigned long long ld_epoch(const unsigned long long* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ double ld_val(const double* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Shared state of one workgroup: two buffers of a staged plane (1/alpha and up
// to two vectors; march_tile alternates them), and red, two buffers of
// per-wave partial sums, which the two block sums of a team reduction use in
// turn.
template <typename R>
struct Smem {
  R a[2][kMaxPlane];
  R v[2][2][kMaxPlane];
  double red[2][kMaxWaves][kNumRed];
  double bc[kNumRed];
  int flag;
};

// Sum NV doubles over the workgroup of WAVES wave64; the result lands in every
// thread's v. Each wave sums its lanes with a butterfly; after one barrier
// every wave loads the waves' sums (lane w holds wave w's) and sums them with
// the same butterfly, so all threads hold the same bits. red must not be
// written again before every thread has passed the next workgroup barrier:
// callers alternate two buffers between consecutive block sums, with a
// barrier in each.
template <int NV, int WAVES>
__device__ __forceinline__ void block_sum(double (&v)[NV], double (*red)[kNumRed]) {
  static_assert(WAVES <= 64, "one lane per wave");
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int i = 0; i < NV; ++i) v[i] = wave_sum(v[i]);
  if (lane == 0) {
#pragma unroll
    for (int i = 0; i < NV; ++i) red[wave][i] = v[i];
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < NV; ++i) v[i] = wave_sum(lane < WAVES ? red[lane][i] : 0.0);
}

// Team all-reduce of NV doubles; also the team's barrier. Every workgroup
// stores its workgroup sum in its slot and releases it with the epoch of this
// reduction (the release also publishes the workgroup's earlier global
// stores). The master (rank 0) waits for every slot, sums the slots in rank
// order with a fixed reduction tree, and releases the result slot; the other
// workgroups wait for that. Waits are bounded by timeout_ticks; a timeout
// returns false and is recorded in err_flag.
template <typename R, int NV, int BLOCK = Cfg<R>::kBlock>
__device__ __forceinline__ bool team_sum(const StepArgs<R>& S, int rank, unsigned long long& epoch,
                                         double (&v)[NV], Smem<R>& sh) {
  // every wave's sweep stores (device-coherent) complete before the workgroup
  // publishes its slot: the slot's release orders only the wave that writes it
  __builtin_amdgcn_s_waitcnt(0);
  block_sum<NV, BLOCK / 64>(v, sh.red[0]);
  if (S.team == 1) {
    __syncthreads();                        // red[0] is free again
    return true;
  }
  const unsigned long long e = ++epoch;
  Slot* slots = (Slot*)S.slots;
  Slot* res = slots + S.team;
  int ok = 1;
  if (rank != 0) {
    if (threadIdx.x == 0) {
#pragma unroll
      for (int i = 0; i < NV; ++i)
        __hip_atomic_store(&slots[rank].v[i], v[i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_store(&slots[rank].epoch, e, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
      const long long t0 = wall_clock64();
      while (ld_epoch(&res->epoch) != e) {
        __builtin_amdgcn_s_sleep(2);
        if (wall_clock64() - t0 > S.timeout_ticks) { ok = 0; break; }
      }
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
#pragma unroll
      for (int i = 0; i < NV; ++i) sh.bc[i] = ld_val(&res->v[i]);
      sh.flag = ok;
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < NV; ++i) v[i] = sh.bc[i];
    ok = sh.flag;
    __syncthreads();
  } else {
    double s[NV];
#pragma unroll
    for (int i = 0; i < NV; ++i) s[i] = 0.0;
    for (int b = threadIdx.x; b < S.team; b += BLOCK) {
      if (b == 0) {
#pragma unroll
        for (int i = 0; i < NV; ++i) s[i] += v[i];
        continue;
      }
      const long long t0 = wall_clock64();
      while (ld_epoch(&slots[b].epoch) != e) {
        __builtin_amdgcn_s_sleep(1);
        if (wall_clock64() - t0 > S.timeout_ticks) { ok = 0; break; }
      }
#pragma unroll
      for (int i = 0; i < NV; ++i) s[i] += ld_val(&slots[b].v[i]);
    }
    ok = __syncthreads_and(ok);
    block_sum<NV, BLOCK / 64>(s, sh.red[1]);
    if (threadIdx.x == 0) {
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
#pragma unroll
      for (int i = 0; i < NV; ++i)
        __hip_atomic_store(&res->v[i], s[i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_store(&res->epoch, e, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < NV; ++i) v[i] = s[i];
  }
  if (!ok && threadIdx.x == 0) atomicOr(S.err_flag, (int)kTimeout);
  return ok != 0;
}

// ---------------------------------------------------------------------------
// tiles

struct Tile {
  int x0, y0, z0, z1;
};

__device__ __forceinline__ Tile tile_of(const Geom& g, int t) {
  const int itz = t % g.ntz;
  const int rest = t / g.ntz;
  const int itx = rest % g.ntx;
  const int ity = rest / g.ntx;
  Tile T;
  T.x0 = itx * g.TX;
  T.y0 = ity * g.TY;
  T.z0 = itz * g.TZ;
  T.z1 = min(T.z0 + g.TZ, g.nz);
  return T;
}

// Workgroup rank -> first tile. With xcd_order the ranks that the hardware
// places on one XCD (rank % 8, dispatch is round-robin over the 8 XCDs) get a
// contiguous tile range, so most halo reads hit that XCD's L2.
__device__ __forceinline__ int first_tile(int rank, int team, int xcd_order) {
  if (xcd_order && (team & 7) == 0) return (rank & 7) * (team >> 3) + (rank >> 3);
  return rank;
}

// The operator's coefficients: 2 dt / h_d^2 per axis, and the Robin sink
// dt beta that the rows of the plane zb (the back face) carry.
template <typename R>
struct Coef {
  R sx, sy, sz, sb;
  int zb;
};

template <typename R>
__device__ __forceinline__ Coef<R> coef_of(const StepArgs<R>& S) {
  return Coef<R>{S.sx, S.sy, S.sz, S.sb, S.g.nz - 1};
}

// Stencil values of one cell: index 0 centre, 1 -x, 2 +x, 3 -y, 4 +y, 5 -z,
// 6 +z; a holds 1/alpha (+inf outside the grid).
template <typename R, int NV>
struct Pt {
  R a[7];
  R v[NV][7];
};

// A load through a global (not flat) pointer.
template <typename T>
__device__ __forceinline__ T gld(const T* p, long long i) {
  return ((const __attribute__((address_space(1))) T*)p)[i];
}

// Buffer loads of one z plane of a vector. The resource covers the plane
// (base p + zp nxy, nxy elements); a lane whose byte offset is kOffLane, a
// null vector and a plane outside the range asked for all read 0, so the
// plane loads need neither branches nor zero fills.
constexpr unsigned kOffLane = 0x80000000u;

template <typename T>
__device__ __forceinline__ __amdgpu_buffer_rsrc_t plane_rsrc(const T* p, long long zp, long long nxy, bool valid) {
  valid = valid && p != nullptr;
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<T*>(p) + (valid ? zp * nxy : 0), 0,
                                           valid ? (int)(nxy * (long long)sizeof(T)) : 0, 0x00020000);
}
template <typename T>
__device__ __forceinline__ T plane_ld(__amdgpu_buffer_rsrc_t r, unsigned off);
template <>
__device__ __forceinline__ float plane_ld<float>(__amdgpu_buffer_rsrc_t r, unsigned off) {
  return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 0));
}
template <>
__device__ __forceinline__ double plane_ld<double>(__amdgpu_buffer_rsrc_t r, unsigned off) {
  const auto v = __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0);
  return __hiloint2double((int)v[1], (int)v[0]);
}

// March one tile along z. Op supplies: NL vectors loaded at the staged cells
// (raw_ptr(k); null reads 0), combined into the NV staged vectors by
// stage(raw, v) when a plane is staged; NO operands of type OT read at the
// cell itself (own_ptr(k)); alpha; and point(P, rc, o, i, kz), which also
// receives the cell's raw values rc. Loads are issued Op::PD planes ahead
// of their use; all queues are rings of Q plane slots with compile-time slot
// numbers (the z loop is unrolled Q times), so no register moves, which would
// wait for loads in flight, rotate them. Arithmetic on loaded values happens
// in stage and point, once the data is needed. The set-up and gradient
// operators, which run once per step and hold the most values per plane,
// prefetch one plane less (their rings would not fit the registers).
constexpr int kPrefetch = 3;

template <typename R, typename Op>
__device__ __forceinline__ void march_tile(const Geom& g, const Tile& T, Op& op, Smem<R>& sh) {
  constexpr int NV = Op::NV;
  constexpr int NL = Op::NL;
  constexpr int NO = Op::NO > 0 ? Op::NO : 1;
  constexpr int PD = Op::PD;
  constexpr int Q = PD + 2;                 // plane slots: z-1 .. z+PD
  using OT = typename Op::OT;
  // the lane's geometry is recomputed in every call (laundered): hoisted out
  // of a caller's iteration loop it would hold registers through the solve
  int tid = threadIdx.x;
  asm volatile("" : "+v"(tid));
  const int TX = g.TX, TY = g.TY, PW = TX + 2;
  const int tx = tid & (TX - 1), ty = tid >> g.txs;
  const int gx = T.x0 + tx, gy = T.y0 + ty;
  const bool own = gx < g.nx && gy < g.ny;
  const long long col = own ? (long long)gx + (long long)g.nx * gy : 0;
  const int oslot = (ty + 1) * PW + tx + 1;
  // the column this thread stages: its own; with periodic lateral faces a
  // thread past the grid edge stages the column across the wrap instead
  const bool ld = own || g.periodic;
  const long long lcol = own ? col : (g.periodic ? (long long)(gx % g.nx) + (long long)g.nx * (gy % g.ny) : 0);

  // the halo cell this thread stages (perimeter of the TX x TY tile)
  int hslot = -1;
  bool hin = false;
  long long hcol = 0;
  {
    int h = tid, hx = 0, hy = 0;
    if (h < TX) { hx = T.x0 + h; hy = T.y0 - 1; hslot = h + 1; }
    else if ((h -= TX) < TX) { hx = T.x0 + h; hy = T.y0 + TY; hslot = (TY + 1) * PW + h + 1; }
    else if ((h -= TX) < TY) { hx = T.x0 - 1; hy = T.y0 + h; hslot = (h + 1) * PW; }
    else if ((h -= TY) < TY) { hx = T.x0 + TX; hy = T.y0 + h; hslot = (h + 1) * PW + TX + 1; }
    if (hslot >= 0) {
      if (g.periodic) {                     // hx, hy >= -1
        hx = (hx + g.nx) % g.nx;
        hy = (hy + g.ny) % g.ny;
      }
      hin = hx >= 0 && hx < g.nx && hy >= 0 && hy < g.ny;
      if (hin) hcol = (long long)hx + (long long)g.nx * hy;
    }
  }
  const unsigned vcol = ld ? (unsigned)lcol * (unsigned)sizeof(R) : kOffLane;
  const unsigned vhalo = hin ? (unsigned)hcol * (unsigned)sizeof(R) : kOffLane;
  const unsigned vown = own ? (unsigned)col * (unsigned)sizeof(OT) : kOffLane;

  // rings; plane zp sits in slot (zp - (z0 - 1)) mod Q
  R qa[Q], ql[Q][NL];                       // staged column: alpha (1/alpha once staged), raw values
  R qv[Q][NV];                              // staged column: staged vectors
  R ha[Q], hl[Q][NL];                       // halo cell: alpha, raw values (staged as 1/alpha)
  OT qo[Q][NO];                             // own operands
  // staged column of plane zp (inside the grid)
  auto load_col = [&](int s, int zp) {
    const bool v = zp >= 0 && zp < g.nz;
    qa[s] = plane_ld<R>(plane_rsrc(op.alpha, zp, g.nxy, v), vcol);
#pragma unroll
    for (int k = 0; k < NL; ++k) ql[s][k] = plane_ld<R>(plane_rsrc(op.raw_ptr(k), zp, g.nxy, v), vcol);
  };
  // own operands and halo cell of plane zp (inside the tile)
  auto load_cell = [&](int s, int zp) {
    const bool v = zp < T.z1;
#pragma unroll
    for (int k = 0; k < NO; ++k)
      qo[s][k] = k < Op::NO ? plane_ld<OT>(plane_rsrc(op.own_ptr(k), zp, g.nxy, v), vown) : OT(0);
    const __amdgpu_buffer_rsrc_t ra = plane_rsrc(op.alpha, zp, g.nxy, v);
    ha[s] = plane_ld<R>(ra, vhalo);
#pragma unroll
    for (int k = 0; k < NL; ++k) hl[s][k] = plane_ld<R>(plane_rsrc(op.raw_ptr(k), zp, g.nxy, v), vhalo);
  };
  // fill: staged column z0-1 .. z0+PD-1, own operands and halo z0 .. z0+PD-1
#pragma unroll
  for (int j = 0; j < Q - 1; ++j) load_col(j, T.z0 - 1 + j);
#pragma unroll
  for (int j = 0; j < PD; ++j) load_cell(j + 1, T.z0 + j);
  op.stage(ql[0], qv[0]);
  op.stage(ql[1], qv[1]);
  qa[0] = inv_alpha<R>(qa[0]);
  qa[1] = inv_alpha<R>(qa[1]);

  for (int zb = T.z0; zb < T.z1; zb += Q) {
#pragma unroll
    for (int u = 0; u < Q; ++u) {
      const int z = zb + u;
      if (z >= T.z1) break;
      const int sm = u % Q, s0 = (u + 1) % Q, sp = (u + 2) % Q, sn = (u + Q - 1) % Q;
      // issue the loads of plane z+PD into the slot plane z-2 has left
      load_col(sn, z + PD);
      load_cell(sn, z + PD);

      // planes alternate between two LDS buffers, so one barrier per plane
      // suffices: a buffer is written again two planes later, after the next
      // plane's barrier, which every wave passes only once it has finished
      // reading this plane
      const int bf = (z - T.z0) & 1;
      R* la = sh.a[bf];
      R (*lv)[kMaxPlane] = sh.v[bf];
      la[oslot] = qa[s0];
#pragma unroll
      for (int k = 0; k < NV; ++k) lv[k][oslot] = qv[s0][k];
      if (hslot >= 0) {
        R hv[NV];
        op.stage(hl[s0], hv);
        la[hslot] = inv_alpha<R>(ha[s0]);
#pragma unroll
        for (int k = 0; k < NV; ++k) lv[k][hslot] = hv[k];
      }
      op.stage(ql[sp], qv[sp]);             // plane z+1: the +z neighbour now, staged next
      qa[sp] = inv_alpha<R>(qa[sp]);
      __syncthreads();

      if (own) {
        Pt<R, NV> P;
        P.a[0] = qa[s0];
        P.a[1] = la[oslot - 1];
        P.a[2] = la[oslot + 1];
        P.a[3] = la[oslot - PW];
        P.a[4] = la[oslot + PW];
        P.a[5] = qa[sm];
        P.a[6] = qa[sp];
#pragma unroll
        for (int k = 0; k < NV; ++k) {
          P.v[k][0] = qv[s0][k];
          P.v[k][1] = lv[k][oslot - 1];
          P.v[k][2] = lv[k][oslot + 1];
          P.v[k][3] = lv[k][oslot - PW];
          P.v[k][4] = lv[k][oslot + PW];
          P.v[k][5] = qv[sm][k];
          P.v[k][6] = qv[sp][k];
        }
        op.point(P, ql[s0], qo[s0], col + (long long)z * g.nxy, z);
      }
    }
  }
  __syncthreads();                          // both plane buffers are free for the next tile
}

// A v and the diagonal D of A at one cell, from staged 1/alpha and v (row k
// of P). A cell of the plane kz carries the Robin sink if kz is the back plane.
template <typename R, int NV>
__device__ __forceinline__ void stencil(const Pt<R, NV>& P, int k, const Coef<R>& cf, int kz, R& Av, R& D) {
  R w[6], n[6];
#pragma unroll
  for (int f = 0; f < 6; ++f) {
    w[f] = face_w<R>(P.a[0], P.a[f + 1]);
    n[f] = P.v[k][f + 1];
  }
  Av = apply_w<R>(cf.sx, cf.sy, cf.sz, w, P.v[k][0], n);
  D = diag_w<R>(cf.sx, cf.sy, cf.sz, w);
  if (kz == cf.zb && cf.sb != R(0)) {
    Av = fma_r(cf.sb, P.v[k][0], Av);
    D = add_rn(D, cf.sb);
  }
}

// ---------------------------------------------------------------------------
// phase operators

// Set-up: b = x0 + top source, r = b - A x0, z = r / D.
template <typename R>
struct InitOp {
  static constexpr int PD = kPrefetch - 1;
  static constexpr int NV = 1;
  static constexpr int NL = 3;
  static constexpr int NO = 0;
  using OT = R;
  const R* alpha;
  const R* src;                             // the previous state h1 (null = zero state)
  const R* h2;                              // with h2 (and h3) the staged x0 extrapolates:
  const R* h3;                              //   x0 = e1 h1 + (e2 h2 + h3); else x0 = h1
  R e1, e2;
  R* xw;                                    // x to initialise with x0 (null = already there)
  R* z;
  const R* top;
  R top_scale;
  Coef<R> cf;
  long long nxy;
  double acc[3];                            // |b|^2, r.z, |r|^2
  // raw: h1, h2, h3 (each 0 where absent)
  __device__ const R* raw_ptr(int k) const { return k == 0 ? src : (k == 1 ? h2 : h3); }
  __device__ void stage(const R (&r)[3], R (&v)[1]) const {
    if (!src) { v[0] = R(0); return; }
    if (!h2) { v[0] = r[0]; return; }
    R t = mul_rn(e2, r[1]);
    if (h3) t = add_rn(t, r[2]);
    v[0] = fma(e1, r[0], t);
  }
  __device__ const R* own_ptr(int) const { return nullptr; }
  __device__ void point(const Pt<R, 1>& P, const R (&rc)[3], const R (&)[1], long long i, int kz) {
    R Av, D;
    stencil<R, 1>(P, 0, cf, kz, Av, D);
    R b = h2 ? rc[0] : P.v[0][0];     // the right-hand side's previous state h1
    if (kz == 0) b += top_scale * top[i];
    const R r = b - Av;
    const R zz = r * rcp<R>(D);
    st_out(z + i, zz);
    if (xw) st_out(xw + i, P.v[0][0]);
    const double bd = b, rd = r;
    acc[0] += bd * bd;
    acc[1] += rd * (double)zz;
    acc[2] += rd * rd;
  }
};

// One step of the Chebyshev iteration for D^-1 A y = z from y_0 = 0 over an
// interval [a, b] of the spectrum of D^-1 A (Y. Saad, Iterative
// Methods for Sparse Linear Systems, 2nd ed., Alg. 12.1, in its three-term
// form):  y_{k+1} = y_k + c1 (y_k - y_{k-1}) + c2 (z - A y_k / D).  y_1 = s z
// and y_0 = 0 are not stored: yk == null stages s z, ykm1 == null gives 0
// (k = 1) or s z (k = 2). The last step also accumulates r . y_m = (D z) . y_m.
template <typename R>
struct ChebOp {
  static constexpr int PD = kPrefetch;
  static constexpr int NV = 1;
  static constexpr int NL = 1;
  static constexpr int NO = 2;
  using OT = R;
  const R* alpha;
  const R* z;
  const R* yk;
  const R* ykm1;
  R* ynext;
  R s, c1, c2;
  int k;
  int last;
  Coef<R> cf;
  double acc[1];
  __device__ const R* raw_ptr(int) const { return yk ? yk : z; }
  __device__ void stage(const R (&r)[1], R (&v)[1]) const { v[0] = yk ? r[0] : s * r[0]; }
  __device__ const R* own_ptr(int j) const { return j == 0 ? z : ykm1; }
  __device__ void point(const Pt<R, 1>& P, const R (&)[1], const R (&o)[2], long long i, int kz) {
    R Ay, D;
    stencil<R, 1>(P, 0, cf, kz, Ay, D);
    const R y = P.v[0][0];
    const R ym = ykm1 ? o[1] : (k == 1 ? R(0) : s * o[0]);
    const R yn = y + c1 * (y - ym) + c2 * (o[0] - Ay * rcp<R>(D));
    st_out(ynext + i, yn);
    if (last) acc[0] += ((double)D * (double)o[0]) * (double)yn;
  }
};

// Phase A: p_new = z + beta p_old, w = A p_new, accumulate p_new . w.
template <typename R>
struct DirOp {
  static constexpr int PD = kPrefetch;
  static constexpr int NV = 1;
  static constexpr int NL = 2;
  static constexpr int NO = 0;
  using OT = R;
  const R* alpha;
  const R* z;
  const R* pold;
  R* pnew;
  R beta;
  int first;
  Coef<R> cf;
  double acc[1];
  __device__ const R* raw_ptr(int k) const { return k == 0 ? z : (first ? nullptr : pold); }
  __device__ void stage(const R (&r)[2], R (&v)[1]) const { v[0] = first ? r[0] : r[0] + beta * r[1]; }
  __device__ const R* own_ptr(int) const { return nullptr; }
  __device__ void point(const Pt<R, 1>& P, const R (&)[2], const R (&)[1], long long i, int kz) {
    R Av, D;
    stencil<R, 1>(P, 0, cf, kz, Av, D);
    st_out(pnew + i, P.v[0][0]);
    acc[0] += (double)P.v[0][0] * (double)Av;
  }
};

// Phase B: x += a p, z -= a (A p) / D, accumulate r.z = D z^2 and |r|^2 = (D z)^2.
template <typename R>
struct UpdOp {
  static constexpr int PD = kPrefetch;
  static constexpr int NV = 1;
  static constexpr int NL = 1;
  static constexpr int NO = 2;
  using OT = R;
  const R* alpha;
  const R* p;
  R* x;
  R* z;
  R a;
  Coef<R> cf;
  double acc[2];
  __device__ const R* raw_ptr(int) const { return p; }
  __device__ void stage(const R (&r)[1], R (&v)[1]) const { v[0] = r[0]; }
  __device__ const R* own_ptr(int k) const { return k == 0 ? x : z; }
  __device__ void point(const Pt<R, 1>& P, const R (&)[1], const R (&o)[2], long long i, int kz) {
    R Ap, D;
    stencil<R, 1>(P, 0, cf, kz, Ap, D);
    st_out(x + i, o[0] + a * P.v[0][0]);
    const R zn = o[1] - a * (Ap * rcp<R>(D));
    st_out(z + i, zn);
    const double zd = zn, rd = (double)D * zd;
    acc[0] += rd * zd;
    acc[1] += rd * rd;
  }
};

// Adjoint epilogue: G_p -= sum_f s_f (a_q/(a_p+a_q))^2 (T_p-T_q)(mu_p-mu_q),
// s_f = 2 dt / h^2, i.e. G += -dt dc_f/da_p dT dmu (eq. grad_assembly); from
// the staged reciprocals, a_q/(a_p+a_q) = (1/a_p)/(1/a_p + 1/a_q).
template <typename R>
struct GradOp {
  static constexpr int PD = kPrefetch - 1;
  static constexpr int NV = 2;
  static constexpr int NL = 2;
  static constexpr int NO = 1;
  using OT = double;
  const R* alpha;
  const R* mu;
  const R* T;
  double* G;
  double sx, sy, sz;
  __device__ const R* raw_ptr(int k) const { return k == 0 ? mu : T; }
  __device__ void stage(const R (&r)[2], R (&v)[2]) const { v[0] = r[0]; v[1] = r[1]; }
  __device__ const double* own_ptr(int) const { return G; }
  __device__ void point(const Pt<R, 2>& P, const R (&)[2], const double (&o)[1], long long i, int) {
    const double ia = P.a[0], m = P.v[0][0], t = P.v[1][0];
    const double s[7] = {0.0, sx, sx, sy, sy, sz, sz};
    double acc = 0.0;
#pragma unroll
    for (int f = 1; f < 7; ++f) {
      const double w = ia / (ia + (double)P.a[f]);
      acc += s[f] * (w * w) * ((t - (double)P.v[1][f]) * (m - (double)P.v[0][f]));
    }
    st_out(G + i, o[0] - acc);
  }
};

// Single-reduction set-up, second part: w = A u, store w / D, accumulate u.w.
template <typename R>
struct WOp {
  static constexpr int PD = kPrefetch;
  static constexpr int NV = 1;
  static constexpr int NL = 1;
  static constexpr int NO = 0;
  using OT = R;
  const R* alpha;
  const R* u;
  R* what;
  Coef<R> cf;
  double acc[1];
  __device__ const R* raw_ptr(int) const { return u; }
  __device__ void stage(const R (&r)[1], R (&v)[1]) const { v[0] = r[0]; }
  __device__ const R* own_ptr(int) const { return nullptr; }
  __device__ void point(const Pt<R, 1>& P, const R (&)[1], const R (&)[1], long long i, int kz) {
    R w, D;
    stencil<R, 1>(P, 0, cf, kz, w, D);
    st_out(what + i, w * rcp<R>(D));
    acc[0] += (double)P.v[0][0] * (double)w;
  }
};

// One iteration of the single-reduction (Chronopoulos-Gear) form of the
// preconditioned CG, with u = r / D, w = A u and s = A p kept as w/D, s/D:
//   s_i = w_i + b s_{i-1},  p_i = u_i + b p_{i-1},  x += a p_i,
//   u_{i+1} = u_i - a s_i   (staged: needed at the halo for the stencil),
//   w_{i+1} = A u_{i+1};  accumulate u.r = D u^2, u.w and |r|^2 = (D u)^2.
// The next a, b follow from these three sums alone, so an iteration needs a
// single team reduction. x moves every second iteration: xmode 1 leaves it
// (the iteration's a p stays pending), xmode 2 applies the pending term of the
// previous iteration (ap, and p_{i-1} read here anyway) and then its own, in
// that order and each rounded as on its own (the same bits as two updates),
// which saves reading and writing x in every other iteration.
template <typename R>
struct FusedOp {
  static constexpr int PD = kPrefetch;
  static constexpr int NV = 1;
  static constexpr int NL = 3;
  static constexpr int NO = 2;
  using OT = R;
  const R* alpha;
  const R* u;                               // u_i
  const R* wh;                              // w_i / D
  const R* sho;                             // s_{i-1} / D
  R* x;
  R* p;                                     // p_{i-1} in, p_i out
  R* un;                                    // u_{i+1}
  R* whn;                                   // w_{i+1} / D
  R* shn;                                   // s_i / D
  R a, b;
  R ap;                                     // a_{i-1} of the pending update (xmode 2)
  int first;
  int xmode;
  Coef<R> cf;
  double acc[3];
  // raw: u_i, w_i / D, s_{i-1} / D; staged: u_{i+1}
  __device__ const R* raw_ptr(int k) const { return k == 0 ? u : (k == 1 ? wh : (first ? nullptr : sho)); }
  __device__ void stage(const R (&r)[3], R (&v)[1]) const {
    const R sv = first ? r[1] : r[1] + b * r[2];
    v[0] = r[0] - a * sv;
  }
  // own: x (when it moves), p_{i-1}
  __device__ const R* own_ptr(int k) const { return k == 0 ? (xmode == 2 ? x : nullptr) : (first ? nullptr : p); }
  __device__ void point(const Pt<R, 1>& P, const R (&rc)[3], const R (&o)[2], long long i, int kz) {
    const R sv = first ? rc[1] : rc[1] + b * rc[2];
    const R pv = first ? rc[0] : rc[0] + b * o[1];
    if (xmode == 2) st_out(x + i, fma_r(a, pv, fma_r(ap, o[1], o[0])));
    st_out(p + i, pv);
    st_out(shn + i, sv);
    R w, D;
    stencil<R, 1>(P, 0, cf, kz, w, D);
    const R uv = P.v[0][0];
    st_out(un + i, uv);
    st_out(whn + i, w * rcp<R>(D));
    const double ud = uv, Dd = D, rd = Dd * ud;
    acc[0] += rd * ud;
    acc[1] += (double)w * ud;
    acc[2] += rd * rd;
  }
};

// y = A x on its own (operator tests).
template <typename R>
struct ApplyOp {
  static constexpr int PD = kPrefetch;
  static constexpr int NV = 1;
  static constexpr int NL = 1;
  static constexpr int NO = 0;
  using OT = R;
  const R* alpha;
  const R* xin;
  R* y;
  Coef<R> cf;
  __device__ const R* raw_ptr(int) const { return xin; }
  __device__ void stage(const R (&r)[1], R (&v)[1]) const { v[0] = r[0]; }
  __device__ const R* own_ptr(int) const { return nullptr; }
  __device__ void point(const Pt<R, 1>& P, const R (&)[1], const R (&)[1], long long i, int kz) {
    R Av, D;
    stencil<R, 1>(P, 0, cf, kz, Av, D);
    y[i] = Av;
  }
};

// One sweep of the paper's fixed-K inner solver (eq. jacobi_iter):
// x_new = D^-1 (b - R x) = x + (b - A x) / D with b = h1 + the top source;
// accumulates |b|^2 and |b - A x|^2 (the residual of the sweep's input).
template <typename R>
struct JacobiOp {
  static constexpr int PD = kPrefetch;
  static constexpr int NV = 1;
  static constexpr int NL = 1;
  static constexpr int NO = 1;
  using OT = R;
  const R* alpha;
  const R* xin;                             // x^(kappa) (null: zero)
  const R* h1;                              // the previous state in b (null: zero)
  R* xout;                                  // x^(kappa+1)
  const R* top;
  R top_scale;
  Coef<R> cf;
  double acc[2];
  __device__ const R* raw_ptr(int) const { return xin; }
  __device__ void stage(const R (&r)[1], R (&v)[1]) const { v[0] = r[0]; }
  __device__ const R* own_ptr(int) const { return h1; }
  __device__ void point(const Pt<R, 1>& P, const R (&)[1], const R (&o)[1], long long i, int kz) {
    R Av, D;
    stencil<R, 1>(P, 0, cf, kz, Av, D);
    R b = o[0];
    if (kz == 0) b += top_scale * top[i];
    const R r = b - Av;
    st_out(xout + i, P.v[0][0] + r * rcp<R>(D));
    const double bd = b, rd = r;
    acc[0] += bd * bd;
    acc[1] += rd * rd;
  }
};

template <typename R, typename Op>
__device__ __forceinline__ void sweep(const Geom& g, int rank, int team, int xcd, Op& op, Smem<R>& sh) {
  for (int t = first_tile(rank, team, xcd); t < g.ntiles; t += team) {
    const Tile T = tile_of(g, t);
    march_tile<R, Op>(g, T, op, sh);
  }
}

// Own cells of the workgroup's tiles (no stencil): fn(i, col, kz).
template <typename F>
__device__ __forceinline__ void own_cells(const Geom& g, int rank, int team, int xcd, F fn) {
  const int tx = threadIdx.x & (g.TX - 1), ty = threadIdx.x >> g.txs;
  for (int t = first_tile(rank, team, xcd); t < g.ntiles; t += team) {
    const Tile T = tile_of(g, t);
    const int gx = T.x0 + tx, gy = T.y0 + ty;
    if (gx >= g.nx || gy >= g.ny) continue;
    const long long col = (long long)gx + (long long)g.nx * gy;
    for (int z = T.z0; z < T.z1; ++z) fn(col + (long long)z * g.nxy, col, z);
  }
}

// Top-plane cells (k = 0) of the workgroup's tiles: fn(col).
template <typename F>
__device__ __forceinline__ void top_cells(const Geom& g, int rank, int team, int xcd, F fn) {
  const int tx = threadIdx.x & (g.TX - 1), ty = threadIdx.x >> g.txs;
  for (int t = first_tile(rank, team, xcd); t < g.ntiles; t += team) {
    const Tile T = tile_of(g, t);
    if (T.z0 != 0) continue;
    const int gx = T.x0 + tx, gy = T.y0 + ty;
    if (gx >= g.nx || gy >= g.ny) continue;
    fn((long long)gx + (long long)g.nx * gy);
  }
}

// ---------------------------------------------------------------------------
// one implicit-Euler step (forward or adjoint) for one team

// What every workgroup of the team knows after a step: the iteration count
// and the flags that follow from reduced values are the same on all of them;
// kTimeout is set only where a wait of this workgroup timed out.
struct StepResult {
  int iters;
  int status;
  double relres;                            // ||r|| / ||b|| at exit (0 when b = 0)
  unsigned long long epoch_end;             // epoch of the step's last team reduction
};

// The fields of a step that change from step to step; run_step takes them
// apart from the rest of StepArgs so that a caller looping over steps keeps
// only these live (the rest can be re-read from memory that does not change).
template <typename R>
struct StepVar {
  R* x;
  const R* xprev;
  const R* xprev2;
  const R* xprev3;
  int gmode;
  const int* gi;
  int gp[3];
  const R* top_src;
  R top_scale;
  R* surf_out;
  R surf_scale;
  R* ckpt_out;
  const R* T_grad;
  int* out_iters;
  double* out_relres;
  int* out_status;
  unsigned long long epoch_base;
  unsigned jtag;                            // blocked fixed-K kernel: tag of the step's first phase
};

// The CG initial guess of a step: x0 = h1 (order 0), the linear
// extrapolation 2 h1 - h2 (order 1) or the quadratic one 3 h1 - 3 h2 + h3
// (order 2) of the states at the preceding time levels, limited by the states
// there are. In mode -1 the order is the one whose probe step took the fewest
// iterations (ties: the higher order); every workgroup reads the same counts,
// written by earlier launches, so the choice is uniform over the team. Mode 3
// takes x0 from xprev2 as given (a projected guess); b still uses h1. Every
// order is one form x0 = e1 h1 + e2 h2 (+ h3) of guess_coef.
template <typename R>
__device__ __forceinline__ int guess_order(const StepVar<R>& V) {
  if (V.gmode == 3) return (V.xprev && V.xprev2) ? 3 : 0;
  int o = V.gmode;
  if (o < 0) {
    const int c0 = V.gi[V.gp[0]], c1 = V.gi[V.gp[1]], c2 = V.gi[V.gp[2]];
    o = 2;
    int best = c2;
    if (c1 < best) { o = 1; best = c1; }
    if (c0 < best) o = 0;
  }
  if (!V.xprev || !V.xprev2) return 0;
  if (o == 2 && !V.xprev3) o = 1;
  return o;
}

// (e1, e2) of x0 = e1 h1 + e2 h2 (+ h3) for guess orders 1..3 (order 3: 0 h1 + h2
// = h2 exactly, h3 unused).
template <typename R>
__device__ __forceinline__ void guess_coef(int order, R& e1, R& e2) {
  e1 = order == 3 ? R(0) : (order == 2 ? R(3) : R(2));
  e2 = order == 3 ? R(1) : (order == 2 ? R(-3) : R(-1));
}

template <typename R>
__host__ __device__ __forceinline__ StepVar<R> step_var(const StepArgs<R>& S) {
  StepVar<R> V;
  V.x = S.x;
  V.xprev = S.xprev;
  V.xprev2 = S.xprev2;
  V.xprev3 = S.xprev3;
  V.gmode = S.gmode;
  V.gi = S.gi;
  V.gp[0] = S.gp[0];
  V.gp[1] = S.gp[1];
  V.gp[2] = S.gp[2];
  V.top_src = S.top_src;
  V.top_scale = S.top_scale;
  V.surf_out = S.surf_out;
  V.surf_scale = S.surf_scale;
  V.ckpt_out = S.ckpt_out;
  V.T_grad = S.T_grad;
  V.out_iters = S.out_iters;
  V.out_relres = S.out_relres;
  V.out_status = S.out_status;
  V.epoch_base = S.epoch_base;
  V.jtag = S.jtag;
  return V;
}

// The end of a step, after the solve: the surface frame (times surf_scale in
// the adjoint) and the checkpoint copy, the gradient pass of an adjoint step,
// and the per-step outputs (written by rank 0). The caller's last team
// reduction is the barrier that makes x complete before this reads it.
template <typename R>
__device__ __forceinline__ StepResult step_epilogue(const StepArgs<R>& S, const StepVar<R>& V, int rank, bool ok, int it,
                                    int status, double bb, double rr, Smem<R>& sh) {
  const Geom& g = S.g;
  if (!(bb < INFINITY) || !(rr < INFINITY) || rr != rr) status |= kNonFinite;
  if (!ok) status |= kTimeout;
  if (S.mode == kForward) {
    if (V.ckpt_out) {
      own_cells(g, rank, S.team, S.xcd_order, [&](long long i, long long col, int kz) {
        const R v = V.x[i];
        if (kz == 0 && V.surf_out) V.surf_out[col] = v;
        V.ckpt_out[i] = v;
      });
    } else if (V.surf_out) {
      top_cells(g, rank, S.team, S.xcd_order, [&](long long col) { V.surf_out[col] = V.x[col]; });
    }
  } else {
    if (V.surf_out)
      top_cells(g, rank, S.team, S.xcd_order, [&](long long col) { V.surf_out[col] = V.surf_scale * V.x[col]; });
  }
  if (S.mode == kAdjoint && V.T_grad && ok) {
    GradOp<R> Gop;
    Gop.alpha = S.alpha; Gop.mu = V.x; Gop.T = V.T_grad; Gop.G = S.G;
    Gop.sx = S.sx; Gop.sy = S.sy; Gop.sz = S.sz;
    sweep<R>(g, rank, S.team, S.xcd_order, Gop, sh);
  }

  const double relres = bb > 0.0 ? sqrt(rr / bb) : 0.0;
  if (V.out_iters && rank == 0 && threadIdx.x == 0) {
    V.out_iters[0] = it;
    V.out_relres[0] = relres;
    V.out_status[0] = status;
  }
  return StepResult{it, status, relres, 0ull};
}

template <typename R>
__device__ __forceinline__ StepResult run_step(const StepArgs<R>& S, const StepVar<R>& V, int rank, Smem<R>& sh) {
  const Geom& g = S.g;
  const Coef<R> cf = coef_of(S);
  unsigned long long red = V.epoch_base;
  bool ok = true;
  int ntr = 0;
  // trace_rank >= 0: that workgroup stamps into trace[0..cap); -1: every
  // workgroup stamps into its own window of cap entries
  const bool tr = S.trace && (rank == S.trace_rank || S.trace_rank < 0) && threadIdx.x == 0;
  long long* trace = S.trace ? S.trace + (S.trace_rank < 0 ? (long long)rank * S.trace_cap : 0) : nullptr;
  auto stamp = [&]() {
    if (tr && ntr < S.trace_cap) trace[ntr++] = wall_clock64();
  };
  stamp();

  int it = 0, status = kOk;
  double bb = 0.0, rr = 0.0;
  if (S.jacobi_k > 0) {
    // the paper's inner solver: K sweeps from x^(0) = h1, alternating between
    // p0 and x so that the last one lands in x; each sweep ends with a team
    // reduction, which is also the barrier before the next sweep reads halos
    const R* xin = V.xprev;
    while (ok && it < S.jacobi_k) {
      JacobiOp<R> J;
      J.alpha = S.alpha;
      J.xin = xin;
      J.h1 = V.xprev;
      J.xout = ((S.jacobi_k - 1 - it) & 1) ? S.p0 : V.x;
      J.top = V.top_src;
      J.top_scale = V.top_scale;
      J.cf = cf;
      J.acc[0] = J.acc[1] = 0.0;
      sweep<R>(g, rank, S.team, S.xcd_order, J, sh);
      stamp();
      double v2[2] = {J.acc[0], J.acc[1]};
      ok &= team_sum<R, 2>(S, rank, red, v2, sh);
      stamp();
      bb = v2[0];
      rr = v2[1];
      xin = J.xout;
      ++it;
    }
  } else {
    // set-up
    InitOp<R> init;
    init.alpha = S.alpha;
    init.cf = cf;
    init.z = S.z;
    init.top = V.top_src;
    init.top_scale = V.top_scale;
    init.nxy = g.nxy;
    init.acc[0] = init.acc[1] = init.acc[2] = 0.0;
    init.src = V.xprev;
    const int order = guess_order(V);
    init.h2 = order >= 1 ? V.xprev2 : nullptr;
    init.h3 = order == 2 ? V.xprev3 : nullptr;
    guess_coef<R>(order, init.e1, init.e2);
    init.xw = (V.xprev == V.x) ? nullptr : V.x;
    sweep<R>(g, rank, S.team, S.xcd_order, init, sh);
    stamp();
    double v3[3] = {init.acc[0], init.acc[1], init.acc[2]};
    ok &= team_sum<R, 3>(S, rank, red, v3, sh);
    stamp();
    bb = v3[0];
    double rz = v3[1];
    rr = v3[2];

    if (ok && bb == 0.0) {
      // b = 0: the solution is x = 0
      own_cells(g, rank, S.team, S.xcd_order, [&](long long i, long long, int) { V.x[i] = R(0); });
      double v0[1] = {0.0};
      ok &= team_sum<R, 1>(S, rank, red, v0, sh);
      rr = 0.0;
    } else if (S.variant == 0) {
      R* pc = S.p0;
      R* pn = S.p1;
      double rz_old = 1.0;
      // Chebyshev preconditioner: z_c = y_m from z = r / D in cheb_m - 1
      // sweeps, each followed by a team reduction (the barrier before the
      // next sweep reads halos); the last reduction returns r . z_c
      const bool cheb = S.cheb_m >= 2;
      auto ybuf = [&](int j) -> R* { return (j & 1) ? S.cheb_y1 : S.cheb_y0; };
      const R* zc = cheb ? ybuf(S.cheb_m) : S.z;
      auto cheb_apply = [&]() {
        double rho = 1.0 / S.cheb_sigma;
        for (int k = 1; ok && k < S.cheb_m; ++k) {
          double c1, c2;
          cheb_coef(S.cheb_sigma, S.cheb_delta, rho, c1, c2);
          ChebOp<R> C;
          C.alpha = S.alpha; C.z = S.z;
          C.yk = k == 1 ? nullptr : ybuf(k);
          C.ykm1 = k <= 2 ? nullptr : ybuf(k - 1);
          C.ynext = ybuf(k + 1);
          C.s = S.cheb_s; C.c1 = (R)c1; C.c2 = (R)c2;
          C.k = k;
          C.last = k + 1 == S.cheb_m;
          C.cf = cf;
          C.acc[0] = 0.0;
          sweep<R>(g, rank, S.team, S.xcd_order, C, sh);
          stamp();
          double vc[1] = {C.acc[0]};
          ok &= team_sum<R, 1>(S, rank, red, vc, sh);
          stamp();
          if (C.last) rz = vc[0];
        }
      };
      if (cheb && rr > S.rtol2 * bb) cheb_apply();
      while (ok && rr > S.rtol2 * bb) {
        if (it >= S.max_iter) { status |= kNoConv; break; }
        DirOp<R> A;
        A.alpha = S.alpha; A.z = zc; A.pold = pc; A.pnew = pn;
        A.first = (it == 0);
        A.beta = (R)(it == 0 ? 0.0 : rz / rz_old);
        A.cf = cf;
        A.acc[0] = 0.0;
        sweep<R>(g, rank, S.team, S.xcd_order, A, sh);
        stamp();
        double v1[1] = {A.acc[0]};
        ok &= team_sum<R, 1>(S, rank, red, v1, sh);
        stamp();
        if (!ok) break;
        const double alpha_cg = rz / v1[0];

        UpdOp<R> B;
        B.alpha = S.alpha; B.p = pn; B.x = V.x; B.z = S.z;
        B.a = (R)alpha_cg;
        B.cf = cf;
        B.acc[0] = B.acc[1] = 0.0;
        sweep<R>(g, rank, S.team, S.xcd_order, B, sh);
        stamp();
        double v2[2] = {B.acc[0], B.acc[1]};
        ok &= team_sum<R, 2>(S, rank, red, v2, sh);
        stamp();
        rz_old = rz;
        rz = v2[0];
        rr = v2[1];
        ++it;
        R* t = pc; pc = pn; pn = t;
        if (cheb && rr > S.rtol2 * bb) cheb_apply();
      }
    } else if (ok && rr > S.rtol2 * bb) {
      // single-reduction form: w_0 = A u_0, then one fused sweep per iteration
      WOp<R> W;
      W.alpha = S.alpha; W.u = S.z; W.what = S.w0;
      W.cf = cf;
      W.acc[0] = 0.0;
      sweep<R>(g, rank, S.team, S.xcd_order, W, sh);
      stamp();
      double vd[1] = {W.acc[0]};
      ok &= team_sum<R, 1>(S, rank, red, vd, sh);
      stamp();
      double gam = rz;
      double a_cg = gam / vd[0], b_cg = 0.0;
      R* ub[2] = {S.z, S.u1};
      R* wb[2] = {S.w0, S.w1};
      R* sb[2] = {S.s0, S.s1};
      int cur = 0;
      int xpend = 0;                        // x += a p of the last iteration still to apply
      R a_pend = R(0);
      while (ok) {
        if (it >= S.max_iter) { status |= kNoConv; break; }
        FusedOp<R> F;
        F.alpha = S.alpha;
        F.u = ub[cur]; F.wh = wb[cur]; F.sho = sb[cur];
        F.x = V.x; F.p = S.p0;
        F.un = ub[cur ^ 1]; F.whn = wb[cur ^ 1]; F.shn = sb[cur ^ 1];
        F.a = (R)a_cg; F.b = (R)b_cg;
        F.first = (it == 0);
        F.xmode = xpend ? 2 : 1;
        F.ap = a_pend;
        F.cf = cf;
        F.acc[0] = F.acc[1] = F.acc[2] = 0.0;
        sweep<R>(g, rank, S.team, S.xcd_order, F, sh);
        xpend = !xpend;
        a_pend = F.a;
        stamp();
        double v3n[3] = {F.acc[0], F.acc[1], F.acc[2]};
        ok &= team_sum<R, 3>(S, rank, red, v3n, sh);
        stamp();
        ++it;
        cur ^= 1;
        rr = v3n[2];
        if (!(rr > S.rtol2 * bb)) break;
        const double gn = v3n[0], dn = v3n[1];
        b_cg = gn / gam;
        a_cg = gn / (dn - b_cg * gn / a_cg);
        gam = gn;
      }
      if (xpend && ok) {
        // the last iteration's x += a p (p holds its p), then a team barrier:
        // the gradient pass and a following step read x at the halo
        const R ap = a_pend;
        const R* pp = S.p0;
        R* xx = V.x;
        own_cells(g, rank, S.team, S.xcd_order, [&](long long i, long long, int) {
          st_out(xx + i, fma_r(ap, gld(pp, i), gld((const R*)xx, i)));
        });
        double vz[1] = {0.0};
        ok &= team_sum<R, 1>(S, rank, red, vz, sh);
      }
    }
  }
  StepResult res = step_epilogue<R>(S, V, rank, ok, it, status, bb, rr, sh);
  res.epoch_end = red;
  return res;
}

template <typename R>
__global__ void __launch_bounds__(Cfg<R>::kBlock, 1) step_kernel(StepArgs<R> S) {
  __shared__ Smem<R> sh;
  run_step<R>(S, step_var(S), blockIdx.x, sh);
}

template <typename R>
__global__ void __launch_bounds__(Cfg<R>::kBlock, 1) apply_kernel(Geom g, const R* alpha, const R* x, R* y,
                                                          Coef<R> cf) {
  __shared__ Smem<R> sh;
  ApplyOp<R> op;
  op.alpha = alpha; op.xin = x; op.y = y;
  op.cf = cf;
  sweep<R>(g, blockIdx.x, gridDim.x, 0, op, sh);
}

// The largest diagonal entry D of A over the grid, as the bit pattern of a
// positive double (ordered like the integers) in *out (cleared by the caller).
// 1 / max D bounds the spectrum of D^-1 A from below (A >= I), 2 - 1 / max D
// from above (A <= 2 D - I); the Chebyshev preconditioner's interval derives
// from them.
template <typename R>
__global__ void __launch_bounds__(256) dmax_kernel(Geom g, const R* __restrict__ alpha, Coef<R> cf,
                                                   unsigned long long* out) {
  const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
  double d = 0.0;
  if (i < g.ng) {
    const int kz = (int)(i / g.nxy);
    const long long col = i - (long long)kz * g.nxy;
    const int iy = (int)(col / g.nx), ix = (int)(col - (long long)iy * g.nx);
    const R a = alpha[i];
    const long long rowx = i - ix, base = i - col;
    R c[6] = {R(0), R(0), R(0), R(0), R(0), R(0)};
    if (ix > 0) c[0] = face<R>(cf.sx, a, alpha[i - 1]);
    else if (g.periodic) c[0] = face<R>(cf.sx, a, alpha[rowx + g.nx - 1]);
    if (ix + 1 < g.nx) c[1] = face<R>(cf.sx, a, alpha[i + 1]);
    else if (g.periodic) c[1] = face<R>(cf.sx, a, alpha[rowx]);
    if (iy > 0) c[2] = face<R>(cf.sy, a, alpha[i - g.nx]);
    else if (g.periodic) c[2] = face<R>(cf.sy, a, alpha[base + (long long)(g.ny - 1) * g.nx + ix]);
    if (iy + 1 < g.ny) c[3] = face<R>(cf.sy, a, alpha[i + g.nx]);
    else if (g.periodic) c[3] = face<R>(cf.sy, a, alpha[base + ix]);
    if (kz > 0) c[4] = face<R>(cf.sz, a, alpha[i - g.nxy]);
    if (kz + 1 < g.nz) c[5] = face<R>(cf.sz, a, alpha[i + g.nxy]);
    d = (double)diag_of<R>(c[0], c[1], c[2], c[3], c[4], c[5], kz == cf.zb ? cf.sb : R(0));
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) d = fmax(d, __shfl_xor(d, off, 64));
  __shared__ double wmax[4];
  if ((threadIdx.x & 63) == 0) wmax[threadIdx.x >> 6] = d;
  __syncthreads();
  if (threadIdx.x == 0) {
    const double m = fmax(fmax(wmax[0], wmax[1]), fmax(wmax[2], wmax[3]));
    atomicMax(out, (unsigned long long)__double_as_longlong(m));
  }
}

// flag |= 1 if some alpha is not finite and positive
template <typename R>
__global__ void validate_kernel(const R* a, long long n, int* flag) {
  int bad = 0;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x) {
    const R v = a[i];
    if (!(v > R(0)) || !(v < R(INFINITY))) bad = 1;
  }
  if (bad) atomicOr(flag, 1);
}

// flag |= 1 if some value is not finite
template <typename R>
__global__ void finite_kernel(const R* a, long long n, int* flag) {
  int bad = 0;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x) {
    const R v = a[i];
    if (!(v == v) || !(v < R(INFINITY)) || !(v > R(-INFINITY))) bad = 1;
  }
  if (bad) atomicOr(flag, 1);
}

template <typename T>
__global__ void fill_kernel(T* p, long long n, T v) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x)
    p[i] = v;
}

template <typename T>
__global__ void copy_kernel(const T* __restrict__ s, T* __restrict__ d, long long n) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x)
    d[i] = s[i];
}


// ---------------------------------------------------------------------------
// gradients of the separable source q^n = q_t[n-1] q_xy (App. D.3: the
// adjoint gives dL/dq^n = dt mu^n on the top plane, here dq[n-1][ny][nx])

constexpr int kSrcBlock = 256;

// dL/dq_xy[c] = sum_n q_t[n-1] dq[n-1][c], summed over n in ascending order.
template <typename R>
__global__ void __launch_bounds__(kSrcBlock) qxy_grad_kernel(const R* __restrict__ dq, const double* __restrict__ qt,
                                                             int nsteps, long long nxy, double* __restrict__ out) {
  for (long long c = blockIdx.x * (long long)kSrcBlock + threadIdx.x; c < nxy; c += (long long)gridDim.x * kSrcBlock) {
    double s = 0.0;
    for (int n = 0; n < nsteps; ++n) s += qt[n] * (double)dq[(size_t)n * nxy + c];
    out[c] = s;
  }
}

// dL/dq_t[n-1] = sum_c dq[n-1][c] q_xy[c]: one workgroup per step, a fixed
// summation order (strided per thread, wave butterfly, waves in order).
template <typename R>
__global__ void __launch_bounds__(kSrcBlock) qt_grad_kernel(const R* __restrict__ dq, const R* __restrict__ qxy,
                                                            long long nxy, double* __restrict__ out) {
  const int n = blockIdx.x;
  const R* f = dq + (size_t)n * nxy;
  double s = 0.0;
  for (long long c = threadIdx.x; c < nxy; c += kSrcBlock) s += (double)f[c] * (double)qxy[c];
  s = wave_sum(s);
  __shared__ double red[kSrcBlock / 64];
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int w = 0; w < kSrcBlock / 64; ++w) t += red[w];
    out[n] = t;
  }
}

}  // namespace nh
