// nh_api.hip -- host runtime and C ABI of the heat solver (include/nefty_heat.h).
//
// The runtime owns one HIP stream per context, the context's device
// workspaces and the saved forward state, and drives the time loop: one
// cooperative launch of nh::step_kernel per implicit-Euler step (Sec. 4.2),
// forward in time for the state and backward in time for the adjoint
// (Sec. 4.3). With checkpointing every k steps the adjoint recomputes each
// k-step segment from its checkpoint before sweeping it backwards; the
// recomputation runs the same kernel with the same launch shape, so it
// reproduces the stored states bit for bit.
#include "nefty_heat.h"
#include "nh_kernels.hpp"
#include "nh_resident.hpp"
#include "nh_jacobi.hpp"
#include "nh_tv.hpp"
#include "nh_proj.hpp"

#include <hip/hip_runtime.h>
#include <rocprofiler-sdk-roctx/roctx.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

namespace nh {

// The streaming sweep's memory access pattern without its arithmetic: tiles
// of 64 x 16 columns (one 1024-thread workgroup each) march the nz planes;
// per cell six loads and five device-coherent stores, one workgroup barrier
// per plane. A measurement of what this traffic reaches on the chip, not part
// of the solver: out_k = in_k + in_{k+1}, and out_4 also adds the -x
// neighbour's in_0 through LDS.
struct ProbeArgs {
  const float* in[6];
  float* out[5];
  int nx, ny, nz;
};

__global__ void __launch_bounds__(1024, 1) stream_probe_kernel(ProbeArgs A) {
  __shared__ float sh[2][1024];
  const int ntx = A.nx >> 6;
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
  const long long col = (long long)((blockIdx.x % ntx) * 64 + tx) + (long long)A.nx * ((blockIdx.x / ntx) * 16 + ty);
  const long long nxy = (long long)A.nx * A.ny;
  for (int z = 0; z < A.nz; ++z) {
    const long long i = col + z * nxy;
    float v[6];
#pragma unroll
    for (int k = 0; k < 6; ++k) v[k] = gld(A.in[k], i);
    sh[z & 1][threadIdx.x] = v[0];
    __syncthreads();
    const float w = tx > 0 ? sh[z & 1][threadIdx.x - 1] : 0.f;
#pragma unroll
    for (int k = 0; k < 4; ++k) st_out(A.out[k] + i, v[k] + v[k + 1]);
    st_out(A.out[4] + i, v[4] + v[5] + w);
  }
}

}  // namespace nh

namespace {

using nh::Geom;
using nh::StepArgs;

// Device scratch of the allocation-free TV entry point (nh_tv_noalloc): the
// per-workgroup partial sums of the regulariser's value. One copy per GPU,
// held until the process ends; host code reaches it only through the
// address hipGetSymbolAddress returns for the device (kept in scratch_ptr).
constexpr int kScratchDoubles = nh::kTvMaxBlocks;
static __device__ __align__(256) double scratch[kScratchDoubles];

std::mutex scratch_mu;
std::vector<double*> scratch_ptr;          // by device ordinal; null until resolved

// The scratch address on `device`, which must be current. Resolved once per device.
hipError_t scratch_of(int device, double** out) {
  std::lock_guard<std::mutex> lk(scratch_mu);
  if ((int)scratch_ptr.size() <= device) scratch_ptr.resize(device + 1, nullptr);
  if (!scratch_ptr[device]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    scratch_ptr[device] = (double*)p;
  }
  *out = scratch_ptr[device];
  return hipSuccess;
}

// A host-side roctx range over one scope: a profiler run with marker tracing
// shows the forward pass, the adjoint pass and each checkpoint segment's
// recompute and adjoint sweep as named ranges (enqueue time on the host; the
// passes end with a stream synchronisation, so their ranges cover the GPU work).
struct Range {
  explicit Range(const char* name) { roctxRangePushA(name); }
  ~Range() { roctxRangePop(); }
  Range(const Range&) = delete;
  Range& operator=(const Range&) = delete;
};

struct Buf {
  void* p = nullptr;
  size_t bytes = 0;
};

}  // namespace

struct nh_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  int num_cu = 0;
  long long wallclock_khz = 100000;
  int occ_f32 = 0, occ_f64 = 0;              // co-resident step kernels per CU
  int res_occ = 0;                           // co-resident resident kernels per CU (0: unusable)
  int jac_occ = 0;                           // co-resident temporally blocked fixed-K kernels per CU

  bool grid_set = false;
  int nx = 0, ny = 0, nz = 0;
  double hx = 1, hy = 1, hz = 1;

  double rtol = 1e-6;
  int max_iter = 1000;
  int ckpt_every = 0;

  // boundary closure and inner solver (App. D.2)
  int periodic = 0;                          // lateral x, y faces wrap around
  double robin = 0;                          // back-face Robin coefficient h (sink h / hz)
  int jacobi_k = 0;                          // > 0: K Jacobi sweeps per solve instead of CG

  int team_max = 0, tile_z = 0, profile = 0;
  double barrier_timeout_s = 20.0;

  // saved forward
  int saved_prec = 0;                        // 0 none, 4 fp32, 8 fp64
  int saved_nsteps = 0;
  double saved_dt = 0;
  std::vector<double> saved_qt;

  // workspaces
  Buf alpha, qxy, z, p0, p1, u1, vw0, vw1, vs0, vs1, traj, seg, slots, steps, flag;
  Buf tvpart;                                // per-workgroup partial sums of the TV regulariser
  Buf xface;                                 // resident kernel: compact x-edge columns of u, w/D, s/D
  Buf srcq, srcqt;                           // source gradients: dL/dq^n series, q_t on the device
  double* scratch = nullptr;                 // this device's scratch array (nh_tv_noalloc)
  Buf jt[2];                                 // tagged iterates of the blocked fixed-K kernel
  unsigned jt_tag = 1;                       // tag of the next launch's first phase (0: cleared)
  // steps of the blocked fixed-K kernel waiting to be launched together
  nh::JacSteps jq{};
  nh::StepArgs<float> jq_base{};
  int jq_ev = -1;                            // event slot of the first queued step (-1: none)
  unsigned long long jq_epoch = 0;
  Buf mu[nh::kProjRing];                     // adjoint states, mu^n in mu[n % ring] (ring 4, or 8 with
                                             //   the projected guess)
  Buf pguess, ppart, pstate;                 // projected guess: A v, then x0; dot partials; ProjState
  Buf w[4];                                  // checkpointed forward: T^n in w[n & 3]
  int guess = 2;                             // initial guess: 0 previous state, 1 extrapolated, 2 adaptive,
                                             //   3 adaptive forward, projected adjoint
  int variant = 2;                           // 0 two reductions per iteration, 1 one, 2 one + register-resident
  int cheb_m = 1;                            // preconditioner: 1 Jacobi, >= 2 Chebyshev polynomial (variant 0)
  double cheb_dmax = 1.0;                    // max D of the saved forward's operator (Chebyshev interval)
  Buf dmaxb;                                 // device result of nh::dmax_kernel
  bool resident = false;                     // the current plan uses nh::resident_step_kernel
  bool jac_tb = false;                       // the current plan uses nh::jacobi_step_kernel
  int jtx = 0, jty = 0;                      //   with this many interior tiles per axis
  unsigned long long launch_ctr = 0;         // makes every launch's reduction epochs unique
  int slot_layout = 0;                       // slots hold: 0 zeros, 1 tagged words (team_sum_dev), 2 team_sum's
  size_t ws_bytes = 0, ws_peak = 0;

  Geom geom{};
  int team = 1;
  nh_stats st{};
  std::string err = "";
  std::vector<hipEvent_t> ev;
  std::vector<char> ev_rec;                  // event pair i was recorded (a queued step records none)
  long long kernel_launches = 0;             // step-kernel launches so far
  // diagnostics: NH_TRACE_STEP=n prints phase timings of forward step n
  int trace_step = 0;
  int trace_rank = 0;
  Buf trace;
};

namespace {

nh_status fail(nh_ctx* c, nh_status s, const std::string& msg) {
  if (c) c->err = msg;
  return s;
}

#define NH_HIP(ctx, call)                                                             \
  do {                                                                                \
    hipError_t e_ = (call);                                                           \
    if (e_ != hipSuccess)                                                             \
      return fail((ctx), NH_EHIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)

#define NH_TRY(expr)                   \
  do {                                 \
    nh_status s_ = (expr);             \
    if (s_ != NH_OK) return s_;        \
  } while (0)

nh_status release(nh_ctx* c, Buf& b) {
  if (b.p) {
    hipError_t e = hipFree(b.p);
    c->ws_bytes -= b.bytes;
    b.p = nullptr;
    b.bytes = 0;
    if (e != hipSuccess) return fail(c, NH_EHIP, std::string("hipFree: ") + hipGetErrorString(e));
  }
  return NH_OK;
}

// Make b hold at least `bytes` (contents are not preserved on growth).
nh_status ensure(nh_ctx* c, Buf& b, size_t bytes) {
  if (b.bytes >= bytes && b.p) return NH_OK;
  NH_TRY(release(c, b));
  if (bytes == 0) return NH_OK;
  hipError_t e = hipMalloc(&b.p, bytes);
  if (e != hipSuccess) {
    b.p = nullptr;
    (void)hipGetLastError();
    return fail(c, NH_ENOMEM, "hipMalloc of " + std::to_string(bytes) + " bytes failed: " +
                                  hipGetErrorString(e));
  }
  b.bytes = bytes;
  c->ws_bytes += bytes;
  if (c->ws_bytes > c->ws_peak) c->ws_peak = c->ws_bytes;
  return NH_OK;
}

void drop_forward(nh_ctx* c) {
  c->saved_prec = 0;
  c->saved_nsteps = 0;
  release(c, c->traj);
  release(c, c->seg);
  for (Buf& b : c->w) release(c, b);
}

template <typename T>
nh_status fill(nh_ctx* c, T* p, long long n, T v) {
  if (n <= 0) return NH_OK;
  int blocks = (int)std::min<long long>((n + 255) / 256, 4096);
  hipLaunchKernelGGL(nh::fill_kernel<T>, dim3(blocks), dim3(256), 0, c->stream, p, n, v);
  NH_HIP(c, hipGetLastError());
  return NH_OK;
}

// Tile shape and team size for the current grid, for workgroups of `block`
// threads; resident_ok allows the register-resident kernel (FP32, variant 2,
// zero-flux walls and the CG inner solver), tb_ok the temporally blocked
// fixed-K kernel (FP32, fixed-K sweeps, nz <= 16, automatic tiling, one
// interior tile per workgroup within what fits on the chip).
void plan(nh_ctx* c, int occ, int block, bool resident_ok = false, bool tb_ok = false) {
  resident_ok = resident_ok && !c->periodic && c->robin == 0 && c->jacobi_k == 0;
  c->jac_tb = false;
  if (tb_ok && c->jacobi_k > 0 && c->nz <= nh::kJacNZ && c->tile_z == 0 && c->jac_occ > 0) {
    const int jtx = (c->nx + nh::kJacIX - 1) / nh::kJacIX, jty = (c->ny + nh::kJacIY - 1) / nh::kJacIY;
    const long long nt = (long long)jtx * jty;
    long long cap = (long long)c->num_cu * c->jac_occ;
    if (c->team_max > 0) cap = std::min<long long>(cap, c->team_max);
    if (nt <= cap) {
      // the epilogue (surface frame, checkpoint, gradient pass) marches 64 x 8 x nz tiles
      Geom g{};
      g.nx = c->nx;
      g.ny = c->ny;
      g.nz = c->nz;
      g.nxy = (long long)c->nx * c->ny;
      g.ng = g.nxy * c->nz;
      g.periodic = c->periodic;
      g.TX = 64;
      g.TY = nh::kJacBlock / 64;
      g.txs = 6;
      g.ntx = (g.nx + g.TX - 1) / g.TX;
      g.nty = (g.ny + g.TY - 1) / g.TY;
      {
        // split in z so that the team shares the gradient pass
        const long long xy = (long long)g.ntx * g.nty;
        const long long want_ntz = std::max<long long>(1, (nt + xy - 1) / xy);
        g.TZ = (int)std::max<long long>(1, (g.nz + want_ntz - 1) / want_ntz);
      }
      g.ntz = (g.nz + g.TZ - 1) / g.TZ;
      g.ntiles = g.ntx * g.nty * g.ntz;
      c->geom = g;
      c->team = (int)nt;
      c->jac_tb = true;
      c->jtx = jtx;
      c->jty = jty;
      c->resident = false;
      c->st.team_blocks = c->team;
      c->st.block_threads = nh::kJacBlock;
      c->st.tile_x = nh::kJacIX;
      c->st.tile_y = nh::kJacIY;
      c->st.tile_z = c->nz;
      c->st.resident = 0;
      c->st.resident_occupancy = c->res_occ;
      c->st.jacobi_blocked = 1;
      return;
    }
  }
  Geom g{};
  g.nx = c->nx;
  g.ny = c->ny;
  g.nz = c->nz;
  g.nxy = (long long)c->nx * c->ny;
  g.ng = g.nxy * c->nz;
  g.periodic = c->periodic;
  g.TX = c->nx > 32 ? 64 : (c->nx > 16 ? 32 : 16);
  g.TY = block / g.TX;
  g.txs = g.TX == 64 ? 6 : (g.TX == 32 ? 5 : 4);
  g.ntx = (g.nx + g.TX - 1) / g.TX;
  g.nty = (g.ny + g.TY - 1) / g.TY;
  const int maxteam_hw = std::max(1, occ * c->num_cu);
  int maxteam = c->team_max > 0 ? std::min(c->team_max, maxteam_hw) : maxteam_hw;
  const long long xy_tiles = (long long)g.ntx * g.nty;
  int tz;
  if (c->tile_z > 0) {
    tz = std::min(c->tile_z, g.nz);
  } else if (c->jacobi_k > 0) {
    // fixed-K sweeps end each sweep with a team barrier and no CG work: as
    // many workgroups as fit, down to one plane per tile (measured on
    // 64x64x16: 24 us per sweep with 4 tiles of 16 planes, 9.2 us with 64
    // tiles of one plane)
    const long long want_ntz = std::max<long long>(1, maxteam / std::max<long long>(1, xy_tiles));
    tz = (int)std::max<long long>(1, (g.nz + want_ntz - 1) / want_ntz);
  } else if (g.ng <= 65536) {
    tz = g.nz;                                // small grids: few workgroups, cheap barriers
  } else {
    long long want_ntz = (maxteam + xy_tiles - 1) / xy_tiles;
    if (want_ntz < 1) want_ntz = 1;
    tz = (int)((g.nz + want_ntz - 1) / want_ntz);
    if (tz < 4) tz = std::min(4, g.nz);
  }
  g.TZ = tz;
  g.ntz = (g.nz + tz - 1) / tz;
  g.ntiles = (int)(xy_tiles * g.ntz);
  int team = std::min(g.ntiles, maxteam);
  if (g.ng <= 65536 && c->team_max == 0 && c->jacobi_k == 0) team = std::min(team, 1 + (int)(g.ng / 16384));
  c->resident = false;
  if (resident_ok && g.TX == 64) {
    // one tile of 64 x 8 columns x TZ cells per CU, the tile's CG state in registers
    Geom r = g;
    r.TY = nh::kResBlock / r.TX;
    r.nty = (r.ny + r.TY - 1) / r.TY;
    const long long rxy = (long long)r.ntx * r.nty;
    const int cap = c->team_max > 0 ? std::min(c->team_max, c->num_cu * c->res_occ) : c->num_cu * c->res_occ;
    // the thinnest tiles that fit: as many workgroups as the chip holds (on 64x64x32, 1 plane
    // per tile and 256 workgroups took 13.3 us per iteration against 14.6 with 4 planes and 64)
    int tz0 = c->tile_z > 0 ? c->tile_z : (int)std::max<long long>(1, ((long long)r.nz * rxy + cap - 1) / cap);
    for (int tz = tz0; tz <= nh::kResTZ && (c->tile_z == 0 || tz == c->tile_z); ++tz) {
      const long long nt = rxy * ((r.nz + tz - 1) / tz);
      if (nt <= cap) {
        r.TZ = std::min(tz, r.nz);
        r.ntz = (r.nz + r.TZ - 1) / r.TZ;
        r.ntiles = (int)(rxy * r.ntz);
        g = r;
        team = r.ntiles;
        block = nh::kResBlock;
        c->resident = true;
        break;
      }
    }
  }
  c->geom = g;
  c->team = std::max(1, team);
  c->st.team_blocks = c->team;
  c->st.block_threads = block;
  c->st.tile_x = g.TX;
  c->st.tile_y = g.TY;
  c->st.tile_z = g.TZ;
  c->st.resident = c->resident ? 1 : 0;
  c->st.resident_occupancy = c->res_occ;
  c->st.jacobi_blocked = 0;
}

template <typename R>
int occupancy(nh_ctx* c) {
  return sizeof(R) == 4 ? c->occ_f32 : c->occ_f64;
}

// Make the reduction slots ready for a launch whose reductions use the
// tagged words of team_sum_dev (tagged) or team_sum's layout, with epochs from
// epoch_base on. Tags are the low 32 bits of the epochs, which repeat every
// 256 launches: the slots are zeroed when a tagged launch starts a new round
// of 256, and whenever the layout changes, so no stale word can carry the
// tag a reader waits for.
nh_status prepare_slots(nh_ctx* c, bool tagged, unsigned long long epoch_base) {
  const int want = tagged ? 1 : 2;
  const bool new_round = tagged && ((epoch_base >> 24) & 0xFF) == 0;
  if (new_round || (c->slot_layout != 0 && c->slot_layout != want))
    NH_TRY(fill<unsigned long long>(c, (unsigned long long*)c->slots.p, (long long)(c->slots.bytes / 8), 0ull));
  c->slot_layout = want;
  return NH_OK;
}

// Launch the queued steps of the blocked fixed-K kernel as one launch, timed
// with the event pair of the first of them.
nh_status flush_steps(nh_ctx* c) {
  if (c->jq.count == 0) return NH_OK;
  NH_TRY(prepare_slots(c, true, c->jq_epoch));
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (c->profile && c->jq_ev >= 0) {
    e0 = c->ev[2 * c->jq_ev];
    e1 = c->ev[2 * c->jq_ev + 1];
    NH_HIP(c, hipEventRecord(e0, c->stream));
  }
  void* args[] = {(void*)&c->jq_base, (void*)&c->jq};
  NH_HIP(c, hipLaunchCooperativeKernel((const void*)nh::jacobi_steps_kernel<nh::kJacH>, dim3(c->jq_base.team),
                                       dim3(nh::kJacBlock), args, 0, c->stream));
  if (e1) {
    NH_HIP(c, hipEventRecord(e1, c->stream));
    c->ev_rec[c->jq_ev] = 1;
  }
  ++c->kernel_launches;
  c->jq.count = 0;
  c->jq_ev = -1;
  return NH_OK;
}

// Queue one step of the blocked fixed-K kernel. Steps of one sweep share
// everything but their StepVar fields; step i of a launch gets the epoch
// base B + i (B even), so consecutive steps' final reductions use
// alternating slot banks. Returns in *launched whether the step was
// launched now (the caller's event slot is then used).
nh_status queue_step(nh_ctx* c, StepArgs<float>& S, int slot_ev, bool* launched) {
  const unsigned phases = (unsigned)((S.jacobi_k + nh::kJacS - 1) / nh::kJacS);
  if (c->jq.count > 0 && (S.mode != c->jq_base.mode || S.G != c->jq_base.G || S.alpha != c->jq_base.alpha))
    NH_TRY(flush_steps(c));
  if (c->jt_tag > 0xFFFFFFF0u - phases) {
    NH_TRY(flush_steps(c));
    for (Buf& b : c->jt) NH_TRY(fill<unsigned long long>(c, (unsigned long long*)b.p, c->geom.ng, 0ull));
    c->jt_tag = 1;
  }
  S.jt[0] = (unsigned long long*)c->jt[0].p;
  S.jt[1] = (unsigned long long*)c->jt[1].p;
  S.jtag = c->jt_tag;
  c->jt_tag += phases;
  if (c->jq.count == 0) {
    c->jq_epoch = (++c->launch_ctr) << 24;
    c->jq_ev = slot_ev;
  }
  S.epoch_base = c->jq_epoch + (unsigned long long)c->jq.count;
  if (c->jq.count == 0) c->jq_base = S;
  c->jq.v[c->jq.count++] = nh::step_var(S);
  *launched = c->jq.count == nh::kJacBatch;
  if (*launched) NH_TRY(flush_steps(c));
  return NH_OK;
}

template <typename R>
nh_status launch_step(nh_ctx* c, StepArgs<R>& S, int slot_ev, double* t_kernel) {
  if constexpr (sizeof(R) == 4) {
    if (c->jac_tb && !S.trace) {
      bool launched = false;
      NH_TRY(queue_step(c, S, slot_ev, &launched));
      (void)t_kernel;
      return NH_OK;
    }
  }
  NH_TRY(flush_steps(c));
  NH_TRY(prepare_slots(c, sizeof(R) == 4 && (c->resident || c->jac_tb), S.epoch_base));
  void* args[] = {(void*)&S};
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (c->profile) {
    e0 = c->ev[2 * slot_ev];
    e1 = c->ev[2 * slot_ev + 1];
    NH_HIP(c, hipEventRecord(e0, c->stream));
  }
  if (sizeof(R) == 4 && c->resident)
    NH_HIP(c, hipLaunchCooperativeKernel((const void*)nh::resident_step_kernel<64>, dim3(S.team),
                                         dim3(nh::kResBlock), args, (unsigned)nh::kResLdsBytes, c->stream));
  else if (sizeof(R) == 4 && c->jac_tb) {
    // phase tags only grow between clears of the tagged buffers, so no stale word can match
    const unsigned phases = (unsigned)((S.jacobi_k + nh::kJacS - 1) / nh::kJacS);
    if (c->jt_tag > 0xFFFFFFF0u - phases) {
      for (Buf& b : c->jt) NH_TRY(fill<unsigned long long>(c, (unsigned long long*)b.p, c->geom.ng, 0ull));
      c->jt_tag = 1;
    }
    S.jt[0] = (unsigned long long*)c->jt[0].p;
    S.jt[1] = (unsigned long long*)c->jt[1].p;
    S.jtag = c->jt_tag;
    c->jt_tag += phases;
    NH_HIP(c, hipLaunchCooperativeKernel((const void*)nh::jacobi_step_kernel<nh::kJacH>, dim3(S.team),
                                         dim3(nh::kJacBlock), args, 0, c->stream));
  }
  else
    NH_HIP(c, hipLaunchCooperativeKernel((const void*)nh::step_kernel<R>, dim3(S.team), dim3(nh::Cfg<R>::kBlock),
                                         args, 0, c->stream));
  if (c->profile) {
    NH_HIP(c, hipEventRecord(e1, c->stream));
    c->ev_rec[slot_ev] = 1;
  }
  ++c->kernel_launches;
  (void)t_kernel;
  return NH_OK;
}

// Events are recorded into a pool of kEvPairs pairs; when the pool is full
// the elapsed times are collected (one stream sync) and the pool reused.
constexpr int kEvPairs = 512;

// Also launches any queued steps first (their events are among those collected).
nh_status collect_events(nh_ctx* c, int used, double* acc) {
  NH_TRY(flush_steps(c));
  if (!c->profile || used == 0) return NH_OK;
  NH_HIP(c, hipStreamSynchronize(c->stream));
  for (int i = 0; i < used; ++i) {
    if (!c->ev_rec[i]) continue;
    float ms = 0;
    NH_HIP(c, hipEventElapsedTime(&ms, c->ev[2 * i], c->ev[2 * i + 1]));
    *acc += ms * 1e-3;
    c->ev_rec[i] = 0;
  }
  return NH_OK;
}

nh_status ensure_events(nh_ctx* c) {
  if (!c->profile || !c->ev.empty()) return NH_OK;
  c->ev.resize(2 * kEvPairs);
  c->ev_rec.assign(kEvPairs, 0);
  for (auto& e : c->ev) NH_HIP(c, hipEventCreate(&e));
  return NH_OK;
}

template <typename R>
void base_args(nh_ctx* c, StepArgs<R>& S, double dt) {
  std::memset(&S, 0, sizeof(S));
  S.g = c->geom;
  S.sx = (R)(2.0 * dt / (c->hx * c->hx));
  S.sy = (R)(2.0 * dt / (c->hy * c->hy));
  S.sz = (R)(2.0 * dt / (c->hz * c->hz));
  S.sb = (R)(dt * c->robin / c->hz);
  S.alpha = (const R*)c->alpha.p;
  S.z = (R*)c->z.p;
  S.p0 = (R*)c->p0.p;
  S.p1 = (R*)c->p1.p;
  S.u1 = (R*)c->u1.p;
  S.w0 = (R*)c->vw0.p;
  S.w1 = (R*)c->vw1.p;
  S.s0 = (R*)c->vs0.p;
  S.s1 = (R*)c->vs1.p;
  S.xface = (R*)c->xface.p;
  S.variant = c->variant == 0 ? 0 : 1;
  S.jacobi_k = c->jacobi_k;
  S.jtx = c->jac_tb ? c->jtx : 0;
  S.jty = c->jac_tb ? c->jty : 0;
  S.slots = c->slots.p;
  S.epoch_base = (++c->launch_ctr) << 24;
  S.rtol2 = c->rtol * c->rtol;
  S.max_iter = c->max_iter;
  S.team = c->team;
  S.xcd_order = 1;
  S.err_flag = (int*)c->flag.p;
  S.timeout_ticks = (long long)(c->barrier_timeout_s * (double)c->wallclock_khz * 1000.0);
  S.trace = nullptr;
  S.cheb_m = 1;
  if (c->variant == 0 && c->cheb_m >= 2 && c->jacobi_k == 0) {
    // Chebyshev interval [lo, hi] of D^-1 A: hi = 2 - 1 / max D bounds the
    // spectrum from above (A <= 2 D - I); lo = max(1 / max D, hi / (2 m^2))
    // targets the upper part, where a degree-m polynomial damps well (a lower
    // bound of the spectrum, 1 / max D, is far below its bulk when the
    // diffusivity contrast is high). Below lo the preconditioned eigenvalues
    // 1 - P_m stay in (0, 1), so M stays symmetric positive definite.
    const int m = c->cheb_m;
    const double dmax = std::max(c->cheb_dmax, 1.0);
    const double hi = 2.0 - 1.0 / dmax, lo = std::max(1.0 / dmax, hi / (2.0 * m * m));
    const double theta = 0.5 * (hi + lo), delta = std::max(0.5 * (hi - lo), 1e-6 * theta);
    S.cheb_m = m;
    S.cheb_s = (R)(1.0 / theta);
    S.cheb_sigma = theta / delta;
    S.cheb_delta = delta;
    S.cheb_y0 = (R*)c->vw0.p;
    S.cheb_y1 = (R*)c->vw1.p;
  }
}

// Per-step device outputs: [3][nsteps] iterations (forward, adjoint, recompute),
// then relres and status in the same arrangement.
struct StepOut {
  int* iters;
  double* relres;
  int* status;
};

size_t relres_offset(int N) { return (sizeof(int) * 3 * (size_t)N + 63) / 64 * 64; }

size_t step_out_bytes(int N) {
  return relres_offset(N) + sizeof(double) * 3 * (size_t)N + sizeof(int) * 3 * (size_t)N;
}

StepOut step_out(nh_ctx* c, int region, int n) {
  const int N = c->saved_nsteps;
  char* base = (char*)c->steps.p;
  int* iters = (int*)base;
  double* relres = (double*)(base + relres_offset(N));
  int* status = (int*)(relres + 3 * (size_t)N);
  StepOut o{iters + region * N + n, relres + region * N + n, status + region * N + n};
  return o;
}

nh_status check_flag(nh_ctx* c) {
  int h = 0;
  NH_HIP(c, hipMemcpyAsync(&h, c->flag.p, sizeof(int), hipMemcpyDeviceToHost, c->stream));
  NH_HIP(c, hipStreamSynchronize(c->stream));
  if (h & nh::kTimeout) {
    // a workgroup left a reduction early; later launches use fresh epochs, so
    // only the flag needs clearing
    NH_HIP(c, hipMemsetAsync(c->flag.p, 0, sizeof(int), c->stream));
    NH_HIP(c, hipStreamSynchronize(c->stream));
    return fail(c, NH_ETIMEOUT, "a device-side team barrier exceeded its time limit");
  }
  return NH_OK;
}

// Sum the per-step outputs of `region` for steps [0, count).
nh_status summarize(nh_ctx* c, int region, int count, long long* iters_sum, int* max_it,
                    double* worst, int* any_status) {
  const int N = c->saved_nsteps;
  std::vector<int> it(count), stv(count);
  std::vector<double> rel(count);
  StepOut o = step_out(c, region, 0);
  NH_HIP(c, hipMemcpyAsync(it.data(), o.iters, sizeof(int) * count, hipMemcpyDeviceToHost, c->stream));
  NH_HIP(c, hipMemcpyAsync(rel.data(), o.relres, sizeof(double) * count, hipMemcpyDeviceToHost, c->stream));
  NH_HIP(c, hipMemcpyAsync(stv.data(), o.status, sizeof(int) * count, hipMemcpyDeviceToHost, c->stream));
  NH_HIP(c, hipStreamSynchronize(c->stream));
  (void)N;
  for (int i = 0; i < count; ++i) {
    *iters_sum += it[i];
    if (it[i] > *max_it) *max_it = it[i];
    if (rel[i] > *worst || rel[i] != rel[i]) *worst = rel[i];
    *any_status |= stv[i];
  }
  return NH_OK;
}

nh_status status_to_code(nh_ctx* c, int any) {
  if (any & nh::kNonFinite) return fail(c, NH_ENONFINITE, "a CG reduction was not finite");
  if (any & nh::kTimeout) return fail(c, NH_ETIMEOUT, "a device-side team barrier timed out");
  if (any & nh::kNoConv) return fail(c, NH_ENOCONV, "a CG solve reached max_iter");
  return NH_OK;
}

template <typename R>
nh_status check_positive(nh_ctx* c, const R* a, long long n, bool positive) {
  NH_HIP(c, hipMemsetAsync(c->flag.p, 0, sizeof(int), c->stream));
  int blocks = (int)std::min<long long>((n + 255) / 256, 2048);
  if (positive)
    hipLaunchKernelGGL(nh::validate_kernel<R>, dim3(blocks), dim3(256), 0, c->stream, a, n, (int*)c->flag.p);
  else
    hipLaunchKernelGGL(nh::finite_kernel<R>, dim3(blocks), dim3(256), 0, c->stream, a, n, (int*)c->flag.p);
  NH_HIP(c, hipGetLastError());
  int h = 0;
  NH_HIP(c, hipMemcpyAsync(&h, c->flag.p, sizeof(int), hipMemcpyDeviceToHost, c->stream));
  NH_HIP(c, hipStreamSynchronize(c->stream));
  NH_HIP(c, hipMemsetAsync(c->flag.p, 0, sizeof(int), c->stream));
  return h ? NH_EINVAL : NH_OK;
}

// Algorithmic bytes of one step, R bytes per vector element: the traffic of
// the textbook two-pass Jacobi-PCG with every vector in HBM, whatever the
// kernel actually keeps on chip. Per iteration and voxel the operator pass
// reads r, p, alpha and writes p, q (5R) and the update pass reads x, p, r,
// q, 1/D and writes x, r (7R): 12R. Per step the residual set-up reads the
// previous state, alpha and the source and writes r, z (5R) and the state is
// stored (R); an adjoint step adds the gradient pass, which reads T^n, mu^n
// and alpha (3R) and reads and writes the FP64 accumulator (16 bytes).
// FP32: 48 bytes per voxel-iteration, 24 per forward step, 52 per adjoint step.
// With the fixed-K Jacobi solver a sweep reads x, alpha and the previous
// state and writes the new x (4R per voxel and sweep); the last sweep writes
// the state itself, and an adjoint step adds the gradient pass (T, mu,
// alpha: 3R; the FP64 accumulator: 16 bytes).
double step_bytes(const Geom& g, int R, int mode, int iters, bool jacobi, int cheb_m = 1) {
  double per_voxel;
  if (jacobi)
    per_voxel = 4.0 * R * iters + (mode == nh::kForward ? 0.0 : 3.0 * R + 16.0);
  else
    // a Chebyshev preconditioner is applied once per iteration (after the
    // set-up and after every iteration but the last): cheb_m - 1 sweeps, each
    // reading y_k, y_{k-1}, z, alpha and writing y_{k+1}
    per_voxel = (12.0 * R + 5.0 * R * (cheb_m - 1)) * iters + (mode == nh::kForward ? 6.0 * R : 9.0 * R + 16.0);
  return per_voxel * (double)g.ng;
}

int cheb_degree(const nh_ctx* c) { return (c->variant == 0 && c->jacobi_k == 0) ? c->cheb_m : 1; }

template <typename R>
nh_status ensure_common(nh_ctx* c, int nsteps) {
  const size_t vb = sizeof(R) * (size_t)c->geom.ng;
  NH_TRY(ensure(c, c->alpha, vb));
  NH_TRY(ensure(c, c->z, vb));
  NH_TRY(ensure(c, c->p0, vb));
  if (c->variant == 0) {
    NH_TRY(ensure(c, c->p1, vb));
    NH_TRY(release(c, c->u1));
    if (c->cheb_m >= 2 && c->jacobi_k == 0) {   // the Chebyshev preconditioner's y buffers
      NH_TRY(ensure(c, c->vw0, vb));
      NH_TRY(ensure(c, c->vw1, vb));
    } else {
      NH_TRY(release(c, c->vw0));
      NH_TRY(release(c, c->vw1));
    }
    NH_TRY(release(c, c->vs0));
    NH_TRY(release(c, c->vs1));
  } else {
    NH_TRY(release(c, c->p1));
    NH_TRY(ensure(c, c->u1, vb));
    NH_TRY(ensure(c, c->vw0, vb));
    NH_TRY(ensure(c, c->vw1, vb));
    NH_TRY(ensure(c, c->vs0, vb));
    NH_TRY(ensure(c, c->vs1, vb));
  }
  if (sizeof(R) == 4 && c->resident)   // three vectors, two banks
    NH_TRY(ensure(c, c->xface, sizeof(float) * 2 * (size_t)c->team * nh::kXfTile));
  else
    NH_TRY(release(c, c->xface));
  const size_t slot_bytes = sizeof(nh::Slot) * (2 * (size_t)c->team + 2);   // streaming: team + 1; resident: 2 banks
  if (c->slots.bytes < slot_bytes || !c->slots.p) {
    NH_TRY(ensure(c, c->slots, slot_bytes));
    NH_HIP(c, hipMemsetAsync(c->slots.p, 0, c->slots.bytes, c->stream));  // epoch 0 is never used
    c->slot_layout = 0;
  }
  if (!c->flag.p) {
    NH_TRY(ensure(c, c->flag, 64));
    NH_HIP(c, hipMemsetAsync(c->flag.p, 0, 64, c->stream));
  }
  NH_TRY(ensure(c, c->steps, step_out_bytes(nsteps)));
  if (c->jac_tb) {
    const size_t tb = sizeof(unsigned long long) * (size_t)c->geom.ng;
    if (c->jt[0].bytes < tb || c->jt[1].bytes < tb) {
      for (Buf& b : c->jt) NH_TRY(ensure(c, b, tb));
      for (Buf& b : c->jt) NH_TRY(fill<unsigned long long>(c, (unsigned long long*)b.p, c->geom.ng, 0ull));
      c->jt_tag = 1;
    }
  }
  return NH_OK;
}

// The previous states h1..h3 and the CG initial-guess policy (c->guess): 0
// x0 = h1; 1 the quadratic extrapolation 3 h1 - 3 h2 + h3 (linear with two
// states); 2 and 3 (3 projects the adjoint's guesses instead, see
// proj_prepare) adaptive: the steps of a sweep are taken in periods of
// kGuessPeriod; its first three steps probe orders 0, 1 and 2, and the others
// use the order whose probe needed the fewest iterations (the kernel compares
// the counts in gi, written by earlier launches). j is the step's position in
// its sweep, step(j) the step number at position j; gi is indexed by step
// number - 1. Null states are zero.
constexpr int kGuessPeriod = 32;

template <typename R, typename StepOf>
void set_guess(const nh_ctx* c, StepArgs<R>& S, const R* const (&h)[3], int j, const int* gi, StepOf step) {
  S.xprev = h[0];
  S.xprev2 = h[1];
  S.xprev3 = h[2];
  S.gi = nullptr;
  S.gp[0] = S.gp[1] = S.gp[2] = 0;
  if (c->guess < 2) {
    S.gmode = c->guess == 0 ? 0 : 2;
    return;
  }
  const int k = j % kGuessPeriod;
  S.gmode = k < 3 ? k : -1;
  if (k >= 3) {
    S.gi = gi;
    for (int d = 0; d < 3; ++d) S.gp[d] = step(j - k + d) - 1;
  }
}

// One forward step n (1-based) into x from the previous states h = T^{n-1},
// T^{n-2}, T^{n-3}; region selects where its iteration count goes (0 forward,
// 2 recompute).
template <typename R>
nh_status forward_step(nh_ctx* c, int n, const R* const (&h)[3], R* x, const R* q_xy, double dt, double qt,
                       R* surf, R* ckpt, int region, int ev_slot) {
  StepArgs<R> S;
  base_args<R>(c, S, dt);
  S.mode = nh::kForward;
  S.x = x;
  // a recomputed step repeats the original forward's choices: same counts
  set_guess<R>(c, S, h, n - 1, step_out(c, 0, 0).iters, [](int jj) { return jj + 1; });
  S.top_src = q_xy;
  S.top_scale = (R)(dt * qt);
  S.surf_out = surf;
  S.surf_scale = R(1);
  S.ckpt_out = ckpt;
  StepOut o = step_out(c, region, n - 1);
  S.out_iters = o.iters;
  S.out_relres = o.relres;
  S.out_status = o.status;
  const bool tracing = region == 0 && n == c->trace_step;
  const int cap = c->trace_rank < 0 ? 256 : 4096;
  const size_t tn = c->trace_rank < 0 ? (size_t)cap * c->team : (size_t)cap;
  if (tracing) {
    NH_TRY(ensure(c, c->trace, sizeof(long long) * tn));
    NH_HIP(c, hipMemsetAsync(c->trace.p, 0, c->trace.bytes, c->stream));
    S.trace = (long long*)c->trace.p;
    S.trace_rank = c->trace_rank < 0 ? -1 : std::min(c->trace_rank, c->team - 1);
    S.trace_cap = cap;
    S.trace_detail = (c->resident && std::getenv("NH_TRACE_DETAIL")) ? 1 : 0;
  }
  NH_TRY(launch_step<R>(c, S, ev_slot, nullptr));
  if (tracing) {
    std::vector<long long> tall(tn);
    NH_HIP(c, hipMemcpyAsync(tall.data(), c->trace.p, sizeof(long long) * tn, hipMemcpyDeviceToHost, c->stream));
    NH_HIP(c, hipStreamSynchronize(c->stream));
    // stamps: start, set-up sweep(s) and reduction(s), then per iteration its
    // sweep(s) and reduction(s): two pairs (variant 0) or one pair (variant 1)
    const double us = 1e3 / (double)c->wallclock_khz;
    if (c->jac_tb) {
      // stamps: start, set-up, then per phase: iterate loaded, sweeps done, barrier passed
      const long long* t = tall.data();
      int m = 0;
      while (m < cap && t[m] != 0) ++m;
      double ld = 0, sw = 0, br = 0;
      const int np = m > 2 ? (m - 2) / 3 : 0;
      for (int k = 0; k < np; ++k) {
        ld += (t[2 + 3 * k] - t[1 + 3 * k]) * us;
        sw += (t[3 + 3 * k] - t[2 + 3 * k]) * us;
        br += (t[4 + 3 * k] - t[3 + 3 * k]) * us;
      }
      std::fprintf(stderr, "[nh trace] step %d rank %d blocked fixed-K: set-up %.2f us, %d phases, mean us per phase: "
                   "load %.2f, sweeps %.2f, store+barrier %.2f\n", n, S.trace_rank, m > 1 ? (t[1] - t[0]) * us : 0.0,
                   np, np ? ld / np : 0.0, np ? sw / np : 0.0, np ? br / np : 0.0);
      return NH_OK;
    }
    const int head = c->variant == 0 ? 3 : 5, per = c->variant == 0 ? 4 : (S.trace_detail ? 5 : 2);
    const int nranks = c->trace_rank < 0 ? c->team : 1;
    for (int r = 0; r < nranks; ++r) {
      const long long* t = tall.data() + (size_t)r * cap;
      int m = 0;
      while (m < cap && t[m] != 0) ++m;
      std::vector<double> acc(per, 0.0);
      const int its = m > head ? (m - head) / per : 0;
      for (int k = 0; k < its; ++k)
        for (int j = 0; j < per; ++j) acc[j] += (t[head + per * k + j] - t[head + per * k + j - 1]) * us;
      std::fprintf(stderr, "[nh trace] step %d rank %d variant %d: set-up %.2f us, %d iterations, mean us per phase:",
                   n, nranks > 1 ? r : S.trace_rank, c->variant, m >= head ? (t[head - 1] - t[0]) * us : 0.0, its);
      for (int j = 0; j < per; ++j) std::fprintf(stderr, " %.2f", its ? acc[j] / its : 0.0);
      std::fprintf(stderr, " | set-up phases:");
      for (int j = 1; j < head && j < m; ++j) std::fprintf(stderr, " %.2f", (t[j] - t[j - 1]) * us);
      const int last = head + per * its - 1;
      if (m - 1 > last && last >= 0) std::fprintf(stderr, " | after the loop %.2f", (t[m - 1] - t[last]) * us);
      std::fprintf(stderr, "\n");
    }
  }
  return NH_OK;
}

template <typename R>
nh_status do_forward(nh_ctx* c, const R* alpha, const R* q_xy, const double* q_t, double dt,
                     int nsteps, R* T_surf) {
  auto t0 = std::chrono::steady_clock::now();
  const Range range(sizeof(R) == 4 ? "nh_forward" : "nh_forward_f64");
  if (!c) return NH_EINVAL;
  if (!c->grid_set) return fail(c, NH_ESTATE, "nh_set_grid has not been called");
  if (!alpha || !q_xy || !q_t || !T_surf) return fail(c, NH_EINVAL, "null pointer argument");
  if (!(dt > 0) || !std::isfinite(dt)) return fail(c, NH_EINVAL, "dt must be finite and > 0");
  if (nsteps < 1) return fail(c, NH_EINVAL, "nsteps must be >= 1");
  for (int i = 0; i < nsteps; ++i)
    if (!std::isfinite(q_t[i])) return fail(c, NH_EINVAL, "q_t holds a non-finite value");

  drop_forward(c);
  plan(c, occupancy<R>(c), nh::Cfg<R>::kBlock, sizeof(R) == 4 && c->variant == 2 && c->res_occ > 0,
       sizeof(R) == 4);
  NH_TRY(ensure_common<R>(c, nsteps));
  NH_TRY(ensure_events(c));
  const Geom& g = c->geom;
  const size_t vb = sizeof(R) * (size_t)g.ng;

  nh_status v = check_positive<R>(c, alpha, g.ng, true);
  if (v == NH_EINVAL) return fail(c, NH_EINVAL, "alpha must be finite and > 0 everywhere");
  NH_TRY(v);
  v = check_positive<R>(c, q_xy, g.nxy, false);
  if (v == NH_EINVAL) return fail(c, NH_EINVAL, "q_xy holds a non-finite value");
  NH_TRY(v);
  NH_HIP(c, hipMemcpyAsync(c->alpha.p, alpha, vb, hipMemcpyDeviceToDevice, c->stream));
  if (c->variant == 0 && c->cheb_m >= 2 && c->jacobi_k == 0) {
    // the largest diagonal entry of A, for the Chebyshev preconditioner's interval
    NH_TRY(ensure(c, c->dmaxb, sizeof(unsigned long long)));
    NH_HIP(c, hipMemsetAsync(c->dmaxb.p, 0, sizeof(unsigned long long), c->stream));
    const nh::Coef<R> cf{(R)(2.0 * dt / (c->hx * c->hx)), (R)(2.0 * dt / (c->hy * c->hy)),
                         (R)(2.0 * dt / (c->hz * c->hz)), (R)(dt * c->robin / c->hz), g.nz - 1};
    const long long blocks = (g.ng + 255) / 256;
    hipLaunchKernelGGL(nh::dmax_kernel<R>, dim3((unsigned)blocks), dim3(256), 0, c->stream, g, (const R*)c->alpha.p,
                       cf, (unsigned long long*)c->dmaxb.p);
    NH_HIP(c, hipGetLastError());
    unsigned long long bits = 0;
    NH_HIP(c, hipMemcpyAsync(&bits, c->dmaxb.p, sizeof(bits), hipMemcpyDeviceToHost, c->stream));
    NH_HIP(c, hipStreamSynchronize(c->stream));
    double d;
    std::memcpy(&d, &bits, sizeof(d));
    if (!(d >= 1.0) || !std::isfinite(d)) return fail(c, NH_EINVAL, "operator diagonal is not finite");
    c->cheb_dmax = d;
  }
  NH_TRY(ensure(c, c->qxy, sizeof(R) * (size_t)g.nxy));
  NH_HIP(c, hipMemcpyAsync(c->qxy.p, q_xy, sizeof(R) * (size_t)g.nxy, hipMemcpyDeviceToDevice, c->stream));
  const R* qsrc = (const R*)c->qxy.p;

  const int k = c->ckpt_every;
  c->saved_nsteps = nsteps;
  R* traj = nullptr;
  if (k == 0) {
    NH_TRY(ensure(c, c->traj, vb * (size_t)nsteps));
    traj = (R*)c->traj.p;
  } else {
    // checkpoint j holds T^{jk}, T^{jk-1}, T^{jk-2} (the states the initial
    // guess of step jk+1 uses), for jk below N
    const int nck = (nsteps - 1) / k;
    if (nck > 0) NH_TRY(ensure(c, c->traj, 3 * vb * (size_t)nck));
    for (Buf& b : c->w) NH_TRY(ensure(c, b, vb));
  }

  c->st.fwd_iters = 0;
  c->st.fwd_steps = nsteps;
  c->st.launches_fwd = 0;
  const long long kl0 = c->kernel_launches;
  c->st.t_kernel_fwd_s = 0;
  double tk = 0;
  int used = 0;
  R* const w[4] = {(R*)c->w[0].p, (R*)c->w[1].p, (R*)c->w[2].p, (R*)c->w[3].p};
  auto state = [&](int m) -> R* {   // T^m, null for T^0 = 0
    if (m < 1) return nullptr;
    return k == 0 ? traj + (size_t)(m - 1) * g.ng : w[m & 3];
  };
  for (int n = 1; n <= nsteps; ++n) {
    const R* const h[3] = {state(n - 1), state(n - 2), state(n - 3)};
    R* x = state(n);
    R* ck = nullptr;
    const bool ckpt = k > 0 && n % k == 0 && n < nsteps;
    if (ckpt) ck = (R*)c->traj.p + (size_t)(n / k - 1) * 3 * g.ng;
    NH_TRY(forward_step<R>(c, n, h, x, qsrc, dt, q_t[n - 1], T_surf + (size_t)(n - 1) * g.nxy,
                           ck, 0, used));
    if (ckpt) {
      NH_TRY(flush_steps(c));               // queued steps precede the copies on the stream
      for (int d = 1; d <= 2 && n - d >= 1; ++d)
        NH_HIP(c, hipMemcpyAsync(ck + (size_t)d * g.ng, state(n - d), vb, hipMemcpyDeviceToDevice, c->stream));
    }
    if (c->profile && ++used == kEvPairs) {
      NH_TRY(collect_events(c, used, &tk));
      used = 0;
    }
  }
  NH_TRY(collect_events(c, used, &tk));
  NH_HIP(c, hipStreamSynchronize(c->stream));
  c->st.t_kernel_fwd_s = tk;
  c->st.launches_fwd = c->kernel_launches - kl0;
  NH_TRY(check_flag(c));

  int max_it = 0, any = 0;
  double worst = 0;
  long long isum = 0;
  NH_TRY(summarize(c, 0, nsteps, &isum, &max_it, &worst, &any));
  c->st.fwd_iters = isum;
  c->st.max_step_iters = max_it;
  c->st.worst_rel_res = worst;
  // algorithmic bytes from the per-step iteration counts
  {
    std::vector<int> it(nsteps);
    NH_HIP(c, hipMemcpyAsync(it.data(), step_out(c, 0, 0).iters, sizeof(int) * nsteps, hipMemcpyDeviceToHost, c->stream));
    NH_HIP(c, hipStreamSynchronize(c->stream));
    double bytes = 0;
    for (int n = 1; n <= nsteps; ++n)
      bytes += step_bytes(g, sizeof(R), nh::kForward, it[n - 1], c->jacobi_k > 0, cheb_degree(c));
    c->st.bytes_alg_fwd = bytes;
  }
  c->saved_prec = sizeof(R);
  c->saved_dt = dt;
  c->saved_qt.assign(q_t, q_t + nsteps);
  c->st.workspace_bytes = c->ws_bytes;
  c->st.peak_workspace_bytes = c->ws_peak;
  c->st.t_fwd_s = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  return status_to_code(c, any);
}

// The projected initial guess of adjoint step n - 1, once mu^n (in M[n % ring])
// is solved: A mu^n, the new row of the window's Gram matrix and the
// right-hand-side projections, the small solve, and x0 into c->pguess. gnext
// is the top-plane source of step n - 1. Queued on the context's stream after
// step n; no host synchronisation.
template <typename R>
nh_status proj_prepare(nh_ctx* c, int n, int N, R* const* M, const R* gnext, double dt) {
  const Geom& g = c->geom;
  nh::ProjWin<R> W{};
  W.k = std::min(nh::kProjMax, N - n + 1);
  for (int j = 0; j < W.k; ++j) {
    W.slot[j] = (n + j) % nh::kProjRing;
    W.w[j] = M[W.slot[j]];
  }
  R* y = (R*)c->pguess.p;
  double* part = (double*)c->ppart.p;
  nh::ProjState* st = (nh::ProjState*)c->pstate.p;
  const nh::Coef<R> cf{(R)(2.0 * dt / (c->hx * c->hx)), (R)(2.0 * dt / (c->hy * c->hy)),
                       (R)(2.0 * dt / (c->hz * c->hz)), (R)(dt * c->robin / c->hz), g.nz - 1};
  const long long blocks = (g.ng + nh::kProjBlock - 1) / nh::kProjBlock;
  hipLaunchKernelGGL(nh::proj_apply_kernel<R>, dim3((unsigned)blocks), dim3(nh::kProjBlock), 0, c->stream, g,
                     (const R*)c->alpha.p, W.w[0], y, cf);
  hipLaunchKernelGGL(nh::proj_dots_kernel<R>, dim3(nh::kProjDotBlocks), dim3(nh::kProjBlock), 0, c->stream, W,
                     (const R*)y, gnext, g.ng, g.nxy, part);
  hipLaunchKernelGGL(nh::proj_solve_kernel<R>, dim3(1), dim3(nh::kProjBlock), 0, c->stream, W,
                     (const double*)part, nh::kProjDotBlocks, st);
  hipLaunchKernelGGL(nh::proj_combine_kernel<R>, dim3((unsigned)blocks), dim3(nh::kProjBlock), 0, c->stream, W,
                     (const nh::ProjState*)st, y, g.ng);
  NH_HIP(c, hipGetLastError());
  return NH_OK;
}

template <typename R>
nh_status do_adjoint(nh_ctx* c, const R* gsurf, double* G, R* dq, R* dT0) {
  auto t0 = std::chrono::steady_clock::now();
  const Range range(sizeof(R) == 4 ? "nh_adjoint" : "nh_adjoint_f64");
  if (!c) return NH_EINVAL;
  if (!gsurf || !G) return fail(c, NH_EINVAL, "null pointer argument");
  if (c->saved_prec != (int)sizeof(R))
    return fail(c, NH_ESTATE, "no saved forward of this precision (call the matching nh_forward first)");
  const Geom& g = c->geom;
  const int N = c->saved_nsteps, k = c->ckpt_every;
  const double dt = c->saved_dt;
  const size_t vb = sizeof(R) * (size_t)g.ng;
  // guess mode 3 projects the adjoint solves' initial guesses (CG only)
  const bool proj = c->guess == 3 && c->jacobi_k == 0;
  const int ring = proj ? nh::kProjRing : 4;
  R* M[nh::kProjRing] = {};
  for (int i = 0; i < ring; ++i) {
    NH_TRY(ensure(c, c->mu[i], vb));
    M[i] = (R*)c->mu[i].p;
  }
  if (proj) {
    NH_TRY(ensure(c, c->pguess, vb));
    NH_TRY(ensure(c, c->ppart, sizeof(double) * nh::kProjVals * nh::kProjDotBlocks));
    NH_TRY(ensure(c, c->pstate, sizeof(nh::ProjState)));
  }
  auto mu_state = [&](int m) -> const R* { return m > N ? nullptr : M[m % ring]; };   // mu^{N+1} = 0
  NH_TRY(fill<double>(c, G, g.ng, 0.0));
  NH_TRY(ensure_events(c));

  c->st.adj_steps = N;
  c->st.recompute_steps = 0;
  c->st.launches_adj = 0;
  const long long kl0 = c->kernel_launches;
  double tk = 0;
  int used = 0;
  double bytes = 0;
  std::vector<int> it_rec;

  auto adj_step = [&](int n, const R* Tn) -> nh_status {
    StepArgs<R> S;
    base_args<R>(c, S, dt);
    S.mode = nh::kAdjoint;
    S.x = M[n % ring];
    S.surf_out = dq ? dq + (size_t)(n - 1) * g.nxy : nullptr;   // dL/dq^n = dt mu^n on k = 0
    S.surf_scale = (R)dt;
    const R* const h[3] = {mu_state(n + 1), mu_state(n + 2), mu_state(n + 3)};
    set_guess<R>(c, S, h, N - n, step_out(c, 1, 0).iters, [N](int jj) { return N - jj; });
    if (proj && n < N) {
      // x0 = the projection that proj_prepare left in pguess; b still from mu^{n+1}
      S.gmode = 3;
      S.xprev2 = (const R*)c->pguess.p;
      S.xprev3 = nullptr;
      S.gi = nullptr;
    }
    S.top_src = gsurf + (size_t)(n - 1) * g.nxy;
    S.top_scale = R(1);
    S.T_grad = Tn;
    S.G = G;
    StepOut o = step_out(c, 1, n - 1);
    S.out_iters = o.iters;
    S.out_relres = o.relres;
    S.out_status = o.status;
    NH_TRY(launch_step<R>(c, S, used, nullptr));
    if (c->profile && ++used == kEvPairs) {
      NH_TRY(collect_events(c, used, &tk));
      used = 0;
    }
    if (proj && n > 1) NH_TRY(proj_prepare<R>(c, n, N, M, gsurf + (size_t)(n - 2) * g.nxy, dt));
    return NH_OK;
  };

  if (k == 0) {
    const R* traj = (const R*)c->traj.p;
    for (int n = N; n >= 1; --n) NH_TRY(adj_step(n, traj + (size_t)(n - 1) * g.ng));
  } else {
    NH_TRY(ensure(c, c->seg, vb * (size_t)std::min(k, N)));
    R* seg = (R*)c->seg.p;
    const int nseg = (N + k - 1) / k;
    const R* qxy = (const R*)c->qxy.p;
    for (int s_idx = nseg - 1; s_idx >= 0; --s_idx) {
      const int s = s_idx * k, e = std::min(s + k, N);
      // T^m of this segment: recomputed into seg above s, from the checkpoint at and below s
      auto state = [&](int m) -> const R* {
        if (m < 1) return nullptr;
        if (m > s) return seg + (size_t)(m - s - 1) * g.ng;
        return (const R*)c->traj.p + ((size_t)(s_idx - 1) * 3 + (size_t)(s - m)) * g.ng;
      };
      {
        const Range rec_range("segment recompute");
        for (int n = s + 1; n <= e; ++n) {
          const R* const h[3] = {state(n - 1), state(n - 2), state(n - 3)};
          NH_TRY(forward_step<R>(c, n, h, seg + (size_t)(n - s - 1) * g.ng, qxy, dt,
                                 c->saved_qt[n - 1], nullptr, nullptr, 2, used));
          ++c->st.recompute_steps;
          if (c->profile && ++used == kEvPairs) {
            NH_TRY(collect_events(c, used, &tk));
            used = 0;
          }
        }
      }
      {
        const Range adj_range("segment adjoint");
        for (int n = e; n >= s + 1; --n) NH_TRY(adj_step(n, seg + (size_t)(n - s - 1) * g.ng));
      }
    }
  }
  NH_TRY(flush_steps(c));                   // queued steps precede the copy on the stream
  if (dT0) NH_HIP(c, hipMemcpyAsync(dT0, M[1 % ring], vb, hipMemcpyDeviceToDevice, c->stream));   // mu^1
  NH_TRY(collect_events(c, used, &tk));
  NH_HIP(c, hipStreamSynchronize(c->stream));
  c->st.launches_adj = c->kernel_launches - kl0;
  c->st.t_kernel_adj_s = tk;
  NH_TRY(check_flag(c));

  int max_it = 0, any = 0;
  double worst = 0;
  long long isum = 0;
  NH_TRY(summarize(c, 1, N, &isum, &max_it, &worst, &any));
  c->st.adj_iters = isum;
  c->st.max_step_iters = max_it;
  c->st.worst_rel_res = worst;
  std::vector<int> it(N);
  NH_HIP(c, hipMemcpyAsync(it.data(), step_out(c, 1, 0).iters, sizeof(int) * N, hipMemcpyDeviceToHost, c->stream));
  NH_HIP(c, hipStreamSynchronize(c->stream));
  for (int n = 1; n <= N; ++n)
    bytes += step_bytes(g, sizeof(R), nh::kAdjoint, it[n - 1], c->jacobi_k > 0, cheb_degree(c));
  c->st.recompute_iters = 0;
  if (k > 0) {
    long long rsum = 0;
    int rmax = 0, rany = 0;
    double rworst = 0;
    NH_TRY(summarize(c, 2, N, &rsum, &rmax, &rworst, &rany));
    c->st.recompute_iters = rsum;
    any |= rany;
    std::vector<int> ir(N);
    NH_HIP(c, hipMemcpyAsync(ir.data(), step_out(c, 2, 0).iters, sizeof(int) * N, hipMemcpyDeviceToHost, c->stream));
    NH_HIP(c, hipStreamSynchronize(c->stream));
    for (int n = 1; n <= N; ++n)
      bytes += step_bytes(g, sizeof(R), nh::kForward, ir[n - 1], c->jacobi_k > 0, cheb_degree(c));
  }
  c->st.bytes_alg_adj = bytes;
  c->st.workspace_bytes = c->ws_bytes;
  c->st.peak_workspace_bytes = c->ws_peak;
  c->st.t_adj_s = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  return status_to_code(c, any);
}

// dL/dq_xy and dL/dq_t of the separable source q^n = q_t[n-1] q_xy (either
// output may be null): the adjoint sweep with its dL/dq^n series, then
// the chain rule through the product on the device (FP64, fixed order).
template <typename R>
nh_status do_source_grad(nh_ctx* c, const R* gsurf, double* G, double* d_qxy, double* d_qt) {
  if (!c) return NH_EINVAL;
  if (!gsurf || !G) return fail(c, NH_EINVAL, "null pointer argument");
  if (c->saved_prec != (int)sizeof(R))
    return fail(c, NH_ESTATE, "no saved forward of this precision (call the matching nh_forward first)");
  const int N = c->saved_nsteps;
  const long long nxy = c->geom.nxy;
  R* dq = nullptr;
  if (d_qxy || d_qt) {
    NH_TRY(ensure(c, c->srcq, sizeof(R) * (size_t)N * (size_t)nxy));
    dq = (R*)c->srcq.p;
  }
  nh_status st = do_adjoint<R>(c, gsurf, G, dq, nullptr);
  if (st != NH_OK && st != NH_ENOCONV) return st;
  if (d_qxy) {
    NH_TRY(ensure(c, c->srcqt, sizeof(double) * (size_t)N));
    NH_HIP(c, hipMemcpyAsync(c->srcqt.p, c->saved_qt.data(), sizeof(double) * (size_t)N, hipMemcpyHostToDevice,
                             c->stream));
    const int blocks = (int)std::min<long long>((nxy + nh::kSrcBlock - 1) / nh::kSrcBlock, 4096);
    hipLaunchKernelGGL(nh::qxy_grad_kernel<R>, dim3(blocks), dim3(nh::kSrcBlock), 0, c->stream, (const R*)dq,
                       (const double*)c->srcqt.p, N, nxy, d_qxy);
    NH_HIP(c, hipGetLastError());
  }
  if (d_qt) {
    hipLaunchKernelGGL(nh::qt_grad_kernel<R>, dim3(N), dim3(nh::kSrcBlock), 0, c->stream, (const R*)dq,
                       (const R*)c->qxy.p, nxy, d_qt);
    NH_HIP(c, hipGetLastError());
  }
  NH_HIP(c, hipStreamSynchronize(c->stream));
  return st;
}

// noalloc: use the device's static scratch for the partial sums instead of a
// context workspace, and return once the work is queued (no allocation, no
// synchronisation).
template <typename R>
nh_status do_tv(nh_ctx* c, const R* alpha, double eps, double weight, double* value, double* grad,
                int accumulate, bool noalloc = false) {
  if (!c) return NH_EINVAL;
  if (!c->grid_set) return fail(c, NH_ESTATE, "nh_set_grid has not been called");
  if (!alpha || !value || !grad) return fail(c, NH_EINVAL, "null pointer argument");
  if (!(eps > 0) || !std::isfinite(eps)) return fail(c, NH_EINVAL, "eps must be finite and > 0");
  if (!std::isfinite(weight)) return fail(c, NH_EINVAL, "weight must be finite");
  if (accumulate != 0 && accumulate != 1) return fail(c, NH_EINVAL, "accumulate must be 0 or 1");
  const long long ng = (long long)c->nx * c->ny * c->nz;
  const int blocks = (int)std::min<long long>((ng + nh::kTvBlock - 1) / nh::kTvBlock, nh::kTvMaxBlocks);
  double* partial = nullptr;
  if (noalloc) {
    if (!c->scratch) return fail(c, NH_ESTATE, "the device scratch array was not resolved");
    if (blocks > kScratchDoubles)
      return fail(c, NH_EINVAL, "grid needs " + std::to_string(blocks) + " partial sums, the scratch holds " +
                                    std::to_string(kScratchDoubles));
    partial = c->scratch;
  } else {
    NH_TRY(ensure(c, c->tvpart, sizeof(double) * (size_t)blocks));
    partial = (double*)c->tvpart.p;
  }
  nh::TvArgs<R> A;
  A.alpha = alpha;
  A.nx = c->nx;
  A.ny = c->ny;
  A.nz = c->nz;
  A.nxy = (long long)c->nx * c->ny;
  A.ng = ng;
  A.ix2 = (R)(1.0 / (c->hx * c->hx));
  A.iy2 = (R)(1.0 / (c->hy * c->hy));
  A.iz2 = (R)(1.0 / (c->hz * c->hz));
  A.eps2 = (R)(eps * eps);
  A.scale = weight * c->hx * c->hy * c->hz;
  A.grad = grad;
  A.accumulate = accumulate;
  A.partial = partial;
  hipLaunchKernelGGL(nh::tv_kernel<R>, dim3(blocks), dim3(nh::kTvBlock), 0, c->stream, A);
  NH_HIP(c, hipGetLastError());
  hipLaunchKernelGGL(nh::tv_finish_kernel, dim3(1), dim3(nh::kTvBlock), 0, c->stream, (const double*)A.partial,
                     blocks, A.scale, value);
  NH_HIP(c, hipGetLastError());
  if (!noalloc) NH_HIP(c, hipStreamSynchronize(c->stream));
  return NH_OK;
}

}  // namespace

extern "C" {

nh_status nh_tv(nh_ctx* c, const float* alpha, double eps, double weight, double* value, double* grad,
                int accumulate) {
  return do_tv<float>(c, alpha, eps, weight, value, grad, accumulate);
}

nh_status nh_tv_f64(nh_ctx* c, const double* alpha, double eps, double weight, double* value, double* grad,
                    int accumulate) {
  return do_tv<double>(c, alpha, eps, weight, value, grad, accumulate);
}

nh_status nh_tv_noalloc(nh_ctx* c, const float* alpha, double eps, double weight, double* value, double* grad,
                        int accumulate) {
  return do_tv<float>(c, alpha, eps, weight, value, grad, accumulate, true);
}

nh_status nh_create(nh_ctx** out, int hip_device, void* hip_stream) {
  if (!out) return NH_EINVAL;
  *out = nullptr;
  nh_ctx* c = new (std::nothrow) nh_ctx();
  if (!c) return NH_ENOMEM;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || hip_device < 0 || hip_device >= ndev) {
    delete c;
    return NH_EINVAL;
  }
  c->device = hip_device;
  if (hipSetDevice(hip_device) != hipSuccess) { delete c; return NH_EHIP; }
  c->stream = (hipStream_t)hip_stream;  // NULL: the null stream
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, hip_device) != hipSuccess) { delete c; return NH_EHIP; }
  c->num_cu = prop.multiProcessorCount;
  int khz = 0;
  if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, hip_device) == hipSuccess && khz > 0)
    c->wallclock_khz = khz;
  int o32 = 0, o64 = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&o32, (const void*)nh::step_kernel<float>,
                                                   nh::Cfg<float>::kBlock, 0) != hipSuccess ||
      hipOccupancyMaxActiveBlocksPerMultiprocessor(&o64, (const void*)nh::step_kernel<double>,
                                                   nh::Cfg<double>::kBlock, 0) != hipSuccess) {
    delete c;
    return NH_EHIP;
  }
  c->occ_f32 = std::max(1, o32);
  c->occ_f64 = std::max(1, o64);
  {
    int ro = 0;
    if (hipFuncSetAttribute((const void*)nh::resident_step_kernel<64>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)nh::kResLdsBytes) == hipSuccess &&
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&ro, (const void*)nh::resident_step_kernel<64>,
                                                     nh::kResBlock, nh::kResLdsBytes) == hipSuccess)
      c->res_occ = ro;
    (void)hipGetLastError();
    if (std::getenv("NH_TRACE_STEP"))
      std::fprintf(stderr, "[nh] resident kernel: %zu B LDS, %d workgroups per CU\n", nh::kResLdsBytes, c->res_occ);
    int jo = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&jo, (const void*)nh::jacobi_step_kernel<nh::kJacH>,
                                                     nh::kJacBlock, 0) == hipSuccess)
      c->jac_occ = jo;
    (void)hipGetLastError();
  }
  if (scratch_of(hip_device, &c->scratch) != hipSuccess) {
    delete c;
    return NH_EHIP;
  }
  if (const char* e = std::getenv("NH_TRACE_STEP")) c->trace_step = std::atoi(e);
  if (const char* e = std::getenv("NH_TRACE_RANK")) c->trace_rank = std::atoi(e);
  *out = c;
  return NH_OK;
}

nh_status nh_set_grid(nh_ctx* c, int nx, int ny, int nz, double hx, double hy, double hz) {
  if (!c) return NH_EINVAL;
  if (nx < 1 || ny < 1 || nz < 1) return fail(c, NH_EINVAL, "grid dimensions must be >= 1");
  if ((long long)nx * ny * nz > (1LL << 40)) return fail(c, NH_EINVAL, "grid too large");
  if (!(hx > 0) || !(hy > 0) || !(hz > 0) || !std::isfinite(hx) || !std::isfinite(hy) || !std::isfinite(hz))
    return fail(c, NH_EINVAL, "spacings must be finite and > 0");
  if (c->periodic && (nx < 3 || ny < 3)) return fail(c, NH_EINVAL, "periodic lateral faces need nx, ny >= 3");
  drop_forward(c);
  c->nx = nx; c->ny = ny; c->nz = nz;
  c->hx = hx; c->hy = hy; c->hz = hz;
  c->grid_set = true;
  NH_TRY(release(c, c->alpha));
  NH_TRY(release(c, c->z));
  NH_TRY(release(c, c->p0));
  NH_TRY(release(c, c->p1));
  for (Buf& b : c->mu) NH_TRY(release(c, b));
  NH_TRY(release(c, c->pguess));
  plan(c, c->occ_f32, nh::Cfg<float>::kBlock);
  return NH_OK;
}

nh_status nh_set_solver(nh_ctx* c, double rtol, int max_iter, int checkpoint_every) {
  if (!c) return NH_EINVAL;
  if (!(rtol > 0) || !(rtol < 1)) return fail(c, NH_EINVAL, "rtol must be in (0, 1)");
  if (max_iter < 1) return fail(c, NH_EINVAL, "max_iter must be >= 1");
  if (checkpoint_every < 0) return fail(c, NH_EINVAL, "checkpoint_every must be >= 0");
  drop_forward(c);
  c->rtol = rtol;
  c->max_iter = max_iter;
  c->ckpt_every = checkpoint_every;
  return NH_OK;
}

nh_status nh_forward(nh_ctx* c, const float* alpha, const float* q_xy, const double* q_t, double dt,
                     int nsteps, float* T_surf) {
  return do_forward<float>(c, alpha, q_xy, q_t, dt, nsteps, T_surf);
}

nh_status nh_adjoint(nh_ctx* c, const float* dL_dTsurf, double* dL_dalpha) {
  return do_adjoint<float>(c, dL_dTsurf, dL_dalpha, nullptr, nullptr);
}

nh_status nh_forward_f64(nh_ctx* c, const double* alpha, const double* q_xy, const double* q_t, double dt,
                         int nsteps, double* T_surf) {
  return do_forward<double>(c, alpha, q_xy, q_t, dt, nsteps, T_surf);
}

nh_status nh_adjoint_f64(nh_ctx* c, const double* dL_dTsurf, double* dL_dalpha) {
  return do_adjoint<double>(c, dL_dTsurf, dL_dalpha, nullptr, nullptr);
}

nh_status nh_adjoint_vjp(nh_ctx* c, const float* dL_dTsurf, double* dL_dalpha, float* dL_dq, float* dL_dT0) {
  return do_adjoint<float>(c, dL_dTsurf, dL_dalpha, dL_dq, dL_dT0);
}

nh_status nh_adjoint_vjp_f64(nh_ctx* c, const double* dL_dTsurf, double* dL_dalpha, double* dL_dq,
                             double* dL_dT0) {
  return do_adjoint<double>(c, dL_dTsurf, dL_dalpha, dL_dq, dL_dT0);
}

nh_status nh_adjoint_source_grad(nh_ctx* c, const float* dL_dTsurf, double* dL_dalpha, double* dL_dqxy,
                                 double* dL_dqt) {
  return do_source_grad<float>(c, dL_dTsurf, dL_dalpha, dL_dqxy, dL_dqt);
}

nh_status nh_adjoint_source_grad_f64(nh_ctx* c, const double* dL_dTsurf, double* dL_dalpha, double* dL_dqxy,
                                     double* dL_dqt) {
  return do_source_grad<double>(c, dL_dTsurf, dL_dalpha, dL_dqxy, dL_dqt);
}

nh_status nh_get_state(nh_ctx* c, int n, void* out) {
  if (!c) return NH_EINVAL;
  if (!out) return fail(c, NH_EINVAL, "null pointer argument");
  if (!c->saved_prec) return fail(c, NH_ESTATE, "no saved forward");
  if (n < 1 || n > c->saved_nsteps) return fail(c, NH_EINVAL, "step index out of range");
  const size_t vb = (size_t)c->saved_prec * (size_t)c->geom.ng;
  const void* src = nullptr;
  if (c->ckpt_every == 0) {
    src = (const char*)c->traj.p + (size_t)(n - 1) * vb;
  } else if (n % c->ckpt_every == 0 && n < c->saved_nsteps) {
    src = (const char*)c->traj.p + (size_t)(n / c->ckpt_every - 1) * 3 * vb;
  } else if (n == c->saved_nsteps) {
    src = c->w[n & 3].p;
  } else {
    return fail(c, NH_ESTATE, "state not held (checkpointing keeps every k-th state and the last)");
  }
  NH_HIP(c, hipMemcpyAsync(out, src, vb, hipMemcpyDeviceToDevice, c->stream));
  NH_HIP(c, hipStreamSynchronize(c->stream));
  return NH_OK;
}

nh_status nh_apply_A(nh_ctx* c, const float* alpha, const float* x, float* y, double dt) {
  if (!c) return NH_EINVAL;
  if (!c->grid_set) return fail(c, NH_ESTATE, "nh_set_grid has not been called");
  if (!alpha || !x || !y) return fail(c, NH_EINVAL, "null pointer argument");
  if (x == y) return fail(c, NH_EINVAL, "y must not alias x");
  if (!(dt >= 0) || !std::isfinite(dt)) return fail(c, NH_EINVAL, "dt must be finite and >= 0");
  plan(c, c->occ_f32, nh::Cfg<float>::kBlock);
  const Geom& g = c->geom;
  const int blocks = std::min(g.ntiles, std::max(1, c->occ_f32 * c->num_cu));
  const nh::Coef<float> cf{(float)(2.0 * dt / (c->hx * c->hx)), (float)(2.0 * dt / (c->hy * c->hy)),
                           (float)(2.0 * dt / (c->hz * c->hz)), (float)(dt * c->robin / c->hz), g.nz - 1};
  hipLaunchKernelGGL(nh::apply_kernel<float>, dim3(blocks), dim3(nh::Cfg<float>::kBlock), 0, c->stream, g, alpha, x, y,
                     cf);
  NH_HIP(c, hipGetLastError());
  NH_HIP(c, hipStreamSynchronize(c->stream));
  return NH_OK;
}

nh_status nh_set_launch(nh_ctx* c, int team_blocks_max, int tile_z, int profile) {
  if (!c) return NH_EINVAL;
  if (team_blocks_max < 0 || tile_z < 0) return fail(c, NH_EINVAL, "negative launch setting");
  drop_forward(c);
  c->team_max = team_blocks_max;
  c->tile_z = tile_z;
  c->profile = profile != 0;
  if (c->grid_set) plan(c, c->occ_f32, nh::Cfg<float>::kBlock);
  return NH_OK;
}

nh_status nh_set_boundary(nh_ctx* c, int periodic_xy, double robin_h) {
  if (!c) return NH_EINVAL;
  if (periodic_xy != 0 && periodic_xy != 1) return fail(c, NH_EINVAL, "periodic_xy must be 0 or 1");
  if (!(robin_h >= 0) || !std::isfinite(robin_h)) return fail(c, NH_EINVAL, "robin_h must be finite and >= 0");
  if (periodic_xy && c->grid_set && (c->nx < 3 || c->ny < 3))
    return fail(c, NH_EINVAL, "periodic lateral faces need nx, ny >= 3");
  drop_forward(c);
  c->periodic = periodic_xy;
  c->robin = robin_h;
  if (c->grid_set) plan(c, c->occ_f32, nh::Cfg<float>::kBlock);
  return NH_OK;
}

nh_status nh_set_jacobi_sweeps(nh_ctx* c, int k) {
  if (!c) return NH_EINVAL;
  if (k < 0 || k > 100000) return fail(c, NH_EINVAL, "the number of Jacobi sweeps must be in [0, 100000]");
  drop_forward(c);
  c->jacobi_k = k;
  if (c->grid_set) plan(c, c->occ_f32, nh::Cfg<float>::kBlock);
  return NH_OK;
}

nh_status nh_set_cg_variant(nh_ctx* c, int variant) {
  if (!c) return NH_EINVAL;
  if (variant < 0 || variant > 2) return fail(c, NH_EINVAL, "variant must be 0, 1 or 2");
  drop_forward(c);
  c->variant = variant;
  if (variant != 0) c->cheb_m = 1;           // the polynomial preconditioner needs the two-reduction form
  return NH_OK;
}

nh_status nh_set_preconditioner(nh_ctx* c, int degree) {
  if (!c) return NH_EINVAL;
  if (degree < 1 || degree > nh::kChebMax)
    return fail(c, NH_EINVAL, "preconditioner degree must be between 1 and 16");
  drop_forward(c);
  c->cheb_m = degree;
  if (degree >= 2) c->variant = 0;
  return NH_OK;
}

nh_status nh_get_step_iters(const nh_ctx* c, int sweep, int* iters) {
  if (!c) return NH_EINVAL;
  nh_ctx* m = const_cast<nh_ctx*>(c);
  if (!iters) return fail(m, NH_EINVAL, "null pointer argument");
  if (sweep < 0 || sweep > 2) return fail(m, NH_EINVAL, "sweep must be 0, 1 or 2");
  if (!c->saved_prec || !c->steps.p) return fail(m, NH_ESTATE, "no saved forward");
  const int N = c->saved_nsteps;
  NH_HIP(m, hipMemcpyAsync(iters, step_out(m, sweep, 0).iters, sizeof(int) * (size_t)N, hipMemcpyDeviceToHost,
                           c->stream));
  NH_HIP(m, hipStreamSynchronize(c->stream));
  return NH_OK;
}

nh_status nh_set_initial_guess(nh_ctx* c, int mode) {
  if (!c) return NH_EINVAL;
  if (mode < 0 || mode > 3) return fail(c, NH_EINVAL, "initial guess mode must be 0, 1, 2 or 3");
  drop_forward(c);
  c->guess = mode;
  return NH_OK;
}

nh_status nh_set_barrier_timeout(nh_ctx* c, double seconds) {
  if (!c) return NH_EINVAL;
  if (!(seconds >= 0) || !std::isfinite(seconds)) return fail(c, NH_EINVAL, "timeout must be finite and >= 0");
  c->barrier_timeout_s = seconds;
  return NH_OK;
}

nh_status nh_get_stats(const nh_ctx* c, nh_stats* out) {
  if (!c || !out) return NH_EINVAL;
  *out = c->st;
  out->workspace_bytes = c->ws_bytes;
  out->peak_workspace_bytes = c->ws_peak;
  return NH_OK;
}

const char* nh_last_error(const nh_ctx* c) {
  if (!c) return "null context";
  return c->err.c_str();
}

void nh_destroy(nh_ctx* c) {
  if (!c) return;
  (void)hipSetDevice(c->device);
  (void)hipStreamSynchronize(c->stream);
  Buf* bufs[] = {&c->trace, &c->alpha, &c->qxy, &c->z, &c->p0, &c->p1, &c->u1, &c->vw0, &c->vw1,
                 &c->vs0, &c->vs1, &c->traj, &c->seg, &c->slots, &c->steps, &c->flag, &c->tvpart, &c->srcq, &c->srcqt,
                 &c->jt[0], &c->jt[1], &c->pguess, &c->ppart, &c->pstate, &c->dmaxb, &c->xface};
  for (Buf* b : bufs) release(c, *b);
  for (Buf& b : c->mu) release(c, b);
  for (Buf& b : c->w) release(c, b);
  for (auto e : c->ev) (void)hipEventDestroy(e);
  delete c;
}

nh_status nh_stream_probe_f32(const float* const* in6, float* const* out5, int nx, int ny, int nz,
                              void* hip_stream) {
  if (!in6 || !out5) return NH_EINVAL;
  if (nx <= 0 || ny <= 0 || nz <= 0 || nx % 64 != 0 || ny % 16 != 0) return NH_EINVAL;
  const long long tiles = (long long)(nx / 64) * (ny / 16);
  if (tiles > 1 << 20 || (long long)nx * ny * nz > (1ll << 40)) return NH_EINVAL;
  nh::ProbeArgs A;
  for (int k = 0; k < 6; ++k) {
    if (!in6[k]) return NH_EINVAL;
    A.in[k] = in6[k];
  }
  for (int k = 0; k < 5; ++k) {
    if (!out5[k]) return NH_EINVAL;
    A.out[k] = out5[k];
  }
  A.nx = nx;
  A.ny = ny;
  A.nz = nz;
  hipLaunchKernelGGL(nh::stream_probe_kernel, dim3((unsigned)tiles), dim3(1024), 0, (hipStream_t)hip_stream, A);
  return hipGetLastError() == hipSuccess ? NH_OK : NH_EHIP;
}

nh_status nh_copy_f32(const float* src, float* dst, size_t n, void* hip_stream) {
  if (!src || !dst) return NH_EINVAL;
  if (n == 0) return NH_OK;
  int blocks = (int)std::min<size_t>((n + 255) / 256, 8192);
  hipLaunchKernelGGL(nh::copy_kernel<float>, dim3(blocks), dim3(256), 0, (hipStream_t)hip_stream, src, dst,
                     (long long)n);
  return hipGetLastError() == hipSuccess ? NH_OK : NH_EHIP;
}

}  // extern "C"
