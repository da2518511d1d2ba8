// nh_serve.hip -- continuous-batching server for forward+adjoint inversion jobs.
//
// A job is one reconstruction request: a diffusivity field, a source, and the
// surface measurements it is compared with (mean squared error). The server
// keeps every admitted job's state resident in HBM and advances all of them
// together: each tick is ONE cooperative launch (nh::batch_resident_kernel,
// or nh::batch_run_kernel with the streaming step code) in which every
// active job's team of workgroups runs implicit-Euler steps
// (forward, or adjoint after its forward has finished) with its own team
// reductions -- the same step code as the single-problem path -- until its
// CG iterations in this launch reach the tick's budget. Between ticks the host
// reads one progress record per job, retires finished jobs, frees their
// memory and admits queued jobs in arrival order while both the HBM budget
// and the co-resident workgroup budget allow -- so requests that arrive while
// others run join at the next tick. A job's team size and tiling depend only
// on the job itself and slices end only between steps, so its result is
// bit-identical whether it runs alone or among others.
#include "nefty_heat.h"
#include "nh_kernels.hpp"
#include "nh_policy.h"
#include "nh_resident.hpp"

#include <hip/hip_runtime.h>
#include <rocprofiler-sdk-roctx/roctx.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <string>
#include <vector>

namespace nh {

// One job's slice of work in a launch. `S` holds the job's buffers and
// constants; the per-step fields are set in the kernel.
struct JobRun {
  StepArgs<float> S;
  const float* qscale;        // forward: top-plane source scale of step n at [n-1]
  float* traj;                // T^n at (n-1) * ng
  float* surf;                // S^n at (n-1) * nxy
  const float* gsurf;         // dL/dS^n at (n-1) * nxy
  int* it_out;                // per-step iterations [2][nsteps]: forward, then adjoint
  double* rel_out;            // per-step relative residuals, same layout
  int* st_out;                // per-step status flags, same layout
  float* mu[4];               // adjoint states, mu^n in mu[n & 3]
  int mode;                   // kForward or kAdjoint
  int n0;                     // first step of the slice (the adjoint counts down to 1)
  int nsteps;
  long long cost;             // cost of one iteration of one workgroup (voxel units)
  long long budget;           // the slice ends once (iterations + steps) * cost would pass this
};

// Per-job progress of a launch, written by the job's rank 0.
struct JobProg {
  int steps;
  int status;
  long long iters;
  long long t0, t1;           // wall clock of rank 0 at the start and end of the slice
};

constexpr int kMaxSliceSteps = 255;       // steps per slice (with max_iter <= 30000 its team
                                           // reductions stay below the 2^24 epochs of a launch)

// The slice of one job for one workgroup: steps of the job until its
// iterations in this launch reach the budget. `step(S, V)` runs one step of
// the team. The loop and its exit test depend only on reduced values, so
// every workgroup of a team runs the same steps (a barrier timeout aside,
// which every member then reaches within its own bounded waits).
typedef __attribute__((address_space(4))) const JobRun CJobRun;

constexpr int kGuessPeriod = 32;

// The loop state of a slice, kept in LDS between steps so that none of it is
// live in registers through the (inlined) step: thread 0 writes it after a
// step, and every thread reads it back after a barrier.
struct SliceState {
  long long t0;
  long long iters;
  unsigned long long ep;
  int n, steps, status;
  int pc[3];
};

template <typename StepF>
__device__ __forceinline__ void run_slice(const CJobRun& J, int2 m, JobProg* prog, SliceState* ss, StepF step) {
  const bool fwd = J.mode == kForward;
  // Adaptive initial guess: in each period of kGuessPeriod steps of a sweep
  // the first step starts from the previous state, the second from the
  // extrapolation, the rest from whichever needed fewer iterations. j is a
  // step's position in its sweep; counts of probes run by earlier launches
  // come from the per-step record, later ones from this loop.
  auto pos = [&](int nn) { return fwd ? nn - 1 : J.nsteps - nn; };
  auto slot_of = [&](int jj) { return fwd ? jj : 2 * J.nsteps - 1 - jj; };
  if (threadIdx.x == 0) {
    ss->t0 = wall_clock64();
    ss->iters = 0;
    ss->n = J.n0;
    ss->steps = 0;
    ss->status = 0;
    // one running epoch through the slice: each step starts from the epoch of
    // its predecessor's last team reduction, so epochs stay unique within the
    // launch and consecutive reductions alternate between the slot banks
    ss->ep = J.S.epoch_base;
    const int j0 = pos(J.n0), base = j0 - j0 % kGuessPeriod;
    for (int d = 0; d < 3; ++d) ss->pc[d] = base + d < j0 ? J.it_out[slot_of(base + d)] : -1;
  }
  __syncthreads();
  const StepArgs<float>& S = (const StepArgs<float>&)J.S;
  while (true) {
    // (wave-uniform: the step's pointers below then live in scalar registers,
    // which leaves the step the vector registers of three planes per barrier)
    const int n = __builtin_amdgcn_readfirstlane(ss->n);
    const int k = pos(n) % kGuessPeriod;
    const long long ng = J.S.g.ng, nxy = J.S.g.nxy;
    StepVar<float> V;
    V.epoch_base = ss->ep;
    V.out_iters = nullptr;                  // per-step outputs are written below
    V.out_relres = nullptr;
    V.out_status = nullptr;
    V.ckpt_out = nullptr;
    // the previous states h1..h3 (T^{n-1..n-3} forward, mu^{n+1..n+3} adjoint; null = zero)
    const float* h[3];
    if (fwd) {
      V.x = J.traj + (long long)(n - 1) * ng;
      for (int d = 1; d <= 3; ++d) h[d - 1] = n - d >= 1 ? J.traj + (long long)(n - d - 1) * ng : nullptr;
      V.top_src = J.S.top_src;
      V.top_scale = J.qscale[n - 1];
      V.surf_out = J.surf + (long long)(n - 1) * nxy;
      V.surf_scale = 1.f;
      V.T_grad = nullptr;
    } else {
      V.x = J.mu[n & 3];
      for (int d = 1; d <= 3; ++d) h[d - 1] = n + d <= J.nsteps ? J.mu[(n + d) & 3] : nullptr;
      V.top_src = J.gsurf + (long long)(n - 1) * nxy;
      V.top_scale = 1.f;
      V.surf_out = nullptr;
      V.surf_scale = 1.f;
      V.T_grad = J.traj + (long long)(n - 1) * ng;
    }
    // initial guess: probes of orders 0, 1, 2 open each period, then the
    // order whose probe needed the fewest iterations (ties: the higher)
    int order = 2;
    if (k < 3) {
      order = k;
    } else {
      const int p0 = __builtin_amdgcn_readfirstlane(ss->pc[0]), p1 = __builtin_amdgcn_readfirstlane(ss->pc[1]),
                p2 = __builtin_amdgcn_readfirstlane(ss->pc[2]);
      if (p0 >= 0 && p1 >= 0 && p2 >= 0) {
        int best = p2;
        if (p1 < best) { order = 1; best = p1; }
        if (p0 < best) order = 0;
      }
    }
    V.xprev = h[0];
    V.xprev2 = h[1];
    V.xprev3 = h[2];
    V.gmode = order;
    V.gi = nullptr;
    V.gp[0] = V.gp[1] = V.gp[2] = 0;
    const StepResult r = step(S, V);
    __syncthreads();                        // every thread has read the state of this step
    if (threadIdx.x == 0) {
      if (m.y == 0) {
        const int slot = (fwd ? 0 : J.nsteps) + n - 1;
        J.it_out[slot] = r.iters;
        J.rel_out[slot] = r.relres;
        J.st_out[slot] = r.status;
      }
      ss->ep = r.epoch_end;
      if (k == 0) ss->pc[0] = ss->pc[1] = ss->pc[2] = -1;
      if (k < 3) ss->pc[k] = r.iters;
      ss->iters += r.iters;
      ss->status |= r.status;
      ss->steps += 1;
      ss->n = n + (fwd ? 1 : -1);
    }
    __syncthreads();
    const bool last = fwd ? n == J.nsteps : n == 1;
    const long long iters = ss->iters;
    const int steps = ss->steps, status = ss->status;
    if (last || (status & (kNonFinite | kTimeout)) || steps >= kMaxSliceSteps) break;
    // the next step is expected to take about as many iterations as this one
    if ((iters + steps + r.iters + 1) * J.cost > J.budget) break;
  }
  if (m.y == 0 && threadIdx.x == 0) {
    JobProg p;
    p.steps = ss->steps;
    p.status = ss->status;
    p.iters = ss->iters;
    p.t0 = ss->t0;
    p.t1 = wall_clock64();
    prog[m.x] = p;
  }
}

// Workgroup b works as rank map[b].y of job map[b].x (streaming step kernel
// code: 1024-thread workgroups, tiles of 64 x 16 columns or narrower).
__global__ void __launch_bounds__(Cfg<float>::kBlock, 1) batch_run_kernel(const JobRun* jobs, const int2* map,
                                                                          JobProg* prog) {
  __shared__ Smem<float> sh;
  __shared__ SliceState ss;
  const int2 m = map[blockIdx.x];
  if (m.x < 0) return;
  // The job table is not written during the launch: reading it through the
  // constant address space makes its loads scalar and invariant.
  const CJobRun& J = *(const CJobRun*)(jobs + m.x);
  run_slice(J, m, prog, &ss, [&](const StepArgs<float>& S, const StepVar<float>& V) {
    return run_step<float>(S, V, m.y, sh);
  });
}

// The same with the register-resident step: 512-thread workgroups, one tile
// of 64 x 8 x (<= 32) cells each, the tile's CG state in registers.
__global__ void __launch_bounds__(kResBlock, 1) batch_resident_kernel(const JobRun* jobs, const int2* map,
                                                                       JobProg* prog) {
  extern __shared__ __align__(16) unsigned char dsm[];
  __shared__ SliceState ss;
  const int2 m = map[blockIdx.x];
  if (m.x < 0) return;
  const CJobRun& J = *(const CJobRun*)(jobs + m.x);
  run_slice(J, m, prog, &ss, [&](const StepArgs<float>& S, const StepVar<float>& V) {
    // three planes per barrier; the x-edge columns from the vectors (the
    // compact copies would spill the slice's state)
    return resident_step<64, 3>(S, V, m.y, dsm, true);
  });
}

constexpr int kMseThreads = 256;

// Mean squared error of the surface series: per-workgroup FP64 partial sums
// of (S - target)^2, and g = scale * (S - target) with scale = 2 / m.
__global__ void __launch_bounds__(kMseThreads) mse_grad_kernel(const float* S, const float* target, float* g,
                                                               long long m, double scale, double* partial) {
  double acc = 0.0;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < m; i += (long long)gridDim.x * blockDim.x) {
    const double d = (double)S[i] - (double)target[i];
    acc += d * d;
    g[i] = (float)(scale * d);
  }
  __shared__ double red[kMseThreads / 64];
  acc = wave_sum(acc);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) partial[blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
}

// loss = (sum of the partials in index order) / m
__global__ void mse_finish_kernel(const double* partial, int n, double inv_m, double* loss) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    double s = 0.0;
    for (int i = 0; i < n; ++i) s += partial[i];
    *loss = s * inv_m;
  }
}

}  // namespace nh

namespace {

constexpr int kMseBlocks = nhp::kMseBlocks;
constexpr long long kVoxelsPerBlock = nhp::kVoxelsPerBlock;
constexpr long long kReductionCost = 8192;   // a team reduction, in voxel units of work
constexpr long long kResCells = 16384;        // cells of a full resident tile
constexpr long long kResFixedCost = 24576;    // per resident iteration: reduction and face exchange
constexpr int kBlock = nh::Cfg<float>::kBlock;
static_assert(nhp::kBlock == kBlock && nhp::kResBlock == nh::kResBlock && nhp::kResTZ == nh::kResTZ &&
                  nhp::kSlotBytes == sizeof(nh::Slot) && sizeof(nh::TSlot) == sizeof(nh::Slot),
              "the host-side policy must size jobs as the kernels tile them");

double now_s() {
  static const auto t0 = std::chrono::steady_clock::now();
  return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
}

size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

// The kernels' tiling of a job from the host-side policy's.
void job_geom_of(int nx, int ny, int nz, const nhp::JobGeom& p, nh::Geom& g, int& team) {
  g = nh::Geom{};
  g.nx = nx; g.ny = ny; g.nz = nz;
  g.nxy = (long long)nx * ny;
  g.ng = g.nxy * nz;
  g.TX = p.TX; g.TY = p.TY; g.TZ = p.TZ; g.txs = p.txs;
  g.ntx = p.ntx; g.nty = p.nty; g.ntz = p.ntz; g.ntiles = p.ntiles;
  team = p.team;
}

struct SJob {
  long long id = 0;
  int state = NH_JOB_QUEUED;
  int nx = 0, ny = 0, nz = 0, nsteps = 0, max_iter = 0;
  double h = 1, dt = 1, rtol = 1e-6;
  std::vector<float> h_alpha, h_qxy, h_target, h_qscale;
  nh::Geom g{};
  int team = 1;
  long long cost = 0;
  size_t bytes = 0;
  void* mem = nullptr;
  float *alpha = nullptr, *qxy = nullptr, *target = nullptr, *traj = nullptr, *z = nullptr, *p0 = nullptr,
        *u1 = nullptr, *w0 = nullptr, *w1 = nullptr, *s0 = nullptr, *s1 = nullptr, *mu[4] = {},
        *surf = nullptr, *gsurf = nullptr, *qscale = nullptr;
  double *G = nullptr, *partial = nullptr, *lossbuf = nullptr, *rel_out = nullptr;
  void* slots = nullptr;
  int *it_out = nullptr, *st_out = nullptr;
  int step = 0;            // the next step to compute (the adjoint counts down from N)
  int steps_done = 0;      // forward and adjoint steps completed
  double busy_s = 0.0;     // measured time of its slices
  long long fwd_iters = 0, adj_iters = 0;
  int status = 0;
  double loss = 0;
  std::vector<double> h_G;
  double t_submit = 0, t_admit = 0, t_done = 0;
};

}  // namespace

struct nh_server {
  int device = 0;
  hipStream_t stream = nullptr;
  int num_cu = 0, max_blocks = 0;
  double budget = 0;
  int resident = 1;        // 1: nh::batch_resident_kernel, 0: nh::batch_run_kernel
  int slice_iters = 512;
  int backfill = 1;        // 1: EASY backfilling, 0: strict arrival order
  std::map<long long, std::pair<double, long long>> shape_time;   // grid -> (seconds, steps) measured
  // grid -> (seconds, iterations + steps) measured: the slice budget's cost of an iteration
  std::map<long long, std::pair<double, long long>> shape_iter;
  double unit_ns = 0.0, unit_cost = 0.0;   // measured ns against the cost model's units, summed
  size_t used_bytes = 0;
  int used_blocks = 0;
  long long next_id = 1;
  unsigned long long launch_ctr = 0;
  long long wallclock_khz = 100000;
  double barrier_timeout_s = 20.0;
  int trace = 0;          // NH_SERVE_TRACE=1: a line per launch; 2: also a line per job
  std::deque<SJob*> queue;
  std::vector<SJob*> active;
  std::map<long long, std::unique_ptr<SJob>> jobs;
  // pinned host staging and device copies of the launch tables
  nh::JobRun* h_runs = nullptr;
  nh::JobProg* h_prog = nullptr;
  int2* h_map = nullptr;
  nh::JobRun* d_runs = nullptr;
  nh::JobProg* d_prog = nullptr;
  int2* d_map = nullptr;
  size_t cap_jobs = 0;
  int* d_flag = nullptr;
  std::string err;
  nh_server_stats st{};
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
};

namespace {

nh_status sfail(nh_server* s, nh_status st, const std::string& m) {
  if (s) s->err = m;
  return st;
}

#define SV_HIP(s, call)                                                                                \
  do {                                                                                                 \
    hipError_t e_ = (call);                                                                            \
    if (e_ != hipSuccess) return sfail((s), NH_EHIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)

// Allocate and fill the job's device state; queues the copies on the stream.
nh_status admit(nh_server* s, SJob* j) {
  if (hipMalloc(&j->mem, j->bytes) != hipSuccess) {
    (void)hipGetLastError();
    j->mem = nullptr;
    return sfail(s, NH_ENOMEM, "hipMalloc for a job failed");
  }
  const size_t ng = (size_t)j->g.ng, nxy = (size_t)j->g.nxy, N = (size_t)j->nsteps;
  char* p = (char*)j->mem;
  auto take = [&](size_t b) {
    char* r = p;
    p += align256(b);
    return r;
  };
  j->alpha = (float*)take(4 * ng);
  j->z = (float*)take(4 * ng);
  j->p0 = (float*)take(4 * ng);
  j->u1 = (float*)take(4 * ng);
  j->w0 = (float*)take(4 * ng);
  j->w1 = (float*)take(4 * ng);
  j->s0 = (float*)take(4 * ng);
  j->s1 = (float*)take(4 * ng);
  for (float*& m : j->mu) m = (float*)take(4 * ng);
  j->traj = (float*)take(4 * ng * N);
  j->G = (double*)take(8 * ng);
  j->qxy = (float*)take(4 * nxy);
  j->target = (float*)take(4 * nxy * N);
  j->surf = (float*)take(4 * nxy * N);
  j->gsurf = (float*)take(4 * nxy * N);
  j->qscale = (float*)take(4 * N);
  j->it_out = (int*)take(4 * 2 * N);
  j->st_out = (int*)take(4 * 2 * N);
  j->rel_out = (double*)take(8 * 2 * N);
  j->slots = take(sizeof(nh::Slot) * (2 * (size_t)j->team + 2));
  j->partial = (double*)take(8 * kMseBlocks);
  j->lossbuf = (double*)take(256);
  if ((size_t)(p - (char*)j->mem) > j->bytes) return sfail(s, NH_EINVAL, "internal: job layout exceeds its size");
  SV_HIP(s, hipMemcpyAsync(j->alpha, j->h_alpha.data(), 4 * ng, hipMemcpyHostToDevice, s->stream));
  SV_HIP(s, hipMemcpyAsync(j->qxy, j->h_qxy.data(), 4 * nxy, hipMemcpyHostToDevice, s->stream));
  SV_HIP(s, hipMemcpyAsync(j->target, j->h_target.data(), 4 * nxy * N, hipMemcpyHostToDevice, s->stream));
  SV_HIP(s, hipMemcpyAsync(j->qscale, j->h_qscale.data(), 4 * N, hipMemcpyHostToDevice, s->stream));
  SV_HIP(s, hipMemsetAsync(j->slots, 0, sizeof(nh::Slot) * (2 * (size_t)j->team + 2), s->stream));
  const int blocks = (int)std::min<size_t>((ng + 255) / 256, 2048);
  hipLaunchKernelGGL(nh::fill_kernel<double>, dim3(blocks), dim3(256), 0, s->stream, j->G, (long long)ng, 0.0);
  SV_HIP(s, hipGetLastError());
  j->state = NH_JOB_FORWARD;
  j->step = 1;
  j->t_admit = now_s();
  s->used_bytes += j->bytes;
  s->used_blocks += j->team;
  return NH_OK;
}

void retire(nh_server* s, SJob* j) {
  if (j->mem) (void)hipFree(j->mem);
  j->mem = nullptr;
  s->used_bytes -= j->bytes;
  s->used_blocks -= j->team;
}

// Job j's slice of the next launch.
long long shape_key(const SJob* j) { return ((long long)j->nx << 42) | ((long long)j->ny << 21) | j->nz; }

// iterations (plus steps) a grid must have run before its measured time per
// iteration prices its slices
constexpr long long kShapeIterMin = 64;

void job_run(const nh_server* s, const SJob* j, unsigned long long epoch_base, nh::JobRun& J) {
  std::memset(&J, 0, sizeof(J));
  nh::StepArgs<float>& S = J.S;
  S.g = j->g;
  const float sd = (float)(2.0 * j->dt / (j->h * j->h));
  S.sx = S.sy = S.sz = sd;
  S.alpha = j->alpha;
  S.z = j->z;
  S.p0 = j->p0;
  S.u1 = j->u1;
  S.w0 = j->w0;
  S.w1 = j->w1;
  S.s0 = j->s0;
  S.s1 = j->s1;
  S.variant = 1;
  S.slots = j->slots;
  S.epoch_base = epoch_base;
  S.rtol2 = j->rtol * j->rtol;
  S.max_iter = j->max_iter;
  S.team = j->team;
  S.xcd_order = 0;
  S.err_flag = s->d_flag;
  S.timeout_ticks = (long long)(s->barrier_timeout_s * (double)s->wallclock_khz * 1000.0);
  if (j->state == NH_JOB_FORWARD) {
    S.mode = nh::kForward;
    S.top_src = j->qxy;
  } else {
    S.mode = nh::kAdjoint;
    S.top_scale = 1.f;
    S.G = j->G;
  }
  for (int k = 0; k < 4; ++k) J.mu[k] = j->mu[k];
  J.qscale = j->qscale;
  J.traj = j->traj;
  J.surf = j->surf;
  J.gsurf = j->gsurf;
  J.it_out = j->it_out;
  J.rel_out = j->rel_out;
  J.st_out = j->st_out;
  J.mode = S.mode;
  J.n0 = j->step;
  J.nsteps = j->nsteps;
  // The slice ends once the job's iterations (and steps, each priced as one
  // iteration) times its cost would pass the budget. Until anything has been
  // measured, cost and budget are in the cost model's units (the cells of a
  // workgroup's tile plus a fixed part per reduction); afterwards in
  // nanoseconds: the budget is the model's budget at the measured ns per model
  // unit, and a job's cost its grid's measured time per iteration, so that
  // every team's slice takes about the same time and few wait for the slowest.
  const long long model_budget =
      (long long)s->slice_iters * (s->resident ? kResCells + kResFixedCost : kVoxelsPerBlock + kReductionCost);
  if (s->unit_cost > 0.0) {
    const double ns_per_unit = s->unit_ns / s->unit_cost;
    J.budget = std::llround((double)model_budget * ns_per_unit);
    auto it = s->shape_iter.find(shape_key(j));
    const double ns = it != s->shape_iter.end() && it->second.second >= kShapeIterMin
                          ? 1e9 * it->second.first / (double)it->second.second
                          : (double)j->cost * ns_per_unit;
    J.cost = std::max<long long>(1, std::llround(ns));
  } else {
    J.cost = j->cost;
    J.budget = model_budget;
  }
}


// Estimated seconds per step of job j: its own measured mean once it has run
// a few steps, else the mean of its grid shape, else of all measured jobs.
double step_estimate(const nh_server* s, const SJob* j) {
  if (j->steps_done >= 4) return j->busy_s / j->steps_done;
  auto it = s->shape_time.find(shape_key(j));
  if (it != s->shape_time.end() && it->second.second > 0) return it->second.first / it->second.second;
  double t = 0.0;
  long long n = 0;
  for (const auto& kv : s->shape_time) {
    t += kv.second.first;
    n += kv.second.second;
  }
  return n > 0 ? t / n : 1e-3;
}

double remaining_steps(const SJob* j) { return (double)std::max(0, 2 * j->nsteps - j->steps_done); }

nh_status ensure_tables(nh_server* s, size_t njobs) {
  if (s->cap_jobs >= njobs) return NH_OK;
  const size_t cap = std::max<size_t>(64, 2 * njobs);
  if (s->h_runs) (void)hipHostFree(s->h_runs);
  if (s->h_prog) (void)hipHostFree(s->h_prog);
  if (s->d_runs) (void)hipFree(s->d_runs);
  if (s->d_prog) (void)hipFree(s->d_prog);
  s->h_runs = nullptr; s->h_prog = nullptr; s->d_runs = nullptr; s->d_prog = nullptr;
  s->cap_jobs = 0;
  SV_HIP(s, hipHostMalloc((void**)&s->h_runs, sizeof(nh::JobRun) * cap, hipHostMallocDefault));
  SV_HIP(s, hipHostMalloc((void**)&s->h_prog, sizeof(nh::JobProg) * cap, hipHostMallocDefault));
  SV_HIP(s, hipMalloc(&s->d_runs, sizeof(nh::JobRun) * cap));
  SV_HIP(s, hipMalloc(&s->d_prog, sizeof(nh::JobProg) * cap));
  s->cap_jobs = cap;
  return NH_OK;
}

}  // namespace

extern "C" {

nh_status nh_server_create(nh_server** out, int hip_device, void* hip_stream, double hbm_budget_bytes,
                           int max_blocks, int resident) {
  if (!out) return NH_EINVAL;
  *out = nullptr;
  if (!(hbm_budget_bytes > 0) || max_blocks < 0 || resident < 0 || resident > 1) return NH_EINVAL;
  now_s();
  std::unique_ptr<nh_server> s(new (std::nothrow) nh_server());
  if (!s) return NH_ENOMEM;
  if (hipSetDevice(hip_device) != hipSuccess) return NH_EINVAL;
  s->device = hip_device;
  s->stream = (hipStream_t)hip_stream;
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, hip_device) != hipSuccess) return NH_EHIP;
  s->num_cu = prop.multiProcessorCount;
  s->resident = resident;
  int occ = 0;
  if (resident) {
    if (hipFuncSetAttribute((const void*)nh::batch_resident_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)nh::kResLdsBytes) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, (const void*)nh::batch_resident_kernel, nh::kResBlock,
                                                     nh::kResLdsBytes) != hipSuccess ||
        occ < 1)
      return NH_EHIP;
  } else if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, (const void*)nh::batch_run_kernel, kBlock, 0) !=
                 hipSuccess ||
             occ < 1) {
    return NH_EHIP;
  }
  s->max_blocks = occ * s->num_cu;
  if (max_blocks > 0) s->max_blocks = std::min(s->max_blocks, max_blocks);
  s->budget = hbm_budget_bytes;
  int khz = 0;
  if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, hip_device) == hipSuccess && khz > 0)
    s->wallclock_khz = khz;
  bool ok = hipMalloc(&s->d_flag, 64) == hipSuccess && hipMemset(s->d_flag, 0, 64) == hipSuccess &&
            hipMalloc(&s->d_map, sizeof(int2) * s->max_blocks) == hipSuccess &&
            hipHostMalloc((void**)&s->h_map, sizeof(int2) * s->max_blocks, hipHostMallocDefault) == hipSuccess &&
            hipEventCreate(&s->ev0) == hipSuccess && hipEventCreate(&s->ev1) == hipSuccess;
  s->st.max_blocks = s->max_blocks;
  if (const char* t = std::getenv("NH_SERVE_TRACE")) s->trace = std::atoi(t);
  nh_server* raw = s.release();
  if (!ok || ensure_tables(raw, 64) != NH_OK) {
    nh_server_destroy(raw);
    return NH_EHIP;
  }
  *out = raw;
  return NH_OK;
}

nh_status nh_server_set_slice(nh_server* s, int iters) {
  if (!s) return NH_EINVAL;
  if (iters < 1) return sfail(s, NH_EINVAL, "slice must be >= 1 iteration");
  s->slice_iters = iters;
  return NH_OK;
}

nh_status nh_server_set_backfill(nh_server* s, int mode) {
  if (!s) return NH_EINVAL;
  if (mode < 0 || mode > 1) return sfail(s, NH_EINVAL, "backfill mode must be 0 or 1");
  s->backfill = mode;
  return NH_OK;
}

nh_status nh_server_submit(nh_server* s, int nx, int ny, int nz, double h, double dt, int nsteps, double rtol,
                           int max_iter, const float* alpha, const float* q_xy, const double* q_t,
                           const float* target, long long* job_id) {
  if (!s) return NH_EINVAL;
  if (!job_id || !alpha || !q_xy || !q_t || !target) return sfail(s, NH_EINVAL, "null pointer argument");
  if (!nhp::job_params_ok(nx, ny, nz, h, dt, nsteps, rtol, max_iter)) return sfail(s, NH_EINVAL, "bad job parameters");
  const size_t ng = (size_t)nx * ny * nz, nxy = (size_t)nx * ny, N = (size_t)nsteps;
  if (nhp::first_bad(alpha, ng, true) >= 0) return sfail(s, NH_EINVAL, "alpha must be finite and > 0");
  if (nhp::first_bad(q_xy, nxy, false) >= 0) return sfail(s, NH_EINVAL, "q_xy holds a non-finite value");
  if (nhp::first_bad(q_t, N, false) >= 0) return sfail(s, NH_EINVAL, "q_t holds a non-finite value");
  if (nhp::first_bad(target, nxy * N, false) >= 0) return sfail(s, NH_EINVAL, "target holds a non-finite value");
  auto j = std::make_unique<SJob>();
  j->nx = nx; j->ny = ny; j->nz = nz;
  j->h = h;
  j->dt = dt;
  j->nsteps = nsteps;
  j->rtol = rtol;
  j->max_iter = max_iter;
  int team = 0;
  if (s->resident) {
    job_geom_of(nx, ny, nz, nhp::job_geom_res(nx, ny, nz), j->g, team);
    if (team > s->max_blocks) return sfail(s, NH_EINVAL, "job needs more tiles than fit on the device");
    j->cost = ((long long)ng + team - 1) / team + kResFixedCost;
  } else {
    job_geom_of(nx, ny, nz, nhp::job_geom(nx, ny, nz, std::max(1, s->max_blocks / 2)), j->g, team);
    j->cost = ((long long)ng + team - 1) / team + (team > 1 ? kReductionCost : 0);
  }
  j->team = team;
  j->bytes = nhp::job_bytes(nx, ny, nz, nsteps, team);
  if ((double)j->bytes > s->budget) return sfail(s, NH_ENOMEM, "job larger than the HBM budget");
  j->h_alpha.assign(alpha, alpha + ng);
  j->h_qxy.assign(q_xy, q_xy + nxy);
  j->h_target.assign(target, target + nxy * N);
  j->h_qscale.resize(N);
  for (size_t n = 0; n < N; ++n) j->h_qscale[n] = (float)(dt * q_t[n]);   // as the single-problem path
  j->id = s->next_id++;
  j->t_submit = now_s();
  *job_id = j->id;
  s->queue.push_back(j.get());
  s->jobs[j->id] = std::move(j);
  return NH_OK;
}

nh_status nh_server_tick(nh_server* s, int* n_active, int* n_queued, long long* finished_ids, int finished_cap,
                         int* n_finished) {
  if (!s) return NH_EINVAL;
  struct TickRange {   // a host-side roctx range per tick, shown by marker tracing
    TickRange() { roctxRangePushA("nh_server_tick"); }
    ~TickRange() { roctxRangePop(); }
  } const tick_range;
  if (finished_cap > 0 && !finished_ids) return sfail(s, NH_EINVAL, "finished_ids is null");
  if (hipSetDevice(s->device) != hipSuccess) return sfail(s, NH_EHIP, "hipSetDevice failed");
  int finished = 0;

  // admission: arrival order, with EASY backfilling (the first job that does
  // not fit holds a reservation; later jobs start only if they do not delay
  // it, judged by run-time estimates from the measured step times)
  {
    std::vector<size_t> qb, ab;
    std::vector<int> qt, at, sel(s->queue.size());
    std::vector<double> qd, ar;
    for (const SJob* j : s->queue) {
      qb.push_back(j->bytes);
      qt.push_back(j->team);
      qd.push_back(2.0 * j->nsteps * step_estimate(s, j));
    }
    for (const SJob* j : s->active) {
      ab.push_back(j->bytes);
      at.push_back(j->team);
      ar.push_back(remaining_steps(j) * step_estimate(s, j));
    }
    const int na = nh_serve_admit_select(qb.data(), qt.data(), qd.data(), (int)qb.size(), ab.data(), at.data(),
                                         ar.data(), (int)ab.size(), s->budget, s->max_blocks, s->backfill, sel.data());
    std::vector<SJob*> admitted;
    nh_status st = NH_OK;
    for (int k = 0; k < na && st == NH_OK; ++k) {
      SJob* j = s->queue[sel[k]];
      st = admit(s, j);
      if (st != NH_OK) break;
      admitted.push_back(j);
      s->active.push_back(j);
    }
    std::deque<SJob*> rest;
    for (SJob* j : s->queue)
      if (j->state == NH_JOB_QUEUED) rest.push_back(j);
    s->queue.swap(rest);
    if (st != NH_OK) return st;
    if (na > 0) {
      // the host copies of the inputs may go once the uploads are done
      SV_HIP(s, hipStreamSynchronize(s->stream));
      for (SJob* j : admitted) {
        std::vector<float>().swap(j->h_alpha);
        std::vector<float>().swap(j->h_target);
        std::vector<float>().swap(j->h_qscale);
      }
    }
  }

  if (!s->active.empty()) {
    const size_t na = s->active.size();
    nh_status ts = ensure_tables(s, na);
    if (ts != NH_OK) return ts;
    const unsigned long long base = (++s->launch_ctr) << 24;
    if (s->resident && (s->launch_ctr & 0xFF) == 0) {
      // the tagged reduction words repeat their tags every 256 launches:
      // zero every admitted job's slots before a new round starts
      for (size_t k = 0; k < na; ++k) {
        const SJob* j = s->active[k];
        SV_HIP(s, hipMemsetAsync(j->slots, 0, sizeof(nh::TSlot) * (2 * (size_t)j->team + 2), s->stream));
      }
    }
    int nb = 0;
    for (size_t k = 0; k < na; ++k) {
      const SJob* j = s->active[k];
      if (nb + j->team > s->max_blocks) return sfail(s, NH_EINVAL, "internal: workgroups exceed the limit");
      job_run(s, j, base, s->h_runs[k]);
      for (int r = 0; r < j->team; ++r) s->h_map[nb++] = make_int2((int)k, r);
    }
    SV_HIP(s, hipMemcpyAsync(s->d_runs, s->h_runs, sizeof(nh::JobRun) * na, hipMemcpyHostToDevice, s->stream));
    SV_HIP(s, hipMemcpyAsync(s->d_map, s->h_map, sizeof(int2) * nb, hipMemcpyHostToDevice, s->stream));
    void* args[] = {(void*)&s->d_runs, (void*)&s->d_map, (void*)&s->d_prog};
    SV_HIP(s, hipEventRecord(s->ev0, s->stream));
    if (s->resident)
      SV_HIP(s, hipLaunchCooperativeKernel((const void*)nh::batch_resident_kernel, dim3((unsigned)nb),
                                           dim3(nh::kResBlock), args, (unsigned)nh::kResLdsBytes, s->stream));
    else
      SV_HIP(s, hipLaunchCooperativeKernel((const void*)nh::batch_run_kernel, dim3((unsigned)nb), dim3(kBlock),
                                           args, 0, s->stream));
    SV_HIP(s, hipEventRecord(s->ev1, s->stream));
    SV_HIP(s, hipMemcpyAsync(s->h_prog, s->d_prog, sizeof(nh::JobProg) * na, hipMemcpyDeviceToHost, s->stream));
    SV_HIP(s, hipStreamSynchronize(s->stream));
    float ms = 0.f;
    SV_HIP(s, hipEventElapsedTime(&ms, s->ev0, s->ev1));
    s->st.kernel_s += 1e-3 * ms;
    ++s->st.ticks;

    // busy time of each team against the launch's span (load balance)
    {
      long long lo = s->h_prog[0].t0, hi = s->h_prog[0].t1;
      double busy = 0.0;
      for (size_t k = 0; k < na; ++k) {
        lo = std::min(lo, s->h_prog[k].t0);
        hi = std::max(hi, s->h_prog[k].t1);
        busy += (double)s->active[k]->team * (double)(s->h_prog[k].t1 - s->h_prog[k].t0);
      }
      const double tick_s = 1.0 / ((double)s->wallclock_khz * 1000.0);
      s->st.busy_block_s += busy * tick_s;
      s->st.span_block_s += (double)s->max_blocks * (double)(hi - lo) * tick_s;
      if (s->trace > 1)
        for (size_t k = 0; k < na; ++k) {
          const SJob* j = s->active[k];
          const nh::JobProg& q = s->h_prog[k];
          std::fprintf(stderr, "[nh_server]   job %lld %dx%dx%d team %d %s steps %d iters %lld busy %.3f ms\n", j->id,
                       j->nx, j->ny, j->nz, j->team, j->state == NH_JOB_FORWARD ? "fwd" : "adj", q.steps, q.iters,
                       (double)(q.t1 - q.t0) * tick_s * 1e3);
        }
      if (s->trace)
        std::fprintf(stderr, "[nh_server] tick %lld: %zu jobs, %d workgroups, launch %.3f ms, span %.3f ms, busy %.1f%%\n",
                     s->st.ticks, na, nb, (double)ms, (double)(hi - lo) * tick_s * 1e3,
                     100.0 * busy / ((double)s->max_blocks * (double)std::max(1LL, hi - lo)));
    }
    std::vector<SJob*> still;
    still.reserve(na);
    for (size_t k = 0; k < na; ++k) {
      SJob* j = s->active[k];
      const nh::JobProg pr = s->h_prog[k];
      j->status |= pr.status;
      {
        const double sec = (double)(pr.t1 - pr.t0) / ((double)s->wallclock_khz * 1000.0);
        j->busy_s += sec;
        j->steps_done += pr.steps;
        auto& st = s->shape_time[shape_key(j)];
        st.first += sec;
        st.second += pr.steps;
        const long long work = pr.iters + pr.steps;
        if (work > 0) {
          auto& si = s->shape_iter[shape_key(j)];
          si.first += sec;
          si.second += work;
          s->unit_ns += 1e9 * sec;
          s->unit_cost += (double)work * (double)j->cost;
        }
      }
      const bool failed = (pr.status & (nh::kNonFinite | nh::kTimeout)) != 0;
      if (j->state == NH_JOB_FORWARD) {
        j->fwd_iters += pr.iters;
        j->step += pr.steps;
        if (j->step > j->nsteps && !failed) {
          // forward done: loss and dL/dS of the mean squared error, ahead of
          // the next launch on the same stream; the adjoint starts at step N
          const long long m = j->g.nxy * (long long)j->nsteps;
          hipLaunchKernelGGL(nh::mse_grad_kernel, dim3(kMseBlocks), dim3(nh::kMseThreads), 0, s->stream, j->surf,
                             j->target, j->gsurf, m, 2.0 / (double)m, j->partial);
          hipLaunchKernelGGL(nh::mse_finish_kernel, dim3(1), dim3(64), 0, s->stream, j->partial, kMseBlocks,
                             1.0 / (double)m, j->lossbuf);
          SV_HIP(s, hipGetLastError());
          j->state = NH_JOB_ADJOINT;
          j->step = j->nsteps;
        }
        if (!failed) {
          still.push_back(j);
          continue;
        }
      } else {
        j->adj_iters += pr.iters;
        j->step -= pr.steps;
        if (j->step >= 1 && !failed) {
          still.push_back(j);
          continue;
        }
      }
      // finished (or failed): results to the host, memory back to the pool
      const size_t ng = (size_t)j->g.ng;
      if (!failed) {
        j->h_G.resize(ng);
        SV_HIP(s, hipMemcpyAsync(j->h_G.data(), j->G, 8 * ng, hipMemcpyDeviceToHost, s->stream));
        SV_HIP(s, hipMemcpyAsync(&j->loss, j->lossbuf, sizeof(double), hipMemcpyDeviceToHost, s->stream));
      }
      SV_HIP(s, hipStreamSynchronize(s->stream));
      j->state = failed ? NH_JOB_FAILED : NH_JOB_DONE;
      j->t_done = now_s();
      retire(s, j);
      if (!failed) {
        s->st.jobs_done += 1;
        s->st.voxel_steps += 2.0 * (double)ng * j->nsteps;
        s->st.cg_iters += j->fwd_iters + j->adj_iters;
      }
      if (finished < finished_cap) finished_ids[finished] = j->id;
      ++finished;
    }
    s->active.swap(still);
  }
  if (n_active) *n_active = (int)s->active.size();
  if (n_queued) *n_queued = (int)s->queue.size();
  if (n_finished) *n_finished = finished;
  return NH_OK;
}

nh_status nh_server_job(nh_server* s, long long job_id, nh_job_info* info, double* dL_dalpha) {
  if (!s) return NH_EINVAL;
  if (!info) return sfail(s, NH_EINVAL, "info is null");
  auto it = s->jobs.find(job_id);
  if (it == s->jobs.end()) return sfail(s, NH_EINVAL, "unknown job id");
  const SJob* j = it->second.get();
  std::memset(info, 0, sizeof(*info));
  info->state = j->state;
  info->status = j->status;
  info->team_blocks = j->team;
  info->nsteps = j->nsteps;
  info->fwd_iters = j->fwd_iters;
  info->adj_iters = j->adj_iters;
  info->loss = j->loss;
  info->t_submit_s = j->t_submit;
  info->t_admit_s = j->t_admit;
  info->t_done_s = j->t_done;
  info->device_bytes = j->bytes;
  if (dL_dalpha && !j->h_G.empty()) std::memcpy(dL_dalpha, j->h_G.data(), sizeof(double) * j->h_G.size());
  return NH_OK;
}

nh_status nh_server_release(nh_server* s, long long job_id) {
  if (!s) return NH_EINVAL;
  auto it = s->jobs.find(job_id);
  if (it == s->jobs.end()) return sfail(s, NH_EINVAL, "unknown job id");
  if (it->second->state != NH_JOB_DONE && it->second->state != NH_JOB_FAILED)
    return sfail(s, NH_ESTATE, "job has not finished");
  s->jobs.erase(it);
  return NH_OK;
}

nh_status nh_server_get_stats(const nh_server* s, nh_server_stats* out) {
  if (!s || !out) return NH_EINVAL;
  *out = s->st;
  out->used_bytes = s->used_bytes;
  out->used_blocks = s->used_blocks;
  out->max_blocks = s->max_blocks;
  out->active = (int)s->active.size();
  out->queued = (int)s->queue.size();
  return NH_OK;
}

const char* nh_server_last_error(const nh_server* s) { return s ? s->err.c_str() : "null server"; }

void nh_server_destroy(nh_server* s) {
  if (!s) return;
  (void)hipSetDevice(s->device);
  (void)hipStreamSynchronize(s->stream);
  for (SJob* j : s->active) retire(s, j);
  if (s->h_runs) (void)hipHostFree(s->h_runs);
  if (s->h_prog) (void)hipHostFree(s->h_prog);
  if (s->h_map) (void)hipHostFree(s->h_map);
  if (s->d_runs) (void)hipFree(s->d_runs);
  if (s->d_prog) (void)hipFree(s->d_prog);
  if (s->d_map) (void)hipFree(s->d_map);
  if (s->d_flag) (void)hipFree(s->d_flag);
  if (s->ev0) (void)hipEventDestroy(s->ev0);
  if (s->ev1) (void)hipEventDestroy(s->ev1);
  delete s;
}

}  // extern "C"
