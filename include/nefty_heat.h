/*
 * nefty_heat.h -- C ABI of the MI355X (gfx950) differentiable implicit-Euler
 * heat solver and its discrete adjoint.
 *
 * The operation (the paper's Sec. 4.2 "Hard-constrained differentiable
 * physics", Sec. 4.3 "Adjoint optimization" and App. D.2-D.3), written with
 * the positive operator L+ = -L so that A = I + dt*L+ (the paper's
 * A = I - dt*L):
 *
 *   c_f    = 2 a_p a_q / (a_p + a_q) / h_d^2        harmonic-mean face conductance (Prop. 1)
 *   (A x)_p = x_p + dt * sum_{interior faces f=(p,q)} c_f (x_p - x_q)  [+ dt beta x_p on k = nz-1]
 *            every boundary face is zero-flux (carries no term) unless
 *            nh_set_boundary makes the lateral faces periodic or gives the
 *            back face a Robin sink beta
 *   A T^n   = T^{n-1} + dt q^n,   T^0 = 0,   q^n = q_t[n-1] * q_xy on the top plane k = 0
 *   S^n     = T^n on k = 0                         (the observation projector of eq. nefty_obj)
 *   A mu^n  = mu^{n+1} + Pi^T dL/dS^n,  mu^{N+1} = 0   (eq. adjoint_eq)
 *   dL/da_p = -dt sum_n sum_{f ni p} 2 a_q^2/(a_p+a_q)^2/h_d^2 (T^n_p-T^n_q)(mu^n_p-mu^n_q)
 *                                                   (eq. grad_assembly, App. D.3)
 *
 * Every linear solve is a Jacobi-preconditioned conjugate gradient run to
 * ||r||_2 <= rtol * ||b||_2, warm-started from the previous state (forward)
 * or from mu^{n+1} (adjoint), as App. D.2 warm-starts its Jacobi sweeps;
 * nh_set_jacobi_sweeps selects those fixed-K sweeps instead.
 *
 * Layout: every volume is [nz][ny][nx], C-contiguous, x fastest, index
 * i + nx*(j + ny*k); k = 0 is the heated and observed top face. Surface
 * series are [nsteps][ny][nx], frame n-1 holding step n = 1..nsteps.
 *
 * Pointers are DEVICE pointers unless marked HOST. The caller owns every
 * buffer it passes; the context owns its workspaces, the saved forward
 * trajectory (or checkpoints) and copies of its inputs. One context is one
 * problem on one HIP stream and is not thread-safe. Each call returns after
 * its work has completed on that stream. Nothing throws across the ABI:
 * every call returns an nh_status and nh_last_error() describes the last
 * failure.
 *
 * Precision: the *_f32 entry points (nh_forward, nh_adjoint) keep the
 * stencil and vectors in FP32 and do every dot product, residual norm and
 * the gradient accumulation in FP64; the *_f64 entry points run the same
 * kernels in FP64 throughout.
 */
#ifndef NEFTY_HEAT_H
#define NEFTY_HEAT_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct nh_ctx nh_ctx;

typedef enum {
    NH_OK = 0,
    NH_EINVAL = -1,     /* bad argument: dims, spacing, dt <= 0, nsteps <= 0, alpha <= 0, null pointer */
    NH_ENOMEM = -2,     /* a device allocation failed */
    NH_ESTATE = -3,     /* adjoint without a matching forward, grid not set, precision mismatch */
    NH_ENOCONV = -4,    /* some solve reached max_iter; outputs are still written */
    NH_ENONFINITE = -5, /* alpha or a reduction was NaN/Inf */
    NH_EHIP = -6,       /* a HIP runtime call failed */
    NH_ETIMEOUT = -7    /* a device-side team barrier exceeded its time limit */
} nh_status;

/* Host-side statistics of the last forward and adjoint calls. */
typedef struct {
    long long fwd_iters;        /* CG iterations summed over the forward steps */
    long long adj_iters;        /* CG iterations summed over the adjoint steps */
    long long recompute_iters;  /* CG iterations of forward steps recomputed from checkpoints */
    int fwd_steps, adj_steps, recompute_steps;
    int max_step_iters;         /* largest per-step iteration count of the last forward/adjoint */
    double worst_rel_res;       /* largest final ||r||/||b|| over those solves */
    double bytes_alg_fwd;       /* algorithmic bytes of the last forward: 12R per voxel and CG iteration, 6R
                                   per voxel and step (textbook two-pass Jacobi-PCG, vectors in HBM) */
    double bytes_alg_adj;       /* same for the last adjoint, with 9R + 16 per voxel and step: the set-up and
                                   state store (6R) plus the gradient pass, which reads T^n, mu^n and alpha
                                   (3R) and the FP64 accumulator (16) (recomputed forward steps counted as
                                   forward).
                                   With fixed-K Jacobi sweeps: 4R per voxel and sweep, plus 3R + 16 per
                                   voxel and adjoint step for the gradient. A degree-m Chebyshev
                                   preconditioner adds 5R (m - 1) per voxel and CG iteration */
    double t_fwd_s, t_adj_s;    /* host wall time of the last forward / adjoint call */
    double t_kernel_fwd_s;      /* summed HIP-event durations of the forward step kernels
                                   (only when profiling is enabled, else 0) */
    double t_kernel_adj_s;      /* same for the adjoint (recomputation included) */
    long long launches_fwd, launches_adj; /* step-kernel launches */
    size_t workspace_bytes;     /* device bytes the context holds now */
    size_t peak_workspace_bytes;/* high-water mark of workspace_bytes */
    int team_blocks;            /* workgroups cooperating on one step */
    int block_threads;          /* threads per workgroup */
    int tile_x, tile_y, tile_z; /* tile extents of the stencil kernels */
    int resident;               /* 1: the register-resident step kernel runs this grid */
    int resident_occupancy;     /* workgroups of that kernel that fit one CU (0: unusable) */
    int jacobi_blocked;         /* 1: fixed-K steps run on the temporally blocked kernel */
} nh_stats;

/* Create a context on HIP device `hip_device`. All work of the context is
 * issued on `hip_stream` (a hipStream_t of that device, borrowed: it must
 * outlive the context); NULL means the device's null stream. Work the
 * caller queued earlier on the same stream is ordered before the context's
 * work. */
nh_status nh_create(nh_ctx **out, int hip_device, void *hip_stream);

/* Set the grid: nx, ny, nz >= 1 cells, spacings hx, hy, hz > 0. Frees the
 * saved forward state; workspaces are (re)allocated lazily by the next
 * forward. */
nh_status nh_set_grid(nh_ctx *ctx, int nx, int ny, int nz, double hx, double hy, double hz);

/* Solver settings: 0 < rtol < 1, max_iter >= 1, checkpoint_every >= 0
 * (0 keeps every state T^1..T^N for the adjoint; k > 0 keeps T^k, T^2k, ...
 * and recomputes each segment during the adjoint). Defaults: 1e-6, 1000, 0.
 * Frees the saved forward state. */
nh_status nh_set_solver(nh_ctx *ctx, double rtol, int max_iter, int checkpoint_every);

/* Boundary closure (App. D.2, boundary conditions and the Robin row sums).
 * periodic_xy = 1 closes the x and y rows into rings, as the paper's circular
 * padding does: cell 0 and cell n-1 of a row share a face with the harmonic-
 * mean conductance (needs nx, ny >= 3, else NH_EINVAL). robin_h >= 0 is the
 * coefficient h of the back-face condition n.(alpha grad T) = -h T on the
 * plane k = nz-1: its rows carry the diagonal sink beta = h / hz, which does
 * not depend on alpha. Default 0, 0: zero flux on all six faces. The plane
 * k = 0 stays adiabatic. Grids with either closure run on the streaming step
 * kernel. Frees the saved forward state. */
nh_status nh_set_boundary(nh_ctx *ctx, int periodic_xy, double robin_h);

/* Inner solver. k = 0 (default): Jacobi-preconditioned CG to rtol. k > 0:
 * the paper's fixed-K solver (eq. jacobi_iter, App. D.2): every solve takes
 * exactly k sweeps x <- D^-1 (b - R x), A = D + R, from the previous time
 * level's state (T^{n-1} forward, mu^{n+1} adjoint); the initial-guess mode
 * does not apply. nh_stats reports k iterations per step, and worst_rel_res
 * the largest ||b - A x|| / ||b|| of a last sweep's input. rtol is ignored
 * and NH_ENOCONV never returned. k <= 100000, else NH_EINVAL. Frees the
 * saved forward state. */
nh_status nh_set_jacobi_sweeps(nh_ctx *ctx, int k);

/* Forward sweep, FP32 vectors with FP64 reductions.
 *   alpha  [nz][ny][nx] diffusivity, every value finite and > 0 (checked on
 *          the device: NH_EINVAL otherwise); copied into the context, so the
 *          caller may change or free it after the call.
 *   q_xy   [ny][nx] top-face source map (finite).
 *   q_t    HOST [nsteps] source amplitude per step: q^n = q_t[n-1] * q_xy.
 *   dt > 0, nsteps >= 1.
 *   T_surf [nsteps][ny][nx] output: T^n on k = 0 for n = 1..nsteps.
 * Saves what the adjoint needs (all states, or checkpoints). Returns
 * NH_ENOCONV if a step hit max_iter (outputs still written). */
nh_status nh_forward(nh_ctx *ctx, const float *alpha, const float *q_xy, const double *q_t,
                     double dt, int nsteps, float *T_surf);

/* Adjoint sweep of the last nh_forward (vector-Jacobian product).
 *   dL_dTsurf [nsteps][ny][nx] derivative of the caller's loss w.r.t. T_surf.
 *   dL_dalpha [nz][ny][nx] FP64 output, overwritten.
 * May be called several times per forward. NH_ESTATE if no FP32 forward is
 * saved. */
nh_status nh_adjoint(nh_ctx *ctx, const float *dL_dTsurf, double *dL_dalpha);

/* The same two calls with FP64 vectors throughout. */
nh_status nh_forward_f64(nh_ctx *ctx, const double *alpha, const double *q_xy, const double *q_t,
                         double dt, int nsteps, double *T_surf);
nh_status nh_adjoint_f64(nh_ctx *ctx, const double *dL_dTsurf, double *dL_dalpha);

/* The adjoint sweep with the other two vector-Jacobian products it yields
 * (App. D.3): besides dL/dalpha, dL_dq[nsteps][ny][nx] receives
 * dL/dq^n = dt * mu^n on the top plane k = 0 (the sensitivity to the source
 * of step n; chain it through q^n = q_t[n-1] * q_xy for q_xy and q_t) and
 * dL_dT0[nz][ny][nx] receives mu^1 = dL/dT^0 (the sensitivity to the initial
 * state). Either may be NULL. Same precision rules and errors as nh_adjoint /
 * nh_adjoint_f64. */
nh_status nh_adjoint_vjp(nh_ctx *ctx, const float *dL_dTsurf, double *dL_dalpha, float *dL_dq, float *dL_dT0);
nh_status nh_adjoint_vjp_f64(nh_ctx *ctx, const double *dL_dTsurf, double *dL_dalpha, double *dL_dq,
                             double *dL_dT0);

/* The adjoint sweep with the gradients of the separable source
 * q^n = q_t[n-1] * q_xy of the last forward (App. D.3, dL/dq^n = dt * mu^n on
 * the top plane, chained through the product):
 *   dL_dqxy [ny][nx] FP64 device: sum_n q_t[n-1] * dL/dq^n (n ascending);
 *   dL_dqt  [nsteps] FP64 device: entry n-1 = sum_ij dL/dq^n_ij * q_xy_ij
 *           (fixed summation order, bit-reproducible).
 * dL/dq^n is rounded to the forward's precision before the sums. Either
 * output may be NULL; dL_dalpha as in nh_adjoint. Same precision rules and
 * errors as nh_adjoint / nh_adjoint_f64 (NH_ENOCONV still writes every
 * output). The context keeps an nsteps x ny x nx workspace for the series. */
nh_status nh_adjoint_source_grad(nh_ctx *ctx, const float *dL_dTsurf, double *dL_dalpha, double *dL_dqxy,
                                 double *dL_dqt);
nh_status nh_adjoint_source_grad_f64(nh_ctx *ctx, const double *dL_dTsurf, double *dL_dalpha,
                                     double *dL_dqxy, double *dL_dqt);

/* Copy the saved state T^n (1 <= n <= nsteps, full storage; or a checkpoint
 * step when checkpointing) of the last forward into `out` ([nz][ny][nx],
 * device, the forward's precision). NH_ESTATE if that state is not held. */
nh_status nh_get_state(nh_ctx *ctx, int n, void *out);

/* y = A x for the operator of Sec. 4.2 with diffusivity alpha and step dt
 * on the current grid (the stencil kernel on its own; for operator tests).
 * alpha, x, y: [nz][ny][nx] FP32 device arrays (y must not alias x). */
nh_status nh_apply_A(nh_ctx *ctx, const float *alpha, const float *x, float *y, double dt);

/* The total-variation regulariser of the inverse problem (eq. tv_discrete,
 * App. D.1) on the context's grid and spacings, value and gradient in one
 * pass:
 *   R(a) = hx hy hz sum_p sqrt((d_x a/hx)^2 + (d_y a/hy)^2 + (d_z a/hz)^2 + eps^2)
 * with forward differences along the array axes; the x and y differences
 * wrap around (the paper's lateral periodicity, whatever nh_set_boundary
 * says) and the z difference is 0 on the plane k = nz-1.
 *   alpha  [nz][ny][nx] device, FP32 (nh_tv) or FP64 (nh_tv_f64); any values.
 *   value  device pointer to one double: receives weight * R(alpha).
 *   grad   [nz][ny][nx] FP64 device: receives weight * dR/dalpha, added to
 *          its contents when accumulate = 1 (e.g. onto the adjoint's
 *          dL/dalpha), written over them when accumulate = 0.
 *   eps > 0 and weight finite, else NH_EINVAL; NH_ESTATE before nh_set_grid.
 * The value is summed in a fixed order (bit-reproducible). */
nh_status nh_tv(nh_ctx *ctx, const float *alpha, double eps, double weight, double *value, double *grad,
                int accumulate);
nh_status nh_tv_f64(nh_ctx *ctx, const double *alpha, double eps, double weight, double *value, double *grad,
                    int accumulate);

/* nh_tv without any device allocation, for callers that cannot allocate
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc). Same arguments, result and errors as nh_tv (FP32 alpha), but
 * the per-workgroup partial sums go to one static device array per GPU
 * (4096 doubles, 32 KiB, held until the process ends; its address is
 * resolved by nh_create) instead of a context workspace, and the call
 * returns as soon as its two kernels are queued on the context's stream:
 * value and grad are ready when that stream reaches them. Every workgroup
 * writes its own partial before the finishing kernel reads it, so nothing
 * carries over between calls; but all calls on one GPU share the array, so
 * calls that overlap in time on one GPU (several streams or host threads)
 * race and must be serialised by the caller. Grids needing more partial
 * sums than the array holds are rejected with NH_EINVAL (the kernel's
 * workgroup count is capped at the array's size, so none does today). */
nh_status nh_tv_noalloc(nh_ctx *ctx, const float *alpha, double eps, double weight, double *value, double *grad,
                        int accumulate);

/* Launch tuning: team_blocks_max caps the workgroups of one step (0 = all
 * that fit on the device), tile_z sets the z extent of a tile (0 = auto).
 * profile != 0 times every step kernel with HIP events (nh_stats.t_kernel_*). */
nh_status nh_set_launch(nh_ctx *ctx, int team_blocks_max, int tile_z, int profile);

/* Form of the preconditioned CG iteration (all reach the same fixed point):
 * 0 = the textbook form with two team reductions per iteration (p.Ap, then
 * r.z and |r|^2); 1 = the single-reduction form of Chronopoulos and Gear,
 * which carries A u and A p as extra vectors so that r.z, u.Au and |r|^2 are
 * reduced together once per iteration; 2 (default) = form 1 with the whole CG
 * state of a tile in registers where the grid fits on the device (FP32,
 * zero-flux walls), else form 1. A variant other than 0 resets the
 * preconditioner to Jacobi. Frees the saved forward. */
nh_status nh_set_cg_variant(nh_ctx *ctx, int variant);

/* Preconditioner of the CG solves (the paper leaves preconditioned solvers to
 * future work, Sec. 6). degree 1 (default) = Jacobi, M = D = diag(A) (App.
 * D.2). degree m in 2..16 = a Chebyshev polynomial in D^-1 A: z = y_m of m
 * steps of the Chebyshev iteration for D^-1 A y = D^-1 r from y_0 = 0 over the
 * interval [max(1/max D, hi/(2 m^2)), hi], hi = 2 - 1/max D. hi bounds the
 * spectrum of D^-1 A from above for any diffusivity (A <= 2D - I), so the
 * preconditioned eigenvalues lie in (0, 2), M is symmetric positive definite
 * and CG converges to the same fixed point. It costs m - 1 more operator
 * sweeps and team reductions per iteration and takes about m times fewer
 * iterations, which pays at high diffusivity contrast (1:1000: degree 8 is
 * 10% faster than the default) and not at moderate contrast. max D is reduced
 * on the device once per forward (one host synchronisation).
 * degree >= 2 selects CG variant 0 (the form with z = M^-1 r explicit); it is
 * ignored by fixed-K Jacobi sweeps. EINVAL outside 1..16. Frees the saved
 * forward. */
nh_status nh_set_preconditioner(nh_ctx *ctx, int degree);

/* CG initial guess of every solve. The states of the preceding time levels
 * are h1 = T^{n-1}, h2 = T^{n-2}, h3 = T^{n-3} (forward) or mu^{n+1},
 * mu^{n+2}, mu^{n+3} (adjoint); the extrapolation of order 1 is 2 h1 - h2 and
 * of order 2 is 3 h1 - 3 h2 + h3 (limited by the states there are). mode 0
 * starts from h1 (order 0); mode 1 from the order-2 extrapolation; mode 2
 * (default) adaptively: in each period of 32 steps of a sweep the first three steps
 * start from orders 0, 1 and 2, and the rest from the order that took the
 * fewest CG iterations (chosen on the device, so nothing synchronises); mode 3
 * as mode 2 in the forward sweep, while every adjoint solve after
 * the first starts from the projection of its right-hand side onto the last
 * (up to 6) adjoint solutions, x0 = W (W^T A W)^-1 W^T c: the point of their
 * span closest to the solution in the A-norm (Fischer's method for successive
 * right-hand sides), computed on the device after each adjoint step (about
 * 2k + 5 vector passes for a window of k, no host synchronisation; needs 8
 * adjoint state buffers instead of 4 and one more vector). Fixed-K Jacobi
 * sweeps ignore the projection. All modes converge to the same tolerance. With
 * checkpointing the three states below each checkpoint are kept and
 * recomputed steps repeat the forward's choices, so recomputation stays bit
 * for bit. Drops any saved forward. */
nh_status nh_set_initial_guess(nh_ctx *ctx, int mode);

/* Time limit of the device-side team barrier in seconds (default 20). A
 * barrier that waits longer makes its kernel exit and the call return
 * NH_ETIMEOUT; the context stays usable. */
nh_status nh_set_barrier_timeout(nh_ctx *ctx, double seconds);

nh_status nh_get_stats(const nh_ctx *ctx, nh_stats *out);

/* CG iterations of every step of the last sweep of one kind, to HOST
 * iters[nsteps] (entry n-1 = step n): sweep 0 forward, 1 adjoint, 2 forward
 * steps recomputed from checkpoints (zeros without checkpointing). Entries of
 * a sweep not yet run since the last forward are stale. */
nh_status nh_get_step_iters(const nh_ctx *ctx, int sweep, int *iters);

/* Text of the last error of this context (never NULL). */
const char *nh_last_error(const nh_ctx *ctx);

void nh_destroy(nh_ctx *ctx);

/* Plain device copy dst[i] = src[i], i < n, on `hip_stream` (NULL = the
 * null stream), asynchronous. Not part of the solver: a kernel of known
 * traffic (8 bytes per element) to calibrate hardware byte counters. */
nh_status nh_copy_f32(const float *src, float *dst, size_t n, void *hip_stream);

/* One pass of the streaming CG sweep's memory access pattern without its
 * arithmetic, on `hip_stream` (NULL = the null stream), asynchronous. Not
 * part of the solver: a measurement of what that traffic reaches on the chip.
 * in6: six device pointers, out5: five device pointers (host arrays of device
 * addresses, read during the call), each an nz x ny x nx FP32 volume, x
 * fastest; tiles of 64 x 16 columns march the nz planes, six loads and five
 * device-coherent stores per cell (44 bytes), one workgroup barrier per plane.
 * Results: out[k] = in[k] + in[k+1] (k < 4), out[4] = in[4] + in[5] + in[0]
 * of the -x neighbour within the 64-cell row (0 at its first cell).
 * NH_EINVAL for null pointers, nx not a multiple of 64, ny not a multiple of
 * 16, or a non-positive size. */
nh_status nh_stream_probe_f32(const float *const *in6, float *const *out5, int nx, int ny, int nz,
                              void *hip_stream);

/* ------------------------------------------------------------------------
 * Serving: continuous batching of inversion jobs (the reconstruction loop
 * of Sec. 4.3 run for many independent requests on one GPU).
 *
 * A job is one forward + adjoint pass of a candidate field alpha against
 * surface measurements: forward sweep T^1..T^N (eq. nefty_obj's implicit
 * Euler steps, FP32 vectors with FP64 reductions), the mean squared error
 * L = mean over all n, i, j of (S^n_ij - target^n_ij)^2 with its gradient
 * dL/dS = 2 (S - target) / (N nx ny), then the adjoint sweep and dL/dalpha
 * (eq. adjoint_eq and eq. grad_assembly), exactly as nh_forward + nh_adjoint
 * compute them with full trajectory storage.
 *
 * The server keeps every admitted job's state in device memory and advances
 * all admitted jobs together: each nh_server_tick() makes one cooperative
 * launch in which each job's own team of workgroups runs implicit-Euler
 * steps (forward, or adjoint once its forward is done) with its own
 * reductions, until its CG iterations in the launch reach the slice budget
 * (nh_server_set_slice) or its sweep ends. Before the launch the tick admits
 * queued jobs in arrival order while the job's device bytes fit the HBM
 * budget and its workgroups fit the co-resident limit; after it, finished
 * jobs are retired and their memory freed. A job's team and tiling depend
 * only on its own grid and slices end between steps, so its result is
 * bit-identical alone and among other jobs.
 *
 * Inputs of nh_server_submit are HOST arrays, copied at submission; results
 * come back to HOST memory. One server is driven from one host thread.
 * ---------------------------------------------------------------------- */
typedef struct nh_server nh_server;

typedef enum {
    NH_JOB_QUEUED = 0,   /* submitted, waiting for memory or workgroups */
    NH_JOB_FORWARD = 1,  /* admitted, forward sweep running */
    NH_JOB_ADJOINT = 2,  /* adjoint sweep running */
    NH_JOB_DONE = 3,     /* loss and dL/dalpha available */
    NH_JOB_FAILED = 4    /* a reduction was non-finite or a barrier timed out */
} nh_job_state;

typedef struct {
    int state;              /* nh_job_state */
    int status;             /* OR of per-step flags: 1 max_iter reached, 2 non-finite, 4 barrier timeout */
    int team_blocks;        /* workgroups of this job's team */
    int nsteps;
    long long fwd_iters;    /* CG iterations summed over the forward steps */
    long long adj_iters;
    double loss;            /* mean squared error (valid when DONE) */
    double t_submit_s;      /* steady clock, seconds since the first server was created */
    double t_admit_s;
    double t_done_s;
    size_t device_bytes;    /* device memory held while admitted */
} nh_job_info;

typedef struct {
    long long ticks;        /* batched launches so far */
    double kernel_s;        /* summed duration of those launches (HIP events) */
    size_t used_bytes;      /* device bytes held by admitted jobs */
    int used_blocks;        /* workgroups held by admitted jobs */
    int max_blocks;         /* co-resident workgroup limit of the batched kernel */
    int active;
    int queued;
    long long jobs_done;
    double voxel_steps;     /* sum over finished jobs of 2 * voxels * nsteps (forward + adjoint) */
    long long cg_iters;     /* CG iterations of finished jobs */
    double busy_block_s;    /* sum over launches and jobs of workgroups * the job's time in the launch */
    double span_block_s;    /* sum over launches of max_blocks * the launch's span; busy / span is the
                               fraction of the chip's workgroup slots that did work */
} nh_server_stats;

/* Create a server on `hip_device` working on `hip_stream` (NULL = the null
 * stream). hbm_budget_bytes bounds the device bytes of admitted jobs;
 * max_blocks > 0 lowers the workgroup limit (0 = all that fit co-resident).
 * resident = 1 runs the jobs with the register-resident step (one 512-thread
 * workgroup per tile of 64 x 8 x <= 32 cells, so a job holds about one CU
 * per 16384 cells, at most all of them); resident = 0 with the streaming
 * step (1024-thread workgroups, about 32768 cells each). */
nh_status nh_server_create(nh_server **out, int hip_device, void *hip_stream, double hbm_budget_bytes,
                           int max_blocks, int resident);

/* Slice budget of a tick: about `iters` CG iterations of a workgroup that
 * holds 32768 voxels (smaller tiles run proportionally more; default 512,
 * which measured 3.7% more jobs/s and a 6% lower p99 than 128 on the 40-job
 * Poisson stream).
 * Each job runs at least one step per tick. */
nh_status nh_server_set_slice(nh_server *s, int iters);

/* Admission order: 1 (default) EASY backfilling -- the first queued job that
 * does not fit holds a reservation, and a later job is admitted ahead of it
 * only if it fits now and, by run-time estimates from the measured step
 * times, either ends before the reserved job could start or leaves it room;
 * 0 strict arrival order. */
nh_status nh_server_set_backfill(nh_server *s, int mode);

/* Queue a job. HOST inputs: alpha [nz][ny][nx] (finite, > 0), q_xy [ny][nx],
 * q_t [nsteps] (FP64), target [nsteps][ny][nx]; uniform spacing h; CG to
 * rtol with at most max_iter (<= 30000) iterations per solve. Writes the job id.
 * NH_ENOMEM if the job alone exceeds the budget. */
nh_status nh_server_submit(nh_server *s, int nx, int ny, int nz, double h, double dt, int nsteps, double rtol,
                           int max_iter, const float *alpha, const float *q_xy, const double *q_t,
                           const float *target, long long *job_id);

/* Admit what fits, advance every admitted job by one slice (one launch),
 * retire finished jobs. Writes up to finished_cap ids of jobs that finished
 * in this tick to HOST finished_ids (may be NULL if finished_cap is 0) and
 * the counts; a tick with nothing admitted does nothing. Blocks until the
 * launch has completed. */
nh_status nh_server_tick(nh_server *s, int *n_active, int *n_queued, long long *finished_ids, int finished_cap,
                         int *n_finished);

/* State of a job; copies dL/dalpha (FP64, [nz][ny][nx], HOST) when the job
 * is DONE or FAILED and dL_dalpha is not NULL. */
nh_status nh_server_job(nh_server *s, long long job_id, nh_job_info *info, double *dL_dalpha);

/* Forget a finished job (its host copy of dL/dalpha). NH_ESTATE if it has
 * not finished. */
nh_status nh_server_release(nh_server *s, long long job_id);

nh_status nh_server_get_stats(const nh_server *s, nh_server_stats *out);
const char *nh_server_last_error(const nh_server *s);

/* Synchronizes the server's stream and frees everything, including the
 * memory of jobs still running. */
void nh_server_destroy(nh_server *s);

/* Host-only helpers of the admission policy (no device needed). */

/* Workgroups of a job's team. resident = 1: one per 64 x 8 x (<= 32) tile
 * (0 if that exceeds max_blocks); resident = 0: one tile of at most about
 * 32768 voxels per workgroup, at most max_blocks / 2 workgroups. 0 on bad
 * arguments. */
int nh_serve_job_team(int nx, int ny, int nz, int max_blocks, int resident);

/* Device bytes a job holds while admitted (0 on bad arguments). */
size_t nh_serve_job_bytes(int nx, int ny, int nz, int nsteps, int team_blocks);

/* The jobs the next tick admits, as indices into the queue (arrival order),
 * written to selected[] (room for n_queued); returns their number. Queued job
 * i needs qbytes[i] device bytes and qteams[i] workgroups and is expected to
 * run qdur[i] seconds; running job i holds abytes[i] and ateams[i] and is
 * expected to end in arem[i] seconds. Walking the queue in order, jobs are
 * admitted while they fit the budget and the workgroup limit. With
 * backfill = 0 the walk ends at the first job that does not fit. With
 * backfill = 1 that job holds a reservation: its shadow time is when enough
 * running jobs (in order of expected end) have ended for it to fit, and its
 * extra room is what it would leave free then; a later job is admitted if it
 * fits now and either ends by the shadow time or fits in the extra room
 * (which it then uses up). qdur and arem may be NULL with backfill = 0. */
int nh_serve_admit_select(const size_t *qbytes, const int *qteams, const double *qdur, int n_queued,
                          const size_t *abytes, const int *ateams, const double *arem, int n_active,
                          double budget_bytes, int max_blocks, int backfill, int *selected);

#ifdef __cplusplus
}
#endif

#endif /* NEFTY_HEAT_H */
