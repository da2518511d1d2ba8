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
 *   (A x)_p = x_p + dt * sum_{interior faces f=(p,q)} c_f (x_p - x_q)
 *            every boundary face is zero-flux (carries no term)
 *   A T^n   = T^{n-1} + dt q^n,   T^0 = 0,   q^n = q_t[n-1] * q_xy on the top plane k = 0
 *   S^n     = T^n on k = 0                         (the observation projector of eq. nefty_obj)
 *   A mu^n  = mu^{n+1} + Pi^T dL/dS^n,  mu^{N+1} = 0   (eq. adjoint_eq)
 *   dL/da_p = -dt sum_n sum_{f ni p} 2 a_q^2/(a_p+a_q)^2/h_d^2 (T^n_p-T^n_q)(mu^n_p-mu^n_q)
 *                                                   (eq. grad_assembly, App. D.3)
 *
 * Every linear solve is a Jacobi-preconditioned conjugate gradient run to
 * ||r||_2 <= rtol * ||b||_2, warm-started from the previous state (forward)
 * or from mu^{n+1} (adjoint), as App. D.2 warm-starts its Jacobi sweeps.
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
    double bytes_alg_fwd;       /* algorithmic HBM bytes of the step kernels, last forward */
    double bytes_alg_adj;       /* same for the last adjoint (recomputation included) */
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

/* Copy the saved state T^n (1 <= n <= nsteps, full storage; or a checkpoint
 * step when checkpointing) of the last forward into `out` ([nz][ny][nx],
 * device, the forward's precision). NH_ESTATE if that state is not held. */
nh_status nh_get_state(nh_ctx *ctx, int n, void *out);

/* y = A x for the operator of Sec. 4.2 with diffusivity alpha and step dt
 * on the current grid (the stencil kernel on its own; for operator tests).
 * alpha, x, y: [nz][ny][nx] FP32 device arrays (y must not alias x). */
nh_status nh_apply_A(nh_ctx *ctx, const float *alpha, const float *x, float *y, double dt);

/* Launch tuning: team_blocks_max caps the workgroups of one step (0 = all
 * that fit on the device), tile_z sets the z extent of a tile (0 = auto).
 * profile != 0 times every step kernel with HIP events (nh_stats.t_kernel_*). */
nh_status nh_set_launch(nh_ctx *ctx, int team_blocks_max, int tile_z, int profile);

/* Form of the preconditioned CG iteration (both reach the same fixed point):
 * 0 = the textbook form with two team reductions per iteration (p.Ap, then
 * r.z and |r|^2); 1 (default) = the single-reduction form of Chronopoulos and
 * Gear, which carries A u and A p as extra vectors so that r.z, u.Au and
 * |r|^2 are reduced together once per iteration. Frees the saved forward. */
nh_status nh_set_cg_variant(nh_ctx *ctx, int variant);

/* Time limit of the device-side team barrier in seconds (default 20). A
 * barrier that waits longer makes its kernel exit and the call return
 * NH_ETIMEOUT; the context stays usable. */
nh_status nh_set_barrier_timeout(nh_ctx *ctx, double seconds);

nh_status nh_get_stats(const nh_ctx *ctx, nh_stats *out);

/* Text of the last error of this context (never NULL). */
const char *nh_last_error(const nh_ctx *ctx);

void nh_destroy(nh_ctx *ctx);

/* Plain device copy dst[i] = src[i], i < n, on `hip_stream` (NULL = the
 * null stream), asynchronous. Not part of the solver: a kernel of known
 * traffic (8 bytes per element) to calibrate hardware byte counters. */
nh_status nh_copy_f32(const float *src, float *dst, size_t n, void *hip_stream);

#ifdef __cplusplus
}
#endif

#endif /* NEFTY_HEAT_H */
