"""Throughput of the differentiable heat solver on one MI355X.

One bench step = one forward sweep plus one adjoint sweep of the whole
workload (every implicit-Euler step, every CG iteration, the surface frames,
the MSE gradient on the surface and dL/dalpha), with inputs resident in HBM.
Default workload: 256x256x64 voxels, 1000 steps, dt = 10, lognormal alpha
(sigma 0.3) with 16 ellipsoidal inclusions, uniform top pulse, CG rtol 1e-6,
FP32 vectors with FP64 reductions and gradient.

Prints one JSON line. ``value`` is fwd+adjoint voxel-steps/s
(voxels * steps / time of one forward plus one adjoint). ``roofline`` prices
the dominant kernel against the HBM peak with algorithmic bytes: 48 bytes per
voxel and CG iteration plus 24 (forward) or 52 (adjoint) bytes per voxel and
step, the traffic of textbook two-pass Jacobi-PCG with its vectors in HBM,
over the kernel's HIP-event time; ``traffic`` is the counter-measured HBM
bytes per launch when a record taken on the same kernel sources is stored
under profiles/. ``paper_fixed_k`` times the paper's own solver set-up
(64x64x16, periodic lateral faces, K = 50 Jacobi sweeps; forward and
backward apart, as in its Table 4); ``invert`` the time per iteration of
the two inversion drivers on its training set-up (Table 9). ``serve`` runs the 200 jobs of the
Poisson serving stream through the batching server and, as the baseline,
one by one through the single-problem path. ``long`` times the 512x512x64
long-horizon line (2000 steps) with a checkpoint every 64 steps against
full trajectory storage, with the peak device workspace of each.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E peak, GB/s


def make_workload(name: str, nsteps: int = 0):
    from paper_2603_11045_amd import workloads as wl

    if name == "stiff_256x256x64":
        w = wl.stiff_256x256x64(nsteps=nsteps or 1000)
    elif name == "contrast_256x256x64":
        w = wl.contrast_256x256x64(nsteps=nsteps or 100)
    elif name == "long_512x512x64":
        w = wl.long_512x512x64(nsteps=nsteps or 2000)
    elif name == "mixed_64x64x32":
        w = wl.mixed_64x64x32(nsteps=nsteps or 200)
    elif name == "plain_fp64_16x16x8":
        w = wl.plain_fp64_16x16x8()
    elif name == "paper_64x64x16":
        w = wl.paper_64x64x16(nsteps=nsteps or 50)
    else:
        raise SystemExit(f"unknown workload {name}")
    return w


def cpu_baseline(w, sample_steps: int, threads: int = 0):
    """The FP64 oracle, as it stands, on the first `sample_steps` steps of the
    same workload (forward + adjoint at the workload's own rtol), on all the
    host's cores or on `threads` of them."""
    from oracle import heat as orc

    if threads > 0:
        orc.set_num_threads(threads)

    src = orc.source_series(w.q_xy, w.q_t)[:sample_steps]
    t0 = time.perf_counter()
    opt = dict(h=w.h, rtol=w.rtol, periodic=w.periodic, robin=w.robin, jacobi_k=w.jacobi_k)
    S, T_all, it_f = orc.forward(w.alpha, src, w.dt, **opt)
    gs = np.random.default_rng(0).standard_normal(S.shape) * 1e-3
    G, _, _, it_a = orc.adjoint(w.alpha, T_all, gs, w.dt, **opt)
    t = time.perf_counter() - t0
    vs = w.ng * sample_steps / t
    solver = (f"{w.jacobi_k} Jacobi sweeps per solve" if w.jacobi_k
              else f"Jacobi-PCG at rtol {w.rtol:g}")
    return {"value": vs, "unit": "voxel-steps/s", "cores": orc.num_threads(), "kind": "oracle",
            "sample": f"{w.nx}x{w.ny}x{w.nz}, first {sample_steps} of {w.nsteps} steps, forward+adjoint, "
                      f"FP64 matrix-free {solver} (OpenMP), {t:.1f} s",
            "cg_iters": int(it_f.sum() + it_a.sum()), "seconds": t}


def stream_probe(dev, reps: int = 20) -> dict:
    """What the streaming sweep's traffic reaches on this chip: nh_stream_probe_f32
    (6 loads and 5 device-coherent stores per cell, 64x16-column tiles marching
    512x512x64, one barrier per plane, no arithmetic), timed with events on its
    stream over `reps` passes after 3 warm-up passes."""
    import ctypes

    import torch

    from paper_2603_11045_amd import _lib

    nx, ny, nz = 512, 512, 64
    bufs = [torch.full((nz, ny, nx), float(k), dtype=torch.float32, device=dev) for k in range(11)]
    vp = ctypes.c_void_p
    ins = (vp * 6)(*[b.data_ptr() for b in bufs[:6]])
    outs = (vp * 5)(*[b.data_ptr() for b in bufs[6:]])
    lib = _lib.load()
    stream = torch.cuda.current_stream()

    def once():
        code = lib.nh_stream_probe_f32(ins, outs, nx, ny, nz, vp(stream.cuda_stream))
        if code != 0:
            raise RuntimeError(f"nh_stream_probe_f32 returned {code}")

    for _ in range(3):
        once()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        once()
    e1.record(stream)
    torch.cuda.synchronize()
    us = e0.elapsed_time(e1) * 1e3 / reps
    ok = bool(torch.all(bufs[6] == 1.0)) and bool(torch.all(bufs[9] == 7.0))
    del bufs
    torch.cuda.empty_cache()
    gbs = 44.0 * nx * ny * nz / us / 1e3
    return {"grid": [nx, ny, nz], "bytes_per_cell": 44, "passes": reps, "us_per_pass": us, "gbs": gbs,
            "frac_of_peak": gbs / 8000.0, "outputs_ok": ok}


def paper_fixed_k(Solver, dev, reps: int):
    """The paper's own solver set-up (App. D.2, Table 5): the 64x64x16
    specimen with periodic lateral faces, dx = dy = 0.156, dz = 0.0625,
    dt = 0.05 and K = 50 Jacobi sweeps per solve, FP32. Forward and backward
    (adjoint) are timed apart, as in the solver benchmark of Table 4 (50
    steps), and together over the 100 frames of the training set-up. Median
    over `reps` repetitions after one warm-up."""
    import torch

    from paper_2603_11045_amd import workloads as wl

    out = {"workload": "paper_64x64x16", "grid": [64, 64, 16], "spacing": [0.156, 0.156, 0.0625], "dt": 0.05,
           "jacobi_k": 50, "lateral": "periodic", "dtype": "f32"}
    for nsteps in (50, 100):
        w = wl.paper_64x64x16(nsteps=nsteps)
        s = Solver(w.nx, w.ny, w.nz, h=w.h, device=0, periodic=True, jacobi_k=w.jacobi_k)
        alpha = torch.from_numpy(w.alpha).to(dev)
        q_xy = torch.from_numpy(w.q_xy).to(dev)
        target = s.forward(torch.from_numpy(w.alpha_target).to(dev), q_xy, w.q_t, w.dt, nsteps).clone()
        tf, tb = [], []
        for r in range(reps + 1):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            S = s.forward(alpha, q_xy, w.q_t, w.dt, nsteps)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            g = (2.0 / S.numel()) * (S - target)
            torch.cuda.synchronize()
            t2 = time.perf_counter()
            s.adjoint(g)
            torch.cuda.synchronize()
            t3 = time.perf_counter()
            if r > 0:
                tf.append(t1 - t0)
                tb.append(t3 - t2)
        st = s.stats()
        fwd, bwd = float(np.median(tf)), float(np.median(tb))
        sweeps = 2 * nsteps * w.jacobi_k
        key = f"steps_{nsteps}"
        out[key] = {"fwd_s": fwd, "bwd_s": bwd, "fwd_bwd_ms": (fwd + bwd) * 1e3,
                    "voxel_sweeps_per_s": w.ng * sweeps / (fwd + bwd),
                    "alg_gb_per_s": (st["bytes_alg_fwd"] + st["bytes_alg_adj"]) / (fwd + bwd) / 1e9,
                    "team_blocks": st["team_blocks"], "peak_workspace_mb": st["peak_workspace_bytes"] / 1e6}
        print(f"[bench] paper fixed-K, {nsteps} steps: fwd {fwd * 1e3:.2f} ms, bwd {bwd * 1e3:.2f} ms",
              file=sys.stderr, flush=True)
        s.close()
    out["paper_table4_context"] = {"fwd_s": 0.46, "bwd_s": 0.50, "peak_mb": 21.9, "steps": 50,
                                   "gpu": "NVIDIA RTX PRO 6000 (the paper's; not this machine)"}
    return out


def invert_iterations(dev, iters: int):
    """Time per optimisation iteration of the two inversion drivers on the
    paper's training set-up (64x64x16, 100 frames, K = 50, TV, Adam; the
    neural field at its full size, 10 layers of width 512 with 12 bands):
    one forward sweep, one adjoint sweep, the TV kernel and the optimiser step
    (plus the MLP forward and backward for the neural field)."""
    import torch

    from paper_2603_11045_amd import workloads as wl
    from paper_2603_11045_amd.invert import InvertConfig, reconstruct
    from paper_2603_11045_amd.solver import Solver

    w = wl.paper_64x64x16(nsteps=100)
    s = Solver(w.nx, w.ny, w.nz, h=w.h, periodic=True, jacobi_k=w.jacobi_k)
    target = s.forward(torch.from_numpy(w.alpha).to(dev), torch.from_numpy(w.q_xy).to(dev), w.q_t, w.dt,
                       w.nsteps).clone()
    s.close()
    out = {"workload": "paper_64x64x16", "nsteps": 100, "jacobi_k": 50, "iters_timed": iters}
    for method in ("grid", "nefty"):
        reconstruct(w, target, InvertConfig(method=method, iters=2), bulk_mean=float(np.median(w.alpha)))
        r = reconstruct(w, target, InvertConfig(method=method, iters=iters), alpha_true=w.alpha,
                        bulk_mean=float(np.median(w.alpha)))
        out[method] = {"ms_per_iter": r.ms_per_iter, "metrics_after": r.metrics}
        print(f"[bench] invert {method}: {r.ms_per_iter:.2f} ms/iteration", file=sys.stderr, flush=True)
    out["paper_table9_context_ms_per_iter"] = {"grid": 47.8, "nefty": 57.5,
                                               "gpu": "NVIDIA RTX PRO 6000 (the paper's; not this machine)"}
    return out


def serve_section(n_jobs: int) -> dict:
    """The first n_jobs of the Poisson serving stream (all 200 by default)
    through the batching server, and one by one through the single-problem
    path as the baseline; also the largest relative difference between a
    job's loss in the two runs."""
    from paper_2603_11045_amd import serve

    print(f"[bench] serving: first {n_jobs} jobs of the Poisson stream (20 jobs/s, seed 5)",
          file=sys.stderr, flush=True)
    sv = serve.benchmark(n_jobs, log=lambda m: print("[bench] " + m, file=sys.stderr, flush=True))
    b, q = sv["batched"], sv["sequential"]
    return {
        "jobs": b["jobs"], "rate_jobs_per_s": sv["rate_jobs_per_s"], "hbm_budget_gb": sv["hbm_budget_gb"],
        "p50_ms": b["p50_ms"], "p99_ms": b["p99_ms"], "jobs_per_s": b["jobs_per_s"],
        "voxel_steps_per_s": b["voxel_steps_per_s"], "workgroup_busy_frac": b["workgroup_busy_frac"],
        "sequential": {"p50_ms": q["p50_ms"], "p99_ms": q["p99_ms"], "jobs_per_s": q["jobs_per_s"]},
        "speedup": {"throughput": sv["speedup_throughput"], "p50": sv["speedup_p50"],
                    "p99": sv["speedup_p99"]},
        "max_rel_loss_diff_vs_sequential": sv["max_rel_loss_diff_vs_sequential"],
    }


def long_section(dev, nsteps: int, k: int) -> dict:
    """The long-horizon memory path: 512x512x64 (four times what the chip's
    registers hold, so the streaming kernel runs it), `nsteps` steps, one
    forward + adjoint pass with a checkpoint every k steps (segments
    recomputed in the adjoint) and one with every state stored: time and the
    library's peak device workspace of each."""
    import torch

    from paper_2603_11045_amd import workloads as wl
    from paper_2603_11045_amd.solver import Solver

    w = wl.long_512x512x64(nsteps=nsteps, checkpoint_every=k)
    alpha = torch.from_numpy(w.alpha).to(dev)
    q_xy = torch.from_numpy(w.q_xy).to(dev)
    out = {"workload": w.name, "grid": [w.nx, w.ny, w.nz], "nsteps": nsteps, "dt": w.dt, "rtol": w.rtol,
           "checkpoint_every": k}
    target = None
    for key, ck in (("checkpointed", k), ("full_storage", 0)):
        s = Solver(w.nx, w.ny, w.nz, h=w.h, rtol=w.rtol, max_iter=2000, checkpoint_every=ck, device=0)
        if target is None:
            target = s.forward(torch.from_numpy(w.alpha_target).to(dev), q_xy, w.q_t, w.dt, nsteps).clone()
        m = target.numel()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        S = s.forward(alpha, q_xy, w.q_t, w.dt, nsteps)
        s.adjoint((2.0 / m) * (S - target))
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        st = s.stats()
        out[key] = {"s_per_pass": el, "voxel_steps_per_s": w.ng * nsteps / el,
                    "peak_workspace_gb": st["peak_workspace_bytes"] / 1e9,
                    "cg_iters": {"fwd": st["fwd_iters"], "adj": st["adj_iters"],
                                 "recompute": st["recompute_iters"]},
                    "kernel": "nh::resident_step_kernel<64>" if st["resident"] else "nh::step_kernel<float>"}
        print(f"[bench] long {key}: {el:.2f} s per pass, peak workspace "
              f"{st['peak_workspace_bytes'] / 1e9:.1f} GB", file=sys.stderr, flush=True)
        s.close()
        del S
        torch.cuda.empty_cache()
    c, f = out["checkpointed"], out["full_storage"]
    out["time_overhead"] = c["s_per_pass"] / f["s_per_pass"] - 1.0
    out["memory_saving"] = 1.0 - c["peak_workspace_gb"] / f["peak_workspace_gb"]
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="stiff_256x256x64")
    ap.add_argument("--nsteps", type=int, default=0, help="override the time-step count (testing)")
    ap.add_argument("--checkpoint-every", type=int, default=-1)
    ap.add_argument("--team", type=int, default=0)
    ap.add_argument("--tile-z", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample-steps", type=int, default=16)
    ap.add_argument("--cpu-threads", type=int, default=0,
                    help="OpenMP threads of the oracle timing (0 = all the host gives it)")
    ap.add_argument("--no-profile", action="store_true", help="skip per-launch HIP event timing")
    ap.add_argument("--guess", default="adaptive", choices=["previous", "extrapolate", "adaptive", "projection"],
                    help="CG initial guess of the solves")
    ap.add_argument("--cheb", type=int, default=1,
                    help="preconditioner: 1 Jacobi, m >= 2 Chebyshev polynomial of degree m (CG variant 0)")
    ap.add_argument("--variant", type=int, default=2, help="CG variant (0 two reductions, 1 one, 2 resident)")
    ap.add_argument("--ckpt-overhead", action="store_true",
                    help="with checkpointing on: also time the same passes with full trajectory storage "
                         "and report peak device memory of both")
    ap.add_argument("--serve-jobs", type=int, default=200,
                    help="jobs of the Poisson serving stream to serve (0 = skip the serving run)")
    ap.add_argument("--long-steps", type=int, default=2000,
                    help="steps of the 512x512x64 long-horizon line, checkpointed vs full storage (0 = skip)")
    ap.add_argument("--paper-reps", type=int, default=5,
                    help="repetitions of the paper-shaped fixed-K timing (0 = skip)")
    ap.add_argument("--invert-iters", type=int, default=20,
                    help="timed iterations of each inversion driver (0 = skip)")
    ap.add_argument("--no-stream-probe", action="store_true",
                    help="skip the access-pattern probe (nh_stream_probe_f32) of the streaming sweep")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="first run a plain 1 GiB device copy (nh_copy_f32) three times, so that "
                         "hardware byte counters can be scaled against a kernel of known traffic")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on exactly one GPU: the solver has no multi-GPU path "
              "(one problem per GPU)", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2603_11045_amd import Solver

    dev = torch.device("cuda", 0)
    if args.calibrate_copy:
        import ctypes

        from paper_2603_11045_amd import _lib

        n = 1 << 28                                   # 2^28 floats = 1 GiB read + 1 GiB written
        src = torch.zeros(n, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        lib = _lib.load()
        for _ in range(3):
            code = lib.nh_copy_f32(ctypes.c_void_p(src.data_ptr()), ctypes.c_void_p(dst.data_ptr()), n,
                                   ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
            assert code == 0, code
        torch.cuda.synchronize()
        del src, dst
        print("[bench] calibration copy: 3 x nh::copy_kernel<float> of 2^28 elements", file=sys.stderr,
              flush=True)
    w = make_workload(args.workload, args.nsteps)
    ck = w.checkpoint_every if args.checkpoint_every < 0 else args.checkpoint_every
    dtype = torch.float32 if w.precision == "f32" else torch.float64
    print(f"[bench] workload {w.name}: {w.nx}x{w.ny}x{w.nz}, {w.nsteps} steps, dt {w.dt}, rtol {w.rtol}, "
          f"checkpoint_every {ck}", file=sys.stderr, flush=True)

    solver = Solver(w.nx, w.ny, w.nz, h=w.h, rtol=w.rtol, max_iter=2000, checkpoint_every=ck,
                    precision=w.precision, device=0, team_blocks_max=args.team, tile_z=args.tile_z,
                    profile=not args.no_profile, periodic=w.periodic, robin=w.robin, jacobi_k=w.jacobi_k,
                    initial_guess=args.guess, cg_variant=args.variant, preconditioner_degree=args.cheb)
    alpha = torch.from_numpy(w.alpha).to(dev)
    q_xy = torch.from_numpy(w.q_xy).to(dev)
    # synthetic measurement: the surface of the target diffusivity
    target = solver.forward(torch.from_numpy(w.alpha_target).to(dev), q_xy, w.q_t, w.dt, w.nsteps).clone()
    m = target.numel()

    def one_step():
        S = solver.forward(alpha, q_xy, w.q_t, w.dt, w.nsteps)
        g = (2.0 / m) * (S - target)           # d/dS of mean((S - target)^2), caller side
        G = solver.adjoint(g)
        return S, G

    for i in range(args.warmup):
        one_step()
        print(f"[bench] warmup {i + 1}/{args.warmup} done", file=sys.stderr, flush=True)
    torch.cuda.synchronize()

    t_fwd = t_adj = tk_f = tk_a = bytes_f = bytes_a = 0.0
    it_f = it_a = it_r = launches = 0
    t0 = time.perf_counter()
    for i in range(args.steps):
        one_step()
        st = solver.stats()
        t_fwd += st["t_fwd_s"]
        t_adj += st["t_adj_s"]
        tk_f += st["t_kernel_fwd_s"]
        tk_a += st["t_kernel_adj_s"]
        bytes_f += st["bytes_alg_fwd"]
        bytes_a += st["bytes_alg_adj"]
        it_f += st["fwd_iters"]
        it_a += st["adj_iters"]
        it_r += st["recompute_iters"]
        launches += st["launches_fwd"] + st["launches_adj"]
        print(f"[bench] step {i + 1}/{args.steps}: fwd {st['t_fwd_s']:.3f} s ({st['fwd_iters']} CG it), "
              f"adj {st['t_adj_s']:.3f} s ({st['adj_iters']} CG it)", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0

    K = args.steps
    vox_steps = float(w.ng) * w.nsteps * K
    value = vox_steps / elapsed
    iters = it_f + it_a + it_r
    st = solver.stats()
    roof = None
    if st["resident"]:
        kname = "nh::resident_step_kernel<64>"
    elif st["jacobi_blocked"]:
        kname = "nh::jacobi_steps_kernel<8>"
    else:
        kname = "nh::step_kernel<float>" if w.precision == "f32" else "nh::step_kernel<double>"
    if not args.no_profile and (tk_f + tk_a) > 0:
        from paper_2603_11045_amd import profiling

        achieved = (bytes_f + bytes_a) / (tk_f + tk_a) / 1e9
        alg_per_launch = (bytes_f + bytes_a) / max(launches, 1)
        tr_path = os.path.join(ROOT, "profiles", f"traffic_{kname.split('::')[1].split('<')[0]}_{w.name}.json")
        tr = profiling.load_traffic(tr_path, kname)
        m = solver.preconditioner_degree
        it_bytes = "48" if m < 2 else f"{48 + 20 * (m - 1)} (Chebyshev degree {m})"
        model = ("16 B/voxel/Jacobi sweep + 28 (adj) B/voxel/step" if w.jacobi_k
                 else f"{it_bytes} B/voxel/CG iteration + 24 (fwd) or 52 (adj) B/voxel/step")
        roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": tr["traffic_bytes_per_launch"] if tr else None,
                "kernel": kname,
                "avg_launch_us": round((tk_f + tk_a) / max(launches, 1) * 1e6, 2),
                "alg_bytes_per_launch": alg_per_launch,
                "alg_bytes_model": model,
                "kernel_time_frac": round((tk_f + tk_a) / elapsed, 4)}
        if tr:
            roof["traffic_over_alg"] = round(tr["traffic_bytes_per_launch"] / alg_per_launch, 4)
            roof["traffic_source"] = os.path.relpath(tr_path, ROOT)
            # the HBM bandwidth the counters show, beside the algorithmic figure
            counter_gbs = tr["traffic_bytes_per_launch"] / ((tk_f + tk_a) / max(launches, 1)) / 1e9
            roof["counter_achieved"] = round(counter_gbs, 1)
            roof["counter_frac"] = round(counter_gbs / HBM_PEAK_GBS, 4)
    rec = {
        "metric": "fwd+adjoint voxel-steps/s",
        "value": value,
        "unit": "voxel-steps/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": args.warmup,
        "ms_per_step": elapsed / K * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": w.precision,
        "data": "synthetic",
        "config": {"workload": w.name, "grid": [w.nx, w.ny, w.nz], "nsteps": w.nsteps, "dt": w.dt,
                   "rtol": w.rtol, "checkpoint_every": ck, "initial_guess": args.guess,
                   "cg_variant": solver.cg_variant, "preconditioner_degree": solver.preconditioner_degree,
                   "team_blocks": st["team_blocks"],
                   "tile": [st["tile_x"], st["tile_y"], st["tile_z"]]},
        "cg_iters_per_s": iters / elapsed,
        "voxel_iters_per_s": iters * float(w.ng) / elapsed,
        "cg_iters_per_step": {"fwd": it_f / K, "adj": it_a / K, "recompute": it_r / K},
        "t_fwd_s": t_fwd / K,
        "t_adj_s": t_adj / K,
        "roofline": roof,
        "peak_workspace_gb": st["peak_workspace_bytes"] / 1e9,
    }
    props = torch.cuda.get_device_properties(dev)
    rec["device"] = {"name": props.name, "arch": getattr(props, "gcnArchName", ""),
                     "compute_units": props.multi_processor_count, "memory_gb": props.total_memory / 1e9,
                     "hbm_peak_gbs": HBM_PEAK_GBS}
    rec["memory"] = {"library_peak_workspace_gb": st["peak_workspace_bytes"] / 1e9,
                     "torch_peak_allocated_gb": torch.cuda.max_memory_allocated(dev) / 1e9,
                     "device_used_gb": (torch.cuda.mem_get_info(dev)[1] - torch.cuda.mem_get_info(dev)[0]) / 1e9}
    if args.ckpt_overhead and ck > 0:
        # the same passes with every state stored: the cost of recomputation
        solver.close()
        torch.cuda.empty_cache()
        full = Solver(w.nx, w.ny, w.nz, h=w.h, rtol=w.rtol, max_iter=2000, checkpoint_every=0,
                      precision=w.precision, device=0, team_blocks_max=args.team, tile_z=args.tile_z)
        print("[bench] full-storage comparison ...", file=sys.stderr, flush=True)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for i in range(args.steps):
            S = full.forward(alpha, q_xy, w.q_t, w.dt, w.nsteps)
            full.adjoint((2.0 / m) * (S - target))
            print(f"[bench] full-storage step {i + 1}/{args.steps} done", file=sys.stderr, flush=True)
        torch.cuda.synchronize()
        el_full = time.perf_counter() - t1
        sf = full.stats()
        rec["checkpointing"] = {
            "checkpoint_every": ck,
            "ms_per_step": elapsed / K * 1e3,
            "peak_workspace_gb": st["peak_workspace_bytes"] / 1e9,
            "recompute_iters_per_step": it_r / K,
            "full_storage": {"ms_per_step": el_full / K * 1e3, "peak_workspace_gb": sf["peak_workspace_bytes"] / 1e9},
            "time_overhead": elapsed / el_full - 1.0,
            "memory_saving": 1.0 - st["peak_workspace_bytes"] / sf["peak_workspace_bytes"],
        }
        full.close()
    # the GPU on the oracle's sample (the first steps of the same workload,
    # which need more CG iterations than the average step), for a like-for-like ratio
    gpu_sample = None
    if not args.no_cpu_baseline and not (args.ckpt_overhead and ck > 0):
        ns = min(args.cpu_sample_steps, w.nsteps)
        solver.forward(alpha, q_xy, w.q_t[:ns], w.dt, ns)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        S = solver.forward(alpha, q_xy, w.q_t[:ns], w.dt, ns)
        solver.adjoint((2.0 / target[:ns].numel()) * (S - target[:ns]))
        torch.cuda.synchronize()
        gpu_sample = float(w.ng) * ns / (time.perf_counter() - t1)
    # release the library's device objects before the run's end, rather than at interpreter teardown
    solver.close()
    del solver, alpha, q_xy, target
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    def section(name, fn):
        # the extra sections never cost the main line: a failure is recorded instead
        try:
            rec[name] = fn()
        except Exception as e:  # noqa: BLE001
            print(f"[bench] section {name} failed: {e!r}", file=sys.stderr, flush=True)
            rec[name] = {"error": repr(e)}

    if not args.no_stream_probe:
        section("stream_probe", lambda: stream_probe(dev))
    if args.paper_reps > 0:
        section("paper_fixed_k", lambda: paper_fixed_k(Solver, dev, args.paper_reps))
    if args.invert_iters > 0:
        section("invert", lambda: invert_iterations(dev, args.invert_iters))
    if args.serve_jobs > 0:
        section("serve", lambda: serve_section(args.serve_jobs))
    if args.long_steps > 0 and args.workload == "stiff_256x256x64":
        section("long", lambda: long_section(dev, args.long_steps, 64))
    if not args.no_cpu_baseline:
        print("[bench] cpu baseline (FP64 oracle) ...", file=sys.stderr, flush=True)
        section("cpu_baseline", lambda: {k: v for k, v in cpu_baseline(w, min(args.cpu_sample_steps, w.nsteps),
                                                                         args.cpu_threads).items()
                                         if k in ("value", "unit", "cores", "kind", "sample")})
        if gpu_sample and "value" in rec["cpu_baseline"]:
            rec["cpu_baseline"]["gpu_value_same_sample"] = gpu_sample
            rec["cpu_baseline"]["gpu_over_cpu_same_sample"] = gpu_sample / rec["cpu_baseline"]["value"]
    torch.cuda.synchronize()
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
