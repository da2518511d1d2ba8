"""Serving front end: a ``Server`` over the library's continuous-batching
server (``nh_server_*``) and a Poisson-arrival driver that measures request
latency, beside the sequential baseline that solves the same jobs one after
another with a single-problem ``Solver`` each.

A job is one forward + adjoint pass of a candidate field against surface
measurements (mean squared error), i.e. one evaluation of the reconstruction
loss and its gradient in the paper's Sec. 4.3 loop. Inputs are host arrays;
the library copies them to the device at admission. Every step of every job
runs in the library's kernels.
"""
from __future__ import annotations

import ctypes
import time
from collections import deque
from dataclasses import dataclass, field
from typing import Dict, List, Optional, Sequence

import numpy as np
import torch

from . import _lib
from .solver import Solver


def _check(code, srv, func, lib):
    if code != _lib.NH_OK:
        msg = lib.nh_server_last_error(srv).decode(errors="replace") if srv is not None else ""
        raise _lib.NHError(code, func, msg)


def _f32(a, shape, name):
    a = np.ascontiguousarray(np.asarray(a, dtype=np.float32))
    if a.size != int(np.prod(shape)):
        raise ValueError(f"{name} must have {int(np.prod(shape))} elements (got {a.size})")
    return a


class Server:
    """Continuous-batching server on one GPU.

    ``submit`` queues a job; each ``tick`` admits what fits (HBM budget and
    co-resident workgroups, arrival order), advances every admitted job by a
    slice of implicit-Euler steps in a single launch, and retires finished
    jobs.
    """

    def __init__(self, hbm_budget_bytes: float = 200e9, max_blocks: int = 0,
                 device: Optional[int] = None, stream: Optional[torch.cuda.Stream] = None,
                 slice_iters: int = 0, backfill: Optional[int] = None, kernel: str = "resident"):
        if kernel not in ("resident", "streaming"):
            raise ValueError("kernel must be 'resident' or 'streaming'")
        self.kernel = kernel
        self.lib = _lib.load()
        self.device = torch.device("cuda", torch.cuda.current_device() if device is None else device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self._srv = ctypes.c_void_p()
        _check(self.lib.nh_server_create(ctypes.byref(self._srv), self.device.index,
                                         ctypes.c_void_p(self.stream.cuda_stream), float(hbm_budget_bytes),
                                         int(max_blocks), int(kernel == "resident")), None, "nh_server_create",
               self.lib)
        self._shapes: Dict[int, tuple] = {}
        self._done = (ctypes.c_longlong * 256)()
        if slice_iters:
            self.set_slice(slice_iters)
        if backfill is not None:
            self.set_backfill(backfill)

    def set_backfill(self, mode: int):
        """1: EASY backfilling (default), 0: strict arrival order."""
        _check(self.lib.nh_server_set_backfill(self._srv, int(mode)), self._srv, "nh_server_set_backfill",
               self.lib)

    def set_slice(self, iters: int):
        """CG iterations per tick of a 32768-voxel workgroup (see the header)."""
        _check(self.lib.nh_server_set_slice(self._srv, int(iters)), self._srv, "nh_server_set_slice", self.lib)

    def submit(self, alpha, q_xy, q_t, target, dt: float, h: float = 1.0, rtol: float = 1e-6,
               max_iter: int = 1000) -> int:
        """Queue a job. ``alpha`` is ``[nz][ny][nx]``, ``q_xy`` ``[ny][nx]``,
        ``q_t`` ``[nsteps]``, ``target`` ``[nsteps][ny][nx]``. Returns its id."""
        alpha = np.asarray(alpha)
        if alpha.ndim != 3:
            raise ValueError("alpha must be [nz][ny][nx]")
        nz, ny, nx = alpha.shape
        qt = np.ascontiguousarray(np.asarray(q_t, dtype=np.float64).reshape(-1))
        nsteps = qt.size
        a = _f32(alpha, (nz, ny, nx), "alpha")
        q = _f32(q_xy, (ny, nx), "q_xy")
        t = _f32(target, (nsteps, ny, nx), "target")
        jid = ctypes.c_longlong()
        _check(self.lib.nh_server_submit(self._srv, nx, ny, nz, float(h), float(dt), nsteps, float(rtol),
                                         int(max_iter), a.ctypes.data, q.ctypes.data, qt.ctypes.data,
                                         t.ctypes.data, ctypes.byref(jid)), self._srv, "nh_server_submit",
               self.lib)
        self._shapes[jid.value] = (nz, ny, nx)
        return jid.value

    def tick(self):
        """One batched launch. Returns ``(n_active, n_queued, finished_ids)``."""
        na, nq, nf = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
        _check(self.lib.nh_server_tick(self._srv, ctypes.byref(na), ctypes.byref(nq), self._done,
                                       len(self._done), ctypes.byref(nf)), self._srv, "nh_server_tick", self.lib)
        n = min(nf.value, len(self._done))
        return na.value, nq.value, [self._done[i] for i in range(n)]

    def info(self, job_id: int) -> dict:
        inf = _lib.nh_job_info()
        _check(self.lib.nh_server_job(self._srv, int(job_id), ctypes.byref(inf), None), self._srv,
               "nh_server_job", self.lib)
        d = inf.as_dict()
        d["state_name"] = _lib.JOB_STATE_NAMES.get(d["state"], str(d["state"]))
        return d

    def result(self, job_id: int):
        """``(loss, dL/dalpha [nz][ny][nx] float64, info)`` of a finished job."""
        G = np.empty(self._shapes[job_id], dtype=np.float64)
        inf = _lib.nh_job_info()
        _check(self.lib.nh_server_job(self._srv, int(job_id), ctypes.byref(inf), G.ctypes.data), self._srv,
               "nh_server_job", self.lib)
        if inf.state not in (_lib.NH_JOB_DONE, _lib.NH_JOB_FAILED):
            raise RuntimeError(f"job {job_id} has not finished (state {inf.state})")
        return inf.loss, G, inf.as_dict()

    def release(self, job_id: int):
        _check(self.lib.nh_server_release(self._srv, int(job_id)), self._srv, "nh_server_release", self.lib)
        self._shapes.pop(job_id, None)

    def stats(self) -> dict:
        s = _lib.nh_server_stats()
        _check(self.lib.nh_server_get_stats(self._srv, ctypes.byref(s)), self._srv, "nh_server_get_stats",
               self.lib)
        return s.as_dict()

    def run_until_idle(self, max_ticks: int = 10_000_000) -> List[int]:
        """Tick until nothing is admitted or queued; returns finished ids."""
        done = []
        for _ in range(max_ticks):
            na, nq, fin = self.tick()
            done += fin
            if na == 0 and nq == 0:
                return done
        raise RuntimeError("server did not drain")

    def close(self):
        if getattr(self, "_srv", None) is not None and self._srv.value:
            self.lib.nh_server_destroy(self._srv)
            self._srv = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---------------------------------------------------------------------------
# Poisson-arrival driver and the sequential baseline

@dataclass
class Request:
    """One job of a stream: arrival time (s from the start) and its inputs."""
    arrival_s: float
    alpha: np.ndarray
    q_xy: np.ndarray
    q_t: np.ndarray
    target: np.ndarray
    dt: float
    h: float = 1.0
    rtol: float = 1e-6
    max_iter: int = 1000
    tag: str = ""


@dataclass
class StreamResult:
    latency_s: List[float]
    makespan_s: float
    losses: List[float]
    voxel_steps: float
    cg_iters: int
    extra: dict = field(default_factory=dict)

    def summary(self) -> dict:
        lat = np.asarray(self.latency_s)
        return {
            "jobs": int(lat.size),
            "p50_ms": float(np.percentile(lat, 50) * 1e3),
            "p99_ms": float(np.percentile(lat, 99) * 1e3),
            "mean_ms": float(lat.mean() * 1e3),
            "makespan_s": self.makespan_s,
            "jobs_per_s": float(lat.size / self.makespan_s),
            "voxel_steps_per_s": self.voxel_steps / self.makespan_s,
            "cg_iters": int(self.cg_iters),
            **self.extra,
        }


def requests_from_specs(specs, targets: Sequence[np.ndarray]) -> List[Request]:
    """Requests from ``workloads.JobSpec`` entries and their target series."""
    out = []
    for s, t in zip(specs, targets):
        w = s.workload
        out.append(Request(s.arrival_s, w.alpha, w.q_xy, w.q_t, t, w.dt, w.h[0], w.rtol, 1000, w.name))
    return out


def target_series(specs, rtol: float = 1e-6) -> List[np.ndarray]:
    """Surface measurements of each job's ``alpha_target`` from the HIP
    forward sweep (one single-problem ``Solver`` per grid shape)."""
    solvers: Dict[tuple, Solver] = {}
    out = []
    for s in specs:
        w = s.workload
        key = (w.nx, w.ny, w.nz)
        if key not in solvers:
            solvers[key] = Solver(w.nx, w.ny, w.nz, h=w.h, rtol=rtol)
        sv = solvers[key]
        a = torch.from_numpy(np.ascontiguousarray(w.alpha_target, dtype=np.float32)).cuda()
        q = torch.from_numpy(np.ascontiguousarray(w.q_xy, dtype=np.float32)).cuda()
        out.append(sv.forward(a, q, w.q_t, w.dt, w.nsteps).cpu().numpy())
    for sv in solvers.values():
        sv.close()
    return out


def serve_stream(reqs: Sequence[Request], hbm_budget_bytes: float = 200e9, max_blocks: int = 0,
                 keep_grads: bool = False, log=None, slice_iters: int = 0,
                 backfill: Optional[int] = None, kernel: str = "resident") -> StreamResult:
    """Feed ``reqs`` to a ``Server`` at their arrival times (wall clock from
    the call) and tick until all are done. Latency = completion - arrival."""
    srv = Server(hbm_budget_bytes, max_blocks, slice_iters=slice_iters, backfill=backfill,
                 kernel=kernel)
    order = sorted(range(len(reqs)), key=lambda i: reqs[i].arrival_s)
    pending = deque(order)
    id2req: Dict[int, int] = {}
    done_t = [0.0] * len(reqs)
    losses = [0.0] * len(reqs)
    grads = [None] * len(reqs)
    ndone = 0
    t0 = time.perf_counter()
    while ndone < len(reqs):
        now = time.perf_counter() - t0
        while pending and reqs[pending[0]].arrival_s <= now:
            i = pending.popleft()
            r = reqs[i]
            id2req[srv.submit(r.alpha, r.q_xy, r.q_t, r.target, r.dt, r.h, r.rtol, r.max_iter)] = i
        na, nq, fin = srv.tick()
        tf = time.perf_counter() - t0
        for jid in fin:
            i = id2req[jid]
            loss, G, inf = srv.result(jid)
            if inf["state"] != _lib.NH_JOB_DONE:
                raise RuntimeError(f"job {i} failed (status {inf['status']})")
            done_t[i] = tf
            losses[i] = loss
            if keep_grads:
                grads[i] = G
            srv.release(jid)
            ndone += 1
            if log and ndone % 10 == 0:
                log(f"served {ndone}/{len(reqs)} jobs at {tf:.2f} s")
        if na == 0 and nq == 0 and pending:
            wait = reqs[pending[0]].arrival_s - (time.perf_counter() - t0)
            if wait > 0:
                time.sleep(wait)
    makespan = max(done_t) - min(r.arrival_s for r in reqs)
    st = srv.stats()
    srv.close()
    lat = [done_t[i] - reqs[i].arrival_s for i in range(len(reqs))]
    res = StreamResult(lat, makespan, losses, st["voxel_steps"], st["cg_iters"],
                       {"ticks": st["ticks"], "kernel_s": st["kernel_s"], "max_blocks": st["max_blocks"],
                        "workgroup_busy_frac": st["busy_block_s"] / max(st["span_block_s"], 1e-30)})
    res.grads = grads
    return res


def sequential_stream(reqs: Sequence[Request], keep_grads: bool = False, log=None) -> StreamResult:
    """Baseline: the same requests solved one at a time in arrival order with
    a single-problem ``Solver`` (all of the GPU per job), inputs uploaded and
    results downloaded per job as the server does."""
    solvers: Dict[tuple, Solver] = {}
    order = sorted(range(len(reqs)), key=lambda i: reqs[i].arrival_s)
    done_t = [0.0] * len(reqs)
    losses = [0.0] * len(reqs)
    grads = [None] * len(reqs)
    vs, iters = 0.0, 0
    dev = torch.device("cuda", torch.cuda.current_device())
    t0 = time.perf_counter()
    for i in order:
        r = reqs[i]
        wait = r.arrival_s - (time.perf_counter() - t0)
        if wait > 0:
            time.sleep(wait)
        nz, ny, nx = r.alpha.shape
        key = (nx, ny, nz, r.h)
        if key not in solvers:
            solvers[key] = Solver(nx, ny, nz, h=(r.h,) * 3, rtol=r.rtol, max_iter=r.max_iter)
        sv = solvers[key]
        a = torch.from_numpy(np.ascontiguousarray(r.alpha, dtype=np.float32)).to(dev)
        q = torch.from_numpy(np.ascontiguousarray(r.q_xy, dtype=np.float32)).to(dev)
        tg = torch.from_numpy(np.ascontiguousarray(r.target, dtype=np.float32)).to(dev)
        S = sv.forward(a, q, r.q_t, r.dt, len(r.q_t))
        d = S.double() - tg.double()
        m = d.numel()
        loss = float((d * d).sum() / m)
        g = (d * (2.0 / m)).float()
        G = sv.adjoint(g).cpu().numpy()
        done_t[i] = time.perf_counter() - t0
        losses[i] = loss
        if keep_grads:
            grads[i] = G
        st = sv.stats()
        vs += 2.0 * nx * ny * nz * len(r.q_t)
        iters += st["fwd_iters"] + st["adj_iters"]
        if log and (order.index(i) + 1) % 10 == 0:
            log(f"sequential {order.index(i) + 1}/{len(reqs)} jobs at {done_t[i]:.2f} s")
    makespan = max(done_t) - min(r.arrival_s for r in reqs)
    for sv in solvers.values():
        sv.close()
    lat = [done_t[i] - reqs[i].arrival_s for i in range(len(reqs))]
    res = StreamResult(lat, makespan, losses, vs, iters)
    res.grads = grads
    return res


def benchmark(n_jobs: int = 40, rate: float = 20.0, seed: int = 5, hbm_budget_bytes: float = 200e9,
              sequential: bool = True, log=None, slice_iters: int = 0,
              backfill: Optional[int] = None, kernel: str = "resident") -> dict:
    """Serve the first ``n_jobs`` of the Poisson stream of mixed grids, then
    (optionally) the same requests sequentially; returns both summaries and
    the speedup of the served stream (throughput and latency)."""
    from . import workloads as wl

    def say(*a):
        if log:
            log(" ".join(str(x) for x in a))

    t = time.perf_counter()
    specs = wl.serving_stream(n_jobs=n_jobs, rate=rate, seed=seed)
    targets = target_series(specs)
    reqs = requests_from_specs(specs, targets)
    torch.cuda.synchronize()
    say(f"serve: {n_jobs} jobs generated with targets in {time.perf_counter() - t:.1f} s")
    a = serve_stream(reqs, hbm_budget_bytes, log=log, slice_iters=slice_iters, backfill=backfill,
                     kernel=kernel)
    out = {"rate_jobs_per_s": rate, "seed": seed, "hbm_budget_gb": hbm_budget_bytes / 1e9, "kernel": kernel,
           "batched": a.summary()}
    say("serve: batched", out["batched"])
    if sequential:
        b = sequential_stream(reqs, log=log)
        out["sequential"] = b.summary()
        say("serve: sequential", out["sequential"])
        out["speedup_throughput"] = out["batched"]["jobs_per_s"] / out["sequential"]["jobs_per_s"]
        out["speedup_p50"] = out["sequential"]["p50_ms"] / out["batched"]["p50_ms"]
        out["speedup_p99"] = out["sequential"]["p99_ms"] / out["batched"]["p99_ms"]
        dl = max(abs(x - y) / abs(y) for x, y in zip(a.losses, b.losses))
        out["max_rel_loss_diff_vs_sequential"] = dl
    return out


def main(argv=None):
    import argparse
    import json
    import sys

    p = argparse.ArgumentParser(description="Serve a Poisson stream of mixed-grid inversion jobs on one GPU")
    p.add_argument("--jobs", type=int, default=40)
    p.add_argument("--rate", type=float, default=20.0)
    p.add_argument("--seed", type=int, default=5)
    p.add_argument("--budget-gb", type=float, default=200.0)
    p.add_argument("--no-sequential", action="store_true")
    p.add_argument("--slice", type=int, default=0, help="CG iterations per tick (0 = library default)")
    p.add_argument("--backfill", type=int, default=None, help="1 EASY backfilling (default), 0 strict order")
    p.add_argument("--kernel", default="resident", choices=["resident", "streaming"])
    args = p.parse_args(argv)
    res = benchmark(args.jobs, args.rate, args.seed, args.budget_gb * 1e9, not args.no_sequential,
                    log=lambda s: print(s, file=sys.stderr, flush=True), slice_iters=args.slice,
                    backfill=args.backfill, kernel=args.kernel)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
