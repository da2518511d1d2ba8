"""Inversion drivers over the solver: the consumers of the library's dL/dalpha.

Two parameterisations of the diffusivity are optimised with Adam through the
same differentiable solver and adjoint (Sec. 4, App. D.1, App. F):

- ``grid``: a learnable voxel tensor started at the bulk mean (the Grid Opt.
  baseline); after every step it is clamped to [alpha_min, alpha_max] so the
  solver's positivity requirement holds.
- ``nefty``: the neural field. Coordinates normalised to [-1, 1]^3, Fourier
  positional encoding with N bands (eq. posenc_appdx) weighted by the cosine
  frequency-annealing schedule (eq. fa_schedule, beta rising linearly from 0
  to N over T_FA steps), a ReLU MLP with Xavier initialisation and one skip
  connection that re-injects the encoding, and the bounded output
  alpha = alpha_min + (alpha_max - alpha_min) * sigmoid(f).

Objective (eq. nefty_obj, discrete form): sum over frames of the squared
surface misfit plus lambda * R(alpha) with the TV regulariser of
eq. tv_discrete. Per iteration: one forward sweep and one adjoint sweep in the
library, the TV value and gradient in the library (added onto dL/dalpha), and,
for the neural field, PyTorch's backward from dL/dalpha to the network
weights (the chain rule of eq. grad_assembly through d alpha / d theta).

Metrics against the ground truth (App. F): MSE, PSNR with the bound range as
peak, and the volumetric IoU of the defect masks alpha < 0.03.
"""
from __future__ import annotations

import math
import time
from dataclasses import dataclass, field
from typing import Callable, Dict, List, Optional

import numpy as np
import torch

from .solver import Solver


@dataclass
class InvertConfig:
    method: str = "nefty"                   # "nefty" or "grid"
    iters: int = 200
    lr: float = 5e-5                        # Table 5 (both methods)
    lr_decay: float = 0.1                   # step decay gamma ...
    lr_decay_every: int = 1000              # ... every this many iterations
    tv_weight: float = 1e-3                 # lambda
    tv_eps: float = 1e-6
    alpha_bounds: tuple = (0.003, 0.25)
    bands: int = 12                         # N
    depth: int = 10                         # L_MLP
    width: int = 512                        # W_MLP
    skip_layer: int = 4
    fa_horizon: int = 2500                  # T_FA
    iou_threshold: float = 0.03
    seed: int = 0


def fa_weights(beta: float, bands: int) -> torch.Tensor:
    """Cosine annealing weight of each band k: (1 - cos(pi clamp(beta - k, 0, 1))) / 2."""
    k = torch.arange(bands, dtype=torch.float64)
    return 0.5 * (1.0 - torch.cos(math.pi * torch.clamp(beta - k, 0.0, 1.0)))


class NeuralField(torch.nn.Module):
    """Coordinate MLP with positional encoding and a bounded output."""

    def __init__(self, shape, cfg: InvertConfig):
        super().__init__()
        nz, ny, nx = shape
        self.shape = shape
        self.cfg = cfg
        # grid-node coordinates normalised to [-1, 1] per axis, order (x, y, z)
        axes = [torch.linspace(-1.0, 1.0, n) if n > 1 else torch.zeros(1) for n in (nx, ny, nz)]
        zz, yy, xx = torch.meshgrid(axes[2], axes[1], axes[0], indexing="ij")
        self.register_buffer("coords", torch.stack([xx, yy, zz], dim=-1).reshape(-1, 3))
        d_in = 2 * 3 * cfg.bands
        layers = []
        for i in range(cfg.depth - 1):
            fan_in = d_in if i == 0 else cfg.width + (d_in if i == cfg.skip_layer else 0)
            layers.append(torch.nn.Linear(fan_in, cfg.width))
        self.hidden = torch.nn.ModuleList(layers)
        self.out = torch.nn.Linear(cfg.width, 1)
        for m in list(self.hidden) + [self.out]:
            torch.nn.init.xavier_uniform_(m.weight)
            torch.nn.init.zeros_(m.bias)
        self.register_buffer("band_w", torch.ones(cfg.bands))

    def set_anneal(self, step: int):
        beta = self.cfg.bands * min(1.0, step / max(self.cfg.fa_horizon, 1))
        self.band_w.copy_(fa_weights(beta, self.cfg.bands).to(self.band_w))

    def encode(self) -> torch.Tensor:
        """gamma(x) = (sin(2^k pi x), cos(2^k pi x))_k per coordinate, each band scaled by its weight."""
        f = (2.0 ** torch.arange(self.cfg.bands, device=self.coords.device, dtype=self.coords.dtype)) * math.pi
        ang = self.coords[:, :, None] * f[None, None, :]                  # [n, 3, N]
        w = self.band_w[None, None, :]
        return torch.cat([torch.sin(ang) * w, torch.cos(ang) * w], dim=1).reshape(self.coords.shape[0], -1)

    def forward(self) -> torch.Tensor:
        g = self.encode()
        h = g
        for i, lin in enumerate(self.hidden):
            if i == self.cfg.skip_layer:
                h = torch.cat([h, g], dim=1)
            h = torch.relu(lin(h))
        f = self.out(h)[:, 0]
        lo, hi = self.cfg.alpha_bounds
        return (lo + (hi - lo) * torch.sigmoid(f)).reshape(self.shape)


def metrics(alpha_hat: np.ndarray, alpha_true: np.ndarray, bounds=(0.003, 0.25), tau: float = 0.03) -> Dict:
    """MSE, PSNR ((alpha_max - alpha_min)^2 / MSE) and the IoU of alpha < tau (App. F)."""
    a, t = np.asarray(alpha_hat, np.float64), np.asarray(alpha_true, np.float64)
    mse = float(np.mean((a - t) ** 2))
    psnr = 10.0 * math.log10((bounds[1] - bounds[0]) ** 2 / mse) if mse > 0 else float("inf")
    ma, mt = a < tau, t < tau
    union = int(np.logical_or(ma, mt).sum())
    iou = float(np.logical_and(ma, mt).sum() / union) if union else 1.0
    return {"mse": mse, "psnr": psnr, "iou": iou}


def objective_and_grad(s: Solver, alpha: torch.Tensor, q_xy: torch.Tensor, w, target: torch.Tensor,
                       tv_weight: float, tv_eps: float):
    """J = sum_n |S^n(alpha) - target^n|^2 + tv_weight * R(alpha) and dJ/dalpha
    (FP64): one forward and one adjoint sweep plus the TV kernel, which adds
    its gradient onto the adjoint's. Returns (data term, weighted TV, grad)."""
    S = s.forward(alpha, q_xy, w.q_t, w.dt, w.nsteps)
    r = S - target
    data = float((r.double() * r.double()).sum())
    G = s.adjoint((2.0 * r).contiguous())
    tv, G = s.tv(alpha, eps=tv_eps, weight=tv_weight, grad=G)
    return data, tv, G


@dataclass
class InvertResult:
    alpha: np.ndarray
    history: List[Dict] = field(default_factory=list)
    seconds: float = 0.0
    ms_per_iter: float = 0.0
    metrics: Optional[Dict] = None


def reconstruct(w, target: torch.Tensor, cfg: InvertConfig, alpha_true: Optional[np.ndarray] = None,
                bulk_mean: Optional[float] = None, log: Optional[Callable[[str], None]] = None,
                log_every: int = 50) -> InvertResult:
    """Recover alpha of workload ``w`` (grid, spacing, dt, source, closure,
    inner solver) from the surface series ``target`` ([nsteps][ny][nx] on the
    GPU, FP32)."""
    dev = target.device
    torch.manual_seed(cfg.seed)
    s = Solver(w.nx, w.ny, w.nz, h=w.h, rtol=w.rtol, max_iter=5000, periodic=w.periodic, robin=w.robin,
               jacobi_k=w.jacobi_k, device=dev.index)
    q_xy = torch.from_numpy(np.ascontiguousarray(w.q_xy, dtype=np.float32)).to(dev)
    if cfg.method == "grid":
        init = float(bulk_mean if bulk_mean is not None else np.mean(w.alpha))
        param = torch.full((w.nz, w.ny, w.nx), init, dtype=torch.float32, device=dev, requires_grad=True)
        params = [param]
        field_fn = lambda: param  # noqa: E731
        net = None
    elif cfg.method == "nefty":
        net = NeuralField((w.nz, w.ny, w.nx), cfg).to(dev)
        params = list(net.parameters())
        field_fn = net
    else:
        raise ValueError("method must be 'grid' or 'nefty'")
    opt = torch.optim.Adam(params, lr=cfg.lr)
    sched = torch.optim.lr_scheduler.StepLR(opt, step_size=cfg.lr_decay_every, gamma=cfg.lr_decay)
    res = InvertResult(alpha=None)
    torch.cuda.synchronize(dev)
    t0 = time.perf_counter()
    for it in range(cfg.iters):
        if net is not None:
            net.set_anneal(it)
        opt.zero_grad(set_to_none=True)
        alpha = field_fn()
        a32 = alpha.detach().contiguous()
        data, tv, G = objective_and_grad(s, a32, q_xy, w, target, cfg.tv_weight, cfg.tv_eps)
        alpha.backward(G.to(alpha.dtype))
        opt.step()
        sched.step()
        if cfg.method == "grid":
            with torch.no_grad():
                param.clamp_(*cfg.alpha_bounds)
        if log and (it % log_every == 0 or it == cfg.iters - 1):
            rec = {"iter": it, "data": data, "tv": tv, "loss": data + tv}
            if alpha_true is not None:
                rec.update(metrics(a32.cpu().numpy(), alpha_true, cfg.alpha_bounds, cfg.iou_threshold))
            res.history.append(rec)
            log(" ".join(f"{k} {v:.4g}" if isinstance(v, float) else f"{k} {v}" for k, v in rec.items()))
    torch.cuda.synchronize(dev)
    res.seconds = time.perf_counter() - t0
    res.ms_per_iter = res.seconds / max(cfg.iters, 1) * 1e3
    with torch.no_grad():
        res.alpha = field_fn().detach().float().cpu().numpy()
    if alpha_true is not None:
        res.metrics = metrics(res.alpha, alpha_true, cfg.alpha_bounds, cfg.iou_threshold)
    s.close()
    return res


def main(argv=None):
    import argparse
    import json

    from . import workloads as wl

    ap = argparse.ArgumentParser(description="reconstruct alpha of a paper-shaped specimen")
    ap.add_argument("--method", default="nefty", choices=["nefty", "grid"])
    ap.add_argument("--iters", type=int, default=200)
    ap.add_argument("--nsteps", type=int, default=100)
    ap.add_argument("--lr", type=float, default=None)
    ap.add_argument("--layered", action="store_true")
    ap.add_argument("--seed", type=int, default=6)
    ap.add_argument("--log-every", type=int, default=100)
    a = ap.parse_args(argv)
    w = wl.paper_64x64x16(seed=a.seed, nsteps=a.nsteps, layered=a.layered)
    dev = torch.device("cuda", 0)
    # synthetic measurement: the surface series of the ground truth
    s = Solver(w.nx, w.ny, w.nz, h=w.h, periodic=True, jacobi_k=w.jacobi_k)
    target = s.forward(torch.from_numpy(w.alpha).to(dev), torch.from_numpy(w.q_xy).to(dev), w.q_t, w.dt,
                       w.nsteps).clone()
    s.close()
    cfg = InvertConfig(method=a.method, iters=a.iters)
    if a.lr is not None:
        cfg.lr = a.lr
    bulk = float(np.median(w.alpha))
    r = reconstruct(w, target, cfg, alpha_true=w.alpha, bulk_mean=bulk, log=lambda m: print(m, flush=True),
                    log_every=a.log_every)
    print(json.dumps({"method": a.method, "iters": a.iters, "ms_per_iter": r.ms_per_iter, "metrics": r.metrics}))


if __name__ == "__main__":
    main()
