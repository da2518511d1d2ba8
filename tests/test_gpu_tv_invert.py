"""The TV regulariser kernel (eq. tv_discrete) against the FP64 oracle,
through the C ABI.

Tolerances: FP64 path 1e-12 relative on the value and on the gradient (global
relative L2); FP32 path 1e-6 on the value and 1e-5 on the gradient (the
differences of FP32 inputs are formed in FP32).
"""
import numpy as np
import pytest
import torch

from oracle import tv as orc_tv
from paper_2603_11045_amd import _lib
from paper_2603_11045_amd import workloads as wl
from paper_2603_11045_amd.solver import Solver

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


def rel_l2(a, b):
    """Relative L2 distance; 0 when both are exactly zero (a one-cell grid has no gradient)."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    nb = np.linalg.norm(b)
    if nb == 0.0:
        return float(np.linalg.norm(a))
    return float(np.linalg.norm(a - b) / nb)


@pytest.fixture(scope="module", autouse=True)
def gpu():
    assert torch.cuda.is_available(), "GPU tests need a ROCm GPU"
    _lib.load()


def dev(a, dtype):
    return torch.from_numpy(np.ascontiguousarray(a)).to(device="cuda", dtype=dtype)


@pytest.mark.parametrize("shape", [(1, 1, 1), (1, 3, 2), (3, 5, 7), (16, 64, 64), (9, 33, 130), (64, 256, 256)])
@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_tv_matches_oracle(shape, precision):
    say("tv", shape, precision)
    nz, ny, nx = shape
    rng = np.random.default_rng(sum(shape))
    a = rng.uniform(0.003, 0.25, size=shape)
    # piecewise-constant regions, as the regulariser favours: exact zeros in the differences
    a[:, : ny // 2, : nx // 2] = 0.15
    h, eps, weight = (0.156, 0.156, 0.0625), 1e-6, 1e-3
    dt_t = torch.float32 if precision == "f32" else torch.float64
    a_in = a.astype(np.float32) if precision == "f32" else a
    s = Solver(nx, ny, nz, h=h, precision=precision)
    v, g = s.tv(dev(a_in, dt_t), eps=eps, weight=weight)
    v_o = weight * orc_tv.tv_value(a_in, h, eps)
    g_o = weight * orc_tv.tv_grad(a_in, h, eps)
    ev, eg = abs(v - v_o) / abs(v_o), rel_l2(g.cpu().numpy(), g_o)
    say("  value rel", ev, "grad rel", eg)
    tol_v, tol_g = (1e-12, 1e-12) if precision == "f64" else (1e-6, 1e-5)
    assert ev <= tol_v and eg <= tol_g
    # accumulate onto a given gradient; a second call reproduces the value bit for bit
    base = torch.full_like(g, 0.5)
    v2, g2 = s.tv(dev(a_in, dt_t), eps=eps, weight=weight, grad=base)
    assert v2 == v
    assert torch.equal(g2, g + 0.5)                     # the same FP64 addition, element by element


def test_tv_errors():
    s = Solver(4, 4, 3)
    a = torch.ones(48, device="cuda")
    with pytest.raises(_lib.NHError) as e:
        s.tv(a, eps=0.0)
    assert e.value.code == _lib.NH_EINVAL
    with pytest.raises(_lib.NHError) as e:
        s.tv(a, eps=1e-6, weight=float("nan"))
    assert e.value.code == _lib.NH_EINVAL


# ------------------------------------------------------------------ inversion driver
def test_objective_gradient_matches_oracle():
    """The driver's dJ/dalpha (data misfit through the adjoint plus lambda times
    the TV gradient) against the oracle's, on the paper-shaped specimen with
    K = 50 sweeps, 10 steps, at a field between the start and the truth."""
    from oracle import heat as orc
    from paper_2603_11045_amd.invert import objective_and_grad

    w = wl.paper_64x64x16(nsteps=10)
    say("objective", w.name)
    src = orc.source_series(w.q_xy, w.q_t)
    opt = dict(h=w.h, periodic=True, jacobi_k=w.jacobi_k)
    target_o, _, _ = orc.forward(w.alpha, src, w.dt, keep_states=False, **opt)
    a = (0.5 * (w.alpha.astype(np.float64) + np.median(w.alpha))).astype(np.float32)
    S_o, T_o, _ = orc.forward(a, src, w.dt, **opt)
    r = S_o - target_o
    G_o, _, _, _ = orc.adjoint(a, T_o, 2.0 * r, w.dt, **opt)
    G_o = G_o + 1e-3 * orc_tv.tv_grad(a, w.h, 1e-6)
    s = Solver(w.nx, w.ny, w.nz, h=w.h, periodic=True, jacobi_k=w.jacobi_k)
    target = dev(target_o, torch.float32)
    data, tv, G = objective_and_grad(s, dev(a, torch.float32), dev(w.q_xy, torch.float32), w, target, 1e-3, 1e-6)
    ed = abs(data - float(np.sum(r * r))) / float(np.sum(r * r))
    eg = rel_l2(G.cpu().numpy(), G_o)
    say("  data rel", ed, "grad rel", eg)
    assert ed <= 1e-4 and eg <= 1e-4


@pytest.mark.parametrize("method", ["grid", "nefty"])
def test_reconstruction_reduces_the_objective(method):
    """A short run of each driver lowers the objective and keeps alpha in bounds."""
    from paper_2603_11045_amd.invert import InvertConfig, reconstruct

    w = wl.paper_64x64x16(nsteps=20)
    say("reconstruct", method)
    s = Solver(w.nx, w.ny, w.nz, h=w.h, periodic=True, jacobi_k=w.jacobi_k)
    target = s.forward(dev(w.alpha, torch.float32), dev(w.q_xy, torch.float32), w.q_t, w.dt, w.nsteps).clone()
    s.close()
    cfg = InvertConfig(method=method, iters=30, lr=2e-3 if method == "grid" else 1e-4, width=128, depth=6,
                       skip_layer=3, fa_horizon=20)
    r = reconstruct(w, target, cfg, alpha_true=w.alpha, bulk_mean=float(np.median(w.alpha)),
                    log=lambda m: say("  " + m), log_every=1)
    losses = [h["loss"] for h in r.history]
    say("  loss first", losses[0], "last", losses[-1], "ms/iter", r.ms_per_iter, "metrics", r.metrics)
    assert np.isfinite(r.alpha).all()
    assert r.alpha.min() >= 0.003 - 1e-7 and r.alpha.max() <= 0.25 + 1e-7
    assert losses[-1] < 0.9 * losses[0]
