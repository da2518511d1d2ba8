"""Parity of the HIP path (through the C ABI) against the FP64 oracle.

Norms (global relative L2 over the whole array) and tolerances: surface
temperature 1e-5 and dL/dalpha 1e-4 for the FP32-vector path; the FP64 path
is held to 1e-9 / 1e-8. The oracle solves every step to 1e-13, the GPU to the
workload's own tolerance, so the CG tolerance (not FP32 rounding) sets the
FP32 gap.
"""
import numpy as np
import pytest
import torch

from oracle import heat as orc
from paper_2603_11045_amd import _lib
from paper_2603_11045_amd import workloads as wl
from paper_2603_11045_amd.solver import HeatSolve, Solver

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


def rel_l2(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.fixture(scope="session", autouse=True)
def gpu():
    assert torch.cuda.is_available(), "GPU tests need a ROCm GPU"
    _lib.load()
    return torch.device("cuda", 0)


def to_dev(a, dtype):
    return torch.from_numpy(np.ascontiguousarray(a)).to(device="cuda", dtype=dtype)


def run_gpu(w, rtol=None, checkpoint_every=0, team=0, tile_z=0, gs=None, precision=None, variant=2,
            guess="adaptive", cheb=1):
    """Forward (and adjoint when gs is given) of workload w on the GPU."""
    prec = precision or w.precision
    dt_t = torch.float32 if prec == "f32" else torch.float64
    s = Solver(w.nx, w.ny, w.nz, h=w.h, rtol=rtol or w.rtol, max_iter=5000,
               checkpoint_every=checkpoint_every, precision=prec, team_blocks_max=team, tile_z=tile_z,
               cg_variant=variant, initial_guess=guess, preconditioner_degree=cheb)
    S = s.forward(to_dev(w.alpha, dt_t), to_dev(w.q_xy, dt_t), w.q_t, w.dt, w.nsteps)
    out = dict(S=S.cpu().numpy().astype(np.float64), stats_fwd=s.stats(), solver=s)
    if gs is not None:
        G = s.adjoint(to_dev(gs, dt_t))
        out["G"] = G.cpu().numpy()
        out["stats_adj"] = s.stats()
    return out


# ------------------------------------------------------------------ operator
@pytest.mark.parametrize("shape", [(3, 5, 7), (9, 33, 65), (11, 17, 130), (8, 16, 16), (32, 64, 64),
                                   (1, 1, 1), (5, 1, 70)])
def test_apply_A_matches_oracle(shape):
    nz, ny, nx = shape
    say("apply_A", shape)
    rng = np.random.default_rng(sum(shape))
    alpha = np.exp(0.7 * rng.standard_normal(shape)).astype(np.float32)
    x = rng.uniform(-1, 1, size=shape).astype(np.float32)
    dt = 1.7
    s = Solver(nx, ny, nz, h=(1.0, 0.8, 1.3))
    y = s.apply_A(to_dev(alpha, torch.float32), to_dev(x, torch.float32), dt).cpu().numpy()
    ref = orc.apply_A(alpha, x, dt, h=(1.0, 0.8, 1.3))
    scale = np.abs(x).max() * (1 + 12 * dt * alpha.max())
    assert np.abs(y - ref).max() <= 4e-6 * scale
    if shape != (1, 1, 1):
        assert rel_l2(y, ref) <= 1e-6


# ------------------------------------------------------------------ small problems
SMALL = [
    # (nx, ny, nz, nsteps, seed, team, tile_z)
    (7, 5, 3, 6, 1, 0, 0),
    (37, 21, 13, 5, 2, 3, 4),
    (70, 40, 9, 4, 3, 5, 3),
    (33, 17, 6, 7, 4, 8, 2),
    (16, 16, 8, 5, 5, 0, 0),
    (130, 9, 5, 3, 6, 0, 1),
    # shapes that the register-resident kernel takes (variant 2): ragged z tiles,
    # a single tile, many tiles
    (70, 40, 9, 4, 7, 0, 0),
    (100, 20, 40, 3, 8, 0, 0),
    (64, 8, 20, 4, 9, 0, 0),
    (65, 17, 33, 3, 10, 0, 0),
]


@pytest.mark.parametrize("case", SMALL, ids=[f"{c[0]}x{c[1]}x{c[2]}_t{c[5]}_z{c[6]}" for c in SMALL])
@pytest.mark.parametrize("precision", ["f64", "f32"])
@pytest.mark.parametrize("variant", [2, 1, 0])
def test_small_forward_adjoint(case, precision, variant):
    nx, ny, nz, nsteps, seed, team, tz = case
    say("small", case, precision, "variant", variant)
    w = wl.small_problem(nx, ny, nz, nsteps, seed=seed, dt=2.5, precision=precision,
                         rtol=1e-12 if precision == "f64" else 1e-7)
    gs = wl.random_surface_weights(nsteps, ny, nx, seed=100 + seed)
    src = orc.source_series(w.q_xy, w.q_t)
    S_o, T_o, _ = orc.forward(w.alpha, src, w.dt)
    G_o, _, _, _ = orc.adjoint(w.alpha, T_o, gs, w.dt)
    out = run_gpu(w, team=team, tile_z=tz, gs=gs, variant=variant)
    tol_s, tol_g = (1e-9, 1e-8) if precision == "f64" else (1e-5, 1e-4)
    es, eg = rel_l2(out["S"], S_o), rel_l2(out["G"], G_o)
    say("  rel-L2 S", es, "G", eg, "team", out["stats_fwd"]["team_blocks"], "block",
        out["stats_fwd"]["block_threads"])
    assert es <= tol_s and eg <= tol_g


@pytest.mark.parametrize("case", SMALL, ids=[f"{c[0]}x{c[1]}x{c[2]}_t{c[5]}_z{c[6]}" for c in SMALL])
@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_small_projected_adjoint(case, precision):
    """The projected initial guess of the adjoint solves (guess mode 3) on the
    same cases, resident and streaming kernels, FP32 and FP64."""
    nx, ny, nz, nsteps, seed, team, tz = case
    say("small projected", case, precision)
    w = wl.small_problem(nx, ny, nz, nsteps, seed=seed, dt=2.5, precision=precision,
                         rtol=1e-12 if precision == "f64" else 1e-7)
    gs = wl.random_surface_weights(nsteps, ny, nx, seed=100 + seed)
    src = orc.source_series(w.q_xy, w.q_t)
    S_o, T_o, _ = orc.forward(w.alpha, src, w.dt)
    G_o, _, _, _ = orc.adjoint(w.alpha, T_o, gs, w.dt)
    out = run_gpu(w, team=team, tile_z=tz, gs=gs, guess="projection")
    tol_s, tol_g = (1e-9, 1e-8) if precision == "f64" else (1e-5, 1e-4)
    es, eg = rel_l2(out["S"], S_o), rel_l2(out["G"], G_o)
    say("  rel-L2 S", es, "G", eg, "adjoint iterations", out["stats_adj"]["adj_iters"])
    assert es <= tol_s and eg <= tol_g


@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_projected_adjoint_degenerate_sources(precision):
    """Projected guesses with degenerate windows: a zero adjoint source (every
    window vector is zero and is dropped, the gradient is exactly zero) and a
    source on one step only (the window then holds one decaying direction)."""
    nx, ny, nz, nsteps = 40, 24, 10, 9
    w = wl.small_problem(nx, ny, nz, nsteps, seed=31, dt=2.0, precision=precision,
                         rtol=1e-12 if precision == "f64" else 1e-7)
    out = run_gpu(w, gs=np.zeros((nsteps, ny, nx)), guess="projection")
    assert not np.any(out["G"])
    gs = np.zeros((nsteps, ny, nx))
    gs[nsteps - 1] = wl.random_surface_weights(1, ny, nx, seed=32)[0]
    src = orc.source_series(w.q_xy, w.q_t)
    S_o, T_o, _ = orc.forward(w.alpha, src, w.dt)
    G_o, _, _, _ = orc.adjoint(w.alpha, T_o, gs, w.dt)
    out = run_gpu(w, gs=gs, guess="projection")
    eg = rel_l2(out["G"], G_o)
    say("one-step source: rel-L2 G", eg, "adjoint iterations", out["stats_adj"]["adj_iters"])
    assert eg <= (1e-8 if precision == "f64" else 1e-4)


CHEB_CASES = [SMALL[1], SMALL[2], SMALL[5], SMALL[7], SMALL[9]]


@pytest.mark.parametrize("case", CHEB_CASES, ids=[f"{c[0]}x{c[1]}x{c[2]}_t{c[5]}_z{c[6]}" for c in CHEB_CASES])
@pytest.mark.parametrize("precision", ["f64", "f32"])
@pytest.mark.parametrize("degree", [2, 4, 7, 16])
def test_chebyshev_preconditioner_matches_oracle(case, precision, degree):
    """CG with the Chebyshev polynomial preconditioner reaches the oracle's
    fixed point (same tolerances as Jacobi-PCG)."""
    nx, ny, nz, nsteps, seed, team, tz = case
    say("chebyshev", degree, case, precision)
    w = wl.small_problem(nx, ny, nz, nsteps, seed=seed, dt=2.5, precision=precision,
                         rtol=1e-12 if precision == "f64" else 1e-7)
    gs = wl.random_surface_weights(nsteps, ny, nx, seed=100 + seed)
    src = orc.source_series(w.q_xy, w.q_t)
    S_o, T_o, _ = orc.forward(w.alpha, src, w.dt)
    G_o, _, _, _ = orc.adjoint(w.alpha, T_o, gs, w.dt)
    out = run_gpu(w, team=team, tile_z=tz, gs=gs, variant=0, cheb=degree)
    assert out["solver"].cg_variant == 0 and out["solver"].preconditioner_degree == degree
    tol_s, tol_g = (1e-9, 1e-8) if precision == "f64" else (1e-5, 1e-4)
    es, eg = rel_l2(out["S"], S_o), rel_l2(out["G"], G_o)
    say("  rel-L2 S", es, "G", eg, "iterations", out["stats_fwd"]["fwd_iters"], out["stats_adj"]["adj_iters"])
    assert es <= tol_s and eg <= tol_g


def test_chebyshev_preconditioner_cuts_iterations_at_high_contrast():
    """A 1:1000 inclusion: the degree-4 polynomial needs well under half the
    Jacobi-PCG iterations, and its result agrees with the oracle."""
    nx, ny, nz, nsteps = 48, 40, 16, 6
    w = wl.small_problem(nx, ny, nz, nsteps, seed=41, dt=4.0, precision="f64", rtol=1e-12)
    w.alpha[4:12, 10:30, 12:36] *= 1000.0
    gs = wl.random_surface_weights(nsteps, ny, nx, seed=42)
    src = orc.source_series(w.q_xy, w.q_t)
    S_o, T_o, _ = orc.forward(w.alpha, src, w.dt)
    G_o, _, _, _ = orc.adjoint(w.alpha, T_o, gs, w.dt)
    its = {}
    for degree in (1, 4):
        out = run_gpu(w, gs=gs, variant=0, cheb=degree)
        its[degree] = out["stats_fwd"]["fwd_iters"] + out["stats_adj"]["adj_iters"]
        es, eg = rel_l2(out["S"], S_o), rel_l2(out["G"], G_o)
        say("  degree", degree, "iterations", its[degree], "rel-L2 S", es, "G", eg)
        assert es <= 1e-6 and eg <= 1e-5
    assert its[4] < 0.5 * its[1]


@pytest.mark.parametrize("degree", [3, 6])
def test_chebyshev_checkpointing_is_bitwise(degree):
    w = wl.small_problem(40, 24, 10, 12, seed=9, dt=3.0, precision="f32", rtol=1e-6)
    gs = wl.random_surface_weights(12, 24, 40, seed=19).astype(np.float32)
    full = run_gpu(w, gs=gs, variant=0, cheb=degree)
    ck = run_gpu(w, gs=gs, checkpoint_every=5, variant=0, cheb=degree)
    assert np.array_equal(ck["S"], full["S"]) and np.array_equal(ck["G"], full["G"])


def test_preconditioner_settings():
    s = Solver(8, 8, 4)
    assert s.cg_variant == 2 and s.preconditioner_degree == 1
    s.set_preconditioner(5)
    assert s.cg_variant == 0
    s.set_cg_variant(1)
    assert s.preconditioner_degree == 1
    for bad in (0, 17):
        with pytest.raises(Exception):
            s.set_preconditioner(bad)


def test_plain_fp64_16x16x8():
    """16x16x8, 50 steps, dt=2, FP64 at rtol 1e-12, MSE against the alpha=0.2 target."""
    w = wl.plain_fp64_16x16x8()
    say("plain fp64", w.name)
    ref = orc.run_workload(w)
    out = run_gpu(w, gs=ref["gs"])
    es, eg = rel_l2(out["S"], ref["S"]), rel_l2(out["G"], ref["G"])
    say("  rel-L2 S", es, "G", eg, "iters", out["stats_fwd"]["fwd_iters"], out["stats_adj"]["adj_iters"])
    assert es <= 1e-10
    assert eg <= 1e-9


# ------------------------------------------------------------------ 64x64x32 mixed precision
@pytest.fixture(scope="module")
def mixed_ref():
    w = wl.mixed_64x64x32()
    say("oracle for", w.name)
    return w, orc.run_workload(w)


@pytest.mark.timeout(600)
@pytest.mark.parametrize("variant", [2, 1, 0])
def test_mixed_64x64x32_forward_and_adjoint(mixed_ref, variant):
    w, ref = mixed_ref
    say("gpu", w.name, "variant", variant)
    out = run_gpu(w, gs=ref["gs"].astype(np.float32), variant=variant)
    es, eg = rel_l2(out["S"], ref["S"]), rel_l2(out["G"], ref["G"])
    mx = float(np.abs(out["G"] - ref["G"]).max() / np.abs(ref["G"]).max())
    say("  rel-L2 S", es, "G", eg, "max|dG|/max|G|", mx, "iters", out["stats_fwd"]["fwd_iters"],
        out["stats_adj"]["adj_iters"], "resident", out["stats_fwd"]["resident"])
    assert es <= 1e-5
    assert eg <= 1e-4


@pytest.mark.timeout(600)
def test_initial_guess_modes(mixed_ref):
    """Every CG starting point reaches the tolerance; the extrapolated one in
    fewer iterations on this smooth trajectory, the adaptive choice too."""
    w, ref = mixed_ref
    its = {}
    for guess in ("previous", "extrapolate", "adaptive", "projection"):
        out = run_gpu(w, gs=ref["gs"].astype(np.float32), guess=guess)
        es, eg = rel_l2(out["S"], ref["S"]), rel_l2(out["G"], ref["G"])
        its[guess] = (out["stats_fwd"]["fwd_iters"], out["stats_adj"]["adj_iters"])
        say("  guess", guess, "rel-L2 S", es, "G", eg, "iters", its[guess])
        assert es <= 1e-5
        assert eg <= 1e-4
    assert its["extrapolate"][0] < its["previous"][0]
    assert its["extrapolate"][1] < its["previous"][1]
    assert sum(its["adaptive"]) < sum(its["previous"])
    # the projection leaves the forward as it is and shortens the adjoint
    assert its["projection"][0] == its["adaptive"][0]
    assert its["projection"][1] < its["adaptive"][1]


# ------------------------------------------------------------------ checkpointing, determinism
@pytest.mark.parametrize("variant,guess", [(2, "adaptive"), (1, "adaptive"), (0, "adaptive"),
                                           (2, "projection"), (1, "projection")])
def test_checkpoint_recompute_is_bitwise(variant, guess):
    w = wl.small_problem(40, 24, 10, 20, seed=9, dt=3.0, precision="f32", rtol=1e-6)
    gs = wl.random_surface_weights(20, 24, 40, seed=19).astype(np.float32)
    say("checkpoint full", variant, guess)
    team, tz = (0, 0) if variant == 2 else (4, 3)
    full = run_gpu(w, gs=gs, team=team, tile_z=tz, variant=variant, guess=guess)
    for k in (1, 2, 3, 7, 64):
        say("checkpoint k", k)
        ck = run_gpu(w, gs=gs, checkpoint_every=k, team=team, tile_z=tz, variant=variant, guess=guess)
        assert np.array_equal(ck["S"], full["S"])
        assert np.array_equal(ck["G"], full["G"])
        if k < 20:
            assert ck["stats_adj"]["recompute_iters"] == full["stats_fwd"]["fwd_iters"]


def test_step_iters_add_up_to_the_stats():
    w = wl.small_problem(40, 24, 10, 12, seed=9, dt=3.0, precision="f32", rtol=1e-6)
    gs = wl.random_surface_weights(12, 24, 40, seed=19).astype(np.float32)
    out = run_gpu(w, gs=gs, checkpoint_every=5)
    s = out["solver"]
    fi, ai, ri = s.step_iters("forward"), s.step_iters("adjoint"), s.step_iters("recompute")
    assert fi.shape == (12,) and (fi > 0).all() and (ai > 0).all()
    assert fi.sum() == out["stats_fwd"]["fwd_iters"]
    assert ai.sum() == out["stats_adj"]["adj_iters"]
    assert ri.sum() == out["stats_adj"]["recompute_iters"]
    # recomputation repeats the forward step for step
    assert np.array_equal(ri, fi)


def test_runs_are_bitwise_deterministic():
    w = wl.small_problem(64, 40, 12, 6, seed=11, dt=4.0, precision="f32", rtol=1e-6)
    gs = wl.random_surface_weights(6, 40, 64, seed=21).astype(np.float32)
    a = run_gpu(w, gs=gs, team=6, tile_z=4)
    b = run_gpu(w, gs=gs, team=6, tile_z=4)
    assert np.array_equal(a["S"], b["S"]) and np.array_equal(a["G"], b["G"])


@pytest.mark.parametrize("guess", ["adaptive", "projection", "extrapolate"])
def test_resident_and_streaming_kernels_agree_bitwise(guess):
    """Both FP32 kernels of the single-reduction iteration build the operator
    from the same staged 1/alpha with every rounding of the face weights, the
    diagonal and A v written out (no contraction left to the compiler), and
    cast the FP64 scalars to FP32: on the same problem, tiled differently, they
    give identical surface frames, gradient and iteration counts."""
    w = wl.small_problem(96, 24, 40, 6, seed=23, dt=4.0, precision="f32", rtol=1e-6)
    gs = wl.random_surface_weights(6, 24, 96, seed=24).astype(np.float32)
    res = run_gpu(w, gs=gs, guess=guess)
    stm = run_gpu(w, gs=gs, tile_z=40, guess=guess)   # columns longer than a resident tile holds
    assert res["stats_fwd"]["resident"] == 1 and stm["stats_fwd"]["resident"] == 0
    say("resident vs streaming: S", rel_l2(res["S"], stm["S"]), "G", rel_l2(res["G"], stm["G"]),
        "iters", res["stats_fwd"]["fwd_iters"], res["stats_adj"]["adj_iters"],
        stm["stats_fwd"]["fwd_iters"], stm["stats_adj"]["adj_iters"])
    assert np.array_equal(res["S"], stm["S"])
    assert np.array_equal(res["G"], stm["G"])
    assert res["stats_fwd"]["fwd_iters"] == stm["stats_fwd"]["fwd_iters"]
    assert res["stats_adj"]["adj_iters"] == stm["stats_adj"]["adj_iters"]


def test_get_state_conserves_heat():
    """Zero flux: total heat after step n is dt * sum of the injected source."""
    w = wl.small_problem(48, 30, 10, 5, seed=12, dt=2.0, precision="f64", rtol=1e-12)
    out = run_gpu(w)
    s = out["solver"]
    injected = np.cumsum(w.dt * w.q_t * w.q_xy.sum())
    for n in range(1, 6):
        T = s.get_state(n).cpu().numpy()
        assert abs(T.sum() - injected[n - 1]) <= 1e-10 * injected[n - 1]


# ------------------------------------------------------------------ autograd
def test_heat_solve_autograd_matches_adjoint_and_gradcheck():
    nx, ny, nz, nsteps = 5, 4, 3, 4
    w = wl.small_problem(nx, ny, nz, nsteps, seed=13, dt=1.5, precision="f64", rtol=1e-13)
    s = Solver(nx, ny, nz, rtol=1e-13, max_iter=2000, precision="f64")
    q = to_dev(w.q_xy, torch.float64)
    a = to_dev(w.alpha, torch.float64).requires_grad_(True)
    T = HeatSolve.apply(a, s, q, w.q_t, w.dt, nsteps)
    gs = torch.from_numpy(wl.random_surface_weights(nsteps, ny, nx, seed=31)).cuda()
    (T * gs).sum().backward()
    src = orc.source_series(w.q_xy, w.q_t)
    _, T_o, _ = orc.forward(w.alpha, src, w.dt)
    G_o, _, _, _ = orc.adjoint(w.alpha, T_o, gs.cpu().numpy(), w.dt)
    assert rel_l2(a.grad.cpu().numpy(), G_o) <= 1e-9
    f = lambda al: HeatSolve.apply(al, s, q, w.q_t, w.dt, nsteps)  # noqa: E731
    assert torch.autograd.gradcheck(f, (a.detach().clone().requires_grad_(True),), eps=1e-6,
                                    atol=1e-7, rtol=1e-5)


# ------------------------------------------------------------------ source and initial-state VJPs
VJP_CASES = [((20, 12, 6), 7, "f64"), ((20, 12, 6), 7, "f32"), ((70, 40, 9), 5, "f32"), ((64, 8, 20), 6, "f32")]


@pytest.mark.parametrize("shape,nsteps,precision", VJP_CASES)
def test_adjoint_vjp_source_and_initial_state(shape, nsteps, precision):
    """dL/dq^n = dt mu^n on the top plane and dL/dT0 = mu^1 (App. D.3) against
    the oracle's adjoint; with checkpointing they are bit for bit the same."""
    nx, ny, nz = shape
    w = wl.small_problem(nx, ny, nz, nsteps, seed=17, dt=2.0, precision=precision, pulse_steps=2,
                         rtol=1e-13 if precision == "f64" else 1e-7)
    gs = wl.random_surface_weights(nsteps, ny, nx, seed=23)
    src = orc.source_series(w.q_xy, w.q_t)
    _, T_o, _ = orc.forward(w.alpha, src, w.dt, rtol=1e-13)
    G_o, dq_o, mu1_o, _ = orc.adjoint(w.alpha, T_o, gs, w.dt, rtol=1e-13)
    dt_t = torch.float32 if precision == "f32" else torch.float64
    outs = []
    for k in (0, 3):
        s = Solver(nx, ny, nz, rtol=w.rtol, max_iter=5000, checkpoint_every=k, precision=precision)
        s.forward(to_dev(w.alpha, dt_t), to_dev(w.q_xy, dt_t), w.q_t, w.dt, nsteps)
        G, dq, dT0 = s.adjoint_vjp(to_dev(gs, dt_t))
        outs.append((G.cpu().numpy(), dq.cpu().numpy(), dT0.cpu().numpy(), s.stats()["resident"]))
    G, dq, dT0, res = outs[0]
    e = (rel_l2(G, G_o), rel_l2(dq, dq_o), rel_l2(dT0, mu1_o))
    say(shape, precision, "resident", res, "rel-L2 G, dq, dT0:", e)
    tol = (1e-8, 1e-9, 1e-9) if precision == "f64" else (1e-4, 1e-5, 1e-5)
    assert all(x <= t for x, t in zip(e, tol))
    for a, b in zip(outs[0][:3], outs[1][:3]):
        assert np.array_equal(a, b)
    # the plain adjoint gives the same dL/dalpha
    s = Solver(nx, ny, nz, rtol=w.rtol, max_iter=5000, precision=precision)
    s.forward(to_dev(w.alpha, dt_t), to_dev(w.q_xy, dt_t), w.q_t, w.dt, nsteps)
    assert np.array_equal(s.adjoint(to_dev(gs, dt_t)).cpu().numpy(), G)


def test_heat_solve_source_gradients():
    """Autograd through HeatSolve for the source map and schedule: against
    the chain rule through the oracle's dL/dq^n, and gradcheck."""
    nx, ny, nz, nsteps = 5, 4, 3, 4
    w = wl.small_problem(nx, ny, nz, nsteps, seed=13, dt=1.5, precision="f64", rtol=1e-13)
    s = Solver(nx, ny, nz, rtol=1e-13, max_iter=2000, precision="f64")
    a = to_dev(w.alpha, torch.float64)
    q = to_dev(w.q_xy, torch.float64).requires_grad_(True)
    qt = torch.tensor(w.q_t, dtype=torch.float64, requires_grad=True)
    T = HeatSolve.apply(a, s, q, qt, w.dt, nsteps)
    gs = torch.from_numpy(wl.random_surface_weights(nsteps, ny, nx, seed=31)).cuda()
    (T * gs).sum().backward()
    src = orc.source_series(w.q_xy, w.q_t)
    _, T_o, _ = orc.forward(w.alpha, src, w.dt)
    _, dq_o, _, _ = orc.adjoint(w.alpha, T_o, gs.cpu().numpy(), w.dt)
    gq_o = np.einsum("n,nij->ij", np.asarray(w.q_t), dq_o)
    gqt_o = np.einsum("nij,ij->n", dq_o, np.asarray(w.q_xy))
    assert rel_l2(q.grad.cpu().numpy(), gq_o) <= 1e-9
    assert rel_l2(qt.grad.numpy(), gqt_o) <= 1e-9
    f = lambda qq, tt: HeatSolve.apply(a, s, qq, tt, w.dt, nsteps)  # noqa: E731
    assert torch.autograd.gradcheck(f, (q.detach().clone().requires_grad_(True),
                                        qt.detach().clone().requires_grad_(True)),
                                    eps=1e-6, atol=1e-7, rtol=1e-5)


# ------------------------------------------------------------------ error paths
def test_error_paths():
    nx, ny, nz = 8, 6, 4
    s = Solver(nx, ny, nz)
    q = torch.ones((ny, nx), device="cuda")
    g = torch.ones((3, ny, nx), device="cuda")
    with pytest.raises(_lib.NHError) as e:
        s.nsteps = 3
        s.adjoint(g)
    assert e.value.code == _lib.NH_ESTATE
    bad = torch.ones((nz, ny, nx), device="cuda")
    bad[1, 2, 3] = 0.0
    with pytest.raises(_lib.NHError) as e:
        s.forward(bad, q, [1.0, 0, 0], 1.0, 3)
    assert e.value.code == _lib.NH_EINVAL
    bad[1, 2, 3] = float("nan")
    with pytest.raises(_lib.NHError) as e:
        s.forward(bad, q, [1.0, 0, 0], 1.0, 3)
    assert e.value.code == _lib.NH_EINVAL
    good = torch.ones((nz, ny, nx), device="cuda")
    with pytest.raises(_lib.NHError) as e:
        s.forward(good, q, [1.0, 0, 0], -1.0, 3)
    assert e.value.code == _lib.NH_EINVAL
    s.set_solver(1e-10, 1, 0)
    T = s.forward(good, q, [1.0, 0, 0], 5.0, 3, allow_noconv=True)
    assert s.last_status == _lib.NH_ENOCONV and torch.isfinite(T).all()
    # a zero time limit on the team barrier makes the kernel leave early; the context recovers
    s2 = Solver(64, 32, 16, rtol=1e-6, team_blocks_max=8, tile_z=2)
    s2.set_barrier_timeout(0.0)
    a2 = torch.ones((16, 32, 64), device="cuda")
    q2 = torch.ones((32, 64), device="cuda")
    with pytest.raises(_lib.NHError) as e:
        s2.forward(a2, q2, [1.0, 0.0], 1.0, 2)
    assert e.value.code == _lib.NH_ETIMEOUT
    s2.set_barrier_timeout(20.0)
    T2 = s2.forward(a2, q2, [1.0, 0.0], 1.0, 2)
    assert torch.isfinite(T2).all()


# ------------------------------------------------------------------ measurement probe
def test_stream_probe_outputs():
    """nh_stream_probe_f32 (the streaming sweep's access pattern, used to measure
    what that traffic reaches): every output element against numpy, on a grid of
    several 64x16-column tiles and five planes."""
    import ctypes

    from paper_2603_11045_amd import _lib
    nx, ny, nz = 128, 48, 5
    rng = np.random.default_rng(41)
    host = [rng.standard_normal((nz, ny, nx)).astype(np.float32) for _ in range(6)]
    ins_t = [torch.from_numpy(h).cuda() for h in host]
    outs_t = [torch.zeros((nz, ny, nx), dtype=torch.float32, device="cuda") for _ in range(5)]
    vp = ctypes.c_void_p
    ins = (vp * 6)(*[t.data_ptr() for t in ins_t])
    outs = (vp * 5)(*[t.data_ptr() for t in outs_t])
    lib = _lib.load()
    assert lib.nh_stream_probe_f32(ins, outs, nx, ny, nz, vp(torch.cuda.current_stream().cuda_stream)) == 0
    torch.cuda.synchronize()
    got = [t.cpu().numpy() for t in outs_t]
    for k in range(4):
        assert np.array_equal(got[k], host[k] + host[k + 1]), k
    left = np.zeros_like(host[0])
    left[:, :, 1:] = host[0][:, :, :-1]
    left[:, :, 64::64] = 0.0                 # the neighbour lies within the 64-cell row of a tile
    assert np.array_equal(got[4], (host[4] + host[5]) + left)
