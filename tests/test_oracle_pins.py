"""Pins of the FP64 oracle against facts that do not come from the oracle itself.

Each test names the passage of the paper (or the piece of mathematics) it
rests on. Together they are chosen so that a plausible slip in the oracle
(arithmetic instead of harmonic mean, a dropped dt or spacing, the wrong
observed plane, a sign error in the gradient, a transposed axis) fails at
least one of them. None of these tests needs a GPU.
"""
import json
import os

import numpy as np
import pytest
import scipy.fft
import scipy.linalg

from oracle import dense_ref
from oracle import heat as orc
from paper_2603_11045_amd import workloads as wl

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _rand_problem(shape, nsteps, seed, sigma=0.6):
    rng = np.random.default_rng(seed)
    nz, ny, nx = shape
    alpha = np.exp(sigma * rng.standard_normal(shape))
    src = rng.uniform(0.0, 5.0, size=(nsteps, ny, nx))
    gs = rng.standard_normal((nsteps, ny, nx))
    return alpha, src, gs


# ---------------------------------------------------------------- P1 closed form
@pytest.mark.parametrize("shape,h,dt,a", [((7, 6, 5), (1.0, 1.0, 1.0), 0.7, 0.9),
                                          ((4, 9, 6), (0.156, 0.3, 0.0625), 0.05, 0.1)])
def test_uniform_alpha_matches_cosine_eigenbasis(shape, h, dt, a):
    """Uniform alpha, zero flux: the cell-centred second difference is
    diagonalised by DCT-II modes cos(pi k (i+1/2)/n) with eigenvalues
    4 sin^2(pi k / 2n) / h^2 (the discrete counterpart of the slab
    eigenfunctions of App. B), so implicit Euler divides each mode by
    (1 + dt a lambda) per step."""
    nz, ny, nx = shape
    rng = np.random.default_rng(1)
    alpha = np.full(shape, a)
    q = rng.uniform(0, 3, size=(ny, nx))
    nsteps = 4
    src = np.zeros((nsteps, ny, nx))
    src[0] = q
    S, T_all, _ = orc.forward(alpha, src, dt, h=h)
    lam = [4.0 * np.sin(np.pi * np.arange(n) / (2 * n)) ** 2 / hh ** 2
           for n, hh in zip((nx, ny, nz), h)]
    Lam = lam[2][:, None, None] + lam[1][None, :, None] + lam[0][None, None, :]
    b1 = np.zeros(shape)
    b1[0] = dt * q
    bh = scipy.fft.dctn(b1, type=2, norm="ortho")
    for n in range(1, nsteps + 1):
        Tn = scipy.fft.idctn(bh / (1.0 + dt * a * Lam) ** n, type=2, norm="ortho")
        np.testing.assert_allclose(T_all[n - 1], Tn, rtol=0, atol=1e-12 * np.abs(Tn).max())
        np.testing.assert_allclose(S[n - 1], Tn[0], rtol=0, atol=1e-12 * np.abs(Tn).max())


# ---------------------------------------------------------------- P2 conservation
def test_total_heat_is_conserved_forward_and_adjoint():
    """Zero flux on every face makes every column of A sum to one (the row
    sums of App. D.2 with no Robin sink), so total heat grows only by the
    injected source, and the adjoint sum by the injected weights."""
    alpha, src, gs = _rand_problem((5, 6, 7), 6, seed=2)
    dt = 1.3
    S, T_all, _ = orc.forward(alpha, src, dt)
    injected = np.cumsum(dt * src.sum(axis=(1, 2)))
    np.testing.assert_allclose(T_all.sum(axis=(1, 2, 3)), injected, rtol=1e-11)
    G, dq, mu1, _ = orc.adjoint(alpha, T_all, gs, dt)
    assert abs(mu1.sum() - gs.sum()) <= 1e-10 * np.abs(gs).sum()
    # dJ/dq^n = dt mu^n on the top plane, so its per-step sum equals dt * sum_{m>=n} sum g^m
    # only for the total; check the first step, where mu^1 collects all weights.
    np.testing.assert_allclose(dq[0], dt * mu1[0], rtol=1e-12, atol=0)


# ---------------------------------------------------------------- P3 dense solves
@pytest.mark.parametrize("shape,h,dt", [((6, 5, 4), (1.0, 1.0, 1.0), 2.0),
                                        ((3, 3, 3), (1.0, 1.0, 1.0), 0.5),
                                        ((3, 4, 5), (0.5, 1.0, 2.0), 1.0)])
def test_forward_and_gradient_match_dense_assembly(shape, h, dt):
    """Independent dense assembly of App. D.2 plus numpy.linalg.solve and the
    explicit derivative of the assembled matrix (eq. grad_assembly)."""
    alpha, src, gs = _rand_problem(shape, 5, seed=3)
    S, T_all, _ = orc.forward(alpha, src, dt, h=h)
    Td, Sd = dense_ref.forward(alpha, src, dt, h)
    np.testing.assert_allclose(S, Sd, rtol=1e-11, atol=1e-12 * np.abs(Sd).max())
    np.testing.assert_allclose(T_all.reshape(Td.shape), Td, rtol=1e-11, atol=1e-12 * np.abs(Td).max())
    G, _, _, _ = orc.adjoint(alpha, T_all, gs, dt, h=h)
    Gd, _ = dense_ref.adjoint_gradient(alpha, src, gs, dt, h)
    np.testing.assert_allclose(G, Gd, rtol=1e-9, atol=1e-11 * np.abs(Gd).max())


# ---------------------------------------------------------------- P4 dot-product tests
def test_adjoint_dot_product_source_map():
    """For fixed alpha, F: q -> S is linear and its transpose applied to w is
    dt mu^n on the top plane (the adjoint recurrence, eq. adjoint_eq)."""
    alpha, src, w = _rand_problem((6, 7, 8), 7, seed=4)
    dt = 3.0
    S, T_all, _ = orc.forward(alpha, src, dt)
    _, dq, _, _ = orc.adjoint(alpha, T_all, w, dt)
    lhs = np.sum(S * w)
    rhs = np.sum(src * dq)
    assert abs(lhs - rhs) <= 1e-11 * max(abs(lhs), 1.0)


def test_adjoint_dot_product_initial_state():
    """With no source, T^0 -> S is linear and its transpose applied to w is
    mu^1 (the adjoint recurrence run down to n = 1, eq. adjoint_eq): the
    initial-state gradient of the linear functional <w, S>."""
    alpha, _, w = _rand_problem((5, 6, 7), 6, seed=14)
    dt = 2.5
    T0 = np.random.default_rng(15).standard_normal(alpha.shape)
    src = np.zeros((6,) + alpha.shape[1:])
    S, T_all, _ = orc.forward(alpha, src, dt, T0=T0, rtol=1e-14)
    _, _, mu1, _ = orc.adjoint(alpha, T_all, w, dt, rtol=1e-14)
    lhs = np.sum(S * w)
    rhs = np.sum(T0 * mu1)
    assert abs(lhs - rhs) <= 1e-11 * max(abs(lhs), 1.0)


def test_tangent_linear_vs_adjoint():
    """<J v, w> = <v, J^T w> with J = dS/dalpha: TLM against the adjoint gradient."""
    alpha, src, w = _rand_problem((5, 6, 7), 6, seed=5)
    dt = 2.0
    v = np.random.default_rng(55).standard_normal(alpha.shape)
    _, T_all, _ = orc.forward(alpha, src, dt)
    dS = orc.tlm(alpha, v, T_all, dt)
    G, _, _, _ = orc.adjoint(alpha, T_all, w, dt)
    lhs = np.sum(dS * w)
    rhs = np.sum(v * G)
    assert abs(lhs - rhs) <= 1e-10 * max(abs(lhs), 1e-3)


# ---------------------------------------------------------------- P5 finite differences
def test_gradient_central_differences_mse():
    """Central differences of the MSE loss in single voxels (h = 1e-5 alpha_p)."""
    w = wl.small_problem(5, 4, 4, 6, seed=6, dt=1.5)
    src = orc.source_series(w.q_xy, w.q_t)
    St, _, _ = orc.forward(w.alpha_target, src, w.dt, keep_states=False)

    def loss(a):
        S, _, _ = orc.forward(a, src, w.dt, keep_states=False)
        return orc.mse_loss_and_grad(S, St)[0]

    S, T_all, _ = orc.forward(w.alpha, src, w.dt)
    _, gs = orc.mse_loss_and_grad(S, St)
    G, _, _, _ = orc.adjoint(w.alpha, T_all, gs, w.dt)
    rng = np.random.default_rng(66)
    for flat in rng.choice(w.alpha.size, size=8, replace=False):
        p = np.unravel_index(flat, w.alpha.shape)
        eps = 1e-5 * w.alpha[p]
        ap, am = w.alpha.copy(), w.alpha.copy()
        ap[p] += eps
        am[p] -= eps
        fd = (loss(ap) - loss(am)) / (2 * eps)
        assert abs(fd - G[p]) <= 1e-6 * max(abs(fd), 1e-3 * np.abs(G).max()), (p, fd, G[p])


def test_gradient_complex_step_direction():
    """Complex-step directional derivative through dense complex solves."""
    alpha, src, gs = _rand_problem((4, 3, 5), 4, seed=7)
    dt = 1.0
    v = np.random.default_rng(77).standard_normal(alpha.shape)
    _, T_all, _ = orc.forward(alpha, src, dt)
    G, _, _, _ = orc.adjoint(alpha, T_all, gs, dt)
    cs = dense_ref.complex_step_directional(alpha, v, src, gs, dt)
    assert abs(np.sum(G * v) - cs) <= 1e-11 * max(abs(cs), 1.0)


# ---------------------------------------------------------------- P6 one-dimensional case
def test_column_reduces_to_tridiagonal_banded_solve():
    """nx = ny = 1 leaves a tridiagonal system; scipy.linalg.solve_banded."""
    rng = np.random.default_rng(8)
    nz, dt, hz = 12, 0.8, 0.7
    alpha = np.exp(rng.standard_normal((nz, 1, 1)))
    src = rng.uniform(0, 2, size=(3, 1, 1))
    S, T_all, _ = orc.forward(alpha, src, dt, h=(1.0, 1.0, hz))
    a = alpha.ravel()
    c = 2 * a[:-1] * a[1:] / (a[:-1] + a[1:]) / hz ** 2  # face k+1/2
    diag = np.ones(nz)
    diag[:-1] += dt * c
    diag[1:] += dt * c
    ab = np.zeros((3, nz))
    ab[0, 1:] = -dt * c
    ab[1] = diag
    ab[2, :-1] = -dt * c
    T = np.zeros(nz)
    for s in range(3):
        b = T.copy()
        b[0] += dt * src[s, 0, 0]
        T = scipy.linalg.solve_banded((1, 1), ab, b)
        np.testing.assert_allclose(T_all[s].ravel(), T, rtol=1e-12)


# ---------------------------------------------------------------- P7 two-cell case (Prop. 1)
def test_two_cells_harmonic_flux():
    """Two cells exchange heat through the harmonic-mean conductance of
    Prop. 1: the difference decays by 1/(1 + 2 dt c) per step and the sum is
    conserved."""
    a1, a2, dx, dt = 0.3, 2.5, 0.8, 0.4
    alpha = np.array([a1, a2]).reshape(1, 1, 2)
    src = np.zeros((3, 1, 2))
    src[0, 0, 0] = 7.0
    S, T_all, _ = orc.forward(alpha, src, dt, h=(dx, 1.0, 1.0))
    c = 2 * a1 * a2 / (a1 + a2) / dx ** 2
    tot = dt * 7.0
    diff = tot / (1 + 2 * dt * c)  # step 1: difference of b is tot, sum is tot
    for s in range(3):
        T1 = 0.5 * (tot + diff)
        T2 = 0.5 * (tot - diff)
        np.testing.assert_allclose(T_all[s].ravel(), [T1, T2], rtol=1e-13)
        diff = diff / (1 + 2 * dt * c)


# ---------------------------------------------------------------- P8 long-time limit
def test_long_time_limit_is_uniform():
    alpha, _, _ = _rand_problem((4, 5, 6), 1, seed=9, sigma=0.3)
    nsteps = 300
    src = np.zeros((nsteps, 5, 6))
    src[0] = np.random.default_rng(10).uniform(0, 1, size=(5, 6))
    dt = 5.0
    _, T_all, _ = orc.forward(alpha, src, dt)
    mean = dt * src[0].sum() / alpha.size
    np.testing.assert_allclose(T_all[-1], mean, rtol=1e-9)


# ---------------------------------------------------------------- P9 variance growth (App. H)
def test_variance_grows_by_two_alpha_dt_per_step():
    """App. H checks that a Gaussian spreads with variance slope 2 alpha. For
    the discrete scheme the x-marginal of a uniform-alpha field evolves by the
    1-D implicit-Euler kernel, whose variance is exactly 2 alpha dt; so the
    marginal's variance grows by exactly 2 alpha dt per step while the heat
    stays far from the walls. The paper's measured slope (golden fixture)
    must sit within its stated 0.16% of ours."""
    with open(os.path.join(GOLDEN, "app_h_variance_slope.json")) as f:
        gold = json.load(f)
    a, dt = gold["alpha"], 0.5
    nx, ny, nz = 161, 3, 2
    alpha = np.full((nz, ny, nx), a)
    nsteps = 8
    src = np.zeros((nsteps, ny, nx))
    src[0, :, nx // 2] = 1.0
    _, T_all, _ = orc.forward(alpha, src, dt)
    x = np.arange(nx)
    var = []
    for s in range(nsteps):
        m = T_all[s].sum(axis=(0, 1))
        mu = (m * x).sum() / m.sum()
        var.append(((x - mu) ** 2 * m).sum() / m.sum())
    growth = np.diff(var)
    np.testing.assert_allclose(growth, 2 * a * dt, rtol=1e-9)
    slope = growth.mean() / dt
    assert abs(slope - gold["analytic_slope"]) < 1e-9
    assert abs(gold["measured_slope"] - slope) / slope <= gold["relative_error"] + 1e-4


# ---------------------------------------------------------------- P10 structure
def test_operator_symmetric_rowsum_one_and_positive():
    """App. D.2: A is symmetric, A 1 = 1 without a Robin sink, and an M-matrix
    (so a non-negative source keeps T non-negative)."""
    alpha, src, _ = _rand_problem((5, 6, 7), 3, seed=11, sigma=1.0)
    dt = 4.0
    rng = np.random.default_rng(12)
    x, y = rng.standard_normal((2,) + alpha.shape)
    Ax, Ay = orc.apply_A(alpha, x, dt), orc.apply_A(alpha, y, dt)
    assert abs(np.sum(Ax * y) - np.sum(x * Ay)) <= 1e-12 * np.abs(Ax * y).sum()
    np.testing.assert_allclose(orc.apply_A(alpha, np.ones_like(alpha), dt), 1.0, rtol=0, atol=1e-13)
    _, T_all, _ = orc.forward(alpha, src, dt)
    assert T_all.min() > 0
    # the diagonal is 1 + dt * (sum of the row's conductances)
    d = orc.diagonal(alpha, dt)
    e = np.zeros(alpha.size)
    e[37] = 1.0
    col = orc.apply_A(alpha, e.reshape(alpha.shape), dt).ravel()
    assert abs(col[37] - d.ravel()[37]) < 1e-14 * d.ravel()[37]
    assert abs(col.sum() - 1.0) < 1e-13


# ---------------------------------------------------------------- P11 Euler homogeneity
def test_euler_homogeneity_of_gradient():
    """The harmonic mean is 1-homogeneous, so sum_p alpha_p dL/dalpha_p equals
    dL(c alpha)/dc at c = 1 (a scalar that a central difference resolves)."""
    w = wl.small_problem(6, 5, 4, 5, seed=13, dt=2.0)
    src = orc.source_series(w.q_xy, w.q_t)
    St, _, _ = orc.forward(w.alpha_target, src, w.dt, keep_states=False)
    S, T_all, _ = orc.forward(w.alpha, src, w.dt)
    _, gs = orc.mse_loss_and_grad(S, St)
    G, _, _, _ = orc.adjoint(w.alpha, T_all, gs, w.dt)
    eps = 1e-5

    def loss(c):
        Sc, _, _ = orc.forward(c * w.alpha, src, w.dt, keep_states=False)
        return orc.mse_loss_and_grad(Sc, St)[0]

    fd = (loss(1 + eps) - loss(1 - eps)) / (2 * eps)
    lhs = float(np.sum(w.alpha * G))
    assert abs(lhs - fd) <= 1e-7 * abs(fd)


# ---------------------------------------------------------------- P12 autograd cross-route
def test_gradient_matches_autograd_through_dense_solves():
    """Autograd through dense solves (the paper's AD route of Table 4) agrees
    with the discrete adjoint (its AM route)."""
    alpha, src, gs = _rand_problem((3, 4, 5), 4, seed=14)
    dt = 1.7
    _, T_all, _ = orc.forward(alpha, src, dt)
    G, _, _, _ = orc.adjoint(alpha, T_all, gs, dt)
    Ga = dense_ref.autograd_gradient(alpha, src, gs, dt)
    np.testing.assert_allclose(G, Ga, rtol=1e-9, atol=1e-12 * np.abs(Ga).max())


# ---------------------------------------------------------------- solver contract
def test_zero_rhs_gives_zero_and_no_iterations():
    alpha = np.ones((2, 3, 4))
    x, it, rel = orc.solve(alpha, np.zeros_like(alpha), 1.0, x0=np.ones_like(alpha))
    assert it == 0 and rel == 0.0 and not x.any()


def test_plain_fp64_workload_converges():
    """The 16x16x8 FP64 workload: every step converges and heat is conserved."""
    w = wl.plain_fp64_16x16x8()
    out = orc.run_workload(w)
    assert out["iters_fwd"].max() < 200 and out["iters_adj"].max() < 200
    tot = out["T_all"].sum(axis=(1, 2, 3))
    np.testing.assert_allclose(tot, w.dt * 100.0 * 256, rtol=1e-11)
    assert np.isfinite(out["G"]).all() and np.abs(out["G"]).max() > 0


# ---------------------------------------------------------------- P13 closures and the fixed-K inner solver
# App. D.2: lateral periodicity by circular padding, a Robin back face with the
# diagonal sink beta = h / dz, and K Jacobi sweeps warm-started from T^{n-1}.

@pytest.mark.parametrize("shape,h,dt,a", [((5, 6, 7), (1.0, 1.0, 1.0), 0.8, 0.7),
                                          ((4, 8, 6), (0.156, 0.156, 0.0625), 0.05, 0.15)])
def test_periodic_uniform_alpha_matches_fourier_cosine_basis(shape, h, dt, a):
    """Uniform alpha, periodic x, y and zero-flux z: the discrete operator is
    diagonal in Fourier (x, y) times DCT-II (z) modes, the grid counterpart of
    the slab eigenfunctions of App. B (step 4), with eigenvalue
    4 sin^2(pi m / nx) / hx^2 + 4 sin^2(pi l / ny) / hy^2 + 4 sin^2(pi p / (2 nz)) / hz^2.
    Each implicit step divides a mode by 1 + dt a lambda."""
    nz, ny, nx = shape
    rng = np.random.default_rng(21)
    T0 = rng.standard_normal(shape)
    nsteps = 3
    alpha = np.full(shape, a)
    S, T_all, _ = orc.forward(alpha, np.zeros((nsteps, ny, nx)), dt, T0=T0, h=h, rtol=1e-14,
                              periodic=True)
    m = np.arange(nx)
    l = np.arange(ny)
    p = np.arange(nz)
    lam = (4 * np.sin(np.pi * p / (2 * nz)) ** 2 / h[2] ** 2)[:, None, None] \
        + (4 * np.sin(np.pi * l / ny) ** 2 / h[1] ** 2)[None, :, None] \
        + (4 * np.sin(np.pi * m / nx) ** 2 / h[0] ** 2)[None, None, :]
    spec = scipy.fft.dct(np.fft.fft2(T0, axes=(1, 2)), type=2, axis=0, norm="ortho")
    for n in range(1, nsteps + 1):
        Tn = np.fft.ifft2(scipy.fft.idct(spec / (1 + dt * a * lam) ** n, type=2, axis=0, norm="ortho"),
                          axes=(1, 2)).real
        np.testing.assert_allclose(T_all[n - 1], Tn, rtol=0, atol=1e-11 * np.abs(T0).max())


def test_robin_single_layer_decays_by_one_plus_dt_beta():
    """nz = 1 and a uniform state: no face carries flux, so the finite-volume
    balance of the Robin face leaves A T = (1 + dt h / dz) T on every cell."""
    shape = (1, 4, 5)
    alpha = np.exp(0.4 * np.random.default_rng(22).standard_normal(shape))
    h, dt, hr = (0.3, 0.4, 0.0625), 0.05, 0.8
    T0 = np.full(shape, 2.0)
    _, T_all, _ = orc.forward(alpha, np.zeros((4, 4, 5)), dt, T0=T0, h=h, rtol=1e-14,
                              periodic=True, robin=hr)
    for n in range(4):
        np.testing.assert_allclose(T_all[n], 2.0 / (1 + dt * hr / h[2]) ** (n + 1), rtol=1e-12)


def test_robin_heat_balance():
    """Column sums of A are 1 + dt beta_p (App. D.2): the heat lost per step is
    dt beta times the back-face heat of the new state."""
    alpha, src, gs = _rand_problem((5, 6, 7), 5, seed=23)
    h, dt, hr = (1.0, 0.7, 0.5), 0.9, 0.3
    _, T_all, _ = orc.forward(alpha, src, dt, h=h, rtol=1e-14, robin=hr, periodic=True)
    prev = 0.0
    for n in range(5):
        lhs = T_all[n].sum() + dt * hr / h[2] * T_all[n][-1].sum()
        np.testing.assert_allclose(lhs, prev + dt * src[n].sum(), rtol=1e-12)
        prev = T_all[n].sum()
    # the adjoint carries the same balance with A^T = A
    _, _, mu1, _ = orc.adjoint(alpha, T_all, gs, dt, h=h, rtol=1e-14, robin=hr, periodic=True)
    assert np.isfinite(mu1).all()


def test_robin_column_reduces_to_tridiagonal():
    """nx = ny = 1 is a 1-D column: the Robin sink sits on the last diagonal
    entry of the tridiagonal system (scipy.linalg.solve_banded)."""
    nz = 9
    rng = np.random.default_rng(24)
    a = np.exp(0.5 * rng.standard_normal(nz))
    hz, dt, hr = 0.1, 0.02, 0.7
    c = 2 * a[:-1] * a[1:] / (a[:-1] + a[1:]) / hz ** 2
    diag = 1 + dt * (np.r_[c, 0.0] + np.r_[0.0, c])
    diag[-1] += dt * hr / hz
    ab = np.zeros((3, nz))
    ab[0, 1:] = -dt * c
    ab[1] = diag
    ab[2, :-1] = -dt * c
    src = rng.uniform(0, 5, size=(3, 1, 1))
    _, T_all, _ = orc.forward(a.reshape(nz, 1, 1), src, dt, h=(1.0, 1.0, hz), rtol=1e-14, robin=hr)
    T = np.zeros(nz)
    for n in range(3):
        b = T.copy()
        b[0] += dt * src[n, 0, 0]
        T = scipy.linalg.solve_banded((1, 1), ab, b)
        np.testing.assert_allclose(T_all[n].ravel(), T, rtol=1e-12)


@pytest.mark.parametrize("periodic,robin", [(True, 0.0), (False, 0.6), (True, 0.6)])
def test_closures_match_dense_assembly(periodic, robin):
    """States and gradient against the dense assembly of App. D.2 with the
    wrapped faces and the Robin rows."""
    alpha, src, gs = _rand_problem((3, 4, 5), 4, seed=25)
    h, dt = (0.5, 0.8, 0.3), 0.2
    opt = dict(periodic=periodic, robin=robin)
    S, T_all, _ = orc.forward(alpha, src, dt, h=h, rtol=1e-14, **opt)
    Td, Sd = dense_ref.forward(alpha, src, dt, h, **opt)
    np.testing.assert_allclose(T_all.reshape(Td.shape), Td, rtol=1e-11, atol=1e-12 * np.abs(Td).max())
    G, _, _, _ = orc.adjoint(alpha, T_all, gs, dt, h=h, rtol=1e-14, **opt)
    Gd, _ = dense_ref.adjoint_gradient(alpha, src, gs, dt, h, **opt)
    np.testing.assert_allclose(G, Gd, rtol=1e-9, atol=1e-11 * np.abs(Gd).max())
    # and the operator itself
    x = np.random.default_rng(26).standard_normal(alpha.shape)
    Ad = dense_ref.system_matrix(alpha, dt, h, **opt)
    np.testing.assert_allclose(orc.apply_A(alpha, x, dt, h=h, **opt).ravel(), Ad @ x.ravel(), rtol=1e-13,
                               atol=1e-13 * np.abs(x).max())
    np.testing.assert_allclose(orc.diagonal(alpha, dt, h=h, **opt).ravel(), np.diag(Ad), rtol=1e-14)


@pytest.mark.parametrize("periodic,robin,K", [(False, 0.0, 1), (True, 0.0, 7), (True, 0.5, 50)])
def test_jacobi_sweeps_match_dense_splitting(periodic, robin, K):
    """K sweeps x <- D^-1 (b - R x) (eq. jacobi_iter) against the dense
    splitting A = D + R, and a whole fixed-K forward and adjoint (warm starts
    T^{n-1} and mu^{n+1}) against the dense run of the same recurrences."""
    alpha, src, gs = _rand_problem((3, 4, 5), 3, seed=27)
    h, dt = (0.5, 0.8, 0.3), 0.05
    opt = dict(periodic=periodic, robin=robin)
    rng = np.random.default_rng(28)
    b, x0 = rng.standard_normal(alpha.shape), rng.standard_normal(alpha.shape)
    A = dense_ref.system_matrix(alpha, dt, h, **opt)
    D = np.diag(A)
    x = x0.ravel().copy()
    for _ in range(K):
        x = (b.ravel() - (A - np.diag(D)) @ x) / D
    np.testing.assert_allclose(orc.jacobi(alpha, b, dt, x0, K, h=h, **opt).ravel(), x, rtol=1e-12,
                               atol=1e-13 * np.abs(x).max())
    S, T_all, it = orc.forward(alpha, src, dt, h=h, jacobi_k=K, **opt)
    assert (it == K).all()
    Td, _ = dense_ref.forward(alpha, src, dt, h, jacobi_k=K, **opt)
    np.testing.assert_allclose(T_all.reshape(Td.shape), Td, rtol=1e-12, atol=1e-13 * np.abs(Td).max())
    G, _, _, _ = orc.adjoint(alpha, T_all, gs, dt, h=h, jacobi_k=K, **opt)
    Gd, _ = dense_ref.adjoint_gradient(alpha, src, gs, dt, h, jacobi_k=K, **opt)
    np.testing.assert_allclose(G, Gd, rtol=1e-10, atol=1e-12 * np.abs(Gd).max())


def test_jacobi_converges_to_the_exact_solve():
    """Strict diagonal dominance (App. D.2) makes the sweeps contract: many
    sweeps reach the PCG fixed point, and the paper's K = 50 on its grid
    spacing and dt leaves a small residual."""
    w = wl.paper_64x64x16(nsteps=4, precision="f64")
    src = orc.source_series(w.q_xy, w.q_t)
    opt = dict(h=w.h, periodic=True)
    S, _, _ = orc.forward(w.alpha, src, w.dt, rtol=1e-14, **opt)
    Sj, _, _ = orc.forward(w.alpha, src, w.dt, jacobi_k=400, **opt)
    assert np.abs(Sj - S).max() <= 1e-10 * np.abs(S).max()
    S50, _, _ = orc.forward(w.alpha, src, w.dt, jacobi_k=50, **opt)
    err = np.abs(S50 - S).max() / np.abs(S).max()
    assert 0 < err < 1e-2


# ---------------------------------------------------------------- P14 total variation (eq. tv_discrete)
from oracle import tv as orc_tv  # noqa: E402


def test_tv_constant_field_is_volume_times_eps():
    """No differences: every term is eps, R = N dx dy dz eps."""
    h, eps = (0.156, 0.156, 0.0625), 1e-3
    a = np.full((4, 5, 6), 0.3)
    assert abs(orc_tv.tv_value(a, h, eps) - 120 * h[0] * h[1] * h[2] * eps) <= 1e-15
    assert np.abs(orc_tv.tv_grad(a, h, eps)).max() == 0.0


def test_tv_step_in_x_counts_both_periodic_jumps():
    """alpha = a on the first half of each x row, b on the second: with the
    lateral wrap every row has two jumps of |a - b|, so as eps -> 0
    R = dx dy dz * 2 |a - b| / dx * ny * nz (plus eps on the flat cells)."""
    nz, ny, nx = 3, 4, 8
    h, eps = (0.5, 0.7, 0.3), 1e-12
    a = np.full((nz, ny, nx), 0.2)
    a[:, :, nx // 2:] = 0.05
    want = h[0] * h[1] * h[2] * (2 * 0.15 / h[0] * ny * nz + (nx - 2) * ny * nz * eps)
    assert abs(orc_tv.tv_value(a, h, eps) - want) <= 1e-13 * want


def test_tv_ramp_in_z_has_no_last_plane_term():
    """alpha_k = c k: nz - 1 vertical differences per column (the last plane's
    is zero by definition), so R = dx dy dz nx ny ((nz - 1) |c| / dz + eps)."""
    nz, ny, nx = 5, 3, 4
    h, eps, c = (1.0, 1.0, 0.25), 1e-12, 0.07
    a = np.broadcast_to((c * np.arange(nz))[:, None, None], (nz, ny, nx)).copy()
    want = h[0] * h[1] * h[2] * nx * ny * ((nz - 1) * c / h[2] + eps)
    assert abs(orc_tv.tv_value(a, h, eps) - want) <= 1e-13 * want


def test_tv_isotropic_combination_in_one_cell():
    """One raised cell p: p's own term combines its +x, +y, +z differences
    under one square root (isotropic TV), not as a sum of absolute values."""
    nz, ny, nx = 3, 3, 3
    h, eps, d = (1.0, 2.0, 0.5), 1e-9, 0.4
    a = np.zeros((nz, ny, nx))
    a[1, 1, 1] = d
    # p: all three forward differences are -d; its -x, -y, -z neighbours each see +d along one axis
    own = np.sqrt((d / h[0]) ** 2 + (d / h[1]) ** 2 + (d / h[2]) ** 2 + eps ** 2)
    nb = [np.sqrt((d / hh) ** 2 + eps ** 2) for hh in h]
    want = h[0] * h[1] * h[2] * (own + sum(nb) + (27 - 4) * eps)
    assert abs(orc_tv.tv_value(a, h, eps) - want) <= 1e-14 * want


def test_tv_gradient_matches_central_differences():
    """Brute-force central differences of R on a small random field."""
    rng = np.random.default_rng(31)
    a = rng.uniform(0.05, 0.2, size=(3, 4, 5))
    h, eps = (0.156, 0.156, 0.0625), 1e-2
    g = orc_tv.tv_grad(a, h, eps)
    step = 1e-6
    for flat in range(a.size):
        p = np.unravel_index(flat, a.shape)
        ap, am = a.copy(), a.copy()
        ap[p] += step
        am[p] -= step
        fd = (orc_tv.tv_value(ap, h, eps) - orc_tv.tv_value(am, h, eps)) / (2 * step)
        assert abs(fd - g[p]) <= 1e-6 * max(abs(fd), 1e-3 * np.abs(g).max()), (p, fd, g[p])
