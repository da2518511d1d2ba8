"""Dense reference for tiny grids, assembled independently of ``heat_oracle.c``.

TEST INFRASTRUCTURE ONLY. It pins the matrix-free oracle: the matrix here is
assembled entry by entry from the listing of App. D.2 of the paper in the
paper's own sign convention (``L`` negative semidefinite,
``A = I - dt*L``), and every solve is a dense ``numpy.linalg.solve`` (or, for
the paper's fixed-K inner solver, K dense Jacobi sweeps). The
gradient is obtained three independent ways: explicit differentiation of the
assembled matrix, complex-step, and torch autograd through dense solves.
"""
from __future__ import annotations

import numpy as np


def _faces(shape, periodic=False):
    """Yield (p, q, axis) for every interior face, q the + neighbour of p;
    with ``periodic`` the x and y rows close into rings (circular padding,
    App. D.2), so the last cell of a row also faces the first."""
    nz, ny, nx = shape
    for k in range(nz):
        for j in range(ny):
            for i in range(nx):
                p = i + nx * (j + ny * k)
                if i + 1 < nx or periodic:
                    yield p, (i + 1) % nx + nx * (j + ny * k), 0
                if j + 1 < ny or periodic:
                    yield p, i + nx * ((j + 1) % ny + ny * k), 1
                if k + 1 < nz:
                    yield p, i + nx * (j + ny * (k + 1)), 2


def assemble_L(alpha, h=(1.0, 1.0, 1.0), periodic=False, robin=0.0):
    """Paper's operator (App. D.2): ``L_pq = a_pq`` for face neighbours,
    ``L_pp = -beta_p - sum_q a_pq``, ``a_pq = hm(alpha_p, alpha_q) / h_axis^2``;
    ``beta_p = robin / h_z`` on the back-face rows (k = nz-1), else 0.
    Works for real or complex ``alpha``."""
    a = np.asarray(alpha).ravel()
    n = a.size
    nz, ny, nx = np.shape(alpha)
    L = np.zeros((n, n), dtype=np.result_type(a.dtype, np.float64))
    hs = (h[0], h[1], h[2])
    for p, q, ax in _faces(np.shape(alpha), periodic):
        c = 2.0 * a[p] * a[q] / (a[p] + a[q]) / hs[ax] ** 2
        L[p, q] += c
        L[q, p] += c
        L[p, p] -= c
        L[q, q] -= c
    if robin:
        back = np.arange((nz - 1) * nx * ny, nz * nx * ny)
        L[back, back] -= robin / h[2]
    return L


def assemble_dL(alpha, p_cell, h=(1.0, 1.0, 1.0), periodic=False):
    """``dL/dalpha_p`` for one cell p, from the derivative of the harmonic mean
    (the Robin sink does not depend on alpha)."""
    a = np.asarray(alpha, dtype=np.float64).ravel()
    n = a.size
    dL = np.zeros((n, n))
    hs = (h[0], h[1], h[2])
    for p, q, ax in _faces(np.shape(alpha), periodic):
        if p_cell == p:
            d = 2.0 * a[q] ** 2 / (a[p] + a[q]) ** 2 / hs[ax] ** 2
        elif p_cell == q:
            d = 2.0 * a[p] ** 2 / (a[p] + a[q]) ** 2 / hs[ax] ** 2
        else:
            continue
        dL[p, q] += d
        dL[q, p] += d
        dL[p, p] -= d
        dL[q, q] -= d
    return dL


def system_matrix(alpha, dt, h=(1.0, 1.0, 1.0), periodic=False, robin=0.0):
    L = assemble_L(alpha, h, periodic, robin)
    return np.eye(L.shape[0], dtype=L.dtype) - dt * L


def _solver(A, jacobi_k):
    """Dense ``A x = b`` with start ``x0``: exact, or ``jacobi_k`` sweeps of the
    splitting ``A = D + R``, ``x <- D^-1 (b - R x)`` (eq. jacobi_iter)."""
    if not jacobi_k:
        return lambda b, x0: np.linalg.solve(A, b)
    D = np.diag(A).copy()
    R = A - np.diag(D)

    def run(b, x0):
        x = x0.copy()
        for _ in range(jacobi_k):
            x = (b - R @ x) / D
        return x
    return run


def top_mask(shape):
    nz, ny, nx = shape
    m = np.zeros(nz * ny * nx, dtype=bool)
    m[: nx * ny] = True
    return m


def forward(alpha, src, dt, h=(1.0, 1.0, 1.0), periodic=False, robin=0.0, jacobi_k=0, T0=None):
    """States T^1..T^N (``[N][ng]``) and surfaces (``[N][ny][nx]``), T^0 = 0
    unless given; each solve exact or ``jacobi_k`` Jacobi sweeps warm-started
    from the previous state (App. D.2)."""
    shape = np.shape(alpha)
    nz, ny, nx = shape
    A = system_matrix(alpha, dt, h, periodic, robin)
    solve = _solver(A, jacobi_k)
    top = top_mask(shape)
    T = np.zeros(A.shape[0], dtype=A.dtype) if T0 is None else np.asarray(T0, dtype=A.dtype).ravel()
    Ts, Ss = [], []
    for s in range(src.shape[0]):
        b = T.copy()
        b[top] += dt * np.asarray(src[s]).ravel()
        T = solve(b, T)
        Ts.append(T)
        Ss.append(T[top].reshape(ny, nx))
    return np.array(Ts), np.array(Ss)


def adjoint_gradient(alpha, src, gs, dt, h=(1.0, 1.0, 1.0), periodic=False, robin=0.0, jacobi_k=0):
    """dJ/dalpha for J with dJ/dS = gs, from the Lagrangian derivation of
    App. D.3 written with dense matrices: ``A^T mu^n = mu^{n+1} + Pi^T g^n`` and
    ``dJ/dalpha_p = dt sum_n mu^n . (dL/dalpha_p) T^n``. With ``jacobi_k`` the
    states and multipliers come from that many Jacobi sweeps per solve, the
    adjoint ones started from mu^{n+1}."""
    shape = np.shape(alpha)
    A = system_matrix(alpha, dt, h, periodic, robin)
    solve_t = _solver(A.T, jacobi_k)
    T_all, _ = forward(alpha, src, dt, h, periodic, robin, jacobi_k)
    top = top_mask(shape)
    n = A.shape[0]
    N = src.shape[0]
    mus = [None] * N
    mu_next = np.zeros(n)
    for s in range(N - 1, -1, -1):
        rhs = mu_next.copy()
        rhs[top] += np.asarray(gs[s]).ravel()
        mus[s] = solve_t(rhs, mu_next)
        mu_next = mus[s]
    G = np.zeros(n)
    for p in range(n):
        dL = assemble_dL(alpha, p, h, periodic)
        G[p] = dt * sum(mus[s] @ (dL @ T_all[s]) for s in range(N))
    return G.reshape(shape), np.array(mus)


def surface_functional(alpha, src, gs, dt, h=(1.0, 1.0, 1.0)):
    """``sum_n <S^n, g^n>`` (a linear functional of the surface series)."""
    _, S = forward(alpha, src, dt, h)
    return np.sum(S * gs)


def complex_step_directional(alpha, v, src, gs, dt, h=(1.0, 1.0, 1.0), eps=1e-30):
    """``d/de sum_n <S^n(alpha + e v), g^n>`` at e = 0 by the complex step."""
    ac = np.asarray(alpha, dtype=np.complex128) + 1j * eps * np.asarray(v)
    return float(np.imag(surface_functional(ac, src, gs, dt, h)) / eps)


def autograd_gradient(alpha, src, gs, dt, h=(1.0, 1.0, 1.0)):
    """dJ/dalpha by torch autograd through dense FP64 solves (CPU)."""
    import torch

    shape = np.shape(alpha)
    nz, ny, nx = shape
    a = torch.tensor(np.asarray(alpha, dtype=np.float64).ravel(), requires_grad=True)
    n = a.numel()
    P, Q, AX = zip(*_faces(shape))
    P = torch.tensor(P)
    Q = torch.tensor(Q)
    hs = torch.tensor([h[0] ** 2, h[1] ** 2, h[2] ** 2], dtype=torch.float64)[torch.tensor(AX)]
    c = 2.0 * a[P] * a[Q] / (a[P] + a[Q]) / hs
    L = torch.zeros((n, n), dtype=torch.float64)
    L = L.index_put((P, Q), c, accumulate=True)
    L = L.index_put((Q, P), c, accumulate=True)
    L = L.index_put((P, P), -c, accumulate=True)
    L = L.index_put((Q, Q), -c, accumulate=True)
    A = torch.eye(n, dtype=torch.float64) - dt * L
    T = torch.zeros(n, dtype=torch.float64)
    J = torch.zeros((), dtype=torch.float64)
    src_t = torch.tensor(np.asarray(src, dtype=np.float64))
    g_t = torch.tensor(np.asarray(gs, dtype=np.float64))
    for s in range(src_t.shape[0]):
        b = T.clone()
        b[: nx * ny] = b[: nx * ny] + dt * src_t[s].reshape(-1)
        T = torch.linalg.solve(A, b)
        J = J + torch.sum(T[: nx * ny] * g_t[s].reshape(-1))
    (g,) = torch.autograd.grad(J, a)
    return g.detach().numpy().reshape(shape)
