"""ctypes front end of the matrix-free FP64 oracle (``heat_oracle.c``).

TEST INFRASTRUCTURE ONLY (see the package docstring). Every function here
takes NumPy arrays, widens them to float64 and calls the C routine; none of
the arithmetic lives in Python.

Conventions (the paper's Sec. 4.2-4.3 and App. D with A = I + dt*L+):
``alpha`` is ``[nz][ny][nx]``, x fastest, ``k = 0`` is the top face; the source
of step n is ``src[n-1]`` on the k = 0 plane, ``src[n-1] = q_t[n-1] * q_xy`` for
the separable pulses of the workloads.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "heat_oracle.c")
_LIB = os.path.join(_HERE, "libheat_oracle.so")

DEFAULT_RTOL = 1e-13
DEFAULT_MAX_ITER = 20000


def build(force: bool = False) -> str:
    """Compile ``heat_oracle.c`` into ``libheat_oracle.so`` (gcc, OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class _Grid(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int), ("ny", ctypes.c_int), ("nz", ctypes.c_int),
                ("hx", ctypes.c_double), ("hy", ctypes.c_double), ("hz", ctypes.c_double),
                ("periodic", ctypes.c_int), ("beta", ctypes.c_double), ("jacobi_k", ctypes.c_int)]


_lib = None


def _load():
    global _lib
    if _lib is None:
        # NH_ORACLE_LIB names another build of heat_oracle.c to use instead (the
        # sanitizer tier's instrumented build)
        lib = ctypes.CDLL(os.environ.get("NH_ORACLE_LIB") or build())
        P = ctypes.POINTER
        dp = P(ctypes.c_double)
        ip = P(ctypes.c_int)
        g = P(_Grid)
        lib.orc_apply_A.argtypes = [g, dp, ctypes.c_double, dp, dp]
        lib.orc_diagonal.argtypes = [g, dp, ctypes.c_double, dp]
        lib.orc_apply_R.argtypes = [g, dp, ctypes.c_double, dp, dp]
        lib.orc_jacobi.argtypes = [g, dp, ctypes.c_double, dp, dp, dp, ctypes.c_int]
        lib.orc_pcg.argtypes = [g, dp, ctypes.c_double, dp, dp, dp, ctypes.c_double, ctypes.c_int, dp]
        lib.orc_pcg.restype = ctypes.c_int
        lib.orc_forward.argtypes = [g, dp, dp, dp, ctypes.c_double, ctypes.c_int, ctypes.c_double,
                                    ctypes.c_int, dp, dp, ip]
        lib.orc_forward.restype = ctypes.c_int
        lib.orc_adjoint.argtypes = [g, dp, ctypes.c_double, ctypes.c_int, dp, dp, ctypes.c_double,
                                    ctypes.c_int, dp, dp, dp, ip]
        lib.orc_adjoint.restype = ctypes.c_int
        lib.orc_tlm.argtypes = [g, dp, dp, ctypes.c_double, ctypes.c_int, dp, ctypes.c_double,
                                ctypes.c_int, dp]
        lib.orc_tlm.restype = ctypes.c_int
        lib.orc_num_threads.restype = ctypes.c_int
        lib.orc_set_num_threads.argtypes = [ctypes.c_int]
        _lib = lib
    return _lib


def _d(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


def _ptr(a: Optional[np.ndarray]):
    if a is None:
        return None
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _grid(alpha: np.ndarray, h=(1.0, 1.0, 1.0), periodic=False, robin=0.0, jacobi_k=0) -> _Grid:
    """Grid, closure and inner solver: ``periodic`` wraps the lateral faces
    (needs nx, ny >= 3), ``robin`` is the coefficient h of the back-face
    condition n.(alpha grad T) = -h T (sink beta = h / dz on k = nz-1),
    ``jacobi_k`` > 0 replaces Jacobi-PCG by that many Jacobi sweeps."""
    nz, ny, nx = alpha.shape
    if periodic and (nx < 3 or ny < 3):
        raise ValueError("lateral periodicity needs nx, ny >= 3")
    if robin < 0 or jacobi_k < 0:
        raise ValueError("robin and jacobi_k must be >= 0")
    return _Grid(nx, ny, nz, float(h[0]), float(h[1]), float(h[2]), int(bool(periodic)),
                 float(robin) / float(h[2]), int(jacobi_k))


def num_threads() -> int:
    return int(_load().orc_num_threads())


def set_num_threads(n: int) -> None:
    """Run the oracle on n OpenMP threads from now on (timing only)."""
    _load().orc_set_num_threads(int(n))


def apply_A(alpha, x, dt, h=(1.0, 1.0, 1.0), periodic=False, robin=0.0) -> np.ndarray:
    """``A x`` with ``A = I + dt L+(alpha)``."""
    a, xx = _d(alpha), _d(x)
    y = np.empty_like(a)
    _load().orc_apply_A(ctypes.byref(_grid(a, h, periodic, robin)), _ptr(a), float(dt), _ptr(xx), _ptr(y))
    return y


def diagonal(alpha, dt, h=(1.0, 1.0, 1.0), periodic=False, robin=0.0) -> np.ndarray:
    a = _d(alpha)
    d = np.empty_like(a)
    _load().orc_diagonal(ctypes.byref(_grid(a, h, periodic, robin)), _ptr(a), float(dt), _ptr(d))
    return d


def solve(alpha, b, dt, x0=None, h=(1.0, 1.0, 1.0), rtol=DEFAULT_RTOL, max_iter=DEFAULT_MAX_ITER,
          periodic=False, robin=0.0):
    """Solve ``A x = b`` by Jacobi-PCG from ``x0`` (default 0). Returns (x, iters, rel_res)."""
    a, bb = _d(alpha), _d(b)
    x = np.zeros_like(a) if x0 is None else _d(x0).copy()
    dg = diagonal(a, dt, h, periodic, robin)
    rel = ctypes.c_double(0.0)
    it = _load().orc_pcg(ctypes.byref(_grid(a, h, periodic, robin)), _ptr(a), float(dt), _ptr(dg),
                         _ptr(bb), _ptr(x), float(rtol), int(max_iter), ctypes.byref(rel))
    return x, int(it), float(rel.value)


def jacobi(alpha, b, dt, x0, K, h=(1.0, 1.0, 1.0), periodic=False, robin=0.0):
    """``K`` Jacobi sweeps ``x <- D^-1 (b - R x)`` on ``A x = b`` from ``x0`` (eq. jacobi_iter)."""
    a, bb = _d(alpha), _d(b)
    x = _d(x0).copy()
    dg = diagonal(a, dt, h, periodic, robin)
    _load().orc_jacobi(ctypes.byref(_grid(a, h, periodic, robin)), _ptr(a), float(dt), _ptr(dg),
                       _ptr(bb), _ptr(x), int(K))
    return x


def source_series(q_xy, q_t) -> np.ndarray:
    """Per-step top-face source ``src[n] = q_t[n] * q_xy``, ``[nsteps][ny][nx]``."""
    return np.asarray(q_t, dtype=np.float64)[:, None, None] * _d(q_xy)[None, :, :]


def forward(alpha, src, dt, T0=None, h=(1.0, 1.0, 1.0), rtol=DEFAULT_RTOL,
            max_iter=DEFAULT_MAX_ITER, keep_states=True, periodic=False, robin=0.0, jacobi_k=0):
    """Forward sweep. ``src`` is ``[nsteps][ny][nx]``.

    Returns ``(S, T_all, iters)``: surface series ``[nsteps][ny][nx]``, all
    states ``[nsteps][nz][ny][nx]`` (None unless ``keep_states``) and the
    inner-solver iterations per step. Raises if a solve does not converge.
    ``periodic``, ``robin`` and ``jacobi_k`` choose the closure and the inner
    solver (see ``_grid``).
    """
    a, s = _d(alpha), _d(src)
    nz, ny, nx = a.shape
    nsteps = s.shape[0]
    assert s.shape == (nsteps, ny, nx)
    S = np.empty((nsteps, ny, nx))
    T_all = np.empty((nsteps, nz, ny, nx)) if keep_states else None
    iters = np.empty(nsteps, dtype=np.int32)
    t0 = None if T0 is None else _d(T0)
    grid = _grid(a, h, periodic, robin, jacobi_k)
    st = _load().orc_forward(ctypes.byref(grid), _ptr(a), _ptr(s), _ptr(t0), float(dt),
                             int(nsteps), float(rtol), int(max_iter), _ptr(S), _ptr(T_all),
                             iters.ctypes.data_as(ctypes.POINTER(ctypes.c_int)))
    if st != 0:
        raise RuntimeError("oracle forward: a solve did not converge")
    return S, T_all, iters


def adjoint(alpha, T_all, gs, dt, h=(1.0, 1.0, 1.0), rtol=DEFAULT_RTOL, max_iter=DEFAULT_MAX_ITER,
            periodic=False, robin=0.0, jacobi_k=0):
    """Adjoint sweep. ``gs = dJ/dS`` is ``[nsteps][ny][nx]``.

    Returns ``(G, dq, mu1, iters)``: ``dJ/dalpha`` ``[nz][ny][nx]``,
    ``dJ/dq^n`` ``[nsteps][ny][nx]``, ``mu^1 = dJ/dT^0`` and the iterations of
    each adjoint solve.
    """
    a, T, g = _d(alpha), _d(T_all), _d(gs)
    nz, ny, nx = a.shape
    nsteps = g.shape[0]
    assert T.shape == (nsteps, nz, ny, nx) and g.shape == (nsteps, ny, nx)
    G = np.empty_like(a)
    dq = np.empty((nsteps, ny, nx))
    mu1 = np.empty_like(a)
    iters = np.empty(nsteps, dtype=np.int32)
    grid = _grid(a, h, periodic, robin, jacobi_k)
    st = _load().orc_adjoint(ctypes.byref(grid), _ptr(a), float(dt), int(nsteps), _ptr(T),
                             _ptr(g), float(rtol), int(max_iter), _ptr(G), _ptr(dq), _ptr(mu1),
                             iters.ctypes.data_as(ctypes.POINTER(ctypes.c_int)))
    if st != 0:
        raise RuntimeError("oracle adjoint: a solve did not converge")
    return G, dq, mu1, iters


def tlm(alpha, v, T_all, dt, h=(1.0, 1.0, 1.0), rtol=DEFAULT_RTOL, max_iter=DEFAULT_MAX_ITER,
        periodic=False, robin=0.0):
    """Directional derivative ``dS`` of the surface series along ``v`` (alpha direction)."""
    a, vv, T = _d(alpha), _d(v), _d(T_all)
    nz, ny, nx = a.shape
    nsteps = T.shape[0]
    dS = np.empty((nsteps, ny, nx))
    st = _load().orc_tlm(ctypes.byref(_grid(a, h, periodic, robin)), _ptr(a), _ptr(vv), float(dt), int(nsteps),
                         _ptr(T), float(rtol), int(max_iter), _ptr(dS))
    if st != 0:
        raise RuntimeError("oracle tlm: a solve did not converge")
    return dS


def mse_loss_and_grad(S, S_target):
    """``L = mean((S - S_target)^2)`` over all steps and pixels and ``dL/dS``."""
    d = _d(S) - _d(S_target)
    m = d.size
    return float(np.sum(d * d) / m), 2.0 * d / m


def run_workload(w, rtol=DEFAULT_RTOL, with_adjoint=True):
    """Forward of ``w.alpha``, target surface from ``w.alpha_target``, MSE
    gradient and adjoint. Returns a dict of FP64 arrays."""
    src = source_series(w.q_xy, w.q_t)
    opt = dict(h=w.h, rtol=rtol, periodic=w.periodic, robin=w.robin, jacobi_k=w.jacobi_k)
    S, T_all, it_f = forward(w.alpha, src, w.dt, **opt)
    St, _, _ = forward(w.alpha_target, src, w.dt, keep_states=False, **opt)
    L, gs = mse_loss_and_grad(S, St)
    out = dict(S=S, S_target=St, loss=L, gs=gs, iters_fwd=it_f, T_all=T_all)
    if with_adjoint:
        G, dq, mu1, it_a = adjoint(w.alpha, T_all, gs, w.dt, **opt)
        out.update(G=G, dq=dq, mu1=mu1, iters_adj=it_a)
    return out
