"""Python front end of the HIP heat solver: a ``Solver`` object over one C
context and the ``HeatSolve`` autograd function.

PyTorch supplies device memory and the stream; every step of the forward
and adjoint sweeps runs in the library's kernels (``libnefty_heat.so``).
The loss stays with the caller: the adjoint takes ``dL/dT_surf`` and returns
``dL/dalpha`` (the vector-Jacobian product of the paper's Sec. 4.3).
"""
from __future__ import annotations

import ctypes
from typing import Optional, Sequence

import numpy as np
import torch

from . import _lib


def _check(code: int, ctx, func: str, allow=()):
    if code != _lib.NH_OK and code not in allow:
        raise _lib.NHError(code, func, _lib.last_error(ctx))
    return code


def _dev_tensor(t: torch.Tensor, name: str, dtype: torch.dtype, numel: int) -> torch.Tensor:
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch.Tensor")
    if t.device.type != "cuda":
        raise ValueError(f"{name} must live on a GPU (got {t.device})")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype} (got {t.dtype})")
    if t.numel() != numel:
        raise ValueError(f"{name} must have {numel} elements (got {t.numel()})")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return t


class Solver:
    """One implicit-Euler heat problem on one GPU (one C context, one stream).

    ``precision`` is ``"f32"`` (FP32 vectors, FP64 reductions and gradient) or
    ``"f64"``. ``checkpoint_every = k > 0`` keeps every k-th state and
    recomputes segments in the adjoint; 0 keeps all states. ``cg_variant``
    selects the CG form: 0 two reductions per iteration, 1 one reduction
    (streaming kernel), 2 one reduction with the register-resident kernel
    where the grid fits on the chip, else as 1. ``initial_guess`` is the CG
    starting point of each solve: ``"adaptive"`` (default), ``"projection"``
    (adaptive in the forward sweep, projected onto the last adjoint solutions
    in the adjoint), ``"extrapolate"`` from the last three states, or
    ``"previous"`` state alone. ``periodic``
    wraps the lateral faces, ``robin`` is the back-face Robin coefficient and
    ``jacobi_k > 0`` replaces CG by the paper's fixed-K Jacobi sweeps (App. D.2).
    ``preconditioner_degree`` m >= 2 replaces the Jacobi preconditioner by a
    degree-m Chebyshev polynomial in D^-1 A (CG variant 0).
    """

    def __init__(self, nx: int, ny: int, nz: int, h: Sequence[float] = (1.0, 1.0, 1.0),
                 rtol: float = 1e-6, max_iter: int = 1000, checkpoint_every: int = 0,
                 precision: str = "f32", device: Optional[int] = None,
                 stream: Optional[torch.cuda.Stream] = None, team_blocks_max: int = 0,
                 tile_z: int = 0, profile: bool = False, cg_variant: int = 2,
                 initial_guess: str = "adaptive", periodic: bool = False, robin: float = 0.0,
                 jacobi_k: int = 0, preconditioner_degree: int = 1):
        if precision not in ("f32", "f64"):
            raise ValueError("precision must be 'f32' or 'f64'")
        self.lib = _lib.load()
        self.nx, self.ny, self.nz = int(nx), int(ny), int(nz)
        self.h = tuple(float(v) for v in h)
        self.precision = precision
        self.dtype = torch.float32 if precision == "f32" else torch.float64
        self.device = torch.device("cuda", torch.cuda.current_device() if device is None else device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self._ctx = ctypes.c_void_p()
        _check(self.lib.nh_create(ctypes.byref(self._ctx), self.device.index,
                                  ctypes.c_void_p(self.stream.cuda_stream)), None, "nh_create")
        _check(self.lib.nh_set_grid(self._ctx, self.nx, self.ny, self.nz, *self.h), self._ctx,
               "nh_set_grid")
        self.set_boundary(periodic, robin)
        self.set_jacobi_sweeps(jacobi_k)
        self.set_cg_variant(cg_variant)
        self.set_preconditioner(preconditioner_degree)
        self.set_initial_guess(initial_guess)
        self.set_solver(rtol, max_iter, checkpoint_every)
        if team_blocks_max or tile_z or profile:
            self.set_launch(team_blocks_max, tile_z, profile)
        self.generation = 0
        self.nsteps = 0
        self.last_status = _lib.NH_OK

    # -- configuration ----------------------------------------------------
    def set_solver(self, rtol: float, max_iter: int, checkpoint_every: int = 0):
        _check(self.lib.nh_set_solver(self._ctx, float(rtol), int(max_iter), int(checkpoint_every)),
               self._ctx, "nh_set_solver")
        self.rtol, self.max_iter, self.checkpoint_every = float(rtol), int(max_iter), int(checkpoint_every)

    def set_launch(self, team_blocks_max: int = 0, tile_z: int = 0, profile: bool = False):
        _check(self.lib.nh_set_launch(self._ctx, int(team_blocks_max), int(tile_z), int(bool(profile))),
               self._ctx, "nh_set_launch")

    def set_boundary(self, periodic: bool = False, robin: float = 0.0):
        """Lateral periodic faces and the back-face Robin coefficient h (the
        sink h / hz on the plane k = nz-1); the defaults are zero flux."""
        _check(self.lib.nh_set_boundary(self._ctx, int(bool(periodic)), float(robin)), self._ctx,
               "nh_set_boundary")
        self.periodic, self.robin = bool(periodic), float(robin)

    def set_jacobi_sweeps(self, k: int):
        """0: Jacobi-PCG to rtol; k > 0: exactly k Jacobi sweeps per solve."""
        _check(self.lib.nh_set_jacobi_sweeps(self._ctx, int(k)), self._ctx, "nh_set_jacobi_sweeps")
        self.jacobi_k = int(k)

    def set_cg_variant(self, variant: int):
        _check(self.lib.nh_set_cg_variant(self._ctx, int(variant)), self._ctx, "nh_set_cg_variant")
        self.cg_variant = int(variant)
        if self.cg_variant != 0:
            self.preconditioner_degree = 1

    def set_preconditioner(self, degree: int = 1):
        """1: Jacobi (default); 2..16: a Chebyshev polynomial of that degree in
        D^-1 A (selects CG variant 0)."""
        _check(self.lib.nh_set_preconditioner(self._ctx, int(degree)), self._ctx, "nh_set_preconditioner")
        self.preconditioner_degree = int(degree)
        if self.preconditioner_degree >= 2:
            self.cg_variant = 0

    def set_initial_guess(self, mode: str):
        """``"previous"`` (the last state), ``"extrapolate"`` (from the last
        three states), ``"adaptive"`` (per period of steps, whichever order
        needed the fewest iterations) or ``"projection"`` (adaptive forward;
        each adjoint solve starts from the A-norm projection of its
        right-hand side onto the last adjoint solutions)."""
        modes = {"previous": 0, "extrapolate": 1, "adaptive": 2, "projection": 3}
        if mode not in modes:
            raise ValueError(f"initial_guess must be one of {sorted(modes)}")
        _check(self.lib.nh_set_initial_guess(self._ctx, modes[mode]), self._ctx, "nh_set_initial_guess")
        self.initial_guess = mode

    def set_barrier_timeout(self, seconds: float):
        _check(self.lib.nh_set_barrier_timeout(self._ctx, float(seconds)), self._ctx,
               "nh_set_barrier_timeout")

    @property
    def ng(self) -> int:
        return self.nx * self.ny * self.nz

    # -- solver ------------------------------------------------------------
    def forward(self, alpha: torch.Tensor, q_xy: torch.Tensor, q_t, dt: float, nsteps: int,
                out: Optional[torch.Tensor] = None, allow_noconv: bool = False) -> torch.Tensor:
        """Surface temperature ``[nsteps][ny][nx]`` of the forward sweep."""
        nsteps = int(nsteps)
        _dev_tensor(alpha, "alpha", self.dtype, self.ng)
        _dev_tensor(q_xy, "q_xy", self.dtype, self.nx * self.ny)
        qt = np.ascontiguousarray(np.asarray(q_t, dtype=np.float64).reshape(-1))
        if qt.size != nsteps:
            raise ValueError(f"q_t must have nsteps={nsteps} entries (got {qt.size})")
        if out is None:
            out = torch.empty((nsteps, self.ny, self.nx), dtype=self.dtype, device=self.device)
        _dev_tensor(out, "T_surf", self.dtype, nsteps * self.nx * self.ny)
        fn = self.lib.nh_forward if self.precision == "f32" else self.lib.nh_forward_f64
        code = fn(self._ctx, alpha.data_ptr(), q_xy.data_ptr(),
                  qt.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), float(dt), nsteps,
                  out.data_ptr())
        allow = (_lib.NH_ENOCONV,) if allow_noconv else ()
        self.last_status = _check(code, self._ctx, "nh_forward", allow)
        self.generation += 1
        self.nsteps = nsteps
        return out

    def adjoint(self, dL_dTsurf: torch.Tensor, out: Optional[torch.Tensor] = None,
                allow_noconv: bool = False) -> torch.Tensor:
        """``dL/dalpha`` (float64, ``[nz][ny][nx]``) of the last forward."""
        _dev_tensor(dL_dTsurf, "dL_dTsurf", self.dtype, self.nsteps * self.nx * self.ny)
        if out is None:
            out = torch.empty((self.nz, self.ny, self.nx), dtype=torch.float64, device=self.device)
        _dev_tensor(out, "dL_dalpha", torch.float64, self.ng)
        fn = self.lib.nh_adjoint if self.precision == "f32" else self.lib.nh_adjoint_f64
        code = fn(self._ctx, dL_dTsurf.data_ptr(), out.data_ptr())
        allow = (_lib.NH_ENOCONV,) if allow_noconv else ()
        self.last_status = _check(code, self._ctx, "nh_adjoint", allow)
        return out

    def adjoint_vjp(self, dL_dTsurf: torch.Tensor, allow_noconv: bool = False):
        """``(dL/dalpha, dL/dq, dL/dT0)`` of the last forward: ``dL/dq`` is
        ``[nsteps][ny][nx]`` (``dt * mu^n`` on the top plane, the sensitivity
        to the source of step n) and ``dL/dT0 = mu^1`` is ``[nz][ny][nx]``."""
        _dev_tensor(dL_dTsurf, "dL_dTsurf", self.dtype, self.nsteps * self.nx * self.ny)
        G = torch.empty((self.nz, self.ny, self.nx), dtype=torch.float64, device=self.device)
        dq = torch.empty((self.nsteps, self.ny, self.nx), dtype=self.dtype, device=self.device)
        dT0 = torch.empty((self.nz, self.ny, self.nx), dtype=self.dtype, device=self.device)
        fn = self.lib.nh_adjoint_vjp if self.precision == "f32" else self.lib.nh_adjoint_vjp_f64
        code = fn(self._ctx, dL_dTsurf.data_ptr(), G.data_ptr(), dq.data_ptr(), dT0.data_ptr())
        allow = (_lib.NH_ENOCONV,) if allow_noconv else ()
        self.last_status = _check(code, self._ctx, "nh_adjoint_vjp", allow)
        return G, dq, dT0

    def adjoint_source_grad(self, dL_dTsurf: torch.Tensor, want_qxy: bool = True, want_qt: bool = True,
                            allow_noconv: bool = False):
        """``(dL/dalpha, dL/dq_xy, dL/dq_t)`` of the last forward, all float64
        on the device: the adjoint sweep, then the library's chain rule through
        ``q^n = q_t[n-1] * q_xy`` (``[ny][nx]`` and ``[nsteps]``; ``None``
        when not wanted)."""
        _dev_tensor(dL_dTsurf, "dL_dTsurf", self.dtype, self.nsteps * self.nx * self.ny)
        G = torch.empty((self.nz, self.ny, self.nx), dtype=torch.float64, device=self.device)
        dqxy = torch.empty((self.ny, self.nx), dtype=torch.float64, device=self.device) if want_qxy else None
        dqt = torch.empty(self.nsteps, dtype=torch.float64, device=self.device) if want_qt else None
        fn = self.lib.nh_adjoint_source_grad if self.precision == "f32" else self.lib.nh_adjoint_source_grad_f64
        code = fn(self._ctx, dL_dTsurf.data_ptr(), G.data_ptr(), dqxy.data_ptr() if want_qxy else None,
                  dqt.data_ptr() if want_qt else None)
        allow = (_lib.NH_ENOCONV,) if allow_noconv else ()
        self.last_status = _check(code, self._ctx, "nh_adjoint_source_grad", allow)
        return G, dqxy, dqt

    def get_state(self, n: int) -> torch.Tensor:
        out = torch.empty((self.nz, self.ny, self.nx), dtype=self.dtype, device=self.device)
        _check(self.lib.nh_get_state(self._ctx, int(n), out.data_ptr()), self._ctx, "nh_get_state")
        return out

    def apply_A(self, alpha: torch.Tensor, x: torch.Tensor, dt: float) -> torch.Tensor:
        """``A x`` with the FP32 stencil kernel (operator tests)."""
        _dev_tensor(alpha, "alpha", torch.float32, self.ng)
        _dev_tensor(x, "x", torch.float32, self.ng)
        y = torch.empty_like(x)
        _check(self.lib.nh_apply_A(self._ctx, alpha.data_ptr(), x.data_ptr(), y.data_ptr(), float(dt)),
               self._ctx, "nh_apply_A")
        return y

    def tv(self, alpha: torch.Tensor, eps: float = 1e-6, weight: float = 1.0,
           grad: Optional[torch.Tensor] = None):
        """The TV regulariser of eq. tv_discrete on this grid: returns
        ``(weight * R(alpha), grad)`` with ``grad`` FP64 holding
        ``weight * dR/dalpha`` -- added to the given ``grad`` (e.g. the
        adjoint's dL/dalpha) in place, or in a new tensor."""
        _dev_tensor(alpha, "alpha", self.dtype, self.ng)
        accumulate = grad is not None
        if grad is None:
            grad = torch.empty((self.nz, self.ny, self.nx), dtype=torch.float64, device=self.device)
        else:
            _dev_tensor(grad, "grad", torch.float64, self.ng)
        value = torch.empty(1, dtype=torch.float64, device=self.device)
        fn = self.lib.nh_tv if self.precision == "f32" else self.lib.nh_tv_f64
        _check(fn(self._ctx, alpha.data_ptr(), float(eps), float(weight), value.data_ptr(), grad.data_ptr(),
                  int(accumulate)), self._ctx, "nh_tv")
        return float(value.item()), grad

    def stats(self) -> dict:
        s = _lib.nh_stats()
        _check(self.lib.nh_get_stats(self._ctx, ctypes.byref(s)), self._ctx, "nh_get_stats")
        return s.as_dict()

    def step_iters(self, sweep: str = "forward") -> np.ndarray:
        """CG iterations per step of the last ``"forward"``, ``"adjoint"`` or
        ``"recompute"`` sweep (entry n-1 = step n)."""
        kinds = {"forward": 0, "adjoint": 1, "recompute": 2}
        out = np.zeros(self.nsteps, dtype=np.int32)
        _check(self.lib.nh_get_step_iters(self._ctx, kinds[sweep], out.ctypes.data), self._ctx,
               "nh_get_step_iters")
        return out

    def close(self):
        if getattr(self, "_ctx", None) is not None and self._ctx.value:
            self.lib.nh_destroy(self._ctx)
            self._ctx = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class HeatSolve(torch.autograd.Function):
    """``T_surf = HeatSolve.apply(alpha, solver, q_xy, q_t, dt, nsteps)``.

    Backward runs the library's adjoint sweep and returns ``dL/dalpha`` in
    ``alpha``'s dtype (accumulated in FP64), and, when they require grad, the
    gradients of the source map ``q_xy`` and of the schedule ``q_t`` (a torch
    tensor then) from ``dL/dq^n = dt mu^n`` on the top plane and
    ``q^n = q_t[n-1] q_xy``. If the solver ran another forward in between, the
    forward of this call is recomputed first.
    """

    @staticmethod
    def forward(ctx, alpha, solver: Solver, q_xy, q_t, dt, nsteps):
        a = alpha.detach().to(solver.dtype).contiguous()
        q = q_xy.detach().to(solver.dtype).contiguous()
        qt = q_t.detach().cpu().double().numpy() if isinstance(q_t, torch.Tensor) else q_t
        T = solver.forward(a, q, qt, dt, nsteps)
        ctx.solver = solver
        ctx.gen = solver.generation
        ctx.args = (q, qt, dt, nsteps)
        ctx.dtypes = (alpha.dtype, q_xy.dtype, q_t.dtype if isinstance(q_t, torch.Tensor) else None)
        ctx.q_t_device = q_t.device if isinstance(q_t, torch.Tensor) else None
        ctx.save_for_backward(a)
        return T

    @staticmethod
    def backward(ctx, g):
        solver: Solver = ctx.solver
        (a,) = ctx.saved_tensors
        if solver.generation != ctx.gen:
            solver.forward(a, *ctx.args)
        gg = g.detach().to(solver.dtype).contiguous()
        want_qxy, want_qt = ctx.needs_input_grad[2], ctx.needs_input_grad[3]
        d_qxy = d_qt = None
        if want_qxy or want_qt:
            G, d_qxy, d_qt = solver.adjoint_source_grad(gg, want_qxy, want_qt)
            if d_qxy is not None:
                d_qxy = d_qxy.to(ctx.dtypes[1])
            if d_qt is not None:
                d_qt = d_qt.to(device=ctx.q_t_device, dtype=ctx.dtypes[2])
        else:
            G = solver.adjoint(gg)
        return G.to(ctx.dtypes[0]), None, d_qxy, d_qt, None, None


def heat_solve(alpha, solver: Solver, q_xy, q_t, dt, nsteps):
    return HeatSolve.apply(alpha, solver, q_xy, q_t, dt, nsteps)
