"""MI355X (gfx950) differentiable implicit-Euler heat solver with a discrete adjoint.

The hot path of neural-field thermal tomography: each step solves
``(I + dt L(alpha)) T^n = T^{n-1} + dt q^n`` with the 7-point harmonic-mean
diffusion operator and zero-flux walls; the adjoint sweep returns
``dL/dalpha``. The work runs in hand-written HIP kernels behind the C ABI of
``include/nefty_heat.h``; ``Solver`` and ``HeatSolve`` are thin bindings.
"""
from .solver import HeatSolve, Solver, heat_solve  # noqa: F401
