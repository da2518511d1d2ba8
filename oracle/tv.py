"""FP64 reference of the discrete total-variation regulariser (eq. tv_discrete, App. D.1).

TEST INFRASTRUCTURE ONLY: used by the test suite and the smoke check, never by
the product path, and sharing no code with the GPU library.

    R(a) = dx dy dz sum_{i,j,k} sqrt( (dx_a / dx)^2 + (dy_a / dy)^2 + (dz_a / dz)^2 + eps^2 )

with forward differences along each axis of the array index: dx_a and dy_a
wrap around (lateral periodicity), dz_a = a[k+1] - a[k] for k < nz-1 and 0 on
the last plane. Layout [nz][ny][nx], x fastest, as everywhere else.
"""
from __future__ import annotations

import numpy as np


def _diffs(a):
    """Forward differences (dx, dy, dz) of a [nz][ny][nx] array."""
    dxa = np.roll(a, -1, axis=2) - a
    dya = np.roll(a, -1, axis=1) - a
    dza = np.zeros_like(a)
    dza[:-1] = a[1:] - a[:-1]
    return dxa, dya, dza


def tv_value(alpha, h=(1.0, 1.0, 1.0), eps=1e-6) -> float:
    """R(alpha) of eq. tv_discrete."""
    a = np.asarray(alpha, dtype=np.float64)
    dxa, dya, dza = _diffs(a)
    t = np.sqrt((dxa / h[0]) ** 2 + (dya / h[1]) ** 2 + (dza / h[2]) ** 2 + eps * eps)
    return float(h[0] * h[1] * h[2] * t.sum())


def tv_grad(alpha, h=(1.0, 1.0, 1.0), eps=1e-6) -> np.ndarray:
    """dR/dalpha: each cell's term t = sqrt(...) depends on the cell itself and
    on its +x, +y (wrapped) and +z neighbours; d t / d(forward neighbour) =
    (difference / h^2) / t and d t / d(cell) is minus the sum of those."""
    a = np.asarray(alpha, dtype=np.float64)
    dxa, dya, dza = _diffs(a)
    t = np.sqrt((dxa / h[0]) ** 2 + (dya / h[1]) ** 2 + (dza / h[2]) ** 2 + eps * eps)
    gx = dxa / (h[0] ** 2 * t)
    gy = dya / (h[1] ** 2 * t)
    gz = dza / (h[2] ** 2 * t)
    g = -(gx + gy + gz)
    g += np.roll(gx, 1, axis=2)          # the cell is the +x neighbour of the cell before it
    g += np.roll(gy, 1, axis=1)
    g[1:] += gz[:-1]
    return h[0] * h[1] * h[2] * g
