"""Seeded synthetic inputs for the heat-solver workloads.

This module only draws data: diffusivity fields, source maps, pulse schedules
and job streams. It holds none of the solver's arithmetic, so both the FP64
CPU oracle and the GPU library consume exactly the same arrays.

Layout convention for every volume: ``[nz][ny][nx]`` C-contiguous, x fastest,
``k = 0`` is the heated and observed top face.

The paper's own data (a 64x64x16 synthetic set made with an external
simulator, and two real PVC thermography sets; Sec. 5.1 and App. F) is not
available, so these generators stand in for it: a lognormal background plus
box or ellipsoid inclusions of lower or higher diffusivity mimics the
"1 to 4 subsurface defects in a homogeneous or layered slab" structure of
App. F.1, at the grid sizes of the workloads below.
"""
from __future__ import annotations

import dataclasses
from typing import List, Optional, Tuple

import numpy as np


# --------------------------------------------------------------------------
# diffusivity fields
# --------------------------------------------------------------------------

def lognormal_field(shape: Tuple[int, int, int], sigma: float,
                    rng: np.random.Generator) -> np.ndarray:
    """iid ``exp(sigma * Z)``, ``Z ~ N(0, 1)`` per voxel, float64, shape (nz, ny, nx)."""
    return np.exp(sigma * rng.standard_normal(shape))


def add_cuboids(alpha: np.ndarray, count: int, lo: float, hi: float,
                size_lo: int, size_hi: int, rng: np.random.Generator) -> List[dict]:
    """Overwrite ``count`` axis-aligned boxes with a constant diffusivity each.

    Edge lengths are drawn uniformly from ``{size_lo..size_hi}`` per axis and
    clipped to the grid; the origin is uniform over positions where the box
    fits. Later boxes win where they overlap. Returns the drawn boxes.
    """
    nz, ny, nx = alpha.shape
    boxes = []
    for _ in range(count):
        ex = min(int(rng.integers(size_lo, size_hi + 1)), nx)
        ey = min(int(rng.integers(size_lo, size_hi + 1)), ny)
        ez = min(int(rng.integers(size_lo, size_hi + 1)), nz)
        x0 = int(rng.integers(0, nx - ex + 1))
        y0 = int(rng.integers(0, ny - ey + 1))
        z0 = int(rng.integers(0, nz - ez + 1))
        val = float(rng.uniform(lo, hi))
        alpha[z0:z0 + ez, y0:y0 + ey, x0:x0 + ex] = val
        boxes.append(dict(x0=x0, y0=y0, z0=z0, ex=ex, ey=ey, ez=ez, alpha=val))
    return boxes


def add_ellipsoids(alpha: np.ndarray, count: int, lo: float, hi: float,
                   r_lo: float, r_hi: float, rng: np.random.Generator) -> List[dict]:
    """Overwrite ``count`` ellipsoids (voxel centres inside) with a constant each.

    Centres are uniform over the grid, semi-axes uniform in ``[r_lo, r_hi]``
    voxels per axis; ellipsoids are clipped at the walls, later ones win.
    """
    nz, ny, nx = alpha.shape
    out = []
    for _ in range(count):
        c = rng.uniform([0, 0, 0], [nx, ny, nz])
        r = rng.uniform(r_lo, r_hi, size=3)
        val = float(rng.uniform(lo, hi))
        x0, x1 = max(int(np.floor(c[0] - r[0])), 0), min(int(np.ceil(c[0] + r[0])) + 1, nx)
        y0, y1 = max(int(np.floor(c[1] - r[1])), 0), min(int(np.ceil(c[1] + r[1])) + 1, ny)
        z0, z1 = max(int(np.floor(c[2] - r[2])), 0), min(int(np.ceil(c[2] + r[2])) + 1, nz)
        if x0 >= x1 or y0 >= y1 or z0 >= z1:
            out.append(dict(center=c.tolist(), radii=r.tolist(), alpha=val))
            continue
        zz, yy, xx = np.meshgrid(np.arange(z0, z1) + 0.5, np.arange(y0, y1) + 0.5,
                                 np.arange(x0, x1) + 0.5, indexing="ij")
        inside = (((xx - c[0]) / r[0]) ** 2 + ((yy - c[1]) / r[1]) ** 2
                  + ((zz - c[2]) / r[2]) ** 2) <= 1.0
        sub = alpha[z0:z1, y0:y1, x0:x1]
        sub[inside] = val
        out.append(dict(center=c.tolist(), radii=r.tolist(), alpha=val))
    return out


# --------------------------------------------------------------------------
# sources
# --------------------------------------------------------------------------

def uniform_pulse(ny: int, nx: int, amp: float = 100.0) -> np.ndarray:
    return np.full((ny, nx), amp, dtype=np.float64)


def gaussian_pulse(ny: int, nx: int, sigma: float, amp: float = 100.0) -> np.ndarray:
    """``amp * exp(-((i-cx)^2 + (j-cy)^2) / (2 sigma^2))`` centred on the grid."""
    cx, cy = (nx - 1) / 2.0, (ny - 1) / 2.0
    i = np.arange(nx)[None, :]
    j = np.arange(ny)[:, None]
    return amp * np.exp(-((i - cx) ** 2 + (j - cy) ** 2) / (2.0 * sigma ** 2))


def first_step_schedule(nsteps: int) -> np.ndarray:
    """Pulse on step 1 only: ``q_t[0] = 1``, zero afterwards (float64, host)."""
    q_t = np.zeros(nsteps, dtype=np.float64)
    q_t[0] = 1.0
    return q_t


# --------------------------------------------------------------------------
# workloads
# --------------------------------------------------------------------------

@dataclasses.dataclass
class Workload:
    """One solver problem: inputs plus solver settings.

    ``alpha``/``q_xy`` carry the dtype the GPU path consumes (float32 for the
    mixed-precision path, float64 for the FP64 path); the oracle widens them.
    ``alpha_target`` is the diffusivity whose simulated surface serves as the
    synthetic measurement (the target surface itself is a solver output and
    is computed by whoever needs it).
    """
    name: str
    nx: int
    ny: int
    nz: int
    dt: float
    nsteps: int
    alpha: np.ndarray
    q_xy: np.ndarray
    q_t: np.ndarray
    alpha_target: np.ndarray
    rtol: float
    h: Tuple[float, float, float] = (1.0, 1.0, 1.0)
    checkpoint_every: int = 0
    precision: str = "f32"
    periodic: bool = False                  # lateral x, y faces wrap around
    robin: float = 0.0                      # back-face Robin coefficient (0: adiabatic)
    jacobi_k: int = 0                       # > 0: that many Jacobi sweeps per solve instead of PCG

    @property
    def ng(self) -> int:
        return self.nx * self.ny * self.nz


def _cast(a: np.ndarray, precision: str) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float32 if precision == "f32" else np.float64)


def plain_fp64_16x16x8() -> Workload:
    """16x16x8, 50 steps, dt=2, alpha=1 with one box alpha=0.1 at x,y in [5,10], z in [3,5]
    (inclusive, 0-based), uniform pulse 100 on step 1, rtol 1e-12, FP64 path.
    Target: the same box at alpha=0.2."""
    nx, ny, nz = 16, 16, 8
    a = np.ones((nz, ny, nx))
    a[3:6, 5:11, 5:11] = 0.1
    at = np.ones((nz, ny, nx))
    at[3:6, 5:11, 5:11] = 0.2
    return Workload("plain_fp64_16x16x8", nx, ny, nz, 2.0, 50, _cast(a, "f64"),
                    uniform_pulse(ny, nx), first_step_schedule(50), _cast(at, "f64"),
                    rtol=1e-12, precision="f64")


def mixed_64x64x32(seed: int = 2, nsteps: int = 200) -> Workload:
    """64x64x32, 200 steps, dt=5, lognormal sigma=0.2 plus 4 boxes alpha~U(0.05,0.3),
    edges 4..12; Gaussian pulse sigma=16 on step 1; rtol 1e-6.
    Target: the same field with every box value doubled."""
    nx, ny, nz = 64, 64, 32
    rng = np.random.default_rng(seed)
    a = lognormal_field((nz, ny, nx), 0.2, rng)
    at = a.copy()
    boxes = add_cuboids(a, 4, 0.05, 0.3, 4, 12, rng)
    for b in boxes:
        at[b["z0"]:b["z0"] + b["ez"], b["y0"]:b["y0"] + b["ey"], b["x0"]:b["x0"] + b["ex"]] = 2 * b["alpha"]
    return Workload("mixed_64x64x32", nx, ny, nz, 5.0, nsteps, _cast(a, "f32"),
                    gaussian_pulse(ny, nx, 16.0).astype(np.float32), first_step_schedule(nsteps),
                    _cast(at, "f32"), rtol=1e-6)


def stiff_256x256x64(seed: int = 3, nsteps: int = 1000, nx: int = 256, ny: int = 256,
                     nz: int = 64, n_incl: int = 16) -> Workload:
    """256x256x64, 1000 steps, dt=10, lognormal sigma=0.3 plus 16 ellipsoids
    alpha~U(0.02,0.5); uniform pulse 100 on step 1; rtol 1e-6.
    Target: inclusions redrawn with seed+1000 over the same background."""
    rng = np.random.default_rng(seed)
    base = lognormal_field((nz, ny, nx), 0.3, rng)
    a = base.copy()
    add_ellipsoids(a, n_incl, 0.02, 0.5, 2.0, 8.0, rng)
    at = base.copy()
    add_ellipsoids(at, n_incl, 0.02, 0.5, 2.0, 8.0, np.random.default_rng(seed + 1000))
    return Workload(f"stiff_{nx}x{ny}x{nz}", nx, ny, nz, 10.0, nsteps, _cast(a, "f32"),
                    uniform_pulse(ny, nx).astype(np.float32), first_step_schedule(nsteps),
                    _cast(at, "f32"), rtol=1e-6)


def contrast_256x256x64(seed: int = 3, nsteps: int = 100, nx: int = 256, ny: int = 256, nz: int = 64,
                        n_incl: int = 16) -> Workload:
    """The 256x256x64 background (lognormal sigma=0.3, median 1, dt=10, uniform
    pulse on step 1, rtol 1e-6) with 16 highly conductive ellipsoids
    alpha~U(100,1000): a contrast up to 1:1000, where Jacobi-PCG needs many
    iterations. Target: inclusions redrawn with seed+1000."""
    rng = np.random.default_rng(seed)
    base = lognormal_field((nz, ny, nx), 0.3, rng)
    a = base.copy()
    add_ellipsoids(a, n_incl, 100.0, 1000.0, 2.0, 8.0, rng)
    at = base.copy()
    add_ellipsoids(at, n_incl, 100.0, 1000.0, 2.0, 8.0, np.random.default_rng(seed + 1000))
    return Workload(f"contrast_{nx}x{ny}x{nz}", nx, ny, nz, 10.0, nsteps, _cast(a, "f32"),
                    uniform_pulse(ny, nx).astype(np.float32), first_step_schedule(nsteps),
                    _cast(at, "f32"), rtol=1e-6)


def long_512x512x64(seed: int = 4, nsteps: int = 2000, checkpoint_every: int = 64,
                    nx: int = 512, ny: int = 512, nz: int = 64) -> Workload:
    """512x512x64, 2000 steps, dt=10, lognormal sigma=0.2 plus 64 boxes
    alpha~U(0.05,0.3), edges 4..12; uniform pulse; rtol 1e-6; checkpoint every 64."""
    rng = np.random.default_rng(seed)
    a = lognormal_field((nz, ny, nx), 0.2, rng)
    at = a.copy()
    boxes = add_cuboids(a, 64, 0.05, 0.3, 4, 12, rng)
    for b in boxes:
        at[b["z0"]:b["z0"] + b["ez"], b["y0"]:b["y0"] + b["ey"], b["x0"]:b["x0"] + b["ex"]] = 2 * b["alpha"]
    return Workload(f"long_{nx}x{ny}x{nz}", nx, ny, nz, 10.0, nsteps, _cast(a, "f32"),
                    uniform_pulse(ny, nx).astype(np.float32), first_step_schedule(nsteps),
                    _cast(at, "f32"), rtol=1e-6, checkpoint_every=checkpoint_every)


def add_defects(alpha: np.ndarray, count: int, lo: float, hi: float,
                rng: np.random.Generator) -> List[dict]:
    """Overwrite ``count`` buried defects, each an ellipsoid, a vertical
    cylinder or a box (kind uniform), with a constant diffusivity ~U(lo, hi).

    Lateral extents are 3..10 voxels (semi-axis or radius) or 6..20 (box
    edge), through-thickness extents 2..6 voxels; the top of each defect lies
    at depth 1..nz/2 and every defect is clipped at the walls. Later defects
    win where they overlap.
    """
    nz, ny, nx = alpha.shape
    zc, yc, xc = np.meshgrid(np.arange(nz) + 0.5, np.arange(ny) + 0.5, np.arange(nx) + 0.5,
                             indexing="ij")
    out = []
    for _ in range(count):
        kind = ("ellipsoid", "cylinder", "box")[int(rng.integers(0, 3))]
        val = float(rng.uniform(lo, hi))
        cx, cy = rng.uniform(0, nx), rng.uniform(0, ny)
        ez = float(rng.uniform(2, 6))
        top = float(rng.uniform(1, max(nz // 2, 2)))
        if kind == "ellipsoid":
            rx, ry = rng.uniform(3, 10, size=2)
            cz = top + ez / 2
            inside = (((xc - cx) / rx) ** 2 + ((yc - cy) / ry) ** 2 + ((zc - cz) / (ez / 2)) ** 2) <= 1.0
        elif kind == "cylinder":
            r = float(rng.uniform(3, 10))
            inside = ((xc - cx) ** 2 + (yc - cy) ** 2 <= r * r) & (zc >= top) & (zc <= top + ez)
        else:
            ex, ey = rng.uniform(6, 20, size=2)
            inside = ((np.abs(xc - cx) <= ex / 2) & (np.abs(yc - cy) <= ey / 2)
                      & (zc >= top) & (zc <= top + ez))
        alpha[inside] = val
        out.append(dict(kind=kind, alpha=val, center=(cx, cy), top=top, thickness=ez))
    return out


def paper_64x64x16(seed: int = 6, nsteps: int = 50, layered: bool = False, jacobi_k: int = 50,
                   robin: float = 0.0, periodic: bool = True, precision: str = "f32") -> Workload:
    """The paper's synthetic specimen shape (App. E, Table 5): 64x64x16 on
    [0,10]^2 x [0,1] (dx = dy = 0.156, dz = 0.0625), dt = 0.05, lateral
    periodic faces, adiabatic or Robin back face, K = 50 Jacobi sweeps per
    solve; 50 steps as in the solver benchmark of Table 4 (100 frames in the
    training set-up). Bulk alpha ~U(0.1, 0.2), constant or in 3..4 strata
    along z (layered); 1..4 buried defects alpha ~U(0.005, 0.015). Uniform
    pulse 100 on step 1. Target: the defects redrawn from seed + 1000 over
    the same bulk."""
    nx, ny, nz = 64, 64, 16
    rng = np.random.default_rng(seed)
    if layered:
        nl = int(rng.integers(3, 5))
        cuts = np.sort(rng.choice(np.arange(2, nz - 1), size=nl - 1, replace=False))
        vals = rng.uniform(0.1, 0.2, size=nl)
        prof = np.empty(nz)
        edges = [0] + cuts.tolist() + [nz]
        for l in range(nl):
            prof[edges[l]:edges[l + 1]] = vals[l]
        bulk = np.broadcast_to(prof[:, None, None], (nz, ny, nx)).copy()
    else:
        bulk = np.full((nz, ny, nx), float(rng.uniform(0.1, 0.2)))
    a = bulk.copy()
    add_defects(a, int(rng.integers(1, 5)), 0.005, 0.015, rng)
    at = bulk.copy()
    trng = np.random.default_rng(seed + 1000)
    add_defects(at, int(trng.integers(1, 5)), 0.005, 0.015, trng)
    name = f"paper_{nx}x{ny}x{nz}" + ("_layered" if layered else "") + ("_robin" if robin else "")
    qdt = np.float64 if precision == "f64" else np.float32
    return Workload(name, nx, ny, nz, 0.05, nsteps, _cast(a, precision),
                    uniform_pulse(ny, nx).astype(qdt), first_step_schedule(nsteps),
                    _cast(at, precision), rtol=1e-6, h=(0.156, 0.156, 0.0625), precision=precision,
                    periodic=periodic, robin=robin, jacobi_k=jacobi_k)


SERVE_GRIDS = [(32, 32, 16), (64, 64, 32), (96, 96, 32), (128, 128, 48), (192, 192, 48)]
SERVE_STEPS = [100, 300, 600]


@dataclasses.dataclass
class JobSpec:
    job_id: int
    arrival_s: float
    workload: Workload


def serving_stream(n_jobs: int = 200, rate: float = 20.0, seed: int = 5,
                   grids=None, steps=None, dt: float = 5.0) -> List[JobSpec]:
    """Poisson stream of forward+adjoint jobs: exponential inter-arrival times
    at ``rate`` jobs/s; grid uniform over ``grids``; steps uniform over
    ``steps``; lognormal sigma=0.25 with 1..8 boxes alpha~U(0.05,0.3);
    uniform pulse on step 1; rtol 1e-6. Target: box values doubled."""
    grids = SERVE_GRIDS if grids is None else grids
    steps = SERVE_STEPS if steps is None else steps
    rng = np.random.default_rng(seed)
    t = 0.0
    jobs = []
    for j in range(n_jobs):
        t += float(rng.exponential(1.0 / rate))
        nx, ny, nz = grids[int(rng.integers(0, len(grids)))]
        ns = int(steps[int(rng.integers(0, len(steps)))])
        jrng = np.random.default_rng([seed, j])
        a = lognormal_field((nz, ny, nx), 0.25, jrng)
        at = a.copy()
        boxes = add_cuboids(a, int(jrng.integers(1, 9)), 0.05, 0.3, 4, 12, jrng)
        for b in boxes:
            at[b["z0"]:b["z0"] + b["ez"], b["y0"]:b["y0"] + b["ey"], b["x0"]:b["x0"] + b["ex"]] = 2 * b["alpha"]
        w = Workload(f"job{j}_{nx}x{ny}x{nz}", nx, ny, nz, dt, ns, _cast(a, "f32"),
                     uniform_pulse(ny, nx).astype(np.float32), first_step_schedule(ns),
                     _cast(at, "f32"), rtol=1e-6)
        jobs.append(JobSpec(j, t, w))
    return jobs


def random_field(shape, seed: int, lo: float = 0.5, hi: float = 2.0,
                 dtype=np.float64) -> np.ndarray:
    """Uniform random positive field (for operator-level tests)."""
    rng = np.random.default_rng(seed)
    return rng.uniform(lo, hi, size=shape).astype(dtype)


def random_surface_weights(nsteps: int, ny: int, nx: int, seed: int,
                           dtype=np.float64) -> np.ndarray:
    """Standard-normal ``[nsteps][ny][nx]`` array (a synthetic dL/dT_surf)."""
    rng = np.random.default_rng(seed)
    return rng.standard_normal((nsteps, ny, nx)).astype(dtype)


def small_problem(nx: int, ny: int, nz: int, nsteps: int, seed: int, dt: float = 1.0,
                  sigma: float = 0.5, precision: str = "f64", pulse_steps: Optional[int] = None,
                  rtol: float = 1e-12) -> Workload:
    """A small random problem for tests: lognormal alpha, random positive top
    source, pulses on the first ``pulse_steps`` steps with random weights."""
    rng = np.random.default_rng(seed)
    a = lognormal_field((nz, ny, nx), sigma, rng)
    at = lognormal_field((nz, ny, nx), sigma, rng)
    q = rng.uniform(0.0, 10.0, size=(ny, nx))
    ps = nsteps if pulse_steps is None else pulse_steps
    q_t = np.zeros(nsteps)
    q_t[:ps] = rng.uniform(0.2, 1.0, size=ps)
    return Workload(f"small_{nx}x{ny}x{nz}_s{seed}", nx, ny, nz, dt, nsteps, _cast(a, precision),
                    _cast(q, precision), q_t, _cast(at, precision), rtol=rtol, precision=precision)
