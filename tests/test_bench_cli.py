"""bench.py's command-line contract that needs no GPU: more than one GPU is
refused with a message and a non-zero exit; the options and the recipe of the
high-contrast workload."""
import os
import subprocess
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_bench_help_lists_the_solver_options():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--help"], capture_output=True, text=True,
                       timeout=120)
    assert r.returncode == 0
    for opt in ("--workload", "--guess", "--cheb", "--variant", "--nsteps", "--cpu-threads"):
        assert opt in r.stdout


def test_contrast_workload_recipe():
    """The 1:1000-contrast workload: the 256x256x64 background with 16
    conductive ellipsoids alpha in [100, 1000], 100 steps by default."""
    sys.path.insert(0, ROOT)
    from paper_2603_11045_amd import workloads as wl

    w = wl.contrast_256x256x64(nx=64, ny=64, nz=16, n_incl=4, nsteps=5)
    assert (w.nz, w.ny, w.nx) == w.alpha.shape == (16, 64, 64) and w.nsteps == 5 and w.dt == 10.0
    hi = w.alpha[w.alpha >= 100.0]
    assert hi.size > 0 and hi.max() <= 1000.0
    assert float(w.alpha.min()) > 0.0 and np.isfinite(w.alpha).all()
    assert not np.array_equal(w.alpha, w.alpha_target)
