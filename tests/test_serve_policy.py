"""Host-side admission policy of the serving path (no GPU needed).

The server admits queued jobs in arrival order: the longest prefix of the
queue whose device bytes and workgroups, added to those in use, fit the HBM
budget and the co-resident workgroup limit. These tests call the library's
host-only helpers through the C ABI.
"""
import ctypes
import os

import numpy as np
import pytest

from paper_2603_11045_amd import _lib
from paper_2603_11045_amd import workloads as wl


@pytest.fixture(scope="module")
def lib():
    # NH_POLICY_LIB names a standalone build of the host-side policy
    # (csrc/nh_policy.cpp; the sanitizer tier's instrumented build) to test
    # instead of the library
    path = os.environ.get("NH_POLICY_LIB")
    if not path:
        return _lib.load()
    pol = ctypes.CDLL(path)
    ip, szp, dp = ctypes.c_int, ctypes.POINTER(ctypes.c_size_t), ctypes.POINTER(ctypes.c_double)
    pol.nh_serve_job_team.argtypes = [ip, ip, ip, ip, ip]
    pol.nh_serve_job_team.restype = ip
    pol.nh_serve_job_bytes.argtypes = [ip, ip, ip, ip, ip]
    pol.nh_serve_job_bytes.restype = ctypes.c_size_t
    pol.nh_serve_admit_select.argtypes = [szp, ctypes.POINTER(ip), dp, ip, szp, ctypes.POINTER(ip), dp, ip,
                                          ctypes.c_double, ip, ip, ctypes.POINTER(ip)]
    pol.nh_serve_admit_select.restype = ip
    return pol


def select(lib, qbytes, qteams, budget, max_blocks, qdur=None, active=(), backfill=0):
    """Indices the next tick admits; active = [(bytes, team, remaining seconds)]."""
    n = len(qbytes)
    qdur = [1.0] * n if qdur is None else qdur
    qb = (ctypes.c_size_t * max(n, 1))(*qbytes)
    qt = (ctypes.c_int * max(n, 1))(*qteams)
    qd = (ctypes.c_double * max(n, 1))(*qdur)
    m = len(active)
    ab = (ctypes.c_size_t * max(m, 1))(*[a[0] for a in active])
    at = (ctypes.c_int * max(m, 1))(*[a[1] for a in active])
    ar = (ctypes.c_double * max(m, 1))(*[a[2] for a in active])
    sel = (ctypes.c_int * max(n, 1))()
    k = lib.nh_serve_admit_select(qb, qt, qd, n, ab, at, ar, m, float(budget), max_blocks, backfill, sel)
    return [sel[i] for i in range(k)]


def admit(lib, qbytes, qteams, used_bytes, used_blocks, budget, max_blocks):
    """Strict arrival order: the number of jobs admitted from the head."""
    active = [(used_bytes, used_blocks, 1.0)] if (used_bytes or used_blocks) else []
    sel = select(lib, qbytes, qteams, budget, max_blocks, active=active)
    assert sel == list(range(len(sel)))
    return len(sel)


def test_admit_prefix_by_budget(lib):
    assert admit(lib, [10, 10, 10], [1, 1, 1], 0, 0, 25, 100) == 2
    assert admit(lib, [10, 10, 10], [1, 1, 1], 0, 0, 30, 100) == 3
    assert admit(lib, [10, 10, 10], [1, 1, 1], 6, 0, 25, 100) == 1
    assert admit(lib, [10], [1], 20, 0, 25, 100) == 0


def test_admit_prefix_by_workgroups(lib):
    assert admit(lib, [1, 1, 1], [100, 100, 100], 0, 0, 1e18, 256) == 2
    assert admit(lib, [1, 1, 1], [100, 100, 100], 0, 100, 1e18, 256) == 1
    assert admit(lib, [1], [256], 0, 0, 1e18, 256) == 1
    assert admit(lib, [1], [257], 0, 0, 1e18, 256) == 0


def test_strict_order_blocks_behind_the_head(lib):
    assert admit(lib, [100, 1, 1], [1, 1, 1], 0, 0, 50, 100) == 0
    assert admit(lib, [1, 100, 1], [1, 1, 1], 0, 0, 50, 100) == 1


def test_easy_backfill(lib):
    # 196 of 256 workgroups busy: 100 until t = 5 s, 96 until t = 9 s
    active = [(1, 100, 5.0), (1, 96, 9.0)]
    # the 144-workgroup head fits once the first job ends (t = 5): at that
    # time 160 are free, 16 of them to spare
    q_teams = [144, 8, 40, 30, 16, 4]
    q_dur = [3.0, 2.0, 6.0, 4.0, 20.0, 1.0]
    sel = select(lib, [1] * 6, q_teams, 1e18, 256, q_dur, active, backfill=1)
    # job 1 (8, ends at 2 s) and job 3 (30, 4 s) end before t = 5 s; job 2 (40
    # workgroups, 6 s) would delay the head; job 4 (16, 20 s) fits in the
    # spare room; job 5 (4) still fits now but the spare room is used up and it
    # ends before the shadow time, so it goes too
    assert sel == [1, 3, 4, 5]
    # strict order admits nothing
    assert select(lib, [1] * 6, q_teams, 1e18, 256, q_dur, active, backfill=0) == []


def test_easy_backfill_bytes(lib):
    # the memory budget, not workgroups, holds the head back
    active = [(60, 1, 5.0)]
    sel = select(lib, [50, 30, 10], [1, 1, 1], 100, 256, [1.0, 9.0, 9.0], active, backfill=1)
    # head needs 50 of 40 free bytes: shadow 5 s, spare 100 - 50 = 50 bytes;
    # job 1 (30 bytes, 9 s) fits the spare room, job 2 (10 bytes) too
    assert sel == [1, 2]
    sel = select(lib, [50, 30, 25], [1, 1, 1], 100, 256, [1.0, 9.0, 9.0], active, backfill=1)
    # after job 1 only 20 spare bytes remain: job 2 would delay the head
    assert sel == [1]


def test_admit_edge_cases(lib):
    assert select(lib, [], [], 10, 10) == []
    assert lib.nh_serve_admit_select(None, None, None, 3, None, None, None, 0, 10.0, 10, 0, None) == 0


def test_job_team_sizes_streaming(lib):
    # about one workgroup per 32768 voxels, one tile each, capped at half the limit
    teams = {g: lib.nh_serve_job_team(*g, 256, 0) for g in wl.SERVE_GRIDS}
    assert teams[(32, 32, 16)] == 1
    assert teams[(64, 64, 32)] == 4
    assert teams[(96, 96, 32)] == 12
    assert teams[(128, 128, 48)] == 32
    assert teams[(192, 192, 48)] == 72
    for g, t in teams.items():
        ng = g[0] * g[1] * g[2]
        assert 1 <= t <= 128
        assert ng / t <= 2 * 32768 + 1
    assert lib.nh_serve_job_team(192, 192, 48, 64, 0) == 32
    assert lib.nh_serve_job_team(0, 1, 1, 256, 0) == 0
    assert lib.nh_serve_job_team(4, 4, 4, 0, 0) == 0


def test_job_team_sizes_resident(lib):
    # one workgroup per tile of 64 x 8 columns and <= 32 cells in z
    teams = {g: lib.nh_serve_job_team(*g, 256, 1) for g in wl.SERVE_GRIDS}
    assert teams == {(32, 32, 16): 4, (64, 64, 32): 8, (96, 96, 32): 24, (128, 128, 48): 64, (192, 192, 48): 144}
    assert lib.nh_serve_job_team(70, 40, 24, 256, 1) == 10
    assert lib.nh_serve_job_team(96, 20, 40, 256, 1) == 12
    assert lib.nh_serve_job_team(256, 256, 64, 256, 1) == 256
    # larger than the device: not servable in this mode
    assert lib.nh_serve_job_team(256, 256, 65, 256, 1) == 0
    assert lib.nh_serve_job_team(192, 192, 48, 100, 1) == 0


def test_job_bytes(lib):
    for (nx, ny, nz) in wl.SERVE_GRIDS:
        for ns in wl.SERVE_STEPS:
            team = lib.nh_serve_job_team(nx, ny, nz, 256, 1)
            b = lib.nh_serve_job_bytes(nx, ny, nz, ns, team)
            ng, nxy = nx * ny * nz, nx * ny
            floor = 4 * ng * (12 + ns) + 8 * ng + 4 * nxy * (1 + 3 * ns)
            assert floor <= b <= floor + 64 * 1024 + 256 * 30
    # monotone in the number of steps
    assert lib.nh_serve_job_bytes(64, 64, 32, 300, 4) > lib.nh_serve_job_bytes(64, 64, 32, 100, 4)
    assert lib.nh_serve_job_bytes(64, 64, 32, 0, 4) == 0


def test_stream_fits_budget(lib):
    # every job of the serving stream fits the 200 GB budget on its own,
    # and the workgroup limit (not memory) bounds the concurrency
    jobs = wl.serving_stream(n_jobs=40)
    sizes = []
    for j in jobs:
        w = j.workload
        t = lib.nh_serve_job_team(w.nx, w.ny, w.nz, 256, 1)
        sizes.append((lib.nh_serve_job_bytes(w.nx, w.ny, w.nz, w.nsteps, t), t))
    assert max(b for b, _ in sizes) < 200e9
    n = admit(lib, [b for b, _ in sizes], [t for _, t in sizes], 0, 0, 200e9, 256)
    assert 1 <= n < len(jobs)
    assert sum(t for _, t in sizes[:n]) <= 256 < sum(t for _, t in sizes[:n + 1])
