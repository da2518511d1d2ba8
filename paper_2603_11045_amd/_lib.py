"""ctypes binding of ``libnefty_heat.so`` (declared in ``include/nefty_heat.h``).

Argument marshalling only: every function forwards to the C entry point of
the same name. Importing this module loads the in-tree library and raises if
it has not been built; there is no fallback implementation.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libnefty_heat.so")

NH_OK = 0
NH_EINVAL = -1
NH_ENOMEM = -2
NH_ESTATE = -3
NH_ENOCONV = -4
NH_ENONFINITE = -5
NH_EHIP = -6
NH_ETIMEOUT = -7

STATUS_NAMES = {0: "NH_OK", -1: "NH_EINVAL", -2: "NH_ENOMEM", -3: "NH_ESTATE", -4: "NH_ENOCONV",
                -5: "NH_ENONFINITE", -6: "NH_EHIP", -7: "NH_ETIMEOUT"}

EXPORTED = ["nh_create", "nh_set_grid", "nh_set_solver", "nh_forward", "nh_adjoint",
            "nh_forward_f64", "nh_adjoint_f64", "nh_adjoint_vjp", "nh_adjoint_vjp_f64",
            "nh_adjoint_source_grad", "nh_adjoint_source_grad_f64", "nh_get_state", "nh_apply_A", "nh_tv", "nh_tv_f64", "nh_tv_noalloc", "nh_set_launch",
            "nh_set_boundary", "nh_set_jacobi_sweeps", "nh_set_cg_variant", "nh_set_preconditioner", "nh_set_initial_guess", "nh_set_barrier_timeout", "nh_get_stats", "nh_get_step_iters", "nh_last_error", "nh_destroy", "nh_copy_f32", "nh_stream_probe_f32",
            "nh_server_create", "nh_server_submit", "nh_server_tick", "nh_server_job", "nh_server_release",
            "nh_server_get_stats", "nh_server_last_error", "nh_server_destroy", "nh_serve_job_team",
            "nh_serve_job_bytes", "nh_serve_admit_select", "nh_server_set_slice",
            "nh_server_set_backfill"]

NH_JOB_QUEUED, NH_JOB_FORWARD, NH_JOB_ADJOINT, NH_JOB_DONE, NH_JOB_FAILED = range(5)
JOB_STATE_NAMES = {0: "queued", 1: "forward", 2: "adjoint", 3: "done", 4: "failed"}


class nh_stats(ctypes.Structure):
    _fields_ = [
        ("fwd_iters", ctypes.c_longlong),
        ("adj_iters", ctypes.c_longlong),
        ("recompute_iters", ctypes.c_longlong),
        ("fwd_steps", ctypes.c_int),
        ("adj_steps", ctypes.c_int),
        ("recompute_steps", ctypes.c_int),
        ("max_step_iters", ctypes.c_int),
        ("worst_rel_res", ctypes.c_double),
        ("bytes_alg_fwd", ctypes.c_double),
        ("bytes_alg_adj", ctypes.c_double),
        ("t_fwd_s", ctypes.c_double),
        ("t_adj_s", ctypes.c_double),
        ("t_kernel_fwd_s", ctypes.c_double),
        ("t_kernel_adj_s", ctypes.c_double),
        ("launches_fwd", ctypes.c_longlong),
        ("launches_adj", ctypes.c_longlong),
        ("workspace_bytes", ctypes.c_size_t),
        ("peak_workspace_bytes", ctypes.c_size_t),
        ("team_blocks", ctypes.c_int),
        ("block_threads", ctypes.c_int),
        ("tile_x", ctypes.c_int),
        ("tile_y", ctypes.c_int),
        ("tile_z", ctypes.c_int),
        ("resident", ctypes.c_int),
        ("resident_occupancy", ctypes.c_int),
        ("jacobi_blocked", ctypes.c_int),
    ]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


class nh_job_info(ctypes.Structure):
    _fields_ = [
        ("state", ctypes.c_int),
        ("status", ctypes.c_int),
        ("team_blocks", ctypes.c_int),
        ("nsteps", ctypes.c_int),
        ("fwd_iters", ctypes.c_longlong),
        ("adj_iters", ctypes.c_longlong),
        ("loss", ctypes.c_double),
        ("t_submit_s", ctypes.c_double),
        ("t_admit_s", ctypes.c_double),
        ("t_done_s", ctypes.c_double),
        ("device_bytes", ctypes.c_size_t),
    ]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


class nh_server_stats(ctypes.Structure):
    _fields_ = [
        ("ticks", ctypes.c_longlong),
        ("kernel_s", ctypes.c_double),
        ("used_bytes", ctypes.c_size_t),
        ("used_blocks", ctypes.c_int),
        ("max_blocks", ctypes.c_int),
        ("active", ctypes.c_int),
        ("queued", ctypes.c_int),
        ("jobs_done", ctypes.c_longlong),
        ("voxel_steps", ctypes.c_double),
        ("cg_iters", ctypes.c_longlong),
        ("busy_block_s", ctypes.c_double),
        ("span_block_s", ctypes.c_double),
    ]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


class NHError(RuntimeError):
    def __init__(self, code: int, func: str, msg: str):
        super().__init__(f"{func}: {STATUS_NAMES.get(code, code)}: {msg}")
        self.code = code


_lib = None


def load():
    """Load the library (once). Raises if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with "
                          "`python -m paper_2603_11045_amd.build` (hipcc, gfx950)")
    lib = ctypes.CDLL(LIB_PATH)
    vp, ip, dp = ctypes.c_void_p, ctypes.c_int, ctypes.c_double
    st = ctypes.c_int
    lib.nh_create.argtypes = [ctypes.POINTER(vp), ip, vp]
    lib.nh_set_grid.argtypes = [vp, ip, ip, ip, dp, dp, dp]
    lib.nh_set_solver.argtypes = [vp, dp, ip, ip]
    lib.nh_forward.argtypes = [vp, vp, vp, ctypes.POINTER(dp), dp, ip, vp]
    lib.nh_adjoint.argtypes = [vp, vp, vp]
    lib.nh_forward_f64.argtypes = [vp, vp, vp, ctypes.POINTER(dp), dp, ip, vp]
    lib.nh_adjoint_f64.argtypes = [vp, vp, vp]
    lib.nh_adjoint_vjp.argtypes = [vp, vp, vp, vp, vp]
    lib.nh_adjoint_vjp_f64.argtypes = [vp, vp, vp, vp, vp]
    lib.nh_adjoint_source_grad.argtypes = [vp, vp, vp, vp, vp]
    lib.nh_adjoint_source_grad_f64.argtypes = [vp, vp, vp, vp, vp]
    lib.nh_get_state.argtypes = [vp, ip, vp]
    lib.nh_apply_A.argtypes = [vp, vp, vp, vp, dp]
    lib.nh_tv.argtypes = [vp, vp, dp, dp, vp, vp, ip]
    lib.nh_tv_f64.argtypes = [vp, vp, dp, dp, vp, vp, ip]
    lib.nh_tv_noalloc.argtypes = [vp, vp, dp, dp, vp, vp, ip]
    lib.nh_set_launch.argtypes = [vp, ip, ip, ip]
    lib.nh_set_boundary.argtypes = [vp, ip, ctypes.c_double]
    lib.nh_set_jacobi_sweeps.argtypes = [vp, ip]
    lib.nh_set_cg_variant.argtypes = [vp, ip]
    lib.nh_set_initial_guess.argtypes = [vp, ip]
    lib.nh_set_preconditioner.argtypes = [vp, ip]
    lib.nh_set_barrier_timeout.argtypes = [vp, dp]
    lib.nh_get_stats.argtypes = [vp, ctypes.POINTER(nh_stats)]
    lib.nh_get_step_iters.argtypes = [vp, ip, vp]
    lib.nh_last_error.argtypes = [vp]
    lib.nh_last_error.restype = ctypes.c_char_p
    lib.nh_destroy.argtypes = [vp]
    lib.nh_destroy.restype = None
    lib.nh_copy_f32.argtypes = [vp, vp, ctypes.c_size_t, vp]
    lib.nh_stream_probe_f32.argtypes = [ctypes.POINTER(vp), ctypes.POINTER(vp), ctypes.c_int, ctypes.c_int,
                                        ctypes.c_int, vp]
    llp = ctypes.POINTER(ctypes.c_longlong)
    lib.nh_server_create.argtypes = [ctypes.POINTER(vp), ip, vp, dp, ip, ip]
    lib.nh_server_submit.argtypes = [vp, ip, ip, ip, dp, dp, ip, dp, ip, vp, vp, vp, vp, llp]
    lib.nh_server_tick.argtypes = [vp, ctypes.POINTER(ip), ctypes.POINTER(ip), llp, ip, ctypes.POINTER(ip)]
    lib.nh_server_job.argtypes = [vp, ctypes.c_longlong, ctypes.POINTER(nh_job_info), vp]
    lib.nh_server_release.argtypes = [vp, ctypes.c_longlong]
    lib.nh_server_set_slice.argtypes = [vp, ip]
    lib.nh_server_get_stats.argtypes = [vp, ctypes.POINTER(nh_server_stats)]
    lib.nh_server_last_error.argtypes = [vp]
    lib.nh_server_last_error.restype = ctypes.c_char_p
    lib.nh_server_destroy.argtypes = [vp]
    lib.nh_server_destroy.restype = None
    lib.nh_serve_job_team.argtypes = [ip, ip, ip, ip, ip]
    lib.nh_serve_job_team.restype = ip
    lib.nh_serve_job_bytes.argtypes = [ip, ip, ip, ip, ip]
    lib.nh_serve_job_bytes.restype = ctypes.c_size_t
    szp, dpp = ctypes.POINTER(ctypes.c_size_t), ctypes.POINTER(dp)
    lib.nh_serve_admit_select.argtypes = [szp, ctypes.POINTER(ip), dpp, ip, szp, ctypes.POINTER(ip), dpp, ip,
                                          dp, ip, ip, ctypes.POINTER(ip)]
    lib.nh_serve_admit_select.restype = ip
    lib.nh_server_set_backfill.argtypes = [vp, ip]
    for name in EXPORTED:
        f = getattr(lib, name)
        if name not in ("nh_last_error", "nh_destroy", "nh_server_last_error", "nh_server_destroy",
                        "nh_serve_job_team", "nh_serve_job_bytes", "nh_serve_admit_select"):
            f.restype = st
    _lib = lib
    return lib


def last_error(ctx) -> str:
    return load().nh_last_error(ctx).decode(errors="replace")


def server_last_error(srv) -> str:
    return load().nh_server_last_error(srv).decode(errors="replace")
