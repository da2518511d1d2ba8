"""The C-ABI library loads on any host and exports every symbol of the header."""
import ctypes
import os
import re

from paper_2603_11045_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    with open(os.path.join(ROOT, "include", "nefty_heat.h")) as f:
        text = f.read()
    return sorted(set(re.findall(r"^(?:nh_status|const char \*|void|int|size_t)\s*(nh_\w+)\s*\(", text, re.M)))


def test_header_and_binding_agree():
    assert header_functions() == sorted(_lib.EXPORTED)


def test_library_exports_every_declared_symbol():
    lib = _lib.load()
    for name in header_functions():
        assert getattr(lib, name) is not None, name


def struct_fields(name):
    with open(os.path.join(ROOT, "include", "nefty_heat.h")) as f:
        text = f.read()
    end = text.index("} %s;" % name)
    body = text[text.rindex("typedef struct {", 0, end):end]
    return re.findall(r"\b([a-z_0-9]+)\s*[;,]", re.sub(r"/\*.*?\*/", "", body, flags=re.S))


def test_structs_match_header_fields():
    for cname, py in (("nh_stats", _lib.nh_stats), ("nh_job_info", _lib.nh_job_info),
                      ("nh_server_stats", _lib.nh_server_stats)):
        assert struct_fields(cname) == [n for n, _ in py._fields_], cname


def test_null_context_calls_fail_cleanly():
    lib = _lib.load()
    assert lib.nh_set_grid(None, 4, 4, 4, 1.0, 1.0, 1.0) == _lib.NH_EINVAL
    assert lib.nh_last_error(None) == b"null context"
    assert lib.nh_copy_f32(None, None, 4, None) == _lib.NH_EINVAL
    lib.nh_destroy(None)
    assert lib.nh_server_tick(None, None, None, None, 0, None) == _lib.NH_EINVAL
    assert lib.nh_server_last_error(None) == b"null server"
    assert lib.nh_server_create(None, 0, None, 1e9, 0, 1) == _lib.NH_EINVAL
    lib.nh_server_destroy(None)


def test_library_marks_its_passes_with_roctx_ranges():
    """The forward pass, the adjoint pass, checkpoint segments and serving ticks are
    host-side roctx ranges: the library links the range library and calls it."""
    import subprocess
    path = _lib.load()._name
    undef = subprocess.run(["nm", "-D", "--undefined-only", path], capture_output=True, text=True,
                           check=True).stdout
    assert "roctxRangePushA" in undef and "roctxRangePop" in undef
    needed = subprocess.run(["readelf", "-d", path], capture_output=True, text=True, check=True).stdout
    assert "librocprofiler-sdk-roctx" in needed
    for src, names in (("nh_api.hip", ("nh_forward", "nh_adjoint", "segment recompute", "segment adjoint")),
                       ("nh_serve.hip", ("nh_server_tick",))):
        with open(os.path.join(ROOT, "paper_2603_11045_amd", "csrc", src)) as f:
            text = f.read()
        for n in names:
            assert re.search(r'Range\w*\(?[^;]*"%s' % re.escape(n), text) or ('roctxRangePushA("%s")' % n) in text, n


def test_stream_probe_rejects_bad_arguments():
    """The access-pattern probe checks its arguments before touching the GPU."""
    lib = _lib.load()
    vp = ctypes.c_void_p
    fake_in = (vp * 6)(*[vp(64 * (k + 1)) for k in range(6)])
    fake_out = (vp * 5)(*[vp(64 * (k + 8)) for k in range(5)])
    einval = -1
    assert lib.nh_stream_probe_f32(None, fake_out, 64, 16, 1, None) == einval
    assert lib.nh_stream_probe_f32(fake_in, None, 64, 16, 1, None) == einval
    assert lib.nh_stream_probe_f32(fake_in, fake_out, 65, 16, 1, None) == einval   # nx not a multiple of 64
    assert lib.nh_stream_probe_f32(fake_in, fake_out, 64, 17, 1, None) == einval   # ny not a multiple of 16
    assert lib.nh_stream_probe_f32(fake_in, fake_out, 64, 16, 0, None) == einval
