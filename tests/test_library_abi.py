"""The C-ABI library loads on any host and exports every symbol of the header."""
import ctypes
import os
import re

from paper_2603_11045_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    with open(os.path.join(ROOT, "include", "nefty_heat.h")) as f:
        text = f.read()
    return sorted(set(re.findall(r"^(?:nh_status|const char \*|void)\s*(nh_\w+)\s*\(", text, re.M)))


def test_header_and_binding_agree():
    assert header_functions() == sorted(_lib.EXPORTED)


def test_library_exports_every_declared_symbol():
    lib = _lib.load()
    for name in header_functions():
        assert getattr(lib, name) is not None, name


def test_stats_struct_matches_header_fields():
    with open(os.path.join(ROOT, "include", "nefty_heat.h")) as f:
        text = f.read()
    body = text[text.index("typedef struct {"):text.index("} nh_stats;")]
    fields = re.findall(r"\b([a-z_0-9]+)\s*[;,]", re.sub(r"/\*.*?\*/", "", body, flags=re.S))
    assert fields == [n for n, _ in _lib.nh_stats._fields_]


def test_null_context_calls_fail_cleanly():
    lib = _lib.load()
    assert lib.nh_set_grid(None, 4, 4, 4, 1.0, 1.0, 1.0) == _lib.NH_EINVAL
    assert lib.nh_last_error(None) == b"null context"
    assert lib.nh_copy_f32(None, None, 4, None) == _lib.NH_EINVAL
    lib.nh_destroy(None)
