"""CPU tier under the compiler's sanitizers: the FP64 oracle
(oracle/heat_oracle.c) and the host-only serving policy
(paper_2603_11045_amd/csrc/nh_policy.cpp: a job's tiling and bytes, the checks
of a submitted job, the admission order) are built with gcc's address and
undefined-behaviour sanitizers, and the oracle's pins and the admission-policy
tests run against those builds in a child interpreter with the address
sanitizer's runtime preloaded. Any sanitizer report fails the test."""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = ["-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
       "-fPIC", "-shared"]


def runtime(name):
    p = subprocess.run(["gcc", f"-print-file-name={name}"], capture_output=True, text=True).stdout.strip()
    return p if os.path.isabs(p) and os.path.exists(p) else None


@pytest.fixture(scope="module")
def builds(tmp_path_factory):
    if not shutil.which("gcc") or not shutil.which("g++") or not runtime("libasan.so"):
        pytest.skip("gcc with the address sanitizer runtime is needed")
    d = tmp_path_factory.mktemp("san")
    orc = str(d / "libheat_oracle_san.so")
    pol = str(d / "libnh_policy_san.so")
    for cmd in (["gcc", *SAN, "-std=c11", "-fopenmp", "-o", orc, os.path.join(ROOT, "oracle", "heat_oracle.c"), "-lm"],
                ["g++", *SAN, "-std=c++17", "-I", os.path.join(ROOT, "include"),
                 "-I", os.path.join(ROOT, "paper_2603_11045_amd", "csrc"), "-o", pol,
                 os.path.join(ROOT, "paper_2603_11045_amd", "csrc", "nh_policy.cpp")]):
        r = subprocess.run(cmd, capture_output=True, text=True, timeout=300)
        assert r.returncode == 0, r.stderr[-3000:]
    return orc, pol


def child_env(orc, pol):
    env = dict(os.environ)
    pre = runtime("libasan.so")
    env["LD_PRELOAD"] = pre + (":" + env["LD_PRELOAD"] if env.get("LD_PRELOAD") else "")
    env["ASAN_OPTIONS"] = "detect_leaks=0:halt_on_error=1:abort_on_error=0"
    env["UBSAN_OPTIONS"] = "halt_on_error=1:print_stacktrace=1"
    env["NH_ORACLE_LIB"] = orc
    env["NH_POLICY_LIB"] = pol
    env["OMP_NUM_THREADS"] = "4"
    return env


def test_instrumented_builds_are_the_ones_loaded(builds):
    orc, pol = builds
    code = ("import ctypes, os; ctypes.CDLL(os.environ['NH_ORACLE_LIB']); ctypes.CDLL(os.environ['NH_POLICY_LIB']);"
            "m = open('/proc/self/maps').read(); print('asan' if 'libasan' in m else 'none')")
    r = subprocess.run([sys.executable, "-c", code], env=child_env(orc, pol), capture_output=True, text=True,
                       timeout=120)
    assert r.returncode == 0, r.stderr[-3000:]
    assert r.stdout.strip() == "asan"


def test_oracle_pins_and_admission_policy_under_sanitizers(builds):
    orc, pol = builds
    cmd = [sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider", "-m", "not gpu",
           os.path.join(ROOT, "tests", "test_oracle_pins.py"), os.path.join(ROOT, "tests", "test_serve_policy.py")]
    r = subprocess.run(cmd, env=child_env(orc, pol), capture_output=True, text=True, timeout=900, cwd=ROOT)
    out = r.stdout + r.stderr
    print(out[-2000:])
    assert "ERROR: AddressSanitizer" not in out
    assert "runtime error:" not in out
    assert r.returncode == 0, out[-3000:]
    assert " passed" in out and " failed" not in out
