"""Resource use of the hot kernels, read from the compiler's gfx950 output (no
GPU needed): the per-step kernels must keep their whole step inlined, with no
private (scratch) segment and no register spills. A function call or a
scratch copy of the step arguments once slowed the streaming kernel by a third
while every numerical test still passed.

The kernels that run several steps in one launch (the serving kernels and the
batched fixed-K kernel) carry their loop's state on top of a step that uses
the whole register file; they must not call functions, and their spills must
stay within the counts they have today (the resident serving kernel reloads
one value per CG iteration, in the team reduction, and none in its plane
sweeps), so that a change that adds spills shows up here."""
import os
import re
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

from paper_2603_11045_amd import build  # noqa: E402

HOT = {
    "_ZN2nh20resident_step_kernelILi64EEEvNS_8StepArgsIfEE": "resident_step_kernel<64>",
    "_ZN2nh11step_kernelIfEEvNS_8StepArgsIT_EE": "step_kernel<float>",
    "_ZN2nh11step_kernelIdEEvNS_8StepArgsIT_EE": "step_kernel<double>",
}


# multi-step kernels: the most VGPR spills allowed. Their values live across
# the steps of a launch; the reloads sit outside the plane loops (checked in
# the assembly when a budget was set: the serving streaming kernel reloads per
# step, per iteration and per tile, never per plane).
BATCHED = {
    "_ZN2nh21batch_resident_kernelEPKNS_6JobRunEPK15HIP_vector_typeIiLj2EEPNS_7JobProgE": ("batch_resident_kernel", 3),
    "_ZN2nh16batch_run_kernelEPKNS_6JobRunEPK15HIP_vector_typeIiLj2EEPNS_7JobProgE": ("batch_run_kernel", 84),
    "_ZN2nh19jacobi_steps_kernelILi8EEEvNS_8StepArgsIfEENS_8JacStepsE": ("jacobi_steps_kernel<8>", 6),
    "_ZN2nh18jacobi_step_kernelILi8EEEvNS_8StepArgsIfEE": ("jacobi_step_kernel<8>", 0),
}


@pytest.fixture(scope="module")
def asm(tmp_path_factory):
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    if not shutil.which(hipcc):
        pytest.skip("hipcc not available")
    d = tmp_path_factory.mktemp("asm")
    flags = [f for f in build.HIPCC_FLAGS if f not in ("-shared", "-fPIC")]
    text = ""
    for src in ("nh_api.hip", "nh_serve.hip"):
        out = d / (src + ".s")
        cmd = [hipcc, *flags, f"-I{build.INCLUDE}", f"-I{build.CSRC}", "--cuda-device-only", "-S", "-o", str(out),
               os.path.join(build.CSRC, src)]
        res = subprocess.run(cmd, capture_output=True, text=True, timeout=600)
        assert res.returncode == 0, res.stderr[-2000:]
        text += out.read_text() + "\n"
    return text


def kernel_meta(text):
    out = {}
    for part in text.split("amdhsa.kernels:")[1:]:
        out.update(_meta_of(part))
    return out


def _meta_of(meta):
    out = {}
    for blk in re.split(r"\n  - ", meta)[1:]:
        name = re.search(r"\.name:\s+(\S+)", blk)
        if not name:
            continue
        out[name.group(1)] = {
            "private": int(re.search(r"\.private_segment_fixed_size:\s+(\d+)", blk).group(1)),
            "vgpr_spill": int(re.search(r"\.vgpr_spill_count:\s+(\d+)", blk).group(1)),
        }
    return out


def kernel_body(text, sym):
    start = text.index(f"\n{sym}:")
    return text[start:text.index("s_endpgm", start)]


@pytest.mark.parametrize("sym", list(HOT), ids=list(HOT.values()))
def test_step_kernels_are_inlined_without_scratch(asm, sym):
    meta = kernel_meta(asm)
    assert sym in meta, f"{HOT[sym]} not found in the device code"
    assert meta[sym]["private"] == 0, f"{HOT[sym]} uses {meta[sym]['private']} bytes of scratch"
    assert meta[sym]["vgpr_spill"] == 0
    assert "s_swappc" not in kernel_body(asm, sym), f"{HOT[sym]} calls a function"


@pytest.mark.parametrize("sym", list(BATCHED), ids=[v[0] for v in BATCHED.values()])
def test_multi_step_kernels_stay_within_their_spill_budget(asm, sym):
    name, budget = BATCHED[sym]
    meta = kernel_meta(asm)
    assert sym in meta, f"{name} not found in the device code"
    assert meta[sym]["vgpr_spill"] <= budget, f"{name} spills {meta[sym]['vgpr_spill']} VGPRs (budget {budget})"
    assert "s_swappc" not in kernel_body(asm, sym), f"{name} calls a function"
