"""Every kernel of the library runs from replayed HIP graphs as well as from
eager launches, and all of them are kept free of private (scratch) memory:
no register spills to memory and no stack.  Compile the kernel sources for
gfx950 exactly as the library build does, with the compiler's resource-usage
remarks switched on, and check every kernel's figures.  (A scalar register
spilled into a vector register lane uses no memory and is allowed.)"""
import os
import re
import shutil
import subprocess

import pytest

from paper_2609_31980_amd import build as B

CSRC = os.path.join(os.path.dirname(os.path.abspath(__file__)), "..", "paper_2609_31980_amd", "csrc")
HIP_SOURCES = [s for s in B.SOURCES if s.endswith(".hip")]

FIELD = re.compile(r"remark:\s+(Function Name|ScratchSize \[bytes/lane\]|VGPRs Spill|Dynamic Stack|VGPRs|"
                   r"Occupancy \[waves/SIMD\]):\s*(\S+)")


def resource_usage(src):
    """{kernel: {field: value}} from the compiler's resource-usage remarks."""
    cmd = [B.HIPCC, "-x", "hip", *B.FLAGS, "--cuda-device-only", "-Rpass-analysis=kernel-resource-usage",
           "-I", CSRC, "-c", os.path.join(CSRC, src), "-o", os.devnull]
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=900)
    assert r.returncode == 0, r.stderr[-2000:]
    out, cur = {}, None
    for m in FIELD.finditer(r.stderr):
        k, v = m.group(1), m.group(2)
        if k == "Function Name":
            cur = v
            out[cur] = {}
        elif cur is not None:
            out[cur][k] = v
    return out


def check_no_scratch(usage):
    bad = []
    for name, f in usage.items():
        if f.get("ScratchSize [bytes/lane]", "0") != "0" or f.get("VGPRs Spill", "0") != "0" \
                or f.get("Dynamic Stack", "False") != "False":
            bad.append(f"{name}: scratch {f.get('ScratchSize [bytes/lane]')} B/lane, "
                       f"VGPR spill {f.get('VGPRs Spill')}, dynamic stack {f.get('Dynamic Stack')}")
    return bad


@pytest.mark.skipif(not os.path.exists(B.HIPCC) and shutil.which(B.HIPCC) is None, reason="hipcc not found")
@pytest.mark.parametrize("src", HIP_SOURCES)
def test_kernels_use_no_scratch(src):
    usage = resource_usage(src)
    assert usage, f"no resource-usage remarks parsed for {src}"
    bad = check_no_scratch(usage)
    assert not bad, "kernels with scratch memory:\n" + "\n".join(bad)


def test_detector_fires_on_a_spilling_kernel(tmp_path):
    """Control: a kernel forced to spill is reported."""
    src = tmp_path / "spill.hip"
    src.write_text(
        "#include <hip/hip_runtime.h>\n"
        "__global__ void __attribute__((amdgpu_num_vgpr(24))) spill(float *p, const int *k) {\n"
        "  float v[48];\n"
        "  #pragma unroll\n"
        "  for (int i = 0; i < 48; ++i) v[i] = p[threadIdx.x + i * 256];\n"
        "  float s = 0.f;\n"
        "  #pragma unroll\n"
        "  for (int i = 0; i < 48; ++i) s += v[i] * v[(i * 7) % 48];\n"
        "  p[threadIdx.x] = s + v[k[threadIdx.x] % 48];\n"
        "}\n")
    cmd = [B.HIPCC, "-x", "hip", *B.FLAGS, "--cuda-device-only", "-Rpass-analysis=kernel-resource-usage",
           "-c", str(src), "-o", os.devnull]
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr[-2000:]
    usage, cur = {}, None
    for m in FIELD.finditer(r.stderr):
        if m.group(1) == "Function Name":
            cur = m.group(2)
            usage[cur] = {}
        else:
            usage[cur][m.group(1)] = m.group(2)
    assert check_no_scratch(usage), "the spilling control kernel was not detected"
