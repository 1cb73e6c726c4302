"""The distance must be three separately rounded FP32 operations per axis
(Sec. 4.2: a fused or reassociated sum changes float32 membership near the
radius), and cell coordinates are one float64 subtract and one multiply.
Compile the kernels for gfx950 exactly as the library build does and check
the device assembly: no fused multiply-add in the kernels that evaluate
distances or cell coordinates, and no packed FP32 anywhere.  (Other kernels
hold FMAs only inside the compiler's expansions of integer division and of
correctly rounded float64 division.)"""
import os
import re
import shutil
import subprocess
from collections import Counter

import pytest

from paper_2609_31980_amd import build as B

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "..", "paper_2609_31980_amd", "csrc", "frnn_kernels.hip")
FMA = re.compile(r"\b(v_fma\w*|v_fmac\w*|v_fmamk\w*|v_fmaak\w*|v_mac_f32\w*|v_mad_f32\w*)\b")
PACKED = re.compile(r"\bv_pk_\w*_f32\w*\b")
EXACT_KERNELS = ("k_query", "k_short_rows", "k_keys", "k_scatter")


def device_asm(tmp_path):
    out = tmp_path / "k.s"
    cmd = [B.HIPCC, "-x", "hip", *B.FLAGS, "--cuda-device-only", "-S", "-I", os.path.dirname(SRC), SRC,
           "-o", str(out)]
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stderr[-2000:]
    asm = out.read_text()
    labels = [(m.start(), m.group(1)) for m in re.finditer(r"^(_ZN4frnn\w+):", asm, re.M)]
    return {name: asm[pos:(labels[i + 1][0] if i + 1 < len(labels) else len(asm))]
            for i, (pos, name) in enumerate(labels)}


@pytest.mark.skipif(not os.path.exists(B.HIPCC) and shutil.which(B.HIPCC) is None, reason="hipcc not found")
def test_distance_kernels_have_no_fma_or_packed_fp32(tmp_path):
    funcs = device_asm(tmp_path)
    exact = [n for n in funcs if any(k in n for k in EXACT_KERNELS)]
    assert sum("k_query" in n for n in exact) >= 6, "query kernels not found in the assembly"
    for n in exact:
        bad = Counter(FMA.findall(funcs[n]))
        assert not bad, f"{n}: fused multiply-add {dict(bad)}"
    for n, body in funcs.items():
        bad = Counter(PACKED.findall(body))
        assert not bad, f"{n}: packed FP32 {dict(bad)}"


@pytest.mark.skipif(not os.path.exists(B.HIPCC) and shutil.which(B.HIPCC) is None, reason="hipcc not found")
def test_detector_sees_contraction_when_allowed(tmp_path):
    """The same check on a copy built with contraction allowed (pragma removed,
    -ffp-contract=fast) must find fused multiply-adds in the query kernels."""
    csrc = os.path.dirname(SRC)
    for f in os.listdir(csrc):
        if f.endswith((".h", ".hip")):
            shutil.copy(os.path.join(csrc, f), tmp_path / f)
    src = (tmp_path / "frnn_kernels.hip").read_text()
    assert "#pragma clang fp contract(off)" in src
    (tmp_path / "frnn_kernels.hip").write_text(src.replace("#pragma clang fp contract(off)", ""))
    flags = [f for f in B.FLAGS if f != "-ffp-contract=off"] + ["-ffp-contract=fast"]
    out = tmp_path / "k.s"
    cmd = [B.HIPCC, "-x", "hip", *flags, "--cuda-device-only", "-S", "-I", str(tmp_path),
           "-I", os.path.join(csrc, "..", ".."), str(tmp_path / "frnn_kernels.hip"), "-o", str(out)]
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stderr[-2000:]
    asm = out.read_text()
    q = [m.start() for m in re.finditer(r"^_ZN4frnn7k_query\w+:", asm, re.M)]
    assert q and FMA.search(asm[q[0]:]), "contraction allowed, yet no FMA found: the check would be vacuous"
