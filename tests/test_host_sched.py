"""Host logic of the serving loop on the CPU: the budget ledger driven by a
multi-threaded simulation with a fake executor, built with ThreadSanitizer
and with AddressSanitizer + UBSan (host code only, g++)."""
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "tests", "cpp", "test_sched.cpp")
INC = os.path.join(ROOT, "paper_2609_31980_amd", "csrc")


@pytest.mark.parametrize("san", ["thread", "address,undefined", "none"])
def test_budget_ledger_simulation(tmp_path, san):
    exe = str(tmp_path / "sched")
    flags = ["-O1", "-g", "-std=c++17", "-pthread"]
    if san != "none":
        flags.append(f"-fsanitize={san}")
    subprocess.run(["g++", *flags, "-I", INC, SRC, "-o", exe], check=True)
    env = dict(os.environ, TSAN_OPTIONS="halt_on_error=1", ASAN_OPTIONS="detect_leaks=1",
               UBSAN_OPTIONS="halt_on_error=1")
    r = subprocess.run([exe, "1500"], capture_output=True, text=True, timeout=120, env=env)
    assert r.returncode == 0, r.stderr[-3000:]
    assert "batches" in r.stdout
