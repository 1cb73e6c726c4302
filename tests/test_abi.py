"""The C-ABI library loads on a machine without a GPU and exports every
function include/frnn.h declares; the binding refuses to run without it."""
import ctypes
import os
import re
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "frnn.h")
LIB = os.path.join(ROOT, "paper_2609_31980_amd", "libfrnn.so")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = set(re.findall(r"\b(frnn_[a-z0-9_]+)\s*\(", src))
    return sorted(names)


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ("frnn_build", "frnn_query", "frnn_query_batch", "frnn_csr_release",
                 "frnn_index_destroy", "frnn_server_create", "frnn_server_submit",
                 "frnn_server_wait", "frnn_server_destroy", "frnn_tune", "frnn_status_str",
                 "frnn_last_error"):
        assert must in names


def test_library_exports_every_symbol():
    assert os.path.exists(LIB), "libfrnn.so not built"
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, f"not exported: {missing}"


def test_pure_host_calls():
    from paper_2609_31980_amd import frnn
    o = frnn.default_opts()
    assert o.grid_axes_max == 6 and o.queries_per_item == 32 and o.row_cap_lds == 512 and o.persistent == 2
    assert o.cells_per_item == 2 and o.stash_cap == 64 and o.graphs == 0 and o.adapt == 1
    lib = frnn._lib
    assert lib.frnn_status_str(0) == b"ok"
    assert lib.frnn_status_str(5).startswith(b"query radius")


def test_binding_refuses_without_library(tmp_path):
    pkg = tmp_path / "paper_2609_31980_amd"
    pkg.mkdir()
    shutil.copy(os.path.join(ROOT, "paper_2609_31980_amd", "frnn.py"), pkg / "frnn.py")
    (pkg / "__init__.py").write_text("")
    r = subprocess.run([sys.executable, "-c", "import paper_2609_31980_amd.frnn"],
                       cwd=tmp_path, capture_output=True, text=True)
    assert r.returncode != 0 and "not built" in r.stderr


def test_product_never_touches_the_oracle():
    pkg = os.path.join(ROOT, "paper_2609_31980_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".cpp", ".hip", ".h")):
                text = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in text and "liboracle" not in text and \
                    "frnn_oracle" not in text, f"{f} refers to the oracle"
