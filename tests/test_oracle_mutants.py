"""The pins are strong enough: each plausible mistake, planted in a private
copy of the oracle source (never in the committed oracle), makes at least one
pin fail."""
import os
import shutil

import numpy as np
import pytest

import oracle
import pinlib
from paper_2609_31980_amd import inputs

# (name, text to find, replacement) applied to a temporary copy of the source
MUTANTS = [
    ("fused multiply-add", "float u = t * t;\n        s = s + u;", "s = fmaf(t, t, s);"),
    ("strict boundary", "if (s <= w->r2)", "if (s < w->r2)"),
    ("distances compared through sqrt", "if (s <= w->r2)", "if (sqrtf(s) <= sqrtf(w->r2))"),
    ("dropped last axis", "for (int32_t d = 0; d < D; ++d)", "for (int32_t d = 0; d < D - 1; ++d)"),
    ("reversed axis order", "for (int32_t d = 0; d < D; ++d)", "for (int32_t d = D - 1; d >= 0; --d)"),
    ("double accumulator", "float s = 0.0f;\n    for", "double s = 0.0;\n    for"),
    ("ties by descending index", "return (x->j > y->j) - (x->j < y->j);", "return (x->j < y->j) - (x->j > y->j);"),
    ("order by index only", "if (x->s < y->s) return -1;\n    if (x->s > y->s) return 1;", ""),
    ("cap off by one", "int64_t keep = (w->K > 0 && n > w->K) ? w->K : n;", "int64_t keep = (w->K > 0 && n > w->K) ? w->K - 1 : n;"),
    ("self never excluded", "if (j == self) continue;", ""),
    ("queries used as references", "w->X + j * (int64_t)w->D", "w->Q + (j % w->M) * (int64_t)w->D"),
    ("absolute instead of square", "float u = t * t;", "float u = fabsf(t);"),
    ("squared radius in double", "if (s <= w->r2)", "if ((double)s <= (double)sqrtf(w->r2) * (double)sqrtf(w->r2))"),
    # mistakes confined to the counts (degrees) path or to the degree field
    ("counts path keeps self", "if (j == self) continue;", "if (w->want_rows && j == self) continue;"),
    ("counts path strict boundary", "if (s <= w->r2) {", "if (w->want_rows ? s <= w->r2 : s < w->r2) {"),
    ("degree recorded after the cap", "w->degree[i] = n;",
     "w->degree[i] = (w->K > 0 && n > w->K) ? w->K : n;"),
    ("counts path self by position", "int64_t self = w->self_ids ? w->self_ids[i] : -1;",
     "int64_t self = w->self_ids ? (w->want_rows ? w->self_ids[i] : i) : -1;"),
    ("counts path skips the last reference", "for (int64_t j = 0; j < w->N; ++j) {",
     "for (int64_t j = 0; j < (w->want_rows ? w->N : w->N - 1); ++j) {"),
]


@pytest.fixture(scope="module")
def X():
    return inputs.c1().points[:1500].copy()


@pytest.mark.parametrize("name,find,repl", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_mutant_is_caught(tmp_path, X, name, find, repl):
    src = open(oracle.SRC).read()
    assert find in src, f"mutation site for '{name}' not found"
    mut = src.replace(find, repl, 1)
    p = tmp_path / "mutant.c"
    p.write_text(mut)
    lib = str(tmp_path / "libmutant.so")
    oracle.build(str(p), lib)
    o = oracle.Oracle(lib)
    failed = pinlib.run_fast_pins(o, X)
    assert failed is not None, f"no pin caught the mutant '{name}'"


def test_unmodified_copy_passes(tmp_path, X):
    lib = str(tmp_path / "libcopy.so")
    oracle.build(oracle.SRC, lib)
    assert pinlib.run_fast_pins(oracle.Oracle(lib), X) is None
