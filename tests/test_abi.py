"""Host-side checks of the C ABI: libaidw.so loads, exports every function
that include/aidw.h declares, and the ctypes structures of the Python binding
have the C layout.  No GPU compute is issued here."""
import ctypes
import os
import re
import subprocess
import tempfile

import pytest

from paper_1511_02186_amd import aidw

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "aidw.h")


def _declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"\b(aidw_[a-z0-9_]+)\s*\(", text)
    return sorted(set(names))


def _lib_or_skip():
    if not os.path.exists(aidw.LIB_PATH):
        pytest.fail("libaidw.so is not built; run __graft_entry__.build()")
    return aidw.lib()


def test_header_declares_the_boundary():
    names = _declared_functions()
    for must in ["aidw_create", "aidw_destroy", "aidw_set_stream", "aidw_interpolate",
                 "aidw_interpolate_ex", "aidw_last_error", "aidw_status_string"]:
        assert must in names


def test_library_exports_every_declared_symbol():
    L = ctypes.CDLL(_lib_or_skip()._name)
    missing = [n for n in _declared_functions() if not hasattr(L, n)]
    assert not missing, missing


def test_binding_covers_every_declared_symbol():
    for n in _declared_functions():
        assert n in aidw._SIGNATURES, n


def test_version_and_status_names():
    _lib_or_skip()
    assert aidw.aidw_version() == (0 << 16) | 1
    assert aidw.status_name(aidw.AIDW_EINVAL) == "AIDW_EINVAL"
    assert aidw.status_name(aidw.AIDW_OK) == "AIDW_OK"


def test_struct_layout_matches_header():
    src = r"""
#include <stddef.h>
#include <stdio.h>
#include "aidw.h"
int main(void) {
  printf("%zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu\n", sizeof(aidw_problem),
         offsetof(aidw_problem, m), offsetof(aidw_problem, k), offsetof(aidw_problem, alpha_levels),
         offsetof(aidw_problem, area), offsetof(aidw_problem, out), offsetof(aidw_problem, knn_idx),
         offsetof(aidw_problem, flags), sizeof(aidw_options), offsetof(aidw_options, hbm_budget_bytes),
         offsetof(aidw_options, tune_path));
  return 0;
}
"""
    with tempfile.TemporaryDirectory() as d:
        c = os.path.join(d, "layout.c")
        exe = os.path.join(d, "layout")
        open(c, "w").write(src)
        subprocess.run(["gcc", "-I" + os.path.join(ROOT, "include"), c, "-o", exe], check=True)
        got = [int(v) for v in subprocess.run([exe], capture_output=True, text=True,
                                              check=True).stdout.split()]
    P, O = aidw.aidw_problem, aidw.aidw_options
    want = [ctypes.sizeof(P), P.m.offset, P.k.offset, P.alpha_levels.offset, P.area.offset,
            P.out.offset, P.knn_idx.offset, P.flags.offset, ctypes.sizeof(O),
            O.hbm_budget_bytes.offset, O.tune_path.offset]
    assert got == want
