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


def test_constants_match_header():
    text = open(HEADER).read()
    assert int(re.search(r"#define AIDW_KMAX (\d+)", text).group(1)) == aidw.AIDW_KMAX
    assert int(re.search(r"#define AIDW_MAX_POINTS (\d+)LL", text).group(1)) == \
        aidw.AIDW_MAX_POINTS
    # the kernels' scan bounds j + 2 * 32 stay below 2^31
    assert aidw.AIDW_MAX_POINTS + 64 < 2 ** 31


def test_version_and_status_names():
    _lib_or_skip()
    assert aidw.aidw_version() == (0 << 16) | 3
    assert aidw.status_name(aidw.AIDW_EINVAL) == "AIDW_EINVAL"
    assert aidw.status_name(aidw.AIDW_OK) == "AIDW_OK"


STRUCTS = ["aidw_options", "aidw_problem", "aidw_tuning", "aidw_issue_costs",
           "aidw_server_options", "aidw_job", "aidw_server_counters"]


def _header_structs():
    text = re.sub(r"/\*.*?\*/", "", open(HEADER).read(), flags=re.S)
    return sorted(set(re.findall(r"typedef\s+struct\s+(aidw_[a-z_]+)\s*\{", text)))


def test_every_header_struct_is_mirrored():
    assert _header_structs() == sorted(STRUCTS)


def test_struct_layout_matches_header():
    """sizeof and the offset of every field of every struct, C against ctypes."""
    lines, want = [], []
    for name in STRUCTS:
        cls = getattr(aidw, name)
        lines.append('printf("%%zu\\n", sizeof(%s));' % name)
        want.append(ctypes.sizeof(cls))
        for field, _ in cls._fields_:
            lines.append('printf("%%zu\\n", offsetof(%s, %s));' % (name, field))
            want.append(getattr(cls, field).offset)
    src = ("#include <stddef.h>\n#include <stdio.h>\n#include \"aidw.h\"\nint main(void) {\n"
           + "\n".join(lines) + "\nreturn 0;\n}\n")
    with tempfile.TemporaryDirectory() as d:
        c = os.path.join(d, "layout.c")
        exe = os.path.join(d, "layout")
        open(c, "w").write(src)
        subprocess.run(["gcc", "-Wall", "-I" + os.path.join(ROOT, "include"), c, "-o", exe],
                       check=True)
        got = [int(v) for v in subprocess.run([exe], capture_output=True, text=True,
                                              check=True).stdout.split()]
    assert got == want


def test_c_field_names_match_binding():
    """Every field the header declares in a struct is in the ctypes mirror, in
    the same order."""
    text = re.sub(r"/\*.*?\*/", "", open(HEADER).read(), flags=re.S)
    for name in STRUCTS:
        body = re.search(r"typedef\s+struct\s+%s\s*\{(.*?)\}\s*%s\s*;" % (name, name), text,
                         flags=re.S).group(1)
        fields = []
        for decl in body.split(";"):
            decl = decl.strip()
            if not decl:
                continue
            decl = re.sub(r"\[[^]]*\]", "", decl)
            # "double R_min, R_max" declares two fields; "const void *a,*b" too
            head, *rest = decl.split(",")
            fields.append(re.findall(r"[A-Za-z_][A-Za-z_0-9]*", head)[-1])
            fields += [re.findall(r"[A-Za-z_][A-Za-z_0-9]*", r)[-1] for r in rest]
        assert fields == [f for f, _ in getattr(aidw, name)._fields_], name


def test_last_error_takes_a_handle():
    L = _lib_or_skip()
    # no handle: the thread's most recent error of any call
    h = ctypes.c_void_p()
    opt = aidw.aidw_options(-7, 0, 0, None, 0)
    st = L.aidw_create(ctypes.byref(h), ctypes.byref(opt))
    assert st != aidw.AIDW_OK
    assert aidw.last_error(None) != ""
