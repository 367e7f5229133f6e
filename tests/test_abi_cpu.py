"""Host-side checks of the C ABI: the library loads without a GPU and exports
every function that include/ss.h declares; the binding refuses to run without
the built library (no CPU fallback)."""
import ctypes
import os
import re
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    text = open(os.path.join(ROOT, "include", "ss.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?[A-Za-z_][\w\s\*]*?\b(ss_\w+)\s*\(", text, flags=re.M)))


def test_header_declares_entry_points():
    names = header_functions()
    assert "ss_filter_batch" in names and "ss_filter_sliced_async" in names
    assert len(names) >= 12


def test_library_exports_every_declared_symbol():
    import paper_1910_09020_amd as ss
    lib = ctypes.CDLL(ss.LIB_PATH)
    missing = [n for n in header_functions() if not hasattr(lib, n)]
    assert not missing, missing
    assert set(header_functions()) <= set(ss.exported_symbols())


def test_status_strings_and_sizes():
    import paper_1910_09020_amd as ss
    assert ss.status_str(ss.SS_EBASE).startswith("SS_EBASE")
    assert ss.ss_sliced_bytes(32, 100) == 4 * 25 * 1 * 16
    assert ss.ss_sliced_bytes(33, 100) == 4 * 25 * 2 * 16
    assert ss.ss_sliced_bytes(-1, 100) == -1
    assert ss.ss_stream_words(0) == 2
    assert ss.ss_stream_words(33) == 4


def test_validation_needs_no_device():
    """Argument errors are caught before any device call."""
    import paper_1910_09020_amd as ss
    L = ss.lib()
    assert L.ss_filter_batch(None, None, None, -1, 5, None, None) == ss.SS_EINVAL
    assert L.ss_filter_batch(None, None, None, 0, 5, None, None) == ss.SS_OK
    assert L.ss_filter_sliced_async(None, None, 10, 100, 5, None, None) == ss.SS_EINVAL
    assert L.ss_create(None, 0) == ss.SS_EINVAL


def test_missing_library_fails_loudly(tmp_path):
    code = ("import paper_1910_09020_amd as ss; ss.LIB_PATH = %r\n"
            "try:\n    ss.lib()\nexcept RuntimeError as e:\n    print('RAISED', e)\n" % str(tmp_path / "none.so"))
    r = subprocess.run([sys.executable, "-c", code], cwd=ROOT, capture_output=True, text=True)
    assert "RAISED" in r.stdout and "no CPU fallback" in r.stdout


def test_header_limits_match_binding():
    """Every SS_MAX_* limit of include/ss.h has the same value in the binding."""
    import paper_1910_09020_amd as ss
    text = open(os.path.join(ROOT, "include", "ss.h")).read()
    found = 0
    for name, expr in re.findall(r"^#define\s+(SS_MAX_\w+)\s+(.+?)\s*(?:/\*.*)?$", text, flags=re.M):
        value = eval(re.sub(r"(\d+)LL", r"\1", expr), {})      # integer literals and shifts only
        assert getattr(ss, name) == value, name
        found += 1
    assert found >= 8


def test_batch_desc_layout_matches_header(tmp_path):
    """The binding's mirror of ss_batch_desc has the C struct's size and field offsets (a C program built
    against include/ss.h prints them)."""
    import paper_1910_09020_amd as ss
    fields = [f for f, _ in ss.BatchDesc._fields_]
    src = tmp_path / "layout.c"
    src.write_text('#include <stdio.h>\n#include <stddef.h>\n#include "ss.h"\nint main(void){\n'
                   '  printf("%zu\\n", sizeof(ss_batch_desc));\n' +
                   "".join(f'  printf("%zu\\n", offsetof(ss_batch_desc, {f}));\n' for f in fields) +
                   "  return 0;\n}\n")
    exe = tmp_path / "layout"
    subprocess.check_call(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)])
    vals = [int(x) for x in subprocess.check_output([str(exe)], text=True).split()]
    assert vals[0] == ctypes.sizeof(ss.BatchDesc)
    assert vals[1:] == [getattr(ss.BatchDesc, f).offset for f in fields]
    assert ss.ss_pack_words(0) == 4 and ss.ss_pack_words(33) == 2 * (2 + 2) and ss.ss_pack_words(-1) == -1
