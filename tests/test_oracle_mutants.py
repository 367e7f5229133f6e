"""Planted mistakes in a copy of the oracle must each fail at least one pin.

Each mutant is a one-token edit of ``oracle/ss_oracle.c`` of the kind a
reader could plausibly make (wrong sign, wrong index, transposed operands, a
dropped boundary term, an off-by-one in the counting or stopping rule).  The
mutant is compiled into a temporary library on the CPU and run against the
same independent pins used for the real oracle: the paper's worked example
and the exhaustive tiny-input properties (Theorem 2 against an exhaustive
search, the edit-distance lower bound, the E = 0 equality case).
"""
import ctypes
import os
import subprocess

import numpy as np
import pytest

import oracle
from tests.test_oracle_pins import all_pairs

SRC = os.path.join(os.path.dirname(oracle.__file__), "ss_oracle.c")

MUTANTS = {
    "deletion_rows_wrong_sign": ("else if (i <= E)     q = j - i;", "else if (i <= E)     q = j + i;"),
    "insertion_rows_off_by_one": ("else                 q = j + i - E - 1;", "else                 q = j + i - E;"),
    "main_row_shifted": ("if (i == E + 1)      q = j;", "if (i == E + 1)      q = j - 1;"),
    "operands_transposed": ("return fold(Q[q - 1]) == fold(R[j - 1]) ? 0 : 1;",
                            "return fold(R[q - 1]) == fold(Q[j - 1]) ? 0 : 1;"),
    "boundary_dropped": ("if (q < 1 || q > m) return 1;", "if (q < 1) q = 1; if (q > m) q = m;"),
    "last_column_not_counted": ("if (end <= m) n++;", "if (end < m) n++;"),
    "checkpoint_skips_column": ("c = end + 1;                                   /* step 3",
                                "c = end + 2;                                   /* step 3"),
    "stops_one_early": ("if (stop_early && n > E) break;", "if (stop_early && n >= E) break;"),
    "accept_strict": ("return n <= E ? 1 : 0;", "return n < E ? 1 : 0;"),
    "shortest_run_taken": ("if (L > best) { best = L; best_row = i; }",
                           "if (best < 0 || L < best) { best = L; best_row = i; }"),
}


def _build_mutant(tmp_path, name, old, new):
    src = open(SRC).read()
    assert src.count(old) == 1, name
    path = tmp_path / f"{name}.c"
    path.write_text(src.replace(old, new))
    so = tmp_path / f"lib{name}.so"
    subprocess.check_call(["gcc", "-O1", "-std=c99", "-D_POSIX_C_SOURCE=199309L", "-shared", "-fPIC",
                           "-pthread", str(path), "-o", str(so)])
    lib = ctypes.CDLL(str(so))
    vp = ctypes.c_void_p
    lib.ss_oracle_cell.argtypes = [vp, vp, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int]
    lib.ss_oracle_batch.argtypes = [vp, vp, vp, vp, ctypes.c_int64, vp, ctypes.c_int32, ctypes.c_int,
                                    ctypes.c_int, vp, vp, vp]
    lib.ss_oracle_batch.restype = ctypes.c_double
    lib.ss_oracle_min_obstacles_batch.argtypes = [vp, vp, vp, vp, ctypes.c_int64, vp, ctypes.c_int32, vp]
    return lib


def _p(a):
    return ctypes.c_void_p(a.ctypes.data)


def _pins_hold(lib, golden):
    """True when every pin holds for this library."""
    R = golden["R"][0].encode()
    Q = golden["Q"][0].encode()
    E = int(golden["E"][0])
    r = np.frombuffer(R, np.uint8).copy()
    q = np.frombuffer(Q, np.uint8).copy()
    off = np.zeros(1, np.int64)
    ln = np.array([len(R)], np.int32)
    acc = np.zeros(1, np.uint8)
    ed = np.zeros(1, np.int32)
    lib.ss_oracle_batch(_p(q), _p(r), _p(off), _p(ln), 1, None, E, 1, 1, _p(acc), _p(ed), None)
    if ed[0] != int(golden["obstacles"][0]) or acc[0] != int(golden["accept"][0]):
        return False
    col = [lib.ss_oracle_cell(_p(r), _p(q), len(R), E, i, 6) for i in range(1, 2 * E + 2)]
    if col != [int(v) for v in golden["column6"]]:
        return False
    for m in (1, 2, 3):
        d = all_pairs(m)
        ed_true = oracle.levenshtein_batch(d["reads"], d["refs"], d["offsets"], d["lengths"])
        equal = np.all(d["A"] == d["B"], axis=1)
        for E in range(0, 4):
            n = len(d["lengths"])
            acc = np.zeros(n, np.uint8); tr = np.zeros(n, np.int32)
            acc2 = np.zeros(n, np.uint8); full = np.zeros(n, np.int32)
            opt = np.zeros(n, np.int32)
            args = (_p(d["reads"]), _p(d["refs"]), _p(d["offsets"]), _p(d["lengths"]), n, None, E, 1)
            lib.ss_oracle_batch(*args, 1, _p(acc), _p(tr), None)
            lib.ss_oracle_batch(*args, 0, _p(acc2), _p(full), None)
            lib.ss_oracle_min_obstacles_batch(_p(d["reads"]), _p(d["refs"]), _p(d["offsets"]),
                                              _p(d["lengths"]), n, None, E, _p(opt))
            if not np.array_equal(full, opt):
                return False
            if not np.array_equal(tr, np.minimum(full, E + 1)):
                return False
            if not np.array_equal(acc, (tr <= E).astype(np.uint8)):
                return False
            if np.any(tr > ed_true) or np.any(acc[ed_true <= E] == 0):
                return False
            if not np.array_equal(full == 0, equal):
                return False
            if E == 0 and not np.array_equal(acc == 1, equal):
                return False
    return True


def test_unmutated_copy_passes(tmp_path, golden_fig2):
    lib = _build_mutant(tmp_path, "unchanged", "int n = 0;", "int n = 0;")
    assert _pins_hold(lib, golden_fig2)


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(tmp_path, golden_fig2, name):
    old, new = MUTANTS[name]
    lib = _build_mutant(tmp_path, name, old, new)
    assert not _pins_hold(lib, golden_fig2), f"planted mistake '{name}' passed every pin"
