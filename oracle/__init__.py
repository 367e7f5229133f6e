"""SneakySnake CPU oracle (test infrastructure only).

Thin ctypes wrapper over ``oracle/ss_oracle.c``: the plain, per-cell CPU
implementation of the chip maze (Equation 1, Section 2.3) and the greedy walk
(Section 2.4), Snake-on-Chip's sub-maze decomposition of it (Section 2.5), pairs of
unequal length (the note of Section 2.4 between steps 4 and 5), plus
the two checkers that pin it (minimum-obstacle search over
all signal nets, Theorem 2; Levenshtein DP, the quantity the filter bounds from
below, Sections 1 and 2.1).

Only the tests, the smoke check and the benchmark's CPU-baseline leg may import
this package.  The GPU library never loads it.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ss_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle with gcc -O2 into oracle/liboracle.so."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-D_POSIX_C_SOURCE=199309L", "-shared",
                               "-fPIC", "-pthread", _SRC, "-o", tmp])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB):
        build(force=False)
    lib = ctypes.CDLL(_LIB)
    u8p = ctypes.POINTER(ctypes.c_uint8)
    i32p = ctypes.POINTER(ctypes.c_int32)
    i64p = ctypes.POINTER(ctypes.c_int64)
    lib.ss_oracle_cell.argtypes = [u8p, u8p, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int]
    lib.ss_oracle_cell.restype = ctypes.c_int
    lib.ss_oracle_pair_ex.argtypes = [u8p, u8p, ctypes.c_int, ctypes.c_int, ctypes.c_int, i32p,
                                      ctypes.c_void_p, i32p, i32p, ctypes.c_int, i32p]
    lib.ss_oracle_pair_ex.restype = ctypes.c_int
    lib.ss_oracle_min_obstacles.argtypes = [u8p, u8p, ctypes.c_int, ctypes.c_int]
    lib.ss_oracle_min_obstacles.restype = ctypes.c_int
    lib.ss_oracle_levenshtein.argtypes = [u8p, ctypes.c_int, u8p, ctypes.c_int]
    lib.ss_oracle_levenshtein.restype = ctypes.c_int
    lib.ss_oracle_batch.argtypes = [u8p, u8p, i64p, i32p, ctypes.c_int64, i32p, ctypes.c_int32,
                                    ctypes.c_int, ctypes.c_int, u8p, i32p, i64p]
    lib.ss_oracle_batch.restype = ctypes.c_double
    lib.ss_oracle_min_obstacles_batch.argtypes = [u8p, u8p, i64p, i32p, ctypes.c_int64, i32p,
                                                  ctypes.c_int32, i32p]
    lib.ss_oracle_min_obstacles_batch.restype = None
    lib.ss_oracle_levenshtein_batch.argtypes = [u8p, u8p, i64p, i32p, ctypes.c_int64, i32p]
    lib.ss_oracle_levenshtein_batch.restype = None
    lib.ss_oracle_submaze.argtypes = [u8p, u8p, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, i32p]
    lib.ss_oracle_submaze.restype = ctypes.c_int
    lib.ss_oracle_submaze_batch.argtypes = [u8p, u8p, i64p, i32p, ctypes.c_int64, ctypes.c_int, ctypes.c_int, u8p,
                                            i32p]
    lib.ss_oracle_submaze_batch.restype = None
    lib.ss_oracle_pair_uneq.argtypes = [u8p, ctypes.c_int, u8p, ctypes.c_int, ctypes.c_int, i32p, i32p, i32p]
    lib.ss_oracle_pair_uneq.restype = ctypes.c_int
    lib.ss_oracle_min_obstacles_uneq.argtypes = [u8p, ctypes.c_int, u8p, ctypes.c_int, ctypes.c_int]
    lib.ss_oracle_min_obstacles_uneq.restype = ctypes.c_int
    lib.ss_oracle_batch_uneq.argtypes = [u8p, i64p, i32p, u8p, i64p, i32p, ctypes.c_int64, i32p, ctypes.c_int32,
                                         ctypes.c_int, u8p, i32p]
    lib.ss_oracle_batch_uneq.restype = ctypes.c_double
    lib.ss_oracle_uneq_checks.argtypes = [u8p, i64p, i32p, u8p, i64p, i32p, ctypes.c_int64, ctypes.c_int32, i32p, i32p,
                                          i32p]
    lib.ss_oracle_uneq_checks.restype = None
    _lib = lib
    return lib


def _u8(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))


def _i32(a):
    return None if a is None else a.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))


def _i64(a):
    return None if a is None else a.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))


def _bytes(s) -> np.ndarray:
    if isinstance(s, str):
        s = s.encode()
    return np.frombuffer(bytes(s), dtype=np.uint8).copy()


def cell(R, Q, E: int, i: int, j: int) -> int:
    """Z[i, j] of Equation 1 (1-based row i in 1..2E+1, column j in 1..m)."""
    r, q = _bytes(R), _bytes(Q)
    assert len(r) == len(q)
    return _load().ss_oracle_cell(_u8(r), _u8(q), len(r), E, i, j)


def maze(R, Q, E: int) -> np.ndarray:
    """The full (2E+1) x m chip maze of Equation 1, row i-1 / column j-1."""
    r, q = _bytes(R), _bytes(Q)
    m = len(r)
    z = np.zeros((2 * E + 1, m), dtype=np.uint8)
    for i in range(1, 2 * E + 2):
        for j in range(1, m + 1):
            z[i - 1, j - 1] = _load().ss_oracle_cell(_u8(r), _u8(q), m, E, i, j)
    return z


def pair(R, Q, E: int, stop_early: bool = True, segments: bool = False):
    """Greedy walk of Section 2.4 on reference R and query Q.

    Returns (accept, edits) or, with segments=True, (accept, edits, [(row, end_col), ...]).
    """
    r, q = _bytes(R), _bytes(Q)
    assert len(r) == len(q)
    m = len(r)
    e = ctypes.c_int32(0)
    cap = m + 1
    rows = np.zeros(cap, dtype=np.int32)
    ends = np.zeros(cap, dtype=np.int32)
    ns = ctypes.c_int32(0)
    acc = _load().ss_oracle_pair_ex(_u8(r), _u8(q), m, E, 1 if stop_early else 0, ctypes.byref(e),
                                    None, _i32(rows), _i32(ends), cap, ctypes.byref(ns))
    if segments:
        return acc, e.value, list(zip(rows[:ns.value].tolist(), ends[:ns.value].tolist()))
    return acc, e.value


def min_obstacles(R, Q, E: int) -> int:
    r, q = _bytes(R), _bytes(Q)
    return _load().ss_oracle_min_obstacles(_u8(r), _u8(q), len(r), E)


def levenshtein(a, b) -> int:
    x, y = _bytes(a), _bytes(b)
    return _load().ss_oracle_levenshtein(_u8(x), len(x), _u8(y), len(y))


def batch(reads: np.ndarray, refs: np.ndarray, offsets: np.ndarray, lengths: np.ndarray, E=None,
          E_per_pair: np.ndarray | None = None, threads: int = 1, stop_early: bool = True,
          want_stats: bool = False):
    """Run the oracle over a concatenated batch (reads = queries, refs = references).

    Returns dict(accept=uint8[n], edits=int32[n], seconds=float[, stats=int64[n,3]]).
    stats columns: checkpoints, last column reached, cells evaluated.
    """
    reads = np.ascontiguousarray(reads, dtype=np.uint8)
    refs = np.ascontiguousarray(refs, dtype=np.uint8)
    offsets = np.ascontiguousarray(offsets, dtype=np.int64)
    lengths = np.ascontiguousarray(lengths, dtype=np.int32)
    n = len(lengths)
    if E_per_pair is not None:
        E_per_pair = np.ascontiguousarray(E_per_pair, dtype=np.int32)
    acc = np.zeros(n, dtype=np.uint8)
    ed = np.zeros(n, dtype=np.int32)
    st = np.zeros((n, 3), dtype=np.int64) if want_stats else None
    secs = _load().ss_oracle_batch(_u8(reads), _u8(refs), _i64(offsets), _i32(lengths), n,
                                   _i32(E_per_pair), int(E if E is not None else 0), int(threads),
                                   1 if stop_early else 0, _u8(acc), _i32(ed), _i64(st))
    out = dict(accept=acc, edits=ed, seconds=secs)
    if want_stats:
        out["stats"] = st
    return out


def min_obstacles_batch(reads, refs, offsets, lengths, E=0, E_per_pair=None) -> np.ndarray:
    n = len(lengths)
    out = np.zeros(n, dtype=np.int32)
    lengths = np.ascontiguousarray(lengths, dtype=np.int32)
    offsets = np.ascontiguousarray(offsets, dtype=np.int64)
    if E_per_pair is not None:
        E_per_pair = np.ascontiguousarray(E_per_pair, dtype=np.int32)
    _load().ss_oracle_min_obstacles_batch(_u8(np.ascontiguousarray(reads)), _u8(np.ascontiguousarray(refs)),
                                          _i64(offsets), _i32(lengths), n, _i32(E_per_pair), int(E), _i32(out))
    return out


def submaze(R, Q, E: int, t: int, stop_early: bool = True):
    """Snake-on-Chip decomposition (Section 2.5): sum of the greedy walk's counts over sub-mazes of
    t columns.  Returns (accept, count)."""
    r, q = _bytes(R), _bytes(Q)
    assert len(r) == len(q)
    n = ctypes.c_int32(0)
    acc = _load().ss_oracle_submaze(_u8(r), _u8(q), len(r), int(E), int(t), 1 if stop_early else 0,
                                    ctypes.byref(n))
    return int(acc), int(n.value)


def submaze_batch(reads, refs, offsets, lengths, E: int, t: int) -> dict:
    n = len(lengths)
    acc = np.zeros(n, dtype=np.uint8)
    ed = np.zeros(n, dtype=np.int32)
    lengths = np.ascontiguousarray(lengths, dtype=np.int32)
    offsets = np.ascontiguousarray(offsets, dtype=np.int64)
    _load().ss_oracle_submaze_batch(_u8(np.ascontiguousarray(reads)), _u8(np.ascontiguousarray(refs)),
                                    _i64(offsets), _i32(lengths), n, int(E), int(t), _u8(acc), _i32(ed))
    return dict(accept=acc, edits=ed)


def levenshtein_batch(reads, refs, offsets, lengths) -> np.ndarray:
    n = len(lengths)
    out = np.zeros(n, dtype=np.int32)
    lengths = np.ascontiguousarray(lengths, dtype=np.int32)
    offsets = np.ascontiguousarray(offsets, dtype=np.int64)
    _load().ss_oracle_levenshtein_batch(_u8(np.ascontiguousarray(reads)), _u8(np.ascontiguousarray(refs)),
                                        _i64(offsets), _i32(lengths), n, _i32(out))
    return out


# ---------------------------------------------------------------------------- unequal lengths
def pair_uneq(R, Q, E: int):
    """Walk of Section 2.4 on a reference R and a query Q of any lengths, with the leading and
    trailing obstacles caused by the fourth case of Equation 1 deducted (the reading is stated in
    ss_oracle.c).  Returns (accept, reported count = min(count after the deduction, E+1), count
    before the deduction)."""
    r, q = _bytes(R), _bytes(Q)
    e, f = ctypes.c_int32(0), ctypes.c_int32(0)
    acc = _load().ss_oracle_pair_uneq(_u8(r), len(r), _u8(q), len(q), int(E), ctypes.byref(e), ctypes.byref(f),
                                      None)
    return int(acc), int(e.value), int(f.value)


def min_obstacles_uneq(R, Q, E: int) -> int:
    """Fewest obstacles outside fourth-case-only columns over all signal nets (exhaustive search)."""
    r, q = _bytes(R), _bytes(Q)
    return int(_load().ss_oracle_min_obstacles_uneq(_u8(r), len(r), _u8(q), len(q), int(E)))


def batch_uneq(reads, read_offsets, read_lengths, refs, ref_offsets, ref_lengths, E=None, E_per_pair=None,
               threads: int = 1) -> dict:
    """pair_uneq over a batch: query p = reads[read_offsets[p]:+read_lengths[p]], reference p likewise
    in refs.  Returns dict(accept=uint8[n], edits=int32[n], seconds)."""
    reads = np.ascontiguousarray(reads, dtype=np.uint8)
    refs = np.ascontiguousarray(refs, dtype=np.uint8)
    ro = np.ascontiguousarray(read_offsets, dtype=np.int64)
    rl = np.ascontiguousarray(read_lengths, dtype=np.int32)
    fo = np.ascontiguousarray(ref_offsets, dtype=np.int64)
    fl = np.ascontiguousarray(ref_lengths, dtype=np.int32)
    n = len(rl)
    assert len(ro) == n and len(fo) == n and len(fl) == n
    if E_per_pair is not None:
        E_per_pair = np.ascontiguousarray(E_per_pair, dtype=np.int32)
    acc = np.zeros(n, dtype=np.uint8)
    ed = np.zeros(n, dtype=np.int32)
    secs = _load().ss_oracle_batch_uneq(_u8(reads), _i64(ro), _i32(rl), _u8(refs), _i64(fo), _i32(fl), n,
                                        _i32(E_per_pair), int(E if E is not None else 0), int(threads), _u8(acc),
                                        _i32(ed))
    return dict(accept=acc, edits=ed, seconds=secs)


def uneq_checks(reads, read_offsets, read_lengths, refs, ref_offsets, ref_lengths, E: int) -> dict:
    """Per pair: the count after the deduction without the stop at E+1 (net), the exhaustive minimum
    over nets (minobs) and the Levenshtein distance (ed); one thread."""
    reads = np.ascontiguousarray(reads, dtype=np.uint8)
    refs = np.ascontiguousarray(refs, dtype=np.uint8)
    ro = np.ascontiguousarray(read_offsets, dtype=np.int64)
    rl = np.ascontiguousarray(read_lengths, dtype=np.int32)
    fo = np.ascontiguousarray(ref_offsets, dtype=np.int64)
    fl = np.ascontiguousarray(ref_lengths, dtype=np.int32)
    n = len(rl)
    net = np.zeros(n, np.int32)
    mo = np.zeros(n, np.int32)
    ed = np.zeros(n, np.int32)
    _load().ss_oracle_uneq_checks(_u8(reads), _i64(ro), _i32(rl), _u8(refs), _i64(fo), _i32(fl), n, int(E),
                                  _i32(net), _i32(mo), _i32(ed))
    return dict(net=net, minobs=mo, ed=ed)
