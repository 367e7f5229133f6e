"""Seeded synthetic read/reference workloads (inputs only; no filter arithmetic).

A ctypes wrapper over ``ssgen.c``.  Each configuration produces ASCII pairs in
the concatenated layout used everywhere in this project: pair i occupies
``[offsets[i], offsets[i] + lengths[i])`` in both ``reads`` (queries) and
``refs`` (references).

Configurations (default sizes; ``n`` overrides the pair count):
  0: 10,000 x 100 bp, k ~ U{0..10} edits, E = 5.
  1: 30 M x 100 bp, 40% k ~ U{0..3}, 40% k ~ U{4..15}, 20% unrelated; E swept 0..10.
  2: 10 M x 250 bp, k = min(Poisson(8), 40), 20% unrelated; E swept 0..25.
  3: 5 M short pairs (m ~ U{100,150,250}) + 20,000 pairs of 10 kbp, per-pair E.
Serving requests (Poisson arrivals, log-uniform sizes) come from ``arrivals`` /
``request``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ssgen.c")
_LIB = os.path.join(_HERE, "libssgen.so")
_lib = None

SEED_BASE = 1910090200
SWEEPS = {0: [5], 1: list(range(0, 11)), 2: list(range(0, 26))}
LONG_PAIRS = 20000


def build(force: bool = True) -> str:
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-shared", "-fPIC", "-pthread", _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB):
        build(force=False)
    lib = ctypes.CDLL(_LIB)
    vp = ctypes.c_void_p
    lib.ssgen_default_pairs.argtypes = [ctypes.c_int]
    lib.ssgen_default_pairs.restype = ctypes.c_int64
    lib.ssgen_plan.argtypes = [ctypes.c_int, ctypes.c_uint64, ctypes.c_int64, ctypes.c_int64, vp, vp, vp]
    lib.ssgen_plan.restype = ctypes.c_int
    lib.ssgen_fill.argtypes = [ctypes.c_int, ctypes.c_uint64, ctypes.c_int64, vp, vp, vp, vp, vp, ctypes.c_int]
    lib.ssgen_fill.restype = ctypes.c_int
    lib.ssgen_arrivals.argtypes = [ctypes.c_uint64, ctypes.c_double, ctypes.c_double, vp, ctypes.c_int64]
    lib.ssgen_arrivals.restype = ctypes.c_int64
    lib.ssgen_long_fill.argtypes = [ctypes.c_uint64, ctypes.c_int64, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                    vp, vp]
    lib.ssgen_long_fill.restype = ctypes.c_int
    lib.ssgen_request_pairs.argtypes = [ctypes.c_uint64, ctypes.c_int64, ctypes.c_int32]
    lib.ssgen_request_pairs.restype = ctypes.c_int32
    lib.ssgen_request_plan.argtypes = [ctypes.c_uint64, ctypes.c_int64, ctypes.c_int32, ctypes.c_int32,
                                       ctypes.c_int32, vp, vp]
    lib.ssgen_request_plan.restype = ctypes.c_int64
    lib.ssgen_request_fill.argtypes = [ctypes.c_uint64, ctypes.c_int64, ctypes.c_int32, vp, vp, vp, vp]
    lib.ssgen_request_fill.restype = ctypes.c_int
    lib.ssgen_drive.argtypes = [ctypes.c_uint64, vp, ctypes.c_int64, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                vp, vp, ctypes.c_int, ctypes.c_int64, ctypes.c_int64, vp, vp, vp, vp, vp, vp, vp,
                                vp, vp, vp]
    lib.ssgen_drive.restype = ctypes.c_int64
    lib.ssgen_drive_free.argtypes = [ctypes.c_int64, vp, vp]
    lib.ssgen_drive_free.restype = None
    lib.ssgen_uneq_plan.argtypes = [ctypes.c_uint64, ctypes.c_int64, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, vp]
    lib.ssgen_uneq_plan.restype = ctypes.c_int64
    lib.ssgen_uneq_fill.argtypes = [ctypes.c_uint64, ctypes.c_int64, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                    vp, vp, vp]
    lib.ssgen_uneq_fill.restype = ctypes.c_int
    _lib = lib
    return lib


def _p(a):
    return ctypes.c_void_p(a.ctypes.data) if a is not None else None


def default_pairs(config: int) -> int:
    return int(_load().ssgen_default_pairs(config))


def make(config: int, n: int | None = None, seed: int | None = None, n_long: int | None = None,
         threads: int | None = None) -> dict:
    """Generate configuration ``config``; returns a dict of numpy arrays."""
    lib = _load()
    if n is None:
        n = default_pairs(config)
    if seed is None:
        seed = SEED_BASE + config
    if n_long is None:
        n_long = min(LONG_PAIRS, n // 251) if config == 3 else 0
    if threads is None:
        threads = min(16, os.cpu_count() or 1)
    cat = np.empty(n, dtype=np.uint8)
    lengths = np.empty(n, dtype=np.int32)
    E = np.empty(n, dtype=np.int32)
    if lib.ssgen_plan(config, seed, n, n_long, _p(cat), _p(lengths), _p(E)) != 0:
        raise ValueError("bad configuration %r" % (config,))
    offsets = np.zeros(n, dtype=np.int64)
    if n:
        np.cumsum(lengths[:-1], out=offsets[1:])
    total = int(offsets[-1] + lengths[-1]) if n else 0
    reads = np.empty(total, dtype=np.uint8)
    refs = np.empty(total, dtype=np.uint8)
    lib.ssgen_fill(config, seed, n, _p(cat), _p(offsets), _p(lengths), _p(reads), _p(refs), threads)
    return dict(config=config, seed=seed, n=n, reads=reads, refs=refs, offsets=offsets, lengths=lengths,
                E=E if config == 3 else None, category=cat)


def arrivals(seed: int, rate: float, duration: float) -> np.ndarray:
    lib = _load()
    cnt = lib.ssgen_arrivals(seed, rate, duration, None, 0)
    t = np.empty(cnt, dtype=np.float64)
    lib.ssgen_arrivals(seed, rate, duration, _p(t), cnt)
    return t


def long_pairs(n: int, m: int, bp_lo: int, bp_hi: int, seed: int = 1910090205) -> dict:
    """n pairs of length m (back to back) at per-pair edit rates ~U[bp_lo, bp_hi] basis points
    (the long-pair model at any length)."""
    lib = _load()
    reads = np.empty(n * m, dtype=np.uint8)
    refs = np.empty(n * m, dtype=np.uint8)
    rc = lib.ssgen_long_fill(seed, n, m, bp_lo, bp_hi, _p(reads), _p(refs))
    if rc != 0:
        raise ValueError("ssgen_long_fill: bad arguments")
    return dict(n=n, reads=reads, refs=refs, offsets=np.arange(n, dtype=np.int64) * m,
                lengths=np.full(n, m, np.int32), E=None)


def request(seed: int, req: int, max_pairs: int = 4096, min_len: int = 100, max_len: int = 10000) -> dict:
    """One serving request: its pairs (ASCII), per-pair lengths and E."""
    lib = _load()
    n = int(lib.ssgen_request_pairs(seed, req, max_pairs))
    lengths = np.empty(n, dtype=np.int32)
    E = np.empty(n, dtype=np.int32)
    total = int(lib.ssgen_request_plan(seed, req, n, min_len, max_len, _p(lengths), _p(E)))
    offsets = np.zeros(n, dtype=np.int64)
    if n:
        np.cumsum(lengths[:-1], out=offsets[1:])
    reads = np.empty(total, dtype=np.uint8)
    refs = np.empty(total, dtype=np.uint8)
    lib.ssgen_request_fill(seed, req, n, _p(offsets), _p(lengths), _p(reads), _p(refs))
    return dict(n=n, reads=reads, refs=refs, offsets=offsets, lengths=lengths, E=E)


class Drive:
    """Result of a native serving-schedule run (see ssgen_drive): tickets, scheduled times and the
    per-request output buffers, which stay owned by the generator library until free()."""

    def __init__(self, n):
        self.n = n
        self.tickets = np.zeros(n, np.uint64)
        self.due_ns = np.zeros(n, np.int64)
        self.call_ns = np.zeros(n, np.int64)      # when the submitter called submit
        self.pairs = np.zeros(n, np.int32)
        self.bases = np.zeros(n, np.int64)
        self._acc = (ctypes.c_void_p * max(n, 1))()
        self._ed = (ctypes.c_void_p * max(n, 1))()
        self.submitted = 0

    def outputs(self, i):
        n = int(self.pairs[i])
        a = np.ctypeslib.as_array((ctypes.c_uint8 * n).from_address(self._acc[i])).copy() if n else np.zeros(0, np.uint8)
        e = np.ctypeslib.as_array((ctypes.c_int32 * n).from_address(self._ed[i])).copy() if n else np.zeros(0, np.int32)
        return a, e

    def free(self):
        if self.n:
            _load().ssgen_drive_free(self.n, ctypes.cast(self._acc, ctypes.c_void_p), ctypes.cast(self._ed, ctypes.c_void_p))
            self.n = 0


def drive(seed: int, arrivals_s: np.ndarray, submit_fn_ptr: int, server: int, threads: int = 8, pool: int = 0,
          t0_ns: int = 0, max_pairs: int = 4096, min_len: int = 100, max_len: int = 10000, staged=None) -> Drive:
    """Generate and submit the requests of a schedule natively (submit_fn_ptr: address of a function with
    the signature of ss_server_submit; server: its first argument).  pool > 0: requests 0..pool-1 are
    generated before the clock starts and schedule position i replays request i mod pool.  staged:
    addresses of (ss_server_stage_alloc, ss_server_stage_free, ss_server_submit_staged) to generate each
    request into the server's staging and submit it without a copy (on the fly only)."""
    lib = _load()
    arr = np.ascontiguousarray(arrivals_s, dtype=np.float64)
    n = len(arr)
    D = Drive(n)
    got = lib.ssgen_drive(seed, _p(arr), n, max_pairs, min_len, max_len, ctypes.c_void_p(submit_fn_ptr),
                          ctypes.c_void_p(server), threads, pool, t0_ns, _p(D.tickets), _p(D.due_ns), _p(D.call_ns), _p(D.pairs),
                          _p(D.bases), ctypes.cast(D._acc, ctypes.c_void_p), ctypes.cast(D._ed, ctypes.c_void_p),
                          *[ctypes.c_void_p(x) for x in (staged or (None, None, None))])
    D.submitted = int(got)
    return D


def uneq(n: int, m: int = 100, kmax: int = 10, unrel_pct: int = 10, seed: int = 1910090206) -> dict:
    """Pairs of unequal length: reads of m bases back to back; each reference is its read with
    k ~ U{0..kmax} single-base edits (1/3 substitutions, insertions, deletions) at its natural length,
    or an unrelated string of length in [m - kmax, m + kmax] for unrel_pct percent of the pairs."""
    lib = _load()
    ref_len = np.empty(n, dtype=np.int32)
    total = int(lib.ssgen_uneq_plan(seed, n, m, kmax, unrel_pct, _p(ref_len)))
    if total < 0:
        raise ValueError("ssgen_uneq_plan: bad arguments")
    ref_off = np.zeros(n, dtype=np.int64)
    if n:
        np.cumsum(ref_len[:-1], out=ref_off[1:])
    reads = np.empty(n * m, dtype=np.uint8)
    refs = np.empty(total, dtype=np.uint8)
    lib.ssgen_uneq_fill(seed, n, m, kmax, unrel_pct, _p(ref_off), _p(reads), _p(refs))
    return dict(n=n, reads=reads, refs=refs, read_offsets=np.arange(n, dtype=np.int64) * m,
                read_lengths=np.full(n, m, np.int32), ref_offsets=ref_off, ref_lengths=ref_len)


def concat(pairs) -> dict:
    """Build a batch dict from a list of (read, ref) strings/bytes of equal length."""
    rd = [p[0].encode() if isinstance(p[0], str) else bytes(p[0]) for p in pairs]
    rf = [p[1].encode() if isinstance(p[1], str) else bytes(p[1]) for p in pairs]
    lengths = np.array([len(x) for x in rd], dtype=np.int32)
    assert all(len(a) == len(b) for a, b in zip(rd, rf))
    offsets = np.zeros(len(rd), dtype=np.int64)
    if len(rd):
        np.cumsum(lengths[:-1], out=offsets[1:])
    reads = np.frombuffer(b"".join(rd), dtype=np.uint8).copy()
    refs = np.frombuffer(b"".join(rf), dtype=np.uint8).copy()
    return dict(n=len(rd), reads=reads, refs=refs, offsets=offsets, lengths=lengths, E=None)
