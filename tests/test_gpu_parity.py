"""GPU parity: every kernel against the CPU oracle, element by element.

The bar is bit-exact equality of the accept bit and the reported obstacle
count (integer arithmetic only).  Inputs are the seeded workloads of
``paper_1910_09020_amd.gen`` plus hand-made edge cases.
"""
import ctypes
import sys

import numpy as np
import pytest

import oracle
from paper_1910_09020_amd import gen

pytestmark = pytest.mark.gpu


def _need_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


@pytest.fixture(scope="module")
def rt():
    _need_gpu()
    import paper_1910_09020_amd as ss
    ss.lib()
    from paper_1910_09020_amd import runner
    return runner


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def expect(b, E=None, Epp=None):
    r = oracle.batch(b["reads"], b["refs"], b["offsets"], b["lengths"], E=E, E_per_pair=Epp, threads=8)
    return r["accept"], r["edits"]


def check(name, got, want):
    ga, ge = got
    wa, we = want
    bad = np.nonzero((ga != wa) | (ge != we))[0]
    assert len(bad) == 0, f"{name}: {len(bad)} mismatches, first {bad[:5]} got {ge[bad[:5]]} want {we[bad[:5]]}"


def uniform_batch(m, n, seed):
    """n pairs of length m: references with ~6% substitutions, every fifth one unrelated."""
    rng = np.random.default_rng(seed)
    A = np.frombuffer(b"ACGT", np.uint8)
    reads = rng.choice(A, size=n * m)
    refs = reads.copy()
    flip = rng.random(n * m) < 0.06
    refs[flip] = rng.choice(A, size=int(flip.sum()))
    for p in range(0, n, 5):
        refs[p * m:(p + 1) * m] = rng.choice(A, size=m)
    return dict(n=n, reads=reads, refs=refs, offsets=np.arange(n, dtype=np.int64) * m,
                lengths=np.full(n, m, np.int32), E=None)


def run_all(rt, b, E, kernels=("sliced", "fused", "plain", "wave")):
    import torch
    db = rt.DeviceBatch(b)
    want = expect(b, E=E)
    if "sliced" in kernels and db.uniform_m is not None and E <= 32:
        say(f"  sliced n={db.n} m={db.uniform_m} E={E}")
        pk = db.pack_sliced()
        out = db.filter_sliced(pk, E)
        torch.cuda.synchronize()
        assert not db.bad_bases()
        check(f"sliced E={E}", rt.results_numpy(out, db.n), want)
    if "fused" in kernels and db.contiguous and db.uniform_m <= 2048 and E <= 32:
        say(f"  fused n={db.n} m={db.uniform_m} E={E}")
        out = db.filter_fused(E)
        torch.cuda.synchronize()
        assert not db.bad_bases()
        check(f"fused E={E}", rt.results_numpy(out, db.n), want)
    ps = None
    if "plain" in kernels and E <= 31:
        say(f"  plain n={db.n} E={E}")
        ps = db.pack_stream()
        out = db.filter_plain(ps, E)
        torch.cuda.synchronize()
        check(f"plain E={E}", rt.results_numpy(out, db.n), want)
    if "wave" in kernels:
        say(f"  wave n={db.n} E={E}")
        ps = db.pack_stream() if ps is None else ps
        out = db.filter_wave(ps, E)
        torch.cuda.synchronize()
        check(f"wave E={E}", rt.results_numpy(out, db.n), want)


def test_fig2_example(rt):
    b = gen.concat([("GGTGAGAGTTGT", "GGTGCAGAGCTC")])   # (read Q, ref R)
    for E in range(0, 6):
        run_all(rt, b, E)


def test_config0_E5(rt):
    run_all(rt, gen.make(0), 5)


@pytest.mark.parametrize("E", list(range(0, 11)))
def test_config1_sweep(rt, E):
    run_all(rt, gen.make(1, n=20000 + 7), E)


@pytest.mark.parametrize("E", [0, 1, 3, 8, 10, 11, 12, 13, 16, 17, 20, 25])
def test_config2_sweep(rt, E):
    run_all(rt, gen.make(2, n=4000 + 19), E)


@pytest.mark.parametrize("m", [1, 2, 3, 4, 5, 7, 31, 32, 33, 63, 64, 65, 127, 128, 129, 200])
def test_ragged_lengths(rt, m):
    rng = np.random.default_rng(m)
    n = 97
    reads = rng.choice(np.frombuffer(b"ACGT", np.uint8), size=n * m)
    refs = reads.copy()
    # mutate a few positions, make some pairs unrelated, some identical
    flip = rng.random(n * m) < 0.06
    refs[flip] = rng.choice(np.frombuffer(b"ACGT", np.uint8), size=int(flip.sum()))
    for p in range(0, n, 5):
        refs[p * m:(p + 1) * m] = rng.choice(np.frombuffer(b"ACGT", np.uint8), size=m)
    b = dict(n=n, reads=reads, refs=refs, offsets=np.arange(n, dtype=np.int64) * m,
             lengths=np.full(n, m, np.int32), E=None)
    # every window size of the one-window sweep (E = 0; 1..4; 5..8; 9, 10; 13..16) and of the
    # three-part one (E = 11, 12; 17..20; 29..32), with each form's first and last threshold
    for E in (0, 1, 2, 3, 4, 5, 6, 7, 8, 9, 10, 11, 12, 13, 16, 17, 20, 29, 31, 32):
        run_all(rt, b, E)


def test_degenerate_pairs(rt):
    pairs = [("A", "A"), ("A", "C"), ("AAAA", "CCCC"), ("ACGTACGT", "ACGTACGA"), ("ACGTTGCA", "CGTTGCAG"),
             ("acgtAC", "ACGTac"), ("T" * 40, "T" * 40), ("G" * 40, "C" * 40)]
    b = gen.concat(pairs)
    for E in (0, 1, 3, 10, 32):
        run_all(rt, b, E, kernels=("plain", "wave") if E > 31 else ("plain", "wave"))
    # equal-length subsets through the sliced kernel
    for m in (1, 4, 8, 40):
        sub = gen.concat([p for p in pairs if len(p[0]) == m])
        for E in (0, 1, 3, 10, 32):
            run_all(rt, sub, E, kernels=("sliced", "fused"))


def test_zero_length_pairs_on_the_equal_length_paths(rt):
    """Pairs of length 0 through the sliced sweep, the one-call entry (aligned and unaligned inputs)
    and the entry that allocates nothing: every pair is accepted with count 0, as the oracle gives;
    the sweep reads nothing (the planes of length 0 are empty)."""
    import torch
    import paper_1910_09020_amd as ss
    n = 100
    b = dict(n=n, reads=np.zeros(0, np.uint8), refs=np.zeros(0, np.uint8),
             offsets=np.zeros(n, np.int64), lengths=np.zeros(n, np.int32), E=None)
    db = rt.DeviceBatch(b)
    ctx = rt.context()
    buf = torch.full((64,), ord("A"), dtype=torch.uint8, device="cuda")
    for E in (0, 5, 9):
        say(f"  m=0 n={n} E={E}")
        want = expect(b, E=E)
        assert np.all(want[0] == 1) and np.all(want[1] == 0)
        pk = db.pack_sliced()
        check(f"sliced m=0 E={E}", rt.results_numpy(db.filter_sliced(pk, E), n), want)
        check(f"one call m=0 E={E}", rt.results_numpy(db.filter_fused(E), n), want)
        for off in (0, 1):
            for entry in (ss.ss_filter_ascii_async, ss.ss_filter_ascii_noalloc):
                out = torch.full((n + 8,), -1, dtype=torch.int16, device="cuda")
                if entry is ss.ss_filter_ascii_async:
                    entry(ctx, buf[off:], buf[off:], n, 0, E, 0, out, db.err)
                else:
                    entry(ctx, buf[off:], buf[off:], n, 0, E, out, db.err)
                torch.cuda.synchronize()
                check(f"{entry.__name__} m=0 E={E} offset {off}", rt.results_numpy(out, n), want)
    assert db.err_bits() == 0


def test_mixed_lengths_per_pair_E(rt):
    import torch
    b = gen.make(3, n=3000, n_long=6)
    db = rt.DeviceBatch(b)
    want = expect(b, Epp=b["E"])
    Emax = int(b["E"].max())
    say(f"  wave mixed n={db.n} Emax={Emax}")
    ps = db.pack_stream()
    out = db.filter_wave(ps, Emax, per_pair=True)
    torch.cuda.synchronize()
    check("wave mixed", rt.results_numpy(out, db.n), want)
    # plain kernel on the short pairs only (its rows are held in registers, E <= 31)
    short = np.nonzero(b["lengths"] < 1000)[0]
    sb = dict(n=len(short), reads=b["reads"], refs=b["refs"], offsets=b["offsets"][short],
              lengths=b["lengths"][short], E=b["E"][short])
    dsb = rt.DeviceBatch(dict(sb))
    # DeviceBatch copies reads/refs in full; offsets index into them
    ps2 = dsb.pack_stream()
    out2 = dsb.filter_plain(ps2, int(sb["E"].max()), per_pair=True)
    torch.cuda.synchronize()
    check("plain mixed", rt.results_numpy(out2, dsb.n), expect(sb, Epp=sb["E"]))


@pytest.mark.parametrize("m,E", [(1000, 33), (1000, 50), (1000, 100), (3000, 300), (10000, 100)])
def test_wave_large_E(rt, m, E):
    rng = np.random.default_rng(E + m)
    n = 24
    A = np.frombuffer(b"ACGT", np.uint8)
    reads = rng.choice(A, size=n * m)
    refs = reads.copy()
    rate = np.linspace(0.0, 0.12, n)
    for p in range(n):
        seg = slice(p * m, (p + 1) * m)
        fl = rng.random(m) < rate[p]
        r = refs[seg].copy()
        r[fl] = rng.choice(A, size=int(fl.sum()))
        if p % 3 == 1:      # a few indels: shift a tail by one
            cut = m // 3
            r = np.concatenate([r[:cut], r[cut + 1:], rng.choice(A, size=1)])
        refs[seg] = r
    b = dict(n=n, reads=reads, refs=refs, offsets=np.arange(n, dtype=np.int64) * m,
             lengths=np.full(n, m, np.int32), E=None)
    run_all(rt, b, E, kernels=("wave",))


def test_invalid_base_is_reported(rt):
    import torch
    b = gen.make(0, n=64)
    b["refs"] = b["refs"].copy()
    b["refs"][1234] = ord("N")
    db = rt.DeviceBatch(b)
    db.pack_sliced()
    torch.cuda.synchronize()
    assert db.bad_bases()
    db2 = rt.DeviceBatch(b)
    db2.pack_stream()
    torch.cuda.synchronize()
    assert db2.bad_bases()


def test_host_api_matches_oracle(rt):
    import paper_1910_09020_amd as ss
    b = gen.make(0, n=3000)
    acc, ed = ss.ss_filter_batch(b["reads"], b["refs"], b["lengths"], 5)
    check("ss_filter_batch", (acc, ed), expect(b, E=5))
    b3 = gen.make(3, n=2000, n_long=3)
    acc, ed = ss.ss_filter_batch_var(b3["reads"], b3["refs"], b3["lengths"], b3["E"])
    check("ss_filter_batch_var", (acc, ed), expect(b3, Epp=b3["E"]))


def test_host_api_errors_leave_outputs(rt):
    import paper_1910_09020_amd as ss
    L = ss.lib()
    b = gen.make(0, n=100)
    refs = b["refs"].copy()
    refs[50] = ord("x")
    acc = np.full(100, 7, np.uint8)
    ed = np.full(100, -9, np.int32)
    rc = L.ss_filter_batch(b["reads"].ctypes.data, refs.ctypes.data, b["lengths"].ctypes.data, 100, 5,
                           acc.ctypes.data, ed.ctypes.data)
    assert rc == ss.SS_EBASE
    assert np.all(acc == 7) and np.all(ed == -9)
    rc = L.ss_filter_batch(b["reads"].ctypes.data, b["refs"].ctypes.data, b["lengths"].ctypes.data, 100, -1,
                           acc.ctypes.data, ed.ctypes.data)
    assert rc == ss.SS_EINVAL
    assert np.all(acc == 7)
    assert L.ss_filter_batch(None, None, None, 0, 5, None, None) == ss.SS_OK


def pinned(a):
    """A copy of a numpy array in pinned host memory (and the tensor that owns it)."""
    import torch
    t = torch.from_numpy(a).pin_memory()
    return t.numpy(), t


@pytest.mark.parametrize("m,E,n", [(100, 5, 700_001), (100, 9, 400_000), (250, 5, 300_003), (2048, 3, 40_000)])
def test_host_api_pipelined_chunks_match_oracle(rt, m, E, n):
    """The host entry point for pairs of one length in pinned memory streams the batch to the device in
    chunks through two staging buffers, copies overlapping the filter (several chunks here, both buffers
    reused, a ragged last chunk; E = 9 takes the two-kernel schedule inside each chunk); from pageable
    memory it copies the batch whole.  Every pair against the oracle, both ways."""
    import paper_1910_09020_amd as ss
    say(f"  ss_filter_batch m={m} E={E} n={n}, pageable and pinned")
    if m == 100:
        b = gen.make(1, n=n, seed=77 + E)
    elif m == 250:
        b = gen.make(2, n=n, seed=78)
    else:
        b = gen.long_pairs(n, m, 300, 900)
    want = expect(b, E=E)
    acc, ed = ss.ss_filter_batch(b["reads"], b["refs"], b["lengths"], E)
    check(f"ss_filter_batch pageable m={m} E={E}", (acc, ed), want)
    pr, tr = pinned(b["reads"])
    pf, tf = pinned(b["refs"])
    acc2, ed2 = ss.ss_filter_batch(pr, pf, b["lengths"], E)
    check(f"ss_filter_batch pinned m={m} E={E}", (acc2, ed2), want)
    del tr, tf


def test_host_api_pipelined_bad_base_in_last_chunk(rt):
    import paper_1910_09020_amd as ss
    L = ss.lib()
    b = gen.make(1, n=700_001, seed=79)
    refs, t_refs = pinned(b["refs"])
    reads, t_reads = pinned(b["reads"])
    refs[-3] = ord("N")
    acc = np.full(b["n"], 7, np.uint8)
    ed = np.full(b["n"], -9, np.int32)
    rc = L.ss_filter_batch(reads.ctypes.data, refs.ctypes.data, b["lengths"].ctypes.data, b["n"], 5,
                           acc.ctypes.data, ed.ctypes.data)
    assert rc == ss.SS_EBASE
    assert np.all(acc == 7) and np.all(ed == -9)
    # the context is usable afterwards
    a2, e2 = ss.ss_filter_batch(b["reads"], b["refs"], b["lengths"], 5)
    check("after the error", (a2, e2), expect(b, E=5))


@pytest.mark.parametrize("m", [1, 7, 33, 100, 129, 250])
def test_sliced_range_matches_each_threshold(rt, m):
    """ss_filter_sliced_range_async: thresholds sharing a pass (0..4, 5..7) and those that take
    their own must give each threshold's ss_filter_sliced_async result and the oracle's, over ranges
    that start and end inside a shared run."""
    import torch
    b = uniform_batch(m, 24 * 32 * 2 + 13, seed=900 + m)
    db = rt.DeviceBatch(b)
    pk = db.pack_sliced()
    for lo, hi in ((0, 10), (0, 25), (3, 9), (5, 7), (0, 4), (6, 12), (11, 13), (4, 4)):
        say(f"  range n={db.n} m={m} E={lo}..{hi}")
        rng = db.filter_sliced_range(pk, lo, hi)
        torch.cuda.synchronize()
        for E in range(lo, hi + 1):
            one = db.filter_sliced(pk, E)
            torch.cuda.synchronize()
            assert torch.equal(rng[E - lo, :db.n], one[:db.n]), f"m={m} E={E} range {lo}..{hi}"
    for E in (0, 2, 4, 5, 7, 9):
        rng = db.filter_sliced_range(pk, E, E if E not in (0, 5) else {0: 4, 5: 7}[E])
        torch.cuda.synchronize()
        check(f"range m={m} E={E}", rt.results_numpy(rng[0], db.n), expect(b, E=E))


def test_sliced_range_argument_errors(rt):
    import torch
    import paper_1910_09020_amd as ss
    L = ss.lib()
    ctx = rt.context(0)
    pk = torch.zeros(1 << 16, dtype=torch.int32, device="cuda")
    out = torch.zeros(4096, dtype=torch.int16, device="cuda")
    p = lambda t, off=0: ctypes.c_void_p(t.data_ptr() + off)
    call = lambda n, m, lo, hi, stride, off=0: L.ss_filter_sliced_range_async(ctx, p(pk), n, m, lo, hi, p(out, off),
                                                                           stride, None)
    assert call(0, 100, 0, 10, 0) == ss.SS_OK
    assert call(100, 100, 3, 2, 104) == ss.SS_EINVAL      # empty range
    assert call(100, 100, -1, 2, 104) == ss.SS_EINVAL
    assert call(100, 100, 0, 33, 104) == ss.SS_ELEN       # past the sweep's threshold limit
    assert call(100, 100, 0, 2, 96) == ss.SS_EINVAL       # stride below n_pairs
    assert call(100, 100, 0, 2, 101) == ss.SS_EINVAL      # stride not a multiple of 8
    assert call(100, 100, 0, 2, 104, off=2) == ss.SS_EINVAL   # misaligned output
    torch.cuda.synchronize()
