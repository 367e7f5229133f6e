"""GPU parity of the fused encode-and-filter kernel (ss_filter_ascii_async).

The fused kernel encodes each workgroup's tile of pairs on chip and sweeps it
there; its results must equal the oracle's bit for bit for every tile shape,
ragged batch size, length and threshold, and equal those of the two-kernel
path (encode to device memory, then sweep).
"""
import ctypes
import sys

import numpy as np
import pytest

import oracle
from paper_1910_09020_amd import gen

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rt():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1910_09020_amd as ss
    ss.lib()
    from paper_1910_09020_amd import runner
    return runner


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def want(b, E):
    r = oracle.batch(b["reads"], b["refs"], b["offsets"], b["lengths"], E=E, threads=8)
    return r["accept"], r["edits"]


def check(name, got, exp):
    bad = np.nonzero((got[0] != exp[0]) | (got[1] != exp[1]))[0]
    assert len(bad) == 0, f"{name}: {len(bad)} mismatches, first {bad[:5]}"


def uniform(m, n, seed, rate=0.05):
    rng = np.random.default_rng(seed)
    A = np.frombuffer(b"ACGT", np.uint8)
    reads = rng.choice(A, size=n * m)
    refs = reads.copy()
    fl = rng.random(n * m) < rate
    refs[fl] = rng.choice(A, size=int(fl.sum()))
    for p in range(0, n, 7):       # some unrelated pairs
        refs[p * m:(p + 1) * m] = rng.choice(A, size=m)
    return dict(n=n, reads=reads, refs=refs, offsets=np.arange(n, dtype=np.int64) * m,
                lengths=np.full(n, m, np.int32), E=None)


@pytest.mark.parametrize("tile", [0, 1, 2, 3, 8, 12, 16, 24, 32, 40])
def test_tile_shapes(rt, tile):
    import torch
    b = gen.make(1, n=24 * 32 * 5 + 17)
    db = rt.DeviceBatch(b)
    exp = want(b, 5)
    say(f"  fused n={db.n} m=100 E=5 tile_groups={tile}")
    out = db.filter_fused(5, tile_groups=tile)
    torch.cuda.synchronize()
    assert not db.bad_bases()
    check(f"tile {tile}", rt.results_numpy(out, db.n), exp)


@pytest.mark.parametrize("n", [1, 31, 32, 33, 255, 257, 24 * 32 + 1, 24 * 32 * 3 - 5])
def test_ragged_batch_sizes(rt, n):
    import torch
    b = gen.make(1, n=n)
    db = rt.DeviceBatch(b)
    for E in (0, 5, 10):
        say(f"  fused n={n} E={E}")
        out = db.filter_fused(E)
        torch.cuda.synchronize()
        check(f"n={n} E={E}", rt.results_numpy(out, n), want(b, E))


@pytest.mark.parametrize("m", [0, 1, 2, 3, 5, 36, 100, 128, 132, 250, 1000, 2048])
def test_lengths_and_thresholds(rt, m):
    import torch
    n = max(40, min(2000, 200000 // max(m, 1)))
    b = uniform(m, n, seed=m)
    db = rt.DeviceBatch(b)
    for E in (0, 3, 10, 25, 32):
        say(f"  fused n={n} m={m} E={E}")
        out = db.filter_fused(E)
        torch.cuda.synchronize()
        assert not db.bad_bases()
        check(f"m={m} E={E}", rt.results_numpy(out, n), want(b, E))


def test_same_as_two_kernel_path(rt):
    import torch
    b = gen.make(1, n=200_000)
    db = rt.DeviceBatch(b)
    pk = db.pack_sliced()
    for E in range(0, 11):
        a = db.filter_sliced(pk, E)
        f = db.filter_fused(E)
        torch.cuda.synchronize()
        assert torch.equal(a[:db.n], f[:db.n]), f"E={E}"


def test_bad_base_sets_flag(rt):
    import torch
    b = gen.make(0, n=1000)
    b["reads"] = b["reads"].copy()
    b["reads"][777] = ord("N")
    db = rt.DeviceBatch(b)
    db.filter_fused(5)
    torch.cuda.synchronize()
    assert db.bad_bases()


def test_argument_errors(rt):
    import torch
    import paper_1910_09020_amd as ss
    L = ss.lib()
    ctx = rt.context(0)
    d = torch.zeros(1 << 16, dtype=torch.uint8, device="cuda")
    out = torch.zeros(1024, dtype=torch.int16, device="cuda")
    err = torch.zeros(1, dtype=torch.int32, device="cuda")
    p = lambda t, off=0: ctypes.c_void_p(t.data_ptr() + off)
    call = lambda n, m, E, tile, o=out, off=0: L.ss_filter_ascii_async(ctx, p(d), p(d), n, m, E, tile, p(o, off),
                                                                      p(err), None)
    assert call(0, 100, 5, 0) == ss.SS_OK
    assert call(10, 2049, 5, 0) == ss.SS_ELEN
    assert call(10, 100, 33, 0) == ss.SS_ELEN
    assert call(10, 100, -1, 0) == ss.SS_EINVAL
    assert call(10, 100, 5, 257) == ss.SS_EINVAL
    assert call(10, 100, 5, 200) == ss.SS_EINVAL          # 200 groups of 100 bp do not fit on chip
    assert call(10, 100, 5, 64) == ss.SS_EINVAL           # nor two tiles of 64 groups
    assert call(10, 100, 5, 40) == ss.SS_OK
    assert call(10, 100, 5, 0, off=2) == ss.SS_EINVAL     # misaligned output
    torch.cuda.synchronize()


def test_unaligned_bases_take_the_byte_path(rt):
    """Inputs that start 1 byte past a 16-byte boundary cannot use the vector-load path; the result
    must not change (fused schedule at E <= 10, chunked above)."""
    import torch
    import paper_1910_09020_amd as ss
    b = gen.make(1, n=5000 + 3)
    n, m = b["n"], 100
    d = torch.device("cuda")
    rd = torch.empty(n * m + 64, dtype=torch.uint8, device=d)
    rf = torch.empty(n * m + 64, dtype=torch.uint8, device=d)
    rd[1:1 + n * m].copy_(torch.from_numpy(b["reads"]))
    rf[1:1 + n * m].copy_(torch.from_numpy(b["refs"]))
    err = torch.zeros(1, dtype=torch.int32, device=d)
    for E in (0, 5, 6, 12):
        out = torch.empty(n + 8, dtype=torch.int16, device=d)
        ss.ss_filter_ascii_async(rt.context(0), rd[1:], rf[1:], n, m, E, 0, out, err)
        torch.cuda.synchronize()
        assert int(err.item()) == 0
        check(f"unaligned E={E}", rt.results_numpy(out, n), want(b, E))


@pytest.mark.parametrize("aligned", [True, False])
def test_many_tiles_per_block(rt, aligned):
    """Small tiles give every persistent block many tiles, so each tile buffer is reused: in wave mode
    (aligned inputs of 100 bp) the encoders wait for the sweep of the buffer's previous tile, in block mode
    (inputs one byte past a 16-byte boundary) the lockstep schedule runs many rounds.  Every pair must
    equal the oracle's result."""
    import torch
    import paper_1910_09020_amd as ss
    b = gen.make(1, n=300_000 + 5)
    n, m = b["n"], 100
    d = torch.device("cuda")
    off = 0 if aligned else 1
    rd = torch.empty(n * m + 64, dtype=torch.uint8, device=d)
    rf = torch.empty(n * m + 64, dtype=torch.uint8, device=d)
    rd[off:off + n * m].copy_(torch.from_numpy(b["reads"]))
    rf[off:off + n * m].copy_(torch.from_numpy(b["refs"]))
    err = torch.zeros(1, dtype=torch.int32, device=d)
    # E = 0: one row; 3, 5, 6: column words counted in three binary digits (wave mode), 7 and 10 in
    # four; block mode counts every threshold with the per-column thermometer
    for E in (0, 3, 5, 6, 7, 10):
        exp = want(b, E)
        for tile in (1, 2, 6):
            say(f"  fused n={n} E={E} tile_groups={tile} aligned={aligned}")
            out = torch.empty(n + 8, dtype=torch.int16, device=d)
            ss.ss_filter_ascii_async(rt.context(0), rd[off:], rf[off:], n, m, E, tile, out, err)
            torch.cuda.synchronize()
            assert int(err.item()) == 0
            check(f"E={E} tile={tile} aligned={aligned}", rt.results_numpy(out, n), exp)


@pytest.mark.parametrize("E", [6, 8, 10])
def test_block_mode_above_five(rt, E):
    """Pairs of 250 bp with an explicit tile take the fused kernel's block mode (the three encoding
    wavefronts share barriers with the sweeping one); at thresholds above 5 its count is the
    per-column thermometer.  Every pair must equal the oracle's result."""
    import torch
    b = uniform(250, 24 * 32 * 3 + 11, seed=250 + E)
    db = rt.DeviceBatch(b)
    exp = want(b, E)
    for tile in (1, 8):
        say(f"  fused n={db.n} m=250 E={E} tile_groups={tile}")
        out = db.filter_fused(E, tile_groups=tile)
        torch.cuda.synchronize()
        db.check_err(f"fused m=250 E={E} tile={tile}")
        check(f"m=250 E={E} tile={tile}", rt.results_numpy(out, db.n), exp)
