"""GPU parity of the verification step (exact edit distance of accepted pairs) and of the
compaction of accepted indices, against the oracle's Levenshtein dynamic programme."""
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
    from paper_1910_09020_amd import runner
    ss.lib()
    return ss, runner, torch


def _pairs(lengths, seed):
    rng = np.random.default_rng(seed)
    A = list("ACGT")
    out = []
    for i, m in enumerate(lengths):
        q = rng.choice(A, size=m)
        r = q.copy()
        rate = (0.0, 0.02, 0.08, 0.3, 1.0)[i % 5]
        mask = rng.random(m) < rate
        r[mask] = rng.choice(A, size=int(mask.sum()))
        r = list(r)
        if m > 3 and i % 3 == 1:                     # one deletion and one insertion
            k = int(rng.integers(0, m))
            r = r[:k] + r[k + 1:]
            k = int(rng.integers(0, len(r) + 1))
            r = r[:k] + [rng.choice(A)] + r[k:]
        out.append(("".join(q), "".join(r)))
    return gen.concat(out)


def test_ragged_lengths_vs_levenshtein(rt):
    ss, runner, torch = rt
    lengths = [0, 1, 2, 3, 7, 31, 32, 33, 63, 64, 65, 100, 127, 128, 129, 150, 200, 250, 255, 256] * 12
    b = _pairs(lengths, 3)
    db = runner.DeviceBatch(b)
    ps = db.pack_stream()
    ed = db.verify(ps)
    torch.cuda.synchronize()
    want = oracle.levenshtein_batch(b["reads"], b["refs"], b["offsets"], b["lengths"])
    got = ed[:db.n].cpu().numpy()
    bad = np.nonzero(got != want)[0]
    assert len(bad) == 0, f"{len(bad)} mismatches, first {bad[:5]} got {got[bad[:5]]} want {want[bad[:5]]}"


@pytest.mark.parametrize("m", [32, 64, 100, 128, 250])
def test_uniform_lengths_each_word_count(rt, m):
    ss, runner, torch = rt
    b = gen.make(1, n=3000) if m == 100 else _pairs([m] * 600, m)
    db = runner.DeviceBatch(b)
    ps = db.pack_stream()
    ed = db.verify(ps, max_len=m)
    torch.cuda.synchronize()
    want = oracle.levenshtein_batch(b["reads"], b["refs"], b["offsets"], b["lengths"])
    assert np.array_equal(ed[:db.n].cpu().numpy(), want)


def test_select_then_verify_accepted(rt):
    """Filter (one call), compact the accepted indices, verify only those: every accepted pair's
    distance equals the oracle's, and the accepted set equals the oracle's accepted set."""
    ss, runner, torch = rt
    b = gen.make(1, n=50_000)
    db = runner.DeviceBatch(b)
    res = db.filter_fused(5)
    idx, cnt = db.select_accepted(res)
    ps = db.pack_stream()
    torch.cuda.synchronize()
    k = int(cnt.item())
    ed = db.verify(ps, index=idx[:k], n=k, max_len=100)
    torch.cuda.synchronize()
    sel = np.sort(idx[:k].cpu().numpy())
    want = oracle.batch(b["reads"], b["refs"], b["offsets"], b["lengths"], E=5, threads=8)
    assert np.array_equal(sel, np.nonzero(want["accept"])[0])
    order = idx[:k].cpu().numpy()
    wl = oracle.levenshtein_batch(b["reads"], b["refs"], b["offsets"][order], b["lengths"][order])
    assert np.array_equal(ed[:k].cpu().numpy(), wl)
    # the filter's guarantee: every pair with ED <= E was accepted (no false rejects)
    all_ed = oracle.levenshtein_batch(b["reads"], b["refs"], b["offsets"], b["lengths"])
    assert np.all(want["accept"][all_ed <= 5] == 1)


def test_empty_and_errors(rt):
    ss, runner, torch = rt
    b = _pairs([10, 20], 1)
    db = runner.DeviceBatch(b)
    ps = db.pack_stream()
    ctx = runner.context()
    out = torch.zeros(4, dtype=torch.int32, device="cuda")
    cnt = torch.full((1,), 7, dtype=torch.int64, device="cuda")
    ss.ss_verify_async(ctx, ps, db.total, db.offsets, db.lengths, None, 0, 20, out)
    with pytest.raises(ss.SSError) as ei:
        ss.ss_verify_async(ctx, ps, db.total, db.offsets, db.lengths, None, 2, ss.SS_MAX_LEN_VERIFY + 1, out)
    assert ei.value.status == ss.SS_ELEN
    res = torch.zeros(1, dtype=torch.int16, device="cuda")
    ss.ss_select_accepted_async(ctx, res, 0, None, cnt)
    torch.cuda.synchronize()
    assert int(cnt.item()) == 0


def _levenshtein_parallel(b, threads=8):
    """The oracle's Levenshtein distance of every pair, pairs spread over host threads."""
    from concurrent.futures import ThreadPoolExecutor
    def one(i):
        o, m = int(b["offsets"][i]), int(b["lengths"][i])
        return oracle.levenshtein(b["reads"][o:o + m], b["refs"][o:o + m])
    with ThreadPoolExecutor(threads) as ex:
        return np.array(list(ex.map(one, range(len(b["lengths"])))), dtype=np.int32)


@pytest.mark.parametrize("max_len,lengths", [
    (2048, [257, 300, 1000, 2047, 2048, 700, 1500, 2000, 257, 2048]),
    (4096, [2049, 3000, 4096, 4095, 2500]),
    (8192, [4097, 5000, 8192, 6000, 7777]),
    (16384, [8193, 10000, 16384, 12000, 10000]),
    (32768, [16385, 30000, 20000]),
    (65536, [40000, 65536]),
])
def test_long_pairs_one_wavefront_each(rt, max_len, lengths):
    """Pairs longer than 256 positions: one pair per wavefront, every word count W (2048 W >= max_len),
    ragged lengths at and just past the word boundaries, edit rates from none to unrelated, with indels."""
    ss, runner, torch = rt
    print(f"  wavefront verify max_len={max_len} lengths={lengths}", flush=True)
    b = _pairs(lengths, max_len)
    db = runner.DeviceBatch(b)
    ps = db.pack_stream()
    ed = db.verify(ps, max_len=max_len)
    torch.cuda.synchronize()
    want = _levenshtein_parallel(b)
    got = ed[:db.n].cpu().numpy()
    bad = np.nonzero(got != want)[0]
    assert len(bad) == 0, f"{len(bad)} mismatches, first {bad[:5]} got {got[bad[:5]]} want {want[bad[:5]]}"


def test_long_pair_past_max_len_reports_minus_one(rt):
    ss, runner, torch = rt
    b = _pairs([3000, 1000], 11)
    db = runner.DeviceBatch(b)
    ps = db.pack_stream()
    ed = db.verify(ps, max_len=2048)          # the 3,000-position pair does not fit 2,048 positions
    torch.cuda.synchronize()
    got = ed[:db.n].cpu().numpy()
    assert got[0] == -1
    assert got[1] == oracle.levenshtein(b["reads"][3000:4000], b["refs"][3000:4000])


def test_mixed_batch_select_then_verify_short_and_long(rt):
    """The mixed-length batch (100/150/250 bp and 10 kbp pairs, per-pair thresholds): filter with the
    batched launch, compact the accepted indices, verify the short ones one pair per lane and the long
    ones one pair per wavefront: distances equal the oracle's, and no pair with distance <= E was
    rejected (the filter is lossless)."""
    ss, runner, torch = rt
    b = gen.make(3, n=20_000, n_long=40)
    db = runner.DeviceBatch(b)
    ps = db.pack_stream()
    res = db.filter_wave(ps, int(b["E"].max()), per_pair=True)
    torch.cuda.synchronize()
    r = res[:db.n].cpu().numpy().astype(np.int64) & 0xFFFF
    accepted = np.nonzero(r >> 15)[0]
    lengths = b["lengths"]
    short = accepted[lengths[accepted] <= 256]
    long_ = accepted[lengths[accepted] > 256]
    assert len(long_) > 0
    for sel, ml in ((short, 256), (long_, 10000)):
        idx = torch.from_numpy(sel.astype(np.int64)).cuda()
        ed = db.verify(ps, index=idx, n=len(sel), max_len=ml)
        torch.cuda.synchronize()
        got = ed[:len(sel)].cpu().numpy()
        sub = dict(reads=b["reads"], refs=b["refs"], offsets=b["offsets"][sel], lengths=lengths[sel])
        want = _levenshtein_parallel(sub)
        assert np.array_equal(got, want), (ml, np.nonzero(got != want)[0][:5])
    # lossless: every pair the filter rejected has distance > E (checked on the short pairs and a sample
    # of the long ones)
    rejected = np.nonzero((r >> 15) == 0)[0]
    rs = np.concatenate([rejected[lengths[rejected] <= 256][:3000], rejected[lengths[rejected] > 256][:8]])
    sub = dict(reads=b["reads"], refs=b["refs"], offsets=b["offsets"][rs], lengths=lengths[rs])
    dist = _levenshtein_parallel(sub)
    assert np.all(dist > b["E"][rs])


def _within(ed, E):
    return np.where(ed <= E, ed, E + 1).astype(np.int32)


@pytest.mark.parametrize("E", [0, 3, 10, 50, 300, 1100])
def test_banded_ragged_lengths(rt, E):
    """Banded verification: the distance when within E, else E + 1, for ragged lengths up to 5,000 at
    every edit rate, with indels; E = 1,100 takes two words per lane."""
    ss, runner, torch = rt
    print(f"  banded verify E={E}", flush=True)
    lengths = [0, 1, 2, 31, 32, 33, 100, 257, 700, 1000, 2047, 2048, 2049, 3000, 5000] * 2
    b = _pairs(lengths, 40 + E)
    db = runner.DeviceBatch(b)
    ps = db.pack_stream()
    ed = db.verify_banded(ps, E)
    torch.cuda.synchronize()
    want = _within(_levenshtein_parallel(b), E)
    got = ed[:db.n].cpu().numpy()
    bad = np.nonzero(got != want)[0]
    assert len(bad) == 0, f"{len(bad)} mismatches, first {bad[:5]} got {got[bad[:5]]} want {want[bad[:5]]}"


def test_banded_per_pair_thresholds_and_limits(rt):
    ss, runner, torch = rt
    lengths = [50, 400, 1200, 3000, 6000] * 4
    b = _pairs(lengths, 77)
    rng = np.random.default_rng(3)
    b["E"] = rng.integers(0, 400, size=len(lengths)).astype(np.int32)
    db = runner.DeviceBatch(b)
    ps = db.pack_stream()
    ed = db.verify_banded(ps, int(b["E"].max()), per_pair=True)
    torch.cuda.synchronize()
    want = _within(_levenshtein_parallel(b), b["E"])
    assert np.array_equal(ed[:db.n].cpu().numpy(), want)
    # the largest threshold the window holds, on short pairs; one past it is refused
    ed2 = db.verify_banded(ps, ss.SS_MAX_E_VERIFY_BANDED)
    torch.cuda.synchronize()
    assert np.array_equal(ed2[:db.n].cpu().numpy(), _levenshtein_parallel(b))
    with pytest.raises(ss.SSError) as ei:
        db.verify_banded(ps, ss.SS_MAX_E_VERIFY_BANDED + 1)
    assert ei.value.status == ss.SS_ELEN


def test_banded_long_pairs_30kbp_and_100kbp(rt):
    """Long pairs at thresholds that need five and six words per lane: 30 kbp at E = 4,500 and
    100 kbp at E = 5,000 (the workload of the 100 kbp row), against the oracle's full Levenshtein."""
    ss, runner, torch = rt
    print("  banded verify 30 kbp E=4500 and 100 kbp E=5000", flush=True)
    b = gen.long_pairs(4, 30000, 300, 2000, seed=91)
    db = runner.DeviceBatch(b)
    ps = db.pack_stream()
    ed = db.verify_banded(ps, 4500)
    torch.cuda.synchronize()
    want = _within(_levenshtein_parallel(b), 4500)
    assert np.array_equal(ed[:db.n].cpu().numpy(), want), (ed[:db.n].cpu().numpy(), want)
    b = gen.long_pairs(2, 100000, 300, 700, seed=92)
    db = runner.DeviceBatch(b)
    ps = db.pack_stream()
    ed = db.verify_banded(ps, 5000)
    torch.cuda.synchronize()
    want = _within(_levenshtein_parallel(b), 5000)
    assert np.array_equal(ed[:db.n].cpu().numpy(), want), (ed[:db.n].cpu().numpy(), want)


def test_banded_equals_full_within_threshold_on_the_mixed_batch(rt):
    """On the mixed batch's 10 kbp pairs, the banded distance at each pair's threshold equals the full
    distance (one pair per wavefront) clipped to threshold + 1."""
    ss, runner, torch = rt
    b = gen.make(3, n=2_000, n_long=200)
    db = runner.DeviceBatch(b)
    ps = db.pack_stream()
    long_idx = np.nonzero(b["lengths"] > 256)[0]
    idx = torch.from_numpy(long_idx.astype(np.int64)).cuda()
    full = db.verify(ps, index=idx, n=len(long_idx), max_len=10000)
    banded = db.verify_banded(ps, int(b["E"].max()), per_pair=True, index=idx, n=len(long_idx))
    torch.cuda.synchronize()
    f = full[:len(long_idx)].cpu().numpy()
    E = b["E"][long_idx]
    assert np.array_equal(banded[:len(long_idx)].cpu().numpy(), _within(f, E))
