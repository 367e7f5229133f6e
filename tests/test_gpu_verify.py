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
        ss.ss_verify_async(ctx, ps, db.total, db.offsets, db.lengths, None, 2, 257, out)
    assert ei.value.status == ss.SS_ELEN
    res = torch.zeros(1, dtype=torch.int16, device="cuda")
    ss.ss_select_accepted_async(ctx, res, 0, None, cnt)
    torch.cuda.synchronize()
    assert int(cnt.item()) == 0
