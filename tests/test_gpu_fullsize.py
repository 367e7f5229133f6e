"""Parity at the full workload sizes, in the launch configuration the benchmark times.

The oracle checks a random sample pair by pair; every pair is checked by
properties that hold at any size: the lane-sliced sweep, the one-call path
(fused or chunked) and the one-pair-per-lane walk agree on all pairs, the accept decision is monotone in E, a reported
count never exceeds E+1 and the decision is exactly count <= E.
"""
import os

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
    return torch, runner


def _sample_check(b, E, acc, ed, k, seed):
    rng = np.random.default_rng(seed)
    idx = np.sort(rng.choice(b["n"], size=k, replace=False))
    w = oracle.batch(b["reads"], b["refs"], b["offsets"][idx], b["lengths"][idx], E=E,
                     threads=min(16, os.cpu_count() or 1))
    bad = np.nonzero((w["accept"] != acc[idx]) | (w["edits"] != ed[idx]))[0]
    assert len(bad) == 0, f"E={E}: {len(bad)} sampled mismatches, first pairs {idx[bad[:5]]}"


def _run(rt, b, Es, plain_E, sample):
    torch, runner = rt
    db = runner.DeviceBatch(b)
    pk = db.pack_sliced()
    out = db.new_out()
    res = {}
    for E in Es:
        print(f"  sliced n={db.n} m={db.uniform_m} E={E}", flush=True)
        db.filter_sliced(pk, E, out=out)
        torch.cuda.synchronize()
        res[E] = runner.results_numpy(out, db.n)
    assert not db.bad_bases()
    del pk
    # the one-call path (fused kernel for small E, chunked two-kernel schedule
    # above) must give the same words for every pair
    for E in Es:
        print(f"  one-call n={db.n} E={E}", flush=True)
        f = db.filter_fused(E)
        torch.cuda.synchronize()
        fa, fe = runner.results_numpy(f, db.n)
        assert np.array_equal(fa, res[E][0]) and np.array_equal(fe, res[E][1]), f"one-call E={E}"
        del f
    ps = db.pack_stream()
    print(f"  plain E={plain_E}", flush=True)
    pout = db.filter_plain(ps, plain_E)
    torch.cuda.synchronize()
    pacc, ped = runner.results_numpy(pout, db.n)
    assert np.array_equal(pacc, res[plain_E][0]) and np.array_equal(ped, res[plain_E][1])
    for E in Es:
        acc, ed = res[E]
        assert np.all(ed <= E + 1)
        assert np.array_equal(acc == 1, ed <= E)
    for E0, E1 in zip(Es, Es[1:]):
        assert np.all(res[E1][0] >= res[E0][0]), f"accept not monotone between E={E0} and E={E1}"
    _sample_check(b, plain_E, *res[plain_E], sample, 3)
    return res


def test_100bp_30M_E5(rt):
    b = gen.make(1)
    _run(rt, b, [4, 5, 6], 5, 100_000)


def test_250bp_10M_E25(rt):
    b = gen.make(2)
    _run(rt, b, [24, 25], 25, 20_000)


def test_mixed_5M_planned(rt, tmp_path):
    """The mixed-length batch at full size (5 M short pairs + 20,000 pairs of 10 kbp, per-pair E), in
    the benchmark's launch configuration: an autotuned plan replayed from a captured graph.  Every
    pair against one unbucketed wavefront launch laid out for the largest threshold; a sample of
    short and long pairs against the oracle."""
    torch, runner = rt
    import paper_1910_09020_amd as ss
    b = gen.make(3, threads=min(16, os.cpu_count() or 1))
    db = runner.DeviceBatch(b)
    ps = db.pack_stream()
    ctx = runner.context()
    out = db.new_out()
    print(f"  tuned plan n={db.n}", flush=True)
    plan, _ = ss.ss_plan_create_tuned(ctx, b["lengths"], b["E"], ps, db.total, db.offsets, db.lengths, db.E, out,
                                      str(tmp_path / "tune.json"))
    ss.ss_plan_capture(ctx, plan, ps, db.total, db.offsets, db.lengths, db.E, out)
    out.fill_(-1)
    ss.ss_plan_launch(plan, torch.cuda.current_stream())
    torch.cuda.synchronize()
    acc, ed = runner.results_numpy(out, db.n)
    ss.ss_plan_destroy(plan)
    assert not db.bad_bases()
    print(f"  unbucketed wavefront launch E={int(b['E'].max())}", flush=True)
    flat = db.filter_wave(ps, int(b["E"].max()), per_pair=True)
    torch.cuda.synchronize()
    fa, fe = runner.results_numpy(flat, db.n)
    assert np.array_equal(acc, fa) and np.array_equal(ed, fe), "planned launch != unbucketed launch"
    assert np.all(ed <= b["E"] + 1) and np.array_equal(acc == 1, ed <= b["E"])
    rng = np.random.default_rng(5)
    long_idx = np.nonzero(b["lengths"] >= 10000)[0]
    short_idx = np.nonzero(b["lengths"] < 10000)[0]
    idx = np.sort(np.concatenate([rng.choice(short_idx, 20_000, replace=False), rng.choice(long_idx, 100, replace=False)]))
    w = oracle.batch(b["reads"], b["refs"], b["offsets"][idx], b["lengths"][idx], E_per_pair=b["E"][idx],
                     threads=min(16, os.cpu_count() or 1))
    bad = np.nonzero((w["accept"] != acc[idx]) | (w["edits"] != ed[idx]))[0]
    assert len(bad) == 0, f"{len(bad)} sampled mismatches, first pairs {idx[bad[:5]]}"
