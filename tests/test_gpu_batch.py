"""GPU tests of the batched launch (plan + persistent kernel + graph + autotune)."""
import json
import os

import numpy as np
import pytest

import oracle
from paper_1910_09020_amd import gen

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1910_09020_amd as ss
    from paper_1910_09020_amd import runner
    ss.lib()
    return ss, runner, torch


def _mixed(n=20000, n_long=40):
    b = gen.make(3, n=n, n_long=n_long)
    want = oracle.batch(b["reads"], b["refs"], b["offsets"], b["lengths"], E_per_pair=b["E"], threads=8)
    return b, (want["accept"], want["edits"])


def _check(got, want, what):
    ga, ge = got
    wa, we = want
    bad = np.nonzero((ga != wa) | (ge != we))[0]
    assert len(bad) == 0, f"{what}: {len(bad)} mismatches, first {bad[:5]}"


def test_planned_matches_oracle(env):
    ss, runner, torch = env
    b, want = _mixed()
    db = runner.DeviceBatch(b)
    ps = db.pack_stream()
    ctx = runner.context()
    for spl in (1, 2, 4, 8):       # 1 and 2: the 10 kbp pairs take 32 or 64 lanes (the permlane votes)
        print(f"  plan slices_per_lane={spl}", flush=True)
        plan = ss.ss_plan_create(ctx, b["lengths"], b["E"], spl)
        info = ss.ss_plan_info(plan)
        assert info["items"] > 0 and info["slices_per_lane"] == spl
        out = db.new_out()
        ss.ss_filter_planned_async(ctx, plan, ps, db.total, db.offsets, db.lengths, db.E, out,
                                   torch.cuda.current_stream())
        torch.cuda.synchronize()
        _check(runner.results_numpy(out, db.n), want, f"planned spl={spl}")
        ss.ss_plan_destroy(plan)


def test_shuffled_mix_equals_per_bucket_launches(env):
    """The persistent launch on a shuffled mix equals separate launches per (length, E) bucket."""
    ss, runner, torch = env
    b, want = _mixed(n=8000, n_long=16)
    db = runner.DeviceBatch(b)
    ps = db.pack_stream()
    plan = ss.ss_plan_create(runner.context(), b["lengths"], b["E"], 8)
    out = db.new_out()
    ss.ss_filter_planned_async(runner.context(), plan, ps, db.total, db.offsets, db.lengths, db.E, out)
    torch.cuda.synchronize()
    got = runner.results_numpy(out, db.n)
    keys = sorted(set(zip(b["lengths"].tolist(), b["E"].tolist())))
    for (m, E) in keys:
        idx = np.nonzero((b["lengths"] == m) & (b["E"] == E))[0]
        sub = dict(n=len(idx), reads=b["reads"], refs=b["refs"], offsets=b["offsets"][idx],
                   lengths=b["lengths"][idx], E=None)
        ds = runner.DeviceBatch(sub)
        p2 = ds.pack_stream()
        o2 = ds.filter_wave(p2, int(E))
        torch.cuda.synchronize()
        a2, e2 = runner.results_numpy(o2, ds.n)
        assert np.array_equal(a2, got[0][idx]) and np.array_equal(e2, got[1][idx]), (m, E)
    ss.ss_plan_destroy(plan)
    _check(got, want, "shuffled mix")


def test_graph_replays(env):
    ss, runner, torch = env
    b, want = _mixed(n=6000, n_long=12)
    db = runner.DeviceBatch(b)
    ps = db.pack_stream()
    torch.cuda.synchronize()
    ctx = runner.context()
    plan = ss.ss_plan_create(ctx, b["lengths"], b["E"], 8)
    out = db.new_out()
    ss.ss_plan_capture(ctx, plan, ps, db.total, db.offsets, db.lengths, db.E, out)
    for rep in range(4):
        out.fill_(-1)                                   # eager work between replays
        ss.ss_plan_launch(plan, torch.cuda.current_stream())
        torch.cuda.synchronize()
        _check(runner.results_numpy(out, db.n), want, f"graph replay {rep}")
        eager = db.filter_wave(ps, int(b["E"].max()), per_pair=True)   # eager launch in between
        torch.cuda.synchronize()
        _check(runner.results_numpy(eager, db.n), want, f"eager after replay {rep}")
    ss.ss_plan_destroy(plan)


def test_autotune_cache(env, tmp_path):
    ss, runner, torch = env
    b, want = _mixed(n=6000, n_long=12)
    db = runner.DeviceBatch(b)
    ps = db.pack_stream()
    torch.cuda.synchronize()
    ctx = runner.context()
    cache = str(tmp_path / "tune.json")
    scratch = db.new_out()
    plan, chosen = ss.ss_plan_create_tuned(ctx, b["lengths"], b["E"], ps, db.total, db.offsets, db.lengths, db.E,
                                           scratch, cache)
    assert chosen in (1, 2, 4, 8)
    entries = json.load(open(cache))
    value = list(entries.values())[0]      # slices + 100 x resident blocks per CU (0: as many as fit)
    assert len(entries) == 1 and value % 100 == chosen and value // 100 in (0, 2)
    out = db.new_out()
    ss.ss_filter_planned_async(ctx, plan, ps, db.total, db.offsets, db.lengths, db.E, out)
    torch.cuda.synchronize()
    _check(runner.results_numpy(out, db.n), want, "tuned plan")
    grid = ss.ss_plan_info(plan)["grid"]
    ss.ss_plan_destroy(plan)
    plan2, chosen2 = ss.ss_plan_create_tuned(ctx, b["lengths"], b["E"], ps, db.total, db.offsets, db.lengths, db.E,
                                             scratch, cache)
    assert chosen2 == chosen and ss.ss_plan_info(plan2)["grid"] == grid      # the cached choice, grid included
    ss.ss_plan_destroy(plan2)


def test_empty_plan(env):
    ss, runner, torch = env
    ctx = runner.context()
    plan = ss.ss_plan_create(ctx, np.zeros(0, np.int32), np.zeros(0, np.int32), 8)
    assert ss.ss_plan_info(plan)["items"] == 0
    ss.ss_plan_destroy(plan)


@pytest.mark.parametrize("E", [1000, 5000])
def test_100kbp_pairs(env, E):
    """Pairs of 100 kbp with thresholds up to 5% of the length (2E+1 = 10,001 rows at E = 5000: one
    wavefront per pair, 64 lanes x 5 slices): the wavefront kernel and the planned persistent launch
    against the oracle."""
    ss, runner, torch = env
    b = gen.long_pairs(8, 100_000, 300, 700)
    b["E"] = np.array([E, E // 2, E, E // 5, E, E, E // 10, E], dtype=np.int32)
    want = oracle.batch(b["reads"], b["refs"], b["offsets"], b["lengths"], E_per_pair=b["E"], threads=8)
    assert 0 < int(want["accept"].sum()) < 8 or E == 1000     # both decisions occur at E = 5000
    db = runner.DeviceBatch(b)
    ps = db.pack_stream()
    print(f"  wave m=100000 Emax={E}", flush=True)
    out = db.filter_wave(ps, E, per_pair=True)
    torch.cuda.synchronize()
    _check(runner.results_numpy(out, db.n), (want["accept"], want["edits"]), f"wave E={E}")
    for spl in (4, 8):
        print(f"  planned m=100000 Emax={E} slices_per_lane={spl}", flush=True)
        plan = ss.ss_plan_create(runner.context(), b["lengths"], b["E"], spl)
        out = db.new_out()
        ss.ss_filter_planned_async(runner.context(), plan, ps, db.total, db.offsets, db.lengths, db.E, out)
        torch.cuda.synchronize()
        _check(runner.results_numpy(out, db.n), (want["accept"], want["edits"]), f"planned E={E} spl={spl}")
        ss.ss_plan_destroy(plan)


def test_plan_width_raised_and_limit(env):
    """A plan raises its slice width to hold the largest threshold's rows in one wavefront and
    refuses thresholds beyond 64 lanes x 8 slices (SS_ELEN, nothing launched); so does the server."""
    ss, runner, torch = env
    ctx = runner.context()
    lengths = np.array([1000, 2000], dtype=np.int32)
    for E, want in ((31, 1), (2047, 2), (2048, 4), (5000, 8), (8191, 8)):
        plan = ss.ss_plan_create(ctx, lengths, np.array([E, 3], dtype=np.int32), 1)
        assert ss.ss_plan_info(plan)["slices_per_lane"] == want, E
        ss.ss_plan_destroy(plan)
    with pytest.raises(ss.SSError) as ei:
        ss.ss_plan_create(ctx, lengths, np.array([8192, 3], dtype=np.int32), 8)
    assert ei.value.status == ss.SS_ELEN
    srv = ss.ss_server_create(ctx, 1 << 30, 2)
    b = gen.concat([("ACGT" * 10, "ACGT" * 10)])
    acc = np.zeros(1, np.uint8)
    ed = np.zeros(1, np.int32)
    with pytest.raises(ss.SSError) as ei:
        ss.ss_server_submit(srv, b["reads"], b["refs"], b["lengths"], np.array([9000], np.int32), acc, ed)
    assert ei.value.status == ss.SS_ELEN
    ss.ss_server_destroy(srv)


def _one_lane_batch(shuffle):
    """Pairs whose rows fit one lane (2E+1 <= 31, and 32..63 at two slices): 100 bp pairs whose
    block items fit the LDS stage, 3 kbp pairs whose items do not, and an empty and two one-base
    pairs at the end of the stream.  shuffle: input order unrelated to stream order (every item's
    span of stream words is then large, so the items read global memory)."""
    rng = np.random.default_rng(7)
    a = gen.make(0, n=700)
    bl = gen.long_pairs(300, 3000, 300, 1500, seed=19)
    base = len(a["reads"]) + len(bl["reads"])
    reads = np.concatenate([a["reads"], bl["reads"], np.frombuffer(b"GA", np.uint8)])
    refs = np.concatenate([a["refs"], bl["refs"], np.frombuffer(b"GC", np.uint8)])
    offsets = np.concatenate([[base], a["offsets"], bl["offsets"] + len(a["reads"]), [base, base + 1]])
    lengths = np.concatenate([[0], a["lengths"], bl["lengths"], [1, 1]])
    n = len(lengths)
    E = np.where(rng.random(n) < 0.2, rng.integers(16, 32, n), rng.integers(0, 16, n)).astype(np.int32)
    order = rng.permutation(n) if shuffle else np.arange(n)
    b = dict(n=n, reads=reads, refs=refs, offsets=offsets[order].astype(np.int64),
             lengths=lengths[order].astype(np.int32), E=E)
    want = oracle.batch(b["reads"], b["refs"], b["offsets"], b["lengths"], E_per_pair=b["E"], threads=8)
    return b, (want["accept"], want["edits"])


@pytest.mark.parametrize("shuffle", [False, True])
def test_one_lane_items_staged_and_global(env, shuffle):
    """Items of one-lane pairs: staged in LDS when their stream span fits, else read from global
    memory; both against the oracle, at three slice widths."""
    ss, runner, torch = env
    b, want = _one_lane_batch(shuffle)
    db = runner.DeviceBatch(b)
    ps = db.pack_stream()
    ctx = runner.context()
    for spl in (1, 4, 8):
        print(f"  shuffle={shuffle} slices_per_lane={spl}", flush=True)
        plan = ss.ss_plan_create(ctx, b["lengths"], b["E"], spl)
        out = db.new_out()
        ss.ss_filter_planned_async(ctx, plan, ps, db.total, db.offsets, db.lengths, db.E, out)
        torch.cuda.synchronize()
        _check(runner.results_numpy(out, db.n), want, f"one-lane items shuffle={shuffle} spl={spl}")
        ss.ss_plan_destroy(plan)


def test_stream_limit_refused_before_launch(env):
    """A bit stream longer than SS_MAX_STREAM_BASES (planes past 4 GiB) is refused with SS_ELEN by the
    wavefront, planned and capture calls before anything is enqueued; outputs stay untouched."""
    ss, runner, torch = env
    b, _ = _mixed(n=2000, n_long=2)
    db = runner.DeviceBatch(b)
    ps = db.pack_stream()
    ctx = runner.context()
    plan = ss.ss_plan_create(ctx, b["lengths"], b["E"], 4)
    out = db.new_out()
    out.fill_(-1)
    torch.cuda.synchronize()
    too_long = ss.SS_MAX_STREAM_BASES + 1
    calls = [lambda: ss.ss_filter_planned_async(ctx, plan, ps, too_long, db.offsets, db.lengths, db.E, out),
             lambda: ss.ss_plan_capture(ctx, plan, ps, too_long, db.offsets, db.lengths, db.E, out),
             lambda: ss.ss_filter_wave_async(ctx, ps, too_long, db.offsets, db.lengths, db.E, db.n,
                                             int(b["E"].max()), out)]
    for call in calls:
        with pytest.raises(ss.SSError) as e:
            call()
        assert e.value.status == ss.SS_ELEN
    torch.cuda.synchronize()
    assert bool((out == -1).all())
    ss.ss_plan_destroy(plan)


def _random_batch(rng, n):
    """n pairs of random lengths (0..2000, 32-bit word edges over-represented) and thresholds (0..250),
    references made from the read by substitutions at a per-pair rate (some unrelated), stored back to back."""
    edges = np.array([0, 1, 2, 31, 32, 33, 63, 64, 65, 95, 96, 97, 127, 128, 129, 255, 256, 257], np.int32)
    lengths = np.where(rng.random(n) < 0.3, rng.choice(edges, n),
                       np.exp(rng.uniform(0, np.log(2000), n)).astype(np.int32))
    E = np.minimum(rng.integers(0, 251, n), np.maximum(lengths // 4, rng.integers(0, 6, n))).astype(np.int32)
    bases = np.frombuffer(b"ACGT", np.uint8)
    reads, refs = [], []
    for m in lengths:
        r = rng.choice(bases, int(m))
        q = r.copy()
        if rng.random() < 0.1:
            q = rng.choice(bases, int(m))
        else:
            hit = rng.random(int(m)) < rng.uniform(0, 0.2)
            q[hit] = rng.choice(bases, int(hit.sum()))
        reads.append(q)
        refs.append(r)
    offsets = np.zeros(n, np.int64)
    offsets[1:] = np.cumsum(lengths[:-1])
    return dict(n=n, reads=np.concatenate(reads) if n else np.zeros(0, np.uint8),
                refs=np.concatenate(refs) if n else np.zeros(0, np.uint8), offsets=offsets,
                lengths=lengths.astype(np.int32), E=E)


@pytest.mark.parametrize("seed", range(6))
def test_random_batches_against_oracle(env, seed):
    """Random lengths and thresholds (every block kind of the wavefront sweep, partial last blocks, 1 to 64
    lanes per pair, staged and unstaged one-lane items), in input order and shuffled, at every slice width:
    the planned launch and the standalone wavefront kernel against the oracle."""
    ss, runner, torch = env
    rng = np.random.default_rng(1000 + seed)
    b = _random_batch(rng, 1500)
    if seed % 2:
        order = rng.permutation(b["n"])
        b = dict(b, offsets=b["offsets"][order], lengths=b["lengths"][order], E=b["E"][order])
    want = oracle.batch(b["reads"], b["refs"], b["offsets"], b["lengths"], E_per_pair=b["E"], threads=8)
    want = (want["accept"], want["edits"])
    db = runner.DeviceBatch(b)
    ps = db.pack_stream()
    ctx = runner.context()
    spl = (1, 2, 4, 8)[seed % 4]
    print(f"  seed={seed} slices_per_lane={spl} Emax={int(b['E'].max())}", flush=True)
    plan = ss.ss_plan_create(ctx, b["lengths"], b["E"], spl)
    out = db.new_out()
    ss.ss_filter_planned_async(ctx, plan, ps, db.total, db.offsets, db.lengths, db.E, out)
    torch.cuda.synchronize()
    _check(runner.results_numpy(out, db.n), want, f"planned seed={seed}")
    ss.ss_plan_destroy(plan)
    wout = db.filter_wave(ps, int(b["E"].max()), per_pair=True)
    torch.cuda.synchronize()
    _check(runner.results_numpy(wout, db.n), want, f"wavefront seed={seed}")
