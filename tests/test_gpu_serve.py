"""GPU tests of the serving loop: exactness alone and in the mix, budget and slot
limits, queueing, time-outs, cancellation, error reporting."""
import numpy as np
import pytest

import oracle
from paper_1910_09020_amd import gen

pytestmark = pytest.mark.gpu
SEED = 1910090204


@pytest.fixture(scope="module")
def env():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1910_09020_amd as ss
    from paper_1910_09020_amd import runner
    ss.lib()
    return ss, runner.context()


def request(i, max_pairs=256, max_len=3000):
    return gen.request(SEED, i, max_pairs=max_pairs, max_len=max_len)


def want(r):
    w = oracle.batch(r["reads"], r["refs"], r["offsets"], r["lengths"], E_per_pair=r["E"], threads=8)
    return w["accept"], w["edits"]


def submit(ss, srv, r):
    acc = np.full(r["n"], 255, np.uint8)
    ed = np.full(r["n"], -1, np.int32)
    t = ss.ss_server_submit(srv, r["reads"], r["refs"], r["lengths"], r["E"], acc, ed)
    return t, acc, ed


def test_alone_and_in_mix_are_identical(env):
    ss, ctx = env
    srv = ss.ss_server_create(ctx, 1 << 30, 4)
    try:
        x = request(7)
        t, acc, ed = submit(ss, srv, x)
        assert ss.ss_server_wait(srv, t, 60_000_000) == ss.SS_OK
        wa, we = want(x)
        assert np.array_equal(acc, wa) and np.array_equal(ed, we)
        mix = [request(100 + i) for i in range(24)]
        mix.insert(11, x)
        subs = [submit(ss, srv, r) for r in mix]
        for r, (t2, a2, e2) in zip(mix, subs):
            assert ss.ss_server_wait(srv, t2, 60_000_000) == ss.SS_OK
            wa2, we2 = want(r)
            assert np.array_equal(a2, wa2) and np.array_equal(e2, we2)
        # the request inside the mix equals the request alone
        assert np.array_equal(subs[11][1], acc) and np.array_equal(subs[11][2], ed)
        st = ss.ss_server_stats(srv)
        assert st["completed"] == 26 and st["peak_in_flight"] >= 1
        # every slice width gives the same results
        for spl in (1, 4, 8):
            ss.ss_server_set_slices(srv, spl)
            t3, a3, e3 = submit(ss, srv, x)
            assert ss.ss_server_wait(srv, t3, 60_000_000) == ss.SS_OK
            assert np.array_equal(a3, acc) and np.array_equal(e3, ed), spl
    finally:
        ss.ss_server_destroy(srv)


def test_budget_and_slot_exhaustion_queue_and_complete(env):
    ss, ctx = env
    reqs = [request(200 + i) for i in range(10)]
    fps = [ss.ss_server_footprint(r["n"], len(r["reads"])) for r in reqs]
    budget = max(fps) + 4096               # room for one request at a time
    srv = ss.ss_server_create(ctx, budget, 3)
    try:
        subs = [submit(ss, srv, r) for r in reqs]
        for r, (t, a, e) in zip(reqs, subs):
            assert ss.ss_server_wait(srv, t, 60_000_000) == ss.SS_OK
            wa, we = want(r)
            assert np.array_equal(a, wa) and np.array_equal(e, we)
        st = ss.ss_server_stats(srv)
        assert st["completed"] == len(reqs)
        assert 0 < st["peak_bytes"] <= budget
    finally:
        ss.ss_server_destroy(srv)
    # a request that alone exceeds the budget is refused at submission
    small = ss.ss_server_create(ctx, 1 << 16, 2)
    try:
        big = request(300, max_pairs=2048, max_len=10000)
        with pytest.raises(ss.SSError) as ei:
            submit(ss, small, big)
        assert ei.value.status == ss.SS_EBUDGET
    finally:
        ss.ss_server_destroy(small)


def test_hold_timeout_and_cancel(env):
    ss, ctx = env
    srv = ss.ss_server_create(ctx, 1 << 30, 2)
    try:
        ss.ss_server_set_hold(srv, True)
        a = request(400)
        b = request(401)
        ta, acc_a, ed_a = submit(ss, srv, a)
        tb, acc_b, ed_b = submit(ss, srv, b)
        assert ss.ss_server_wait(srv, ta, 20_000) == ss.SS_ETIMEOUT      # held: the deadline passes
        assert not ss.ss_server_poll(srv, ta)
        assert ss.ss_server_cancel(srv, tb) == ss.SS_OK
        ss.ss_server_set_hold(srv, False)
        assert ss.ss_server_wait(srv, ta, 60_000_000) == ss.SS_OK
        assert ss.ss_server_wait(srv, tb, 1000) == ss.SS_EAGAIN          # cancelled
        assert np.all(acc_b == 255)                                       # never written
        wa, we = want(a)
        assert np.array_equal(acc_a, wa) and np.array_equal(ed_a, we)
        s, ad, d = ss.ss_server_times(srv, ta)
        assert s <= ad <= d
        assert ss.ss_server_release(srv, ta) == ss.SS_OK
    finally:
        ss.ss_server_destroy(srv)


def test_bad_base_and_empty(env):
    ss, ctx = env
    srv = ss.ss_server_create(ctx, 1 << 30, 2)
    try:
        r = request(500)
        r["refs"] = r["refs"].copy()
        r["refs"][3] = ord("N")
        t, acc, ed = submit(ss, srv, r)
        assert ss.ss_server_wait(srv, t, 60_000_000) == ss.SS_EBASE
        assert np.all(acc == 255) and np.all(ed == -1)
        e = dict(reads=np.zeros(0, np.uint8), refs=np.zeros(0, np.uint8), lengths=np.zeros(0, np.int32),
                 E=np.zeros(0, np.int32), n=0)
        t0, _, _ = submit(ss, srv, e)
        assert ss.ss_server_wait(srv, t0, 1000) == ss.SS_OK
    finally:
        ss.ss_server_destroy(srv)


def test_staged_submissions_on_slot_streams(env):
    """Staged submissions (bases written into blocks of the server's staging, copied to the device
    from there on the slot's stream) mixed with copied ones, with the slots full: every result
    equals the oracle's; a bad base in a staged request is reported with the outputs untouched."""
    ss, ctx = env
    print("host server: staged submissions", flush=True)
    srv = ss.ss_server_create(ctx, 1 << 28, 4)
    try:
        def staged(r):
            T = len(r["reads"])
            roff = (T + 15) // 16 * 16
            blk = ss.ss_server_stage_alloc(srv, roff + max(T, 1))
            assert blk
            v = ss.stage_view(blk, roff + T)
            v[:T] = r["reads"]
            v[roff:roff + T] = r["refs"]
            acc = np.full(r["n"], 255, np.uint8)
            ed = np.full(r["n"], -1, np.int32)
            return ss.ss_server_submit_staged(srv, blk, roff, r["lengths"], r["E"], acc, ed), acc, ed

        reqs = [request(1300 + i, max_pairs=512, max_len=6000) for i in range(24)]
        subs = [staged(r) if i % 2 else submit(ss, srv, r) for i, r in enumerate(reqs)]
        for r, (t, a, e) in zip(reqs, subs):
            assert ss.ss_server_wait(srv, t, 60_000_000) == ss.SS_OK
            wa, we = want(r)
            assert np.array_equal(a, wa) and np.array_equal(e, we)
        bad = dict(reqs[3])
        bad["refs"] = bad["refs"].copy()
        bad["refs"][5] = ord("N")
        t, a, e = staged(bad)
        assert ss.ss_server_wait(srv, t, 60_000_000) == ss.SS_EBASE
        assert np.all(a == 255) and np.all(e == -1)
    finally:
        ss.ss_server_destroy(srv)
