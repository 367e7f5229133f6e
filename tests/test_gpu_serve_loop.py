"""GPU tests of the device-resident serving loop (ss_server_create_loop): exactness against the
oracle alone and in the mix, slot reuse, admission by the arena budget, the loop kernel ending when
idle and being launched again, queueing controls, error reporting and refusals."""
import time

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


def planes_bytes(total):
    return (((total + 31) // 32 + 2) * 16 + 255) // 256 * 256


def test_loop_alone_and_in_mix_match_oracle(env):
    ss, ctx = env
    print("loop server: 1 request alone, then 40 in flight together", flush=True)
    srv = ss.ss_server_create_loop(ctx, 1 << 30, 16, 1)
    try:
        x = request(7)
        t, acc, ed = submit(ss, srv, x)
        assert ss.ss_server_wait(srv, t, 60_000_000) == ss.SS_OK
        wa, we = want(x)
        assert np.array_equal(acc, wa) and np.array_equal(ed, we)
        mix = [request(100 + i) for i in range(40)]
        mix.insert(17, x)
        subs = [submit(ss, srv, r) for r in mix]
        for r, (t2, a2, e2) in zip(mix, subs):
            assert ss.ss_server_wait(srv, t2, 60_000_000) == ss.SS_OK
            wa2, we2 = want(r)
            assert np.array_equal(a2, wa2) and np.array_equal(e2, we2)
        assert np.array_equal(subs[17][1], acc) and np.array_equal(subs[17][2], ed)
        st = ss.ss_server_stats(srv)
        assert st["completed"] == 42 and st["peak_in_flight"] >= 2
        for t2, _, _ in subs:
            h2d, comp = ss.ss_server_stages(srv, t2)[1:3]
            assert h2d >= 0 and comp > 0
    finally:
        ss.ss_server_destroy(srv)


def test_loop_large_and_small_requests_together(env):
    """A request of many encoding units (thousands of 10 kbp pairs) beside small ones, every slot reused."""
    ss, ctx = env
    print("loop server: large + small requests, 4 slots", flush=True)
    srv = ss.ss_server_create_loop(ctx, 1 << 30, 4, 1)
    try:
        reqs = [request(600, max_pairs=4096, max_len=10000)] + [request(610 + i, max_pairs=64) for i in range(30)]
        assert len(reqs[0]["reads"]) > 32 * 1024 * 8          # several encoding units
        subs = [submit(ss, srv, r) for r in reqs]
        for r, (t, a, e) in zip(reqs, subs):
            assert ss.ss_server_wait(srv, t, 120_000_000) == ss.SS_OK
            wa, we = want(r)
            assert np.array_equal(a, wa) and np.array_equal(e, we)
    finally:
        ss.ss_server_destroy(srv)


def test_loop_budget_admission_and_refusal(env):
    ss, ctx = env
    print("loop server: arena budget of one request at a time", flush=True)
    reqs = [request(200 + i) for i in range(10)]
    budget = max(planes_bytes(len(r["reads"])) for r in reqs)
    srv = ss.ss_server_create_loop(ctx, budget, 8, 1)
    try:
        subs = [submit(ss, srv, r) for r in reqs]
        for r, (t, a, e) in zip(reqs, subs):
            assert ss.ss_server_wait(srv, t, 60_000_000) == ss.SS_OK
            wa, we = want(r)
            assert np.array_equal(a, wa) and np.array_equal(e, we)
        st = ss.ss_server_stats(srv)
        assert st["completed"] == len(reqs)
        assert 0 < st["peak_bytes"] <= budget
        # all ten requests as one: its planes alone exceed the arena
        big = dict(reads=np.concatenate([r["reads"] for r in reqs]), refs=np.concatenate([r["refs"] for r in reqs]),
                   lengths=np.concatenate([r["lengths"] for r in reqs]), E=np.concatenate([r["E"] for r in reqs]))
        big["n"] = len(big["lengths"])
        assert planes_bytes(len(big["reads"])) > budget
        with pytest.raises(ss.SSError) as ei:
            submit(ss, srv, big)
        assert ei.value.status == ss.SS_EBUDGET
    finally:
        ss.ss_server_destroy(srv)


def test_loop_ends_when_idle_and_restarts(env):
    ss, ctx = env
    print("loop server: requests 0.5 s apart (the kernel ends after 0.2 s idle)", flush=True)
    srv = ss.ss_server_create_loop(ctx, 1 << 28, 4, 2)
    try:
        for k in range(3):
            r = request(700 + k)
            t, a, e = submit(ss, srv, r)
            assert ss.ss_server_wait(srv, t, 60_000_000) == ss.SS_OK
            wa, we = want(r)
            assert np.array_equal(a, wa) and np.array_equal(e, we)
            time.sleep(0.5)
    finally:
        ss.ss_server_destroy(srv)


def test_loop_hold_cancel_bad_base_empty_and_refusals(env):
    ss, ctx = env
    print("loop server: hold, cancel, bad base, empty and zero-length requests, refusals", flush=True)
    srv = ss.ss_server_create_loop(ctx, 1 << 28, 2, 1)
    try:
        ss.ss_server_set_hold(srv, True)
        a = request(400)
        b = request(401)
        ta, acc_a, ed_a = submit(ss, srv, a)
        tb, acc_b, _ = submit(ss, srv, b)
        assert ss.ss_server_wait(srv, ta, 20_000) == ss.SS_ETIMEOUT
        assert ss.ss_server_cancel(srv, tb) == ss.SS_OK
        ss.ss_server_set_hold(srv, False)
        assert ss.ss_server_wait(srv, ta, 60_000_000) == ss.SS_OK
        assert ss.ss_server_wait(srv, tb, 1000) == ss.SS_EAGAIN
        assert np.all(acc_b == 255)
        wa, we = want(a)
        assert np.array_equal(acc_a, wa) and np.array_equal(ed_a, we)

        r = request(500)
        r["refs"] = r["refs"].copy()
        r["refs"][3] = ord("N")
        t, acc, ed = submit(ss, srv, r)
        assert ss.ss_server_wait(srv, t, 60_000_000) == ss.SS_EBASE
        assert np.all(acc == 255) and np.all(ed == -1)
        # the slot and its arena room are reusable after the error
        r2 = request(501)
        t2, a2, e2 = submit(ss, srv, r2)
        assert ss.ss_server_wait(srv, t2, 60_000_000) == ss.SS_OK
        wa2, we2 = want(r2)
        assert np.array_equal(a2, wa2) and np.array_equal(e2, we2)

        e = dict(reads=np.zeros(0, np.uint8), refs=np.zeros(0, np.uint8), lengths=np.zeros(0, np.int32),
                 E=np.zeros(0, np.int32), n=0)
        t0, _, _ = submit(ss, srv, e)
        assert ss.ss_server_wait(srv, t0, 1000) == ss.SS_OK
        z = dict(reads=np.zeros(0, np.uint8), refs=np.zeros(0, np.uint8), lengths=np.zeros(5, np.int32),
                 E=np.array([0, 1, 2, 3, 4], np.int32), n=5)
        tz, az, ez = submit(ss, srv, z)
        assert ss.ss_server_wait(srv, tz, 60_000_000) == ss.SS_OK
        assert np.all(az == 1) and np.all(ez == 0)

        # a threshold that needs two slices per lane on a one-slice loop is refused
        w = request(502, max_pairs=4)
        w["E"] = np.full(w["n"], 1500, np.int32)
        with pytest.raises(ss.SSError) as ei:
            submit(ss, srv, w)
        assert ei.value.status == ss.SS_ELEN
        with pytest.raises(ss.SSError):
            ss.ss_server_set_slices(srv, 2)
        # one device-resident loop per device
        with pytest.raises(ss.SSError) as ei:
            ss.ss_server_create_loop(ctx, 1 << 20, 2, 1)
        assert ei.value.status == ss.SS_EAGAIN
    finally:
        ss.ss_server_destroy(srv)
    # free again once the first is gone
    srv2 = ss.ss_server_create_loop(ctx, 1 << 20, 2, 1)
    ss.ss_server_destroy(srv2)


def test_loop_destroy_waits_for_requests_in_flight(env):
    ss, ctx = env
    print("loop server: destroy with 64 requests in flight", flush=True)
    srv = ss.ss_server_create_loop(ctx, 1 << 30, 64, 1)
    reqs = [request(800 + i, max_pairs=128) for i in range(64)]
    subs = [submit(ss, srv, r) for r in reqs]
    ss.ss_server_destroy(srv)
    # every admitted request finished before destroy returned; queued ones were cancelled (outputs untouched)
    done = 0
    for r, (_, a, e) in zip(reqs, subs):
        if np.all(a == 255) and np.all(e == -1):
            continue
        wa, we = want(r)
        assert np.array_equal(a, wa) and np.array_equal(e, we)
        done += 1
    assert done >= 1


def test_loop_staging_beyond_the_pinned_region(env):
    """Staging is taken at submission: with the server on hold, 90 requests of about 0.3 MB of
    staging each outgrow the 16 MiB region pinned at creation (the smallest, for a 4 MiB budget),
    so the later ones take blocks pinned on demand.  Released, every result equals the oracle's,
    and the region's ranges are reused by the next requests."""
    ss, ctx = env
    print("loop server: 90 held requests past the staging region, then 20 more", flush=True)
    srv = ss.ss_server_create_loop(ctx, 4 << 20, 16, 1)
    try:
        ss.ss_server_set_hold(srv, True)
        reqs = [request(1000 + i, max_pairs=256, max_len=4000) for i in range(90)]
        staged = sum(2 * len(r["reads"]) + 24 * r["n"] for r in reqs)      # a lower bound of the staging
        assert staged > 20 << 20, staged
        subs = [submit(ss, srv, r) for r in reqs]
        ss.ss_server_set_hold(srv, False)
        more = [request(1100 + i, max_pairs=256, max_len=4000) for i in range(20)]
        subs += [submit(ss, srv, r) for r in more]
        for r, (t, a, e) in zip(reqs + more, subs):
            assert ss.ss_server_wait(srv, t, 60_000_000) == ss.SS_OK
            wa, we = want(r)
            assert np.array_equal(a, wa) and np.array_equal(e, we)
    finally:
        ss.ss_server_destroy(srv)


def submit_staged(ss, srv, r):
    """Write the request's bases into a block of the server's staging and submit it without a copy."""
    T = len(r["reads"])
    roff = (T + 15) // 16 * 16
    blk = ss.ss_server_stage_alloc(srv, roff + max(T, 1))
    assert blk
    v = ss.stage_view(blk, roff + T)
    v[:T] = r["reads"]
    v[roff:roff + T] = r["refs"]
    acc = np.full(r["n"], 255, np.uint8)
    ed = np.full(r["n"], -1, np.int32)
    t = ss.ss_server_submit_staged(srv, blk, roff, r["lengths"], r["E"], acc, ed)
    return t, acc, ed


def test_loop_staged_submissions(env):
    """Requests whose bases are written into blocks of the server's staging and read from there on the
    device (no copy at submission), mixed with copied ones: every result equals the oracle's.
    Refusals leave the block with the caller; a submitted block is no longer the caller's."""
    ss, ctx = env
    print("loop server: staged submissions", flush=True)
    srv = ss.ss_server_create_loop(ctx, 1 << 28, 16, 1)
    try:
        reqs = [request(1200 + i, max_pairs=512, max_len=6000) for i in range(30)]
        subs = [(submit_staged if i % 3 else submit)(ss, srv, r) for i, r in enumerate(reqs)]
        for r, (t, a, e) in zip(reqs, subs):
            assert ss.ss_server_wait(srv, t, 60_000_000) == ss.SS_OK
            wa, we = want(r)
            assert np.array_equal(a, wa) and np.array_equal(e, we)
        # refusals: the sides overlap, or the references run past the block
        r = reqs[0]
        T = len(r["reads"])
        blk = ss.ss_server_stage_alloc(srv, 2 * T + 16)
        acc = np.zeros(r["n"], np.uint8)
        ed = np.zeros(r["n"], np.int32)
        L = ss.lib()
        for roff in (T - 1, T + 32):
            rc = L.ss_server_submit_staged(srv, blk, roff, ss._ptr(r["lengths"]), ss._ptr(r["E"]), r["n"],
                                           ss._ptr(acc), ss._ptr(ed), ss.ctypes.byref(ss.ctypes.c_uint64(0)))
            assert rc == ss.SS_EINVAL
        ss.ss_server_stage_free(srv, blk)                 # still the caller's after the refusals
        with pytest.raises(ss.SSError):
            ss.ss_server_stage_free(srv, blk)             # not twice
        with pytest.raises(ss.SSError):
            ss.ss_server_stage_free(srv, 4096)            # not a block of the staging
        t, a, e = submit_staged(ss, srv, reqs[1])
        assert ss.ss_server_wait(srv, t, 60_000_000) == ss.SS_OK
        # held and cancelled: the block returns to the staging with the request
        ss.ss_server_set_hold(srv, True)
        t2, _, _ = submit_staged(ss, srv, reqs[2])
        assert ss.ss_server_cancel(srv, t2) == ss.SS_OK
        ss.ss_server_set_hold(srv, False)
        # an empty staged request completes at once
        z = dict(reads=np.zeros(0, np.uint8), refs=np.zeros(0, np.uint8), lengths=np.zeros(0, np.int32),
                 E=np.zeros(0, np.int32), n=0)
        tz, _, _ = submit_staged(ss, srv, z)
        assert ss.ss_server_wait(srv, tz, 1000) == ss.SS_OK
        assert ss.ss_server_stage_alloc(srv, 0) is None
        assert ss.ss_server_stage_alloc(srv, 1 << 62) is None    # beyond the staging's cap
        left = ss.ss_server_stage_alloc(srv, 1 << 20)     # held at destroy: freed with the server
        assert left
    finally:
        ss.ss_server_destroy(srv)


def test_loop_relaunch_race_with_a_tiny_idle_time(env):
    """With the loop's idle time at 20 microseconds the kernel ends between requests over and over, so
    requests are published just as it ends (the host launches it again when it finds the last launch
    done with a request waiting); requests come from four threads at random gaps, two of them
    submitting staged (taking, filling and handing over blocks of the staging concurrently).  Every
    result equals the oracle's."""
    import random
    import threading
    ss, ctx = env
    print("loop server: 20 us idle time, 4 submitting threads", flush=True)
    srv = ss.ss_server_create_loop(ctx, 1 << 28, 8, 1)
    try:
        ss.ss_server_set_loop_idle(srv, 20)
        reqs = [request(900 + i, max_pairs=64, max_len=1500) for i in range(48)]
        subs = [None] * len(reqs)
        errors = []

        def work(k):
            rng = random.Random(k)
            try:
                for i in range(k, len(reqs), 4):
                    time.sleep(rng.choice([0, 0, 0.00005, 0.0003, 0.002]))
                    subs[i] = (submit_staged if k % 2 else submit)(ss, srv, reqs[i])
            except Exception as ex:          # reported below
                errors.append(repr(ex))

        th = [threading.Thread(target=work, args=(k,)) for k in range(4)]
        for t in th:
            t.start()
        for t in th:
            t.join()
        assert not errors, errors
        for r, (t, a, e) in zip(reqs, subs):
            assert ss.ss_server_wait(srv, t, 60_000_000) == ss.SS_OK
            wa, we = want(r)
            assert np.array_equal(a, wa) and np.array_equal(e, we)
    finally:
        ss.ss_server_destroy(srv)
    with pytest.raises(ss.SSError):
        host = ss.ss_server_create(ctx, 1 << 20, 2)
        try:
            ss.ss_server_set_loop_idle(host, 100)      # not a loop server
        finally:
            ss.ss_server_destroy(host)
