"""The batch-descriptor boundary (ss_pack, ss_filter_batch_ex, ss_filter_batch_pairs) on the GPU.

Every kernel choice, forced and automatic, every input form (ASCII, each side packed apart by ss_pack,
the lane-sliced buffer) and pairs of unequal length are compared with the CPU oracle on every pair;
forcing a kernel a batch does not fit is an error before any work is enqueued; the one-call host entry
points give each caller its own results when called from several threads at once.
"""
import threading

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
    return torch, ss, runner


def say(msg):
    print(msg, flush=True)


def check(name, got, want):
    bad = np.nonzero((got[0] != want[0]) | (got[1] != want[1]))[0]
    assert len(bad) == 0, f"{name}: {len(bad)} of {len(want[0])} pairs differ from the oracle, first {bad[:5]}"


def oracle_eq(b, E=None, Epp=None):
    w = oracle.batch(b["reads"], b["refs"], b["offsets"], b["lengths"], E=E, E_per_pair=Epp, threads=8)
    return w["accept"], w["edits"]


class Dev:
    """A batch on the device with every input form the descriptor takes."""

    def __init__(self, rt, b, Epp=None):
        torch, ss, runner = rt
        self.torch, self.ss, self.runner = torch, ss, runner
        self.b = b
        self.db = runner.DeviceBatch(b)
        self.n = self.db.n
        d = torch.device("cuda")
        self.err = torch.zeros(1, dtype=torch.int32, device=d)
        self.out = torch.empty(max(8, self.n), dtype=torch.int16, device=d)
        self.E = None if Epp is None else torch.from_numpy(np.ascontiguousarray(Epp, dtype=np.int32)).to(d)
        total = self.db.total
        self.q = torch.empty(ss.ss_pack_words(total), dtype=torch.int32, device=d)
        self.r = torch.empty(ss.ss_pack_words(total), dtype=torch.int32, device=d)
        ctx = runner.context()
        ss.ss_pack(ctx, self.db.reads, total, self.q, self.err, torch.cuda.current_stream())
        ss.ss_pack(ctx, self.db.refs, total, self.r, self.err, torch.cuda.current_stream())
        torch.cuda.synchronize()
        assert int(self.err.item()) == 0

    def run(self, flags, E, packed=False, uniform=None, offsets=True, Epp=False, plan=None, sliced=None):
        ss, torch = self.ss, self.torch
        self.out.fill_(-1)
        desc = ss.batch_desc(
            sliced if sliced is not None else (self.q if packed else self.db.reads),
            None if sliced is not None else (self.r if packed else self.db.refs),
            self.n, E, flags, self.out, err=self.err,
            offsets=self.db.offsets if offsets else None,
            lengths=self.db.lengths if offsets else None,
            E_per_pair=self.E if Epp else None, plan=plan,
            read_bases=self.db.total, ref_bases=self.db.total,
            length=-1 if uniform is None else uniform)
        ss.ss_filter_batch_ex(self.runner.context(), desc, torch.cuda.current_stream())
        torch.cuda.synchronize()
        assert int(self.err.item()) == 0
        return self.runner.results_numpy(self.out, self.n)


def test_every_kernel_equal_lengths(rt):
    torch, ss, runner = rt
    b = gen.make(1, n=40_000 + 13)
    D = Dev(rt, b)
    m = 100
    ascii_ = ss.SS_INPUT_ASCII
    pk = ss.SS_INPUT_PACKED
    sl = D.db.pack_sliced()
    torch.cuda.synchronize()
    for E in (0, 3, 5, 9):
        want = oracle_eq(b, E)
        say(f"  E={E}")
        check(f"auto ascii back to back E={E}", D.run(ascii_ | ss.SS_KERNEL_AUTO, E, uniform=m, offsets=False), want)
        check(f"fused E={E}", D.run(ascii_ | ss.SS_KERNEL_FUSED, E, uniform=m, offsets=False), want)
        check(f"auto ascii with offsets E={E}", D.run(ascii_ | ss.SS_KERNEL_AUTO, E, uniform=m), want)
        check(f"sliced from ascii E={E}", D.run(ascii_ | ss.SS_KERNEL_SLICED, E, uniform=m), want)
        check(f"sliced input E={E}", D.run(ss.SS_INPUT_PACKED_SLICED, E, uniform=m, offsets=False, sliced=sl), want)
        check(f"plain from ascii E={E}", D.run(ascii_ | ss.SS_KERNEL_PLAIN, E), want)
        check(f"plain packed E={E}", D.run(pk | ss.SS_KERNEL_PLAIN, E, packed=True), want)
        check(f"wave packed E={E}", D.run(pk | ss.SS_KERNEL_WAVE, E, packed=True), want)
        check(f"auto packed E={E}", D.run(pk | ss.SS_KERNEL_AUTO, E, packed=True), want)
        check(f"wave packed, uniform without arrays E={E}",
              D.run(pk | ss.SS_KERNEL_WAVE, E, packed=True, uniform=m, offsets=False), want)


def test_mixed_lengths_per_pair_E_and_plan(rt):
    torch, ss, runner = rt
    b = gen.make(3, n=30_000, n_long=12)
    D = Dev(rt, b, Epp=b["E"])
    Emax = int(b["E"].max())
    want = oracle_eq(b, Epp=b["E"])
    pk = ss.SS_INPUT_PACKED
    say("  auto, mixed lengths, per-pair thresholds")
    check("auto ascii", D.run(ss.SS_INPUT_ASCII, Emax, Epp=True), want)
    check("wave packed", D.run(pk | ss.SS_KERNEL_WAVE, Emax, packed=True, Epp=True), want)
    ctx = runner.context()
    plan = ss.ss_plan_create(ctx, b["lengths"], b["E"], 4)
    try:
        say("  persistent launch of a plan")
        check("persistent packed", D.run(pk | ss.SS_KERNEL_PERSISTENT, Emax, packed=True, Epp=True, plan=plan), want)
        check("auto with a plan, ascii", D.run(ss.SS_INPUT_ASCII, Emax, Epp=True, plan=plan), want)
    finally:
        ss.ss_plan_destroy(plan)
    short = b["lengths"] < 1000
    if int(b["E"][short].max()) <= 31:
        pass   # the one-pair-per-lane kernel needs E <= 31 for every pair; covered in the equal-length test


def test_unequal_lengths(rt):
    """Pairs of unequal length through the descriptor (each side packed apart, the references at offsets and
    lengths of their own) and through the host one-call, against the oracle's unequal-length walk."""
    torch, ss, runner = rt
    d = gen.uneq(50_000, m=100, kmax=12, unrel_pct=10)
    n = d["n"]
    dev = torch.device("cuda")
    qt, rt_ = int(d["reads"].size), int(d["refs"].size)
    reads = torch.from_numpy(d["reads"]).to(dev)
    refs = torch.from_numpy(d["refs"]).to(dev)
    qoff = torch.from_numpy(d["read_offsets"]).to(dev)
    qlen = torch.from_numpy(d["read_lengths"]).to(dev)
    roff = torch.from_numpy(d["ref_offsets"]).to(dev)
    rlen = torch.from_numpy(d["ref_lengths"]).to(dev)
    err = torch.zeros(1, dtype=torch.int32, device=dev)
    out = torch.empty(n + 8, dtype=torch.int16, device=dev)
    qp = torch.empty(ss.ss_pack_words(qt), dtype=torch.int32, device=dev)
    rp = torch.empty(ss.ss_pack_words(rt_), dtype=torch.int32, device=dev)
    ctx = runner.context()
    st = torch.cuda.current_stream()
    ss.ss_pack(ctx, reads, qt, qp, err, st)
    ss.ss_pack(ctx, refs, rt_, rp, err, st)
    rng = np.random.default_rng(3)
    Epp = rng.integers(0, 16, size=n).astype(np.int32)
    dE = torch.from_numpy(Epp).to(dev)
    for E, per_pair in ((0, False), (3, False), (8, False), (15, True)):
        w = oracle.batch_uneq(d["reads"], d["read_offsets"], d["read_lengths"], d["refs"], d["ref_offsets"],
                              d["ref_lengths"], E=E, E_per_pair=Epp if per_pair else None, threads=8)
        want = (w["accept"], w["edits"])
        for form in ("ascii", "packed"):
            say(f"  unequal lengths E={E} per_pair={per_pair} {form}")
            out.fill_(-1)
            desc = ss.batch_desc(reads if form == "ascii" else qp, refs if form == "ascii" else rp, n, E,
                                 (ss.SS_INPUT_ASCII if form == "ascii" else ss.SS_INPUT_PACKED) | ss.SS_KERNEL_AUTO,
                                 out, err=err, offsets=qoff, lengths=qlen, ref_offsets=roff, ref_lengths=rlen,
                                 E_per_pair=dE if per_pair else None, read_bases=qt, ref_bases=rt_)
            ss.ss_filter_batch_ex(ctx, desc, st)
            torch.cuda.synchronize()
            assert int(err.item()) == 0
            check(f"uneq {form} E={E}", runner.results_numpy(out, n), want)
        say(f"  host one-call, unequal lengths, E={E}")
        acc, ed = ss.ss_filter_batch_pairs(d["reads"], d["read_lengths"], d["refs"], d["ref_lengths"], E=E,
                                           E_per_pair=Epp if per_pair else None)
        check(f"ss_filter_batch_pairs E={E}", (acc, ed), want)


def test_unequal_edge_cases(rt):
    """Empty sides, a reference that is a prefix of its query, references longer than their query by more
    than E, long pairs (several 32-column blocks and lanes per pair)."""
    torch, ss, runner = rt
    rng = np.random.default_rng(11)
    A = np.frombuffer(b"ACGT", np.uint8)
    pairs = []
    for n_q, n_r in ((0, 0), (0, 7), (7, 0), (1, 1), (5, 40), (40, 5), (31, 33), (33, 31), (64, 64), (100, 160),
                     (160, 100), (700, 720), (2000, 1990)):
        q = rng.choice(A, size=n_q)
        if n_r <= n_q:
            r = q[:n_r].copy()
        else:
            r = np.concatenate([q, rng.choice(A, size=n_r - n_q)])
        if n_r > 3:
            r[rng.integers(0, n_r, size=max(1, n_r // 20))] = rng.choice(A, size=max(1, n_r // 20))
        pairs.append((q, r))
    reads = np.concatenate([p[0] for p in pairs]) if pairs else np.zeros(0, np.uint8)
    refs = np.concatenate([p[1] for p in pairs])
    ql = np.array([len(p[0]) for p in pairs], np.int32)
    rl = np.array([len(p[1]) for p in pairs], np.int32)
    qo = np.concatenate([[0], np.cumsum(ql)[:-1]]).astype(np.int64)
    ro = np.concatenate([[0], np.cumsum(rl)[:-1]]).astype(np.int64)
    for E in (0, 2, 7, 40, 300):
        w = oracle.batch_uneq(reads, qo, ql, refs, ro, rl, E=E)
        acc, ed = ss.ss_filter_batch_pairs(reads, ql, refs, rl, E=E)
        check(f"edge cases E={E}", (acc, ed), (w["accept"], w["edits"]))
    # equal lengths through the unequal-length entry point give ss_filter_batch's results
    b = gen.make(0, n=3000)
    acc, ed = ss.ss_filter_batch_pairs(b["reads"], b["lengths"], b["refs"], b["lengths"], E=5)
    a2, e2 = ss.ss_filter_batch(b["reads"], b["refs"], b["lengths"], 5)
    assert np.array_equal(acc, a2) and np.array_equal(ed, e2)


def test_descriptor_errors(rt):
    """Forcing a kernel the batch does not fit, or a malformed descriptor, is refused before any work."""
    torch, ss, runner = rt
    b = gen.make(0, n=1000)
    D = Dev(rt, b, Epp=np.full(1000, 5, np.int32))
    ctx = runner.context()
    st = torch.cuda.current_stream()

    def rc(**kw):
        base = dict(reads=D.db.reads, refs=D.db.refs, n_pairs=D.n, E=5, flags=ss.SS_INPUT_ASCII, out=D.out,
                    err=D.err, offsets=D.db.offsets, lengths=D.db.lengths, read_bases=D.db.total,
                    ref_bases=D.db.total)
        base.update(kw)
        desc = ss.batch_desc(**base)
        return int(ss.lib().ss_filter_batch_ex(ctx, ss.ctypes.byref(desc), st.cuda_stream))

    D.out.fill_(-7)
    assert rc(flags=ss.SS_INPUT_ASCII | ss.SS_KERNEL_FUSED) == ss.SS_EINVAL            # offsets given
    assert rc(flags=ss.SS_INPUT_ASCII | ss.SS_KERNEL_FUSED, offsets=None, lengths=None, length=100,
              E_per_pair=D.E) == ss.SS_EINVAL                                          # per-pair thresholds
    assert rc(flags=ss.SS_INPUT_ASCII | ss.SS_KERNEL_SLICED, length=100, E=33) == ss.SS_ELEN
    assert rc(flags=ss.SS_INPUT_ASCII | ss.SS_KERNEL_PLAIN, E=32) == ss.SS_ELEN
    assert rc(flags=ss.SS_INPUT_ASCII | ss.SS_KERNEL_PERSISTENT, E_per_pair=D.E) == ss.SS_EINVAL   # no plan
    assert rc(flags=ss.SS_INPUT_PACKED | ss.SS_KERNEL_SLICED, length=100) == ss.SS_EINVAL         # bit streams
    assert rc(err=None) == ss.SS_EINVAL                                                # ASCII needs the error word
    assert rc(flags=0x60) == ss.SS_EINVAL and rc(flags=0x3) == ss.SS_EINVAL and rc(flags=0x100) == ss.SS_EINVAL
    assert rc(E=ss.SS_MAX_E + 1) == ss.SS_ELEN
    assert rc(offsets=None) == ss.SS_EINVAL                                            # several lengths need arrays
    # pairs back to back at i * length beyond the declared bases (bit-stream kernels)
    for kern in (ss.SS_KERNEL_PLAIN, ss.SS_KERNEL_WAVE):
        assert rc(flags=ss.SS_INPUT_ASCII | kern, offsets=None, lengths=None, length=100,
                  read_bases=100 * D.n - 1) == ss.SS_EINVAL
        assert rc(flags=ss.SS_INPUT_ASCII | kern, offsets=None, lengths=None, length=100,
                  ref_bases=100 * D.n - 1) == ss.SS_EINVAL
        assert rc(flags=ss.SS_INPUT_ASCII | kern, offsets=None, lengths=None, length=1 << 20,
                  n_pairs=1 << 62) == ss.SS_EINVAL                                     # the product overflows
    assert rc(n_pairs=0) == ss.SS_OK
    torch.cuda.synchronize()
    assert bool((D.out == -7).all())                                                   # nothing was written
    # a byte outside the alphabet is reported through the error word
    bad = dict(b)
    bad["reads"] = b["reads"].copy()
    bad["reads"][1234] = ord("N")
    Db = Dev.__new__(Dev)
    try:
        Dev.__init__(Db, rt, bad)
    except AssertionError:
        pass                                   # ss_pack already saw it
    Db.err.zero_()
    desc = ss.batch_desc(Db.db.reads, Db.db.refs, Db.n, 5, ss.SS_INPUT_ASCII | ss.SS_KERNEL_WAVE, Db.out, err=Db.err,
                         offsets=Db.db.offsets, lengths=Db.db.lengths, read_bases=Db.db.total, ref_bases=Db.db.total)
    ss.ss_filter_batch_ex(ctx, desc, st)
    torch.cuda.synchronize()
    assert int(Db.err.item()) & 1


def test_one_call_from_several_threads(rt):
    """The one-call host entry points share one context per device: calls from several host threads at once
    must each get their own results (they run one at a time)."""
    torch, ss, runner = rt
    batches = [gen.make(1, n=200_000 + 17 * k, seed=1000 + k) for k in range(4)]
    solo = [ss.ss_filter_batch(b["reads"], b["refs"], b["lengths"], 4) for b in batches]
    got = [None] * len(batches)
    errors = []

    def work(k):
        try:
            for _ in range(3):
                got[k] = ss.ss_filter_batch(batches[k]["reads"], batches[k]["refs"], batches[k]["lengths"], 4)
                a, e = got[k]
                if not (np.array_equal(a, solo[k][0]) and np.array_equal(e, solo[k][1])):
                    errors.append(k)
        except Exception as ex:          # reported below
            errors.append(repr(ex))

    th = [threading.Thread(target=work, args=(k,)) for k in range(len(batches))]
    for t in th:
        t.start()
    for t in th:
        t.join(timeout=300)
    assert not any(t.is_alive() for t in th)
    assert not errors, errors
    for k, b in enumerate(batches):
        check(f"batch {k}", solo[k], oracle_eq(b, 4))
