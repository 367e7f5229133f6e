"""Parity at the full workload sizes, in the launch configurations the benchmark times.

Every pair of every size is compared with the CPU oracle (run on the host cores, 16 threads), bit for
bit on the accept decision and the reported count:
  - 30 M pairs of 100 bp at E = 0, 3, 5 (the one-call path runs the fused kernel) and E = 6, 10 (the
    chunked two-kernel schedule), through the lane-sliced sweep on the resident planes and through the
    one-call path from ASCII; the one-pair-per-lane kernel at E = 5;
  - 10 M pairs of 250 bp at E = 0, 8, 25, lane-sliced sweep and one-call path; the wavefront kernel at
    E = 25 and the one-pair-per-lane kernel at E = 8;
  - the mixed batch (5 M short pairs + 20,000 pairs of 10 kbp, per-pair E) through an autotuned plan
    replayed from a captured graph.
"""
import os

import numpy as np
import pytest

import oracle
from paper_1910_09020_amd import gen

pytestmark = pytest.mark.gpu

THREADS = min(16, os.cpu_count() or 1)


@pytest.fixture(scope="module")
def rt():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1910_09020_amd as ss
    from paper_1910_09020_amd import runner
    ss.lib()
    return torch, runner


def say(msg):
    print(msg, flush=True)


def oracle_all(b, E=None, E_per_pair=None):
    w = oracle.batch(b["reads"], b["refs"], b["offsets"], b["lengths"], E=E, E_per_pair=E_per_pair,
                     threads=THREADS)
    return w["accept"], w["edits"]


def check(name, got, want):
    acc, ed = got
    wa, we = want
    bad = np.nonzero((acc != wa) | (ed != we))[0]
    assert len(bad) == 0, f"{name}: {len(bad)} of {len(wa)} pairs differ from the oracle, first {bad[:5]}"


def _every_pair(rt, b, Es, plain_E, wave_E=None):
    torch, runner = rt
    db = runner.DeviceBatch(b)
    pk = db.pack_sliced()
    out = db.new_out()
    for E in Es:
        say(f"  oracle n={db.n} m={db.uniform_m} E={E}")
        want = oracle_all(b, E)
        say(f"  sliced E={E}")
        db.filter_sliced(pk, E, out=out)
        torch.cuda.synchronize()
        check(f"sliced E={E}", runner.results_numpy(out, db.n), want)
        say(f"  one-call E={E}")
        db.filter_fused(E, out=out)
        torch.cuda.synchronize()
        db.check_err(f"one-call E={E}")
        check(f"one-call E={E}", runner.results_numpy(out, db.n), want)
        if E == plain_E or E == wave_E:
            ps = db.pack_stream()
            if E == plain_E:
                say(f"  one pair per lane E={E}")
                db.filter_plain(ps, E, out=out)
                torch.cuda.synchronize()
                check(f"plain E={E}", runner.results_numpy(out, db.n), want)
            if E == wave_E:
                say(f"  wavefront E={E}")
                db.filter_wave(ps, E, out=out)
                torch.cuda.synchronize()
                check(f"wave E={E}", runner.results_numpy(out, db.n), want)
            del ps
        del want
    db.check_err("encode")


def test_100bp_30M_every_pair(rt):
    _every_pair(rt, gen.make(1, threads=THREADS), [0, 3, 5, 6, 10], plain_E=5)


def test_250bp_10M_every_pair(rt):
    _every_pair(rt, gen.make(2, threads=THREADS), [0, 8, 25], plain_E=8, wave_E=25)


def test_mixed_5M_planned_every_pair(rt, tmp_path):
    """The mixed-length batch at full size in the benchmark's launch configuration: an autotuned plan
    replayed from a captured graph, every pair (short and long) against the oracle."""
    torch, runner = rt
    import paper_1910_09020_amd as ss
    b = gen.make(3, threads=THREADS)
    db = runner.DeviceBatch(b)
    ps = db.pack_stream()
    ctx = runner.context()
    out = db.new_out()
    say(f"  tuned plan n={db.n}")
    plan, _ = ss.ss_plan_create_tuned(ctx, b["lengths"], b["E"], ps, db.total, db.offsets, db.lengths, db.E, out,
                                      str(tmp_path / "tune.json"))
    ss.ss_plan_capture(ctx, plan, ps, db.total, db.offsets, db.lengths, db.E, out)
    out.fill_(-1)
    ss.ss_plan_launch(plan, torch.cuda.current_stream())
    torch.cuda.synchronize()
    got = runner.results_numpy(out, db.n)
    ss.ss_plan_destroy(plan)
    db.check_err("encode")
    say("  oracle on every pair")
    check("planned launch", got, oracle_all(b, E_per_pair=b["E"]))
