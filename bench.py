#!/usr/bin/env python3
"""Benchmark: filtered pairs/s on one MI355X for 100 bp pairs at E = 5.

One step is one threshold's pass of the filter over the 30 M pairs of 100 bp
(the 100 bp workload's sweep is one launch per E over data encoded once into
2-bit planes and resident in HBM): the lane-sliced column sweep builds the
Equation 1 rows of every pair and runs the greedy walk of Section 2.4,
writing each pair's accept bit and obstacle count (ss_filter_sliced_async at
E = 5).  The encoding (ASCII in HBM to 2-bit planes, run once per batch and
reused by every threshold) is timed on its own beside it, and so is the
one-call path that encodes and filters ASCII in one kernel.  Reported with
them: every pair's result against the CPU oracle (whose run on the host cores
is the cpu_baseline), the roofline of the step's kernel, the one-pair-per-lane
kernel on the same batch, the threshold sweeps, verification of the accepted
pairs, the mixed-length batch in one persistent launch and the serving loop.

Prints one JSON line.  Only one GPU is used; --gpus above 1 is refused.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, GB/s
VALU_PEAK_TOPS = 39.3          # 256 CU x 64 lanes x 2.4 GHz, 32-bit lane ops / s (1e12)


def measured_traffic(name, profile="fused_encode_sweep_100bp_E5_pmc.md"):
    """HBM bytes per launch of a kernel from a committed rocprofv3 PMC summary, or None when one of
    the kernel's source files has changed since the counters were taken (the summary line carries a
    hash of those files, concatenated in the order listed)."""
    import hashlib
    try:
        text = open(os.path.join(ROOT, "profiles", profile)).read()
    except OSError:
        return None
    for line in text.splitlines():
        f = line.split()
        if len(f) == 5 and f[0] == "traffic" and f[1] == name:
            kv = dict(x.split("=", 1) for x in f[2:])
            h = hashlib.sha256()
            try:
                for src in kv["source"].split(","):
                    h.update(open(os.path.join(ROOT, src), "rb").read())
            except OSError:
                return None
            return float(kv["bytes"]) if h.hexdigest()[:16] == kv["sha256_16"] else None
    return None


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def timed_loop(fns, steps, torch, means=None):
    """Run each callable in fns per step, bracketed by HIP events on the current stream (the stream
    every callable here launches on).  Returns (wall seconds for all steps, [median ms per
    callable over the steps]); means, if a list, receives the mean ms per callable."""
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(len(fns) + 1)] for _ in range(steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(steps):
        evs[s][0].record()
        for i, f in enumerate(fns):
            f()
            evs[s][i + 1].record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = [[evs[s][i].elapsed_time(evs[s][i + 1]) for s in range(steps)] for i in range(len(fns))]
    if means is not None:
        means[:] = [float(np.mean(x)) for x in ms]
    return wall, [float(np.median(x)) for x in ms]


def verify_leg(torch, runner, db, out, n, E, steps):
    """Filter then verify: exact edit distance (GPU) of every pair, the filter's false accept rate
    against it, and the pipeline filter -> compact accepted -> verify accepted, against verifying
    every pair (what the filter saves the aligner)."""
    ps = db.pack_stream()
    ed = db.verify(ps, max_len=db.uniform_m)
    torch.cuda.synchronize()
    _, (all_ms,) = timed_loop([lambda: db.verify(ps, max_len=db.uniform_m, out=ed)], steps, torch)
    res = out
    idx, cnt = db.select_accepted(res)
    torch.cuda.synchronize()
    k = int(cnt.item())
    ved = torch.empty(max(1, k), dtype=torch.int32, device="cuda")
    fused = lambda: db.filter_fused(E, out=res)
    sel = lambda: db.select_accepted(res, index_out=idx, count=cnt)
    ver = lambda: db.verify(ps, index=idx[:k], n=k, max_len=db.uniform_m, out=ved)
    _, (f_ms, s_ms, v_ms) = timed_loop([fused, sel, ver], steps, torch)
    acc = (res[:n].to(torch.int32) & 0x8000) != 0
    far_num = int((acc & (ed[:n] > E)).sum().item())
    far_den = int((ed[:n] > E).sum().item())
    missed = int(((~acc) & (ed[:n] <= E)).sum().item())
    pipe_ms = f_ms + s_ms + v_ms
    # Snake-on-Chip's decomposition at the paper's sub-maze width (8 columns): underestimates, so it
    # accepts more; same false-reject guarantee
    pk = db.pack_sliced()
    sub = db.filter_submaze(pk, E, 8)
    torch.cuda.synchronize()
    _, (sub_ms,) = timed_loop([lambda: db.filter_submaze(pk, E, 8, out=sub)], steps, torch)
    sacc = (sub[:n].to(torch.int32) & 0x8000) != 0
    sub_far = int((sacc & (ed[:n] > E)).sum().item())
    sub_missed = int(((~sacc) & (ed[:n] <= E)).sum().item())
    del pk
    log(f"verify: all {all_ms:.3f} ms; filter {f_ms:.3f} + select {s_ms:.3f} + verify {k} accepted {v_ms:.3f} ms; "
        f"FAR {far_num}/{far_den}; false rejects {missed}; sub-mazes of 8: FAR {sub_far}/{far_den}, "
        f"false rejects {sub_missed}, sweep {sub_ms:.3f} ms")
    r = dict(verify_all_ms=round(all_ms, 4), filter_ms=round(f_ms, 4), select_ms=round(s_ms, 4),
             verify_accepted_ms=round(v_ms, 4), accepted=k, pipeline_ms=round(pipe_ms, 4),
             speedup_vs_verify_all=all_ms / pipe_ms,
             false_accept_rate=far_num / far_den if far_den else None, false_accepts=far_num,
             pairs_over_E=far_den, false_rejects=missed,
             submaze_t8=dict(sweep_ms=round(sub_ms, 4), accepted=int(sacc.sum().item()),
                             false_accept_rate=sub_far / far_den if far_den else None, false_rejects=sub_missed))
    del ps, ed, ved, idx, cnt
    return r


def sweep_leg(torch, ss, gen, runner, config, Es, steps, batch=None, plain_and_wave=False):
    """Threshold sweep on one resident batch: the two-kernel path encodes once and sweeps each E;
    the one-call path (fused up to E = 10, chunked above) runs per E; and the range call sweeps every E
    with thresholds sharing passes over the planes (outputs checked equal).  plain_and_wave: also the
    one-pair-per-lane kernel and the wavefront-cooperative kernel on the bit-stream encoding, per E,
    with outputs checked equal to the sweep's.  Mean ms per launch."""
    b = batch if batch is not None else gen.make(config, threads=min(16, os.cpu_count() or 1))
    db = runner.DeviceBatch(b)
    n, m = db.n, db.uniform_m
    packed = torch.empty(max(4, ss.ss_sliced_bytes(n, m) // 4), dtype=torch.int32, device="cuda")
    out = torch.empty(n, dtype=torch.int16, device="cuda")
    out1 = torch.empty(n, dtype=torch.int16, device="cuda")
    db.pack_sliced(packed=packed)
    torch.cuda.synchronize()
    _, (enc_ms,) = timed_loop([lambda: db.pack_sliced(packed=packed)], steps, torch)
    ps = db.pack_stream() if plain_and_wave else None
    rng = db.filter_sliced_range(packed, Es[0], Es[-1])
    torch.cuda.synchronize()
    per_E = {}
    same = True
    same_pw = True
    same_rng = True
    for E in Es:
        db.filter_sliced(packed, E, out=out)
        db.filter_fused(E, out=out1)
        torch.cuda.synchronize()
        same = same and bool(torch.equal(out, out1))
        same_rng = same_rng and bool(torch.equal(out, rng[E - Es[0], :n]))
        _, (sw_ms, one_ms) = timed_loop([lambda: db.filter_sliced(packed, E, out=out),
                                         lambda: db.filter_fused(E, out=out1)], steps, torch)
        per_E[E] = dict(sweep_ms=round(sw_ms, 4), one_call_ms=round(one_ms, 4))
        if plain_and_wave:
            db.filter_plain(ps, E, out=out1)
            torch.cuda.synchronize()
            same_pw = same_pw and bool(torch.equal(out, out1))
            db.filter_wave(ps, E, out=out1)
            torch.cuda.synchronize()
            same_pw = same_pw and bool(torch.equal(out, out1))
            _, (pl_ms, wv_ms) = timed_loop([lambda: db.filter_plain(ps, E, out=out1),
                                            lambda: db.filter_wave(ps, E, out=out1)], steps, torch)
            per_E[E].update(plain_ms=round(pl_ms, 4), wave_ms=round(wv_ms, 4))
    _, (rng_ms,) = timed_loop([lambda: db.filter_sliced_range(packed, Es[0], Es[-1], out=rng)], steps, torch)
    db.check_err(f"sweep config {config}")
    total_sweep = enc_ms + sum(v["sweep_ms"] for v in per_E.values())
    log(f"sweep config {config} ({n} x {m} bp): encode {enc_ms:.3f} ms, E={Es[0]}..{Es[-1]} "
        f"sweeps {sum(v['sweep_ms'] for v in per_E.values()):.3f} ms, identical={same}; "
        f"range call {rng_ms:.3f} ms, identical={same_rng}")
    res = dict(n_pairs=n, m=m, encode_ms=round(enc_ms, 4), per_E=per_E,
               whole_sweep_ms=round(total_sweep, 4),
               whole_sweep_pair_thresholds_per_s=n * len(Es) / (1e-3 * total_sweep),
               one_call_equals_two_kernel=same,
               range_call=dict(entry="ss_filter_sliced_range_async", ms=round(rng_ms, 4),
                               identical_to_per_E=same_rng,
                               whole_sweep_ms=round(enc_ms + rng_ms, 4),
                               pair_thresholds_per_s=n * len(Es) / (1e-3 * (enc_ms + rng_ms))))
    if plain_and_wave:
        pl = sum(v["plain_ms"] for v in per_E.values())
        wv = sum(v["wave_ms"] for v in per_E.values())
        res.update(plain_all_E_ms=round(pl, 4), wave_all_E_ms=round(wv, 4), plain_and_wave_identical=same_pw)
        log(f"sweep config {config}: one pair per lane {pl:.3f} ms, wavefront-cooperative {wv:.3f} ms over "
            f"E={Es[0]}..{Es[-1]} on the bit stream, identical={same_pw}")
    del db, packed, out, out1, ps, rng
    torch.cuda.empty_cache()
    return res


def long_leg(torch, ss, gen, runner, oracle, n=2000, m=100_000, E=5000, steps=3):
    """Pairs of 100 kbp at E = 5000 (5% of the length; 2E+1 = 10,001 rows per column), edit rates
    3-7%: one standalone wavefront launch and one planned persistent launch (8 slices per lane),
    with a sample checked against the oracle."""
    b = gen.long_pairs(n, m, 300, 700)
    db = runner.DeviceBatch(b)
    ps = db.pack_stream()
    out = db.new_out()
    db.filter_wave(ps, E, out=out)
    torch.cuda.synchronize()
    _, (wave_ms,) = timed_loop([lambda: db.filter_wave(ps, E, out=out)], steps, torch)
    db.check_err("100 kbp encode")
    Es = np.full(n, E, dtype=np.int32)
    dE = torch.from_numpy(Es).to("cuda")
    plan = ss.ss_plan_create(runner.context(), b["lengths"], Es, 8)
    pout = db.new_out()
    run = lambda: ss.ss_filter_planned_async(runner.context(), plan, ps, db.total, db.offsets, db.lengths, dE,
                                             pout, torch.cuda.current_stream())
    run()
    torch.cuda.synchronize()
    _, (plan_ms,) = timed_loop([run], steps, torch)
    acc, ed = runner.results_numpy(out, n)
    pacc, ped = runner.results_numpy(pout, n)
    k = 16
    w = oracle.batch(b["reads"], b["refs"], b["offsets"][:k], b["lengths"][:k], E=E,
                     threads=min(16, os.cpu_count() or 1))
    mism = int(np.sum((w["accept"] != acc[:k]) | (w["edits"] != ed[:k])))
    same = bool(np.array_equal(acc, pacc) and np.array_equal(ed, ped))
    ss.ss_plan_destroy(plan)
    # banded verification of every pair (distance when within E, else E + 1): false accept rate, no false reject
    vout = torch.empty(n, dtype=torch.int32, device="cuda")
    vb = lambda: db.verify_banded(ps, E, out=vout)
    vb(); torch.cuda.synchronize()
    _, (vb_ms,) = timed_loop([vb], 1, torch)
    vd = vout.cpu().numpy()
    over = vd > E
    verify = dict(banded_verify_ms=round(vb_ms, 3), pairs_over_E=int(over.sum()),
                  false_accepts=int((acc.astype(bool) & over).sum()),
                  false_accept_rate=float((acc.astype(bool) & over).sum() / max(1, over.sum())),
                  false_rejects=int((~acc.astype(bool) & ~over).sum()))
    log(f"100 kbp: {n} pairs at E={E}: wave {wave_ms:.2f} ms, planned {plan_ms:.2f} ms, identical={same}, "
        f"accepted {int(acc.sum())}, oracle mismatches {mism}/{k}; banded verify {verify}")
    res = dict(workload=f"{n} pairs of {m} bp, edit rate U[3%,7%], E={E}", n_pairs=n, m=m, E=E,
               wave_ms=round(wave_ms, 3), planned_ms=round(plan_ms, 3),
               pairs_per_s=n / (1e-3 * min(wave_ms, plan_ms)),
               cells_per_s=n * m * (2 * E + 1) / (1e-3 * min(wave_ms, plan_ms)),
               accepted=int(acc.sum()), identical_outputs=same, oracle_sample_pairs=k, oracle_sample_mismatches=mism,
               verify=verify)
    del db, ps, out, pout, vout
    torch.cuda.empty_cache()
    return res


def latency_leg(torch, ss, gen, runner, E=5, reps=200):
    """Single-call latency on the small 10,000-pair batch: eager calls, and the same call
    captured once in a HIP graph and replayed (each replay checked against the eager result)."""
    b = gen.make(0)
    db = runner.DeviceBatch(b)
    out = torch.empty(db.n, dtype=torch.int16, device="cuda")
    db.filter_fused(E, out=out)
    torch.cuda.synchronize()
    db.check_err("latency leg")
    ref = out.clone()
    t0 = time.perf_counter()
    for _ in range(reps):
        db.filter_fused(E, out=out)
    torch.cuda.synchronize()
    eager_us = 1e6 * (time.perf_counter() - t0) / reps
    _, (eager_dev_ms,) = timed_loop([lambda: db.filter_fused(E, out=out)], reps, torch)
    g = torch.cuda.CUDAGraph()
    gout = torch.empty_like(out)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        db.filter_fused(E, out=gout, stream=s)          # warm-up on the capture stream
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    with torch.cuda.graph(g, stream=s):
        db.filter_fused(E, out=gout, stream=s)
    ok = True
    for _ in range(3):
        gout.zero_()
        g.replay()
        torch.cuda.synchronize()
        ok = ok and bool(torch.equal(gout, ref))
        db.filter_fused(E, out=out)                       # eager work between replays
        torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        g.replay()
    torch.cuda.synchronize()
    graph_us = 1e6 * (time.perf_counter() - t0) / reps
    db.check_err("latency leg")
    log(f"latency (10,000 pairs, E={E}): eager {eager_us:.1f} us/call, graph {graph_us:.1f} us/replay, "
        f"replays identical={ok}")
    res = dict(n_pairs=db.n, E=E, eager_us_per_call=eager_us, eager_kernel_us=1e3 * eager_dev_ms,
               graph_us_per_replay=graph_us, graph_replays_identical=ok)
    del g, db
    return res


def mixed_leg(a, torch, ss, gen, runner, oracle):
    """Mixed-length batch (5 M short pairs of 100/150/250 bp + 20,000 pairs of 10 kbp, per-pair E):
    one persistent launch from an autotuned plan, replayed from a captured HIP graph, against one
    unbucketed launch of the wavefront kernel over the batch in input order (every pair laid out for
    the largest threshold).  Both run on the same bit-stream encoding resident in HBM."""
    t = time.perf_counter()
    b = gen.make(3, n=a.mixed_n, threads=min(16, os.cpu_count() or 1))
    n = b["n"]
    log(f"mixed: generated {n} pairs ({int((b['lengths'] >= 10000).sum())} long) in {time.perf_counter() - t:.1f}s")
    db = runner.DeviceBatch(b)
    ps = db.pack_stream()
    torch.cuda.synchronize()
    enc = lambda: db.pack_stream(packed=ps)
    _, (enc_ms,) = timed_loop([enc], 3, torch)
    ctx = runner.context()
    out = db.new_out()
    cache = os.environ.get("SS_TUNE_CACHE", "/tmp/ss_tune_cache.json")
    t = time.perf_counter()
    plan, chosen = ss.ss_plan_create_tuned(ctx, b["lengths"], b["E"], ps, db.total, db.offsets, db.lengths, db.E,
                                           out, cache)
    plan_s = time.perf_counter() - t
    info = ss.ss_plan_info(plan)
    ss.ss_plan_capture(ctx, plan, ps, db.total, db.offsets, db.lengths, db.E, out)
    stream = torch.cuda.current_stream()
    run = lambda: ss.ss_plan_launch(plan, stream)
    for _ in range(max(1, a.warmup)):
        run()
    torch.cuda.synchronize()
    _, (bat_ms,) = timed_loop([run], max(10, a.steps // 2), torch)
    db.check_err("mixed encode")
    acc, ed = runner.results_numpy(out, n)
    emax = int(b["E"].max())
    uout = db.new_out()
    flat = lambda: db.filter_wave(ps, emax, per_pair=True, out=uout)
    flat(); torch.cuda.synchronize()
    _, (flat_ms,) = timed_loop([flat], 2, torch)
    uacc, ued = runner.results_numpy(uout, n)
    identical = bool(np.array_equal(acc, uacc) and np.array_equal(ed, ued))
    # sampled oracle check: short pairs and long pairs separately
    rng = np.random.default_rng(11)
    long_idx = np.nonzero(b["lengths"] >= 10000)[0]
    short_idx = np.nonzero(b["lengths"] < 10000)[0]
    idx = np.sort(np.concatenate([rng.choice(short_idx, size=min(50000, len(short_idx)), replace=False),
                                  rng.choice(long_idx, size=min(400, len(long_idx)), replace=False)]))
    w = oracle.batch(b["reads"], b["refs"], b["offsets"][idx], b["lengths"][idx], E_per_pair=b["E"][idx],
                     threads=min(16, os.cpu_count() or 1), want_stats=True)
    mism = int(np.sum((w["accept"] != acc[idx]) | (w["edits"] != ed[idx])))
    ss.ss_plan_destroy(plan)
    # verification of every pair on the GPU (short pairs one per lane, long ones one per wavefront): the
    # false accept rate over the whole batch, long pairs included, and no false reject
    ver = {}
    ed_all = np.zeros(n, dtype=np.int64)
    for name, cls_idx, ml in (("short", short_idx, int(b["lengths"][short_idx].max())),
                              ("long", long_idx, int(b["lengths"][long_idx].max()) if len(long_idx) else 0)):
        if not len(cls_idx):
            continue
        ix = torch.from_numpy(cls_idx.astype(np.int64)).cuda()
        vout = torch.empty(len(cls_idx), dtype=torch.int32, device="cuda")
        fn = lambda: db.verify(ps, index=ix, n=len(cls_idx), max_len=ml, out=vout)
        fn(); torch.cuda.synchronize()
        _, (v_ms,) = timed_loop([fn], 2, torch)
        ed_all[cls_idx] = vout.cpu().numpy()
        ver[f"{name}_verify_ms"] = round(v_ms, 4)
        ver[f"{name}_pairs"] = int(len(cls_idx))
    over = ed_all > b["E"]
    fa = acc.astype(bool) & over
    ver.update(pairs_over_E=int(over.sum()), false_accepts=int(fa.sum()),
               false_accept_rate=float(fa.sum() / max(1, over.sum())),
               false_accept_rate_long=float(fa[long_idx].sum() / max(1, over[long_idx].sum())) if len(long_idx) else None,
               false_rejects=int((~acc.astype(bool) & ~over).sum()),
               verified_sample_vs_oracle_levenshtein=None)
    # the GPU distances against the oracle's Levenshtein on a few pairs of each class
    chk = np.concatenate([short_idx[:2000], long_idx[:8]])
    lev = oracle.levenshtein_batch(b["reads"], b["refs"], b["offsets"][chk], b["lengths"][chk])
    ver["verified_sample_vs_oracle_levenshtein"] = {"pairs": int(len(chk)),
                                                    "mismatches": int(np.sum(lev != ed_all[chk]))}
    del vout
    log(f"mixed verify: {ver}")
    # the oracle's rate on this batch, per class (short, long) on the same samples, timed apart:
    # the whole batch would take n_short / short rate + n_long / long rate on these threads
    threads = min(16, os.cpu_count() or 1)
    rates = {}
    for name, cls_idx in (("short", idx[b["lengths"][idx] < 10000]), ("long", idx[b["lengths"][idx] >= 10000])):
        t0 = time.perf_counter()
        oracle.batch(b["reads"], b["refs"], b["offsets"][cls_idx], b["lengths"][cls_idx], E_per_pair=b["E"][cls_idx],
                     threads=threads)
        rates[name] = len(cls_idx) / max(time.perf_counter() - t0, 1e-9)
    oracle_batch_s = len(short_idx) / rates["short"] + len(long_idx) / rates["long"]
    # roofline by the op model of a row-wise bit-parallel walk: (2E+1) (5 ceil(c_last/32) + 3 K) 32-bit ops
    # per pair, c_last and the checkpoints K from the oracle's stats on the sample, scaled to the batch
    # by class (short / long)
    Es = b["E"][idx].astype(np.float64)
    ops = (2 * Es + 1) * (5 * np.ceil(w["stats"][:, 1] / 32.0) + 3 * w["stats"][:, 0])
    is_long = b["lengths"][idx] >= 10000
    model_ops = float(ops[~is_long].mean() * len(short_idx) + (ops[is_long].mean() * len(long_idx) if len(long_idx) else 0))
    achieved_tops = model_ops / (bat_ms * 1e-3) / 1e12
    res = dict(workload="5M short (100/150/250 bp) + 20k x 10 kbp, per-pair E = ceil(rate x m), rate in "
                        "{1,2,5,10}%", n_pairs=n, encode_ms=round(enc_ms, 4), batched_ms=round(bat_ms, 4),
               batched_pairs_per_s=n / (1e-3 * bat_ms), step_pairs_per_s=n / (1e-3 * (bat_ms + enc_ms)),
               unbucketed_ms=round(flat_ms, 4), unbucketed_pairs_per_s=n / (1e-3 * flat_ms),
               speedup_vs_unbucketed=flat_ms / bat_ms, identical_outputs=identical, plan_seconds=round(plan_s, 3),
               plan=info, tuned_slices_per_lane=chosen, oracle_sample_pairs=int(len(idx)),
               oracle_sample_mismatches=mism, verify=ver,
               cpu_oracle={"threads": threads, "short_pairs_per_s": rates["short"], "long_pairs_per_s": rates["long"],
                           "whole_batch_s": oracle_batch_s, "gpu_speedup": oracle_batch_s / (1e-3 * bat_ms),
                           "sample": f"{int((b['lengths'][idx] < 10000).sum())} short and "
                                     f"{int((b['lengths'][idx] >= 10000).sum())} long pairs of the batch, timed "
                                     "apart; whole batch = n_short / short rate + n_long / long rate"},
               roofline={"bound": "alu", "model": "(2E+1)(5 ceil(c_last/32) + 3 checkpoints) 32-bit ops per pair "
                                                   "(oracle stats on the sample, scaled to the batch by class)",
                         "model_ops": model_ops, "achieved": achieved_tops, "peak": VALU_PEAK_TOPS,
                         "unit": "T ops/s", "frac": achieved_tops / VALU_PEAK_TOPS})
    log(f"mixed: batched {bat_ms:.3f} ms, unbucketed {flat_ms:.3f} ms, identical={identical}, "
        f"oracle mismatches {mism}/{len(idx)}, plan {plan_s:.2f}s {info}; op model {model_ops / 1e9:.1f} G ops "
        f"-> {achieved_tops:.1f} T ops/s ({100 * achieved_tops / VALU_PEAK_TOPS:.0f}% of {VALU_PEAK_TOPS} T); oracle on "
        f"{threads} threads: {rates['short'] / 1e6:.2f} M short + {rates['long']:.0f} long pairs/s -> whole batch "
        f"{oracle_batch_s:.2f} s ({oracle_batch_s / (1e-3 * bat_ms):.0f}x the launch)")
    del db, ps, out, uout
    torch.cuda.empty_cache()
    return res


def serving_leg(a, ss, gen, runner, oracle, mode=None, seconds=None):
    """Continuous batching: Poisson arrivals, requests of 1..4096 pairs of 100..10,000 bp (log-uniform)
    with one threshold rate per request, generated by native worker threads just ahead of their arrival
    and submitted at their scheduled times to one server; latency = completion - scheduled arrival."""
    import ctypes
    seed = 1910090204
    mode = mode or a.serve_mode
    seconds = seconds or a.serve_seconds
    arr = gen.arrivals(seed, a.serve_rate, seconds)
    nreq = len(arr)
    ctx = runner.context()
    if mode == "loop":
        # device-resident loop: one persistent kernel, requests handed over through host memory
        budget = 4 << 30
        srv = ss.ss_server_create_loop(ctx, budget, a.serve_loop_slots, a.serve_slices)
    else:
        budget = 32 << 30
        srv = ss.ss_server_create(ctx, budget, a.serve_slots)
        ss.ss_server_set_slices(srv, a.serve_slices)
    submit_ptr = ctypes.cast(ss.lib().ss_server_submit, ctypes.c_void_p).value
    pool = min(nreq, a.serve_pool)
    # on the fly, requests are generated into blocks of the server's pinned staging and submitted without
    # a copy (ss_server_submit_staged), unless --serve-copy asks for the copying submission
    staged = None
    if pool == 0 and not getattr(a, "serve_copy", False):
        L = ss.lib()
        staged = tuple(ctypes.cast(f, ctypes.c_void_p).value
                       for f in (L.ss_server_stage_alloc, L.ss_server_stage_free, L.ss_server_submit_staged))
    # on the fly: generator threads run up to 2,048 requests ahead of the clock (a head start of as many
    # before it starts), and 8 submitter threads hand each request over at its due time
    # (12 generator threads leave the server's threads cores of their own on a 16-core host share)
    D = gen.drive(seed, arr, submit_ptr, srv, threads=12 if pool == 0 else min(16, max(4, os.cpu_count() or 1)),
                  pool=pool, staged=staged)
    assert D.submitted == nreq, f"submission failed: {D.submitted}"
    for t in D.tickets:
        rc = ss.ss_server_wait(srv, int(t), -1)
        assert rc == ss.SS_OK, rc
    lat, svc, wait, lag, dlag, stages = [], [], [], [], [], []
    done_last = 0
    for i in range(nreq):
        sub, adm, done = ss.ss_server_times(srv, int(D.tickets[i]))
        due = int(D.due_ns[i])
        lat.append((done - due) / 1e6)
        svc.append((done - adm) / 1e6)
        wait.append((adm - sub) / 1e6)
        lag.append((sub - due) / 1e6)
        dlag.append((int(D.call_ns[i]) - due) / 1e6)
        stages.append(ss.ss_server_stages(srv, int(D.tickets[i])))
        done_last = max(done_last, done)
    lat = np.array(lat)
    # where the time of a request goes: the driver's lag behind the schedule (due time to its submit
    # call), the submission itself (planning and staging inside ss_server_submit), queue, host enqueue,
    # device spans (copy in, encode + filter, copy out), and the rest of the service time (waiting on
    # the device behind other slots' work, and the completion thread's polling); means over all
    # requests and over those at or above the p99 latency
    st = np.array(stages, dtype=np.float64) / 1e6
    parts = np.stack([np.array(dlag), np.array(lag) - np.array(dlag), np.array(wait), st[:, 0], st[:, 1], st[:, 2],
                      st[:, 3], np.array(svc) - st.sum(axis=1)], axis=1)
    names = ["driver_lag", "submit", "queue", "host_enqueue", "copy_in", "encode_filter", "copy_out",
             "device_wait_and_poll"]
    tail = lat >= np.percentile(lat, 99)
    breakdown = {"all_mean_ms": dict(zip(names, [round(float(x), 4) for x in parts.mean(axis=0)])),
                 "p99_tail_mean_ms": dict(zip(names, [round(float(x), 4) for x in parts[tail].mean(axis=0)])),
                 "p99_tail_requests": int(tail.sum()),
                 "p99_tail_mean_pairs": float(np.mean(D.pairs[tail])),
                 "all_mean_pairs": float(np.mean(D.pairs))}
    pct = lambda v, q: float(np.percentile(np.array(v), q))
    pairs = int(D.pairs.sum())
    bases = int(D.bases.sum())
    st = ss.ss_server_stats(srv)
    t0 = int(D.due_ns[0]) - int(arr[0] * 1e9)
    span = (done_last - t0) / 1e9
    # exactness: a sample of requests against the oracle
    rng = np.random.default_rng(5)
    chk = rng.choice(nreq, size=min(40, nreq), replace=False)
    mism = 0
    for i in chk:
        r = gen.request(seed, int(i) % pool if pool else int(i))
        acc, ed = D.outputs(int(i))
        w = oracle.batch(r["reads"], r["refs"], r["offsets"], r["lengths"], E_per_pair=r["E"],
                         threads=min(16, os.cpu_count() or 1))
        mism += int(np.sum((w["accept"] != acc) | (w["edits"] != ed)))
    D.free()
    ss.ss_server_destroy(srv)
    res = dict(mode=("device-resident loop (one persistent kernel)" if mode == "loop" else
                     "host dispatcher (kernels and copies on slot streams)"),
               arrival_rate=a.serve_rate, seconds=seconds, requests=nreq, pairs=pairs, bases=bases,
               pairs_per_s=pairs / span, p50_ms=float(np.percentile(lat, 50)), p99_ms=float(np.percentile(lat, 99)),
               max_ms=float(lat.max()), service_p50_ms=pct(svc, 50), service_p99_ms=pct(svc, 99),
               queue_p50_ms=pct(wait, 50), queue_p99_ms=pct(wait, 99), submit_lag_p50_ms=pct(lag, 50),
               submit_lag_p99_ms=pct(lag, 99), driver_lag_p50_ms=pct(dlag, 50), driver_lag_p99_ms=pct(dlag, 99),
               slots=a.serve_loop_slots if mode == "loop" else a.serve_slots,
               hbm_budget_bytes=budget, stats=st,
               hw_queues=os.environ.get("GPU_MAX_HW_QUEUES", "HIP default"), distinct_requests=pool or nreq,
               breakdown=breakdown,
               generation=(f"every request generated from its own seed, up to {512 if staged else 2048} ahead of "
                           "the clock" if not pool else f"{pool} requests generated before the clock, replayed in a cycle"),
               submission=("staged: generated into blocks of the server's pinned staging, submitted without a copy "
                           "(ss_server_submit_staged)" if staged else "copied into staging (ss_server_submit)"),
               slices_per_lane=a.serve_slices,
               oracle_checked_requests=int(len(chk)), oracle_mismatches=mism)
    log(f"serving ({mode}): {nreq} requests, {pairs} pairs in {span:.2f}s, p50 {res['p50_ms']:.3f} ms, "
        f"p99 {res['p99_ms']:.3f} ms, service p50/p99 {res['service_p50_ms']:.3f}/{res['service_p99_ms']:.3f} ms, "
        f"tail breakdown {breakdown['p99_tail_mean_ms']}, "
        f"queue p50/p99 {res['queue_p50_ms']:.3f}/{res['queue_p99_ms']:.3f} ms, submit lag p50/p99 "
        f"{res['submit_lag_p50_ms']:.3f}/{res['submit_lag_p99_ms']:.3f} ms (of which the driver's "
        f"{res['driver_lag_p50_ms']:.3f}/{res['driver_lag_p99_ms']:.3f} ms), stats {st}, oracle mismatches {mism}")
    return res


def sclk_leg(step, seconds=1.5):
    """Shader clock while the step's kernel runs back to back: rocm-smi is sampled from a thread
    during ~seconds of launches.  Returns dict(mhz=[...], samples) or None when no tool answers."""
    import re
    import subprocess
    import threading
    import torch
    samples = []
    stop = threading.Event()

    def poll():
        while not stop.is_set():
            try:
                r = subprocess.run(["rocm-smi", "--showclocks", "--json"], capture_output=True, text=True,
                                   timeout=10)
                d = json.loads(r.stdout[r.stdout.index("{"):]) if "{" in r.stdout else {}
                for card, kv in d.items():
                    for k, v in kv.items():
                        if "sclk" in k.lower():
                            mm = re.search(r"(\d+)\s*[Mm][Hh]z", str(v))
                            if mm:
                                samples.append(int(mm.group(1)))
            except Exception:
                return
    th = threading.Thread(target=poll, daemon=True)
    th.start()
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < seconds:
        for _ in range(64):
            step()
        torch.cuda.synchronize()
    stop.set()
    th.join(timeout=15)
    if not samples:
        return None
    return dict(mhz=samples, median_mhz=float(np.median(samples)), tool="rocm-smi --showclocks",
                note="sampled while the step's kernel ran back to back")


# the paper's own end-to-end speedups (filter + aligner over the aligner alone), quoted as context: they
# are ratios on other hardware, not figures this benchmark measures
PAPER_CONTEXT = [
    {"what": "Snake-on-GPU + Edlib over Edlib alone", "value": "up to 413x", "workload": "100bp_2, E=5%",
     "hardware": "NVIDIA RTX 2080Ti (filter), aligner on the host CPU", "where": "Section 3.4"},
    {"what": "Snake-on-GPU + Parasail over Parasail alone", "value": "up to 689x", "workload": "100bp_2, E=5%",
     "hardware": "NVIDIA RTX 2080Ti (filter), aligner on the host CPU", "where": "Section 3.4"},
    {"what": "CPU SneakySnake + Edlib / + Parasail", "value": "up to 37.7x / 43.9x", "workload": "250bp_2",
     "hardware": "one core of an Intel E3-1225 (3.3 GHz)", "where": "Section 3.3"},
    {"what": "SneakySnake + Parasail, long reads", "value": "up to 979x", "workload": "100Kbp, E up to 5%",
     "hardware": "Intel Xeon Gold 5118, 40 threads", "where": "Section 3.5, Table 1"},
]


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--E", type=int, default=5)
    ap.add_argument("--n", type=int, default=None, help="pairs (default: 30 M, the 100 bp workload)")
    ap.add_argument("--cpu-pairs", type=int, default=None, help="oracle baseline sample (default: all pairs)")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--mixed-n", type=int, default=None, help="pairs of the mixed-length batch (default 5.02 M)")
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--serve-seconds", type=float, default=60.0, help="serving schedule length (60 s in full)")
    ap.add_argument("--serve-rate", type=float, default=2000.0, help="Poisson arrival rate, requests/s")
    ap.add_argument("--serve-slots", type=int, default=8, help="slot streams of the host-dispatch server")
    ap.add_argument("--serve-loop-slots", type=int, default=64, help="request slots of the device-resident loop")
    ap.add_argument("--serve-mode", choices=["loop", "host"], default="loop",
                    help="serving leg: device-resident loop (default) or host dispatcher")
    ap.add_argument("--serve-slices", type=int, default=1, help="32-row slices per lane for served requests")
    ap.add_argument("--serve-pool", type=int, default=0,
                    help="0 (default): every request generated from its own seed, ahead of its arrival; N > 0: "
                         "N distinct requests generated before the clock starts and replayed in a cycle")
    ap.add_argument("--serve-copy", action="store_true",
                    help="submit requests with ss_server_submit (bases copied into staging) instead of generating "
                         "them into the server's staging")
    ap.add_argument("--serve-only", action="store_true", help="run only the serving leg (diagnostics)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-sclk", action="store_true")
    ap.add_argument("--no-sweep", action="store_true", help="skip the threshold sweeps and the latency leg")
    a = ap.parse_args()
    if a.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {a.gpus} is not supported (pairs shard independently "
              "across GPUs with no collective on the path).", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_1910_09020_amd as ss
    from paper_1910_09020_amd import gen, runner

    ss.lib()
    torch.cuda.set_device(0)
    if a.serve_only:
        import oracle
        print(json.dumps(serving_leg(a, ss, gen, runner, oracle)), flush=True)
        return
    E = a.E
    n = a.n or gen.default_pairs(1)
    t = time.perf_counter()
    b = gen.make(1, n=n, threads=min(16, os.cpu_count() or 1))
    log(f"generated {n} pairs in {time.perf_counter() - t:.1f}s")
    m = 100
    db = runner.DeviceBatch(b)
    torch.cuda.synchronize()

    # row a1: the batch's 2-bit planes (lane-sliced layout), encoded once from the ASCII in HBM and
    # reused by every threshold of the sweep; timed on its own
    packed = torch.empty(max(4, ss.ss_sliced_bytes(n, m) // 4), dtype=torch.int32, device="cuda")
    pack = lambda: db.pack_sliced(packed=packed)
    pack()
    torch.cuda.synchronize()
    db.check_err("encode")
    _, (pack_ms,) = timed_loop([pack], max(10, a.steps), torch)
    db.check_err("encode")

    # the step: one threshold's filter launch over the resident planes (rows a2-a5)
    out = torch.empty(n, dtype=torch.int16, device="cuda")
    step = lambda: db.filter_sliced(packed, E, out=out)
    for _ in range(a.warmup):
        step()
    torch.cuda.synchronize()
    step_mean = [0.0]
    wall, (step_ms,) = timed_loop([step], a.steps, torch, means=step_mean)
    ms_per_step = 1e3 * wall / a.steps
    value = n / (ms_per_step / 1e3)
    if a.steps < 10:
        # the kernel's median (and mean) over at least 10 launches
        _, (step_ms,) = timed_loop([step], 10, torch, means=step_mean)
    step_mean_ms = step_mean[0]
    acc, ed = runner.results_numpy(out, n)
    log(f"step {ms_per_step:.4f} ms (sweep E={E} on resident planes; kernel median {step_ms:.4f} ms, "
        f"mean {step_mean_ms:.4f} ms) "
        f"{value / 1e9:.2f} G pairs/s; encode {pack_ms:.4f} ms")

    # the one-call path from ASCII in HBM (encode + filter in one kernel up to E = 10)
    out1 = torch.empty(n, dtype=torch.int16, device="cuda")
    one = lambda: db.filter_fused(E, out=out1)
    one()
    torch.cuda.synchronize()
    db.check_err("one-call")
    _, (one_ms,) = timed_loop([one], max(10, a.steps), torch)
    db.check_err("one-call")
    one_call = dict(entry="ss_filter_ascii_async", kernel=("fused encode + sweep (k_fused<%d, true>)" % E
                                                             if E <= 10 else "encode + sweep in chunks"),
                    ms=round(one_ms, 4), pairs_per_s=n / (1e-3 * one_ms),
                    identical_outputs=bool(torch.equal(out[:n], out1[:n])),
                    ascii_bytes_read=n * 2 * m,
                    roofline={"bound": "hbm", "achieved": n * (2 * m + 2) / (one_ms * 1e-3) / 1e9,
                              "peak": HBM_PEAK_GBS, "unit": "GB/s",
                              "frac": n * (2 * m + 2) / (one_ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
                              "algorithmic_bytes": n * (2 * m + 2),
                              "bytes_rule": "ASCII in (2m) + result (2 B) per pair: what this entry point must read",
                              "frac_at_packed_bytes": n * (m // 2 + 2) / (one_ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
                              "traffic": measured_traffic("k_fused_E%d" % E) if (n == 30_000_000 and E == 5) else None})
    log(f"one call (ASCII in): {one_ms:.4f} ms, identical={one_call['identical_outputs']}")
    del out1

    plain = None
    if not a.no_plain:
        ps = db.pack_stream()
        pout = torch.empty(n, dtype=torch.int16, device="cuda")
        pstream = lambda: db.pack_stream(packed=ps)
        pfilt = lambda: db.filter_plain(ps, E, out=pout)
        pfilt(); torch.cuda.synchronize()
        _, (ps_ms, pf_ms) = timed_loop([pstream, pfilt], 10, torch)
        db.check_err("bit-stream encode")
        pacc, ped = runner.results_numpy(pout, n)
        plain = dict(kernel="one pair per lane (k_plain)", encode_ms=round(ps_ms, 4), filter_ms=round(pf_ms, 4),
                     filter_pairs_per_s=n / (1e-3 * pf_ms),
                     identical_outputs=bool(np.array_equal(pacc, acc) and np.array_equal(ped, ed)),
                     step_over_plain=pf_ms / step_ms)
        log(f"plain: encode {ps_ms:.3f} ms filter {pf_ms:.3f} ms identical={plain['identical_outputs']}")
        del ps, pout

    sclk = None if a.no_sclk else sclk_leg(step)
    if sclk:
        log(f"sclk under the step: median {sclk['median_mhz']:.0f} MHz over {len(sclk['mhz'])} samples")

    verify = None if a.no_sweep else verify_leg(torch, runner, db, torch.empty(n, dtype=torch.int16, device="cuda"),
                                                  n, E, 10)
    if verify is not None:
        db.check_err("verify leg")

    # PCIe-inclusive rate of the host entry point (host ASCII in, accept/edits out): not the headline
    host = None
    if not a.no_sweep:
        ss.ss_filter_batch(b["reads"], b["refs"], b["lengths"], E)          # first call sizes the buffers
        t0 = time.perf_counter()
        hacc, hed = ss.ss_filter_batch(b["reads"], b["refs"], b["lengths"], E)
        host_s = time.perf_counter() - t0
        host = dict(entry="ss_filter_batch", input="pageable", seconds=round(host_s, 4), pairs_per_s=n / host_s,
                    host_bytes_in=int(len(b["reads"]) + len(b["refs"])),
                    identical_outputs=bool(np.array_equal(hacc, acc) and np.array_equal(hed, ed)))
        del hacc, hed
        # the same from pinned host arrays: chunks copied straight to the device, overlapping the filter
        pr, pf = torch.from_numpy(b["reads"]).pin_memory(), torch.from_numpy(b["refs"]).pin_memory()
        ss.ss_filter_batch(pr.numpy(), pf.numpy(), b["lengths"], E)
        t0 = time.perf_counter()
        hacc, hed = ss.ss_filter_batch(pr.numpy(), pf.numpy(), b["lengths"], E)
        pin_s = time.perf_counter() - t0
        host["pinned_input"] = dict(seconds=round(pin_s, 4), pairs_per_s=n / pin_s,
                                    identical_outputs=bool(np.array_equal(hacc, acc) and np.array_equal(hed, ed)))
        del hacc, hed, pr, pf
        log(f"host entry point (PCIe-inclusive): pageable {host_s:.3f} s -> {n / host_s / 1e6:.1f} M pairs/s, "
            f"pinned {pin_s:.3f} s -> {n / pin_s / 1e6:.1f} M pairs/s, identical={host['identical_outputs']}/"
            f"{host['pinned_input']['identical_outputs']}")

    # HBM calibration: a device-to-device copy of 2 GiB (reads and writes 2 GiB each)
    del db.reads, db.refs, packed
    torch.cuda.empty_cache()
    src = torch.empty(2 << 30, dtype=torch.uint8, device="cuda")
    dst = torch.empty_like(src)
    src.fill_(1)
    cp = lambda: dst.copy_(src)
    cp(); torch.cuda.synchronize()
    _, (cp_ms,) = timed_loop([cp], 10, torch)
    copy_gbs = 2 * src.numel() / (cp_ms * 1e-3) / 1e9
    log(f"device copy: {copy_gbs:.0f} GB/s (read + write)")
    # read-only kernel of known size (2 GiB summed as int64): calibrates the fetch counter
    rd = lambda: src.view(torch.int64).sum()
    rd(); torch.cuda.synchronize()
    _, (rd_ms,) = timed_loop([rd], 10, torch)
    read_gbs = src.numel() / (rd_ms * 1e-3) / 1e9
    log(f"device read: {read_gbs:.0f} GB/s")
    del src, dst

    import oracle
    sweeps = None
    if not a.no_sweep:
        sweeps = {"100bp_30M_E0-10": sweep_leg(torch, ss, gen, runner, 1, list(range(0, 11)), 10, batch=b),
                  "250bp_10M_E0-25": sweep_leg(torch, ss, gen, runner, 2, list(range(0, 26)), 10,
                                               plain_and_wave=True)}
    long_pairs = None if a.no_sweep else long_leg(torch, ss, gen, runner, oracle)

    mixed = None
    if not a.no_mixed:
        mixed = mixed_leg(a, torch, ss, gen, runner, oracle)

    serving = serving_host = None
    if not a.no_serve:
        serving = serving_leg(a, ss, gen, runner, oracle)
        if a.serve_mode == "loop":
            # the host-dispatch server on the same schedule's first seconds, for comparison
            serving_host = serving_leg(a, ss, gen, runner, oracle, mode="host", seconds=min(15.0, a.serve_seconds))

    latency = None
    if not a.no_sweep:
        try:
            latency = latency_leg(torch, ss, gen, runner)
        except Exception as e:          # reported, not fatal: the headline is already measured
            latency = {"error": repr(e)}
            log(f"latency leg failed: {e!r}")

    # the oracle on the host cores over the same pairs: its outputs are compared with the step's for
    # every pair, and its rate is the CPU baseline
    cpu = None
    full_mism = None
    if not a.no_cpu:
        threads = min(16, os.cpu_count() or 1)
        k = min(a.cpu_pairs or n, n)
        r = oracle.batch(b["reads"], b["refs"], b["offsets"][:k], b["lengths"][:k], E=E, threads=threads)
        full_mism = int(np.sum((r["accept"] != acc[:k]) | (r["edits"] != ed[:k])))
        what = "all" if k == n else f"the first {k} of the"
        cpu = dict(value=k / r["seconds"], unit="pairs/s", cores=threads, kind="oracle",
                   sample=f"{what} {n} pairs of the 100 bp workload at E={E}, {threads} threads "
                          f"({r['seconds']:.2f} s wall, {r['seconds'] * threads:.1f} CPU-seconds at most); its "
                          f"outputs are compared with the step's on every pair")
        log(f"oracle: {cpu['value'] / 1e6:.2f} M pairs/s on {threads} threads, {full_mism} mismatches over {k} pairs")
        # the same oracle on one thread, over a fixed prefix of the batch
        k1 = min(2_000_000, n)
        r1 = oracle.batch(b["reads"], b["refs"], b["offsets"][:k1], b["lengths"][:k1], E=E, threads=1)
        cpu["one_thread"] = dict(value=k1 / r1["seconds"], unit="pairs/s", cores=1,
                                 sample=f"first {k1} pairs at E={E} ({r1['seconds']:.2f} s)")
        cpu["gpu_over_oracle"] = value / cpu["value"]
        cpu["gpu_over_oracle_one_thread"] = value / cpu["one_thread"]["value"]
        log(f"oracle, one thread: {cpu['one_thread']['value'] / 1e6:.2f} M pairs/s; GPU / oracle "
            f"{cpu['gpu_over_oracle']:.0f}x ({threads} threads), {cpu['gpu_over_oracle_one_thread']:.0f}x (1 thread)")

    # roofline of the step's kernel: algorithmic bytes per launch (2-bit planes of both sequences,
    # m/2 bytes per pair, plus the 2-byte result) over its mean launch time from HIP events on its
    # stream over the timed steps (the median is reported beside it)
    bytes_ = n * (m // 2 + 2)
    achieved = bytes_ / (step_mean_ms * 1e-3) / 1e9
    traffic = measured_traffic("k_sliced_E%d" % E, profile="sliced_sweep_100bp_E5_pmc.md") if n == 30_000_000 else None
    line = {
        "metric": "filtered pairs/sec at 1 GPU (100bp E=5)",
        "value": value,
        "unit": "pairs/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32 bitwise",
        "data": "synthetic (seeded generator; stands in for the paper's 100bp datasets)",
        "config": {"workload": f"100 bp pairs, 30M, 40% k~U{{0..3}} / 40% k~U{{4..15}} / 20% unrelated, E={E}; "
                               "one threshold's launch over the batch encoded once in 2-bit planes resident in HBM",
                   "n_pairs": n, "m": m, "E": E, "kernel": "lane-sliced column sweep (k_sliced<%d>)" % E},
        "step_kernel_median_ms": round(step_ms, 4),
        "step_kernel_mean_ms": round(step_mean_ms, 4),
        "encode_ms": round(pack_ms, 4),
        "encode_plus_step_pairs_per_s": n / (1e-3 * (pack_ms + step_ms)),
        "one_call_ascii": one_call,
        "oracle_full_mismatches": full_mism,
        "oracle_full_pairs": (min(a.cpu_pairs or n, n) if cpu else 0),
        "plain": plain,
        "roofline": {"bound": "hbm", "kernel": "lane-sliced column sweep (k_sliced<%d>)" % E, "achieved": achieved,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "algorithmic_bytes": bytes_, "duration": "mean of the step's HIP events over the timed steps",
                     "bytes_rule": "2-bit planes of read and reference (m/2 B) + 2 B result per pair"},
        "sclk": sclk,
        "cpu_baseline": cpu,
        "paper_context": PAPER_CONTEXT,
        "hbm_copy_calibration_gbs": copy_gbs,
        "hbm_read_calibration_gbs": read_gbs,
        "filter_then_verify": verify,
        "threshold_sweeps": sweeps,
        "latency_10k": latency,
        "host_entry_pcie_inclusive": host,
        "long_100kbp": long_pairs,
        "mixed": mixed,
        "serving": serving,
        "serving_host_dispatch": serving_host,
    }
    print(json.dumps(line), flush=True)
    if full_mism:
        sys.exit(1)


if __name__ == "__main__":
    main()
