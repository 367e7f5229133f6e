"""Pins of the oracle's Snake-on-Chip decomposition (Section 2.5): sub-mazes of t columns solved
one by one by the greedy walk, counts summed.  What fixes it besides its own code:

- t >= m leaves one sub-maze, the whole maze: the count is SneakySnake's own (Section 2.4);
- t = 1: a one-column sub-maze contributes an obstacle exactly when no query character within
  distance E of the column's position equals the reference character there (all 2E+1 cells of
  Equation 1 are obstacles), so the count is the number of such columns, found here by a direct
  scan of the two strings;
- a finer partition (t dividing t') never counts more: any net of a coarse sub-maze, cut at the fine
  boundaries, is a net of each fine sub-maze with no more obstacles;
- no t counts more than the whole-maze walk, so the filter stays a lower bound on the edit distance
  whenever that distance is <= E (Section 2.5: underestimation, never overestimation).
"""
import itertools

import numpy as np
import pytest

import oracle


def _rand(m, seed, rate=0.15):
    rng = np.random.default_rng(seed)
    q = rng.choice(list("ACGT"), size=m)
    r = q.copy()
    mask = rng.random(m) < rate
    r[mask] = rng.choice(list("ACGT"), size=int(mask.sum()))
    return "".join(r), "".join(q)


def test_whole_maze_equals_sneakysnake():
    for seed in range(200):
        m = 1 + seed % 60
        R, Q = _rand(m, seed)
        for E in (0, 1, 3, 6):
            for t in (m, m + 5, 1000):
                assert oracle.submaze(R, Q, E, t) == oracle.pair(R, Q, E)
                assert oracle.submaze(R, Q, E, t, stop_early=False)[1] == oracle.pair(R, Q, E, stop_early=False)[1]


def test_unit_width_counts_unmatched_columns():
    for seed in range(300):
        m = 1 + seed % 40
        R, Q = _rand(m, seed, rate=0.5)
        for E in (0, 1, 2, 5):
            # columns j whose reference character equals no query character at distance <= E
            lonely = sum(1 for j in range(m) if all(Q[x] != R[j] for x in range(max(0, j - E), min(m, j + E + 1))))
            assert oracle.submaze(R, Q, E, 1, stop_early=False)[1] == lonely


def test_refinement_and_lower_bound_small():
    """Pairs over {A,C,G,T} of length 5 (6,000 drawn from all 4^10, and 64 identical pairs):
    refinement, count <= whole-maze count, and count <= edit distance whenever that is <= E."""
    m = 5
    seqs = ["".join(p) for p in itertools.product("ACGT", repeat=m)]
    rng = np.random.default_rng(0)
    pairs = [(seqs[i], seqs[j]) for i, j in zip(rng.integers(0, len(seqs), 6000), rng.integers(0, len(seqs), 6000))]
    pairs += [(s, s) for s in seqs[:64]]
    for R, Q in pairs:
        ed = oracle.levenshtein(R, Q)
        for E in (0, 1, 2, 3):
            full = oracle.pair(R, Q, E, stop_early=False)[1]
            c = {t: oracle.submaze(R, Q, E, t, stop_early=False)[1] for t in (1, 2, 3, 4)}
            assert c[1] <= c[2] <= c[4] <= full
            assert c[1] <= c[3] <= full
            if ed <= E:
                assert all(v <= ed for v in c.values())
                assert all(oracle.submaze(R, Q, E, t)[0] == 1 for t in (1, 2, 3, 4))


def test_truncation_and_batch():
    reads, refs, offs, lens = [], [], [], []
    pos = 0
    for seed in range(64):
        m = 20 + seed
        R, Q = _rand(m, seed, rate=0.3)
        reads.append(Q); refs.append(R); offs.append(pos); lens.append(m); pos += m
    rd = np.frombuffer("".join(reads).encode(), np.uint8)
    rf = np.frombuffer("".join(refs).encode(), np.uint8)
    for E, t in ((2, 8), (5, 8), (5, 16)):
        b = oracle.submaze_batch(rd, rf, np.array(offs), np.array(lens), E, t)
        for i in range(64):
            full = oracle.submaze(refs[i], reads[i], E, t, stop_early=False)[1]
            assert b["edits"][i] == min(full, E + 1)
            assert b["accept"][i] == (full <= E)
