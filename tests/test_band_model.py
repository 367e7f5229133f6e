"""CPU model of the banded verifier's window (k_verify_band in ss_verify.hip), checked against the
oracle's Levenshtein distance.

The model runs the same steps on Python integers (the whole window as one bit-vector, so the
carries the kernel resolves across lanes are plain integer addition): a window of NW words of WB
positions, bottom position lo; before every WB columns the bottom word is dropped once it lies
wholly below the band (lo + WB <= j - E), its vertical deltas going into the value B of the row
under the window and a word of +1 deltas entering at the top; each column is Myers' step with the
row under the window growing by one (bottom shift-in +1); at the end D = B + the vertical deltas of
the window's rows below m.  Small word sizes (4, 8) drop many words on short pairs.  Expected:
the distance when it is <= E, else E + 1.
"""
import random

import oracle


def band(q: bytes, r: bytes, E: int, WB: int = 32, drop_to_B: bool = True) -> int:
    m = len(q)
    NW = (2 * E + 2 * WB + 1 + WB - 1) // WB
    CAP = NW * WB
    FULL = (1 << CAP) - 1
    lo, pv, mv, B = 0, FULL, 0, 0
    for jb in range(0, m, WB):
        if lo + WB <= jb - E:
            low = (1 << WB) - 1
            if drop_to_B:
                B += bin(pv & low).count("1") - bin(mv & low).count("1")
            pv = (pv >> WB) | (low << (CAP - WB))
            mv >>= WB
            lo += WB
        for j in range(jb, min(m, jb + WB)):
            eq = 0
            for x in range(min(CAP, m - lo)):
                if q[lo + x] == r[j]:
                    eq |= 1 << x
            xv = eq | mv
            xh = ((((eq & pv) + pv) & FULL) ^ pv) | eq
            ph = mv | (~(xh | pv) & FULL)
            mh = pv & xh
            ph = ((ph << 1) | 1) & FULL
            mh = (mh << 1) & FULL
            pv = mh | (~(xv | ph) & FULL)
            mv = ph & xv
            B += 1
    keep = max(0, min(CAP, m - lo))
    mask = (1 << keep) - 1
    D = B + bin(pv & mask).count("1") - bin(mv & mask).count("1")
    return D if D <= E else E + 1


def pairs(rng, count, max_m=120):
    out = []
    for _ in range(count):
        m = rng.randint(0, max_m)
        q = [rng.choice(b"ACGT") for _ in range(m)]
        r = list(q)
        rate = rng.choice([0, 0.02, 0.05, 0.1, 0.3, 1.0])
        for i in range(m):
            if rng.random() < rate:
                r[i] = rng.choice(b"ACGT")
        if m > 3 and rng.random() < 0.5:
            for _ in range(rng.randint(1, 4)):
                del r[rng.randrange(len(r))]
                r.insert(rng.randrange(len(r) + 1), rng.choice(b"ACGT"))
        r = (r + [rng.choice(b"ACGT") for _ in range(m)])[:m]
        out.append((bytes(q), bytes(r)))
    return out


def test_band_window_matches_levenshtein():
    rng = random.Random(5)
    for q, r in pairs(rng, 1500):
        E = rng.randint(0, 30)
        WB = rng.choice([4, 8, 32])
        L = oracle.levenshtein(q, r)
        assert band(q, r, E, WB) == (L if L <= E else E + 1), (len(q), E, WB, L)


def test_a_dropped_word_left_out_of_B_is_caught():
    """Dropping the bottom word without adding its deltas to the boundary value is wrong, and the
    model's check sees it."""
    rng = random.Random(6)
    wrong = 0
    for q, r in pairs(rng, 400):
        E = rng.randint(0, 10)
        L = oracle.levenshtein(q, r)
        wrong += band(q, r, E, 4, drop_to_B=False) != (L if L <= E else E + 1)
    assert wrong > 0
