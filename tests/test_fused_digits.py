"""CPU model of the fused kernel's counted-column arithmetic (ss_fused.h, wave mode, E >= 3).

The sweeping wavefront stores, per group and column, the word "some row is free" (bit s for pair
slot s of the group).  After the group's last column each of the group's four lanes counts the
columns of its quarter where no row was free, in binary digits saturating at E + 1 (count_digits,
sat_eq, digits_inc), and two butterfly steps over the quad (lane pairs 1,0,3,2 then 2,3,0,1) add
the four shares with a saturating add (sat_add).  The result must equal min(columns with no row
free, E + 1) for every slot: that is the obstacle count the walk of Section 2.4 reports, stopped
once it exceeds E.

This restates the kernel's bitwise steps on 32-bit words held in Python integers and checks them
against the plain count over random column words, for every threshold the fused kernel takes in
this mode and for thresholds up to 14 (four digits).
"""
import random

M32 = 0xFFFFFFFF


def count_digits(S):
    return 1 if S < 2 else 1 + count_digits(S >> 1)


def sat_eq(c, S):
    r = M32
    for d, w in enumerate(c):
        if (S >> d) & 1:
            r &= w
    return r


def digits_inc(c, inc):
    for d in range(len(c)):
        k = c[d] & inc
        c[d] ^= inc
        inc = k


def sat_add(a, b, S):
    nd = len(a)
    s = [0] * nd
    k = 0
    for d in range(nd):
        s[d] = a[d] ^ b[d] ^ k
        k = (a[d] & b[d]) | (a[d] & k) | (b[d] & k)     # majority
    ge = M32
    for d in range(nd):
        ge = (s[d] & ge) if (S >> d) & 1 else (s[d] | ge)
    ge |= k
    return [((s[d] | ge) if (S >> d) & 1 else (s[d] & ~ge & M32)) for d in range(nd)]


def lanes_count(dead, E, lanes=4):
    """The kernel's finish step for one group: dead[j] is the column's "some row is free" word."""
    S = E + 1
    nd = count_digits(S)
    m = len(dead)
    q = (m + lanes - 1) // lanes
    shares = []
    for h in range(lanes):
        c = [0] * nd
        for j in range(h * q, min(m, (h + 1) * q)):
            digits_inc(c, ~dead[j] & ~sat_eq(c, S) & M32)
        shares.append(c)
    # butterfly: lane h adds lane h ^ 1, then lane h ^ 2
    shares = [sat_add(shares[h], shares[h ^ 1], S) for h in range(lanes)]
    shares = [sat_add(shares[h], shares[h ^ 2], S) for h in range(lanes)]
    assert all(x == shares[0] for x in shares), "every lane of the quad ends with the same count"
    c = shares[0]
    accept = ~sat_eq(c, S) & M32
    return [sum(((c[d] >> s) & 1) << d for d in range(nd)) for s in range(32)], accept


def plain(dead, E):
    return [min(E + 1, sum(1 for w in dead if not (w >> s) & 1)) for s in range(32)]


def test_digits_match_the_plain_count():
    rng = random.Random(19100902)
    for E in range(3, 15):
        for trial in range(60):
            m = rng.choice([1, 2, 3, 4, 5, 7, 8, 31, 33, 64, 100, 101, 150, 224])
            p_dead = rng.choice([0.0, 0.02, 0.1, 0.3, 0.7, 1.0])
            dead = []
            for _ in range(m):
                w = 0
                for s in range(32):
                    if rng.random() >= p_dead:
                        w |= 1 << s
                dead.append(w)
            got, accept = lanes_count(dead, E)
            want = plain(dead, E)
            assert got == want, (E, m, trial)
            for s in range(32):
                assert ((accept >> s) & 1) == (want[s] <= E), (E, m, trial, s)


def test_digit_counts_per_threshold():
    # three digits up to E = 6 (count 7), four up to E = 14 (count 15)
    assert [count_digits(E + 1) for E in (3, 5, 6, 7, 10, 14)] == [3, 3, 3, 4, 4, 4]


def test_a_dropped_carry_is_caught():
    """A saturating add that drops the carry out of the top digit is caught: two saturated shares
    added first (the lanes of the first half of the columns) wrap, and the second step's shares of a
    clean half cannot bring the count back."""
    E = 10

    def bad_sat_add(a, b, S):
        nd = len(a)
        s, k = [0] * nd, 0
        for d in range(nd):
            s[d] = a[d] ^ b[d] ^ k
            k = (a[d] & b[d]) | (a[d] & k) | (b[d] & k)
        ge = M32
        for d in range(nd):
            ge = (s[d] & ge) if (S >> d) & 1 else (s[d] | ge)
        return [((s[d] | ge) if (S >> d) & 1 else (s[d] & ~ge & M32)) for d in range(nd)]

    global sat_add
    good = sat_add
    sat_add = bad_sat_add
    try:
        dead = [0] * 50 + [M32] * 50          # no row free in the first half, every row in the second
        assert plain(dead, E) == [E + 1] * 32
        assert lanes_count(dead, E)[0] != plain(dead, E)
    finally:
        sat_add = good
