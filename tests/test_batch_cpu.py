"""Host-side checks of the batched-launch planner (no device work)."""
import numpy as np
import pytest

import paper_1910_09020_amd as ss


def test_plan_validation_without_device():
    L = ss.lib()
    assert L.ss_plan_create(None, None, None, 0, 8, None) == ss.SS_EINVAL
    bad = ss.SS_EINVAL
    assert L.ss_plan_info(None, None, None, None, None) == bad
    assert L.ss_plan_launch(None, None) == bad
    assert L.ss_plan_destroy(None) == bad


def _shape_for(E, rsmax):
    """Lanes per pair and slices per lane for threshold E at width rsmax (2E+1 rows in 32-row slices)."""
    SL = (2 * E + 1 + 31) // 32
    if SL <= rsmax:
        return 1, SL
    L = 1
    while L * rsmax < SL:
        L <<= 1
    return L, (SL + L - 1) // L


def _level(x):
    l = 0
    while x >= 4:
        x *= 0.25
        l += 1
    return l


@pytest.mark.parametrize("spl", [1, 4, 8])
def test_host_plan_invariants(spl):
    """The planner's items on a mixed batch (short and 10 kbp pairs, per-pair E): the permutation covers
    every pair once, items cut it into contiguous runs of one shape with their largest threshold, one-lane
    items are 256-pair chunks of their class in input order (longest first inside), and the queue goes by
    cost level, then (items of several lanes) threshold level, then input position."""
    from paper_1910_09020_amd import gen
    b = gen.make(3, n=40000, n_long=60)
    lengths, E = b["lengths"], b["E"]
    n = len(lengths)
    items, perm = ss.ss_plan_items_host(lengths, E, spl)
    slices = (2 * int(E.max()) + 1 + 31) // 32
    rsmax = max(spl, min(r for r in (1, 2, 4, 8) if 64 * r >= slices))
    assert np.array_equal(np.sort(perm), np.arange(n))
    by_first = items[np.argsort(items[:, 0])]
    assert by_first[0, 0] == 0 and by_first[-1, 0] + by_first[-1, 1] == n
    assert np.all(by_first[1:, 0] == by_first[:-1, 0] + by_first[:-1, 1])
    shapes = [_shape_for(int(e), rsmax) for e in E]
    members = {}
    for i in range(n):
        if shapes[i][0] == 1:
            members.setdefault(shapes[i], []).append(i)
    chunks = {frozenset(v[k:k + 256]) for v in members.values() for k in range(0, len(v), 256)}
    keys = []
    for first, count, lp, rs, emax in items:
        pairs = perm[first:first + count]
        assert 0 < count <= 4 * 64 // lp
        assert all(shapes[p] == (lp, rs) for p in pairs)
        assert emax == E[pairs].max()
        if lp == 1:
            assert frozenset(pairs.tolist()) in chunks
            assert np.all(np.diff(lengths[pairs]) <= 0)
        cost = float(lengths[pairs].max()) * rs * 4
        elevel = int(np.floor(np.log2(emax + 1))) if lp > 1 else 0
        keys.append((-_level(cost), -elevel, int(perm[first])))
    assert keys == sorted(keys)


@pytest.mark.parametrize("spl", [1, 8])
def test_host_plan_order_is_the_plain_sort(spl):
    """The permutation is exactly the plain sort of the pairs by (shape class in order of first
    appearance, 256-pair chunk of one-lane classes in input order, length descending, threshold
    descending, input position), on lengths up to the limit and many ties."""
    rng = np.random.default_rng(19100)
    for trial in range(6):
        n = int(rng.integers(500, 3000))
        lengths = rng.choice(np.array([0, 1, 100, 250, 10_000, (1 << 24) - 1, 1 << 24], np.int32), n)
        if trial % 2:
            lengths = rng.integers(0, (1 << 24) + 1, n).astype(np.int32)
        E = rng.choice(np.array([0, 1, 5, 15, 16, 100, 127, 128, 1000, 4000], np.int32), n)
        items, perm = ss.ss_plan_items_host(lengths, E, spl)
        slices = (2 * int(E.max()) + 1 + 31) // 32
        rsmax = max(spl, min(r for r in (1, 2, 4, 8) if 64 * r >= slices))
        shapes = [_shape_for(int(e), rsmax) for e in E]
        cid, seen, key = {}, {}, []
        for i in range(n):
            c = cid.setdefault(shapes[i], len(cid))
            chunk = 0
            if shapes[i][0] == 1:
                chunk = seen.get(c, 0) // 256
                seen[c] = seen.get(c, 0) + 1
            key.append((c, chunk, -int(lengths[i]), -int(E[i]), i))
        assert perm.tolist() == [k[4] for k in sorted(key)], trial


def test_host_plan_errors():
    lengths = np.full(4, 100, np.int32)
    with pytest.raises(ss.SSError) as e:
        ss.ss_plan_items_host(lengths, np.array([5, 5, 5, 8192], np.int32), 8)
    assert e.value.status == ss.SS_ELEN
    with pytest.raises(ss.SSError) as e:
        ss.ss_plan_items_host(lengths, np.full(4, 5, np.int32), 3)
    assert e.value.status == ss.SS_EINVAL
    with pytest.raises(ss.SSError) as e:
        ss.ss_plan_items_host(np.array([100, -1, 100, 100], np.int32), np.full(4, 5, np.int32), 4)
    assert e.value.status == ss.SS_EINVAL
    items, perm = ss.ss_plan_items_host(np.zeros(0, np.int32), np.zeros(0, np.int32), 4)
    assert items.shape == (0, 5) and perm.shape == (0,)
