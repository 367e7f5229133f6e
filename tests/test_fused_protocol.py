"""CPU model of the fused kernel's synchronisation (ss_fused.h, k_fused), checked under random schedules.

Wave mode: three encoding wavefronts take the block's units k = w, w+3, ... (unit k: tile k // upt of
the block, U groups); a unit of tile i >= 2 first waits until the sweep count reaches i - 1 (the
buffer's previous tile, i - 2, swept), then encodes into buffer i % 2, then adds one to that
buffer's done count.  The sweeping wavefront takes tile i once buffer i % 2's done count reaches
upt * (i // 2 + 1), sweeps it and adds one to the sweep count.  The model runs these steps as
separate events under a random scheduler and checks that the block drains (no wait is left
unsatisfied), that no unit writes a buffer whose previous tile is still unswept or being swept, and
that no sweep starts before every unit of its tile with groups has been encoded.

Block mode: the encoders pass four barriers per step of GB groups, and the sweeping wavefront passes
as many while it sweeps the previous tile in as many pieces; the model checks that both sides pass
the same number of barriers and that every (group pass, item) of every tile is swept once.
"""
import random

import pytest


def wave_mode_run(nmine, T, U, last_groups, rng, wait_for_empty_units=True, enc_steps=3, sweep_steps=3):
    """One random schedule of a block with nmine tiles of T groups (the last one holding last_groups),
    units of U groups.  Returns a list of violations (empty when the schedule is correct)."""
    upt = T // U
    tiles = [T] * nmine
    tiles[-1] = last_groups

    def unit_groups(k):
        if k >= nmine * upt:
            return 0
        i, u = divmod(k, upt)
        return min(U, tiles[i] - u * U)

    done = [0, 0]
    swept = 0
    encoded = [[False] * upt for _ in range(nmine)]
    sweeping = None               # tile being swept
    writing = {}                  # wave -> tile it is writing
    violations = []
    # encoder state: (list of its units, index, phase, steps left)
    enc = []
    for w in range(3):
        units = list(range(w, nmine * upt, 3))
        enc.append({"units": units, "i": 0, "phase": "wait", "left": 0})
    sw = {"tile": 0, "phase": "wait", "left": 0}

    def enc_runnable(e):
        if e["i"] >= len(e["units"]):
            return False
        k = e["units"][e["i"]]
        i = k // upt
        if e["phase"] == "wait":
            needs_wait = i >= 2 and (unit_groups(k) > 0 or wait_for_empty_units)
            return (not needs_wait) or swept >= i - 1
        return True

    def sw_runnable():
        i = sw["tile"]
        if i >= nmine:
            return False
        if sw["phase"] == "wait":
            return done[i % 2] >= upt * (i // 2 + 1)
        return True

    for _ in range(100000):
        agents = [("e", w) for w in range(3) if enc_runnable(enc[w])] + ([("s", 0)] if sw_runnable() else [])
        if not agents:
            break
        kind, w = rng.choice(agents)
        if kind == "e":
            e = enc[w]
            k = e["units"][e["i"]]
            i, u = divmod(k, upt)
            if e["phase"] == "wait":
                if unit_groups(k) > 0:
                    e["phase"], e["left"] = "encode", rng.randint(1, enc_steps)
                    writing[w] = i
                    # the buffer must not hold an unswept earlier tile of its parity
                    if i >= 2 and (swept < i - 1 or sweeping == i - 2):
                        violations.append(f"unit {u} of tile {i} writes buffer {i % 2} before tile {i - 2} is swept")
                else:
                    e["phase"] = "arrive"
            elif e["phase"] == "encode":
                if sweeping is not None and sweeping % 2 == i % 2 and sweeping != i:
                    violations.append(f"tile {i} written while tile {sweeping} is swept from the same buffer")
                e["left"] -= 1
                if e["left"] == 0:
                    encoded[i][u] = True
                    writing.pop(w, None)
                    e["phase"] = "arrive"
            else:
                done[i % 2] += 1
                e["i"] += 1
                e["phase"] = "wait"
        else:
            i = sw["tile"]
            if sw["phase"] == "wait":
                missing = [u for u in range(upt) if unit_groups(i * upt + u) > 0 and not encoded[i][u]]
                if missing:
                    violations.append(f"tile {i} swept before units {missing} were encoded")
                sweeping = i
                sw["phase"], sw["left"] = "sweep", rng.randint(1, sweep_steps)
            else:
                sw["left"] -= 1
                if sw["left"] == 0:
                    swept += 1
                    sweeping = None
                    sw["tile"] += 1
                    sw["phase"] = "wait"
    left = [w for w in range(3) if enc[w]["i"] < len(enc[w]["units"])]
    if left or sw["tile"] < nmine:
        violations.append(f"deadlock: encoders {left} unfinished, sweep at tile {sw['tile']} of {nmine}")
    return violations


def test_wave_mode_protocol_random_schedules():
    rng = random.Random(1910)
    for trial in range(3000):
        T = rng.choice([2, 4, 8, 16, 32])
        U = rng.choice([u for u in (1, 2) if T % u == 0])
        nmine = rng.randint(1, 9)
        last = rng.randint(1, T)
        v = wave_mode_run(nmine, T, U, last, rng)
        assert not v, (trial, nmine, T, U, last, v[:3])


def test_units_without_groups_must_wait_too():
    """A unit past the batch's last group encodes nothing, but it still counts toward its buffer's done
    count; without the wait it could raise that count before the tile two back is complete (the model
    finds such schedules), which is why every unit of tile i >= 2 waits for the sweep count."""
    rng = random.Random(7)
    found = False
    for _ in range(20000):
        v = wave_mode_run(4, 16, 2, rng.randint(1, 10), rng, wait_for_empty_units=False, enc_steps=8)
        if any("swept before" in x for x in v):
            found = True
            break
    assert found


def block_mode_counts(G, T, GB, grid, block, GPP=16, nci=13):
    """Barriers each role passes and the sweep items it covers, for one block of the block-mode
    schedule (tiles of T groups dealt round-robin over the grid; GB groups per encoding step)."""
    ntiles = -(-G // T)
    mine = list(range(block, ntiles, grid))
    tg = [min(T, G - t * T) for t in mine]
    steps = [-(-g // GB) for g in tg]
    enc_barriers = sum(4 * s for s in steps)
    sweep_barriers = 0
    swept = []
    for i in range(len(mine) + 1):
        nint = 4 * steps[i] if i < len(mine) else 0
        if i == 0:
            sweep_barriers += nint
            continue
        g = tg[i - 1]
        work = -(-g // GPP) * nci
        it, pas, c = 0, 0, 0
        items = []
        for b in range(max(nint, 1)):
            end = work * (b + 1) // nint if nint > 0 else work
            while it < end:
                items.append((pas, c))
                it += 1
                c += 1
                if c == nci:
                    c, pas = 0, pas + 1
            if nint > 0:
                sweep_barriers += 1
        swept.append((g, items))
    return enc_barriers, sweep_barriers, swept


def test_block_mode_barriers_and_coverage():
    rng = random.Random(3)
    for _ in range(3000):
        GB = rng.choice([1, 2, 4, 8])
        T = GB * rng.randint(1, 8)
        G = rng.randint(1, 400)
        grid = rng.randint(1, 40)
        nci = rng.randint(1, 30)
        for block in {0, grid - 1, rng.randrange(grid)}:
            if block * T >= G:
                continue
            e, s, swept = block_mode_counts(G, T, GB, grid, block, nci=nci)
            assert e == s, (G, T, GB, grid, block)
            for g, items in swept:
                passes = -(-g // 16)
                assert items == [(p, c) for p in range(passes) for c in range(nci)], (G, T, GB, grid, block)
