"""CPU model of the device-resident serving loop's claim protocol (ss_loop.h, ss_loop.hip), checked
under random schedules.

The host publishes requests into slots and publishes a new request in a slot only after the
previous one finished.  The scheduler activates a published request: it resets the slot's done
counts, stores the closed item counter (generation, count 0, next 0) and then the encoding-unit
counter (generation, n_pack, 0), and sets the slot's active bit.  A worker looks at the slots (a
snapshot of every active slot's counters), picks the oldest one with next < count on its
encoding-unit counter, else on its item counter, and later (any number of other steps may pass in
between, so its snapshot may be stale and the slot may even hold a newer request by then) adds one
to that counter.  The returned value is its claim: valid when its next is below its count, for the
request whose generation it carries.  A valid encoding unit is run and counted; the block that
counts a request's last one opens the item counter (generation, n_items, 0).  A valid item is run
and counted; the block that counts the last one finishes the request (clears the active bit, marks
the slot done for the host).

Checked: every encoding unit and every item of every request runs exactly once, no item of a request
runs before all of its encoding units have finished, every request finishes (no schedule leaves
work unclaimable), and no counter's next field runs more than the number of workers past its
count.
"""
import random


def ctr(gen, count, nxt=0):
    return (gen & 0xFFFF, count, nxt)


def run(rng, n_slots, n_workers, n_requests, max_pack=3, max_items=4, stale_delay=6):
    reqs = [dict(n_pack=rng.randint(1, max_pack), n_items=rng.randint(1, max_items)) for _ in range(n_requests)]
    slot_req = [None] * n_slots           # request index held by the slot (device side)
    pub = [0] * n_slots                   # generation published by the host
    seen = [0] * n_slots
    gen_of = {}                           # (slot, gen) -> request index
    fin = [0] * n_slots
    pack_ctr = [ctr(0, 0)] * n_slots
    item_ctr = [ctr(0, 0)] * n_slots
    pack_done = [0] * n_slots
    item_done = [0] * n_slots
    active = [False] * n_slots
    adm = [0] * n_slots
    adm_next = 0
    next_req = 0
    gen_next = [0] * n_slots
    ran_pack = {}
    ran_item = {}
    pack_finished = {}                    # request -> number of encoding units finished
    finished = set()
    violations = []
    max_over = 0
    # worker state: ("look",) | ("add", slot, kind, delay) | ("run", kind, slot, gen, unit, steps, request)
    workers = [("look",) for _ in range(n_workers)]

    def host_step():
        nonlocal next_req
        for s in range(n_slots):
            if next_req < n_requests and (pub[s] == 0 or fin[s] == pub[s]):
                gen_next[s] += 1
                pub[s] = gen_next[s]
                gen_of[(s, pub[s])] = next_req
                next_req += 1
                return True
        return False

    def sched_step():
        nonlocal adm_next
        for s in range(n_slots):
            if pub[s] != seen[s]:
                r = gen_of[(s, pub[s])]
                slot_req[s] = (r, pub[s])
                pack_done[s] = 0
                item_done[s] = 0
                adm[s] = adm_next
                adm_next += 1
                item_ctr[s] = ctr(pub[s], 0)
                pack_ctr[s] = ctr(pub[s], reqs[r]["n_pack"])
                active[s] = True
                seen[s] = pub[s]
                return True
        return False

    def worker_step(w):
        nonlocal max_over
        st = workers[w]
        if st[0] == "look":
            best = None
            for s in range(n_slots):
                if not active[s]:
                    continue
                g, c, nx = pack_ctr[s]
                if nx < c:
                    kind = "pack"
                else:
                    g, c, nx = item_ctr[s]
                    if nx >= c:
                        continue
                    kind = "item"
                if best is None or adm[s] < best[0]:
                    best = (adm[s], s, kind)
            if best is None:
                return False
            workers[w] = ("add", best[1], best[2], rng.randint(0, stale_delay))
            return True
        if st[0] == "add":
            _, s, kind, delay = st
            if delay > 0:
                workers[w] = ("add", s, kind, delay - 1)
                return True
            arr = pack_ctr if kind == "pack" else item_ctr
            g, c, nx = arr[s]
            arr[s] = (g, c, nx + 1)
            max_over = max(max_over, nx + 1 - c)
            if nx < c:
                # the counter always carries the generation of the request now in the slot
                r, full = slot_req[s]
                assert g == full & 0xFFFF
                if kind == "item" and pack_finished.get(r, 0) != reqs[r]["n_pack"]:
                    violations.append(f"item {nx} of request {r} runs before its planes are complete")
                workers[w] = ("run", kind, s, g, nx, rng.randint(1, 3), r)
            else:
                workers[w] = ("look",)
            return True
        # running a claimed unit
        _, kind, s, g, unit, steps, r = st
        if steps > 1:
            workers[w] = ("run", kind, s, g, unit, steps - 1, r)
            return True
        if kind == "pack":
            key = (r, unit)
            ran_pack[key] = ran_pack.get(key, 0) + 1
            pack_finished[r] = pack_finished.get(r, 0) + 1
            pack_done[s] += 1
            if pack_done[s] == reqs[r]["n_pack"]:
                item_ctr[s] = ctr(g, reqs[r]["n_items"])
        else:
            key = (r, unit)
            ran_item[key] = ran_item.get(key, 0) + 1
            item_done[s] += 1
            if item_done[s] == reqs[r]["n_items"]:
                active[s] = False
                fin[s] = slot_req[s][1]
                finished.add(r)
        workers[w] = ("look",)
        return True

    for _ in range(200000):
        agents = ["h", "s"] + list(range(n_workers))
        rng.shuffle(agents)
        moved = False
        for a in agents:
            if a == "h":
                moved = host_step()
            elif a == "s":
                moved = sched_step()
            else:
                moved = worker_step(a)
            if moved:
                break
        if not moved:
            break
    for r in range(n_requests):
        for u in range(reqs[r]["n_pack"]):
            if ran_pack.get((r, u), 0) != 1:
                violations.append(f"encoding unit {u} of request {r} ran {ran_pack.get((r, u), 0)} times")
        for u in range(reqs[r]["n_items"]):
            if ran_item.get((r, u), 0) != 1:
                violations.append(f"item {u} of request {r} ran {ran_item.get((r, u), 0)} times")
    if len(finished) != n_requests:
        violations.append(f"{n_requests - len(finished)} requests never finished")
    if max_over > n_workers:
        violations.append(f"a counter ran {max_over} past its count with {n_workers} workers")
    return violations


def test_claims_under_random_schedules():
    rng = random.Random(19100902)
    for trial in range(1500):
        n_slots = rng.randint(1, 4)
        n_workers = rng.randint(1, 6)
        v = run(rng, n_slots, n_workers, rng.randint(1, 12))
        assert not v, (trial, n_slots, n_workers, v[:3])


def mutant(old, new):
    """run() with one line of the protocol changed (the model must be able to fail)."""
    import inspect
    src = inspect.getsource(run)
    assert old in src
    g = dict(globals())
    exec(compile(src.replace(old, new), __file__, "exec"), g)
    return g["run"]


def test_an_open_item_counter_at_activation_is_caught():
    """Publishing the item counter open (count n_items) at activation lets items run before the
    planes exist; the model finds such schedules."""
    bad = mutant('item_ctr[s] = ctr(pub[s], 0)', 'item_ctr[s] = ctr(pub[s], reqs[r]["n_items"])')
    rng = random.Random(3)
    assert any(any("before its planes" in x for x in bad(rng, 2, 4, 6)) for _ in range(300))


def test_a_lost_claim_is_caught():
    """Dropping a valid claim (a block that claims and then does not run the unit) leaves a request
    unfinished; the model reports it."""
    bad = mutant('workers[w] = ("run", kind, s, g, nx, rng.randint(1, 3), r)', 'workers[w] = ("look",)')
    rng = random.Random(4)
    assert any(any("never finished" in x for x in bad(rng, 2, 3, 5)) for _ in range(50))
