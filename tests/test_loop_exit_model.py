"""CPU model of how the device-resident serving loop's kernel ends and is launched again
(ss_loop.hip, ss_serve.cpp), checked under random schedules on a discrete clock.

The scheduler of a launch looks at the slots every step and stores its heartbeat (the step); it
activates a published request, and returns once nothing has been active or new for `idle` steps,
raising the launch's quit epoch.  A worker takes a unit of an active request when one is left (one
worker per unit, the others lose the race); otherwise it returns when it sees the quit epoch, or,
as a last guard, when no slot is active and the heartbeat (and its own start) are older than
`orphan` steps.  The host publishes requests at random gaps, and launches the kernel again when it
finds a request published and the last launch over (every block returned).

Checked: no worker returns while its launch's scheduler is running (the pool of workers never
shrinks under a live scheduler), every launch ends (its workers drain once its scheduler has
quit), and every request finishes.  The rule the guard replaced (return after four idle periods
without a claim of its own, whenever no slot is active) is caught shrinking the pool.
"""
import random


def run(rng, n_workers, n_requests, idle=6, orphan=24, old_rule=False, max_units=2, steps=4000, launches=None):
    pending = []                  # published, not activated: [units]
    active = []                   # activated requests: [units left to claim, units running]
    published = 0
    finished = 0
    next_pub = 0
    launch = None                 # dict(epoch, sched_alive, quit, beat, t_busy, workers)
    epoch = 0
    violations = []
    for now in range(steps):
        # host: publish at random gaps; relaunch when a request waits and the last launch is over
        if published < n_requests and now >= next_pub:
            pending.append(rng.randint(1, max_units))
            published += 1
            next_pub = now + rng.choice([0, 1, 2, idle // 2, idle, 2 * idle, 3 * idle])
        if pending and (launch is None or not launch["workers"] and not launch["sched_alive"]):
            epoch += 1
            launch = dict(epoch=epoch, sched_alive=True, quit=False, beat=now, t_busy=now,
                          workers=[dict(state="look", t_start=now, t_claim=now, left=0)
                                   for _ in range(n_workers)])
        if launch is None:
            continue
        agents = ["s"] + list(range(len(launch["workers"])))
        rng.shuffle(agents)
        gone = []
        for a in agents:
            if a == "s":
                if not launch["sched_alive"]:
                    continue
                launch["beat"] = now
                fresh = bool(pending)
                while pending:
                    active.append([pending.pop(0), 0])
                if fresh or active:
                    launch["t_busy"] = now
                elif now - launch["t_busy"] > idle:
                    launch["quit"] = True
                    launch["sched_alive"] = False
                continue
            w = launch["workers"][a]
            if w["state"] == "run":
                w["left"] -= 1
                if w["left"] == 0:
                    req = w["req"]
                    req[1] -= 1
                    if req[0] == 0 and req[1] == 0:
                        active.remove(req)
                        finished += 1
                    w["state"] = "look"
                continue
            cand = [r for r in active if r[0] > 0]
            if cand:
                r = cand[0]
                r[0] -= 1
                r[1] += 1
                w.update(state="run", req=r, left=rng.randint(1, 3), t_claim=now)
                continue
            leave = False
            if launch["quit"]:
                leave = True
            elif old_rule:
                leave = not active and now - w["t_claim"] > 4 * idle
            elif not active:
                leave = now - max(launch["beat"], w["t_start"]) > orphan
            if leave:
                if launch["sched_alive"]:
                    violations.append(f"step {now}: a worker of launch {launch['epoch']} left under a live scheduler")
                gone.append(a)
        for a in sorted(gone, reverse=True):
            launch["workers"].pop(a)
        if launch["sched_alive"] is False and launch["quit"] and launch["workers"]:
            # every worker still there leaves within a few steps of the quit
            launch.setdefault("quit_at", now)
            if now - launch["quit_at"] > 8:
                violations.append(f"launch {launch['epoch']} did not drain")
                break
        if finished == n_requests and not pending:
            break
    if finished != n_requests:
        violations.append(f"{n_requests - finished} of {n_requests} requests never finished")
    if launches is not None:
        launches.append(epoch)
    return violations


def test_exit_rules_under_random_schedules():
    rng = random.Random(1910090211)
    launches = []
    for trial in range(400):
        v = run(rng, rng.randint(1, 6), rng.randint(1, 40), launches=launches)
        assert not v, (trial, v[:3])
    # the schedules end the kernel and launch it again many times (the gaps exceed the idle time)
    assert sum(x > 3 for x in launches) > 100, sorted(launches)[-10:]


def test_the_old_worker_exit_is_caught():
    """Counting idleness from a worker's own last claim lets a worker that lost every race leave
    while the scheduler still runs (the pool shrinks); the model finds such schedules."""
    rng = random.Random(7)
    hits = 0
    for _ in range(200):
        v = run(rng, rng.randint(3, 6), 40, old_rule=True)
        hits += any("live scheduler" in x for x in v)
    assert hits > 0
