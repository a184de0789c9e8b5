"""CPU model check of the persistent serving launch's protocol (the host ring, the teams'
barriers, stop and relaunch), replayed step by step under random interleavings.

Each workgroup and the host are generators that yield at every access to shared memory;
a seeded scheduler interleaves them (sequentially consistent memory: within a batch the
launch's cross-workgroup words are device-coherent atomics, each wave's accesses complete
before it arrives at a barrier, and the ring words are system-scope atomics with fences;
the arena's reuse under write-back caches is modelled in test_serve_cache_model).  Checked over many seeds and shapes (teams, workgroups per team, batches):
- every published batch is served exactly once, with the descriptors the host wrote;
- within a batch, no workgroup starts a step before every workgroup of its team finished
  the previous one;
- a stop ends the launch only after every published batch is complete, and a relaunch
  numbers its batches from 0 again;
- nothing deadlocks.
Planted mistakes (a barrier that reads its generation after arriving, an exit decision
that skips the barrier, a host that publishes before it writes the slot) each fail.
"""
import random

import pytest

RING = 8
STEPS = 4


class Deadlock(Exception):
    pass


def run(seed, teams, per_team, n_batches, relaunch_every=None, mistake=None):
    rng = random.Random(seed)
    mem = {"published": 0, "stop": 0}
    for s in range(RING):
        mem[("done", s)] = 0
        mem[("slot", s)] = None
    for t in range(teams):
        mem[("count", t)] = mem[("gen", t)] = mem[("exit", t)] = 0
        mem[("cur", t)] = None
    served = []   # (launch, batch seq, content) per team's first workgroup
    trace = []    # (launch, team, seq, step, wg, "begin"/"end")
    G = per_team

    def barrier(t):
        if mistake == "late-generation":
            c = yield ("add", ("count", t), 1)
            g = yield ("load", ("gen", t))
        else:
            g = yield ("load", ("gen", t))
            c = yield ("add", ("count", t), 1)
        if c == G - 1:
            yield ("store", ("count", t), 0)
            yield ("add", ("gen", t), 1)
            return
        while True:
            cur = yield ("load", ("gen", t))
            if cur != g:
                return

    def workgroup(launch, t, w):
        b = t
        while True:
            slot = b % RING
            if w == 0:
                state = None
                while state is None:
                    pub = yield ("load", "published")
                    if pub > b:
                        state = 0
                        break
                    stop = yield ("load", "stop")
                    if stop:
                        if mistake == "stop-without-recheck":
                            state = 1
                            break
                        pub = yield ("load", "published")  # after seeing stop, the count is final
                        state = 0 if pub > b else 1
                if state == 0:
                    content = yield ("load", ("slot", slot))
                    served.append((launch, b, content))
                    yield ("store", ("cur", t), content)
                else:
                    yield ("store", ("exit", t), 1)
                    if mistake == "exit-without-barrier":
                        return
            yield from barrier(t)
            ex = yield ("load", ("exit", t))
            if ex:
                return
            for step in range(STEPS):
                trace.append((launch, t, b, step, w, "begin"))
                yield ("work",)
                trace.append((launch, t, b, step, w, "end"))
                yield from barrier(t)
            if w == 0:
                yield ("store", ("done", slot), b + 1)
            b += teams

    def reset_launch():
        mem["published"] = 0
        mem["stop"] = 0
        for s in range(RING):
            mem[("done", s)] = 0
        for t in range(teams):
            mem[("count", t)] = mem[("gen", t)] = mem[("exit", t)] = 0

    published_total = []  # (launch, seq, content)
    procs = {}
    launch_id = [0]

    def start():
        reset_launch()
        for t in range(teams):
            for w in range(G):
                procs[(launch_id[0], t, w)] = workgroup(launch_id[0], t, w)

    def host():
        sent = 0
        seq = 0
        inflight = []
        start()
        while sent < n_batches or inflight:
            if relaunch_every and sent and sent % relaunch_every == 0 and seq > 0:
                # a new scene version: stop with batches possibly in flight, as the host does
                # when a frame falls due; every published batch must be complete at the exit
                mem["stop"] = 1
                yield ("wait-exit",)
                inflight = [s for s in inflight if mem[("done", s % RING)] != s + 1]
                assert not inflight, "the launch left before serving a published batch"
                launch_id[0] += 1
                seq = 0
                start()
            if sent < n_batches and len(inflight) < RING and all(s % RING != seq % RING for s in inflight):
                content = (launch_id[0], seq, sent)
                if mistake == "publish-first":
                    mem["published"] = seq + 1
                    yield ("host",)
                    mem[("slot", seq % RING)] = content
                else:
                    mem[("slot", seq % RING)] = content
                    yield ("host",)
                    mem["published"] = seq + 1
                published_total.append(content)
                inflight.append(seq)
                seq += 1
                sent += 1
                yield ("host-progress",)
            yield ("host",)
            before = len(inflight)
            inflight = [s for s in inflight if mem[("done", s % RING)] != s + 1]
            if len(inflight) != before:
                yield ("host-progress",)
        mem["stop"] = 1
        yield ("wait-exit",)

    h = host()
    pending = {}  # value to send to each process when it next runs
    host_waiting = False
    idle = 0
    while True:
        alive = list(procs.keys())
        host_can = not host_waiting or not any(k[0] == launch_id[0] for k in alive)
        choices = alive + (["host"] if h is not None and host_can else [])
        if not choices:
            break
        if idle > 20000:
            raise Deadlock(f"no progress (seed {seed})")
        c = rng.choice(choices)
        if c == "host":
            host_waiting = False
            try:
                op = next(h)
            except StopIteration:
                h = None
                continue
            if op[0] == "wait-exit":
                host_waiting = True
            if op[0] == "host":
                idle += 1
            else:
                idle = 0
            continue
        g = procs[c]
        try:
            op = g.send(pending.pop(c, None))
        except StopIteration:
            del procs[c]
            idle = 0
            continue
        kind = op[0]
        if kind == "load":
            pending[c] = mem[op[1]]
            idle += 1
        elif kind == "store":
            mem[op[1]] = op[2]
            idle = 0
        elif kind == "add":
            pending[c] = mem[op[1]]
            mem[op[1]] += op[2]
            idle = 0
        else:
            idle = 0
    return served, trace, published_total


def check(served, trace, published, teams, per_team):
    assert all(c is not None and (launch, b) == c[:2] for launch, b, c in served), "stale or missing descriptors"
    assert sorted(c for _, _, c in served) == sorted(published), "a batch served twice or missed"
    by = {}
    for i, (launch, t, b, step, w, ev) in enumerate(trace):
        by.setdefault((launch, t, b), []).append((i, step, w, ev))
    for key, evs in by.items():
        for step in range(1, STEPS):
            first_begin = min(i for i, s, w, ev in evs if s == step and ev == "begin")
            last_end = max(i for i, s, w, ev in evs if s == step - 1 and ev == "end")
            assert last_end < first_begin, f"step {step} began before step {step - 1} ended in {key}"
        assert len({w for _, s, w, ev in evs}) == per_team


SHAPES = [(1, 1, 5), (1, 3, 6), (2, 2, 9), (4, 2, 13), (3, 3, 10)]


@pytest.mark.parametrize("teams,per_team,n", SHAPES)
def test_protocol_random_interleavings(teams, per_team, n):
    for seed in range(40):
        served, trace, published = run(seed, teams, per_team, n, relaunch_every=4 if seed % 2 else None)
        check(served, trace, published, teams, per_team)


@pytest.mark.parametrize("mistake", ["late-generation", "exit-without-barrier", "publish-first",
                                     "stop-without-recheck"])
def test_planted_mistakes_fail(mistake):
    failed = False
    for seed in range(400):
        teams, per_team = (2, 1) if seed % 2 else (2, 3)
        try:
            served, trace, published = run(seed, teams, per_team, 12, relaunch_every=2, mistake=mistake)
            check(served, trace, published, teams, per_team)
        except (AssertionError, Deadlock, KeyError):
            failed = True
            break
    assert failed, mistake
