"""Model check, on the CPU, of the open-addressing map's protocol (one device thread per
operation, Sec. 5 semantics): each operation's steps are replayed as a generator that
yields at every memory access, interleaved at random, in the memory model of
test_chain_protocol_model (each word coherent on its own, loads possibly returning
older values of a word).  Key words only move EMPTY -> key -> TOMB and a value word
only PENDING -> value, so the key CAS decides every race and a reader that sees a key
with a PENDING value reads the value again.

Checked: per-key linearizability of random same-key batches (PENDING shares its bit
pattern with ABSENT, so a find that returned an unpublished value fails it) and no key in
two slots.  Planted mistakes - an insert that reuses tombstones, a find that stops at one
- fail within the first seeds.
"""
import random

import pytest

from test_chain_protocol_model import ABSENT, Lane, Memory, serial_ok

EMPTY, TOMB, PENDING = -1, -2, -(1 << 31)


class OpenModel:
    def __init__(self, slots):
        self.n = slots
        words = {}
        for i in range(slots):
            words[("k", i)] = EMPTY
            words[("v", i)] = PENDING
        self.mem = Memory(words)

    def home(self, key):
        return (key * 2654435761) % self.n

    def load(self, L, w):
        yield
        return L.ld(w)

    def op(self, L, op, key, val, out, idx):
        p = self.home(key)
        n = 0
        while n < self.n:
            cur = yield from self.load(L, ("k", p))
            step = 1
            if cur == key:
                if op == 0:
                    out[idx] = 0
                    return
                if op == 2:
                    yield
                    out[idx] = 1 if L.cas(("k", p), key, TOMB) else 0
                    return
                v = yield from self.load(L, ("v", p))
                if v != PENDING:
                    out[idx] = v
                    return
                step = 0  # the value is not published yet: read this slot again
            elif cur == EMPTY:
                if op != 0:
                    out[idx] = ABSENT if op == 1 else 0
                    return
                yield
                h = self.mem.hist[("k", p)]
                old = h[-1]
                if L.cas(("k", p), EMPTY, key):
                    yield
                    L.st(("v", p), val)
                    out[idx] = 1
                    return
                if old == key:
                    out[idx] = 0
                    return
            p = (p + step) % self.n
            n += step
        out[idx] = -4 if op == 0 else (ABSENT if op == 1 else 0)

    def batch(self, ops, keys, vals, rng):
        out = [None] * len(ops)
        lanes = [self.op(Lane(self.mem, rng), o, k, v, out, i) for i, (o, k, v) in enumerate(zip(ops, keys, vals))]
        live = list(range(len(lanes)))
        while live:
            j = rng.choice(live)
            try:
                next(lanes[j])
            except StopIteration:
                live.remove(j)
        self.mem.settle()
        return out

    def contents(self):
        got = {}
        for i in range(self.n):
            k = self.mem.latest(("k", i))
            if k >= 0:
                assert k not in got, "key in two slots"
                v = self.mem.latest(("v", i))
                assert v != PENDING
                got[k] = v
        return got


@pytest.mark.parametrize("seed", range(60))
def test_random_interleavings_are_linearizable(seed):
    rng = random.Random(1000 + seed)
    m = OpenModel(512)  # room for every key and its tombstones over the run
    state = {}
    for _ in range(25):
        keys_pool = rng.sample(range(1, 40), 5)
        ops, keys, vals = [], [], []
        for k in keys_pool:
            for _ in range(rng.randint(1, 3)):
                ops.append(rng.randint(0, 2))
                keys.append(k)
                vals.append(1000 + k)
        order = list(range(len(ops)))
        rng.shuffle(order)
        ops, keys, vals = [ops[i] for i in order], [keys[i] for i in order], [vals[i] for i in order]
        out = m.batch(ops, keys, vals, rng)
        got = m.contents()
        assert all(o is not None and o != -4 for o in out), out
        for k in keys_pool:
            sel = [i for i, kk in enumerate(keys) if kk == k]
            assert serial_ok([ops[i] for i in sel], [out[i] for i in sel], [vals[i] for i in sel],
                             k in state, state.get(k)), (k, [(ops[i], out[i]) for i in sel])
            state.pop(k, None)
            if k in got:
                state[k] = got[k]
        assert got == state
