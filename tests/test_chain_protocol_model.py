"""Model check, on the CPU, of the chained hash map's concurrency protocol (the paper's
Sec. 5 design as built for gfx950): the steps of one device lane are replayed as a
Python generator that yields at every memory access, and a random scheduler
interleaves the lanes of a batch.

Memory model: every 64-bit word is coherent on its own (a compare-and-swap sees and
extends the latest value, and a lane never reads a value older than one it already
saw), but a plain load may return any value the word has held since the batch began,
not yet superseded in the lane's view - so a lane may see a new link word together
with an old key word, as on hardware without ordering fences.  Kernel boundaries (batch
start and the after-batch pass) make everything visible.

Checked for every batch of random same-key operations: the per-key outcome equals some
serial order of that key's operations, keys stay unique, and every excess entry is
either in exactly one list or on the free stack.
"""
import itertools
import random

import pytest

ABSENT = -(1 << 31)
LOCK, OCC, LIFE_B, DEAD = 1 << 63, 1 << 62, 1 << 61, 1 << 60
LINK_SHIFT, LINK_MASK = 32, (1 << 28) - 1
KEY_BITS = (1 << 63) - 1


def link_of(b):
    return (b >> LINK_SHIFT) & LINK_MASK


def with_link(b, e):
    return (b & ~(LINK_MASK << LINK_SHIFT)) | (e << LINK_SHIFT)


def life_b(b):
    return (b >> 61) & 1


def life_a(a):
    return a >> 63


class Memory:
    def __init__(self, words):
        self.hist = {w: [v] for w, v in words.items()}

    def settle(self):  # kernel boundary
        for w, h in self.hist.items():
            self.hist[w] = [h[-1]]

    def latest(self, w):
        return self.hist[w][-1]


class Lane:
    def __init__(self, mem, rng):
        self.mem, self.rng, self.seen = mem, rng, {}

    def ld(self, w):
        h = self.mem.hist[w]
        lo = self.seen.get(w, 0)
        i = self.rng.randint(lo, len(h) - 1)
        self.seen[w] = i
        return h[i]

    def st(self, w, v):
        self.mem.hist[w].append(v)
        self.seen[w] = len(self.mem.hist[w]) - 1

    def cas(self, w, expect, new):
        h = self.mem.hist[w]
        self.seen[w] = len(h) - 1
        if h[-1] != expect:
            return False
        h.append(new)
        self.seen[w] = len(h) - 1
        return True


class Model:
    def __init__(self, nb, nx):
        self.nb, self.nx, self.total = nb, nx, nb + nx
        words = {}
        for i in range(self.total):
            words[("a", i)] = 0
            words[("b", i)] = 0
        self.mem = Memory(words)
        self.stack = [nb + nx - 1 - j for j in range(nx)]  # pops take from the end
        self.top = nx

    def bucket(self, key):
        return (key * 2654435761) % self.nb

    # ------------------------------------------------------------ one lane's steps
    def walk(self, L, bucket, key):
        i, prev, prev_b = bucket, -1, 0
        b = yield from self.load(L, ("b", bucket))
        a = yield from self.load(L, ("a", bucket))
        bucket_b = b
        for _ in range(self.total):
            if b & OCC:
                if life_a(a) != life_b(b):
                    return dict(again=True)
                if (a & KEY_BITS) == key:
                    return dict(again=False, hit=i, hit_b=b, prev=prev, prev_b=prev_b, bucket_b=bucket_b)
            n = link_of(b)
            if n == 0:
                return dict(again=False, hit=-1, last=i, last_b=b, bucket_b=bucket_b)
            assert n < self.total
            prev, prev_b, i = i, b, n
            b = yield from self.load(L, ("b", i))
            a = yield from self.load(L, ("a", i))
        raise AssertionError("walk longer than the entry array")

    def load(self, L, w):
        yield
        return L.ld(w)

    def lane(self, L, op, key, val, out, idx, pops, retired):
        bucket = self.bucket(key)
        for _ in range(100000):
            w = yield from self.walk(L, bucket, key)
            if w["again"]:
                continue
            if op == 1:
                out[idx] = (w["hit_b"] & 0xFFFFFFFF) if w["hit"] >= 0 else ABSENT
                return
            if op == 0:
                bb = w["bucket_b"]
                if w["hit"] >= 0:
                    out[idx] = 0
                    return
                if not (bb & (OCC | DEAD)):
                    yield
                    if not (bb & LOCK) and L.cas(("b", bucket), bb, bb | LOCK):
                        life = life_b(bb) ^ 1
                        yield
                        L.st(("a", bucket), key | (life << 63))
                        yield
                        L.st(("b", bucket), (bb & (LINK_MASK << LINK_SHIFT)) | OCC | (life << 61) | val)
                        out[idx] = 1
                        return
                    continue
                last, lb = w["last"], w["last_b"]
                if not (lb & LOCK) and (last == bucket or (lb & OCC)):
                    yield
                    if L.cas(("b", last), lb, lb | LOCK):
                        yield  # the pop (one counter for the batch)
                        slot = pops[0]
                        pops[0] += 1
                        if slot < self.top:
                            e = self.stack[self.top - 1 - slot]
                            eb = yield from self.load(L, ("b", e))
                            life = life_b(eb) ^ 1
                            yield
                            L.st(("a", e), key | (life << 63))
                            yield
                            L.st(("b", e), OCC | (life << 61) | val)
                            yield
                            L.st(("b", last), with_link(lb, e))
                            out[idx] = 1
                        else:
                            yield
                            L.st(("b", last), lb)
                            out[idx] = -4
                        return
                continue
            # erase
            if w["hit"] < 0:
                out[idx] = 0
                return
            c, cb = w["hit"], w["hit_b"]
            if cb & LOCK:
                continue
            if w["prev"] < 0:
                yield
                if L.cas(("b", bucket), cb, (cb & ~OCC) | DEAD):
                    retired.append(bucket)
                    out[idx] = 1
                    return
                continue
            p, pb = w["prev"], w["prev_b"]
            if (pb & LOCK) or not (p == bucket or (pb & OCC)):
                continue
            yield
            if not L.cas(("b", p), pb, pb | LOCK):
                continue
            yield
            if not L.cas(("b", c), cb, cb | LOCK):
                yield
                L.st(("b", p), pb)
                continue
            yield
            L.st(("b", c), cb & ~OCC)
            yield
            L.st(("b", p), with_link(pb, link_of(cb)))
            retired.append(c)
            out[idx] = 1
            return
        raise AssertionError("lane did not finish")

    # ------------------------------------------------------------ batch
    def batch(self, ops, keys, vals, rng):
        out = [None] * len(ops)
        pops, retired = [0], []
        lanes = [self.lane(Lane(self.mem, rng), o, k, v, out, i, pops, retired)
                 for i, (o, k, v) in enumerate(zip(ops, keys, vals))]
        live = list(range(len(lanes)))
        while live:
            j = rng.choice(live)
            try:
                next(lanes[j])
            except StopIteration:
                live.remove(j)
        self.mem.settle()
        # after-batch pass: dead buckets usable again, emptied list entries back on the stack
        used = min(pops[0], self.top)
        base = self.top - used
        xs = [e for e in retired if e >= self.nb]
        assert len(set(retired)) == len(retired), "an entry was emptied twice in one batch"
        for e in retired:
            w = ("b", e)
            v = self.mem.latest(w)
            self.mem.hist[w] = [v & ~DEAD if e < self.nb else v & ~(LINK_MASK << LINK_SHIFT)]
        del self.stack[base:]
        self.stack.extend(xs)
        self.top = len(self.stack)
        return out

    def contents(self):
        got, in_list = {}, set()
        for bkt in range(self.nb):
            i, steps = bkt, 0
            while True:
                b, a = self.mem.latest(("b", i)), self.mem.latest(("a", i))
                if b & OCC:
                    assert life_a(a) == life_b(b)
                    k = a & KEY_BITS
                    assert k not in got, "duplicate key"
                    got[k] = b & 0xFFFFFFFF
                if i >= self.nb:
                    assert i not in in_list, "entry in two lists"
                    in_list.add(i)
                    assert b & OCC, "an emptied entry is still linked after the batch"
                n = link_of(b)
                if n == 0:
                    break
                i, steps = n, steps + 1
                assert steps <= self.total
        free = set(self.stack)
        assert len(free) == len(self.stack), "an entry is on the stack twice"
        assert not (free & in_list), "a linked entry is on the free stack"
        assert free | in_list == set(range(self.nb, self.total)), "an excess entry was lost"
        return got


def serial_ok(ops, outs, vals, present0, stored0):
    for perm in itertools.permutations(range(len(ops))):
        present, stored, ok = present0, stored0, True
        for i in perm:
            if ops[i] == 0:
                want = 0 if present else 1
                if not present:
                    present, stored = True, vals[i]
            elif ops[i] == 1:
                want = stored if present else ABSENT
            else:
                want = 1 if present else 0
                present = False
            if outs[i] != want:
                ok = False
                break
        if ok:
            return True
    return False


@pytest.mark.parametrize("seed", range(60))
def test_random_interleavings_are_linearizable(seed):
    rng = random.Random(seed)
    m = Model(nb=4, nx=64)  # 4 buckets: long lists, much contention; room for all 39 keys
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
        assert all(o is not None and o != -4 for o in out), out  # there is room for every key
        for k in keys_pool:
            sel = [i for i, kk in enumerate(keys) if kk == k]
            assert serial_ok([ops[i] for i in sel], [out[i] for i in sel], [vals[i] for i in sel],
                             k in state, state.get(k)), (k, [(ops[i], out[i]) for i in sel])
            state.pop(k, None)
            if k in got:
                state[k] = got[k]
        assert got == state
