"""CPU model of the persistent serving launch's use of arena memory under per-XCD L2
caches, and of the write-back that ends each batch.

The device has several XCDs, each with its own write-back L2.  In the model:
- a plain store (the gather's keys and MC voxels) writes a dirty line into the storing
  XCD's cache;
- a device-scope store (counts, selected pool blocks, request results) goes through to
  memory, and a device-scope load reads memory;
- at any time an XCD may evict a dirty line, which writes it to memory;
- a write-back writes every dirty line of its XCD to memory.
The host hands each batch a range of a first-fit arena and takes it back when the batch
is complete, so a later batch's counts and selections may land where an earlier batch's
outputs were.  Checked over many seeds: with the write-back at the barrier that ends a
batch, every device-scope load returns what the batch itself stored; without it (the
planted mistake), a late eviction of an earlier batch's output overwrites a later batch's
counts or selections, which the later steps read as ranks and pool indices.
"""
import random

import pytest


class FirstFit:
    """First fit over word offsets, as the serving loop's arena hands out ranges."""

    def __init__(self, total):
        self.free = [(0, total)]

    def alloc(self, n):
        for i, (o, s) in enumerate(self.free):
            if s >= n:
                self.free[i] = (o + n, s - n)
                if s == n:
                    del self.free[i]
                return o
        return -1

    def release(self, off, n):
        self.free.append((off, n))
        self.free.sort()
        merged = []
        for o, s in self.free:
            if merged and merged[-1][0] + merged[-1][1] == o:
                merged[-1] = (merged[-1][0], merged[-1][1] + s)
            else:
                merged.append((o, s))
        self.free = merged


def run(seed, write_back, xcds=4, batches=40, evict_p=0.05):
    rng = random.Random(seed)
    mem = {}
    cache = [dict() for _ in range(xcds)]  # addr -> (value, dirty)
    arena = FirstFit(1 << 12)

    def maybe_evict():
        if rng.random() < evict_p:
            c = cache[rng.randrange(xcds)]
            dirty = [a for a, (_, d) in c.items() if d]
            if dirty:
                a = rng.choice(dirty)
                mem[a] = c[a][0]
                del c[a]

    def plain_store(x, a, v):
        cache[x][a] = (v, True)
        maybe_evict()

    def dev_store(x, a, v):
        mem[a] = v
        cache[x].pop(a, None)
        maybe_evict()

    def dev_load(a):
        maybe_evict()
        return mem.get(a)

    pending = []  # (batch, range) in flight
    for b in range(batches):
        limit = rng.randrange(1, 24)
        size = 2 * limit + limit * 4  # selections, counts, then outputs
        off = arena.alloc(size)
        while off < 0:  # the oldest batch completes first
            ob, (ooff, osize) = pending.pop(0)
            arena.release(ooff, osize)
            off = arena.alloc(size)
        sel, cnt, out = off, off + limit, off + 2 * limit
        # count and selection steps: device-scope stores from random workgroups' XCDs
        for i in range(limit):
            dev_store(rng.randrange(xcds), cnt + i, (b, "cnt", i))
            dev_store(rng.randrange(xcds), sel + i, (b, "sel", i))
        # gather: each wave reads its selection, then plain-stores the outputs
        for i in range(limit):
            x = rng.randrange(xcds)
            got = dev_load(sel + i)
            if got != (b, "sel", i):
                return f"batch {b} read selection {i} as {got}"
            if dev_load(cnt + i) != (b, "cnt", i):
                return f"batch {b} read count {i} as {dev_load(cnt + i)}"
            for k in range(4):
                plain_store(x, out + 4 * i + k, (b, "out", i, k))
        # the barrier that ends the batch
        if write_back:
            for c in cache:
                for a, (v, d) in list(c.items()):
                    if d:
                        mem[a] = v
                        c[a] = (v, False)
        pending.append((b, (off, size)))
        if rng.random() < 0.5:  # the host sees a completion and frees its range
            ob, (ooff, osize) = pending.pop(0)
            arena.release(ooff, osize)
    return None


@pytest.mark.parametrize("seed", range(40))
def test_write_back_keeps_reused_ranges_intact(seed):
    assert run(seed, write_back=True) is None


def test_missing_write_back_is_caught():
    failures = [run(seed, write_back=False) for seed in range(40)]
    assert any(f is not None for f in failures)
