"""Seeded int3 key streams and operation batches for the concurrent hash map.

Keys are int3 block coordinates stored as int32 [n,3].  `pack_key` is the 63-bit
offset-binary packing ((x+2^20)<<42 | (y+2^20)<<21 | (z+2^20)) used only to draw
distinct keys and to derive values; the map implementations do their own packing.
"""
from __future__ import annotations

import numpy as np

OP_INSERT, OP_FIND, OP_ERASE = 0, 1, 2
_OFF = 1 << 20
_M21 = (1 << 21) - 1


def pack_key(k: np.ndarray) -> np.ndarray:
    k = np.asarray(k, np.int64)
    return (((k[..., 0] + _OFF) << 42) | ((k[..., 1] + _OFF) << 21) | (k[..., 2] + _OFF)).astype(np.uint64)


def unpack_key(p: np.ndarray) -> np.ndarray:
    p = np.asarray(p, np.uint64).astype(np.int64)
    return np.stack([((p >> 42) & _M21) - _OFF, ((p >> 21) & _M21) - _OFF, (p & _M21) - _OFF],
                    -1).astype(np.int32)


def fmix64(x: np.ndarray) -> np.ndarray:
    """MurmurHash3 64-bit finalizer (public domain, Austin Appleby)."""
    x = np.asarray(x, np.uint64).copy()
    with np.errstate(over="ignore"):
        x ^= x >> np.uint64(33)
        x *= np.uint64(0xFF51AFD7ED558CCD)
        x ^= x >> np.uint64(33)
        x *= np.uint64(0xC4CEB9FE1A85EC53)
        x ^= x >> np.uint64(33)
    return x


def value_of(keys: np.ndarray) -> np.ndarray:
    """Value attached to a key: (int32)(fmix64(packed) & 0x7FFFFFFF); never INT32_MIN."""
    return (fmix64(pack_key(keys)) & np.uint64(0x7FFFFFFF)).astype(np.int32)


def _distinct(rng, n: int, lo: int, hi: int, exclude=None) -> np.ndarray:
    """n distinct int3 keys uniform in [lo,hi)^3 (rejection against a set), in random
    order, avoiding the packed keys in `exclude`."""
    out = np.empty(0, np.uint64)
    while out.size < n:
        need = int((n - out.size) * 1.05) + 64
        cand = pack_key(rng.integers(lo, hi, size=(need, 3), dtype=np.int64))
        out = np.unique(np.concatenate([out, cand]))
        if exclude is not None and exclude.size:
            out = np.setdiff1d(out, exclude, assume_unique=False)
    sel = rng.permutation(out.size)[:n]
    return out[sel]


def bulk_keys(seed: int = 3709, n_unique: int = 1 << 23, lo: int = -1024, hi: int = 1024):
    """n_unique distinct keys, each duplicated once, shuffled: int32 [2n,3] keys and their
    int32 values."""
    rng = np.random.default_rng(seed)
    u = _distinct(rng, n_unique, lo, hi)
    allk = np.concatenate([u, u])
    allk = allk[rng.permutation(allk.size)]
    keys = unpack_key(allk)
    return keys, value_of(keys)


def mixed_batches(present: np.ndarray, seed: int = 3709, n_batches: int = 16,
                  batch: int = 1 << 20, lo: int = -1024, hi: int = 1024):
    """Mixed batches of 40 % insert / 40 % find / 20 % erase.

    present: packed uint64 keys in the map before the first batch.
    Inserts are half present keys and half new keys (new ones repeated within the
    batch); finds are half present, half absent; erases are present keys with some
    repeats.  The three kinds use pairwise disjoint keys inside one batch, so the final
    key set and every find result are independent of the order the ops run in.
    Yields (ops uint8 [n], keys int32 [n,3], vals int32 [n]) and tracks the present set.
    """
    rng = np.random.default_rng(seed + 1)
    present = np.unique(np.asarray(present, np.uint64))
    n_ins, n_find = int(batch * 0.4), int(batch * 0.4)
    n_er = batch - n_ins - n_find
    for _ in range(n_batches):
        perm = rng.permutation(present.size)
        n_ins_present = n_ins // 2
        n_find_present = n_find // 2
        n_er_unique = (n_er * 3) // 4
        a = 0
        ins_present = present[perm[a:a + n_ins_present]]; a += n_ins_present
        find_present = present[perm[a:a + n_find_present]]; a += n_find_present
        er_unique = present[perm[a:a + n_er_unique]]; a += n_er_unique
        er = np.concatenate([er_unique, er_unique[rng.integers(0, n_er_unique, n_er - n_er_unique)]])
        n_new_unique = (n_ins - n_ins_present) // 2
        fresh = _distinct(rng, n_new_unique + (n_find - n_find_present), lo, hi, exclude=present)
        new_unique = fresh[:n_new_unique]
        absent = fresh[n_new_unique:]
        ins_new = np.concatenate([new_unique, new_unique[rng.integers(0, n_new_unique,
                                                                      n_ins - n_ins_present - n_new_unique)]])
        ins = np.concatenate([ins_present, ins_new])
        fnd = np.concatenate([find_present, absent])
        ops = np.concatenate([np.full(ins.size, OP_INSERT, np.uint8),
                              np.full(fnd.size, OP_FIND, np.uint8),
                              np.full(er.size, OP_ERASE, np.uint8)])
        keys = np.concatenate([ins, fnd, er])
        order = rng.permutation(ops.size)
        ops, keys = ops[order], unpack_key(keys[order])
        yield ops, keys, value_of(keys)
        present = np.setdiff1d(np.union1d(present, new_unique), er_unique)


def adversarial_batch(seed: int, n_keys: int = 64, ops_per_key: int = 6, lo=-8, hi=8):
    """Same-key contention: each of n_keys keys gets ops_per_key random operations in
    one batch (interleaved).  Returns (ops, keys, vals)."""
    rng = np.random.default_rng(seed)
    u = _distinct(rng, n_keys, lo, hi)
    keys = np.repeat(u, ops_per_key)
    ops = rng.integers(0, 3, keys.size).astype(np.uint8)
    order = rng.permutation(keys.size)
    keys = unpack_key(keys[order])
    return ops[order], keys, value_of(keys)
