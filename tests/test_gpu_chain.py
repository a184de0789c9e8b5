"""GPU parity of the paper's chained hash map design (Sec. 5: buckets, linked-list excess
entries, free-entry stack, occupancy flags and locks) behind the same C ABI as the
open-addressing map: against the oracle, per-key linearizability under heavy
contention on long chains, set algebra at full size, capacity, and the open map as a
second implementation run on the same batches."""
import numpy as np
import pytest
import torch

import datagen
from gpu_util import keyset, require_gpu, say, sort_keys, to_dev
from test_gpu_hash import ABSENT, linearizable

pytestmark = pytest.mark.gpu
KINDS = [0, 1]


def spatial_bucket(keys, nb):
    k = keys.astype(np.int64) & 0xFFFFFFFF
    h = ((k[:, 0] * 73856093) & 0xFFFFFFFF) ^ ((k[:, 1] * 19349669) & 0xFFFFFFFF) ^ ((k[:, 2] * 83492791) & 0xFFFFFFFF)
    return h & (nb - 1)


@pytest.mark.parametrize("kind", KINDS)
@pytest.mark.parametrize("seed", range(3))
def test_chained_small_mixed_batches_vs_oracle(orc, kind, seed):
    vbh = require_gpu()
    say(f"[chain small] kind={kind} seed={seed}")
    keys, vals = datagen.bulk_keys(seed=seed, n_unique=3000, lo=-40, hi=40)
    present = np.unique(datagen.pack_key(keys))
    m, o = vbh.ChainedMap(1 << 11, 1 << 12, kind), orc.Map()
    st = m.vbh_insert(to_dev(keys), to_dev(vals)).cpu().numpy()
    ost, _ = o.insert(keys, vals)
    assert st.sum() == ost.sum() == present.size
    pk = datagen.pack_key(keys)
    for key in np.unique(pk)[:200]:
        assert st[pk == key].sum() == 1
    assert np.array_equal(m.vbh_find(to_dev(keys)).cpu().numpy(), o.find(keys))
    for ops, k, v in datagen.mixed_batches(present, seed=seed, n_batches=4, batch=4096, lo=-40, hi=40):
        out = m.vbh_apply(to_dev(ops), to_dev(k), to_dev(v)).cpu().numpy()
        oout, _ = o.apply(ops, k, v)
        f = ops == 1
        assert np.array_equal(out[f], oout[f])
        for kind_ in (0, 2):
            assert out[ops == kind_].sum() == oout[ops == kind_].sum()
        gk, gv = m.vbh_map_export()
        ok, ov = o.export()
        gks, order = sort_keys(gk.cpu().numpy())
        assert np.array_equal(gks, ok) and np.array_equal(gv.cpu().numpy()[order], ov)
    assert m.vbh_map_status() == 0
    assert m.vbh_map_size() == (o.size(), 0)


@pytest.mark.parametrize("kind", KINDS)
def test_chained_adversarial_long_chains(kind):
    """64 buckets for up to 729 keys: chains of ~10 entries, every op of a batch on one of
    32 keys, 5 ops per key, all concurrent."""
    vbh = require_gpu()
    m = vbh.ChainedMap(64, 4096, kind)
    state = {}
    for seed in range(40):
        say(f"[chain adversarial] kind={kind} seed={seed}")
        ops, keys, vals = datagen.adversarial_batch(seed, n_keys=32, ops_per_key=5, lo=-4, hi=4)
        out = m.vbh_apply(to_dev(ops), to_dev(keys), to_dev(vals)).cpu().numpy()
        assert m.vbh_map_status() == 0
        pk = datagen.pack_key(keys)
        gk, gv = m.vbh_map_export()
        final = {tuple(k): int(v) for k, v in zip(gk.cpu().numpy(), gv.cpu().numpy())}
        assert len(final) == gk.shape[0], "duplicate key in the table"
        for key in np.unique(pk):
            sel = np.flatnonzero(pk == key)
            k3 = tuple(keys[sel[0]])
            ok, pres = linearizable(ops[sel], out[sel], vals[sel], k3 in state, state.get(k3))
            assert ok, (k3, ops[sel], out[sel])
            assert pres == (k3 in final)
            state.pop(k3, None)
            if k3 in final:
                state[k3] = final[k3]
        # keys not touched by the batch are unchanged
        assert {k: v for k, v in final.items() if k not in set(map(tuple, keys))} == \
            {k: v for k, v in state.items() if k not in set(map(tuple, keys))}
    # fill the remaining key range into the long chains, then look everything up
    allk = np.stack(np.meshgrid(*[np.arange(-4, 5)] * 3, indexing="ij"), -1).reshape(-1, 3).astype(np.int32)
    st = m.vbh_insert(to_dev(allk), to_dev(datagen.value_of(allk))).cpu().numpy()
    assert st.sum() == allk.shape[0] - len(state) and m.vbh_map_status() == 0
    got = m.vbh_find(to_dev(allk)).cpu().numpy()
    want = np.array([state.get(tuple(k), v) for k, v in zip(allk, datagen.value_of(allk))])
    assert np.array_equal(got, want)
    assert m.vbh_map_size() == (allk.shape[0], 0)


def test_chained_full_size_bulk_and_mixed():
    """2^24 keys (2^23 unique) into 2^24 buckets + 2^24 excess entries (the memory of the
    2^25-slot open map), then 16 mixed 1M-op batches; set algebra at full size, the
    oracle on a sample of keys."""
    vbh = require_gpu()
    import oracle
    say("[chain full] generating")
    keys, vals = datagen.bulk_keys()
    m = vbh.ChainedMap(1 << 24, 1 << 24, 0)
    dk, dv = to_dev(keys), to_dev(vals)
    st = m.vbh_insert(dk, dv)
    pk = datagen.pack_key(keys)
    uniq = np.unique(pk)
    assert int(st.sum()) == uniq.size == 1 << 23
    assert torch.equal(m.vbh_find(dk).cpu(), torch.as_tensor(vals))
    assert m.vbh_map_size() == (uniq.size, 0)
    o = oracle.Map()
    rng = np.random.default_rng(1)
    sample_keys = keys[rng.choice(keys.shape[0], 50000, replace=False)]
    o.insert(sample_keys, datagen.value_of(sample_keys))
    present = uniq
    for b, (ops, k, v) in enumerate(datagen.mixed_batches(present)):
        say(f"[chain full] batch={b}")
        out = m.vbh_apply(to_dev(ops), to_dev(k), to_dev(v)).cpu().numpy()
        p = datagen.pack_key(k)
        ins, er, fnd = ops == 0, ops == 2, ops == 1
        was = np.isin(p, present)
        assert np.array_equal(out[fnd], np.where(was[fnd], v[fnd], ABSENT))
        assert out[ins].sum() == np.unique(p[ins & ~was]).size
        assert out[er].sum() == np.unique(p[er]).size
        osel = np.isin(p, datagen.pack_key(sample_keys))
        oout, _ = o.apply(ops[osel], k[osel], v[osel])
        fsel = ops[osel] == 1
        assert np.array_equal(out[osel][fsel], oout[fsel])
        present = np.setdiff1d(np.union1d(present, p[ins]), p[er])
    gk, _ = m.vbh_map_export()
    assert np.array_equal(np.sort(datagen.pack_key(gk.cpu().numpy())), present)
    assert m.vbh_map_size() == (present.size, 0)
    assert m.vbh_map_status() == 0


def test_chained_capacity_and_reuse():
    """A key needs its bucket or a free excess entry; entries emptied by a batch are free
    again from the next batch on."""
    vbh = require_gpu()
    nb, nx = 64, 16
    m = vbh.ChainedMap(nb, nx, 0)
    keys = np.stack(np.meshgrid(np.arange(5), np.arange(5), np.arange(4), indexing="ij"), -1).reshape(-1, 3)
    keys = keys.astype(np.int32)
    used = np.unique(spatial_bucket(keys, nb)).size
    st = m.vbh_insert(to_dev(keys), to_dev(np.arange(100, dtype=np.int32))).cpu().numpy()
    fits = used + min(nx, keys.shape[0] - used)
    assert (st == 1).sum() == fits and (st == -4).sum() == keys.shape[0] - fits
    assert m.vbh_map_status() == vbh.binding.VBH_EFULL_TABLE
    assert m.vbh_map_status() == 0
    stored = keys[st == 1]
    assert keyset(m.vbh_map_export()[0]) == keyset(stored)
    # erase every stored key, then insert the keys that failed: all fit now
    er = m.vbh_erase(to_dev(stored)).cpu().numpy()
    assert (er == 1).all() and m.vbh_map_size() == (0, 0)
    rest = keys[st != 1]
    st2 = m.vbh_insert(to_dev(rest), to_dev(np.arange(rest.shape[0], dtype=np.int32))).cpu().numpy()
    assert (st2 == 1).all() and m.vbh_map_status() == 0
    assert np.array_equal(m.vbh_find(to_dev(rest)).cpu().numpy(), np.arange(rest.shape[0]))
    m.vbh_map_clear()
    bad = np.array([[1 << 20, 0, 0], [0, -(1 << 20) - 1, 0]], np.int32)
    assert (m.vbh_insert(to_dev(bad), to_dev(np.array([1, 2], np.int32))).cpu().numpy() == -1).all()
    assert m.vbh_map_status() == vbh.binding.VBH_EINVAL
    assert (m.vbh_find(to_dev(bad)).cpu().numpy() == ABSENT).all()
    m.vbh_map_status()
    assert m.vbh_map_size() == (0, 0)
    # no excess entries at all: a key needs its bucket
    z = vbh.ChainedMap(nb, 0, 0)
    stz = z.vbh_insert(to_dev(keys), to_dev(np.arange(100, dtype=np.int32))).cpu().numpy()
    assert (stz == 1).sum() == used and z.vbh_map_status() == vbh.binding.VBH_EFULL_TABLE
    assert (z.vbh_erase(to_dev(keys[stz == 1])).cpu().numpy() == 1).all() and z.vbh_map_size() == (0, 0)
    stz2 = z.vbh_insert(to_dev(keys[::-1].copy()), to_dev(np.arange(100, dtype=np.int32))).cpu().numpy()
    assert (stz2 == 1).sum() == used
    z.vbh_map_status()
    with pytest.raises(vbh.VbhError):
        vbh.ChainedMap(96, 16, 0)  # buckets not a power of two
    with pytest.raises(vbh.VbhError):
        vbh.ChainedMap(64, 1 << 28, 0)  # links hold 28 bits


@pytest.mark.parametrize("kind", KINDS)
def test_chained_equals_open_addressing(kind):
    """The two designs give the same results on the same batches (up to which duplicate
    insert of a batch wins, where both report one success per key)."""
    vbh = require_gpu()
    keys, vals = datagen.bulk_keys(seed=11, n_unique=400_000, lo=-200, hi=200)
    a, b = vbh.Map(1 << 20, kind), vbh.ChainedMap(1 << 19, 1 << 19, kind)
    dk, dv = to_dev(keys), to_dev(vals)
    sa, sb = a.vbh_insert(dk, dv), b.vbh_insert(dk, dv)
    pk = datagen.pack_key(keys)
    assert int(sa.sum()) == int(sb.sum()) == np.unique(pk).size
    present = np.unique(pk)
    for i, (ops, k, v) in enumerate(datagen.mixed_batches(present, seed=12, n_batches=6, batch=1 << 18,
                                                          lo=-200, hi=200)):
        say(f"[chain vs open] kind={kind} batch={i}")
        oa = a.vbh_apply(to_dev(ops), to_dev(k), to_dev(v)).cpu().numpy()
        ob = b.vbh_apply(to_dev(ops), to_dev(k), to_dev(v)).cpu().numpy()
        f = ops == 1
        assert np.array_equal(oa[f], ob[f])
        for kind_ in (0, 2):
            assert oa[ops == kind_].sum() == ob[ops == kind_].sum()
    ka, va = a.vbh_map_export()
    kb, vb = b.vbh_map_export()
    sa_, oa_ = sort_keys(ka.cpu().numpy())
    sb_, ob_ = sort_keys(kb.cpu().numpy())
    assert np.array_equal(sa_, sb_) and np.array_equal(va.cpu().numpy()[oa_], vb.cpu().numpy()[ob_])
    assert a.vbh_map_status() == 0 and b.vbh_map_status() == 0


def test_chained_churn_reuses_entries_without_duplicates():
    """Many batches of inserts (with repeats), finds and erases over a small table, so that
    list entries emptied by one batch are reused by the next while other lanes walk the
    same lists: after every batch the key set equals the set algebra, with no duplicate."""
    vbh = require_gpu()
    m = vbh.ChainedMap(256, 1 << 13, 0)
    keys, vals = datagen.bulk_keys(seed=21, n_unique=6000, lo=-14, hi=14)
    m.vbh_insert(to_dev(keys), to_dev(vals))
    present = np.unique(datagen.pack_key(keys))
    for b, (ops, k, v) in enumerate(datagen.mixed_batches(present, seed=22, n_batches=30, batch=2048,
                                                          lo=-14, hi=14)):
        out = m.vbh_apply(to_dev(ops), to_dev(k), to_dev(v)).cpu().numpy()
        p = datagen.pack_key(k)
        ins, er, fnd = ops == 0, ops == 2, ops == 1
        was = np.isin(p, present)
        assert np.array_equal(out[fnd], np.where(was[fnd], v[fnd], ABSENT)), b
        assert out[ins].sum() == np.unique(p[ins & ~was]).size, b
        assert out[er].sum() == np.unique(p[er]).size, b
        present = np.setdiff1d(np.union1d(present, p[ins]), p[er])
        gk, _ = m.vbh_map_export()
        got = np.sort(datagen.pack_key(gk.cpu().numpy()))
        assert np.array_equal(got, present), b
    say(f"[chain churn] 30 batches, {present.size} keys at the end")
    assert m.vbh_map_status() == 0
