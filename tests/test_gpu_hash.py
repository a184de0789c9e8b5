"""GPU parity of the concurrent hash map (Sec. 5) against the oracle and set algebra."""
import itertools

import numpy as np
import pytest
import torch

import datagen
from gpu_util import keyset, require_gpu, say, sort_keys, to_dev

pytestmark = pytest.mark.gpu
ABSENT = -(1 << 31)
KINDS = [0, 1]


@pytest.mark.parametrize("kind", KINDS)
@pytest.mark.parametrize("seed", range(3))
def test_small_mixed_batches_vs_oracle(orc, kind, seed):
    vbh = require_gpu()
    say(f"[hash small] kind={kind} seed={seed}")
    keys, vals = datagen.bulk_keys(seed=seed, n_unique=3000, lo=-40, hi=40)
    present = np.unique(datagen.pack_key(keys))
    m, o = vbh.Map(1 << 14, kind), orc.Map()
    st = m.vbh_insert(to_dev(keys), to_dev(vals)).cpu().numpy()
    ost, _ = o.insert(keys, vals)
    assert st.sum() == ost.sum() == present.size
    # one of each duplicate pair returns 1
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


def linearizable(ops, outs, vals, present0, stored0):
    """Brute force: some serial order of one key's ops yields these results."""
    idx = list(range(len(ops)))
    for perm in itertools.permutations(idx):
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
            return True, present
    return False, None


@pytest.mark.parametrize("kind", KINDS)
def test_adversarial_same_key_batches(kind):
    vbh = require_gpu()
    m = vbh.Map(1 << 14, kind)
    state = {}
    for seed in range(40):
        say(f"[hash adversarial] kind={kind} seed={seed}")
        ops, keys, vals = datagen.adversarial_batch(seed, n_keys=32, ops_per_key=5, lo=-4, hi=4)
        out = m.vbh_apply(to_dev(ops), to_dev(keys), to_dev(vals)).cpu().numpy()
        assert m.vbh_map_status() == 0
        pk = datagen.pack_key(keys)
        gk, gv = m.vbh_map_export()
        final = {tuple(k): int(v) for k, v in zip(gk.cpu().numpy(), gv.cpu().numpy())}
        for key in np.unique(pk):
            sel = np.flatnonzero(pk == key)
            k3 = tuple(keys[sel[0]])
            ok, pres = linearizable(ops[sel], out[sel], vals[sel], k3 in state, state.get(k3))
            assert ok, (k3, ops[sel], out[sel])
            assert pres == (k3 in final)
            state.pop(k3, None)
            if k3 in final:
                state[k3] = final[k3]
        if seed % 10 == 9:
            m.vbh_map_rebuild()
            assert {tuple(k) for k in m.vbh_map_export()[0].cpu().numpy()} == set(final)
    # keys stay unique: export has no duplicates
    gk, _ = m.vbh_map_export()
    assert len(keyset(gk)) == gk.shape[0]


@pytest.mark.parametrize("kind", [0, 1])
def test_full_size_bulk_and_mixed(kind):
    """2^24 keys (2^23 unique) into 2^25 slots, then 16 mixed 1M-op batches; checked by set
    algebra at full size and against the oracle on a sample of keys."""
    vbh = require_gpu()
    import oracle
    say(f"[hash full] kind={kind} generating")
    keys, vals = datagen.bulk_keys()
    m = vbh.Map(1 << 25, kind)
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
        say(f"[hash full] kind={kind} batch={b}")
        out = m.vbh_apply(to_dev(ops), to_dev(k), to_dev(v)).cpu().numpy()
        p = datagen.pack_key(k)
        ins, er, fnd = ops == 0, ops == 2, ops == 1
        was = np.isin(p, present)
        assert np.array_equal(out[fnd], np.where(was[fnd], v[fnd], ABSENT))
        assert out[ins].sum() == np.unique(p[ins & ~was]).size
        assert out[er].sum() == np.unique(p[er]).size
        # oracle on the sampled keys: apply the batch ops touching them, serially
        osel = np.isin(p, datagen.pack_key(sample_keys))
        oout, _ = o.apply(ops[osel], k[osel], v[osel])
        fsel = ops[osel] == 1
        assert np.array_equal(out[osel][fsel], oout[fsel])
        present = np.setdiff1d(np.union1d(present, p[ins]), p[er])
    gk, _ = m.vbh_map_export()
    assert np.array_equal(np.sort(datagen.pack_key(gk.cpu().numpy())), present)
    live, tomb = m.vbh_map_size()
    assert live == present.size and tomb > 0
    m.vbh_map_rebuild()
    assert m.vbh_map_size() == (present.size, 0)
    assert m.vbh_map_status() == 0


def test_errors_are_reported():
    vbh = require_gpu()
    m = vbh.Map(64, 0)
    keys = np.stack(np.meshgrid(np.arange(5), np.arange(5), np.arange(4), indexing="ij"), -1).reshape(-1, 3)
    keys = keys.astype(np.int32)
    st = m.vbh_insert(to_dev(keys), to_dev(np.arange(100, dtype=np.int32))).cpu().numpy()
    assert (st == 1).sum() == 64 and (st == -4).sum() == 36
    assert m.vbh_map_status() == vbh.binding.VBH_EFULL_TABLE
    assert m.vbh_map_status() == 0  # cleared
    m.vbh_map_clear()
    bad = np.array([[1 << 20, 0, 0], [0, -(1 << 20) - 1, 0]], np.int32)
    st = m.vbh_insert(to_dev(bad), to_dev(np.array([1, 2], np.int32))).cpu().numpy()
    assert (st == -1).all()
    assert m.vbh_map_status() == vbh.binding.VBH_EINVAL
    assert (m.vbh_find(to_dev(bad)).cpu().numpy() == ABSENT).all()
    m.vbh_map_status()
    assert m.vbh_map_size() == (0, 0)
    # the reserved value is refused at insert; the key stays absent and a find returns at once
    k = np.array([[3, 4, 5], [6, 7, 8]], np.int32)
    for mm in (m, vbh.ChainedMap(64, 64, 0)):
        st = mm.vbh_insert(to_dev(k), to_dev(np.array([ABSENT, 9], np.int32))).cpu().numpy()
        assert st.tolist() == [-1, 1]
        assert mm.vbh_map_status() == vbh.binding.VBH_EINVAL
        assert mm.vbh_find(to_dev(k)).cpu().numpy().tolist() == [ABSENT, 9]
        assert mm.vbh_map_status() == 0


def test_cas_ceiling_helper():
    """The measurement helper's compare-and-swaps land at the SplitMix64-chosen words: the
    successes equal the distinct words hit, and each hit word holds one of its operations."""
    vbh = require_gpu()
    n_words, n_ops, seed = 1 << 12, 3000, 99
    words = torch.zeros(n_words, dtype=torch.int64, device="cuda")
    won = torch.zeros(1, dtype=torch.int64, device="cuda")
    vbh.binding.vbh_cas_ceiling(words, n_ops, seed, won)
    torch.cuda.synchronize()
    M = (1 << 64) - 1
    hits = {}
    for i in range(n_ops):
        z = (seed + i * 0x9E3779B97F4A7C15) & M
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & M
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & M
        z ^= z >> 31
        hits.setdefault(z & (n_words - 1), set()).add(i + 1)
    w = words.cpu().numpy()
    assert int(won.item()) == len(hits)
    assert set(np.flatnonzero(w).tolist()) == set(hits)
    assert all(int(w[k]) in v for k, v in hits.items())
