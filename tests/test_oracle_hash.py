"""Pins of the oracle's hash-map semantics (Sec. 5: retrieval, insertion, removal with
success guarantee and key uniqueness) against a Python dict and set invariants."""
import numpy as np
import pytest

import datagen

ABSENT = -(1 << 31)


def brute(ops, keys, vals, d):
    out = []
    for o, k, v in zip(ops, map(tuple, keys), vals):
        if o == 0:
            if k in d:
                out.append(0)
            else:
                d[k] = int(v)
                out.append(1)
        elif o == 1:
            out.append(d.get(k, ABSENT))
        else:
            out.append(1 if d.pop(k, None) is not None else 0)
    return np.array(out, np.int32)


@pytest.mark.parametrize("seed", range(5))
def test_apply_matches_dict(orc, seed):
    rng = np.random.default_rng(seed)
    m, d = orc.Map(), {}
    for _ in range(4):
        n = 500
        keys = rng.integers(-6, 6, size=(n, 3)).astype(np.int32)
        ops = rng.integers(0, 3, n).astype(np.uint8)
        vals = rng.integers(0, 1 << 30, n).astype(np.int32)
        out, rc = m.apply(ops, keys, vals)
        assert rc == 0
        assert np.array_equal(out, brute(ops, keys, vals, d))
        assert m.size() == len(d)
        k, v = m.export()
        assert {tuple(x): int(y) for x, y in zip(k, v)} == d


def test_invariants_bulk(orc):
    keys, vals = datagen.bulk_keys(seed=11, n_unique=1 << 14)
    m = orc.Map()
    st, rc = m.insert(keys, vals)
    assert rc == 0
    uniq = np.unique(datagen.pack_key(keys))
    # exactly one "inserted" per unique key, size = |unique keys|
    assert st.sum() == uniq.size and m.size() == uniq.size
    # inserted set equals found set, with the value of the first insert
    assert np.array_equal(m.find(keys), vals)
    ek, _ = m.export()
    assert np.array_equal(np.sort(datagen.pack_key(ek)), uniq)
    # erased keys are absent, others remain
    er = keys[: 1 << 12]
    est, _ = m.erase(er)
    assert est.sum() == np.unique(datagen.pack_key(er)).size
    assert (m.find(er) == ABSENT).all()
    assert m.size() == uniq.size - est.sum()


def test_insert_does_not_overwrite(orc):
    m = orc.Map()
    k = np.array([[4, -3, 2]], np.int32)
    assert m.insert(k, np.array([5], np.int32))[0][0] == 1
    assert m.insert(k, np.array([9], np.int32))[0][0] == 0
    assert m.find(k)[0] == 5


def test_key_range(orc):
    m = orc.Map()
    ok = np.array([[-(1 << 20), (1 << 20) - 1, 0]], np.int32)
    bad = np.array([[1 << 20, 0, 0]], np.int32)
    assert m.insert(ok, np.array([1], np.int32))[0][0] == 1
    st, rc = m.insert(bad, np.array([1], np.int32))
    assert st[0] == -1 and rc == -1
    assert m.find(ok)[0] == 1


def test_mixed_batch_result_is_order_free(orc):
    """Conflict-free batches: any serial order gives the same final set and finds."""
    keys, vals = datagen.bulk_keys(seed=5, n_unique=1 << 12)
    present = np.unique(datagen.pack_key(keys))
    m1, m2 = orc.Map(), orc.Map()
    m1.insert(keys, vals)
    m2.insert(keys, vals)
    rng = np.random.default_rng(0)
    for ops, k, v in datagen.mixed_batches(present, seed=5, n_batches=2, batch=1 << 11):
        o1, _ = m1.apply(ops, k, v)
        perm = rng.permutation(ops.size)
        o2p, _ = m2.apply(ops[perm], k[perm], v[perm])
        o2 = np.empty_like(o2p)
        o2[perm] = o2p
        find = ops == 1
        assert np.array_equal(o1[find], o2[find])
        for kind in (0, 2):
            assert o1[ops == kind].sum() == o2[ops == kind].sum()
        assert np.array_equal(m1.export()[0], m2.export()[0])
