"""Pins of the oracle's serving replay: per-client stream sets (Sec. 4.2).

What fixes the stream sets independently of their code:
- a (re)connecting client is owed every block of the model (Sec. 4.2, 4.3);
- a client that keeps the MC voxels it receives and finally drains its set holds exactly
  the server's current model: no update is lost (the guarantee the stream sets exist for);
- a hash set holds a block once, so between two updates no block is sent twice;
- the update log with per-client cursors (the other formulation, c5) yields answers that
  the stream sets accept, request after request;
- an answer of the wrong size, with a duplicate, with a block not owed, or that leaves an
  older update behind a newer one, is rejected.
Planted mistakes in the oracle's source each fail one of these.
"""
import numpy as np
import pytest

import oracle
from datagen import configs
from oracle_variant import build_variant

N_FRAMES = 8


@pytest.fixture(scope="module")
def frames():
    _, depth, rgb, poses = configs.tiny_inputs(N_FRAMES)
    return depth.numpy(), rgb.numpy(), poses


def keyset(k):
    return set(map(tuple, np.asarray(k).reshape(-1, 3).tolist()))


def fuse(O, frames, f):
    depth, rgb, poses = frames
    assert O.integrate(depth[f], rgb[f], poses[f], f + 1) == 0


def pin_reconnect(L, frames):
    O = oracle.Scene(configs.TINY_VOL, configs.TINY_CAM, L=L)
    for f in range(3):
        fuse(O, frames, f)
    T = oracle.Streams(O, 2)
    k, fr = T.pending(0)
    assert keyset(k) == keyset(O.blocks()) and k.shape[0] == O.n_blocks()
    # blocks of the last update carry its frame id; the others an earlier one
    last = keyset(O.last_mc_updated())
    for key, f in zip(map(tuple, k.tolist()), fr.tolist()):
        assert (f == 3) == (key in last) and 1 <= f <= 3
    # an outage: served half, then reconnected - owed everything again
    T.serve(1, k.shape[0] // 2)
    T.reconnect(1)
    assert keyset(T.pending(1)[0]) == keyset(O.blocks())


def pin_client_model(L, frames, seed=0):
    """Clients keep what they receive; after a final drain each holds the current model."""
    O = oracle.Scene(configs.TINY_VOL, configs.TINY_CAM, L=L)
    fuse(O, frames, 0)
    T = oracle.Streams(O, 3)
    rng = np.random.default_rng(seed)
    model = [dict() for _ in range(3)]
    for f in range(1, N_FRAMES):
        sent_this_version = [set() for _ in range(3)]
        for _ in range(4):
            c = int(rng.integers(3))
            keys = T.serve(c, int(rng.integers(0, 400)))
            got = keyset(keys)
            assert len(got) == keys.shape[0], "a block sent twice in one answer"
            assert not (got & sent_this_version[c]), "a block sent twice between two updates"
            sent_this_version[c] |= got
            if keys.shape[0]:
                mc, rgb = O.stored_mc(keys)
                for key, m, r in zip(map(tuple, keys.tolist()), mc, rgb):
                    model[c][key] = (m.copy(), r.copy())
        fuse(O, frames, f)
        T.sync()
    every = O.blocks()
    cur_mc, cur_rgb = O.stored_mc(every)
    for c in range(3):
        keys = T.serve(c, 1 << 30)
        if keys.shape[0]:
            mc, rgb = O.stored_mc(keys)
            for key, m, r in zip(map(tuple, keys.tolist()), mc, rgb):
                model[c][key] = (m, r)
        assert set(model[c]) == keyset(every), f"client {c} misses blocks"
        for i, key in enumerate(map(tuple, every.tolist())):
            m, r = model[c][key]
            assert np.array_equal(m, cur_mc[i]) and np.array_equal(r, cur_rgb[i]), f"client {c} holds a stale block"


def pin_log_formulation(L, frames, seed=1):
    """Pages of the update log walked from per-client cursors are accepted answers."""
    O = oracle.Scene(configs.TINY_VOL, configs.TINY_CAM, L=L)
    fuse(O, frames, 0)
    T = oracle.Streams(O, 2)
    cursor = [0, 0]
    rng = np.random.default_rng(seed)
    n_checked = 0
    for f in range(1, N_FRAMES):
        for _ in range(6):
            c = int(rng.integers(2))
            limit = int(rng.integers(0, 300))
            keys, cursor[c] = O.updated_since(cursor[c], limit)
            assert T.take(c, limit, keys) == 0, "log page rejected by the stream sets"
            n_checked += 1
        fuse(O, frames, f)
        T.sync()
    for c in range(2):
        keys, cursor[c] = O.updated_since(cursor[c], 1 << 30)
        assert T.take(c, 1 << 30, keys) == 0
        assert T.pending(c)[0].shape[0] == 0
    assert n_checked >= 30


def test_reconnect_owes_every_block(frames):
    pin_reconnect(oracle.lib(), frames)


def test_clients_end_with_the_current_model(frames):
    pin_client_model(oracle.lib(), frames)


def test_log_pages_are_valid_answers(frames):
    pin_log_formulation(oracle.lib(), frames)


def test_take_rejects_invalid_answers(frames):
    O = oracle.Scene(configs.TINY_VOL, configs.TINY_CAM)
    fuse(O, frames, 0)
    T = oracle.Streams(O, 1)
    fuse(O, frames, 1)
    T.sync()
    k, fr = T.pending(0)
    old, new = k[fr == 1], k[fr == 2]
    assert old.shape[0] > 10 and new.shape[0] > 10
    n_before = k.shape[0]
    assert T.take(0, 5, old[:4]) == oracle.SERVE_ECOUNT
    assert T.take(0, 5, np.concatenate([old[:4], old[:1]])) == oracle.SERVE_EDUP
    assert T.take(0, 1, np.array([[900, 900, 900]], np.int32)) == oracle.SERVE_ENOTPENDING
    # a newer update sent while an older one stays behind
    assert T.take(0, 3, np.concatenate([old[:2], new[:1]])) == oracle.SERVE_EORDER
    assert T.pending(0)[0].shape[0] == n_before, "a rejected answer changed the set"
    # every older block plus any of the newest update's blocks is fine
    assert T.take(0, old.shape[0] + 3, np.concatenate([old, new[-3:]])) == 0
    assert T.pending(0)[0].shape[0] == n_before - old.shape[0] - 3
    # nothing owed: only the empty answer is right
    assert T.take(0, 1 << 20, T.pending(0)[0]) == 0
    assert T.take(0, 10, np.zeros((0, 3), np.int32)) == 0


PLANTED = {
    "sync feeds one client": ("for (auto &m : T.set) m[e.second] = e.first;  // newest update of the block",
                              "T.set[0][e.second] = e.first;"),
    "serve keeps what it sent": ("T.set[size_t(client)].erase(v[size_t(i)].second);", "(void)0;"),
    "sync keeps the older frame": ("for (auto &m : T.set) m[e.second] = e.first;  // newest update of the block",
                                   "for (auto &m : T.set) m.emplace(e.second, e.first);"),
}


@pytest.mark.parametrize("name", sorted(PLANTED))
def test_planted_stream_mistakes_are_caught(frames, name):
    L = build_variant("oracle.cpp", *PLANTED[name])
    failed = []
    for pin in (pin_reconnect, pin_client_model, pin_log_formulation):
        try:
            pin(L, frames)
        except AssertionError:
            failed.append(pin.__name__)
    assert failed, f"planted mistake '{name}' passed every pin"
