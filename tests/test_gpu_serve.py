"""Serving loop: continuous batching of client requests for updated MC voxel blocks.

- alone == in the mix: every request of a mixed, overlapping run replayed alone (same
  cursor, limit and scene version) gives bit-identical keys, MC voxels, count and cursor;
- the selection equals vbh_updated_blocks_since and the MC voxels equal the MC pool;
- with frames fused concurrently, each result equals the expected page at the request's
  scene version, computed from the append-only update log;
- admission by memory, request-size errors, reconnection from cursor 0.
"""
import numpy as np
import pytest
import torch

from datagen import configs
from gpu_util import keyset, require_gpu, say

pytestmark = pytest.mark.gpu


def tiny_scene(vbh, n_frames):
    _, depth, rgb, poses = configs.tiny_inputs(32)
    S = vbh.Scene(vbh.make_params(configs.TINY_VOL, configs.TINY_CAM))
    for f in range(n_frames):
        S.vbh_integrate_frame(depth[f].cuda(), rgb[f].cuda(), poses[f], f + 1)
    assert S.vbh_scene_status() == 0
    return S, depth.cuda(), rgb.cuda(), poses


def out_buffers(limits):
    return [(torch.zeros((max(l, 1), 3), dtype=torch.int32, device="cuda"),
             torch.zeros((max(l, 1), 512), dtype=torch.int32, device="cuda")) for l in limits]


def log_uniform(rng, n, lo, hi):
    return np.floor(10 ** rng.uniform(np.log10(lo), np.log10(hi), n)).astype(np.int64)


def test_alone_equals_mix_static_scene():
    vbh = require_gpu()
    S, _, _, _ = tiny_scene(vbh, 32)
    nb = S.vbh_scene_stats()["n_blocks"]
    srv = vbh.Server(S, arena_bytes=256 << 20, max_inflight=32, n_streams=4, n_clients=8, max_batch=12)
    rng = np.random.default_rng(0)
    n = 64
    clients = np.arange(n) % 8
    limits = log_uniform(rng, n, 10, 3000)
    arrivals = np.sort(rng.uniform(0, 0.02, n))
    outs = out_buffers(limits)
    res = srv.vbh_server_run(clients, limits, arrivals, outs)
    assert (res["status"] == 0).all()
    say(f"[serve static] {nb} blocks, {n} requests, {res['count'].sum()} blocks served")
    # continuous batching: some request was admitted while an earlier one was in flight
    overl = [(i, j) for i in range(n) for j in range(n)
             if res["admit_s"][i] < res["admit_s"][j] < res["done_s"][i]]
    assert overl, "no overlap between requests"
    # per-client cursor chaining
    for c in range(8):
        idx = np.flatnonzero(clients == c)
        assert res["cursor_in"][idx[0]] == 0
        assert (res["cursor_in"][idx[1:]] == res["cursor_out"][idx[:-1]]).all()
    # alone replay, bit-exact
    for i in range(n):
        srv.vbh_server_set_cursor(int(clients[i]), int(res["cursor_in"][i]))
        o2 = out_buffers([limits[i]])
        r2 = srv.vbh_server_run([clients[i]], [limits[i]], [0.0], o2)
        k = int(res["count"][i])
        assert r2["count"][0] == k and r2["cursor_out"][0] == res["cursor_out"][i]
        assert torch.equal(o2[0][0][:k], outs[i][0][:k]) and torch.equal(o2[0][1][:k], outs[i][1][:k])
    # the same page as the scene's paged walk, and MC voxels from the MC pool
    for i in range(0, n, 5):
        k = int(res["count"][i])
        keys, meta = S.vbh_updated_blocks_since(int(res["cursor_in"][i]), int(limits[i]))
        assert int(meta[0]) == k and int(meta[1]) == res["cursor_out"][i]
        assert torch.equal(keys[:k], outs[i][0][:k])
        if k:
            mc, rgb = S.vbh_stored_mc(outs[i][0][:k].contiguous())
            packed = (mc.to(torch.int64) | rgb[..., 0].to(torch.int64) << 8 | rgb[..., 1].to(torch.int64) << 16
                      | rgb[..., 2].to(torch.int64) << 24)
            assert torch.equal(packed, outs[i][1][:k].to(torch.int64) & 0xFFFFFFFF)
    # reconnection: cursor 0 delivers every block
    srv.vbh_server_set_cursor(3, 0)
    o3 = out_buffers([nb + 10])
    r3 = srv.vbh_server_run([3], [nb + 10], [0.0], o3)
    assert r3["count"][0] == nb
    assert keyset(o3[0][0][:nb]) == keyset(S.vbh_scene_export_blocks())


def expected_pages(fr, keys, cursor, limit, version):
    """First `limit` entries at positions >= cursor of the log prefix of `version` that are
    the latest update of their block as of that version."""
    pk = (keys[:, 0].astype(np.int64) + (1 << 20)) << 42 | (keys[:, 1].astype(np.int64) + (1 << 20)) << 21 | \
        (keys[:, 2].astype(np.int64) + (1 << 20))
    n = pk.size
    order = np.lexsort((np.arange(n), pk))
    nxt = np.full(n, np.iinfo(np.int64).max)
    same = pk[order][1:] == pk[order][:-1]
    nxt[order[:-1][same]] = fr[order[1:][same]]
    end = int(np.searchsorted(fr, version, side="right"))
    pos = np.arange(cursor, end)
    live = (fr[pos] <= version) & (nxt[pos] > version)
    sel = pos[live][:limit]
    nxt_cursor = int(sel[-1] + 1) if (limit > 0 and sel.size == limit) else (cursor if limit == 0 else end)
    return sel, nxt_cursor, nxt


def test_concurrent_integration_versions():
    vbh = require_gpu()
    S, depth, rgb, poses = tiny_scene(vbh, 8)
    srv = vbh.Server(S, arena_bytes=512 << 20, max_inflight=64, n_streams=4, n_clients=8, max_batch=16)
    frames = [(depth[f].contiguous(), rgb[f].contiguous(), poses[f], 0.004 * (f - 7), f + 1) for f in range(8, 32)]
    rng = np.random.default_rng(1)
    n = 160
    clients = rng.integers(0, 8, n)
    limits = log_uniform(rng, n, 10, 2000)
    arrivals = np.sort(rng.uniform(0, 0.1, n))
    outs = out_buffers(limits)
    res = srv.vbh_server_run(clients, limits, arrivals, outs, frames=frames)
    assert (res["status"] == 0).all() and S.vbh_scene_status() == 0
    vers = np.unique(res["version"])
    say(f"[serve concurrent] versions served: {vers.tolist()}")
    assert vers.size >= 3, "requests were not spread over several scene versions"
    L = S.vbh_scene_stats()["log_length"]
    fr, keys = (t.cpu().numpy() for t in S.vbh_scene_log_entries(0, L))
    assert (np.diff(fr) >= 0).all()
    checked_mc = 0
    stored = {}
    for i in range(n):
        sel, nxt, nxt_frame = expected_pages(fr, keys, int(res["cursor_in"][i]), int(limits[i]),
                                             int(res["version"][i]))
        k = int(res["count"][i])
        assert k == sel.size and int(res["cursor_out"][i]) == nxt, i
        got = outs[i][0][:k].cpu().numpy()
        assert np.array_equal(got, keys[sel]), i
        # MC voxels of blocks not updated after the request's version equal today's MC pool
        final = nxt_frame[sel] == np.iinfo(np.int64).max
        if final.any():
            kk = torch.as_tensor(keys[sel][final]).cuda()
            mc, c3 = S.vbh_stored_mc(kk)
            packed = (mc.to(torch.int64) | c3[..., 0].to(torch.int64) << 8 | c3[..., 1].to(torch.int64) << 16
                      | c3[..., 2].to(torch.int64) << 24)
            assert torch.equal(packed, outs[i][1][:k][torch.as_tensor(final).cuda()].to(torch.int64) & 0xFFFFFFFF)
            checked_mc += int(final.sum())
    say(f"[serve concurrent] {n} requests checked against the log; MC voxels checked for {checked_mc} blocks")
    assert checked_mc > 1000


def test_admission_by_memory_and_errors():
    vbh = require_gpu()
    S, _, _, _ = tiny_scene(vbh, 16)
    per_req = 1000 * (4 + 12 + 2048) + 4096
    srv = vbh.Server(S, arena_bytes=int(2.5 * per_req), max_inflight=16, n_streams=4, n_clients=8, max_batch=8)
    n = 12
    clients = np.arange(n) % 8
    limits = np.full(n, 1000)
    limits[5] = 100_000  # larger than the whole arena: rejected, the rest proceed
    res = srv.vbh_server_run(clients, limits, np.zeros(n))
    assert res["status"][5] != 0 and (np.delete(res["status"], 5) == 0).all()
    ok = np.delete(np.arange(n), 5)
    # at most two results fit at once: no instant has three requests in flight
    ev = sorted([(res["admit_s"][i], 1) for i in ok] + [(res["done_s"][i], -1) for i in ok], key=lambda e: (e[0], e[1]))
    live, peak = 0, 0
    for _, d in ev:
        live += d
        peak = max(peak, live)
    assert peak <= 2
    assert (res["admit_s"][ok] > res["arrival_s"][ok]).sum() >= 1
