"""Serving loop: continuous batching of client requests for updated MC voxel blocks.

- alone == in the mix: every request of a mixed, overlapping run replayed alone (same
  cursor, limit and scene version) gives bit-identical keys, MC voxels, count and cursor;
- the selection equals vbh_updated_blocks_since and the MC voxels equal the MC pool;
- with frames fused concurrently, each result equals the expected page at the request's
  scene version, computed from the append-only update log;
- admission by memory, request-size errors, reconnection from cursor 0;
- against the oracle's serving replay (per-client stream sets, Sec. 4.2): replayed in
  order of scene version, every answer is a valid answer of its client's stream set (its
  size, no block twice, only owed blocks, oldest updates first), and its MC voxels equal
  the oracle's at that version - bit-exact on an analytically written scene of 150k
  blocks with request sizes log-uniform up to 10^5, and on fused scenes wherever no cell
  corner has |F_oracle| <= 1e-5.
"""
import numpy as np
import pytest
import torch

from datagen import configs
import oracle
from gpu_util import corner_min_abs, keyset, pack_mc, require_gpu, say, to_dev

pytestmark = pytest.mark.gpu


def tiny_scene(vbh, n_frames, with_oracle=False):
    _, depth, rgb, poses = configs.tiny_inputs(32)
    S = vbh.Scene(vbh.make_params(configs.TINY_VOL, configs.TINY_CAM))
    O = oracle.Scene(configs.TINY_VOL, configs.TINY_CAM) if with_oracle else None
    for f in range(n_frames):
        S.vbh_integrate_frame(depth[f].cuda(), rgb[f].cuda(), poses[f], f + 1)
        if O is not None:
            assert O.integrate(depth[f].numpy(), rgb[f].numpy(), poses[f], f + 1) == 0
    assert S.vbh_scene_status() == 0
    if with_oracle:
        return S, O, depth, rgb, poses
    return S, depth.cuda(), rgb.cuda(), poses


def oracle_replay(O, n_clients, clients, limits, res, outs, advance=None, exact_mc=False):
    """Replays the served requests against the oracle's per-client stream sets, version by
    version (advance(v) brings the oracle scene to version v).  Every GPU answer must be a
    valid answer of its client's set; its MC voxels are compared with the oracle's stored MC
    voxels at that version: bit-exact when exact_mc, else differences only at cells with a
    corner |F_oracle| <= 1e-5.  Returns (blocks checked, MC voxels allowed to differ)."""
    T = oracle.Streams(O, n_clients)
    order = np.lexsort((np.arange(len(clients)), res["version"]))
    blocks, near = 0, 0
    for i in order:
        v = int(res["version"][i])
        if advance is not None:
            advance(v)
        T.sync()
        k = int(res["count"][i])
        keys = outs[i][0][:k].cpu().numpy()
        rc = T.take(int(clients[i]), int(limits[i]), keys)
        assert rc == 0, (i, int(clients[i]), v, k, rc)
        if k == 0:
            continue
        omc, orgb = O.stored_mc(keys)
        want = pack_mc(omc, orgb).numpy()
        got = outs[i][1][:k].cpu().numpy().astype(np.int64) & 0xFFFFFFFF
        bad = np.nonzero(got != want)
        if exact_mc:
            assert bad[0].size == 0, (i, bad[0].size)
        elif bad[0].size:
            assert (corner_min_abs(O, keys, *bad) <= 1e-5).all(), i
            near += bad[0].size
        blocks += k
    return blocks, near


def out_buffers(limits):
    return [(torch.zeros((max(l, 1), 3), dtype=torch.int32, device="cuda"),
             torch.zeros((max(l, 1), 512), dtype=torch.int32, device="cuda")) for l in limits]


def log_uniform(rng, n, lo, hi):
    return np.floor(10 ** rng.uniform(np.log10(lo), np.log10(hi), n)).astype(np.int64)


MODES = [0, 1]  # rounds of kernels on streams; one persistent launch per scene version


@pytest.mark.parametrize("mode", MODES)
def test_alone_equals_mix_static_scene(mode):
    vbh = require_gpu()
    S, O, _, _, _ = tiny_scene(vbh, 32, with_oracle=True)
    nb = S.vbh_scene_stats()["n_blocks"]
    srv = vbh.Server(S, arena_bytes=256 << 20, max_inflight=32, n_streams=4, n_clients=8, max_batch=12, mode=mode)
    rng = np.random.default_rng(0)
    n = 64
    clients = np.arange(n) % 8
    limits = log_uniform(rng, n, 10, 3000)
    arrivals = np.sort(rng.uniform(0, 0.02, n))
    outs = out_buffers(limits)
    res = srv.vbh_server_run(clients, limits, arrivals, outs)
    assert (res["status"] == 0).all()
    say(f"[serve static mode={mode}] {nb} blocks, {n} requests, {res['count'].sum()} blocks served")
    blocks, near = oracle_replay(O, 8, clients, limits, res, outs)
    say(f"[serve static] oracle replay: {blocks} blocks, {near} MC voxels at |F| <= 1e-5")
    assert blocks == res["count"].sum()
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


@pytest.mark.parametrize("mode", MODES)
def test_concurrent_integration_versions(mode):
    vbh = require_gpu()
    S, O, hdepth, hrgb, poses = tiny_scene(vbh, 8, with_oracle=True)
    depth, rgb = hdepth.cuda(), hrgb.cuda()
    srv = vbh.Server(S, arena_bytes=512 << 20, max_inflight=64, n_streams=4, n_clients=8, max_batch=16, mode=mode)
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
    # the oracle, fused in step with the served versions
    at = [8]

    def advance(v):
        while at[0] < v:
            f = at[0]
            assert O.integrate(hdepth[f].numpy(), hrgb[f].numpy(), poses[f], f + 1) == 0
            at[0] += 1

    blocks, near = oracle_replay(O, 8, clients, limits, res, outs, advance=advance)
    say(f"[serve concurrent] oracle replay: {blocks} blocks over {vers.size} versions, "
        f"{near} MC voxels at |F| <= 1e-5")
    assert blocks == res["count"].sum()


@pytest.mark.parametrize("mode", MODES)
def test_large_written_scene_against_oracle(mode):
    """150k blocks of the serving scene written analytically (two updates), 8 clients,
    48 requests with sizes log-uniform in [10^2, 10^5] arriving together: every answer and
    its MC voxels against the oracle's stream sets, bit-exact."""
    vbh = require_gpu()
    say("[serve large] building analytic blocks")
    keys, F, W, rgb = configs.analytic_blocks(configs.serve_scene(), configs.SERVE_VOL.voxel_size,
                                              configs.SERVE_VOL.trunc, device="cuda")
    n_blk = 150_000
    keys, F, W, rgb = (t[:n_blk].contiguous() for t in (keys, F, W, rgb))
    vol = configs.Volume(**{**configs.SERVE_VOL.__dict__, "slots": 1 << 19, "pool_blocks": 1 << 18,
                            "log_capacity": 1 << 21})
    S = vbh.Scene(vbh.make_params(vol, configs.FULL_CAM))
    O = oracle.Scene(vol, configs.FULL_CAM)
    hk, hF, hW, hc = (t.cpu().numpy() for t in (keys, F, W, rgb))
    half = n_blk // 2
    for lo, hi, fid in ((0, half, 1), (half, n_blk, 2)):
        S.vbh_scene_write_blocks(keys[lo:hi], F[lo:hi], W[lo:hi], rgb[lo:hi], fid)
        assert O.write(hk[lo:hi], hF[lo:hi], hW[lo:hi], hc[lo:hi], fid) == 0
    assert S.vbh_scene_status() == 0 and S.vbh_scene_stats()["n_blocks"] == n_blk
    assert S.vbh_scene_stats()["log_length"] == O.log_length()
    del F, W, rgb
    rng = np.random.default_rng(6464)
    n = 48
    clients = np.arange(n) % 8
    limits = log_uniform(rng, n, 100, 100_000)
    limits[3] = 100_000
    arrivals = np.zeros(n)
    outs = out_buffers(limits)
    srv = vbh.Server(S, arena_bytes=1 << 30, max_inflight=32, n_streams=4, n_clients=8, max_batch=16, mode=mode)
    res = srv.vbh_server_run(clients, limits, arrivals, outs)
    assert (res["status"] == 0).all()
    say(f"[serve large] {n} requests, {res['count'].sum()} blocks served, "
        f"largest answer {res['count'].max()}")
    assert res["count"].max() == 100_000
    blocks, _ = oracle_replay(O, 8, clients, limits, res, outs, exact_mc=True)
    assert blocks == res["count"].sum()


@pytest.mark.parametrize("mode", MODES)
def test_arena_outputs_reused(mode):
    """Answers kept in the server's arena (no caller buffers), so later batches reuse the
    ranges of earlier batches' MC voxel outputs (hundreds of MB through a 512 MiB arena):
    on a written scene whose log entries are all live, request i of a client takes
    count = min(limit, blocks left after its cursor) and moves the cursor by that much."""
    vbh = require_gpu()
    say(f"[serve arena reuse] mode {mode}: building analytic blocks")
    keys, F, W, rgb = configs.analytic_blocks(configs.serve_scene(), configs.SERVE_VOL.voxel_size,
                                              configs.SERVE_VOL.trunc, device="cuda")
    n_blk = 150_000
    keys, F, W, rgb = (t[:n_blk].contiguous() for t in (keys, F, W, rgb))
    vol = configs.Volume(**{**configs.SERVE_VOL.__dict__, "slots": 1 << 19, "pool_blocks": 1 << 18,
                            "log_capacity": 1 << 21})
    S = vbh.Scene(vbh.make_params(vol, configs.FULL_CAM))
    S.vbh_scene_write_blocks(keys, F, W, rgb, 1)
    assert S.vbh_scene_status() == 0 and S.vbh_scene_stats()["log_length"] == n_blk
    del keys, F, W, rgb
    rng = np.random.default_rng(2064)
    n = 80
    clients = np.arange(n) % 8
    limits = log_uniform(rng, n, 2000, 60_000)
    srv = vbh.Server(S, arena_bytes=1 << 29, max_inflight=32, n_streams=4, n_clients=8, max_batch=16, mode=mode)
    res = srv.vbh_server_run(clients, limits, np.zeros(n))
    assert (res["status"] == 0).all()
    cur = np.zeros(8, np.int64)
    for i in range(n):
        c = clients[i]
        want = min(int(limits[i]), n_blk - int(cur[c]))
        assert res["cursor_in"][i] == cur[c], i
        assert res["count"][i] == want, (i, int(res["count"][i]), want)
        cur[c] += want
        assert res["cursor_out"][i] == cur[c], i
    say(f"[serve arena reuse] {res['count'].sum()} blocks served")


@pytest.mark.parametrize("mode", MODES)
def test_admission_by_memory_and_errors(mode):
    vbh = require_gpu()
    S, _, _, _ = tiny_scene(vbh, 16)
    per_req = 1000 * (4 + 12 + 2048) + 4096
    srv = vbh.Server(S, arena_bytes=int(2.5 * per_req), max_inflight=16, n_streams=4, n_clients=8, max_batch=8,
                     mode=mode)
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
