"""Benchmark of the fused voxel-block-hashing path on one MI355X.

A step is one frame through the whole hot path (band allocation, TSDF/colour
integration, MC update-set marking and MC voxel extraction, update log) of the
2000-frame 640x480 noisy sequence in the 10x10x3 m room (5 mm voxels, 2 cm truncation,
2^22 slots).  Frames are pre-staged in HBM; the timed region is K consecutive frames into
a fresh volume, handed to the multi-frame entry point in one call.  Prints one JSON line on stdout (progress goes to stderr).

Also reported (secondary fields): the rate with per-frame PCIe uploads; MC against TSDF
packet bandwidth for 128-1024-block requests at 100 Hz; client triangulation and scene
reset on the fused scene; hash-map Mops/s on 2^24 keys (open addressing in 2^25 slots,
and the chained design in the same memory) with 1M-op mixed batches; the differentiable
form; the serving loop; and the oracle timed on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# Algorithmic bytes per unit of work, for the whole-block formulation of each step:
# integration reads and writes F (4 B) and W+RGB (4 B) of all 512 voxels of a touched
# block (8 KiB) and reads each pixel's depth (4 B) and colour (3 B); extraction of one
# MC-set block reads F and W (5 B) of its 729 voxels including the +1 halo and the RGB
# (3 B) of its 512 voxels, and writes 512 4-byte MC voxels.  The kernels move fewer
# bytes than this where they can (only updated voxels change, sign bits stand in for F
# and W in extraction); rocprofv3's measured traffic is reported beside it.
INT_BYTES_PER_BLOCK, INT_BYTES_PER_PIXEL = 16 * 512, 7
MC_BYTES_PER_BLOCK = 5 * 729 + 3 * 512 + 4 * 512


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def stage_frames(K, device):
    import torch
    from datagen import configs
    from datagen.scenes import render_frames, trajectory_c3
    scene = configs.full_scene()
    traj = trajectory_c3(scene, K)
    depth = torch.empty((K, 480, 640), dtype=torch.float32, device=device)
    rgb = torch.empty((K, 480, 640, 3), dtype=torch.uint8, device=device)
    t0 = time.time()
    for f in range(K):
        d, c = render_frames(scene, configs.FULL_CAM, [traj[f]], device=device, noise_seed=5203, first_frame=f)
        depth[f], rgb[f] = d[0], c[0]
        if f % 250 == 0:
            log(f"[bench] staged frame {f}/{K} ({time.time() - t0:.1f}s)")
    return depth, rgb, traj


def measured_traffic(kernel):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter summary (FETCH_SIZE
    and WRITE_SIZE scaled by a plain-copy calibration), or None if the kernel source changed
    since the counters were taken."""
    import hashlib
    try:
        t = json.load(open(os.path.join(ROOT, "profiles", "fusion_full_traffic.json")))
        src = open(os.path.join(ROOT, "paper_1805_03709_amd", "csrc", "scene.hip"), "rb").read()
    except OSError:
        return None
    if hashlib.sha1(src).hexdigest() != t.get("scene_hip_sha1") or ("k_" + kernel) not in t["per_dispatch"]:
        return None
    d = t["per_dispatch"]["k_" + kernel]
    return {"fetch_bytes": d["fetch_MB"] * 1e6, "write_bytes": d["write_MB"] * 1e6,
            "bytes": (d["fetch_MB"] + d["write_MB"]) * 1e6, "valu_insts": d.get("valu_insts"),
            "workload": t["workload"]}


# Vector-ALU issue peak: 256 CUs x 4 SIMDs x one wave64 instruction per 4 cycles x 2.4 GHz
# (full-rate instructions), in wave64 VALU instructions per second.
VALU_PEAK_WAVE_INSTR_S = 256 * 4 / 4 * 2.4e9


def valu_issue(t, kernel_ms):
    """The dominant kernel against the vector-ALU issue peak: measured VALU instructions per
    launch (rocprofv3 SQ_INSTS_VALU, committed with the traffic counters) over the kernel
    time measured in this run."""
    if not t or not t.get("valu_insts") or kernel_ms <= 0:
        return None
    rate = t["valu_insts"] / (kernel_ms * 1e-3)
    return {"valu_instructions_per_launch": t["valu_insts"], "achieved": rate / 1e9,
            "peak": VALU_PEAK_WAVE_INSTR_S / 1e9, "unit": "G wave64 VALU instructions/s",
            "frac": rate / VALU_PEAK_WAVE_INSTR_S}


def run_fusion(vbh, depth, rgb, traj, K, W, period=4):
    import torch
    from datagen import configs
    params = vbh.make_params(configs.FULL_VOL, configs.FULL_CAM)
    if W > 0:
        warm = vbh.Scene(params)
        for f in range(W):
            warm.vbh_integrate_frame(depth[f], rgb[f], traj[f], f + 1)
        torch.cuda.synchronize()
        assert warm.vbh_scene_status() == 0
        warm.close()
    S = vbh.Scene(params)
    S.vbh_scene_enable_timing(period)  # kernel start/stop events on every period-th frame
    poses = traj[:K]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    # all K frames in one call of the multi-frame entry point: the same kernels per frame as
    # K single-frame calls (bit-exact, tested), without a Python call per frame on the host
    S.vbh_integrate_frames(depth[:K], rgb[:K], poses, 1)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    stage_ms, frames, timed_blocks = S.vbh_scene_timing(with_blocks=True)
    stats = S.vbh_scene_stats()
    status = S.vbh_scene_status()
    if status != 0:
        raise RuntimeError(f"scene reported error {status}")
    return t1 - t0, stage_ms, frames, timed_blocks, stats, S


def per_frame_calls(vbh, depth, rgb, traj, K):
    """Frames/s when every frame is its own vbh_integrate_frame call from Python (the host's
    per-call cost then adds to each frame where it exceeds the GPU time)."""
    import torch
    from datagen import configs
    S = vbh.Scene(vbh.make_params(configs.FULL_VOL, configs.FULL_CAM))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for f in range(K):
        S.vbh_integrate_frame(depth[f], rgb[f], traj[f], f + 1)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    if S.vbh_scene_status() != 0:
        raise RuntimeError("scene reported an error")
    S.close()
    return {"frames": K, "frames_per_s": K / dt}


def h2d_fusion(vbh, depth, rgb, traj, K):
    """Frames/s when the frames start in pinned host memory: vbh_integrate_frames_host
    copies each frame over PCIe in front of its kernels."""
    import torch
    from datagen import configs
    K = min(K, depth.shape[0])
    hd = depth[:K].cpu().pin_memory()
    hc = rgb[:K].cpu().pin_memory()
    # the first DMA read of freshly pinned pages is slow (about 2.5 GB/s here, against
    # 57 GB/s afterwards): touch them once from the device before timing
    torch.empty(hd.shape, dtype=hd.dtype, device="cuda").copy_(hd)
    torch.empty(hc.shape, dtype=hc.dtype, device="cuda").copy_(hc)
    S = vbh.Scene(vbh.make_params(configs.FULL_VOL, configs.FULL_CAM))
    S.vbh_integrate_frames_host(hd[:2], hc[:2], traj[:2], 1)  # allocates the device frame buffers
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    S.vbh_integrate_frames_host(hd[2:], hc[2:], traj[2:K], 3)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    if S.vbh_scene_status() != 0:
        raise RuntimeError("scene reported an error")
    S.close()
    return {"frames": K - 2, "frames_per_s": (K - 2) / dt,
            "MB_per_frame_uploaded": (hd[0].numel() * 4 + hc[0].numel()) / 1e6, "pinned": True}


def hash_bench(vbh, log_phases=True):
    """Hash map Mops/s: bulk insert/find of 2^24 keys into 2^25 slots, 16 mixed 1M batches,
    for the open-addressing map and the chained design."""
    import numpy as np
    import torch
    import datagen
    keys, vals = datagen.bulk_keys()
    dk, dv = torch.as_tensor(keys).cuda(), torch.as_tensor(vals).cuda()
    present = np.unique(datagen.pack_key(keys))
    batches = []
    for i, (ops, k, v) in enumerate(datagen.mixed_batches(present)):
        batches.append((torch.as_tensor(ops).cuda(), torch.as_tensor(k).cuda(), torch.as_tensor(v).cuda()))
        if log_phases and i % 4 == 3:
            log(f"[bench] hash batches generated: {i + 1}")
    out = {}
    reps = 5
    # the open-addressing map (2^25 slots) and the paper's chained design in the same
    # memory (2^24 buckets + 2^24 excess entries), on identical batches
    designs = ((0, "spatial", lambda k: vbh.Map(1 << 25, k)), (1, "mix64", lambda k: vbh.Map(1 << 25, k)),
               (0, "chained_spatial", lambda k: vbh.ChainedMap(1 << 24, 1 << 24, k)),
               (1, "chained_mix64", lambda k: vbh.ChainedMap(1 << 24, 1 << 24, k)))
    for kind, name, make in designs:
        m = make(kind)
        st = torch.empty(dk.shape[0], dtype=torch.int32, device="cuda")
        res = torch.empty(1 << 20, dtype=torch.int32, device="cuda")
        e = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
        ins, fnd, mix = [], [], []
        for rep in range(reps):  # each rep starts from an empty table (cleared outside the timing)
            m.vbh_map_clear()
            torch.cuda.synchronize()
            e[0].record()
            m.vbh_insert(dk, dv, st)
            e[1].record()
            m.vbh_find(dk, st)
            e[2].record()
            for ops, k, v in batches:
                m.vbh_apply(ops, k, v, res)
            e[3].record()
            torch.cuda.synchronize()
            if m.vbh_map_status() != 0:
                raise RuntimeError("hash map reported an error")
            ins.append(e[0].elapsed_time(e[1]))
            fnd.append(e[1].elapsed_time(e[2]))
            mix.append(e[2].elapsed_time(e[3]))
        n = dk.shape[0]
        nm = sum(b[0].shape[0] for b in batches)
        out[name] = {"insert_mops": n / float(np.median(ins)) / 1e3,
                     "find_mops": n / float(np.median(fnd)) / 1e3,
                     "mixed_mops": nm / float(np.median(mix)) / 1e3, "reps": reps}
        m.close()
        log(f"[bench] hash {name}: {out[name]}")
    # the ceiling: uncontended random 64-bit compare-and-swaps over a 512 MiB array (larger
    # than the 2^25-slot table and than the Infinity Cache), as many as the bulk insert makes
    words = torch.zeros(1 << 26, dtype=torch.int64, device="cuda")
    won = torch.zeros(1, dtype=torch.int64, device="cuda")
    n_ops = 1 << 24
    times = []
    for rep in range(reps):
        words.zero_()
        won.zero_()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        vbh.binding.vbh_cas_ceiling(words, n_ops, 1234 + rep, won)
        e1.record()
        torch.cuda.synchronize()
        times.append(e0.elapsed_time(e1))
    out["cas_ceiling"] = {"gops": n_ops / float(np.median(times)) / 1e6, "ops": n_ops, "words": int(words.numel()),
                          "succeeded": int(won.item()), "reps": reps,
                          "workload": "2^24 uncontended random 64-bit atomicCAS over a 2^26-word (512 MiB) array"}
    log(f"[bench] hash cas ceiling: {out['cas_ceiling']}")
    return out


def bandwidth_bench(vbh, depth, rgb, traj, n_frames=300, fps=30.0, rate=100.0, sizes=(128, 256, 512, 1024),
                    drain_s=60.0, tsdf_sample=16):
    """Synthetic analogue of the paper's bandwidth table: the first n_frames of the
    sequence are fused at `fps` while benchmark clients request k updated MC blocks at
    `rate` Hz (one client per k, each from its own cursor) until the model is streamed.
    Every MC packet is built and zstd-compressed (level 1); bandwidth is compressed bytes
    per 1-s window.  The TSDF stream sends, unlimited, every block updated since its last
    step in 512-block packets of 12-byte voxels; its bytes are the exact block counts
    times the compressed bytes per block of 1 in `tsdf_sample` packets (compressing all
    of them would take minutes of host time)."""
    import numpy as np
    import torch
    from datagen import configs
    from paper_1805_03709_amd import packets
    S = vbh.Scene(vbh.make_params(configs.FULL_VOL, configs.FULL_CAM))
    n_frames = min(n_frames, depth.shape[0])
    cur = {k: 0 for k in sizes}
    sent = {k: [] for k in sizes}     # (time, compressed bytes, blocks)
    done = {k: None for k in sizes}
    tsdf_cur, tsdf_steps, tsdf_sampled = 0, [], [0, 0]  # sampled: [compressed bytes, blocks]
    fused, step, i = 0, 1.0 / rate, 0
    t_host = time.perf_counter()
    while any(v is None for v in done.values()):
        t = i * step
        if t > n_frames / fps + drain_s:
            break
        due = min(n_frames, int(t * fps) + 1)
        while fused < due:
            S.vbh_integrate_frame(depth[fused], rgb[fused], traj[fused], fused + 1)
            fused += 1
        for k in sizes:
            if done[k] is not None:
                continue
            keys, meta = S.vbh_updated_blocks_since(cur[k], k)
            cnt, nxt = (int(v) for v in meta.tolist())
            if cnt:
                kk = keys[:cnt].contiguous()
                mc, c3 = S.vbh_stored_mc(kk)
                mc, c3 = mc.cpu().numpy().astype(np.uint32), c3.cpu().numpy().astype(np.uint32)
                packed = mc | (c3[..., 0] << 8) | (c3[..., 1] << 16) | (c3[..., 2] << 24)
                z = packets.zstd_compress(packets.mc_packet(kk.cpu().numpy(), packed))
                sent[k].append((t, len(z), cnt))
            cur[k] = nxt
            if fused == n_frames and cnt < k:
                done[k] = t
        if fused < n_frames or i % int(rate) == 0:
            keys, meta = S.vbh_updated_blocks_since(tsdf_cur, 1 << 22)
            cnt, nxt = (int(v) for v in meta.tolist())
            tsdf_steps.append((t, cnt))
            if cnt and len(tsdf_steps) % tsdf_sample == 1:
                kk = keys[:min(cnt, 512)].contiguous()
                F, Wt, c3, found = S.vbh_scene_read_blocks(kk)
                z = packets.zstd_compress(packets.tsdf_packet(kk.cpu().numpy(), F.cpu().numpy(), Wt.cpu().numpy(),
                                                              c3.cpu().numpy()))
                tsdf_sampled[0] += len(z)
                tsdf_sampled[1] += kk.shape[0]
            tsdf_cur = nxt
        if i % int(5 * rate) == 0:
            log(f"[bench] bandwidth: simulated {t:.0f} s, {fused} frames fused, "
                f"{time.perf_counter() - t_host:.1f} s host time")
        i += 1
    if S.vbh_scene_status() != 0:
        raise RuntimeError("scene reported an error during the bandwidth run")

    def windows(events, end):
        nwin = max(1, int(np.ceil(end)))
        acc = np.zeros(nwin)
        for tt, b in events:
            acc[min(int(tt), nwin - 1)] += b
        mbit = acc * 8 / 1e6
        return float(mbit.mean()), float(mbit.max())

    out = {"workload": f"first {n_frames} frames of the 640x480 sequence fused at {fps:g} Hz, 5 mm voxels, "
                       f"2 cm truncation; requests at {rate:g} Hz; zstd level 1",
           "model_blocks": S.vbh_scene_stats()["n_blocks"], "mc": {}}
    for k in sizes:
        ev = sent[k]
        end = done[k] if done[k] is not None else n_frames / fps + drain_s
        mean, mx = windows([(tt, b) for tt, b, _ in ev], end)
        nb = sum(c for _, _, c in ev)
        out["mc"][str(k)] = {"mean_mbit_s": mean, "max_mbit_s": mx, "complete_s": done[k], "blocks_sent": nb,
                             "bytes_per_block": sum(b for _, b, _ in ev) / max(nb, 1)}
    bpb = tsdf_sampled[0] / max(tsdf_sampled[1], 1)
    end = n_frames / fps
    mean, mx = windows([(tt, c * bpb) for tt, c in tsdf_steps if tt < end], end)
    out["tsdf_512"] = {"mean_mbit_s": mean, "max_mbit_s": mx, "bytes_per_block": bpb,
                       "blocks_sent": sum(c for _, c in tsdf_steps), "sampled_blocks": tsdf_sampled[1],
                       "uncompressed_bytes_per_block": packets.TSDF_BLOCK_BYTES}
    out["mc_vs_tsdf_bytes_per_block"] = out["mc"]["512"]["bytes_per_block"] / max(bpb, 1e-9)
    out["host_seconds"] = time.perf_counter() - t_host
    S.close()
    return out


def client_bench(vbh, S, pose, frame_id, reps=5):
    """On the fused full-size scene: client triangulation of every block's MC voxels, then
    a scene reset of the blocks visible from `pose` (selection, clearing and MC update)."""
    import numpy as np
    import torch
    from datagen import configs
    keys = S.vbh_scene_export_blocks()
    mc, c3 = S.vbh_stored_mc(keys)
    mcv = (mc.to(torch.int64) | c3[..., 0].to(torch.int64) << 8 | c3[..., 1].to(torch.int64) << 16
           | c3[..., 2].to(torch.int64) << 24).to(torch.uint32).view(torch.int32).contiguous()
    del mc, c3
    vs = configs.FULL_VOL.voxel_size
    pos, rgb = vbh.vbh_mc_triangulate(keys, mcv, vs)  # warm-up, and the output size
    n, m = keys.shape[0], pos.shape[0]
    ts = []
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record()
        pos, rgb = vbh.vbh_mc_triangulate(keys, mcv, vs)
        e1.record()
        torch.cuda.synchronize()
        ts.append(e0.elapsed_time(e1))
    ms = float(np.median(ts))
    alg = n * (2048 + 12) + m * (36 + 3)
    mesh = {"blocks": n, "triangles": m, "ms": ms, "mtri_per_s": m / ms / 1e3, "algorithmic_GBps": alg / ms / 1e6,
            "note": "two calls' worth of work: count + scan, a host read of the total, then emission"}
    del pos, rgb
    t0 = time.perf_counter()
    vis = S.vbh_scene_visible_blocks(pose)
    t1 = time.perf_counter()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    S.vbh_scene_reset_blocks(vis, frame_id)
    e1.record()
    torch.cuda.synchronize()
    st = S.vbh_scene_stats()
    if S.vbh_scene_status() != 0:
        raise RuntimeError("scene reported an error in the reset")
    reset = {"visible_blocks": int(vis.shape[0]), "select_ms": (t1 - t0) * 1e3, "reset_ms": e0.elapsed_time(e1),
             "mc_blocks_republished": st["n_mc"], "scene_blocks": n}
    return {"mesh": mesh, "reset": reset}


def diff_bench(vbh, reps=5):
    """Differentiable form on 16 frames of the 640x480 sequence (2 cm voxels, 8 cm
    truncation, 100k samples): forward and backward kernel time (torch events on the
    stream the library launches on)."""
    import torch
    from datagen import configs
    from paper_1805_03709_amd.autograd import DiffFusion
    _, depth, _, poses, sf, sp = configs.diff_inputs(device="cuda")
    E = DiffFusion(vbh.make_params(configs.DIFF_VOL, configs.FULL_CAM), depth.shape[0])
    d = depth.contiguous()
    f = torch.as_tensor(sf).cuda()
    p = torch.as_tensor(sp).cuda()
    one = torch.ones((), device="cuda")
    E.vbh_diff_forward(d, poses, f, p)  # warm-up
    E.vbh_diff_backward(d, poses, f, p, one)
    torch.cuda.synchronize()
    fw, bw = [], []
    for _ in range(reps):
        e = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
        e[0].record()
        loss, _ = E.vbh_diff_forward(d, poses, f, p, with_samples=False)
        e[1].record()
        E.vbh_diff_backward(d, poses, f, p, one)
        e[2].record()
        torch.cuda.synchronize()
        fw.append(e[0].elapsed_time(e[1]))
        bw.append(e[1].elapsed_time(e[2]))
    fwd, bwd = sorted(fw)[reps // 2], sorted(bw)[reps // 2]
    n = depth.shape[0]
    return {"frames": n, "samples": int(f.numel()), "forward_ms": fwd, "backward_ms": bwd,
            "backward_ms_per_frame": bwd / n, "backward_over_forward": bwd / fwd, "loss": float(loss)}


def large_batch_bench(vbh, vs=0.003, wall=3.9):
    """Integration and MC extraction of more than a million blocks in one launch each,
    beyond the 256 MB Infinity Cache: every block of a 3 mm volume (2.4 cm blocks) whose
    centre lies in the 640x480 camera's frustum between 0.45 m and wall - 5 cm, in front of
    a fronto-parallel wall at `wall` metres (every voxel that projects into the image is
    in free space, so it is read and written).  The list is integrated twice (the first
    pass allocates the blocks); the second pass is the one measured, with kernel start and
    stop events attached to its dispatches."""
    import torch
    from datagen import configs
    cam = configs.FULL_CAM
    bs = 8 * vs
    vol = configs.Volume(slots=1 << 23, pool_blocks=1 << 21, voxel_size=vs, trunc=4 * vs, depth_min=0.4,
                         depth_max=4.0, log_capacity=1 << 23)
    zs = torch.arange(int(0.45 / bs), int((wall - 0.05) / bs), device="cuda", dtype=torch.int64)
    zc = (zs.to(torch.float64) + 0.5) * bs
    keys = []
    for z, c in zip(zs.tolist(), zc.tolist()):
        hx = c * (cam.width / 2) / cam.fx
        hy = c * (cam.height / 2) / cam.fy
        xs = torch.arange(int(-hx / bs) - 1, int(hx / bs) + 1, device="cuda")
        ys = torch.arange(int(-hy / bs) - 1, int(hy / bs) + 1, device="cuda")
        xc, yc = (xs.to(torch.float64) + 0.5) * bs, (ys.to(torch.float64) + 0.5) * bs
        xs, ys = xs[xc.abs() <= hx], ys[yc.abs() <= hy]
        g = torch.stack(torch.meshgrid(xs, ys, indexing="ij"), -1).reshape(-1, 2)
        keys.append(torch.cat([g, torch.full((g.shape[0], 1), z, device="cuda")], 1))
    keys = torch.cat(keys).to(torch.int32).contiguous()
    depth = torch.full((cam.height, cam.width), wall, dtype=torch.float32, device="cuda")
    rgb = torch.full((cam.height, cam.width, 3), 128, dtype=torch.uint8, device="cuda")
    pose = [[1.0, 0, 0, 0], [0, 1.0, 0, 0], [0, 0, 1.0, 0]]
    S = vbh.Scene(vbh.make_params(vol, cam))
    S.vbh_integrate_blocks(keys, depth, rgb, pose, 1)
    torch.cuda.synchronize()
    S.vbh_scene_enable_timing(1)
    S.vbh_scene_timing()  # discard the first pass
    S.vbh_integrate_blocks(keys, depth, rgb, pose, 2)
    ms, n_timed = S.vbh_scene_timing()
    st = S.vbh_scene_stats()
    if S.vbh_scene_status() != 0:
        raise RuntimeError("large-batch scene reported an error")
    out = {"workload": f"{keys.shape[0]} blocks of a {vs * 1e3:g} mm volume in the 640x480 frustum in front of a "
                       f"wall at {wall} m, integrated (second pass) and MC-extracted in one launch each",
           "blocks": int(st["n_touched"]), "mc_blocks": int(st["n_mc"]),
           "voxel_updates": int(st["n_voxel_updates"])}
    for stage, nbytes in (("integrate", INT_BYTES_PER_BLOCK * st["n_touched"] + INT_BYTES_PER_PIXEL * cam.width * cam.height),
                          ("mc_extract", MC_BYTES_PER_BLOCK * st["n_mc"])):
        t = ms[stage] / max(n_timed, 1)
        gbs = nbytes / (t * 1e-3) / 1e9
        out[stage] = {"kernel_ms": t, "algorithmic_bytes": float(nbytes), "achieved": gbs, "peak": HBM_PEAK_GBS,
                      "unit": "GB/s", "frac": gbs / HBM_PEAK_GBS}
    S.close()
    del keys, depth, rgb
    torch.cuda.empty_cache()
    out["stream_ceiling"] = stream_ceiling(out["integrate"]["algorithmic_bytes"])
    return out


def stream_ceiling(nbytes, reps=5):
    """What plain streaming kernels (PyTorch's own, not this library's) reach over a working
    set of the large-batch integration's size: an in-place add (every byte read and
    written back, the integration's access pattern) and a copy, in GB/s of read plus
    written bytes, median of `reps`."""
    import numpy as np
    import torch
    n = int(nbytes / 2) // 4
    a = torch.zeros(n, dtype=torch.int32, device="cuda")
    b = torch.zeros(n, dtype=torch.int32, device="cuda")
    res = {"bytes_each": 4 * n}
    for name, fn in (("inplace_add", lambda: a.add_(1)), ("copy", lambda: b.copy_(a))):
        fn()
        times = []
        for _ in range(reps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            fn()
            e1.record()
            torch.cuda.synchronize()
            times.append(e0.elapsed_time(e1))
        res[name + "_GBps"] = 2 * 4 * n / (float(np.median(times)) * 1e-3) / 1e9
    del a, b
    torch.cuda.empty_cache()
    log(f"[bench] stream ceiling: {res}")
    return res


SERVE_MODES = {0: "rounds", 1: "persistent"}


def serve_bench(vbh, seconds=60.0, warmup=10.0, clients=64, rate=30.0, n_unique_frames=600, mode=0):
    """Serving: ~2M-block scene resident on the device, `clients` clients with Poisson
    arrivals (`rate` req/s each), request sizes floor(10^U(2,5)) blocks, every client
    starting from cursor 0, while 640x480 frames are fused at 30 Hz.  Latency = arrival to
    results in device memory; statistics over requests arriving after the warm-up.
    mode: 0 rounds of kernels on 4 streams, 1 one persistent launch per scene version
    (4 teams)."""
    import numpy as np
    import torch
    from datagen import configs
    t0 = time.time()
    scene = configs.serve_scene()
    keys, F, W, rgb = configs.analytic_blocks(scene, configs.SERVE_VOL.voxel_size, configs.SERVE_VOL.trunc,
                                              device="cuda")
    S = vbh.Scene(vbh.make_params(configs.SERVE_VOL, configs.FULL_CAM))
    S.vbh_scene_write_blocks(keys.contiguous(), F.contiguous(), W.contiguous(), rgb.contiguous(), 1)
    st = S.vbh_scene_stats()
    if S.vbh_scene_status() != 0:
        raise RuntimeError("serving scene load failed")
    del F, W, rgb
    log(f"[bench] serve scene: {st['n_blocks']} blocks, log {st['log_length']} ({time.time() - t0:.1f}s)")
    depth, rgbf, traj = configs.serve_frames(n_unique_frames, device="cuda")
    total = seconds + warmup
    nf = int(total * 30)
    frames = [(depth[f % n_unique_frames], rgbf[f % n_unique_frames], traj[f % n_unique_frames], f / 30.0, f + 2)
              for f in range(nf)]
    rng = np.random.default_rng(6464)
    arr, cl = [], []
    for c in range(clients):
        t = np.cumsum(rng.exponential(1.0 / rate, int(total * rate * 1.5) + 50))
        t = t[t < total]
        arr.append(t)
        cl.append(np.full(t.size, c))
    arr, cl = np.concatenate(arr), np.concatenate(cl)
    order = np.argsort(arr, kind="stable")
    arr, cl = arr[order], cl[order]
    lim = np.floor(10 ** rng.uniform(2, 5, arr.size)).astype(np.int64)
    srv = vbh.Server(S, arena_bytes=24 << 30, max_inflight=512, n_streams=4, n_clients=clients, max_batch=64,
                     mode=mode)
    log(f"[bench] serving {arr.size} requests over {total:.0f}s with {nf} fused frames")
    res = srv.vbh_server_run(cl, lim, arr, frames=frames)
    if (res["status"] != 0).any() or S.vbh_scene_status() != 0:
        raise RuntimeError("serving reported an error")
    m = res["arrival_s"] >= warmup
    lat = (res["done_s"] - res["arrival_s"])[m] * 1e3
    queue = (res["admit_s"] - res["arrival_s"])[m] * 1e3
    blocks = res["count"][m].sum()
    span = res["done_s"][m].max() - warmup
    out = {"mode": SERVE_MODES[mode], "requests": int(m.sum()), "clients": clients, "rate_per_client": rate,
           "seconds": seconds,
           "scene_blocks": int(st["n_blocks"]), "frames_fused": nf,
           "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
           "p50_queue_ms": float(np.percentile(queue, 50)), "p99_queue_ms": float(np.percentile(queue, 99)),
           "blocks_per_s": float(blocks / span), "MB_per_s": float(blocks * 2060 / span / 1e6),
           "versions_served": int(np.unique(res["version"][m]).size)}
    srv.close()
    S.close()
    return out


def cpu_baseline(depth, rgb, traj, budget_s):
    """The oracle, as it stands, on the first frames of the same sequence until the time
    budget is spent (host copies excluded)."""
    import oracle
    from datagen import configs
    frames = [(depth[i].cpu().numpy(), rgb[i].cpu().numpy()) for i in range(depth.shape[0])]
    O = oracle.Scene(configs.FULL_VOL, configs.FULL_CAM)
    used, n = 0.0, 0
    for i, (d, c) in enumerate(frames):
        ts = time.perf_counter()
        O.integrate(d, c, traj[i], i + 1)
        used += time.perf_counter() - ts
        n += 1
        if used >= budget_s:
            break
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    model = ""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {"value": n / used, "unit": "frames/s", "cores": cores, "kind": "oracle",
            "host": {"nproc": os.cpu_count(), "cpu_model": model, "omp_threads": cores},
            "sample": f"first {n} frames of the 640x480 sequence: allocation, integration and MC "
                      f"update into the same 5 mm volume ({used:.1f} s of oracle time)"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=2000)
    ap.add_argument("--no-hash", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-diff", action="store_true")
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--no-bandwidth", action="store_true")
    ap.add_argument("--no-client", action="store_true")
    ap.add_argument("--no-h2d", action="store_true")
    ap.add_argument("--no-per-frame", action="store_true")
    ap.add_argument("--no-large", action="store_true", help="skip the large-batch integration/extraction run")
    ap.add_argument("--serve-seconds", type=float, default=60.0)
    ap.add_argument("--serve-mode", type=int, default=0, choices=[0, 1],
                    help="serving form of the headline serve run: 0 rounds of kernels, 1 persistent launch")
    ap.add_argument("--serve-ab-seconds", type=float, default=20.0,
                    help="length of the A/B run of the other serving form (0: skip)")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--timing-period", type=int, default=0,
                    help="attach kernel start/stop events to every n-th frame of the timed run "
                         "(0: every frame up to 125 frames, then about 125 frames spread evenly)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain 1 GiB device copy (scale reference for HBM counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU: --gpus {args.gpus} is not supported; the path runs on a "
              "single GPU only", file=sys.stderr)
        sys.exit(2)
    import torch
    import paper_1805_03709_amd as vbh
    if not torch.cuda.is_available():
        print("no HIP device", file=sys.stderr)
        sys.exit(1)
    torch.cuda.set_device(0)
    vbh.lib()
    K, W = args.steps, args.warmup
    if args.copy_calibration:
        src = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        log("[bench] copy calibration: 3 x 1 GiB device copies")
        del src, dst
    depth, rgb, traj = stage_frames(max(K, W), "cuda")
    log("[bench] frames staged; fusing")
    period = args.timing_period or max(1, K // 125)
    dt, stage_ms, frames, timed_blocks, stats, S = run_fusion(vbh, depth, rgb, traj, K, W, period)
    value = K / dt
    # kernel milliseconds per frame, averaged over the timed frames (every period-th frame)
    ms_frame = {s: v / max(frames, 1) for s, v in stage_ms.items()}
    log(f"[bench] {K} frames in {dt:.3f}s = {value:.1f} frames/s; kernel us/frame over {frames} timed frames: "
        + ", ".join(f"{s} {1e3 * v:.1f}" for s, v in ms_frame.items()))
    # algorithmic bytes per frame, from the blocks of exactly the timed frames
    hw = 640 * 480
    nt = max(frames, 1)
    bytes_frame = {
        "integrate": INT_BYTES_PER_BLOCK * timed_blocks[0] / nt + INT_BYTES_PER_PIXEL * hw,
        "mc_extract": MC_BYTES_PER_BLOCK * float(timed_blocks[1]) / nt,
    }
    dom = max(bytes_frame, key=lambda s: ms_frame[s])
    achieved = bytes_frame[dom] / (ms_frame[dom] * 1e-3) / 1e9
    per_stage = {s: {"ms_per_frame": v} for s, v in ms_frame.items()}
    for s, b in bytes_frame.items():
        per_stage[s]["GBps"] = b / (ms_frame[s] * 1e-3) / 1e9
    result = {
        "metric": "frames/s fused @640x480",
        "value": value, "unit": "frames/s", "n_gpus": 1, "steps": K, "warmup": W,
        "ms_per_step": dt * 1e3 / K, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "full: 640x480 noisy depth+RGB, 10x10x3 m room, 5 mm voxels, "
                               "2 cm truncation, 2^22 slots, 2^21-block pool, per-frame MC update",
                   "frames": K, "parallelism": "single-gpu"},
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": (measured_traffic(dom) or {}).get("bytes"),
                     "traffic_detail": measured_traffic(dom),
                     "traffic_source": "replayed from profiles/fusion_full_traffic.json (rocprofv3 "
                                       "FETCH_SIZE + WRITE_SIZE per launch, scaled by a plain-copy "
                                       "calibration, over the default 2000-frame run); not measured in "
                                       "this run; null once the kernel source differs from the "
                                       "profiled one",
                     "algorithmic_bytes_per_launch": bytes_frame[dom],
                     "timed_blocks_per_frame": {"touched": timed_blocks[0] / nt, "mc_set": timed_blocks[1] / nt},
                     "kernel_ms": ms_frame[dom], "timed_frames": frames, "timing_period": period,
                     "valu_issue": valu_issue(measured_traffic(dom), ms_frame[dom])},
        "stages": per_stage,
        "scene": {"blocks": stats["n_blocks"], "touched_per_frame": stats["total_touched"] / K,
                  "mc_blocks_per_frame": stats["total_mc"] / K,
                  "voxel_updates_per_frame": stats["total_voxel_updates"] / K},
    }
    if not args.no_large:
        log("[bench] large-batch integration and extraction")
        lb = large_batch_bench(vbh)
        result["roofline"]["large_batch"] = lb
        log(f"[bench] large batch: {lb}")
    if not args.no_client:
        log("[bench] client triangulation and scene reset on the fused scene")
        result["client"] = client_bench(vbh, S, traj[K - 1], K + 1)
        log(f"[bench] client: {result['client']}")
    S.close()
    if not args.no_per_frame:
        result["fusion_per_frame_calls"] = per_frame_calls(vbh, depth, rgb, traj, K)
        log(f"[bench] one Python call per frame: {result['fusion_per_frame_calls']}")
    if not args.no_h2d:
        log("[bench] fusion with per-frame host-to-device upload")
        result["fusion_with_h2d"] = h2d_fusion(vbh, depth, rgb, traj, min(K, 500))
        log(f"[bench] {result['fusion_with_h2d']}")
    if not args.no_bandwidth:
        log("[bench] streaming bandwidth (MC packets vs TSDF packets)")
        result["bandwidth"] = bandwidth_bench(vbh, depth, rgb, traj)
        log(f"[bench] bandwidth: {result['bandwidth']}")
    del depth
    if not args.no_hash:
        log("[bench] hash map phase")
        result["hash_mops"] = hash_bench(vbh)
    if not args.no_diff:
        log("[bench] differentiable form")
        result["diff"] = diff_bench(vbh)
        log(f"[bench] diff: {result['diff']}")
    if not args.no_serve:
        log("[bench] serving")
        result["serve"] = serve_bench(vbh, seconds=args.serve_seconds, mode=args.serve_mode)
        log(f"[bench] serve: {result['serve']}")
        if args.serve_ab_seconds > 0:
            result["serve_ab"] = serve_bench(vbh, seconds=args.serve_ab_seconds, mode=1 - args.serve_mode)
            log(f"[bench] serve A/B: {result['serve_ab']}")
    if not args.no_cpu:
        log("[bench] cpu baseline (oracle)")
        d2, c2, t2 = stage_frames(200, "cuda")
        result["cpu_baseline"] = cpu_baseline(d2, c2, t2, args.cpu_seconds)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
