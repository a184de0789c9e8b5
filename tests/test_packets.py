"""Streaming packet layouts (Sec. 4.2: the 4-byte MC voxel against the 12-byte TSDF voxel)
and the zstd round trip, on the CPU."""
import numpy as np

from paper_1805_03709_amd import packets


def test_mc_packet_layout_and_round_trip():
    rng = np.random.default_rng(0)
    keys = rng.integers(-1000, 1000, (7, 3)).astype(np.int32)
    mcv = rng.integers(0, 1 << 32, (7, 512), dtype=np.uint64).astype(np.uint32)
    b = packets.mc_packet(keys, mcv)
    assert len(b) == 7 * packets.MC_BLOCK_BYTES == 7 * (12 + 2048)
    raw = np.frombuffer(b, np.uint8).reshape(7, -1)
    assert np.array_equal(raw[:, :12].copy().view("<i4"), keys)
    assert np.array_equal(raw[:, 12:].copy().view("<u4"), mcv)
    z = packets.zstd_compress(b)
    assert packets.zstd_decompress(z, len(b)) == b


def test_tsdf_packet_layout():
    rng = np.random.default_rng(1)
    keys = rng.integers(-5, 5, (3, 3)).astype(np.int32)
    F = rng.standard_normal((3, 512)).astype(np.float32)
    W = rng.integers(0, 256, (3, 512)).astype(np.uint8)
    rgb = rng.integers(0, 256, (3, 512, 3)).astype(np.uint8)
    b = packets.tsdf_packet(keys, F, W, rgb)
    assert len(b) == 3 * packets.TSDF_BLOCK_BYTES == 3 * (12 + 512 * 12)
    raw = np.frombuffer(b, np.uint8).reshape(3, -1)
    assert np.array_equal(raw[:, :12].copy().view("<i4"), keys)
    vox = raw[:, 12:].reshape(3, 512, 12)
    assert np.array_equal(vox[..., 0:4].copy().view("<f4")[..., 0], F)
    assert np.array_equal(vox[..., 4:8].copy().view("<f4")[..., 0], W.astype(np.float32))
    assert np.array_equal(vox[..., 8:11], rgb) and (vox[..., 11] == 0).all()


def test_zstd_compresses_cut_off_voxels():
    # a block whose MC voxels are all cut to zero (indices 0 and 255) costs only its key
    keys = np.zeros((512, 3), np.int32)
    keys[:, 0] = np.arange(512)
    z = packets.zstd_compress(packets.mc_packet(keys, np.zeros((512, 512), np.uint32)))
    assert len(z) < 512 * 12
