// Scene state shared by the fusion kernels (scene.hip) and the differentiable form
// (diff.hip): device layout of a block-hashed TSDF volume with its MC voxel pool and
// update log, the per-frame camera constants, and the host-side handle.
#pragma once

#include <cstddef>
#include <hip/hip_runtime.h>

#include <array>
#include <vector>

#include "device.hpp"
#include "host.hpp"
#include "vbh.h"

namespace vbh {

int table_init(Slot *T, uint64_t n, hipStream_t st);

constexpr int kBlock = 256;
constexpr int kWaves = kBlock / 64;
constexpr int kChunk = 2048;  // log entries per workgroup chunk in the paged walk
constexpr int kRing = 8;      // per-frame counter ring
constexpr int kMaxPartials = 1 << 16;
// Start/stop events of the fusion kernels of one timed update; bit i of `ran` is set if
// stage i was launched.  Stages: 0 allocation (with MC-set marking), 1 integration,
// 2 stand-alone MC-set marking, 3 MC extraction.
constexpr int kStages = 4;
struct StageTimer {
    std::array<hipEvent_t, 2 * kStages> ev{};
    unsigned ran = 0;
};

// Same-address atomics serialise in L2 (about 10 ns each), so every kernel claims list
// space and reports statistics once per workgroup, never once per wave.

struct FrameCounters {
    unsigned int n_touched;  // n_touched and n_mc share an aligned 64-bit word: the
    unsigned int n_mc;       // allocation kernel reserves space in both lists with one atomic
                             // (n_mc: blocks in the update's MC set, entries of the MC list)
    unsigned int n_new;
    unsigned int pad;
    unsigned long long voxel_updates;
    unsigned long long log_base;  // log length when the update started; the extraction
                                  // kernel writes the MC list to [log_base, log_base + n_mc)
};

static_assert(offsetof(FrameCounters, n_mc) == 4 && alignof(FrameCounters) == 8, "shared 64-bit counter word");

struct Counters {
    FrameCounters fc[kRing];
    unsigned long long pool_next;  // pool blocks handed out (may exceed capacity)
    unsigned long long log_len;    // log entries written or attempted
    unsigned long long tot_touched;  // sums over all updates so far
    unsigned long long tot_mc;
    unsigned long long tot_voxel_updates;
    uint32_t err;
    uint32_t pad;
    unsigned long long visible;  // result count of the last visible-block selection
    unsigned long long timed_touched;  // touched and MC-set blocks of the updates whose
    unsigned long long timed_mc;       // kernels were timed, since the last timing read
};

// Device view of a scene, passed by value to kernels.
struct Dev {
    Slot *T;
    uint64_t mask;
    int kind;
    float *F;            // [P][512]
    uint32_t *WRGB;      // [P][512] W | R<<8 | G<<16 | B<<24
    uint32_t *MCV;       // [P][512] index | R<<8 | G<<16 | B<<24
    uint16_t *SGN;       // [P][64] per voxel column (x, y), index x + 8 y: bit z "F < 0 and
                         // observed", bit 8 + z "observed" (W > 0, F not NaN); kept in step with F/W
    uint64_t *pool_key;  // [P]
    uint32_t *mc_stamp;  // [P]
    int32_t *touched;    // [2][slots] slot indices, by update parity
    int32_t *mclist;     // [2][P] pool indices of an update's MC set, by update parity
    uint64_t *log;       // [L] (frame << 32) | pool
    int64_t *prefix;     // [max_chunks + 1] scratch of the paged walk
    unsigned long long *partial;  // [kMaxPartials] per-workgroup statistics, reduced later
    uint2 *PIX;          // [H*W] the current frame's pixels as written by the allocation kernel:
                         // x = depth bits, y = r | g << 8 | b << 16 (0 without colour)
    int64_t pool_cap;
    uint64_t log_cap;
    Counters *C;
};

// Camera, pose and volume constants of one frame.
struct Frame {
    float P[12];  // camera-to-world, row-major [R|t]
    float fx, fy, cx, cy;
    int W, H;
    float dmin, dmax;
    float dlo;  // max(dmin, 2^-149): d >= dlo is d > 0 && d >= dmin (NaN fails both)
    float vs, mu;
    int m_band;
    int fast_div;  // 1: coordinates and focal lengths admit the reciprocal-based quotient
    int fast_bs;   // 1: band-sample world coordinates and the block size admit it in allocation
                   // (2: also for coordinates below 2^-90, as bs <= 1)
    int local_keys;  // 1: every band sample's block B satisfies 0 <= B - kb < 1024 per axis
    int kb[3];       // base of the allocation's 32-bit tile-local keys (block coordinates)
    uint32_t kb_packed;  // (kb_x << 20) + (kb_y << 10) + kb_z modulo 2^32
};

// The touched list and MC list of update `seq`: double-buffered, so that the allocation
// of one update may run while the previous update's integration and extraction read
// theirs.
__device__ __forceinline__ int32_t *touched_of(const Dev &S, int seq) {
    return S.touched + int64_t(seq & 1) * int64_t(S.mask + 1);
}
__device__ __forceinline__ int32_t *mclist_of(const Dev &S, int seq) {
    return S.mclist + int64_t(seq & 1) * S.pool_cap;
}

// The depth validity rule: positive and inside [dmin, dmax] (float32 tests; the smallest
// positive float 2^-149 folds the sign test into the lower bound).
__device__ __forceinline__ bool depth_valid(float d, const Frame &f) {
    return d >= f.dlo && d <= f.dmax;
}

}  // namespace vbh

// Host-side handle of a scene.
struct vbh_scene {
    uint32_t tag = vbh::kTagScene;  // handle kind, read by vbh_status
    vbh_params p{};
    int m_band = 0;
    vbh::Dev d{};
    vbh::Counters *C = nullptr;
    unsigned long long *hostbuf = nullptr;  // device staging for counters
    int64_t max_chunks = 0;
    int seq = 0;        // number of updates so far (ring index of the next one)
    int cus = 256;      // compute units of the device the scene lives on
    unsigned g_int = 0;  // workgroups of the integration launch: as many as are resident at once
    unsigned g_ext = 0;  // workgroups of the extraction launch, likewise
    uint32_t last_frame = 0;
    void *mem[15] = {};
    int timing_period = 0;  // time the kernels of every n-th update (0: off)
    // the host-input multi-frame form's two device frame buffers (depth then colour),
    // allocated on first use
    void *up_buf[2] = {};
    std::vector<vbh::StageTimer> ev_pending, ev_free;
};


namespace vbh {
// Camera/volume constants for one frame with pose `pose` (row-major 3x4, camera to world).
Frame make_frame(const vbh_scene *s, const float *pose);
// Enqueues band allocation and integration of one frame (and, if with_mc, the MC update
// and log) as update `frame` of the scene; the caller validated the arguments.
int scene_fuse(vbh_scene *s, const float *d_depth, const uint8_t *d_rgb, const float *pose, uint32_t frame,
               bool with_mc, hipStream_t st);
// Enqueues n consecutive frames (depth [n][H][W], rgb [n][H][W][3] or null, host poses
// [n][12], ids first..first+n-1) with their MC updates, as n scene_fuse calls.
int scene_fuse_frames(vbh_scene *s, const float *d_depth, const uint8_t *d_rgb, const float *poses, uint32_t first,
                      int64_t n, hipStream_t st);
// The same for frames in host memory: each frame is copied into one of two device buffers
// on `st` before its kernels.
int scene_fuse_frames_host(vbh_scene *s, const float *h_depth, const uint8_t *h_rgb, const float *poses,
                           uint32_t first, int64_t n, hipStream_t st);
// Enqueues only the band allocation of one frame (touched list, new blocks, no MC set) as
// update `frame`, for callers that compute the voxel state themselves.
int scene_alloc_only(vbh_scene *s, const float *d_depth, const float *pose, uint32_t frame, hipStream_t st);
// Enqueues the MC update (update-set marking, MC voxels, stamps, log) of the scene's last
// update, which must have been fused with with_mc = false as update `frame`.
int scene_mc_update(vbh_scene *s, uint32_t frame, hipStream_t st);
// Empties the scene (table, used pool blocks, stamps, log, counters) on `st`.
int scene_reset(vbh_scene *s, hipStream_t st);
}  // namespace vbh
