// Voxel block hashing volume with the server's MC voxel representation (Sec. 4.1-4.2):
// band allocation, TSDF fusion, MC voxel extraction, update log - kernels and C ABI.
//
// Every discrete decision (band-sample block keys, voxel->pixel index, depth validity,
// the -trunc skip) is computed in IEEE float32 in the operation order written in the
// comments, with contraction off and correctly rounded division, so its outcome is fully
// determined by the float32 inputs.
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <cstring>
#include <new>
#include <vector>

#include "fastdiv.hpp"
#include "scene.hpp"

using namespace vbh;

namespace {


// Blocks in the MC update set of the update whose counters are fc (valid once its
// marking has finished).
__device__ __forceinline__ int64_t update_set_size(const FrameCounters &fc) { return int64_t(fc.n_mc); }

// Starts update `seq`: clears the counters two updates ahead in the ring and records
// where this update's log segment begins: after the previous update's segment, whose size
// is final once that update's allocation (or marking) kernel has finished, even while its
// extraction kernel, which writes the segment, still runs.  Called by exactly one thread.
__device__ __forceinline__ void begin_update(const Dev &S, int seq) {
    FrameCounters z = {};
    S.C->fc[(seq + 2) & (kRing - 1)] = z;
    const FrameCounters &prev = S.C->fc[(seq - 1) & (kRing - 1)];
    S.C->fc[seq & (kRing - 1)].log_base = seq > 0 ? prev.log_base + prev.n_mc : S.C->log_len;
}

// Workgroup staging buffer for list appends: waves reserve space with one LDS atomic,
// and the workgroup claims global space with one atomic per flush.
template <int CAP>
struct StageBuf {
    int32_t item[CAP];
    unsigned int count;
    unsigned long long base;
};

template <int CAP>
__device__ __forceinline__ void stage_reset(StageBuf<CAP> &b) {
    if (threadIdx.x == 0) b.count = 0;
    __syncthreads();
}

// Every lane of every wave may call; lanes with `put` store `v`.
template <int CAP>
__device__ __forceinline__ void stage_put(StageBuf<CAP> &b, bool put, int32_t v) {
    const unsigned long long m = __ballot(put);
    if (!m) return;
    const int leader = __builtin_ctzll(m);
    unsigned int pos = 0;
    if (lane_id() == leader) pos = atomicAdd(&b.count, unsigned(__popcll(m)));
    pos = unsigned(__builtin_amdgcn_readlane(int(pos), leader));
    if (put) b.item[pos + unsigned(lanes_below(m))] = v;
}

// ---------------------------------------------------------------- MC update set
// Block B - e of a touched block B, e in {0,1}^3, joins the frame's MC update set (the
// touched blocks and their seven negative neighbours, Sec. 4.2) if it exists.  The first
// thread to raise its MC stamp appends it to the update's MC list; the extraction kernel
// later copies the list into the update log.
__device__ __forceinline__ bool try_mark(const Dev &S, int32_t target, uint32_t frame) {
    return target >= 0 && atomicMax(&S.mc_stamp[target], frame) < frame;
}

// Pool index of the block B - e (e in {0,1}^3 \ {0}) if it exists and its pool block is
// published, else -1.
__device__ __forceinline__ int32_t negative_neighbour(const Dev &S, int32_t bx, int32_t by, int32_t bz, int e) {
    const int32_t nx = bx - (e & 1), ny = by - ((e >> 1) & 1), nz = bz - ((e >> 2) & 1);
    if (!key_ok(nx, ny, nz)) return -1;
    const uint64_t nk = pack_key(nx, ny, nz);
    // the slot's key and value are read together at every probe step
    uint64_t p = home_slot(nx, ny, nz, nk, S.kind, S.mask);
    for (uint64_t n = 0; n <= S.mask; ++n) {
        const uint64_t k = ld_key(S.T + p);
        const int32_t v = __hip_atomic_load(&S.T[p].val, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (k == nk) return v >= 0 ? v : -1;
        if (k == kEmpty) return -1;
        p = (p + 1) & S.mask;
    }
    return -1;
}

// Appends the workgroup's staged MC-set blocks to the update's MC list (one atomic) and
// empties the buffer.  Called by every thread of the workgroup.
template <int CAP>
__device__ __forceinline__ void flush_mc(int32_t *mclist, FrameCounters *fc, StageBuf<CAP> &b) {
    __syncthreads();
    if (threadIdx.x == 0) b.base = b.count ? atomicAdd(&fc->n_mc, b.count) : 0u;
    __syncthreads();
    for (unsigned int k = threadIdx.x; k < b.count; k += blockDim.x) mclist[b.base + k] = b.item[k];
    __syncthreads();
    if (threadIdx.x == 0) b.count = 0;
    __syncthreads();
}

// ------------------------------------------------------------------ allocation
// One workgroup per 32x16-pixel tile, thread = pixel.  Each valid pixel takes 2m+1 band
// samples at camera depth lam = (d - mu) + s*vs:
//   xn = ((float)u - cx) / fx, yn = ((float)v - cy) / fy, pc = (lam*xn, lam*yn, lam),
//   pw_i = ((R_i0 pc_x + R_i1 pc_y) + R_i2 pc_z) + t_i,  B_i = floor(pw_i / (8 vs)).
// About a hundred samples of a tile fall into each block, so the keys are first made
// unique inside the workgroup: a sample whose key equals the pixel's previous sample or
// the same sample of the left or upper pixel of its 8x8 wave tile is dropped at once, and
// the rest go into an LDS hash set.  Only the tile's distinct keys then reach the global
// table, one thread each: its home slot's key and frame stamp are read together, absent
// keys are claimed with a CAS (and get pool blocks from one reservation per wave, issued
// together with the frame-stamp raise), and the thread that raises a block's frame stamp
// appends it to the touched list (one atomic per workgroup and round, shared with the
// MC-list space).
//
// With `mark`, the kernel also forms the update's MC set.  Blocks that existed before the
// frame are found by any probe (keys never move); a block allocated by this frame is
// touched, so it enters the set as a touched block whether or not a neighbour's probe
// saw it.  Hence: the appending thread of a touched block B marks B's existing negative
// neighbours and, if B's pool block is already known, B itself; the workgroup that claims
// a new block marks it in the same marking step.
//
constexpr int kAllocThreads = 512;  // 32x16 pixels: eight 8x8 wave tiles
constexpr int kSetSlots = 2048;     // LDS hash set of keys (load <= 1/2, see kListFlush)
constexpr int kListCap = 1024;      // distinct keys collected before they are processed
constexpr int kListFlush = kListCap - kAllocThreads;  // one sample step adds <= 512 keys
constexpr int kMcCap = 2048;        // staged MC-set blocks (flushed above kMcCap - 512
                                    // after each marking round of <= 512 items)

// Workgroup-shared state of the allocation.
struct AllocShared {
    unsigned long long set[kSetSlots];
    unsigned long long list[kListCap];
    int32_t appended[kListCap];
    uint16_t app_idx[kListCap];  // list index of each appended block
    int32_t app_pool[kListCap];  // its pool block if it still has to be marked, else -1
    int32_t self_pool[kListCap]; // pool blocks this workgroup claimed (marked by it)
    StageBuf<kMcCap> mcb;
    unsigned int n_list, n_app, n_self, n_new_wg;
    unsigned long long pool_base;
};

// A float that is integral and finite to int32, saturating (v_cvt_i32_f32 clamps to the
// int32 range), where a C++ conversion of an out-of-range value is undefined.
__device__ __forceinline__ int32_t cvt_sat_i32(float x) {
    int32_t r;
    asm("v_cvt_i32_f32 %0, %1" : "=v"(r) : "v"(x));
    return r;
}
// floor(x) as int32 in one instruction, for x whose floor is known to lie in int32 range.
__device__ __forceinline__ int32_t cvt_flr_i32(float x) {
    int32_t r;
    asm("v_cvt_flr_i32_f32 %0, %1" : "=v"(r) : "v"(x));
    return r;
}

__device__ __forceinline__ uint32_t set_hash(uint64_t k) {
    return uint32_t((k * 0x9E3779B97F4A7C15ull) >> 40);
}
__device__ __forceinline__ uint32_t set_hash(uint32_t k) { return (k * 0x9E3779B1u) >> 20; }

// The key of a sample from the lane-1 and lane-8 neighbours (DPP row shifts by 1 and 8
// within 16-lane rows); lanes without such a neighbour in their row read `old`.
template <int kCtrl>
__device__ __forceinline__ uint32_t row_shift(uint32_t v) {
    return uint32_t(__builtin_amdgcn_update_dpp(0, int(v), kCtrl, 0xf, 0xf, false));
}
template <int kCtrl>
__device__ __forceinline__ uint64_t row_shift(uint64_t v) {
    return uint64_t(row_shift<kCtrl>(uint32_t(v))) | uint64_t(row_shift<kCtrl>(uint32_t(v >> 32))) << 32;
}

// Block coordinates of a collected key: a 64-bit table key, or with local keys the 10-bit
// offsets (x << 20 | y << 10 | z) from the frame's base kb.
__device__ __forceinline__ void collected_coords(uint64_t k, const Frame &, int32_t &x, int32_t &y, int32_t &z) {
    unpack_key(k, x, y, z);
}
__device__ __forceinline__ void collected_coords(uint32_t k, const Frame &fr, int32_t &x, int32_t &y, int32_t &z) {
    x = int32_t(k >> 20) + fr.kb[0];
    y = int32_t((k >> 10) & 1023u) + fr.kb[1];
    z = int32_t(k & 1023u) + fr.kb[2];
}

// Allocation (and, with mark, MC-set marking) of the 32x16-pixel tile (tx, ty) for update
// seq.  Called by all kAllocThreads threads of a workgroup.  K is the collected key:
// uint64_t (table keys), or uint32_t when the host has shown that every band sample's
// block lies within [kb, kb + 1024) per axis (Frame::local_keys); the LDS set then holds
// twice as many 4-byte keys in the same bytes and no sample needs the key-range check.
template <class K>
__device__ __forceinline__ void alloc_tile(const Dev &S, const Frame &fr, const float *__restrict__ depth,
                                           const uint8_t *__restrict__ rgb, uint32_t frame, int seq, int mark, int tx,
                                           int ty, AllocShared &sh) {
    constexpr bool kLocal = sizeof(K) == 4;
    constexpr K kNone = K(~K(0));
    constexpr int kSlotsK = kSetSlots * int(8 / sizeof(K));
    K *set = reinterpret_cast<K *>(sh.set);
    K *list = reinterpret_cast<K *>(sh.list);
    int32_t *appended = sh.appended;
    uint16_t *app_idx = sh.app_idx;
    int32_t *app_pool = sh.app_pool;
    StageBuf<kMcCap> &mcb = sh.mcb;
    int32_t *self_pool = sh.self_pool;
    unsigned int &n_list = sh.n_list, &n_app = sh.n_app, &n_self = sh.n_self, &n_new_wg = sh.n_new_wg;
    unsigned long long &pool_base = sh.pool_base;
    FrameCounters *fc = &S.C->fc[seq & (kRing - 1)];
    if (tx == 0 && ty == 0 && threadIdx.x == 0) begin_update(S, seq);
    for (int i = threadIdx.x; i < kSlotsK; i += kAllocThreads) set[i] = kNone;
    if (threadIdx.x == 0) {
        n_list = 0;
        n_app = 0;
        n_self = 0;
        n_new_wg = 0;
        mcb.count = 0;
    }
    const int lane = lane_id();
    const int wave = threadIdx.x >> 6;
    const int lx = lane & 7, ly = lane >> 3;
    const int u = (tx * 4 + (wave & 3)) * 8 + lx;
    const int v = (ty * 2 + (wave >> 2)) * 8 + ly;
    const bool inb = u < fr.W && v < fr.H;
    const uint32_t pix = inb ? uint32_t(v * fr.W + u) : 0u;
    const float d = inb ? depth[pix] : 0.0f;
    if (inb) {  // the pixel record that integration gathers: depth and colour in 8 bytes
        uint32_t c = 0u;
        if (rgb) c = uint32_t(rgb[3 * pix]) | uint32_t(rgb[3 * pix + 1]) << 8 | uint32_t(rgb[3 * pix + 2]) << 16;
        S.PIX[pix] = make_uint2(__float_as_uint(d), c);
    }
    const bool valid = inb && depth_valid(d, fr);
    const bool wave_any = __ballot(valid) != 0;  // uniform per wave
    const float xn = (float(u) - fr.cx) / fr.fx;
    const float yn = (float(v) - fr.cy) / fr.fy;
    const float bs = 8.0f * fr.vs;
    const float ybs = refine_rcp(bs, __builtin_amdgcn_rcpf(bs));
    const int n_samples = 2 * fr.m_band + 1;
    K prev = kNone;
    __syncthreads();
    for (int s = 0; s < n_samples; ++s) {  // workgroup-uniform
        if (wave_any) {
            const float lam = (d - fr.mu) + float(s) * fr.vs;
            bool ok = valid && lam > 0.0f;
            K key = kNone;
            if (ok) {
                const float pc[3] = {lam * xn, lam * yn, lam};
                float pw[3], q[3];
#pragma unroll
                for (int c = 0; c < 3; ++c)
                    pw[c] = ((fr.P[c * 4 + 0] * pc[0] + fr.P[c * 4 + 1] * pc[1]) + fr.P[c * 4 + 2] * pc[2]) +
                            fr.P[c * 4 + 3];
                // wave-uniform: the reciprocal-based quotient (the host bounds the coordinates
                // above); with fast_bs 1, not for a wave where some sample has a world
                // coordinate below its range; with fast_bs 2 (bs <= 1) such a coordinate's
                // quotient still has the floor of the true one, so every wave takes it
                bool full = fr.fast_bs == 0;
                if (fr.fast_bs == 1) {
                    const float small = fminf(fminf(fabsf(pw[0]), fabsf(pw[1])), fabsf(pw[2]));
                    full = __ballot(small < 0x1p-90f) != 0ull;
                }
                if (full) {
#pragma unroll
                    for (int c = 0; c < 3; ++c) q[c] = pw[c] / bs;
                } else {
#pragma unroll
                    for (int c = 0; c < 3; ++c) q[c] = corrected_quotient(pw[c], bs, ybs);
                }
                if constexpr (kLocal) {  // 0 <= B - kb < 1024 per axis, B = floor(q): packed in 10 bits
                    key = ((uint32_t(cvt_flr_i32(q[0])) << 20) + (uint32_t(cvt_flr_i32(q[1])) << 10) +
                           uint32_t(cvt_flr_i32(q[2]))) - fr.kb_packed;
                } else {
#pragma unroll
                    for (int c = 0; c < 3; ++c) q[c] = floorf(q[c]);
                    int32_t B[3];
#pragma unroll
                    for (int c = 0; c < 3; ++c) {
                        if (!(q[c] >= -1048576.0f && q[c] < 1048576.0f)) ok = false;
                        B[c] = ok ? int32_t(q[c]) : 0;
                    }
                    if (ok)
                        key = pack_key(B[0], B[1], B[2]);
                    else
                        raise_err(&S.C->err, kErrKeyRange);
                }
            }
            // lane - 1 (row_shr:1) and lane - 8 (row_shr:8, within a 16-lane row, so only odd
            // pixel rows compare with the row above); a filter only: the set removes the rest
            const K left = row_shift<0x111>(key);
            const K up = row_shift<0x118>(key);
            const bool dup = key == prev || (lx > 0 && key == left) || ((ly & 1) && key == up);
            prev = ok ? key : kNone;
            bool fresh = false;
            if (ok && !dup) {  // insert into the workgroup's set; the inserting thread owns the key
                uint32_t h = set_hash(key) & uint32_t(kSlotsK - 1);
                for (int n = 0; n < kSlotsK; ++n) {
                    const K old = atomicCAS(&set[h], kNone, key);
                    if (old == kNone) {
                        fresh = true;
                        break;
                    }
                    if (old == key) break;
                    h = (h + 1) & uint32_t(kSlotsK - 1);
                }
            }
            // the compiler turns the wave's LDS atomics on one address into one atomic and
            // each lane's rank among the active lanes
            if (fresh) list[atomicAdd(&n_list, 1u)] = key;
        }
        __syncthreads();
        const unsigned int nl = n_list;
        __syncthreads();  // every thread has read n_list before it changes again
        if (nl <= unsigned(kListFlush) && s + 1 < n_samples) continue;  // uniform
        // the collected distinct keys against the global table, one thread per key
        for (unsigned int r = 0; r < nl; r += kAllocThreads) {  // uniform
            const unsigned int i = r + threadIdx.x;
            int32_t slot = -1, pool = -1;  // pool: the block's pool index if known, else -1
            bool claimed = false, stamp_now = false;
            uint64_t key = kEmpty;
            if (i < nl) {
                int32_t x, y, z;
                collected_coords(list[i], fr, x, y, z);
                key = pack_key(x, y, z);
                const uint32_t home = uint32_t(home_slot(x, y, z, key, S.kind, S.mask));
                const uint64_t first = ld_key(S.T + home);
                const int32_t hv = __hip_atomic_load(&S.T[home].val, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                const uint32_t st = __hip_atomic_load(&S.T[home].stamp, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                if (first == key) {
                    slot = int32_t(home);
                    stamp_now = st == frame;  // already touched by this frame
                    pool = hv >= 0 ? hv : -1;
                } else {
                    slot = int32_t(probe_claim(S.T, S.mask, key, home, claimed));
                    if (slot < 0) {
                        raise_err(&S.C->err, kErrTableFull);
                    } else if (!claimed && mark) {
                        const int32_t v = __hip_atomic_load(&S.T[slot].val, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                        pool = v >= 0 ? v : -1;
                    }
                }
            }
            // A claimed key's pool block (one reservation per wave that claims) and every
            // found key's frame stamp are requested together: neither waits for the other.
            const unsigned long long cm = __ballot(claimed);
            unsigned long long pb = 0;
            if (cm && lane == __builtin_ctzll(cm)) {
                pb = atomicAdd(&S.C->pool_next, (unsigned long long)__popcll(cm));
                atomicAdd(&n_new_wg, unsigned(__popcll(cm)));  // LDS
            }
            const bool raise = slot >= 0 && !stamp_now;
            const uint32_t old_stamp = raise ? atomicMax(&S.T[slot].stamp, frame) : frame;
            if (cm) {
                {
                    const int cl = __builtin_ctzll(cm);
                    pb = (unsigned long long)(unsigned(__builtin_amdgcn_readlane(int(pb), cl))) |
                         (unsigned long long)(unsigned(__builtin_amdgcn_readlane(int(pb >> 32), cl))) << 32;
                    pb += (unsigned long long)lanes_below(cm);
                }
                if (claimed) {
                    if (int64_t(pb) < S.pool_cap) {
                        S.pool_key[pb] = key;
                        st_val(S.T + slot, int32_t(pb));
                        pool = int32_t(pb);
                    } else {
                        st_val(S.T + slot, kNoPool);
                        raise_err(&S.C->err, kErrPoolFull);
                    }
                }
                // a new block is marked by its claimer (in the marking step below)
                const bool self = mark && claimed && pool >= 0;
                const unsigned long long sm = __ballot(self);
                if (sm) {
                    const int leader = __builtin_ctzll(sm);
                    unsigned int p0 = 0;
                    if (lane == leader) p0 = atomicAdd(&n_self, unsigned(__popcll(sm)));
                    p0 = unsigned(__builtin_amdgcn_readlane(int(p0), leader));
                    if (self) self_pool[p0 + unsigned(lanes_below(sm))] = pool;
                }
            }
            const bool app = raise && old_stamp < frame;
            const unsigned long long m = __ballot(app);
            if (m) {
                const int leader = __builtin_ctzll(m);
                unsigned int p0 = 0;
                if (lane == leader) p0 = atomicAdd(&n_app, unsigned(__popcll(m)));
                p0 = unsigned(__builtin_amdgcn_readlane(int(p0), leader));
                if (app) {
                    const unsigned int q = p0 + unsigned(lanes_below(m));
                    appended[q] = slot;
                    app_idx[q] = uint16_t(i);
                    app_pool[q] = claimed ? -1 : pool;
                }
            }
        }
        __syncthreads();
        if (mark) {  // uniform: MC-set marking, thread per (appended block, e in {0,1}^3) and
                     // per block this workgroup claimed
            const unsigned int n8 = n_app * 8u, items = n8 + n_self;
            for (unsigned int r = 0; r < items; r += kAllocThreads) {
                const unsigned int it = r + threadIdx.x;
                int32_t target = -1;
                if (it < n8) {
                    const unsigned int b = it >> 3, e = it & 7u;
                    if (e == 0) {
                        target = app_pool[b];
                    } else {
                        int32_t x, y, z;
                        collected_coords(list[app_idx[b]], fr, x, y, z);
                        target = negative_neighbour(S, x, y, z, int(e));
                    }
                } else if (it < items) {
                    target = self_pool[it - n8];
                }
                stage_put(mcb, try_mark(S, target, frame), target);
                __syncthreads();
                const unsigned int c = mcb.count;
                __syncthreads();  // every thread has read the count before it changes again
                if (c > unsigned(kMcCap - kAllocThreads)) flush_mc(mclist_of(S, seq), fc, mcb);
            }
            __syncthreads();
        }
        // touched-list space and the rest of the MC-list space in one 64-bit atomic (the two
        // counts share a word); the new-block count needs no reply
        if (threadIdx.x == 0) {
            const unsigned int nm = mark ? mcb.count : 0u;
            const unsigned long long add = (unsigned long long)nm << 32 | n_app;
            const unsigned long long old =
                add ? atomicAdd(reinterpret_cast<unsigned long long *>(&fc->n_touched), add) : 0ull;
            pool_base = old & 0xFFFFFFFFull;  // reused as the touched-list base
            mcb.base = old >> 32;
            if (n_new_wg) atomicAdd(&fc->n_new, n_new_wg);
            n_new_wg = 0;
        }
        __syncthreads();
        for (unsigned int i = threadIdx.x; i < n_app; i += kAllocThreads) touched_of(S, seq)[pool_base + i] = appended[i];
        if (mark) {
            int32_t *mcl = mclist_of(S, seq);
            for (unsigned int k = threadIdx.x; k < mcb.count; k += kAllocThreads) mcl[mcb.base + k] = mcb.item[k];
        }
        if (s + 1 < n_samples) {  // start a new collection
            for (int i = threadIdx.x; i < kSlotsK; i += kAllocThreads) set[i] = kNone;
            prev = kNone;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            n_list = 0;
            n_app = 0;
            n_self = 0;
            mcb.count = 0;
        }
        __syncthreads();
    }
}

template <class K>
__global__ void __launch_bounds__(kAllocThreads) k_alloc(Dev S, Frame fr, const float *__restrict__ depth,
                                                         const uint8_t *__restrict__ rgb, uint32_t frame, int seq,
                                                         int mark) {
    __shared__ AllocShared sh;
    alloc_tile<K>(S, fr, depth, rgb, frame, seq, mark, int(blockIdx.x), int(blockIdx.y), sh);
}

__device__ __forceinline__ uint64_t first_lane64(uint64_t v) {
    const uint32_t lo = uint32_t(__builtin_amdgcn_readfirstlane(int(uint32_t(v))));
    const uint32_t hi = uint32_t(__builtin_amdgcn_readfirstlane(int(uint32_t(v >> 32))));
    return uint64_t(hi) << 32 | lo;
}

// ----------------------------------------------------------------- integration
// One wave per touched block; lane = lx + 8 ly handles voxels (lx, ly, lz), lz = 0..7.
//   pw_i = (float)g_i * vs, dl_i = pw_i - t_i, pc_j = (R_0j dl_0 + R_1j dl_1) + R_2j dl_2;
//   skip if pc_z <= 0; u = floor((fx (pc_x / pc_z) + cx) + 0.5) (same for v); skip if
//   outside the image; skip unless the pixel depth d is valid; sdf = d - pc_z; skip if
//   sdf < -mu.  Then F <- (W F + min(sdf, mu)) / (W + 1), W <- min(W + 1, 255) and each
//   colour channel c <- (W c + c_obs + floor(n / 2)) / n with n = W + 1.

// The eight voxels (lx, ly, 0..7) of a lane are projected first, then their pixel records
// (depth and colour, 8 bytes, written by the allocation kernel) are gathered together,
// then the TSDF state of the passing voxels is loaded together; the slot of the wave's
// next block is fetched while the current one is processed.  Offsets from wave-uniform
// bases are 32-bit, so the loads take a scalar base plus a vector offset.
template <bool kRgb>
__global__ void __launch_bounds__(kBlock) k_integrate(Dev S, Frame fr, int seq, int timed) {
    const FrameCounters *fc = &S.C->fc[seq & (kRing - 1)];
    const int64_t n = fc->n_touched;
    if (timed && blockIdx.x == 0 && threadIdx.x == 0) {  // the work of a timed update
        atomicAdd(&S.C->timed_touched, (unsigned long long)n);
        atomicAdd(&S.C->timed_mc, (unsigned long long)fc->n_mc);
    }
    const int lane = lane_id();
    const int lx = lane & 7, ly = lane >> 3;
    const int64_t gw = int64_t(blockIdx.x) * kWaves + (threadIdx.x >> 6);
    const int64_t nw = int64_t(gridDim.x) * kWaves;
    const int32_t *touched = touched_of(S, seq);
    const uint2 *__restrict__ pixrec = S.PIX;
    unsigned long long updates = 0;
    Slot cur = {};
    if (gw < n) cur = S.T[touched[gw]];
    for (int64_t t = gw; t < n; t += nw) {
        const int32_t next_idx = t + nw < n ? touched[t + nw] : -1;
        // every lane loaded the same slot: make it wave-uniform (scalar registers)
        const int32_t pool = __builtin_amdgcn_readfirstlane(cur.val);
        int32_t bx, by, bz;
        unpack_key(first_lane64(cur.key), bx, by, bz);
        const float dlx = float(8 * bx + lx) * fr.vs - fr.P[3];
        const float dly = float(8 * by + ly) * fr.vs - fr.P[7];
        float *const Fb = S.F + int64_t(pool) * 512;  // wave-uniform block bases
        uint32_t *const Wb = S.WRGB + int64_t(pool) * 512;
        int32_t pix[8];
        float pz[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const float dlz = float(8 * bz + j) * fr.vs - fr.P[11];
            const float pcx = (fr.P[0] * dlx + fr.P[4] * dly) + fr.P[8] * dlz;
            const float pcy = (fr.P[1] * dlx + fr.P[5] * dly) + fr.P[9] * dlz;
            const float pcz = (fr.P[2] * dlx + fr.P[6] * dly) + fr.P[10] * dlz;
            pz[j] = pcz;
            pix[j] = -1;
            if (pool >= 0 && pcz > 0.0f) {
                if (fr.fast_div && pcz >= 0x1p-32f) {  // one reciprocal for both quotients
                    const float y = refine_rcp(pcz, __builtin_amdgcn_rcpf(pcz));
                    const float qx = corrected_quotient(pcx, pcz, y);
                    const float qy = corrected_quotient(pcy, pcz, y);
                    // |pc| <= 2^32, pc_z >= 2^-32 and |fx|, |fy| <= 2^20 keep fu, fv finite, so
                    // the saturating conversion and one unsigned compare per axis decide
                    // 0 <= fu < W and 0 <= fv < H
                    const int32_t iu = cvt_sat_i32(floorf((fr.fx * qx + fr.cx) + 0.5f));
                    const int32_t iv = cvt_sat_i32(floorf((fr.fy * qy + fr.cy) + 0.5f));
                    if (uint32_t(iu) < uint32_t(fr.W) && uint32_t(iv) < uint32_t(fr.H))
                        pix[j] = int32_t(__umul24(uint32_t(iv), uint32_t(fr.W)) + uint32_t(iu));
                } else {
                    const float fu = floorf((fr.fx * (pcx / pcz) + fr.cx) + 0.5f);
                    const float fv = floorf((fr.fy * (pcy / pcz) + fr.cy) + 0.5f);
                    if (fu >= 0.0f && fu < float(fr.W) && fv >= 0.0f && fv < float(fr.H))
                        pix[j] = int32_t(__umul24(uint32_t(fv), uint32_t(fr.W)) + uint32_t(fu));
                }
            }
        }
        // a voxel outside the image reads pixel 0 (any valid address) and is dropped below
        uint2 rec[8];
#pragma unroll
        for (int j = 0; j < 8; ++j)
            rec[j] = *reinterpret_cast<const uint2 *>(reinterpret_cast<const char *>(pixrec) +
                                                      (uint32_t(pix[j] >= 0 ? pix[j] : 0) << 3));
        const Slot nxt = next_idx >= 0 ? S.T[next_idx] : Slot{};
        bool ok[8];
        float d[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            d[j] = __uint_as_float(rec[j].x);
            ok[j] = pix[j] >= 0 && depth_valid(d[j], fr) && !(d[j] - pz[j] < -fr.mu);
        }
        const uint32_t col = pool >= 0 ? S.SGN[int64_t(pool) * 64 + lane] : 0u;  // this lane's column
        float F[8];
        uint32_t w[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            F[j] = 0.0f;
            w[j] = 0u;
            if (ok[j]) {
                F[j] = Fb[uint32_t(lane + 64 * j)];
                w[j] = Wb[uint32_t(lane + 64 * j)];
            }
        }
        float Fn[8];
        uint32_t Wn[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) {  // branch-free: computed for every voxel, stored if ok
            // n = W + 1 observations (256 once W saturates at 255); 1/n from the hardware
            // reciprocal (relative error below 2^-22)
            const float tsdf = fminf(d[j] - pz[j], fr.mu);
            const uint32_t w_old = w[j] & 0xFFu;
            const float wf = float(w_old);
            const float inv = __builtin_amdgcn_rcpf(wf + 1.0f);
            Fn[j] = fmaf(wf, F[j], tsdf) * inv;
            uint32_t out = min(w_old + 1u, 255u);
            if constexpr (kRgb) {
                // c <- floor((W c + c_obs + floor(n/2)) / n), taken as the truncation of
                // fma(W c + c_obs, 1/n, (floor(n/2) + 1/2) / n).  W c + c_obs is an integer
                // below 2^17, exact in float.  The true value (W c + c_obs + floor(n/2) + 1/2) / n
                // lies at least 1/(2n) >= 1/512 away from an integer and below 256; the computed
                // one is off by at most 256 (2^-22 + 2^-23) + 2^-24 < 1/512 (reciprocal, product
                // and sum errors), so truncation gives the exact floor.
                const float hinv = (float((w_old + 1u) >> 1) + 0.5f) * inv;
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    const float cur_c = float((w[j] >> (8 * (c + 1))) & 0xFFu);
                    const float obs_c = float((rec[j].y >> (8 * c)) & 0xFFu);
                    const float num = fmaf(wf, cur_c, obs_c);
                    out |= uint32_t(fmaf(num, inv, hinv)) << (8 * (c + 1));
                }
            } else {
                out |= w[j] & 0xFFFFFF00u;
            }
            Wn[j] = out;
        }
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            if (ok[j]) {
                Fb[uint32_t(lane + 64 * j)] = Fn[j];
                Wb[uint32_t(lane + 64 * j)] = Wn[j];
            }
        }
        // updated voxels replace their sign/observed bits (W >= 1 after an update)
        uint32_t upd = 0, bits = 0;
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            upd |= uint32_t(ok[j]) * (0x101u << j);
            bits |= uint32_t(ok[j] && Fn[j] < 0.0f) << j;
            bits |= uint32_t(ok[j] && Fn[j] == Fn[j]) << (8 + j);
        }
        updates += uint32_t(__popc(upd & 0xFFu));
        if (upd) S.SGN[int64_t(pool) * 64 + lane] = uint16_t((col & ~upd) | bits);
        cur = nxt;
    }
    __shared__ unsigned long long wg_updates;
    if (threadIdx.x == 0) wg_updates = 0;
    __syncthreads();
    updates = wave_sum(updates);
    if (lane == 0 && updates) atomicAdd(&wg_updates, updates);  // LDS atomic
    __syncthreads();
    if (threadIdx.x == 0) S.partial[blockIdx.x] = wg_updates;
}

// Stand-alone MC-set marking for updates fused without it (the serving loop fuses a
// frame first and runs its MC update later): thread per (touched block, e in {0,1}^3),
// appends staged per workgroup in LDS and claimed with one atomic per flush.
constexpr int kMarkThreads = 1024;
__global__ void __launch_bounds__(kMarkThreads) k_mc_mark(Dev S, uint32_t frame, int seq) {
    constexpr int kCap = 4 * kMarkThreads;
    __shared__ StageBuf<kCap> mb;
    FrameCounters *fc = &S.C->fc[seq & (kRing - 1)];
    const int64_t total = int64_t(fc->n_touched) * 8;
    const int64_t stride = int64_t(gridDim.x) * kMarkThreads;
    stage_reset(mb);
    for (int64_t b0 = int64_t(blockIdx.x) * kMarkThreads; b0 < total; b0 += stride) {  // uniform per workgroup
        const int64_t i = b0 + threadIdx.x;
        int32_t target = -1;
        if (i < total) {
            const Slot *sl = S.T + touched_of(S, seq)[i >> 3];
            const int32_t pool = sl->val;
            const int e = int(i & 7);
            if (pool >= 0) {
                if (e == 0) {
                    target = pool;
                } else {
                    int32_t bx, by, bz;
                    unpack_key(sl->key, bx, by, bz);
                    target = negative_neighbour(S, bx, by, bz, e);
                }
            }
        }
        stage_put(mb, try_mark(S, target, frame), target);
        __syncthreads();
        const unsigned int c = mb.count;
        __syncthreads();  // every thread has read the count before it changes again
        if (c > unsigned(kCap - kMarkThreads) || b0 + stride >= total) flush_mc(mclist_of(S, seq), fc, mb);
    }
}

// ------------------------------------------------------------- MC extraction
// One wave per block, lane = cell column (x, y), working on the blocks' sign/observed
// columns rather than on their voxels.  A lane loads the columns (x + dx, y + dy),
// dx, dy in {0, 1}, from the block or its +x / +y / +x+y neighbours, and the z = 8 bit of
// each from the +z neighbours; the eight corner bits of its eight cells then come out of
// one 8x8 bit transpose.  Corners follow the Lorensen-Cline order; a cell with an
// unobserved corner, or a corner in a missing block, gets index 0; indices 0 and 255 are
// cut to 0 together with their colour.

// 8x8 bit-matrix transpose: bit c of byte r moves to bit r of byte c.
__device__ __forceinline__ uint64_t transpose8(uint64_t x) {
    uint64_t t;
    t = (x ^ (x >> 7)) & 0x00AA00AA00AA00AAull;
    x = x ^ t ^ (t << 7);
    t = (x ^ (x >> 14)) & 0x0000CCCC0000CCCCull;
    x = x ^ t ^ (t << 14);
    t = (x ^ (x >> 28)) & 0x00000000F0F0F0F0ull;
    x = x ^ t ^ (t << 28);
    return x;
}

// Computes the 512 MC voxels of block `pool` (key B) into out[j] for voxel lane + 64 j.
__device__ __forceinline__ void mc_block(const Dev &S, int32_t pool, uint64_t key, uint32_t (&out)[8]) {
    const int lane = lane_id();
    const int x = lane & 7, y = lane >> 3;
    int32_t bx, by, bz;
    unpack_key(key, bx, by, bz);
    // lane e in 1..7 finds neighbour B + (e & 1, e >> 1 & 1, e >> 2 & 1); each probe step
    // reads the slot's key and value together
    int32_t nb = pool;
    if (lane >= 1 && lane < 8) {
        nb = -1;
        const int32_t nx = bx + (lane & 1), ny = by + ((lane >> 1) & 1), nz = bz + ((lane >> 2) & 1);
        if (key_ok(nx, ny, nz)) {
            const uint64_t nk = pack_key(nx, ny, nz);
            uint64_t p = home_slot(nx, ny, nz, nk, S.kind, S.mask);
            for (uint64_t m = 0; m <= S.mask; ++m) {
                const uint64_t k = ld_key(S.T + p);
                const int32_t v = __hip_atomic_load(&S.T[p].val, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                if (k == nk) {
                    nb = v;
                    break;
                }
                if (k == kEmpty) break;
                p = (p + 1) & S.mask;
            }
        }
    }
    int32_t nbs[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) nbs[e] = __builtin_amdgcn_readlane(nb, e);
    // columns (x, y), (x + 1, y), (x + 1, y + 1), (x, y + 1): corners 0..3 at z, 4..7 at z + 1
    uint32_t lo[4], hi[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        const int xx = x + (c == 1 || c == 2), yy = y + (c >= 2);
        const int e = (xx >> 3) | ((yy >> 3) << 1);
        const int o = (xx & 7) + 8 * (yy & 7);
        const int32_t pl = e == 0 ? nbs[0] : e == 1 ? nbs[1] : e == 2 ? nbs[2] : nbs[3];
        const int32_t pu = e == 0 ? nbs[4] : e == 1 ? nbs[5] : e == 2 ? nbs[6] : nbs[7];
        // unconditional loads (a missing block reads pool block 0) keep the loads of the
        // eight columns free of branches
        const uint32_t vl = S.SGN[int64_t(pl >= 0 ? pl : 0) * 64 + o];
        const uint32_t vu = S.SGN[int64_t(pu >= 0 ? pu : 0) * 64 + o];
        lo[c] = pl >= 0 ? vl : 0u;
        hi[c] = pu >= 0 ? vu : 0u;
    }
    uint32_t neg[4], obs[4];  // 9-bit columns, z = 0..8
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        neg[c] = (lo[c] & 0xFFu) | (hi[c] & 1u) << 8;
        obs[c] = (lo[c] >> 8) | ((hi[c] >> 8) & 1u) << 8;
    }
    // byte k = corner k's bits over the lane's eight cells (bit j = cell z = j)
    const uint64_t rows = uint64_t((neg[0] & 0xFFu) | (neg[1] & 0xFFu) << 8 | (neg[2] & 0xFFu) << 16 |
                                   (neg[3] & 0xFFu) << 24) |
                          uint64_t((neg[0] >> 1) | (neg[1] >> 1) << 8 | (neg[2] >> 1) << 16 | (neg[3] >> 1) << 24)
                              << 32;
    const uint64_t idx = transpose8(rows);  // byte j = case index of cell z = j
    const uint32_t all_obs = obs[0] & obs[1] & obs[2] & obs[3];
    const uint32_t any_neg = neg[0] | neg[1] | neg[2] | neg[3];
    const uint32_t all_neg = neg[0] & neg[1] & neg[2] & neg[3];
    const uint32_t keep = all_obs & (all_obs >> 1) & (any_neg | (any_neg >> 1)) & ~(all_neg & (all_neg >> 1));
    uint32_t colour[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) colour[j] = S.WRGB[int64_t(pool) * 512 + lane + 64 * j];
#pragma unroll
    for (int j = 0; j < 8; ++j)
        out[j] = (keep >> j) & 1u ? (uint32_t(idx >> (8 * j)) & 0xFFu) | (colour[j] & 0xFFFFFF00u) : 0u;
}

// Per-frame form: MC list -> MC pool, and the MC list appended to the update log as
// entries (frame << 32 | pool) at [log_base, log_base + n).
// Workgroup 0 also folds the integration kernel's n_partials per-workgroup voxel counts
// into the update's statistics and advances the log length.
// Workgroup wg of n_wg (kBlock threads) of the extraction of update seq.
__device__ __forceinline__ void extract_wg(const Dev &S, int seq, int n_partials, uint32_t frame, int64_t wg,
                                           int64_t n_wg, unsigned long long *red) {
    FrameCounters &fcr = S.C->fc[seq & (kRing - 1)];
    const int64_t n = update_set_size(fcr);
    const unsigned long long log_base = fcr.log_base;
    if (wg == 0) {
        unsigned long long v = 0;
        for (int i = threadIdx.x; i < n_partials; i += kBlock) v += S.partial[i];
        v = wave_sum(v);
        if (lane_id() == 0) red[threadIdx.x >> 6] = v;
        __syncthreads();
        if (threadIdx.x == 0) {
            unsigned long long tot = 0;
            for (int w = 0; w < kWaves; ++w) tot += red[w];
            fcr.voxel_updates = tot;
            S.C->log_len = log_base + (unsigned long long)n;
            if (log_base + (unsigned long long)n > S.log_cap) raise_err(&S.C->err, kErrLogFull);
            S.C->tot_mc += n;
            S.C->tot_touched += fcr.n_touched;
            S.C->tot_voxel_updates += tot;
        }
    }
    const int lane = lane_id();
    const int64_t gw = wg * kWaves + (threadIdx.x >> 6);
    const int64_t nw = n_wg * kWaves;
    const int32_t *ml = mclist_of(S, seq);
    // each list entry and its key are fetched one block ahead
    int32_t pool = gw < n ? ml[gw] : 0;
    uint64_t key = gw < n ? S.pool_key[pool] : 0ull;
    for (int64_t t = gw; t < n; t += nw) {
        const int64_t tn = t + nw;
        const int32_t npool = tn < n ? ml[tn] : 0;
        if (lane == 0 && log_base + t < S.log_cap) S.log[log_base + t] = (uint64_t(frame) << 32) | uint32_t(pool);
        uint32_t out[8];
        mc_block(S, pool, key, out);
        const uint64_t nkey = tn < n ? S.pool_key[npool] : 0ull;
#pragma unroll
        for (int j = 0; j < 8; ++j) S.MCV[int64_t(pool) * 512 + lane + 64 * j] = out[j];
        pool = npool;
        key = nkey;
    }
}

__global__ void __launch_bounds__(kBlock) k_mc_extract(Dev S, int seq, int n_partials, uint32_t frame) {
    __shared__ unsigned long long red[kWaves];
    extract_wg(S, seq, n_partials, frame, blockIdx.x, gridDim.x, red);
}

// API form: keys -> uint8 index [n][512] and optional uint8 RGB [n][512][3].
__global__ void __launch_bounds__(kBlock) k_mc_keys(Dev S, const int32_t *__restrict__ keys, int64_t n, uint8_t *mc,
                                                    uint8_t *rgb) {
    const int lane = lane_id();
    const int64_t gw = int64_t(blockIdx.x) * kWaves + (threadIdx.x >> 6);
    const int64_t nw = int64_t(gridDim.x) * kWaves;
    for (int64_t t = gw; t < n; t += nw) {
        const int32_t x = keys[3 * t], y = keys[3 * t + 1], z = keys[3 * t + 2];
        int32_t pool = -1;
        if (key_ok(x, y, z)) {
            const uint64_t k = pack_key(x, y, z);
            const int64_t ps = probe_locate(S.T, S.mask, k, home_slot(x, y, z, k, S.kind, S.mask));
            if (ps >= 0) pool = S.T[ps].val;
        }
        uint32_t out[8] = {0, 0, 0, 0, 0, 0, 0, 0};
        if (pool >= 0) mc_block(S, pool, pack_key(x, y, z), out);
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const int64_t o = t * 512 + lane + 64 * j;
            mc[o] = uint8_t(out[j]);
            if (rgb) {
                rgb[3 * o] = uint8_t(out[j] >> 8);
                rgb[3 * o + 1] = uint8_t(out[j] >> 16);
                rgb[3 * o + 2] = uint8_t(out[j] >> 24);
            }
        }
    }
}

// ---------------------------------------------------------------- block I/O
__device__ __forceinline__ int32_t lookup_pool(const Dev &S, int32_t x, int32_t y, int32_t z) {
    if (!key_ok(x, y, z)) return -1;
    const uint64_t k = pack_key(x, y, z);
    const int64_t ps = probe_locate(S.T, S.mask, k, home_slot(x, y, z, k, S.kind, S.mask));
    return ps >= 0 ? S.T[ps].val : -1;
}

__global__ void __launch_bounds__(kBlock) k_read_blocks(Dev S, const int32_t *keys, int64_t n, float *F, uint8_t *W,
                                                        uint8_t *rgb, int32_t *found, int mcmode) {
    const int lane = lane_id();
    const int64_t gw = int64_t(blockIdx.x) * kWaves + (threadIdx.x >> 6);
    const int64_t nw = int64_t(gridDim.x) * kWaves;
    for (int64_t t = gw; t < n; t += nw) {
        const int32_t pool = lookup_pool(S, keys[3 * t], keys[3 * t + 1], keys[3 * t + 2]);
        if (found && lane == 0) found[t] = pool >= 0;
        for (int j = 0; j < 8; ++j) {
            const int64_t o = t * 512 + lane + 64 * j;
            const int64_t src = int64_t(pool) * 512 + lane + 64 * j;
            const uint32_t w = pool >= 0 ? (mcmode ? S.MCV[src] : S.WRGB[src]) : 0u;
            if (F) F[o] = pool >= 0 ? S.F[src] : 0.0f;
            if (W) W[o] = uint8_t(w);
            if (rgb) {
                rgb[3 * o] = uint8_t(w >> 8);
                rgb[3 * o + 1] = uint8_t(w >> 16);
                rgb[3 * o + 2] = uint8_t(w >> 24);
            }
        }
    }
}

// Thread per key: insert (allocating a pool block), stamp as touched by `frame`.
__global__ void __launch_bounds__(kBlock) k_load_claim(Dev S, const int32_t *keys, int64_t n, uint32_t frame, int seq) {
    FrameCounters *fc = &S.C->fc[seq & (kRing - 1)];
    if (blockIdx.x == 0 && threadIdx.x == 0) begin_update(S, seq);
    const int64_t stride = int64_t(gridDim.x) * kBlock;
    for (int64_t b = int64_t(blockIdx.x) * kBlock + (threadIdx.x & ~63); b < n; b += stride) {
        const int64_t i = b + lane_id();
        bool append = false, fresh = false;
        int64_t slot = -1;
        if (i < n) {
            const int32_t x = keys[3 * i], y = keys[3 * i + 1], z = keys[3 * i + 2];
            if (!key_ok(x, y, z)) {
                raise_err(&S.C->err, kErrKeyRange);
            } else {
                const uint64_t key = pack_key(x, y, z);
                bool claimed;
                slot = probe_claim(S.T, S.mask, key, home_slot(x, y, z, key, S.kind, S.mask), claimed);
                if (slot < 0) {
                    raise_err(&S.C->err, kErrTableFull);
                } else {
                    Slot *sl = S.T + slot;
                    if (claimed) {
                        fresh = true;
                        const unsigned long long pool = atomicAdd(&S.C->pool_next, 1ull);
                        if (int64_t(pool) < S.pool_cap) {
                            S.pool_key[pool] = key;
                            st_val(sl, int32_t(pool));
                        } else {
                            st_val(sl, kNoPool);
                            raise_err(&S.C->err, kErrPoolFull);
                        }
                    }
                    append = atomicMax(&sl->stamp, frame) < frame;
                }
            }
        }
        const unsigned int pos = wave_append<unsigned int>(append, &fc->n_touched);
        if (append) touched_of(S, seq)[pos] = int32_t(slot);
        const unsigned long long nm = __ballot(fresh);
        if (nm && lane_id() == __builtin_ctzll(nm)) atomicAdd(&fc->n_new, unsigned(__popcll(nm)));
    }
}

// Thread per pixel: the pixel records integration gathers (depth bits, colour), for
// updates whose blocks are not found by the allocation kernel.
__global__ void __launch_bounds__(kBlock) k_pix_pack(Dev S, int64_t hw, const float *__restrict__ depth,
                                                     const uint8_t *__restrict__ rgb) {
    for (int64_t p = int64_t(blockIdx.x) * kBlock + threadIdx.x; p < hw; p += int64_t(gridDim.x) * kBlock) {
        uint32_t c = 0u;
        if (rgb) c = uint32_t(rgb[3 * p]) | uint32_t(rgb[3 * p + 1]) << 8 | uint32_t(rgb[3 * p + 2]) << 16;
        S.PIX[p] = make_uint2(__float_as_uint(depth[p]), c);
    }
}

__global__ void __launch_bounds__(kBlock) k_load_copy(Dev S, const int32_t *keys, int64_t n, const float *F,
                                                      const uint8_t *W, const uint8_t *rgb) {
    const int lane = lane_id();
    const int64_t gw = int64_t(blockIdx.x) * kWaves + (threadIdx.x >> 6);
    const int64_t nw = int64_t(gridDim.x) * kWaves;
    for (int64_t t = gw; t < n; t += nw) {
        const int32_t pool = lookup_pool(S, keys[3 * t], keys[3 * t + 1], keys[3 * t + 2]);
        if (pool < 0) continue;
        uint32_t bits = 0;
        for (int j = 0; j < 8; ++j) {
            const int64_t i = t * 512 + lane + 64 * j;
            const int64_t o = int64_t(pool) * 512 + lane + 64 * j;
            uint32_t w = W[i];
            if (rgb) w |= uint32_t(rgb[3 * i]) << 8 | uint32_t(rgb[3 * i + 1]) << 16 | uint32_t(rgb[3 * i + 2]) << 24;
            const float f = F[i];
            S.F[o] = f;
            S.WRGB[o] = w;
            const bool seen = (w & 0xFFu) && f == f;
            bits |= uint32_t(seen && f < 0.0f) << j | uint32_t(seen) << (8 + j);
        }
        S.SGN[int64_t(pool) * 64 + lane] = uint16_t(bits);
    }
}

// ------------------------------------------------------------------ scene reset
// Reset (Sec. 4.1, quasi-static scenes): thread per listed key.  A key whose block exists
// is stamped as touched by `frame` and appended to the update's touched list, from which
// the MC update set (the block and its seven negative neighbours) is formed as for a
// fused frame; absent keys are skipped and nothing is allocated.
__global__ void __launch_bounds__(kBlock) k_reset_claim(Dev S, const int32_t *keys, int64_t n, uint32_t frame,
                                                        int seq) {
    FrameCounters *fc = &S.C->fc[seq & (kRing - 1)];
    if (blockIdx.x == 0 && threadIdx.x == 0) begin_update(S, seq);
    const int64_t stride = int64_t(gridDim.x) * kBlock;
    for (int64_t b = int64_t(blockIdx.x) * kBlock + (threadIdx.x & ~63); b < n; b += stride) {
        const int64_t i = b + lane_id();
        bool append = false;
        int64_t slot = -1;
        if (i < n) {
            const int32_t x = keys[3 * i], y = keys[3 * i + 1], z = keys[3 * i + 2];
            if (!key_ok(x, y, z)) {
                raise_err(&S.C->err, kErrKeyRange);
            } else {
                const uint64_t key = pack_key(x, y, z);
                slot = probe_locate(S.T, S.mask, key, home_slot(x, y, z, key, S.kind, S.mask));
                if (slot >= 0 && ld_val(S.T + slot) >= 0) append = atomicMax(&S.T[slot].stamp, frame) < frame;
            }
        }
        const unsigned int pos = wave_append<unsigned int>(append, &fc->n_touched);
        if (append) touched_of(S, seq)[pos] = int32_t(slot);
    }
}

// Wave per block of the update's touched list: distance, weight, colour and the sign /
// observed columns become zero, so the block reads as never observed.
__global__ void __launch_bounds__(kBlock) k_reset_clear(Dev S, int seq) {
    const int64_t n = S.C->fc[seq & (kRing - 1)].n_touched;
    const int32_t *touched = touched_of(S, seq);
    const int lane = lane_id();
    const int64_t gw = int64_t(blockIdx.x) * kWaves + (threadIdx.x >> 6);
    const int64_t nw = int64_t(gridDim.x) * kWaves;
    for (int64_t t = gw; t < n; t += nw) {
        const int64_t pool = S.T[touched[t]].val;
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            S.F[pool * 512 + lane + 64 * j] = 0.0f;
            S.WRGB[pool * 512 + lane + 64 * j] = 0u;
        }
        S.SGN[pool * 64 + lane] = 0;
    }
}

// Blocks whose central voxel, local (4, 4, 4), projects into the image at a valid depth
// (the float32 steps of integration); compacted in no particular order.
__global__ void __launch_bounds__(kBlock) k_visible(Dev S, Frame fr, int64_t cap, int32_t *out) {
    const unsigned long long pn = S.C->pool_next;
    const int64_t n = int64_t(pn) < S.pool_cap ? int64_t(pn) : S.pool_cap;
    const int64_t stride = int64_t(gridDim.x) * kBlock;
    for (int64_t b = int64_t(blockIdx.x) * kBlock + (threadIdx.x & ~63); b < n; b += stride) {
        const int64_t i = b + lane_id();
        bool vis = false;
        int32_t x = 0, y = 0, z = 0;
        if (i < n) {
            unpack_key(S.pool_key[i], x, y, z);
            const float dlx = float(8 * x + 4) * fr.vs - fr.P[3];
            const float dly = float(8 * y + 4) * fr.vs - fr.P[7];
            const float dlz = float(8 * z + 4) * fr.vs - fr.P[11];
            const float pcx = (fr.P[0] * dlx + fr.P[4] * dly) + fr.P[8] * dlz;
            const float pcy = (fr.P[1] * dlx + fr.P[5] * dly) + fr.P[9] * dlz;
            const float pcz = (fr.P[2] * dlx + fr.P[6] * dly) + fr.P[10] * dlz;
            if (pcz > 0.0f && depth_valid(pcz, fr)) {
                const float fu = floorf((fr.fx * (pcx / pcz) + fr.cx) + 0.5f);
                const float fv = floorf((fr.fy * (pcy / pcz) + fr.cy) + 0.5f);
                vis = fu >= 0.0f && fu < float(fr.W) && fv >= 0.0f && fv < float(fr.H);
            }
        }
        const unsigned long long pos = wave_append<unsigned long long>(vis, &S.C->visible);
        if (vis && int64_t(pos) < cap) {
            out[3 * pos] = x;
            out[3 * pos + 1] = y;
            out[3 * pos + 2] = z;
        }
    }
}

__global__ void k_zero_visible(Counters *C) { C->visible = 0; }

__global__ void __launch_bounds__(kBlock) k_keys_of(Dev S, int which, int seq, int64_t cap, int32_t *out) {
    // which: 0 = pool order (all blocks), 1 = last touched list, 2 = last MC list
    int64_t n;
    if (which == 0) {
        const unsigned long long pn = S.C->pool_next;
        n = int64_t(pn) < S.pool_cap ? int64_t(pn) : S.pool_cap;
    } else {
        const FrameCounters &fc = S.C->fc[seq & (kRing - 1)];
        n = which == 1 ? int64_t(fc.n_touched) : update_set_size(fc);
    }
    if (n > cap) n = cap;
    for (int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x; i < n; i += int64_t(gridDim.x) * kBlock) {
        uint64_t key;
        if (which == 0) key = S.pool_key[i];
        else if (which == 1) key = S.T[touched_of(S, seq)[i]].key;
        else key = S.pool_key[mclist_of(S, seq)[i]];
        int32_t x, y, z;
        unpack_key(key, x, y, z);
        out[3 * i] = x;
        out[3 * i + 1] = y;
        out[3 * i + 2] = z;
    }
}

// ------------------------------------------------------------ paged log walk
// Entry (f, b) is live iff mc_stamp[b] == f (the block's latest MC update).  Chunks of
// kChunk entries are counted (k_log_count), scanned (k_log_scan, one workgroup) and
// emitted in log order (k_log_emit) up to `cap` keys.
__device__ __forceinline__ uint64_t log_end(const Dev &S) {
    const unsigned long long L = S.C->log_len;
    return L < S.log_cap ? L : S.log_cap;
}

__device__ __forceinline__ bool log_live(const Dev &S, uint64_t pos, uint64_t end) {
    if (pos >= end) return false;
    const uint64_t e = S.log[pos];
    return S.mc_stamp[uint32_t(e)] == uint32_t(e >> 32);
}

__global__ void __launch_bounds__(kBlock) k_log_count(Dev S, uint64_t cursor) {
    __shared__ int part[kWaves];
    const uint64_t end = log_end(S);
    const int64_t nch = cursor < end ? int64_t((end - cursor + kChunk - 1) / kChunk) : 0;
    for (int64_t c = blockIdx.x; c < nch; c += gridDim.x) {
        int cnt = 0;
        for (int k = 0; k < kChunk / kBlock; ++k)
            cnt += log_live(S, cursor + uint64_t(c) * kChunk + uint64_t(k) * kBlock + threadIdx.x, end);
        cnt = wave_sum(cnt);
        if (lane_id() == 0) part[threadIdx.x >> 6] = cnt;
        __syncthreads();
        if (threadIdx.x == 0) {
            int s = 0;
            for (int w = 0; w < kWaves; ++w) s += part[w];
            S.prefix[c] = s;
        }
        __syncthreads();
    }
}

constexpr int kScan = 1024;
__global__ void __launch_bounds__(kScan) k_log_scan(Dev S, uint64_t cursor, int64_t cap, int64_t *d_count,
                                                    uint64_t *d_next) {
    __shared__ int64_t part[kScan];
    const uint64_t end = log_end(S);
    const int64_t nch = cursor < end ? int64_t((end - cursor + kChunk - 1) / kChunk) : 0;
    const int64_t per = (nch + kScan - 1) / kScan;
    const int64_t lo = threadIdx.x * per, hi = lo + per < nch ? lo + per : nch;
    int64_t s = 0;
    for (int64_t c = lo; c < hi; ++c) s += S.prefix[c];
    part[threadIdx.x] = s;
    __syncthreads();
    for (int o = 1; o < kScan; o <<= 1) {  // inclusive Hillis-Steele scan
        const int64_t v = threadIdx.x >= o ? part[threadIdx.x - o] : 0;
        __syncthreads();
        part[threadIdx.x] += v;
        __syncthreads();
    }
    int64_t run = part[threadIdx.x] - s;  // exclusive prefix of this thread's range
    for (int64_t c = lo; c < hi; ++c) {
        const int64_t v = S.prefix[c];
        S.prefix[c] = run;
        run += v;
    }
    if (threadIdx.x == kScan - 1) {
        const int64_t total = part[kScan - 1];
        const int64_t cnt = total < cap ? total : cap;
        *d_count = cnt;
        if (cap == 0)
            *d_next = cursor;
        else if (total < cap)
            *d_next = end;
        // otherwise k_log_emit writes the position after the cap-th live entry
    }
}

__global__ void __launch_bounds__(kBlock) k_log_emit(Dev S, uint64_t cursor, int64_t cap, int32_t *keys,
                                                     uint64_t *d_next) {
    __shared__ int wcount[kWaves];
    const uint64_t end = log_end(S);
    const int64_t nch = cursor < end ? int64_t((end - cursor + kChunk - 1) / kChunk) : 0;
    const int lane = lane_id(), wave = threadIdx.x >> 6;
    for (int64_t c = blockIdx.x; c < nch; c += gridDim.x) {
        int64_t rank = S.prefix[c];
        if (rank >= cap) continue;  // uniform per workgroup
        for (int k = 0; k < kChunk / kBlock; ++k) {
            const uint64_t pos = cursor + uint64_t(c) * kChunk + uint64_t(k) * kBlock + threadIdx.x;
            const bool live = log_live(S, pos, end);
            const unsigned long long m = __ballot(live);
            if (lane == 0) wcount[wave] = __popcll(m);
            __syncthreads();
            int64_t before = rank;
            int64_t total = 0;
            for (int w = 0; w < kWaves; ++w) {
                if (w < wave) before += wcount[w];
                total += wcount[w];
            }
            const int64_t r = before + lanes_below(m);
            if (live && r < cap) {
                int32_t x, y, z;
                unpack_key(S.pool_key[uint32_t(S.log[pos])], x, y, z);
                keys[3 * r] = x;
                keys[3 * r + 1] = y;
                keys[3 * r + 2] = z;
                if (r == cap - 1) *d_next = pos + 1;
            }
            rank += total;
            __syncthreads();
        }
    }
}

__global__ void k_read_counters(const Counters *C, int seq, unsigned long long *out) {
    const FrameCounters &fc = C->fc[seq & (kRing - 1)];
    out[7] = C->tot_touched;
    out[8] = C->tot_mc;
    out[9] = C->tot_voxel_updates;
    out[0] = fc.n_touched;
    out[1] = fc.n_new;
    out[2] = fc.n_mc;
    out[3] = fc.voxel_updates;
    out[4] = C->pool_next;
    out[5] = C->log_len;
    out[6] = C->err;
}

__global__ void k_clear_err(Counters *C) { C->err = 0; }

__global__ void __launch_bounds__(kBlock) k_log_entries(Dev S, uint64_t start, int64_t n, uint32_t *frame,
                                                        int32_t *keys) {
    for (int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x; i < n; i += int64_t(gridDim.x) * kBlock) {
        const uint64_t e = S.log[start + uint64_t(i)];
        if (frame) frame[i] = uint32_t(e >> 32);
        if (keys) {
            int32_t x, y, z;
            unpack_key(S.pool_key[uint32_t(e)], x, y, z);
            keys[3 * i] = x;
            keys[3 * i + 1] = y;
            keys[3 * i + 2] = z;
        }
    }
}

// Zeroes the voxel, MC and stamp state of every handed-out pool block, then the counters.
__global__ void __launch_bounds__(kBlock) k_reset_blocks(Dev S) {
    const unsigned long long pn = S.C->pool_next;
    const int64_t n = int64_t(pn) < S.pool_cap ? int64_t(pn) : S.pool_cap;
    for (int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x; i < n * 512; i += int64_t(gridDim.x) * kBlock) {
        S.F[i] = 0.0f;
        S.WRGB[i] = 0u;
        S.MCV[i] = 0u;
        if ((i & 511) < 64) S.SGN[(i >> 9) * 64 + (i & 511)] = 0;
        if ((i & 511) == 0) {
            S.pool_key[i >> 9] = 0;
            S.mc_stamp[i >> 9] = 0;
        }
    }
}

__global__ void k_zero_counters(Counters *C) {
    uint32_t *w = reinterpret_cast<uint32_t *>(C);
    for (unsigned i = threadIdx.x; i < sizeof(Counters) / 4; i += blockDim.x) w[i] = 0;
}

}  // namespace

namespace {

unsigned wave_grid(const vbh_scene *s, int64_t cap_items) {
    // waves-per-item kernels: enough workgroups to fill every CU several times over
    const int64_t want = int64_t(s->cus) * 8;
    const int64_t need = (cap_items + kWaves - 1) / kWaves;
    return unsigned(need < want ? (need > 0 ? need : 1) : want);
}

// Start/stop events for the kernels of update seq if it is one of the timed updates.
StageTimer *timer_for(vbh_scene *s, int seq) {
    if (s->timing_period <= 0 || seq % s->timing_period != 0) return nullptr;
    if (s->ev_free.empty()) {
        StageTimer t;
        for (auto &e : t.ev)
            if (hipEventCreate(&e) != hipSuccess) return nullptr;
        s->ev_free.push_back(t);
    }
    s->ev_pending.push_back(s->ev_free.back());
    s->ev_free.pop_back();
    StageTimer *tm = &s->ev_pending.back();
    tm->ran = 0;
    return tm;
}

// Launches a kernel; a timed one gets start/stop events attached to its dispatch (no
// extra packets between the kernels).
template <typename... Args, typename F>
void launch(StageTimer *tm, int stage, hipStream_t st, F kern, dim3 grid, dim3 block, Args... args) {
    if (tm) {
        tm->ran |= 1u << stage;
        hipExtLaunchKernelGGL(kern, grid, block, 0, st, tm->ev[2 * stage], tm->ev[2 * stage + 1], 0, args...);
    } else {
        hipLaunchKernelGGL(kern, grid, block, 0, st, args...);
    }
}

// Runs the MC update for the blocks in the touched list of update `seq`.
// n_partials: workgroups of the update's integration kernel whose statistics the
// extraction kernel reduces (0 if none ran).
int mc_update(vbh_scene *s, uint32_t frame, int seq, hipStream_t st, StageTimer *tm = nullptr, int n_partials = 0) {
    launch(tm, 2, st, k_mc_mark, dim3(unsigned(s->cus) * 2), dim3(kMarkThreads), s->d, frame, seq);
    launch(tm, 3, st, k_mc_extract, dim3(s->g_ext), dim3(kBlock), s->d, seq, n_partials, frame);
    VBH_LAUNCHED();
    return VBH_OK;
}

int read_counters(vbh_scene *s, int seq, unsigned long long (&h)[10], hipStream_t st) {
    k_read_counters<<<1, 1, 0, st>>>(s->C, seq, s->hostbuf);
    VBH_LAUNCHED();
    VBH_HIP(hipMemcpyAsync(h, s->hostbuf, sizeof(h), hipMemcpyDeviceToHost, st));
    VBH_HIP(hipStreamSynchronize(st));
    return VBH_OK;
}

int keys_of(vbh_scene *s, int which, int32_t *d_keys, int64_t cap, int64_t *h_count, void *stream) {
    if (!s || cap < 0 || (cap > 0 && !d_keys)) return VBH_EINVAL;
    hipStream_t st = as_stream(stream);
    unsigned long long h[10];
    const int seq = s->seq - 1;
    if (int rc = read_counters(s, seq < 0 ? 0 : seq, h, st)) return rc;
    int64_t n;
    if (which == 0) n = int64_t(h[4]) < s->p.pool_blocks ? int64_t(h[4]) : s->p.pool_blocks;
    else n = s->seq == 0 ? 0 : int64_t(which == 1 ? h[0] : h[2]);
    if (h_count) *h_count = n;
    const int64_t m = n < cap ? n : cap;
    if (m > 0) {
        k_keys_of<<<grid_for(m, kBlock, 4096), kBlock, 0, st>>>(s->d, which, seq < 0 ? 0 : seq, cap, d_keys);
        VBH_LAUNCHED();
        VBH_HIP(hipStreamSynchronize(st));
    }
    return VBH_OK;
}

}  // namespace

namespace vbh {
Frame make_frame(const vbh_scene *s, const float *pose) {
    Frame f{};
    std::memcpy(f.P, pose, sizeof(f.P));
    f.fx = s->p.fx;
    f.fy = s->p.fy;
    f.cx = s->p.cx;
    f.cy = s->p.cy;
    f.W = s->p.width;
    f.H = s->p.height;
    f.dmin = s->p.depth_min;
    f.dmax = s->p.depth_max;
    f.dlo = std::max(f.dmin, 0x1p-149f);
    f.vs = s->p.voxel_size;
    f.mu = s->p.trunc;
    f.m_band = s->m_band;
    // The integration kernel's reciprocal-based quotients pc_x / pc_z and pc_y / pc_z equal
    // the correctly rounded ones for |pc| <= 2^32 and pc_z >= 2^-32 (the kernel checks the
    // latter); a quotient below 2^-56 yields the same pixel as the exact one if |fx|, |fy|
    // <= 2^20.  A voxel's camera coordinate is at most the largest column sum of |R| times
    // the largest |voxel centre - t|, with block coordinates below 2^20 in magnitude.
    double col = 0.0, tmax = 0.0;
    for (int j = 0; j < 3; ++j) {
        col = std::max(col, std::fabs(double(pose[j])) + std::fabs(double(pose[4 + j])) + std::fabs(double(pose[8 + j])));
        tmax = std::max(tmax, std::fabs(double(pose[4 * j + 3])));
    }
    const double bound = 1.001 * col * ((double(1 << 23) + 8.0) * double(f.vs) + tmax);
    f.fast_div = int(bound <= 0x1p32 && std::fabs(double(f.fx)) <= 0x1p20 && std::fabs(double(f.fy)) <= 0x1p20);
    // Allocation divides world coordinates pw of band samples by the block size bs = 8 vs;
    // the reciprocal-based quotient equals the correctly rounded one for 2^-32 <= bs <= 2^32
    // and 2^-90 <= |pw| <= 2^32 (the kernel takes the full division for smaller |pw|).  A
    // sample lies at camera depth at most dmax + mu on a ray with |x/z|, |y/z| at most the
    // image's extent over the focal lengths.
    const double bsd = 8.0 * double(f.vs);
    const double xr = std::max(std::fabs(double(f.cx)), std::fabs(double(f.W) - 1.0 - double(f.cx))) / std::fabs(double(f.fx));
    const double yr = std::max(std::fabs(double(f.cy)), std::fabs(double(f.H) - 1.0 - double(f.cy))) / std::fabs(double(f.fy));
    const double pc_max = (double(f.dmax) + 2.0 * double(f.mu) + double(f.vs)) * std::max(1.0, std::max(xr, yr));
    double pw_max = 0.0;
    for (int c = 0; c < 3; ++c)
        pw_max = std::max(pw_max, std::fabs(double(pose[4 * c + 3])) +
                                      (std::fabs(double(pose[4 * c])) + std::fabs(double(pose[4 * c + 1])) +
                                       std::fabs(double(pose[4 * c + 2]))) * pc_max);
    pw_max *= 1.001;
    f.fast_bs = int(bsd >= 0x1p-32 && bsd <= 0x1p32 && pw_max <= 0x1p32);
    // A band sample's coordinate below 2^-90 in magnitude divided by bs <= 1 gives a
    // nonzero product with the reciprocal (at least 1) of the dividend's sign and below 1
    // in magnitude, so its floor is that of the true quotient: no fallback is needed.
    if (f.fast_bs && bsd <= 1.0) f.fast_bs = 2;
    // Allocation may collect 32-bit keys B - kb (10 bits per axis) when every band sample's
    // block lies within 1024 blocks of kb = floor(t / bs) - 512: a sample's camera depth is
    // at most lam_max = dmax - mu + 2 m vs, so |pw_c - t_c| is at most the row sum of |R|
    // times lam_max max(1, |x/z|, |y/z|), with slack for rounding; the blocks must also lie
    // inside the key range, so that no sample needs the range check.
    f.local_keys = 0;
    const double lam_max = double(f.dmax) + std::fabs(double(f.mu)) + 2.0 * double(f.m_band) * double(f.vs) + double(f.vs);
    const double reach_pc = lam_max * std::max(1.0, std::max(xr, yr));
    if (std::isfinite(reach_pc) && std::isfinite(bsd) && bsd > 0.0) {
        bool ok = true;
        for (int c = 0; c < 3 && ok; ++c) {
            const double t = double(pose[4 * c + 3]);
            const double span = 1.01 * (std::fabs(double(pose[4 * c])) + std::fabs(double(pose[4 * c + 1])) +
                                        std::fabs(double(pose[4 * c + 2]))) * reach_pc +
                                0x1p-20 * (std::fabs(t) + 1.0);
            const double base = std::floor(t / bsd);
            const double reach = std::ceil(span / bsd) + 3.0;
            ok = std::isfinite(base) && reach <= 511.0 && std::fabs(base) + reach <= double(1 << 20) - 1.0;
            if (ok) f.kb[c] = int(base) - 512;
        }
        f.local_keys = int(ok);
        if (ok)  // (B_x << 20) + (B_y << 10) + B_z - kb_packed, modulo 2^32, packs B - kb
            f.kb_packed = (uint32_t(f.kb[0]) << 20) + (uint32_t(f.kb[1]) << 10) + uint32_t(f.kb[2]);
    }
    return f;
}
}  // namespace vbh

namespace {
dim3 alloc_grid(const vbh_scene *s) { return dim3(unsigned((s->p.width + 31) / 32), unsigned((s->p.height + 15) / 16)); }
}  // namespace

namespace vbh {
int scene_fuse(vbh_scene *s, const float *d_depth, const uint8_t *d_rgb, const float *pose, uint32_t frame,
               bool with_mc, hipStream_t st) {
    const Frame fr = make_frame(s, pose);
    const int seq = s->seq;
    StageTimer *tm = timer_for(s, seq);
    launch(tm, 0, st, fr.local_keys ? k_alloc<uint32_t> : k_alloc<uint64_t>, alloc_grid(s), dim3(kAllocThreads), s->d, fr, d_depth, d_rgb, frame, seq,
           int(with_mc));
    launch(tm, 1, st, d_rgb ? k_integrate<true> : k_integrate<false>, dim3(s->g_int), dim3(kBlock), s->d, fr, seq,
           int(tm != nullptr && with_mc));
    if (with_mc) launch(tm, 3, st, k_mc_extract, dim3(s->g_ext), dim3(kBlock), s->d, seq, int(s->g_int), frame);
    VBH_LAUNCHED();
    s->seq = seq + 1;
    s->last_frame = frame;
    return VBH_OK;
}

// At most kInFlight frames are enqueued ahead of the device: a deeper queue of launches
// only stalls submission once the hardware queue is full.
int scene_fuse_frames(vbh_scene *s, const float *d_depth, const uint8_t *d_rgb, const float *poses, uint32_t first,
                      int64_t n, hipStream_t st) {
    constexpr int64_t kStep = 16, kInFlight = 64;
    const int64_t hw = int64_t(s->p.width) * s->p.height;
    hipEvent_t ring[kInFlight / kStep] = {};
    int rc = VBH_OK;
    for (int64_t i = 0; i < n && rc == VBH_OK; ++i) {
        if (i % kStep == 0) {
            hipEvent_t &e = ring[(i / kStep) % (kInFlight / kStep)];
            if (e && hipEventSynchronize(e) != hipSuccess) rc = VBH_EHIP;
            if (!e && hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) rc = VBH_EHIP;
            if (rc == VBH_OK && hipEventRecord(e, st) != hipSuccess) rc = VBH_EHIP;
        }
        if (rc == VBH_OK)
            rc = scene_fuse(s, d_depth + i * hw, d_rgb ? d_rgb + i * hw * 3 : nullptr, poses + 12 * i,
                            first + uint32_t(i), true, st);
    }
    for (hipEvent_t e : ring)
        if (e) (void)hipEventDestroy(e);
    return rc;
}

// Copies go on the caller's stream, in front of each frame's kernels, into one of two
// device buffers.  (A second stream for the copies, ordered by events, measured slower:
// the cross-stream waits cost more than the overlap gains.)
int scene_fuse_frames_host(vbh_scene *s, const float *h_depth, const uint8_t *h_rgb, const float *poses,
                           uint32_t first, int64_t n, hipStream_t st) {
    constexpr int64_t kStep = 16, kInFlight = 64;
    const size_t hw = size_t(s->p.width) * size_t(s->p.height);
    const size_t dbytes = hw * 4, cbytes = hw * 3, stride = (dbytes + cbytes + 255) & ~size_t(255);
    for (int b = 0; b < 2; ++b)
        if (!s->up_buf[b] && hipMalloc(&s->up_buf[b], stride) != hipSuccess) return VBH_ENOMEM;
    hipEvent_t ring[kInFlight / kStep] = {};
    int rc = VBH_OK;
    for (int64_t i = 0; i < n && rc == VBH_OK; ++i) {
        if (i % kStep == 0) {
            hipEvent_t &e = ring[(i / kStep) % (kInFlight / kStep)];
            if (e && hipEventSynchronize(e) != hipSuccess) rc = VBH_EHIP;
            if (!e && hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) rc = VBH_EHIP;
            if (rc == VBH_OK && hipEventRecord(e, st) != hipSuccess) rc = VBH_EHIP;
            if (rc != VBH_OK) break;
        }
        float *dd = static_cast<float *>(s->up_buf[i & 1]);
        uint8_t *dc = static_cast<uint8_t *>(s->up_buf[i & 1]) + dbytes;
        if (hipMemcpyAsync(dd, h_depth + int64_t(i) * int64_t(hw), dbytes, hipMemcpyHostToDevice, st) != hipSuccess ||
            (h_rgb && hipMemcpyAsync(dc, h_rgb + int64_t(i) * int64_t(hw) * 3, cbytes, hipMemcpyHostToDevice, st) !=
                          hipSuccess)) {
            rc = VBH_EHIP;
            break;
        }
        rc = scene_fuse(s, dd, h_rgb ? dc : nullptr, poses + 12 * i, first + uint32_t(i), true, st);
    }
    for (hipEvent_t e : ring)
        if (e) (void)hipEventDestroy(e);
    return rc;
}

int scene_alloc_only(vbh_scene *s, const float *d_depth, const float *pose, uint32_t frame, hipStream_t st) {
    const int seq = s->seq;
    const Frame fr = make_frame(s, pose);
    launch(timer_for(s, seq), 0, st, fr.local_keys ? k_alloc<uint32_t> : k_alloc<uint64_t>, alloc_grid(s),
           dim3(kAllocThreads), s->d, fr, d_depth, static_cast<const uint8_t *>(nullptr), frame, seq, 0);
    VBH_LAUNCHED();
    s->seq = seq + 1;
    s->last_frame = frame;
    return VBH_OK;
}

int scene_mc_update(vbh_scene *s, uint32_t frame, hipStream_t st) {
    const int seq = s->seq - 1;
    if (seq < 0) return VBH_EINVAL;
    k_mc_mark<<<unsigned(s->cus) * 2, kMarkThreads, 0, st>>>(s->d, frame, seq);
    k_mc_extract<<<s->g_ext, kBlock, 0, st>>>(s->d, seq, int(s->g_int), frame);
    VBH_LAUNCHED();
    return VBH_OK;
}

int scene_reset(vbh_scene *s, hipStream_t st) {
    if (int rc = table_init(s->d.T, s->p.slots, st)) return rc;
    k_reset_blocks<<<unsigned(s->cus) * 8, kBlock, 0, st>>>(s->d);
    k_zero_counters<<<1, 256, 0, st>>>(s->C);
    VBH_LAUNCHED();
    s->seq = 0;
    s->last_frame = 0;
    return VBH_OK;
}
}  // namespace vbh

extern "C" {

int vbh_scene_create(const vbh_params *p, vbh_scene **out) {
    if (!out || !p) return VBH_EINVAL;
    *out = nullptr;
    if (!is_pow2(p->slots) || p->slots < 64 || p->slots > (1ull << 31) || p->pool_blocks < 1 ||
        p->pool_blocks > (int64_t(1) << 30) || p->log_capacity < 1 || !(p->voxel_size > 0) ||
        !(p->trunc >= p->voxel_size) || p->width <= 0 || p->height <= 0 || p->width > 16384 ||
        p->height > 16384 || !(p->fx > 0) || !(p->fy > 0) ||
        p->hash_kind < 0 || p->hash_kind > 1 || !(p->depth_max >= p->depth_min))
        return VBH_EINVAL;
    vbh_scene *s = new (std::nothrow) vbh_scene();
    if (!s) return VBH_ENOMEM;
    s->p = *p;
    s->m_band = int(floorf(p->trunc / p->voxel_size + 0.5f));
    s->cus = vbh::device_cus();
    // The per-frame integration and extraction launches have one workgroup per slot that
    // the device can hold at once: a grid of several partial generations leaves the last
    // one running on few CUs (for integration, 5 workgroups per CU by its registers).
    {
        int n = 0;
        s->g_int = unsigned(s->cus) *
                   unsigned(hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_integrate<true>, kBlock, 0) == hipSuccess && n > 0
                                ? n
                                : 4);
        n = 0;
        s->g_ext = unsigned(s->cus) *
                   unsigned(hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_mc_extract, kBlock, 0) == hipSuccess && n > 0
                                ? n
                                : 8);
    }
    const uint64_t P = uint64_t(p->pool_blocks);
    s->max_chunks = (p->log_capacity + kChunk - 1) / kChunk + 1;
    const size_t sizes[] = {p->slots * sizeof(Slot), P * 512 * sizeof(float), P * 512 * 4, P * 512 * 4,
                            P * 8,                  P * 4,                     2 * p->slots * 4, 2 * P * 4,
                            size_t(p->log_capacity) * 8, size_t(s->max_chunks) * 8, sizeof(Counters), 64 * 8,
                            size_t(kMaxPartials) * 8, P * 64 * 2, size_t(p->width) * size_t(p->height) * 8};
    for (int i = 0; i < 15; ++i) {
        if (hipMalloc(&s->mem[i], sizes[i]) != hipSuccess) {
            vbh_scene_destroy(s);
            return VBH_ENOMEM;
        }
    }
    Dev &d = s->d;
    d.T = static_cast<Slot *>(s->mem[0]);
    d.mask = p->slots - 1;
    d.kind = p->hash_kind;
    d.F = static_cast<float *>(s->mem[1]);
    d.WRGB = static_cast<uint32_t *>(s->mem[2]);
    d.MCV = static_cast<uint32_t *>(s->mem[3]);
    d.pool_key = static_cast<uint64_t *>(s->mem[4]);
    d.mc_stamp = static_cast<uint32_t *>(s->mem[5]);
    d.touched = static_cast<int32_t *>(s->mem[6]);
    d.mclist = static_cast<int32_t *>(s->mem[7]);
    d.log = static_cast<uint64_t *>(s->mem[8]);
    d.prefix = static_cast<int64_t *>(s->mem[9]);
    d.pool_cap = p->pool_blocks;
    d.log_cap = uint64_t(p->log_capacity);
    s->C = static_cast<Counters *>(s->mem[10]);
    d.C = s->C;
    s->hostbuf = static_cast<unsigned long long *>(s->mem[11]);
    d.partial = static_cast<unsigned long long *>(s->mem[12]);
    d.SGN = static_cast<uint16_t *>(s->mem[13]);
    d.PIX = static_cast<uint2 *>(s->mem[14]);
    bool ok = vbh::table_init(d.T, p->slots, nullptr) == VBH_OK;
    for (int i : {1, 2, 3, 4, 5, 13})
        if (ok) ok = hipMemset(s->mem[i], 0, sizes[i]) == hipSuccess;
    ok = ok && hipMemset(s->C, 0, sizeof(Counters)) == hipSuccess && hipDeviceSynchronize() == hipSuccess;
    if (!ok) {
        vbh_scene_destroy(s);
        return VBH_EHIP;
    }
    *out = s;
    return VBH_OK;
}

void vbh_scene_destroy(vbh_scene *s) {
    if (!s) return;
    for (void *b : s->up_buf)
        if (b) (void)hipFree(b);
    for (auto *v : {&s->ev_pending, &s->ev_free})
        for (auto &tm : *v)
            for (auto e : tm.ev) (void)hipEventDestroy(e);
    for (void *m : s->mem)
        if (m) (void)hipFree(m);
    delete s;
}

int vbh_integrate_frame(vbh_scene *s, const float *d_depth, const uint8_t *d_rgb, const float *pose_c2w,
                        uint32_t frame_id, void *stream) {
    if (!s || !d_depth || !pose_c2w || frame_id == 0 || frame_id <= s->last_frame) return VBH_EINVAL;
    for (int i = 0; i < 12; ++i)
        if (!std::isfinite(pose_c2w[i])) return VBH_EINVAL;
    return vbh::scene_fuse(s, d_depth, d_rgb, pose_c2w, frame_id, true, as_stream(stream));
}

int vbh_integrate_blocks(vbh_scene *s, const int32_t *d_keys, int64_t n, const float *d_depth, const uint8_t *d_rgb,
                         const float *pose_c2w, uint32_t frame_id, void *stream) {
    if (!s || n < 0 || (n > 0 && !d_keys) || !d_depth || !pose_c2w || frame_id == 0 || frame_id <= s->last_frame)
        return VBH_EINVAL;
    for (int i = 0; i < 12; ++i)
        if (!std::isfinite(pose_c2w[i])) return VBH_EINVAL;
    hipStream_t st = as_stream(stream);
    const Frame fr = make_frame(s, pose_c2w);
    const int seq = s->seq;
    StageTimer *tm = timer_for(s, seq);
    const int64_t hw = int64_t(s->p.width) * s->p.height;
    k_load_claim<<<grid_for(n, kBlock, 8192), kBlock, 0, st>>>(s->d, d_keys, n, frame_id, seq);
    k_pix_pack<<<grid_for(hw, kBlock, 4096), kBlock, 0, st>>>(s->d, hw, d_depth, d_rgb);
    VBH_LAUNCHED();
    launch(tm, 1, st, d_rgb ? k_integrate<true> : k_integrate<false>, dim3(s->g_int), dim3(kBlock), s->d, fr, seq, 0);
    if (int rc = mc_update(s, frame_id, seq, st, tm, int(s->g_int))) return rc;
    s->seq = seq + 1;
    s->last_frame = frame_id;
    return VBH_OK;
}

int vbh_integrate_frames(vbh_scene *s, const float *d_depth, const uint8_t *d_rgb, const float *poses_c2w,
                         uint32_t first_frame_id, int64_t n, void *stream) {
    if (!s || n < 0 || (n > 0 && (!d_depth || !poses_c2w)) || first_frame_id == 0 ||
        first_frame_id <= s->last_frame || uint64_t(first_frame_id) + uint64_t(n > 0 ? n - 1 : 0) > 0xFFFFFFFFull)
        return VBH_EINVAL;
    for (int64_t i = 0; i < 12 * n; ++i)
        if (!std::isfinite(poses_c2w[i])) return VBH_EINVAL;
    return vbh::scene_fuse_frames(s, d_depth, d_rgb, poses_c2w, first_frame_id, n, as_stream(stream));
}

int vbh_integrate_frames_host(vbh_scene *s, const float *h_depth, const uint8_t *h_rgb, const float *poses_c2w,
                              uint32_t first_frame_id, int64_t n, void *stream) {
    if (!s || n < 0 || (n > 0 && (!h_depth || !poses_c2w)) || first_frame_id == 0 ||
        first_frame_id <= s->last_frame || uint64_t(first_frame_id) + uint64_t(n > 0 ? n - 1 : 0) > 0xFFFFFFFFull)
        return VBH_EINVAL;
    for (int64_t i = 0; i < 12 * n; ++i)
        if (!std::isfinite(poses_c2w[i])) return VBH_EINVAL;
    return vbh::scene_fuse_frames_host(s, h_depth, h_rgb, poses_c2w, first_frame_id, n, as_stream(stream));
}

int vbh_extract_mc_indices(vbh_scene *s, const int32_t *d_keys, int64_t n, uint8_t *d_mc, uint8_t *d_rgb,
                           void *stream) {
    if (!s || n < 0 || (n > 0 && (!d_keys || !d_mc))) return VBH_EINVAL;
    if (n == 0) return VBH_OK;
    k_mc_keys<<<wave_grid(s, n), kBlock, 0, as_stream(stream)>>>(s->d, d_keys, n, d_mc, d_rgb);
    VBH_LAUNCHED();
    return VBH_OK;
}

int vbh_stored_mc(vbh_scene *s, const int32_t *d_keys, int64_t n, uint8_t *d_mc, uint8_t *d_rgb, void *stream) {
    if (!s || n < 0 || (n > 0 && (!d_keys || !d_mc))) return VBH_EINVAL;
    if (n == 0) return VBH_OK;
    k_read_blocks<<<wave_grid(s, n), kBlock, 0, as_stream(stream)>>>(s->d, d_keys, n, nullptr, d_mc, d_rgb, nullptr, 1);
    VBH_LAUNCHED();
    return VBH_OK;
}

int vbh_updated_blocks_since(vbh_scene *s, uint64_t cursor, int64_t cap, int32_t *d_keys_out, int64_t *d_count,
                             uint64_t *d_next_cursor, void *stream) {
    if (!s || cap < 0 || !d_count || !d_next_cursor || (cap > 0 && !d_keys_out)) return VBH_EINVAL;
    hipStream_t st = as_stream(stream);
    const unsigned g = unsigned(s->cus) * 4;
    k_log_count<<<g, kBlock, 0, st>>>(s->d, cursor);
    k_log_scan<<<1, kScan, 0, st>>>(s->d, cursor, cap, d_count, d_next_cursor);
    if (cap > 0) k_log_emit<<<g, kBlock, 0, st>>>(s->d, cursor, cap, d_keys_out, d_next_cursor);
    VBH_LAUNCHED();
    return VBH_OK;
}

int vbh_scene_status(vbh_scene *s, void *stream) {
    if (!s) return VBH_EINVAL;
    hipStream_t st = as_stream(stream);
    unsigned long long h[10];
    if (int rc = read_counters(s, s->seq > 0 ? s->seq - 1 : 0, h, st)) return rc;
    if (h[6]) {
        k_clear_err<<<1, 1, 0, st>>>(s->C);
        VBH_LAUNCHED();
        VBH_HIP(hipStreamSynchronize(st));
    }
    return code_from_bits(uint32_t(h[6]));
}

int vbh_scene_stats(vbh_scene *s, vbh_stats *o, void *stream) {
    if (!s || !o) return VBH_EINVAL;
    unsigned long long h[10];
    if (int rc = read_counters(s, s->seq > 0 ? s->seq - 1 : 0, h, as_stream(stream))) return rc;
    const bool any = s->seq > 0;
    o->n_touched = any ? int64_t(h[0]) : 0;
    o->n_new = any ? int64_t(h[1]) : 0;
    o->n_mc = any ? int64_t(h[2]) : 0;
    o->n_voxel_updates = any ? int64_t(h[3]) : 0;
    o->n_blocks = int64_t(h[4]) < s->p.pool_blocks ? int64_t(h[4]) : s->p.pool_blocks;
    o->log_length = h[5] < uint64_t(s->p.log_capacity) ? h[5] : uint64_t(s->p.log_capacity);
    o->last_frame = s->last_frame;
    o->error = code_from_bits(uint32_t(h[6]));
    o->total_touched = int64_t(h[7]);
    o->total_mc = int64_t(h[8]);
    o->total_voxel_updates = int64_t(h[9]);
    return VBH_OK;
}

int vbh_scene_export_blocks(vbh_scene *s, int32_t *d_keys, int64_t cap, int64_t *h_count, void *stream) {
    return keys_of(s, 0, d_keys, cap, h_count, stream);
}
int vbh_scene_last_touched(vbh_scene *s, int32_t *d_keys, int64_t cap, int64_t *h_count, void *stream) {
    return keys_of(s, 1, d_keys, cap, h_count, stream);
}
int vbh_scene_last_mc(vbh_scene *s, int32_t *d_keys, int64_t cap, int64_t *h_count, void *stream) {
    return keys_of(s, 2, d_keys, cap, h_count, stream);
}

int vbh_scene_read_blocks(vbh_scene *s, const int32_t *d_keys, int64_t n, float *d_F, uint8_t *d_W, uint8_t *d_rgb,
                          int32_t *d_found, void *stream) {
    if (!s || n < 0 || (n > 0 && !d_keys)) return VBH_EINVAL;
    if (n == 0) return VBH_OK;
    k_read_blocks<<<wave_grid(s, n), kBlock, 0, as_stream(stream)>>>(s->d, d_keys, n, d_F, d_W, d_rgb, d_found, 0);
    VBH_LAUNCHED();
    return VBH_OK;
}

int vbh_scene_write_blocks(vbh_scene *s, const int32_t *d_keys, int64_t n, const float *d_F, const uint8_t *d_W,
                           const uint8_t *d_rgb, uint32_t frame_id, void *stream) {
    if (!s || n < 0 || (n > 0 && (!d_keys || !d_F || !d_W)) || frame_id == 0 || frame_id <= s->last_frame)
        return VBH_EINVAL;
    hipStream_t st = as_stream(stream);
    const int seq = s->seq;
    k_load_claim<<<grid_for(n, kBlock, 8192), kBlock, 0, st>>>(s->d, d_keys, n, frame_id, seq);
    if (n > 0) k_load_copy<<<wave_grid(s, n), kBlock, 0, st>>>(s->d, d_keys, n, d_F, d_W, d_rgb);
    VBH_LAUNCHED();
    if (int rc = mc_update(s, frame_id, seq, st)) return rc;
    s->seq = seq + 1;
    s->last_frame = frame_id;
    return VBH_OK;
}

int vbh_scene_reset_blocks(vbh_scene *s, const int32_t *d_keys, int64_t n, uint32_t frame_id, void *stream) {
    if (!s || n < 0 || (n > 0 && !d_keys) || frame_id == 0 || frame_id <= s->last_frame) return VBH_EINVAL;
    hipStream_t st = as_stream(stream);
    const int seq = s->seq;
    k_reset_claim<<<grid_for(n, kBlock, 8192), kBlock, 0, st>>>(s->d, d_keys, n, frame_id, seq);
    k_reset_clear<<<wave_grid(s, n), kBlock, 0, st>>>(s->d, seq);
    VBH_LAUNCHED();
    if (int rc = mc_update(s, frame_id, seq, st)) return rc;
    s->seq = seq + 1;
    s->last_frame = frame_id;
    return VBH_OK;
}

int vbh_scene_visible_blocks(vbh_scene *s, const float *pose_c2w, int32_t *d_keys, int64_t cap, int64_t *h_count,
                             void *stream) {
    if (!s || !pose_c2w || cap < 0 || (cap > 0 && !d_keys)) return VBH_EINVAL;
    hipStream_t st = as_stream(stream);
    k_zero_visible<<<1, 1, 0, st>>>(s->C);
    k_visible<<<unsigned(s->cus) * 8, kBlock, 0, st>>>(s->d, make_frame(s, pose_c2w), cap, d_keys);
    VBH_LAUNCHED();
    unsigned long long h = 0;
    VBH_HIP(hipMemcpyAsync(&h, &s->C->visible, sizeof(h), hipMemcpyDeviceToHost, st));
    VBH_HIP(hipStreamSynchronize(st));
    if (h_count) *h_count = int64_t(h);
    return VBH_OK;
}

int vbh_scene_log_entries(vbh_scene *s, uint64_t start, int64_t n, uint32_t *d_frame, int32_t *d_keys,
                          void *stream) {
    if (!s || n < 0) return VBH_EINVAL;
    unsigned long long h[10];
    hipStream_t st = as_stream(stream);
    if (int rc = read_counters(s, s->seq > 0 ? s->seq - 1 : 0, h, st)) return rc;
    const uint64_t end = h[5] < uint64_t(s->p.log_capacity) ? h[5] : uint64_t(s->p.log_capacity);
    if (start > end || uint64_t(n) > end - start) return VBH_EINVAL;
    if (n > 0) {
        k_log_entries<<<grid_for(n, kBlock, 4096), kBlock, 0, st>>>(s->d, start, n, d_frame, d_keys);
        VBH_LAUNCHED();
    }
    return VBH_OK;
}

int vbh_scene_enable_timing(vbh_scene *s, int32_t period) {
    if (!s || period < 0) return VBH_EINVAL;
    s->timing_period = period;
    return VBH_OK;
}

int vbh_scene_timing(vbh_scene *s, double *ms_out, int64_t *h_frames, int64_t *h_blocks, void *stream) {
    if (!s || !ms_out) return VBH_EINVAL;
    VBH_HIP(hipStreamSynchronize(as_stream(stream)));
    unsigned long long blk[2] = {0, 0};
    VBH_HIP(hipMemcpy(blk, &s->C->timed_touched, sizeof(blk), hipMemcpyDeviceToHost));
    VBH_HIP(hipMemset(&s->C->timed_touched, 0, sizeof(blk)));
    if (h_blocks) {
        h_blocks[0] = int64_t(blk[0]);
        h_blocks[1] = int64_t(blk[1]);
    }
    for (int i = 0; i < 4; ++i) ms_out[i] = 0.0;
    for (auto &tm : s->ev_pending) {
        for (int i = 0; i < kStages; ++i) {
            float ms = 0.0f;
            if (tm.ran >> i & 1u) VBH_HIP(hipEventElapsedTime(&ms, tm.ev[2 * i], tm.ev[2 * i + 1]));
            ms_out[i] += ms;
        }
        s->ev_free.push_back(tm);
    }
    if (h_frames) *h_frames = int64_t(s->ev_pending.size());
    s->ev_pending.clear();
    return VBH_OK;
}

}  // extern "C"
