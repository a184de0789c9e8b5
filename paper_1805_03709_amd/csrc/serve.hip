// Serving loop for exploration clients (Sec. 4.2-4.3): the scene stays resident on the
// device; clients ask for the MC voxel blocks updated since their last request (at most
// `limit` blocks, the client-chosen request size); requests are admitted as request slots
// and result memory free up and are launched in rounds on a pool of streams, so work of
// requests admitted at different times overlaps on the device (continuous batching);
// depth frames keep being fused concurrently on another stream.
//
// Consistency: a request is served against one scene version V (the last fully published
// MC update).  A frame's allocation and integration run concurrently with serving, but its
// MC update (which rewrites MC voxels, stamps and appends to the log) waits behind a gate
// until the requests in flight have completed, and no request is launched while it runs.
// So every result equals the result of the same request run alone at version V.
//
// Per request, against the log prefix [0, end_V): the live entries after the client's
// cursor are counted per chunk, the chunk counts are scanned, the first `limit` live
// entries are emitted in log order, and each selected block's key and its 512 MC voxels
// (index | R<<8 | G<<16 | B<<24, the 4-byte MC voxel) are gathered into the request's
// slice of the result arena.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <new>
#include <thread>
#include <vector>

#include "sched.hpp"
#include "scene.hpp"

using namespace vbh;

namespace {

constexpr int kSvChunk = 2048;  // log entries per counting workgroup
constexpr int kSvWG = 256;
constexpr int kMaxBatch = 256;

// Device descriptor of one admitted request (byte offsets into the arena).
struct SvReq {
    uint64_t cursor;     // first log position to consider
    uint64_t end;        // log end of the request's scene version
    int64_t limit;
    int64_t chunk_base;  // first counting item of this request in the round
    int64_t n_chunks;
    int64_t item_base;   // first gather item (prefix of limits) in the round
    int64_t off_sel;     // int32 [limit] selected pool indices
    int64_t off_cnt;     // int64 [n_chunks] chunk counts, then exclusive prefixes
    int64_t off_keys;    // int32 [limit][3]
    int64_t off_mc;      // uint32 [limit][512]
    int64_t off_meta;    // int64 count, uint64 next cursor
    int32_t *keys_out;   // the caller's result buffers, written directly by the gather
    uint32_t *mc_out;    // (NULL: the arena slices above)
};

struct SvRound {
    const SvReq *req;
    int n;
    int64_t total_chunks;
    int64_t total_items;
    char *arena;
};

__device__ __forceinline__ int find_req(const SvRound &R, int64_t item, bool by_chunk) {
    int lo = 0, hi = R.n - 1;  // last request whose base <= item
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        const int64_t b = by_chunk ? R.req[mid].chunk_base : R.req[mid].item_base;
        if (b <= item) lo = mid; else hi = mid - 1;
    }
    return lo;
}

__device__ __forceinline__ bool entry_live(const Dev &S, uint64_t pos, uint64_t end) {
    if (pos >= end) return false;
    const uint64_t e = S.log[pos];
    return S.mc_stamp[uint32_t(e)] == uint32_t(e >> 32);
}

// Words that one workgroup writes and another reads within a launch (chunk counts and
// prefixes, selected pool blocks, counts and cursors) are device-scope relaxed atomics:
// coherent across the XCDs' L2s by themselves, so the persistent launch's barriers only
// wait for their completion and need no invalidate.  The gather's outputs are plain
// stores; the barrier that ends a batch writes them back (see team_sync).
__device__ __forceinline__ int64_t ld_dc(const int64_t *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_dc(int64_t *p, int64_t v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ int32_t ld_dc(const int32_t *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_dc(int32_t *p, int32_t v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// The four steps of a round, for workgroup wg of G (a kernel's grid, or the workgroups of
// the persistent launch).
__device__ __forceinline__ void sv_count(const Dev &S, const SvRound &R, int64_t wg, int64_t G) {
    __shared__ int part[kSvWG / 64];
    for (int64_t it = wg; it < R.total_chunks; it += G) {
        const int r = find_req(R, it, true);
        const SvReq q = R.req[r];
        const int64_t c = it - q.chunk_base;
        int cnt = 0;
        for (int k = 0; k < kSvChunk / kSvWG; ++k)
            cnt += entry_live(S, q.cursor + uint64_t(c) * kSvChunk + uint64_t(k) * kSvWG + threadIdx.x, q.end);
        cnt = wave_sum(cnt);
        if (lane_id() == 0) part[threadIdx.x >> 6] = cnt;
        __syncthreads();
        if (threadIdx.x == 0) {
            int64_t s = 0;
            for (int w = 0; w < kSvWG / 64; ++w) s += part[w];
            st_dc(reinterpret_cast<int64_t *>(R.arena + q.off_cnt) + c, s);
        }
        __syncthreads();
    }
}

// One workgroup per request: exclusive scan of its chunk counts, count and (when fewer
// than `limit` live entries exist) the next cursor.
__device__ __forceinline__ void sv_scan_one(const SvRound &R, int r) {
    __shared__ int64_t part[kSvWG];
    const SvReq q = R.req[r];
    int64_t *cnt = reinterpret_cast<int64_t *>(R.arena + q.off_cnt);
    const int64_t per = (q.n_chunks + kSvWG - 1) / kSvWG;
    const int64_t lo = threadIdx.x * per, hi = lo + per < q.n_chunks ? lo + per : q.n_chunks;
    int64_t s = 0;
    for (int64_t c = lo; c < hi; ++c) s += ld_dc(cnt + c);
    part[threadIdx.x] = s;
    __syncthreads();
    for (int o = 1; o < kSvWG; o <<= 1) {
        const int64_t v = threadIdx.x >= o ? part[threadIdx.x - o] : 0;
        __syncthreads();
        part[threadIdx.x] += v;
        __syncthreads();
    }
    int64_t run = part[threadIdx.x] - s;
    for (int64_t c = lo; c < hi; ++c) {
        const int64_t v = ld_dc(cnt + c);
        st_dc(cnt + c, run);
        run += v;
    }
    if (threadIdx.x == kSvWG - 1) {
        const int64_t total = part[kSvWG - 1];
        int64_t *meta = reinterpret_cast<int64_t *>(R.arena + q.off_meta);
        st_dc(meta, total < q.limit ? total : q.limit);
        if (q.limit == 0) st_dc(meta + 1, int64_t(q.cursor));
        else if (total < q.limit) st_dc(meta + 1, int64_t(q.end));
    }
}

__device__ __forceinline__ void sv_emit(const Dev &S, const SvRound &R, int64_t wg, int64_t G) {
    __shared__ int wc[kSvWG / 64];
    const int lane = lane_id(), wave = threadIdx.x >> 6;
    for (int64_t it = wg; it < R.total_chunks; it += G) {
        const int r = find_req(R, it, true);
        const SvReq q = R.req[r];
        const int64_t c = it - q.chunk_base;
        int64_t rank = ld_dc(reinterpret_cast<const int64_t *>(R.arena + q.off_cnt) + c);
        if (rank >= q.limit) continue;  // uniform per workgroup
        int32_t *sel = reinterpret_cast<int32_t *>(R.arena + q.off_sel);
        int64_t *meta = reinterpret_cast<int64_t *>(R.arena + q.off_meta);
        for (int k = 0; k < kSvChunk / kSvWG; ++k) {
            const uint64_t pos = q.cursor + uint64_t(c) * kSvChunk + uint64_t(k) * kSvWG + threadIdx.x;
            const bool live = entry_live(S, pos, q.end);
            const unsigned long long m = __ballot(live);
            if (lane == 0) wc[wave] = __popcll(m);
            __syncthreads();
            int64_t before = rank, total = 0;
            for (int w = 0; w < kSvWG / 64; ++w) {
                if (w < wave) before += wc[w];
                total += wc[w];
            }
            const int64_t rr = before + lanes_below(m);
            if (live && rr < q.limit) {
                st_dc(sel + rr, int32_t(uint32_t(S.log[pos])));
                if (rr == q.limit - 1) st_dc(meta + 1, int64_t(pos + 1));
            }
            rank += total;
            __syncthreads();
        }
    }
}

// One wave per selected block: its key and 512 MC voxels into the arena (or the caller's
// buffers).
__device__ __forceinline__ void sv_gather(const Dev &S, const SvRound &R, int64_t wg, int64_t G) {
    const int lane = lane_id();
    const int64_t gw = wg * (kSvWG / 64) + (threadIdx.x >> 6);
    const int64_t nw = G * (kSvWG / 64);
    for (int64_t it = gw; it < R.total_items; it += nw) {
        const int r = find_req(R, it, false);
        const SvReq q = R.req[r];
        const int64_t b = it - q.item_base;
        const int64_t count = ld_dc(reinterpret_cast<const int64_t *>(R.arena + q.off_meta));
        if (b >= count) continue;
        const int32_t pool = ld_dc(reinterpret_cast<const int32_t *>(R.arena + q.off_sel) + b);
        const uint4 *src = reinterpret_cast<const uint4 *>(S.MCV + int64_t(pool) * 512);
        uint4 *dst = reinterpret_cast<uint4 *>(q.mc_out ? reinterpret_cast<char *>(q.mc_out) : R.arena + q.off_mc) +
                     b * 128;
        dst[lane] = src[lane];
        dst[lane + 64] = src[lane + 64];
        if (lane < 3) {
            int32_t k[3];
            unpack_key(S.pool_key[pool], k[0], k[1], k[2]);
            int32_t *kd = q.keys_out ? q.keys_out : reinterpret_cast<int32_t *>(R.arena + q.off_keys);
            kd[b * 3 + lane] = k[lane];
        }
    }
}

__global__ void __launch_bounds__(kSvWG) k_sv_count(Dev S, SvRound R) { sv_count(S, R, blockIdx.x, gridDim.x); }
__global__ void __launch_bounds__(kSvWG) k_sv_scan(SvRound R) { sv_scan_one(R, int(blockIdx.x)); }
__global__ void __launch_bounds__(kSvWG) k_sv_emit(Dev S, SvRound R) { sv_emit(S, R, blockIdx.x, gridDim.x); }
__global__ void __launch_bounds__(kSvWG) k_sv_gather(Dev S, SvRound R) { sv_gather(S, R, blockIdx.x, gridDim.x); }

// ----------------------------------------------------------------- persistent form
// One launch serves batches of admitted requests from a ring in pinned host memory until
// the host asks it to stop.  Its workgroups form `teams`; team t takes batches t, t +
// teams, ..., so a batch admitted while another is on the device starts at once on a free
// team.  Within a batch a team runs the four steps of a round, separated by barriers among
// the team's workgroups (all of them resident: the grid is sized to fit the device).  The
// team's first workgroup waits for the batch to be published, copies its descriptors to
// device memory, and after the last step writes each request's count and next cursor and
// the batch's completion word to host memory.  Every wait is bounded in time: a wait that
// expires raises the abort word, and all workgroups leave.
constexpr int kPRing = 8;      // batch slots of the ring
constexpr int kMaxTeams = 4;

struct PBatch {
    int32_t n;  // requests
    int32_t pad;
    int64_t total_chunks, total_items;
    SvReq req[kMaxBatch];
};

// Shared with the host (pinned, coherent, mapped).
struct PHost {
    unsigned long long published;  // batches published in this launch (host)
    unsigned long long stop;       // host: leave once every published batch is done
    unsigned long long err;        // device: a wait expired
    unsigned long long pad;
    unsigned long long done[kPRing];  // batch sequence number + 1, once complete (device)
    int64_t meta[kPRing][kMaxBatch][2];  // count and next cursor per request (device)
    PBatch batch[kPRing];                 // descriptors (host)
};

struct PTeam {
    unsigned int count, gen;  // team barrier
    unsigned int exit, pad;
    PBatch cur;               // the batch being served, copied from host memory
};

struct PDev {
    unsigned int abort;
    unsigned int pad[63];
    PTeam team[kMaxTeams];
};

__device__ __forceinline__ unsigned long long ld_sys(const unsigned long long *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}
__device__ __forceinline__ unsigned int ld_dev(const unsigned int *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Barrier of the team's G workgroups; false if the abort word was raised or the wait took
// longer than `ticks` of the constant wall clock (then this workgroup raises it).  Every
// word that one workgroup writes and another reads within a batch is a device-coherent
// atomic, so a wave only waits for its own accesses to complete before the arrival.
// With `write_back`, the workgroup also writes its XCD's L2 back to memory before it
// arrives: the gather's outputs are plain stores that may sit dirty in that cache, and the
// host hands their arena range to a later batch once this one is complete.  Left dirty,
// such a line could be evicted after the later batch has written its counts or selected
// blocks there (device-scope stores go through to memory) and overwrite them.
__device__ bool team_sync(PDev *P, PTeam &T, unsigned int G, long long ticks, bool write_back = false) {
    __shared__ int ok;
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    if (threadIdx.x == 0) {
        if (write_back) {  // every wave's stores are in L2; the write-back completes before the arrival
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
            __builtin_amdgcn_s_waitcnt(0);
        }
        ok = 1;
        const unsigned int g = ld_dev(&T.gen);
        if (atomicAdd(&T.count, 1u) == G - 1) {
            __hip_atomic_store(&T.count, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __builtin_amdgcn_s_waitcnt(0);
            atomicAdd(&T.gen, 1u);
        } else {
            const long long t0 = wall_clock64();
            while (ld_dev(&T.gen) == g) {
                if (ld_dev(&P->abort) || wall_clock64() - t0 > ticks) {
                    atomicOr(&P->abort, 1u);
                    ok = 0;
                    break;
                }
                __builtin_amdgcn_s_sleep(2);
            }
        }
        if (ld_dev(&P->abort)) ok = 0;
    }
    __syncthreads();
    return ok != 0;
}

__global__ void __launch_bounds__(kSvWG) k_sv_pinit(PDev *P) {
    for (int i = threadIdx.x; i < kMaxTeams; i += blockDim.x) {
        P->team[i].count = 0;
        P->team[i].gen = 0;
        P->team[i].exit = 0;
    }
    if (threadIdx.x == 0) P->abort = 0;
}

__global__ void __launch_bounds__(kSvWG) k_sv_persistent(Dev S, PHost *H, PDev *P, char *arena, int teams,
                                                         long long ticks_idle, long long ticks_step) {
    const int team = int(blockIdx.x) % teams;
    const unsigned int wg = blockIdx.x / unsigned(teams);
    const unsigned int G = (gridDim.x - unsigned(team) + unsigned(teams) - 1) / unsigned(teams);
    PTeam &T = P->team[team];
    __shared__ int state;  // 0 serve, 1 stop, 2 expired
    __shared__ SvReq s_req[kMaxBatch];
    for (unsigned long long b = unsigned(team);; b += unsigned(teams)) {
        const int slot = int(b % kPRing);
        if (wg == 0) {
            if (threadIdx.x == 0) {
                int st = 0;
                const long long t0 = wall_clock64();
                while (ld_sys(&H->published) <= b) {
                    if (ld_sys(&H->stop)) {
                        // the host raises stop after its last publication: a second read of
                        // the count after seeing stop is final
                        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "");
                        if (ld_sys(&H->published) <= b) st = 1;
                        break;
                    }
                    if (ld_dev(&P->abort) || wall_clock64() - t0 > ticks_idle) {
                        st = 2;
                        break;
                    }
                    __builtin_amdgcn_s_sleep(8);
                }
                state = st;
            }
            __syncthreads();
            if (state == 0) {
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "");  // the host's descriptor writes
                const PBatch &src = H->batch[slot];
                const int n = src.n;
                const int64_t *w = reinterpret_cast<const int64_t *>(src.req);
                int64_t *d = reinterpret_cast<int64_t *>(T.cur.req);
                for (int i = threadIdx.x; i < n * int(sizeof(SvReq) / 8); i += kSvWG) st_dc(d + i, w[i]);
                if (threadIdx.x == 0) {
                    st_dc(&T.cur.total_chunks, src.total_chunks);
                    st_dc(&T.cur.total_items, src.total_items);
                    st_dc(&T.cur.n, int32_t(n));
                }
            } else if (threadIdx.x == 0) {
                if (state == 2) atomicOr(&P->abort, 1u);
                __hip_atomic_store(&T.exit, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
        }
        // the other workgroups wait here for the batch (bounded by the idle limit)
        if (!team_sync(P, T, G, ticks_idle) || ld_dev(&T.exit)) break;
        const int n = ld_dc(&T.cur.n);
        {  // this workgroup's copy of the descriptors
            const int64_t *w = reinterpret_cast<const int64_t *>(T.cur.req);
            int64_t *d = reinterpret_cast<int64_t *>(s_req);
            for (int i = threadIdx.x; i < n * int(sizeof(SvReq) / 8); i += kSvWG) d[i] = ld_dc(w + i);
        }
        __syncthreads();
        const SvRound R{s_req, n, ld_dc(&T.cur.total_chunks), ld_dc(&T.cur.total_items), arena};
        sv_count(S, R, wg, G);
        if (!team_sync(P, T, G, ticks_step)) break;
        for (unsigned int r = wg; r < unsigned(R.n); r += G) sv_scan_one(R, int(r));
        if (!team_sync(P, T, G, ticks_step)) break;
        sv_emit(S, R, wg, G);
        if (!team_sync(P, T, G, ticks_step)) break;
        sv_gather(S, R, wg, G);
        if (!team_sync(P, T, G, ticks_step, true)) break;
        if (wg == 0) {  // results to the host, then the completion word
            for (int i = threadIdx.x; i < 2 * R.n; i += kSvWG) {
                const int64_t v = ld_dc(reinterpret_cast<const int64_t *>(arena + R.req[i >> 1].off_meta) + (i & 1));
                __hip_atomic_store(reinterpret_cast<unsigned long long *>(&H->meta[slot][i >> 1][i & 1]),
                                   (unsigned long long)v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
            }
            __builtin_amdgcn_s_waitcnt(0);  // every wave's result stores have completed
            __syncthreads();
            if (threadIdx.x == 0)
                __hip_atomic_store(&H->done[slot], b + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
        }
    }
    if (wg == 0 && threadIdx.x == 0 && ld_dev(&P->abort))
        __hip_atomic_store(&H->err, 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}

__global__ void k_sv_read_log_len(const Counters *C, unsigned long long *out, uint64_t cap) {
    const unsigned long long L = C->log_len;
    out[0] = L < cap ? L : cap;
}

using Clock = std::chrono::steady_clock;


}  // namespace

struct vbh_server {
    vbh_scene *scene = nullptr;
    vbh_server_config cfg{};
    char *arena = nullptr;
    Admission adm;  // client queues, cursors, result slots and arena ranges
    std::vector<hipStream_t> streams;
    hipStream_t istream = nullptr;
    SvReq *d_desc = nullptr;    // [max_inflight][max_batch] device descriptors, one row per round
    SvReq *h_desc = nullptr;    // pinned staging for the same (a row is reused only after its
                                // round completed, so its upload has been consumed)
    int64_t *h_meta = nullptr;  // pinned [max_inflight][2] results copied back
    unsigned long long *d_len = nullptr, *h_len = nullptr;
    uint64_t end_v = 0;            // log end of the published version
    uint32_t version = 0;
    // persistent form
    PHost *H = nullptr;             // pinned, coherent ring shared with the launch (host address)
    PHost *dH = nullptr;            // the same memory as the device addresses it
    PDev *P = nullptr;              // device-side barrier and abort state
    unsigned pgrid = 0;             // workgroups of the launch
    long long ticks_per_s = 100000000;  // constant wall clock of the device
};

namespace {

struct RoundRec {
    hipEvent_t ev;
    int stream;
    int row;  // descriptor row
    std::vector<Admitted> items;
};

double secs(Clock::time_point t0) { return std::chrono::duration<double>(Clock::now() - t0).count(); }

// The device descriptor of an admitted request: its arena range split into the selected
// pool indices, chunk counts, keys, MC voxels and count / next cursor (req_bytes' layout).
void fill_req(SvReq &q, const Admitted &a, const vbh_request &r, int64_t chunk_base, int64_t item_base) {
    q.cursor = a.cursor;
    q.end = a.end;
    q.limit = a.limit;
    q.chunk_base = chunk_base;
    q.n_chunks = a.n_chunks;
    q.item_base = item_base;
    q.off_sel = a.off;
    q.off_cnt = q.off_sel + align256(a.limit * 4);
    q.off_keys = q.off_cnt + align256(a.n_chunks * 8);
    q.off_mc = q.off_keys + align256(a.limit * 12);
    q.off_meta = q.off_mc + align256(a.limit * 2048);
    q.keys_out = r.d_keys_out;
    q.mc_out = reinterpret_cast<uint32_t *>(r.d_mc_out);
}

int read_log_end(vbh_server *v, hipStream_t st, uint64_t *out) {
    k_sv_read_log_len<<<1, 1, 0, st>>>(v->scene->C, v->d_len, uint64_t(v->scene->p.log_capacity));
    VBH_LAUNCHED();
    VBH_HIP(hipMemcpyAsync(v->h_len, v->d_len, 8, hipMemcpyDeviceToHost, st));
    VBH_HIP(hipStreamSynchronize(st));
    *out = v->h_len[0];
    return VBH_OK;
}

// The persistent form of vbh_server_run.  One launch serves the batches of one scene
// version: when a frame is due, the launch is stopped (it finishes the published batches),
// the frame is fused with its MC update, and a new launch serves the next version.  The
// launch is also stopped while no work is pending, and restarted when some arrives.
int run_persistent(vbh_server *v, const vbh_request *reqs, int64_t n_req, const vbh_frame_feed *frames,
                   int64_t n_frames, vbh_request_result *res, Clock::time_point t0) {
    vbh_scene *sc = v->scene;
    PHost *H = v->H;
    hipStream_t st = v->streams[0];
    const int teams = std::min(v->cfg.n_streams, kMaxTeams);
    const long long ticks_idle = 10 * v->ticks_per_s, ticks_step = 5 * v->ticks_per_s;
    struct Batch {
        unsigned long long seq;
        std::vector<Admitted> items;
    };
    Admission &adm = v->adm;
    std::vector<Admitted> admitted;
    std::vector<int64_t> rejected;
    std::deque<Batch> inflight;
    bool running = false;
    unsigned long long published = 0;
    int64_t next_arrival = 0, n_done = 0, fi = 0;
    int rc = VBH_OK;

    auto finish = [&](Batch &bt, int slot, double tdone) {
        for (size_t i = 0; i < bt.items.size(); ++i) {
            const Admitted &f = bt.items[i];
            vbh_request_result &r = res[f.req];
            r.count = H->meta[slot][i][0];
            r.cursor_out = uint64_t(H->meta[slot][i][1]);
            r.done_s = tdone;
            r.status = VBH_OK;
            adm.complete(f, r.cursor_out);
            ++n_done;
        }
    };
    auto poll = [&]() {
        const double tdone = secs(t0);
        for (auto it = inflight.begin(); it != inflight.end();) {
            const int slot = int(it->seq % kPRing);
            if (__atomic_load_n(&H->done[slot], __ATOMIC_ACQUIRE) == it->seq + 1) {
                finish(*it, slot, tdone);
                it = inflight.erase(it);
            } else {
                ++it;
            }
        }
    };
    auto launch = [&]() -> int {
        H->published = 0;
        H->stop = 0;
        H->err = 0;
        for (auto &d : H->done) d = 0;
        published = 0;
        k_sv_pinit<<<1, 64, 0, st>>>(v->P);
        k_sv_persistent<<<v->pgrid, kSvWG, 0, st>>>(sc->d, v->dH, v->P, v->arena, teams, ticks_idle, ticks_step);
        if (hipGetLastError() != hipSuccess) return VBH_EHIP;
        running = true;
        return VBH_OK;
    };
    auto stop = [&]() -> int {
        if (!running) return VBH_OK;
        __atomic_store_n(&H->stop, 1ull, __ATOMIC_RELEASE);
        const hipError_t e = hipStreamSynchronize(st);
        running = false;
        poll();
        if (e != hipSuccess || __atomic_load_n(&H->err, __ATOMIC_ACQUIRE) || !inflight.empty()) return VBH_EHIP;
        return VBH_OK;
    };
    auto fuse = [&](const vbh_frame_feed &fr) -> int {
        if (!fr.d_depth || fr.frame_id <= sc->last_frame) return VBH_EINVAL;
        int r = scene_fuse(sc, fr.d_depth, fr.d_rgb, fr.pose_c2w, fr.frame_id, true, v->istream);
        uint64_t end = 0;
        if (r == VBH_OK) r = read_log_end(v, v->istream, &end);
        if (r == VBH_OK) {
            v->end_v = end;
            v->version = fr.frame_id;
        }
        return r;
    };

    while (n_done < n_req && rc == VBH_OK) {
        const double now = secs(t0);
        while (next_arrival < n_req && reqs[next_arrival].arrival_s <= now) {
            adm.arrive(reqs[next_arrival].client, next_arrival, reqs[next_arrival].limit);
            ++next_arrival;
        }
        if (fi < n_frames && frames[fi].time_s <= now) {  // a new scene version
            rc = stop();
            if (rc == VBH_OK) rc = fuse(frames[fi]);
            ++fi;
            continue;
        }
        // admit one batch into a free ring slot (a stopped launch is restarted first, since a
        // new launch numbers its batches from 0)
        if (!running) {
            if (adm.work_pending()) rc = launch();
            if (rc != VBH_OK) break;
        }
        const int slot = int(published % kPRing);
        bool slot_free = running && inflight.size() < size_t(kPRing);
        for (const Batch &bt : inflight) slot_free = slot_free && int(bt.seq % kPRing) != slot;
        if (slot_free) {
            PBatch &B = H->batch[slot];
            Batch bt;
            bt.seq = published;
            int64_t chunks = 0, items = 0;
            adm.build(v->end_v, admitted, rejected);
            for (const int64_t ri : rejected) {
                res[ri].status = VBH_EINVAL;  // can never fit
                ++n_done;
            }
            for (const Admitted &a : admitted) {
                fill_req(B.req[bt.items.size()], a, reqs[a.req], chunks, items);
                chunks += a.n_chunks;
                items += a.limit;
                res[a.req].arrival_s = reqs[a.req].arrival_s;
                res[a.req].admit_s = now;
                res[a.req].cursor_in = a.cursor;
                res[a.req].version = v->version;
                bt.items.push_back(a);
            }
            if (!bt.items.empty()) {
                B.n = int32_t(bt.items.size());
                B.total_chunks = chunks;
                B.total_items = items;
                __atomic_store_n(&H->published, published + 1, __ATOMIC_RELEASE);
                ++published;
                inflight.push_back(std::move(bt));
            }
        }
        poll();
        if (running && !inflight.empty() && hipStreamQuery(st) != hipErrorNotReady) rc = VBH_EHIP;  // the launch left
        // idle: nothing in flight or queued and the next event is not imminent
        if (running && inflight.empty()) {
            const double next = std::min(next_arrival < n_req ? reqs[next_arrival].arrival_s : 1e300,
                                         fi < n_frames ? frames[fi].time_s : 1e300);
            if (!adm.any_queued() && next - now > 0.5) rc = stop();
        }
        std::this_thread::yield();
    }
    const int rs = stop();
    if (rc == VBH_OK) rc = rs;
    for (; rc == VBH_OK && fi < n_frames; ++fi) {  // the rest of the frame schedule
        while (secs(t0) < frames[fi].time_s) std::this_thread::sleep_for(std::chrono::microseconds(50));
        rc = fuse(frames[fi]);
    }
    return rc;
}

}  // namespace

extern "C" {

int vbh_server_create(vbh_scene *scene, const vbh_server_config *cfg, vbh_server **out) {
    if (!out || !scene || !cfg || cfg->arena_bytes < 4096 || cfg->max_inflight < 1 || cfg->max_inflight > 4096 ||
        cfg->n_streams < 1 || cfg->n_streams > 8 || cfg->n_clients < 1 || cfg->max_batch < 1 ||
        cfg->max_batch > kMaxBatch || int64_t(cfg->max_inflight) * cfg->max_batch > (int64_t(1) << 18) ||
        (cfg->mode != VBH_SERVE_ROUNDS && cfg->mode != VBH_SERVE_PERSISTENT) || cfg->workgroups < 0 ||
        cfg->workgroups > 4096 || (cfg->mode == VBH_SERVE_PERSISTENT && cfg->n_streams > kMaxTeams))
        return VBH_EINVAL;
    *out = nullptr;
    vbh_server *v = new (std::nothrow) vbh_server();
    if (!v) return VBH_ENOMEM;
    v->scene = scene;
    v->cfg = *cfg;
    bool ok = hipMalloc(&v->arena, size_t(cfg->arena_bytes)) == hipSuccess &&
              hipMalloc(&v->d_desc, sizeof(SvReq) * size_t(cfg->max_batch) * cfg->max_inflight) == hipSuccess &&
              hipHostMalloc(&v->h_desc, sizeof(SvReq) * size_t(cfg->max_batch) * cfg->max_inflight) == hipSuccess &&
              hipHostMalloc(&v->h_meta, 16 * size_t(cfg->max_inflight)) == hipSuccess &&
              hipMalloc(&v->d_len, 8) == hipSuccess && hipHostMalloc(&v->h_len, 8) == hipSuccess;
    for (int i = 0; ok && i < cfg->n_streams; ++i) {
        hipStream_t s;
        ok = hipStreamCreateWithFlags(&s, hipStreamNonBlocking) == hipSuccess;
        if (ok) v->streams.push_back(s);
    }
    ok = ok && hipStreamCreateWithFlags(&v->istream, hipStreamNonBlocking) == hipSuccess;
    if (ok && cfg->mode == VBH_SERVE_PERSISTENT) {
        int dev = 0, khz = 0;
        ok = hipHostMalloc(reinterpret_cast<void **>(&v->H), sizeof(PHost), hipHostMallocCoherent | hipHostMallocMapped) ==
                 hipSuccess &&
             hipHostGetDevicePointer(reinterpret_cast<void **>(&v->dH), v->H, 0) == hipSuccess &&
             hipMalloc(&v->P, sizeof(PDev)) == hipSuccess && hipGetDevice(&dev) == hipSuccess &&
             hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev) == hipSuccess;
        if (ok) {
            std::memset(v->H, 0, sizeof(PHost));
            v->ticks_per_s = khz > 0 ? (long long)khz * 1000 : v->ticks_per_s;
            const int64_t want = cfg->workgroups > 0 ? cfg->workgroups : int64_t(scene->cus) * 2;
            v->pgrid = unsigned(std::max<int64_t>(want, std::min(cfg->n_streams, kMaxTeams)));
        }
    }
    if (!ok) {
        vbh_server_destroy(v);
        return VBH_ENOMEM;
    }
    v->adm.init(cfg->n_clients, cfg->max_inflight, cfg->max_batch, cfg->arena_bytes, kSvChunk,
                (scene->p.log_capacity + kSvChunk - 1) / kSvChunk + 1);
    if (read_log_end(v, v->istream, &v->end_v) != VBH_OK) {
        vbh_server_destroy(v);
        return VBH_EHIP;
    }
    v->version = scene->last_frame;
    *out = v;
    return VBH_OK;
}

void vbh_server_destroy(vbh_server *v) {
    if (!v) return;
    for (hipStream_t s : v->streams) {
        (void)hipStreamSynchronize(s);
        (void)hipStreamDestroy(s);
    }
    if (v->istream) {
        (void)hipStreamSynchronize(v->istream);
        (void)hipStreamDestroy(v->istream);
    }
    if (v->arena) (void)hipFree(v->arena);
    if (v->d_desc) (void)hipFree(v->d_desc);
    if (v->h_desc) (void)hipHostFree(v->h_desc);
    if (v->h_meta) (void)hipHostFree(v->h_meta);
    if (v->d_len) (void)hipFree(v->d_len);
    if (v->h_len) (void)hipHostFree(v->h_len);
    if (v->H) (void)hipHostFree(v->H);
    if (v->P) (void)hipFree(v->P);
    delete v;
}

int vbh_server_set_cursor(vbh_server *v, int32_t client, uint64_t cursor) {
    if (!v || client < 0 || client >= v->cfg.n_clients) return VBH_EINVAL;
    v->adm.set_cursor(client, cursor);
    return VBH_OK;
}

int vbh_server_get_cursor(vbh_server *v, int32_t client, uint64_t *cursor) {
    if (!v || !cursor || client < 0 || client >= v->cfg.n_clients) return VBH_EINVAL;
    *cursor = v->adm.cursor(client);
    return VBH_OK;
}

int vbh_server_run(vbh_server *v, const vbh_request *reqs, int64_t n_req, const vbh_frame_feed *frames,
                   int64_t n_frames, vbh_request_result *res) {
    if (!v || n_req < 0 || n_frames < 0 || (n_req > 0 && (!reqs || !res)) || (n_frames > 0 && !frames))
        return VBH_EINVAL;
    for (int64_t i = 0; i < n_req; ++i) {
        if (reqs[i].client < 0 || reqs[i].client >= v->cfg.n_clients || reqs[i].limit < 0 ||
            (i > 0 && reqs[i].arrival_s < reqs[i - 1].arrival_s))
            return VBH_EINVAL;
        res[i] = vbh_request_result{};
        res[i].status = 1;  // pending
    }
    vbh_scene *sc = v->scene;
    // The scene may have changed through its own entry points since the last run (frames,
    // written or reset blocks): serve from its state now.
    if (read_log_end(v, v->istream, &v->end_v) != VBH_OK) return VBH_EHIP;
    v->version = sc->last_frame;
    v->adm.begin_run();
    const auto t0 = Clock::now();
    if (v->cfg.mode == VBH_SERVE_PERSISTENT) return run_persistent(v, reqs, n_req, frames, n_frames, res, t0);
    // --- gate between serving and the MC update of fused frames
    McGate gate_mc;
    std::atomic<int> int_error{VBH_OK};
    std::atomic<bool> int_done{n_frames == 0};
    std::thread integ([&]() {
        for (int64_t f = 0; f < n_frames; ++f) {
            const vbh_frame_feed &fr = frames[f];
            while (secs(t0) < fr.time_s) std::this_thread::sleep_for(std::chrono::microseconds(50));
            if (!fr.d_depth || fr.frame_id <= sc->last_frame) {
                int_error = VBH_EINVAL;
                break;
            }
            int rc = scene_fuse(sc, fr.d_depth, fr.d_rgb, fr.pose_c2w, fr.frame_id, false, v->istream);
            if (rc == VBH_OK) rc = hipStreamSynchronize(v->istream) == hipSuccess ? VBH_OK : VBH_EHIP;
            if (rc != VBH_OK) {
                int_error = rc;
                break;
            }
            gate_mc.acquire();
            rc = scene_mc_update(sc, fr.frame_id, v->istream);
            uint64_t end = 0;
            if (rc == VBH_OK) rc = read_log_end(v, v->istream, &end);
            gate_mc.release([&] {
                if (rc == VBH_OK) {
                    v->end_v = end;
                    v->version = fr.frame_id;
                }
            });
            if (rc != VBH_OK) {
                int_error = rc;
                break;
            }
        }
        int_done = true;
        gate_mc.finish();
    });

    // --- scheduler (this thread)
    Admission &adm = v->adm;
    std::vector<Admitted> admitted;
    std::vector<int64_t> rejected;
    std::vector<int> free_rows;
    for (int i = v->cfg.max_inflight - 1; i >= 0; --i) free_rows.push_back(i);
    std::deque<RoundRec> rounds;
    std::vector<hipEvent_t> ev_pool;
    int64_t next_arrival = 0, n_done = 0;
    int next_stream = 0;
    int rc_all = VBH_OK;
    while (n_done < n_req && rc_all == VBH_OK) {
        const double now = secs(t0);
        while (next_arrival < n_req && reqs[next_arrival].arrival_s <= now) {
            adm.arrive(reqs[next_arrival].client, next_arrival, reqs[next_arrival].limit);
            ++next_arrival;
        }
        uint64_t end_v = 0;
        uint32_t ver = 0;
        const bool gate = gate_mc.poll(rounds.empty(), [&] {
            end_v = v->end_v;
            ver = v->version;
        });
        // admit and launch one round
        if (!gate && !free_rows.empty()) {
            const int si = next_stream;
            const int row = free_rows.back();
            SvReq *hd = v->h_desc + int64_t(row) * v->cfg.max_batch;
            RoundRec rr;
            rr.stream = si;
            rr.row = row;
            int64_t chunks = 0, items = 0;
            adm.build(end_v, admitted, rejected);
            for (const int64_t ri : rejected) {
                res[ri].status = VBH_EINVAL;  // can never fit
                ++n_done;
            }
            for (const Admitted &a : admitted) {
                fill_req(hd[rr.items.size()], a, reqs[a.req], chunks, items);
                chunks += a.n_chunks;
                items += a.limit;
                res[a.req].arrival_s = reqs[a.req].arrival_s;
                res[a.req].admit_s = now;
                res[a.req].cursor_in = a.cursor;
                res[a.req].version = ver;
                rr.items.push_back(a);
            }
            if (!rr.items.empty()) {
                free_rows.pop_back();
                hipStream_t st = v->streams[size_t(si)];
                SvReq *dd = v->d_desc + int64_t(row) * v->cfg.max_batch;
                const int n = int(rr.items.size());
                int e = hipMemcpyAsync(dd, hd, sizeof(SvReq) * size_t(n), hipMemcpyHostToDevice, st) != hipSuccess;
                SvRound R{dd, n, chunks, items, v->arena};
                const unsigned gc = unsigned(std::min<int64_t>(std::max<int64_t>(chunks, 1), int64_t(sc->cus) * 8));
                const unsigned gg =
                    unsigned(std::min<int64_t>(std::max<int64_t>((items + 3) / 4, 1), int64_t(sc->cus) * 16));
                if (chunks > 0) k_sv_count<<<gc, kSvWG, 0, st>>>(sc->d, R);
                k_sv_scan<<<unsigned(n), kSvWG, 0, st>>>(R);
                if (chunks > 0) k_sv_emit<<<gc, kSvWG, 0, st>>>(sc->d, R);
                if (items > 0) k_sv_gather<<<gg, kSvWG, 0, st>>>(sc->d, R);
                e |= hipGetLastError() != hipSuccess;
                for (int i = 0; i < n; ++i)
                    e |= hipMemcpyAsync(v->h_meta + 2 * rr.items[size_t(i)].slot, v->arena + hd[i].off_meta, 16,
                                        hipMemcpyDeviceToHost, st) != hipSuccess;
                if (ev_pool.empty()) {
                    hipEvent_t ev;
                    e |= hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess;
                    ev_pool.push_back(ev);
                }
                rr.ev = ev_pool.back();
                ev_pool.pop_back();
                e |= hipEventRecord(rr.ev, st) != hipSuccess;
                if (e) {
                    rc_all = VBH_EHIP;
                    break;
                }
                rounds.push_back(std::move(rr));
                next_stream = (next_stream + 1) % v->cfg.n_streams;
            }
        }
        // completions (rounds on one stream finish in order; poll all)
        for (auto it = rounds.begin(); it != rounds.end();) {
            const hipError_t q = hipEventQuery(it->ev);
            if (q == hipErrorNotReady) {
                ++it;
                continue;
            }
            if (q != hipSuccess) {
                rc_all = VBH_EHIP;
                break;
            }
            const double tdone = secs(t0);
            for (const Admitted &f : it->items) {
                const int64_t *m = v->h_meta + 2 * f.slot;
                vbh_request_result &r = res[f.req];
                r.count = m[0];
                r.cursor_out = uint64_t(m[1]);
                r.done_s = tdone;
                r.status = VBH_OK;
                adm.complete(f, r.cursor_out);
                ++n_done;
            }
            ev_pool.push_back(it->ev);
            free_rows.push_back(it->row);
            it = rounds.erase(it);
        }
        if (int_error != VBH_OK) rc_all = int_error;
        std::this_thread::yield();
    }
    // drain outstanding GPU work and let integration finish its schedule
    for (hipStream_t s : v->streams) (void)hipStreamSynchronize(s);
    rounds.clear();
    while (!int_done) {
        (void)gate_mc.poll(true, [] {});
        std::this_thread::sleep_for(std::chrono::microseconds(50));
    }
    integ.join();
    for (hipEvent_t e : ev_pool) (void)hipEventDestroy(e);
    if (rc_all == VBH_OK && int_error != VBH_OK) rc_all = int_error;
    return rc_all;
}

}  // extern "C"
