// Client geometry from MC voxels (Sec. 4.3): the exploration client turns received MC
// voxel blocks into triangles, placing each vertex at the midpoint of a cube edge whose
// corners lie on different sides of the surface (no interpolation, Sec. 6).
//
// Triangulation rule per case (a fixed table built on the host at first use):
//   - corner k (Lorensen-Cline numbering) is inside iff bit k of the case index is set;
//   - on each of the 6 cube faces the crossing edges are paired: two crossings make one
//     segment; four (the face's inside corners diagonal) make one segment around each
//     inside corner, so the two cells sharing a face always pair it alike;
//   - the segments close into loops, found in order of their lowest edge number; a loop
//     runs so that its normal points from the inside corners to the outside ones, starts
//     at its lowest edge and is cut into a fan (e0, ei, ei+1).
// Output order: block, then cell (x fastest), then the cell's triangles in table order.
//
// Launches: per-block triangle counts (wave per block), per-chunk exclusive scan (one
// workgroup per 1024 blocks), a scan of the chunk totals (one workgroup), and the
// emission (wave per block, one 64-cell slice at a time, consecutive lanes writing
// consecutive output words).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>
#include <vector>

#include "device.hpp"
#include "host.hpp"
#include "vbh.h"

namespace vbh {
namespace {

constexpr int kBlock = 256;
constexpr int kWaves = kBlock / 64;
constexpr int kChunk = 1024;  // blocks per scan chunk (one 1024-thread workgroup)
constexpr int kMaxTri = 5;    // the rule never yields more triangles per cell (checked on build)

__constant__ uint8_t c_ntri[256];
__constant__ int8_t c_tri[256][3 * kMaxTri];
__constant__ uint8_t c_edge_mid[12][3];  // corner_a + corner_b per axis (doubled midpoint)

// ---------------------------------------------------------------- table (host)
const int kCube[8][3] = {{0, 0, 0}, {1, 0, 0}, {1, 1, 0}, {0, 1, 0}, {0, 0, 1}, {1, 0, 1}, {1, 1, 1}, {0, 1, 1}};
const int kEdgeEnds[12][2] = {{0, 1}, {1, 2}, {2, 3}, {3, 0}, {4, 5}, {5, 6},
                              {6, 7}, {7, 4}, {0, 4}, {1, 5}, {2, 6}, {3, 7}};

int edge_between(int a, int b) {
    for (int e = 0; e < 12; ++e) {
        const int p = kEdgeEnds[e][0], q = kEdgeEnds[e][1];
        if ((p == a && q == b) || (p == b && q == a)) return e;
    }
    return -1;
}

struct Table {
    uint8_t ntri[256];
    int8_t tri[256][3 * kMaxTri];
    uint8_t mid[12][3];
    bool ok = true;
};

// The 6 faces as corner cycles: corners sharing coordinate `axis` = `side`, in cyclic order.
void face_cycles(int out[6][4]) {
    int f = 0;
    for (int axis = 0; axis < 3; ++axis) {
        for (int side = 0; side < 2; ++side) {
            const int u = (axis + 1) % 3, v = (axis + 2) % 3;
            const int ring[4][2] = {{0, 0}, {1, 0}, {1, 1}, {0, 1}};
            for (int i = 0; i < 4; ++i) {
                for (int k = 0; k < 8; ++k) {
                    if (kCube[k][axis] == side && kCube[k][u] == ring[i][0] && kCube[k][v] == ring[i][1]) {
                        out[f][i] = k;
                        break;
                    }
                }
            }
            ++f;
        }
    }
}

Table build_table() {
    Table T{};
    for (int e = 0; e < 12; ++e)
        for (int c = 0; c < 3; ++c) T.mid[e][c] = uint8_t(kCube[kEdgeEnds[e][0]][c] + kCube[kEdgeEnds[e][1]][c]);
    int faces[6][4];
    face_cycles(faces);
    for (int idx = 0; idx < 256; ++idx) {
        const auto inside = [idx](int k) { return (idx >> k) & 1; };
        int link[12][2], deg[12] = {};
        const auto join = [&](int a, int b) {
            link[a][deg[a]++] = b;
            link[b][deg[b]++] = a;
        };
        for (const auto &cyc : faces) {
            int cr[4], n = 0;
            for (int i = 0; i < 4; ++i)
                if (inside(cyc[i]) != inside(cyc[(i + 1) % 4])) cr[n++] = edge_between(cyc[i], cyc[(i + 1) % 4]);
            if (n == 2) join(cr[0], cr[1]);
            if (n == 4)
                for (int i = 0; i < 4; ++i)
                    if (inside(cyc[i]))
                        join(edge_between(cyc[(i + 3) % 4], cyc[i]), edge_between(cyc[i], cyc[(i + 1) % 4]));
        }
        std::vector<int> out;
        bool seen[12] = {};
        for (int start = 0; start < 12; ++start) {
            if (deg[start] == 0 || seen[start]) continue;
            std::vector<int> loop;
            int from = -1, at = start;
            do {
                loop.push_back(at);
                seen[at] = true;
                const int to = (from < 0) ? std::min(link[at][0], link[at][1])
                                          : (link[at][0] == from ? link[at][1] : link[at][0]);
                from = at;
                at = to;
            } while (at != start);
            // orientation: Newell normal of the doubled midpoints against inside -> outside
            long nx = 0, ny = 0, nz = 0, dx = 0, dy = 0, dz = 0;
            const int L = int(loop.size());
            for (int i = 0; i < L; ++i) {
                const uint8_t *p = T.mid[loop[i]], *q = T.mid[loop[(i + 1) % L]];
                nx += long(p[1] - q[1]) * long(p[2] + q[2]);
                ny += long(p[2] - q[2]) * long(p[0] + q[0]);
                nz += long(p[0] - q[0]) * long(p[1] + q[1]);
                const int a = kEdgeEnds[loop[i]][0], b = kEdgeEnds[loop[i]][1];
                const int in = inside(a) ? a : b, outc = inside(a) ? b : a;
                dx += kCube[outc][0] - kCube[in][0];
                dy += kCube[outc][1] - kCube[in][1];
                dz += kCube[outc][2] - kCube[in][2];
            }
            if (nx * dx + ny * dy + nz * dz < 0) std::reverse(loop.begin(), loop.end());
            std::rotate(loop.begin(), std::min_element(loop.begin(), loop.end()), loop.end());
            for (int i = 1; i + 1 < L; ++i) {
                out.push_back(loop[0]);
                out.push_back(loop[i]);
                out.push_back(loop[i + 1]);
            }
        }
        if (out.size() > size_t(3 * kMaxTri)) {
            T.ok = false;
            continue;
        }
        T.ntri[idx] = uint8_t(out.size() / 3);
        for (int i = 0; i < 3 * kMaxTri; ++i) T.tri[idx][i] = i < int(out.size()) ? int8_t(out[size_t(i)]) : int8_t(-1);
    }
    // cut-off: indices 0 and 255 have no crossing edge, so no triangle
    return T;
}

// Uploads the table to the current device once (each device holds its own constants).
int ensure_table() {
    static std::mutex mu;
    static std::vector<int> ready;
    static Table T = build_table();
    if (!T.ok) return VBH_EINVAL;
    int dev = 0;
    VBH_HIP(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lock(mu);
    if (std::find(ready.begin(), ready.end(), dev) != ready.end()) return VBH_OK;
    VBH_HIP(hipMemcpyToSymbol(HIP_SYMBOL(c_ntri), T.ntri, sizeof(T.ntri)));
    VBH_HIP(hipMemcpyToSymbol(HIP_SYMBOL(c_tri), T.tri, sizeof(T.tri)));
    VBH_HIP(hipMemcpyToSymbol(HIP_SYMBOL(c_edge_mid), T.mid, sizeof(T.mid)));
    VBH_HIP(hipDeviceSynchronize());
    ready.push_back(dev);
    return VBH_OK;
}

// ---------------------------------------------------------------- kernels
__device__ __forceinline__ int cell_ntri(uint32_t v) { return c_ntri[v & 0xFFu]; }

__device__ __forceinline__ int wave_excl_scan(int v, int &total) {
    int x = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int y = __shfl_up(x, o);
        if (lane_id() >= o) x += y;
    }
    total = __shfl(x, 63);
    return x - v;
}

__global__ void __launch_bounds__(kBlock) k_tri_count(const uint32_t *mcv, int64_t n, int64_t *cnt) {
    const int lane = lane_id();
    const int64_t gw = int64_t(blockIdx.x) * kWaves + (threadIdx.x >> 6);
    const int64_t nw = int64_t(gridDim.x) * kWaves;
    for (int64_t b = gw; b < n; b += nw) {
        int c = 0;
#pragma unroll
        for (int j = 0; j < 8; ++j) c += cell_ntri(mcv[b * 512 + lane + 64 * j]);
        c = wave_sum(c);
        if (lane == 0) cnt[b] = c;
    }
}

// Exclusive scan of a chunk of kChunk counts in place; chunk total to sums[chunk].
__global__ void __launch_bounds__(kChunk) k_tri_chunk(int64_t *cnt, int64_t n, int64_t *sums) {
    __shared__ int64_t wsum[kChunk / 64];
    const int64_t i = int64_t(blockIdx.x) * kChunk + threadIdx.x;
    const int64_t v = i < n ? cnt[i] : 0;
    int64_t x = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int64_t y = __shfl_up(x, o);
        if (lane_id() >= o) x += y;
    }
    const int w = threadIdx.x >> 6;
    if (lane_id() == 63) wsum[w] = x;
    __syncthreads();
    if (threadIdx.x < 64) {
        int64_t s = threadIdx.x < kChunk / 64 ? wsum[threadIdx.x] : 0;
        int64_t t = s;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const int64_t y = __shfl_up(t, o);
            if (lane_id() >= o) t += y;
        }
        if (threadIdx.x < kChunk / 64) wsum[threadIdx.x] = t - s;
        if (threadIdx.x == kChunk / 64 - 1) sums[blockIdx.x] = t;
    }
    __syncthreads();
    if (i < n) cnt[i] = x - v + wsum[w];
}

// Exclusive scan of the chunk totals (one workgroup, tiles of kChunk); sums[nchunks] = total.
__global__ void __launch_bounds__(kChunk) k_tri_scan_sums(int64_t *sums, int64_t nchunks) {
    __shared__ int64_t wsum[kChunk / 64];
    __shared__ int64_t carry;
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    for (int64_t base = 0; base < nchunks; base += kChunk) {
        const int64_t i = base + threadIdx.x;
        const int64_t v = i < nchunks ? sums[i] : 0;
        int64_t x = v;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const int64_t y = __shfl_up(x, o);
            if (lane_id() >= o) x += y;
        }
        const int w = threadIdx.x >> 6;
        if (lane_id() == 63) wsum[w] = x;
        __syncthreads();
        if (threadIdx.x < 64) {
            int64_t s = threadIdx.x < kChunk / 64 ? wsum[threadIdx.x] : 0;
            int64_t t = s;
#pragma unroll
            for (int o = 1; o < 64; o <<= 1) {
                const int64_t y = __shfl_up(t, o);
                if (lane_id() >= o) t += y;
            }
            if (threadIdx.x < kChunk / 64) wsum[threadIdx.x] = t - s;
        }
        __syncthreads();
        const int64_t c = carry;
        if (i < nchunks) sums[i] = c + x - v + wsum[w];
        __syncthreads();  // everyone has read carry
        if (threadIdx.x == kChunk - 1) carry = c + x + wsum[w];
        __syncthreads();
    }
    if (threadIdx.x == 0) sums[nchunks] = carry;
}

// LDS written by one lane and read by another lane of the same wavefront: the wavefront
// executes its LDS operations in order, so only the compiler must not move them across.
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

constexpr int kSlabTri = 64 * kMaxTri;  // triangles of one wavefront's 64 cells, at most

// Wave per block, 64 cells (one z slice) at a time.  The slice's triangles are contiguous
// in the output; each lane records in LDS which of its triangles it holds, then
// consecutive lanes write consecutive words of the slice's output, each looking up the
// lane (cell) its word belongs to, so every store is coalesced.
__global__ void __launch_bounds__(kBlock) k_tri_emit(const int32_t *keys, const uint32_t *mcv, int64_t n,
                                                     const int64_t *off, const int64_t *sums, float half, float *pos,
                                                     uint8_t *rgb, int64_t cap) {
    // the case table in LDS: every output word looks up its triangle's edge
    __shared__ int8_t s_tri[256 * 3 * kMaxTri];
    __shared__ uint8_t s_mid[12 * 3];
    __shared__ uint8_t s_owner[kWaves][kSlabTri];  // lane holding each triangle of the slice
    for (int i = threadIdx.x; i < 256 * 3 * kMaxTri; i += kBlock) s_tri[i] = (&c_tri[0][0])[i];
    if (threadIdx.x < 36) s_mid[threadIdx.x] = (&c_edge_mid[0][0])[threadIdx.x];
    __syncthreads();
    const int lane = lane_id();
    const int64_t gw = int64_t(blockIdx.x) * kWaves + (threadIdx.x >> 6);
    const int64_t nw = int64_t(gridDim.x) * kWaves;
    for (int64_t b = gw; b < n; b += nw) {
        int64_t base = sums[b / kChunk] + off[b];
        const int64_t kx2 = 16 * int64_t(keys[3 * b]), ky2 = 16 * int64_t(keys[3 * b + 1]);
        const int64_t kz2 = 16 * int64_t(keys[3 * b + 2]);
        for (int j = 0; j < 8; ++j) {
            const uint32_t v = mcv[b * 512 + lane + 64 * j];
            const int idx = int(v & 0xFFu);
            int total;
            const int nt = c_ntri[idx];
            const int lo = wave_excl_scan(nt, total);
            if (total == 0) continue;
            uint8_t *const own = s_owner[threadIdx.x >> 6];
            for (int t = 0; t < nt; ++t) own[lo + t] = uint8_t(lane);
            wave_lds_sync();
            const int64_t room = cap - base;  // triangles of this slice that fit the output
            const int keep = room >= total ? total : (room > 0 ? int(room) : 0);
            float *const gp = pos + base * 9;
            for (int q0 = 0; q0 < keep * 9; q0 += 64) {
                const int q = q0 + lane;
                const int qq = q < keep * 9 ? q : keep * 9 - 1;
                const int t = qq / 9, comp = qq - 9 * (qq / 9);
                const int L = own[t];
                const int oidx = __shfl(idx, L), olo = __shfl(lo, L);
                const int e = s_tri[oidx * 3 * kMaxTri + 3 * (t - olo) + comp / 3];
                const int c = comp % 3;
                const int64_t g2 = c == 0 ? kx2 + 2 * (L & 7) : (c == 1 ? ky2 + 2 * (L >> 3) : kz2 + 2 * j);
                const float val = float(g2 + s_mid[3 * e + c]) * half;
                if (q < keep * 9) gp[q] = val;
            }
            if (rgb) {
                uint8_t *const gc = rgb + base * 3;
                for (int q0 = 0; q0 < keep * 3; q0 += 64) {
                    const int q = q0 + lane;
                    const int qq = q < keep * 3 ? q : keep * 3 - 1;
                    const int t = qq / 3;
                    const uint32_t ov = __shfl(v, int(own[t]));
                    if (q < keep * 3) gc[q] = uint8_t(ov >> (8 * (qq - 3 * t + 1)));
                }
            }
            wave_lds_sync();  // the slice's owners are read before the next slice writes them
            base += total;
        }
    }
}

unsigned waves_grid(int64_t items) {
    const int64_t want = int64_t(device_cus()) * 8;
    const int64_t need = (items + kWaves - 1) / kWaves;
    return unsigned(need < want ? (need > 0 ? need : 1) : want);
}

}  // namespace
}  // namespace vbh

using namespace vbh;

extern "C" {

int vbh_mc_case(int32_t index, int8_t *h_edges) {
    static const Table T = build_table();
    if (index < 0 || index > 255 || !T.ok) return VBH_EINVAL;
    if (h_edges)
        for (int i = 0; i < 3 * kMaxTri; ++i) h_edges[i] = T.tri[index][i];
    return T.ntri[index];
}

int64_t vbh_mc_work_size(int64_t n) {
    if (n < 0) return -1;
    return n + (n + kChunk - 1) / kChunk + 1;
}

}  // extern "C"

namespace {
// Workspace of the allocation-free triangulation: the per-block counts and chunk sums of
// up to VBH_MC_STATIC_MAX_BLOCKS blocks, resident on every device the library runs on.
constexpr int64_t kStaticWork = VBH_MC_STATIC_MAX_BLOCKS + (VBH_MC_STATIC_MAX_BLOCKS + kChunk - 1) / kChunk + 1;
__device__ __align__(256) int64_t scratch[kStaticWork];

// Device address of `scratch` on the current device, looked up once per device.
int static_work(int64_t **out) {
    static std::mutex mu;
    static std::vector<std::pair<int, int64_t *>> addr;
    int dev = 0;
    VBH_HIP(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lock(mu);
    for (const auto &a : addr)
        if (a.first == dev) {
            *out = a.second;
            return VBH_OK;
        }
    void *p = nullptr;
    VBH_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) return VBH_EHIP;
    addr.emplace_back(dev, static_cast<int64_t *>(p));
    *out = static_cast<int64_t *>(p);
    return VBH_OK;
}
}  // namespace

extern "C" {

int vbh_mc_triangulate_static(const int32_t *d_keys, const uint32_t *d_mcv, int64_t n, float voxel_size,
                              float *d_pos, uint8_t *d_rgb, int64_t cap, int64_t *h_count, void *stream) {
    if (n < 0 || n > VBH_MC_STATIC_MAX_BLOCKS) return VBH_EINVAL;
    int64_t *work = nullptr;
    if (int rc = static_work(&work)) return rc;
    return vbh_mc_triangulate(d_keys, d_mcv, n, voxel_size, d_pos, d_rgb, cap, work, h_count, stream);
}

int vbh_mc_triangulate(const int32_t *d_keys, const uint32_t *d_mcv, int64_t n, float voxel_size, float *d_pos,
                       uint8_t *d_rgb, int64_t cap, int64_t *d_work, int64_t *h_count, void *stream) {
    if (n < 0 || cap < 0 || !(voxel_size > 0.0f) || (n > 0 && (!d_keys || !d_mcv || !d_work)) ||
        (cap > 0 && !d_pos))
        return VBH_EINVAL;
    if (int rc = ensure_table()) return rc;
    if (n == 0) {
        if (h_count) *h_count = 0;
        return VBH_OK;
    }
    hipStream_t st = as_stream(stream);
    const int64_t nchunks = (n + kChunk - 1) / kChunk;
    int64_t *off = d_work, *sums = d_work + n;
    k_tri_count<<<waves_grid(n), kBlock, 0, st>>>(d_mcv, n, off);
    k_tri_chunk<<<unsigned(nchunks), kChunk, 0, st>>>(off, n, sums);
    k_tri_scan_sums<<<1, kChunk, 0, st>>>(sums, nchunks);
    VBH_LAUNCHED();
    int64_t total = 0;
    VBH_HIP(hipMemcpyAsync(&total, sums + nchunks, sizeof(total), hipMemcpyDeviceToHost, st));
    VBH_HIP(hipStreamSynchronize(st));
    if (h_count) *h_count = total;
    if (cap > 0 && total > 0) {
        k_tri_emit<<<waves_grid(n), kBlock, 0, st>>>(d_keys, d_mcv, n, off, sums, 0.5f * voxel_size, d_pos, d_rgb,
                                                     cap);
        VBH_LAUNCHED();
    }
    return VBH_OK;
}

}  // extern "C"
