// Concurrent GPU hash map (Sec. 5: retrieval, insertion, removal) - kernels and C ABI.
//
// One device thread per operation; a batch is one launch.  See device.hpp for the
// probing protocol and why every operation completes below capacity.  A map created by
// vbh_map_create_chained holds the paper's chained design instead (chain.hip); every
// other entry point dispatches on which of the two a handle holds.
#include <hip/hip_runtime.h>

#include <cstdlib>
#include <new>

#include "chain.hpp"
#include "device.hpp"
#include "host.hpp"
#include "vbh.h"

using namespace vbh;

struct vbh_map {
    uint32_t tag = kTagMap;  // handle kind, read by vbh_status
    Slot *table = nullptr;
    uint64_t slots = 0;
    int hash_kind = 0;
    uint32_t *err = nullptr;        // sticky error bits
    unsigned long long *cnt = nullptr;  // [0] live, [1] tombstones (scratch for size/export)
    ChainMap *chain = nullptr;          // set for the chained design (then table is unused)
};

namespace {

constexpr int kBlock = 256;

__global__ void __launch_bounds__(kBlock) k_table_init(Slot *T, uint64_t n) {
    for (uint64_t i = blockIdx.x * uint64_t(kBlock) + threadIdx.x; i < n; i += uint64_t(gridDim.x) * kBlock) {
        Slot s;
        s.key = kEmpty;
        s.val = kPending;
        s.stamp = 0;
        T[i] = s;
    }
}

// Single-kind or mixed batch.  OPC < 0: the kind is read from ops[i].
template <int OPC>
__global__ void __launch_bounds__(kBlock) k_map_batch(Slot *T, uint64_t mask, int kind, const uint8_t *ops,
                                                      const int32_t *keys, const int32_t *vals, int64_t n,
                                                      int32_t *out, uint32_t *err) {
    const int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x;
    if (i >= n) return;
    const int op = OPC >= 0 ? OPC : int(ops[i]);
    const int32_t x = keys[3 * i], y = keys[3 * i + 1], z = keys[3 * i + 2];
    int32_t r;
    if (op > 2) {
        raise_err(err, kErrKeyRange);
        r = -1;
    } else {
        r = map_op(T, mask, kind, op, x, y, z, (op == 0 && vals) ? vals[i] : 0, err);
    }
    out[i] = r;
}

__global__ void __launch_bounds__(kBlock) k_zero_u64(unsigned long long *p, int n) {
    if (threadIdx.x < n) p[threadIdx.x] = 0;
}

// Counts live keys and tombstones.
__global__ void __launch_bounds__(kBlock) k_count(const Slot *T, uint64_t n, unsigned long long *cnt) {
    unsigned long long live = 0, tomb = 0;
    for (uint64_t i = blockIdx.x * uint64_t(kBlock) + threadIdx.x; i < n; i += uint64_t(gridDim.x) * kBlock) {
        const uint64_t k = T[i].key;
        live += (k >> 63) == 0;
        tomb += k == kTomb;
    }
    live = wave_sum(live);
    tomb = wave_sum(tomb);
    if (lane_id() == 0) {
        if (live) atomicAdd(&cnt[0], live);
        if (tomb) atomicAdd(&cnt[1], tomb);
    }
}

// Compacts live entries (slot order is not preserved across waves).
__global__ void __launch_bounds__(kBlock) k_export(const Slot *T, uint64_t n, int32_t *keys, int32_t *vals,
                                                   int64_t cap, unsigned long long *cnt) {
    const uint64_t stride = uint64_t(gridDim.x) * kBlock;
    const uint64_t start = blockIdx.x * uint64_t(kBlock) + threadIdx.x;
    // iterate uniformly per wave so the wave-aggregated append sees every lane
    const uint64_t wave_base = start - uint64_t(lane_id());
    for (uint64_t b = wave_base; b < n; b += stride) {
        const uint64_t i = b + uint64_t(lane_id());
        const bool live = i < n && (T[i].key >> 63) == 0;
        const unsigned long long pos = wave_append<unsigned long long>(live, &cnt[0]);
        if (live && int64_t(pos) < cap) {
            int32_t x, y, z;
            unpack_key(T[i].key, x, y, z);
            keys[3 * pos] = x;
            keys[3 * pos + 1] = y;
            keys[3 * pos + 2] = z;
            if (vals) vals[pos] = T[i].val;
        }
    }
}

// Re-inserts live entries of `src` into the fresh table `dst` (keys are unique, so each
// claims a distinct EMPTY slot).
__global__ void __launch_bounds__(kBlock) k_rebuild(const Slot *src, uint64_t n, Slot *dst, uint64_t mask, int kind,
                                                    uint32_t *err) {
    for (uint64_t i = blockIdx.x * uint64_t(kBlock) + threadIdx.x; i < n; i += uint64_t(gridDim.x) * kBlock) {
        const Slot s = src[i];
        if (s.key >> 63) continue;
        int32_t x, y, z;
        unpack_key(s.key, x, y, z);
        bool claimed;
        const int64_t p = probe_claim(dst, mask, s.key, home_slot(x, y, z, s.key, kind, mask), claimed);
        if (p < 0) {
            raise_err(err, kErrTableFull);
            continue;
        }
        dst[p].val = s.val;
        dst[p].stamp = s.stamp;
    }
}

// Thread per operation: one 64-bit compare-and-swap at a pseudo-random word of `a` (a
// SplitMix64 step of the operation index picks it), expecting the word's initial value,
// so with n_words >> n_ops nearly every CAS is uncontended.  The count of successes goes
// to *won (one atomic per workgroup).
__global__ void __launch_bounds__(kBlock) k_cas_ceiling(unsigned long long *a, uint64_t mask, int64_t n_ops,
                                                        uint64_t seed, unsigned long long *won) {
    __shared__ unsigned long long wg;
    if (threadIdx.x == 0) wg = 0;
    __syncthreads();
    unsigned long long mine = 0;
    for (int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x; i < n_ops; i += int64_t(gridDim.x) * kBlock) {
        uint64_t z = seed + uint64_t(i) * 0x9E3779B97F4A7C15ull;
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
        z ^= z >> 31;
        const uint64_t w = z & mask;
        mine += atomicCAS(a + w, 0ull, uint64_t(i) + 1) == 0ull;
    }
    mine = wave_sum(mine);
    if (lane_id() == 0 && mine) atomicAdd(&wg, mine);
    __syncthreads();
    if (threadIdx.x == 0 && wg) atomicAdd(won, wg);
}

int launch_init(Slot *T, uint64_t n, hipStream_t st) {
    k_table_init<<<grid_for(int64_t(n), kBlock, 8192), kBlock, 0, st>>>(T, n);
    VBH_LAUNCHED();
    return VBH_OK;
}

int batch(vbh_map *m, int opc, const uint8_t *ops, const int32_t *keys, const int32_t *vals, int64_t n, int32_t *out,
          void *stream) {
    if (!m || n < 0 || (n > 0 && (!keys || !out))) return VBH_EINVAL;
    if (opc < 0 && n > 0 && !ops) return VBH_EINVAL;
    if (n == 0) return VBH_OK;
    hipStream_t st = as_stream(stream);
    if (m->chain) return chain_batch(m->chain, m->hash_kind, opc, ops, keys, vals, n, out, m->err, st);
    const unsigned g = grid_for(n, kBlock);
    const uint64_t mask = m->slots - 1;
    switch (opc) {
        case 0: k_map_batch<0><<<g, kBlock, 0, st>>>(m->table, mask, m->hash_kind, ops, keys, vals, n, out, m->err); break;
        case 1: k_map_batch<1><<<g, kBlock, 0, st>>>(m->table, mask, m->hash_kind, ops, keys, vals, n, out, m->err); break;
        case 2: k_map_batch<2><<<g, kBlock, 0, st>>>(m->table, mask, m->hash_kind, ops, keys, vals, n, out, m->err); break;
        default: k_map_batch<-1><<<g, kBlock, 0, st>>>(m->table, mask, m->hash_kind, ops, keys, vals, n, out, m->err);
    }
    VBH_LAUNCHED();
    return VBH_OK;
}

}  // namespace

namespace vbh {
int table_init(Slot *T, uint64_t n, hipStream_t st) { return launch_init(T, n, st); }

int device_cus() {
    int dev = 0, cus = 256;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        return 256;
    return cus > 0 ? cus : 256;
}
}  // namespace vbh

extern "C" {

const char *vbh_strerror(int code) {
    switch (code) {
        case VBH_OK: return "ok";
        case VBH_EINVAL: return "invalid argument or key out of range";
        case VBH_ENOMEM: return "device allocation failed";
        case VBH_EHIP: return "HIP runtime error";
        case VBH_EFULL_TABLE: return "hash table full";
        case VBH_EFULL_POOL: return "voxel block pool exhausted";
        case VBH_EFULL_LOG: return "update log full";
        case VBH_ESPIN: return "bounded wait for a concurrent insert expired";
        default: return "unknown error";
    }
}

int vbh_version(void) { return 1; }

int vbh_map_create(uint64_t slots, int32_t hash_kind, vbh_map **out) {
    if (!out || !is_pow2(slots) || slots < 64 || slots > (1ull << 31) || hash_kind < 0 || hash_kind > 1)
        return VBH_EINVAL;
    *out = nullptr;
    vbh_map *m = new (std::nothrow) vbh_map();
    if (!m) return VBH_ENOMEM;
    m->slots = slots;
    m->hash_kind = hash_kind;
    if (hipMalloc(&m->table, slots * sizeof(Slot)) != hipSuccess || hipMalloc(&m->err, 256) != hipSuccess) {
        vbh_map_destroy(m);
        return VBH_ENOMEM;
    }
    m->cnt = reinterpret_cast<unsigned long long *>(reinterpret_cast<char *>(m->err) + 64);
    if (hipMemset(m->err, 0, 256) != hipSuccess || launch_init(m->table, slots, nullptr) != VBH_OK ||
        hipDeviceSynchronize() != hipSuccess) {
        vbh_map_destroy(m);
        return VBH_EHIP;
    }
    *out = m;
    return VBH_OK;
}

int vbh_map_create_chained(uint64_t buckets, uint64_t excess, int32_t hash_kind, vbh_map **out) {
    if (!out || !is_pow2(buckets) || buckets < 64 || excess > kChainMaxEntries ||
        buckets + excess > kChainMaxEntries || hash_kind < 0 || hash_kind > 1)
        return VBH_EINVAL;
    *out = nullptr;
    vbh_map *m = new (std::nothrow) vbh_map();
    if (!m) return VBH_ENOMEM;
    m->slots = buckets;
    m->hash_kind = hash_kind;
    if (chain_create(buckets, excess, &m->chain) != VBH_OK || hipMalloc(&m->err, 256) != hipSuccess) {
        vbh_map_destroy(m);
        return VBH_ENOMEM;
    }
    m->cnt = reinterpret_cast<unsigned long long *>(reinterpret_cast<char *>(m->err) + 64);
    if (hipMemset(m->err, 0, 256) != hipSuccess || chain_clear(m->chain, nullptr) != VBH_OK ||
        hipDeviceSynchronize() != hipSuccess) {
        vbh_map_destroy(m);
        return VBH_EHIP;
    }
    *out = m;
    return VBH_OK;
}

void vbh_map_destroy(vbh_map *m) {
    if (!m) return;
    if (m->chain) chain_destroy(m->chain);
    if (m->table) (void)hipFree(m->table);
    if (m->err) (void)hipFree(m->err);
    delete m;
}

int vbh_insert(vbh_map *m, const int32_t *d_keys, const int32_t *d_vals, int64_t n, int32_t *d_status, void *stream) {
    if (n > 0 && !d_vals) return VBH_EINVAL;
    return batch(m, 0, nullptr, d_keys, d_vals, n, d_status, stream);
}
int vbh_find(vbh_map *m, const int32_t *d_keys, int64_t n, int32_t *d_vals_out, void *stream) {
    return batch(m, 1, nullptr, d_keys, nullptr, n, d_vals_out, stream);
}
int vbh_erase(vbh_map *m, const int32_t *d_keys, int64_t n, int32_t *d_status, void *stream) {
    return batch(m, 2, nullptr, d_keys, nullptr, n, d_status, stream);
}
int vbh_apply(vbh_map *m, const uint8_t *d_ops, const int32_t *d_keys, const int32_t *d_vals, int64_t n,
              int32_t *d_out, void *stream) {
    return batch(m, -1, d_ops, d_keys, d_vals, n, d_out, stream);
}

int vbh_map_size(vbh_map *m, int64_t *h_live, int64_t *h_tombstones, void *stream) {
    if (!m) return VBH_EINVAL;
    hipStream_t st = as_stream(stream);
    k_zero_u64<<<1, 64, 0, st>>>(m->cnt, 2);
    if (m->chain) {
        if (chain_count(m->chain, m->cnt, st) != VBH_OK) return VBH_EHIP;
    } else {
        k_count<<<grid_for(int64_t(m->slots), kBlock, 2048), kBlock, 0, st>>>(m->table, m->slots, m->cnt);
    }
    VBH_LAUNCHED();
    unsigned long long h[2];
    VBH_HIP(hipMemcpyAsync(h, m->cnt, sizeof(h), hipMemcpyDeviceToHost, st));
    VBH_HIP(hipStreamSynchronize(st));
    if (h_live) *h_live = int64_t(h[0]);
    if (h_tombstones) *h_tombstones = int64_t(h[1]);
    return VBH_OK;
}

int vbh_map_export(vbh_map *m, int32_t *d_keys, int32_t *d_vals, int64_t cap, int64_t *h_count, void *stream) {
    if (!m || cap < 0 || (cap > 0 && !d_keys)) return VBH_EINVAL;
    hipStream_t st = as_stream(stream);
    k_zero_u64<<<1, 64, 0, st>>>(m->cnt, 2);
    if (m->chain) {
        if (chain_export(m->chain, d_keys, d_vals, cap, m->cnt, st) != VBH_OK) return VBH_EHIP;
    } else {
        k_export<<<grid_for(int64_t(m->slots), kBlock, 4096), kBlock, 0, st>>>(m->table, m->slots, d_keys, d_vals,
                                                                                cap, m->cnt);
    }
    VBH_LAUNCHED();
    unsigned long long h = 0;
    VBH_HIP(hipMemcpyAsync(&h, m->cnt, sizeof(h), hipMemcpyDeviceToHost, st));
    VBH_HIP(hipStreamSynchronize(st));
    if (h_count) *h_count = int64_t(h);
    return VBH_OK;
}

int vbh_map_rebuild(vbh_map *m, void *stream) {
    if (!m) return VBH_EINVAL;
    if (m->chain) return VBH_OK;  // no tombstones: emptied entries are reused directly
    hipStream_t st = as_stream(stream);
    Slot *fresh = nullptr;
    if (hipMalloc(&fresh, m->slots * sizeof(Slot)) != hipSuccess) return VBH_ENOMEM;
    if (launch_init(fresh, m->slots, st) != VBH_OK) {
        (void)hipFree(fresh);
        return VBH_EHIP;
    }
    k_rebuild<<<grid_for(int64_t(m->slots), kBlock, 8192), kBlock, 0, st>>>(m->table, m->slots, fresh, m->slots - 1,
                                                                             m->hash_kind, m->err);
    if (hipGetLastError() != hipSuccess || hipStreamSynchronize(st) != hipSuccess) {
        (void)hipFree(fresh);
        return VBH_EHIP;
    }
    (void)hipFree(m->table);
    m->table = fresh;
    return VBH_OK;
}

int vbh_cas_ceiling(unsigned long long *d_words, int64_t n_words, int64_t n_ops, uint64_t seed,
                    unsigned long long *d_won, void *stream) {
    if (!d_words || !d_won || n_words < 1 || (n_words & (n_words - 1)) || n_ops < 0) return VBH_EINVAL;
    hipStream_t st = as_stream(stream);
    k_cas_ceiling<<<grid_for(n_ops, kBlock, 1u << 16), kBlock, 0, st>>>(d_words, uint64_t(n_words - 1), n_ops, seed,
                                                                        d_won);
    VBH_LAUNCHED();
    return VBH_OK;
}

int vbh_map_clear(vbh_map *m, void *stream) {
    if (!m) return VBH_EINVAL;
    if (m->chain) return chain_clear(m->chain, as_stream(stream));
    return launch_init(m->table, m->slots, as_stream(stream));
}

int vbh_map_status(vbh_map *m, void *stream) {
    if (!m) return VBH_EINVAL;
    hipStream_t st = as_stream(stream);
    uint32_t bits = 0;
    VBH_HIP(hipMemcpyAsync(&bits, m->err, sizeof(bits), hipMemcpyDeviceToHost, st));
    VBH_HIP(hipStreamSynchronize(st));
    if (bits) VBH_HIP(hipMemset(m->err, 0, sizeof(uint32_t)));
    return code_from_bits(bits);
}

}  // extern "C"
