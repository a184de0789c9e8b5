// Chained concurrent hash map of Sec. 5 - the paper's own design, kept beside the
// open-addressing map as a second implementation of the same C ABI.
//
// Layout.  An entry array holds nb buckets followed by nx excess entries.  A key hashes
// to its bucket; keys that collide there are kept in a singly linked list of excess
// entries hanging off the bucket, reached through each entry's link field.  A stack
// holds the excess entries that are free.  Every entry carries an occupancy flag and a
// lock bit (Sec. 5, Insertion and Removal).
//
// Invariant (Sec. 5): while a batch runs, an entry never changes position and the link
// out of an entry is never cleared, so a thread that stands on an entry unlinked by a
// concurrent removal still reaches the rest of the list.  Retrieval is therefore
// read-only.
//
// Operations are non-blocking attempts retried until they succeed (Sec. 5, Insertion):
//   find    walk from the bucket; a key counts when its entry is occupied;
//   insert  walk (retrieval); if the key is absent and the bucket holds no key, lock the
//           bucket, check again that it is free, store, mark occupied, unlock; otherwise
//           lock the list's last entry, check again that it is still last, pop a free
//           entry from the stack, store, mark occupied with an empty link, link, unlock;
//   erase   at the bucket: lock, check, mark unoccupied (the first list entry is not
//           moved into the bucket); inside the list: lock the previous and the current
//           entry, mark the current entry unoccupied keeping its link, relink the
//           previous entry past it, unlock both.
// Locks are only ever tried, never waited for: a failed try releases what it holds and
// the attempt is repeated in the next iteration of the lane's loop, in which every lane
// of the wavefront takes part, so a lock holder in the same wavefront always proceeds.
//
// gfx950 adaptations (the data structure and the steps above are the paper's):
//   * Lock, occupancy flag, link and value share one 64-bit link word, so taking a lock
//     with a compare-and-swap also re-checks the entry's state in the same atomic step
//     (the paper's second check after locking), and a single-entry change folds lock,
//     check and unlock into that one CAS.
//   * The key lives in a second word.  Both words carry a lifetime bit that flips each
//     time an entry is reused; a reader pairs the two words only when the bits agree and
//     otherwise repeats the attempt.  With this, device-scope relaxed atomics suffice:
//     no release/acquire fence (an L2 write-back or invalidate per access on gfx950)
//     orders the key store against the link store.
//   * Entries emptied by a batch return to the stack, and emptied buckets become usable,
//     only in a short pass after the batch (a per-batch retire log).  Within a batch an
//     entry therefore has at most one new lifetime, which makes one lifetime bit enough,
//     and keeps an emptied entry (whose link is still followed by concurrent readers)
//     from being re-linked elsewhere while they stand on it.  The same pass clears the
//     link of an emptied list entry (the paper clears it when the entry is reused): a
//     reader that reaches a reused entry through its new link may still see the entry's
//     previous link word, which must then end the walk rather than lead elsewhere.
#include <hip/hip_runtime.h>

#include <new>

#include "chain.hpp"
#include "device.hpp"
#include "host.hpp"

namespace vbh {
namespace {

constexpr int kBlock = 256;
constexpr int kBatchBlock = 1024;
constexpr uint64_t kLock = 1ull << 63;
constexpr uint64_t kOcc = 1ull << 62;
constexpr uint64_t kDead = 1ull << 60;  // bucket emptied by the running batch
constexpr uint64_t kLinkMask = kChainMaxEntries << 32;
constexpr uint64_t kKeyBits = ~0ull >> 1;

__device__ __forceinline__ uint64_t link_of(uint64_t b) { return (b >> 32) & kChainMaxEntries; }
__device__ __forceinline__ uint64_t with_link(uint64_t b, uint64_t e) { return (b & ~kLinkMask) | (e << 32); }
__device__ __forceinline__ uint64_t life_b(uint64_t b) { return (b >> 61) & 1ull; }
__device__ __forceinline__ uint64_t life_a(uint64_t a) { return a >> 63; }
__device__ __forceinline__ int32_t value_of(uint64_t b) { return int32_t(uint32_t(b)); }

__device__ __forceinline__ uint64_t ld_a(const ChainEntry *E, uint64_t i) {
    return __hip_atomic_load(&E[i].a, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint64_t ld_b(const ChainEntry *E, uint64_t i) {
    return __hip_atomic_load(&E[i].b, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_a(ChainEntry *E, uint64_t i, uint64_t v) {
    __hip_atomic_store(&E[i].a, (unsigned long long)v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_b(ChainEntry *E, uint64_t i, uint64_t v) {
    __hip_atomic_store(&E[i].b, (unsigned long long)v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
// Try-lock / conditional update: succeeds only if the link word is still `expect`.
__device__ __forceinline__ bool cas_b(ChainEntry *E, uint64_t i, uint64_t expect, uint64_t desired) {
    return atomicCAS(&E[i].b, (unsigned long long)expect, (unsigned long long)desired) == expect;
}

// Result of one retrieval walk (Sec. 5, Retrieval) from a bucket.
struct Walk {
    int64_t hit;        // entry holding the key, or -1
    int64_t prev;       // entry whose link led to `hit` (-1: hit is the bucket)
    uint64_t hit_b, prev_b;
    int64_t last;       // last entry of the list when the key is absent
    uint64_t last_b;
    uint64_t bucket_b;  // link word of the bucket as read by this walk
    bool again;         // an entry was caught between lifetimes: repeat the attempt
    bool broken;        // a link out of range or a walk longer than the array (never expected)
};

__device__ __forceinline__ Walk walk(const ChainEntry *E, uint64_t bucket, uint64_t key, uint64_t total,
                                     uint32_t *err) {
    Walk w;
    w.hit = -1;
    w.prev = -1;
    w.hit_b = w.prev_b = 0;
    w.last = -1;
    w.last_b = 0;
    w.again = false;
    w.broken = false;
    uint64_t i = bucket, prev_b = 0;
    int64_t prev = -1;
    // Both words of an entry are requested together (one trip per entry); the lifetime
    // check below accepts them in either order of arrival.
    w.bucket_b = ld_b(E, bucket);
    uint64_t b = w.bucket_b, a = ld_a(E, bucket);
    // A link only ever points at an entry linked after the one holding it, so a walk
    // visits each entry at most once.
    for (uint64_t s = 0; s < total; ++s) {
        if (b & kOcc) {
            if (life_a(a) != life_b(b)) {
                w.again = true;
                return w;
            }
            if ((a & kKeyBits) == key) {
                w.hit = int64_t(i);
                w.hit_b = b;
                w.prev = prev;
                w.prev_b = prev_b;
                return w;
            }
        }
        const uint64_t n = link_of(b);
        if (n == 0) {
            w.last = int64_t(i);
            w.last_b = b;
            return w;
        }
        if (n >= total) break;  // never happens; guards the next load
        prev = int64_t(i);
        prev_b = b;
        i = n;
        b = ld_b(E, i);
        a = ld_a(E, i);
    }
    raise_err(err, kErrSpin);
    w.broken = true;
    return w;
}

// Batch kernel.  Updating batches run a workgroup-wide loop so that the stack pops and the
// retire-log appends of all 1024 lanes of an iteration cost one global atomic each (the
// counters are single words that every workgroup hits); retrieval-only batches run a
// wavefront-wide loop in 256-lane workgroups.  Either way every lane of a wavefront runs every iteration, so a
// lock taken by one lane is released within that iteration whatever the other lanes do,
// and no lane ever waits for another workgroup inside an iteration.
template <int OPC>
__global__ void __launch_bounds__(kBatchBlock) k_chain_batch(ChainEntry *E, const uint32_t *stack, uint32_t *retire,
                                                             ChainCtl *ctl, uint64_t nb, uint64_t total, int kind,
                                                             const uint8_t *ops, const int32_t *keys,
                                                             const int32_t *vals, int64_t n, int32_t *out,
                                                             uint32_t *err) {
    constexpr bool kUpdates = OPC != 1;
    __shared__ unsigned long long s_cnt[3];  // this iteration's pops, list and bucket retirements
    const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (!kUpdates && t >= n) return;
    const bool in = t < n;
    const int op = !in ? 1 : (OPC >= 0 ? OPC : int(ops[t]));
    const int32_t x = in ? keys[3 * t] : 0, y = in ? keys[3 * t + 1] : 0, z = in ? keys[3 * t + 2] : 0;
    const int32_t val = (in && op == 0 && vals) ? vals[t] : 0;
    int32_t res = -1;
    bool active = in;
    if (in && op > 2) {
        raise_err(err, kErrKeyRange);
        active = false;
    } else if (in && (!key_ok(x, y, z) || (op == 0 && val == kAbsent))) {
        // a key out of range, or an insert of the reserved value VBH_ABSENT
        raise_err(err, kErrKeyRange);
        res = op == 1 ? kAbsent : -1;
        active = false;
    }
    const uint64_t key = active ? pack_key(x, y, z) : 0;
    const uint64_t bucket = active ? home_slot(x, y, z, key, kind, nb - 1) : 0;
    const unsigned long long top = ctl->top;  // fixed while the batch runs
    uint32_t tries = 0;
    if (kUpdates) {
        if (threadIdx.x < 3) s_cnt[threadIdx.x] = 0;
        __syncthreads();
    }
    while (kUpdates ? __syncthreads_or(active) != 0 : __ballot(active) != 0) {
        bool need_entry = false, retired = false, again = false;
        uint64_t last = 0, last_b = 0, emptied = 0;
        if (active) {
            const Walk w = walk(E, bucket, key, total, err);
            if (w.broken) {
                res = op == 1 ? kAbsent : VBH_ESPIN;
                active = false;
            } else if (w.again) {
                again = true;
            } else if (op == 1) {
                res = w.hit >= 0 ? value_of(w.hit_b) : kAbsent;
                active = false;
            } else if (op == 0) {
                const uint64_t bb = w.bucket_b;
                if (w.hit >= 0) {
                    res = 0;
                    active = false;
                } else if (!(bb & (kOcc | kDead))) {
                    // The bucket holds no key: lock it, checking in the same CAS that it is
                    // still free and unchanged, store the key, mark occupied, unlock.
                    if (!(bb & kLock) && cas_b(E, bucket, bb, bb | kLock)) {
                        const uint64_t life = life_b(bb) ^ 1ull;
                        st_a(E, bucket, key | (life << 63));
                        st_b(E, bucket, (bb & kLinkMask) | kOcc | (life << 61) | uint64_t(uint32_t(val)));
                        res = 1;
                        active = false;
                    } else {
                        again = true;  // a concurrent insert may be storing this very key
                    }
                } else if (w.last >= 0 && !(w.last_b & kLock) &&
                           (uint64_t(w.last) == bucket || (w.last_b & kOcc))) {
                    // Append: lock the last entry, checking in the same CAS that it is still
                    // last and occupied; a free entry is popped below for the whole wave.
                    if (cas_b(E, uint64_t(w.last), w.last_b, w.last_b | kLock)) {
                        need_entry = true;
                        last = uint64_t(w.last);
                        last_b = w.last_b;
                    } else {
                        again = true;
                    }
                } else {
                    again = true;  // last entry locked or between lifetimes
                }
            } else {
                if (w.hit < 0) {
                    res = 0;
                    active = false;
                } else if (w.hit_b & kLock) {
                    again = true;
                } else if (w.prev < 0) {
                    // At the bucket: unoccupied, link kept; the bucket is reusable after the batch.
                    if (cas_b(E, bucket, w.hit_b, (w.hit_b & ~kOcc) | kDead)) {
                        res = 1;
                        active = false;
                        retired = true;
                        emptied = bucket;
                    } else {
                        again = true;
                    }
                } else {
                    const uint64_t p = uint64_t(w.prev), pb = w.prev_b, c = uint64_t(w.hit), cb = w.hit_b;
                    if ((pb & kLock) || !(p == bucket || (pb & kOcc)) || !cas_b(E, p, pb, pb | kLock)) {
                        again = true;
                    } else if (!cas_b(E, c, cb, cb | kLock)) {
                        st_b(E, p, pb);  // release the previous entry unchanged
                        again = true;
                    } else {
                        st_b(E, c, cb & ~kOcc);                  // unoccupied, link kept, unlocked
                        st_b(E, p, with_link(pb, link_of(cb)));  // skip it, unlocked
                        res = 1;
                        active = false;
                        retired = true;
                        emptied = c;
                    }
                }
            }
        }
        if (kUpdates) {
            // Pops and retirements of the whole workgroup: wavefront counts into LDS, one
            // global atomic per counter, then each lane's position.
            const bool ret_x = retired && emptied >= nb, ret_b = retired && emptied < nb;
            const unsigned long long mp = __ballot(need_entry), mx = __ballot(ret_x), mb = __ballot(ret_b);
            unsigned long long wp = 0, wx = 0, wb = 0;
            if (lane_id() == 0) {
                if (mp) wp = atomicAdd(&s_cnt[0], (unsigned long long)__popcll(mp));
                if (mx) wx = atomicAdd(&s_cnt[1], (unsigned long long)__popcll(mx));
                if (mb) wb = atomicAdd(&s_cnt[2], (unsigned long long)__popcll(mb));
            }
            __syncthreads();
            // three lanes claim the three global ranges at once (used, retired_x, retired_b
            // are consecutive words of the control block)
            if (threadIdx.x < 3) {
                const unsigned long long c = s_cnt[threadIdx.x];
                s_cnt[threadIdx.x] = c ? atomicAdd(&ctl->used + threadIdx.x, c) : 0ull;
            }
            __syncthreads();
            const unsigned long long slot = s_cnt[0] + __shfl(wp, 0) + (unsigned long long)lanes_below(mp);
            const unsigned long long rx = s_cnt[1] + __shfl(wx, 0) + (unsigned long long)lanes_below(mx);
            const unsigned long long rb = s_cnt[2] + __shfl(wb, 0) + (unsigned long long)lanes_below(mb);
            __syncthreads();
            if (threadIdx.x < 3) s_cnt[threadIdx.x] = 0;  // next adds follow the loop's barrier
            if (need_entry) {
                if (slot < top) {
                    const uint64_t e = stack[top - 1 - slot];
                    const uint64_t life = life_b(ld_b(E, e)) ^ 1ull;  // e is unreachable until linked
                    st_a(E, e, key | (life << 63));
                    st_b(E, e, kOcc | (life << 61) | uint64_t(uint32_t(val)));  // empty link, unlocked
                    st_b(E, last, with_link(last_b, e));                         // link, unlock
                    res = 1;
                } else {
                    st_b(E, last, last_b);  // unlock unchanged
                    raise_err(err, kErrTableFull);
                    res = VBH_EFULL_TABLE;
                }
                active = false;
            }
            // an entry empties at most once per batch, so the two ends never meet
            if (ret_x && rx < total) retire[rx] = uint32_t(emptied);
            if (ret_b && rb < total) retire[total - 1 - rb] = uint32_t(emptied);
        }
        if (again && ++tries > kSpinLimit) {
            raise_err(err, kErrSpin);
            res = op == 1 ? kAbsent : VBH_ESPIN;
            active = false;
        }
    }
    if (in) out[t] = res;
}

// After a batch: emptied buckets become usable, emptied list entries go back on the stack
// (at the positions the batch's pops freed, then above).
__global__ void __launch_bounds__(kBlock) k_chain_retire(ChainEntry *E, uint32_t *stack, const uint32_t *retire,
                                                         const ChainCtl *ctl, uint64_t total, uint64_t nx,
                                                         int64_t cap) {
    const int64_t t = int64_t(blockIdx.x) * kBlock + threadIdx.x;
    if (t >= cap) return;
    const unsigned long long used = ctl->used < ctl->top ? ctl->used : ctl->top;
    const unsigned long long base = ctl->top - used;
    if (t < int64_t(ctl->retired_x)) {
        const uint64_t e = retire[t];
        // The link of an emptied list entry was kept while the batch ran (readers standing
        // on it still follow it); now that no reader is left, clear it, so that a reader of
        // the next batch that meets the entry before its new contents are visible sees an
        // empty entry ending the list instead of a link into a list it left.
        E[e].b &= ~kLinkMask;
        if (base + t < nx) stack[base + t] = uint32_t(e);  // it was in use, so there is room
    }
    if (t < int64_t(ctl->retired_b)) E[retire[total - 1 - t]].b &= ~kDead;
}

__global__ void k_chain_finish(ChainCtl *ctl) {
    const unsigned long long used = ctl->used < ctl->top ? ctl->used : ctl->top;
    ctl->top = ctl->top - used + ctl->retired_x;
    ctl->used = 0;
    ctl->retired_x = 0;
    ctl->retired_b = 0;
}

__global__ void __launch_bounds__(kBlock) k_chain_init(ChainEntry *E, uint64_t total, uint32_t *stack, uint64_t nb,
                                                       uint64_t nx, ChainCtl *ctl) {
    const uint64_t stride = uint64_t(gridDim.x) * kBlock;
    for (uint64_t i = blockIdx.x * uint64_t(kBlock) + threadIdx.x; i < total; i += stride) {
        E[i].a = 0;
        E[i].b = 0;
        // the first pops take the lowest excess entries
        if (i < nx) stack[i] = uint32_t(nb + nx - 1 - i);
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        ctl->top = nx;
        ctl->used = ctl->retired_x = ctl->retired_b = 0;
    }
}

__global__ void __launch_bounds__(kBlock) k_chain_count(const ChainEntry *E, uint64_t total, unsigned long long *cnt) {
    unsigned long long live = 0;
    for (uint64_t i = blockIdx.x * uint64_t(kBlock) + threadIdx.x; i < total; i += uint64_t(gridDim.x) * kBlock)
        live += (E[i].b & kOcc) != 0;
    live = wave_sum(live);
    if (lane_id() == 0 && live) atomicAdd(cnt, live);
}

__global__ void __launch_bounds__(kBlock) k_chain_export(const ChainEntry *E, uint64_t total, int32_t *keys,
                                                         int32_t *vals, int64_t cap, unsigned long long *cnt) {
    const uint64_t stride = uint64_t(gridDim.x) * kBlock;
    const uint64_t wave_base = blockIdx.x * uint64_t(kBlock) + threadIdx.x - uint64_t(lane_id());
    for (uint64_t base = wave_base; base < total; base += stride) {
        const uint64_t i = base + uint64_t(lane_id());
        const bool live = i < total && (E[i].b & kOcc);
        const unsigned long long pos = wave_append<unsigned long long>(live, cnt);
        if (live && int64_t(pos) < cap) {
            int32_t x, y, z;
            unpack_key(E[i].a & kKeyBits, x, y, z);
            keys[3 * pos] = x;
            keys[3 * pos + 1] = y;
            keys[3 * pos + 2] = z;
            if (vals) vals[pos] = value_of(E[i].b);
        }
    }
}

}  // namespace

int chain_create(uint64_t buckets, uint64_t excess, ChainMap **out) {
    *out = nullptr;
    ChainMap *c = new (std::nothrow) ChainMap();
    if (!c) return VBH_ENOMEM;
    c->nb = buckets;
    c->nx = excess;
    const uint64_t total = buckets + excess;
    if (hipMalloc(&c->E, total * sizeof(ChainEntry)) != hipSuccess ||
        hipMalloc(&c->stack, (excess ? excess : 1) * sizeof(uint32_t)) != hipSuccess ||
        hipMalloc(&c->retire, total * sizeof(uint32_t)) != hipSuccess ||
        hipMalloc(&c->ctl, sizeof(ChainCtl)) != hipSuccess) {
        chain_destroy(c);
        return VBH_ENOMEM;
    }
    *out = c;
    return VBH_OK;
}

void chain_destroy(ChainMap *c) {
    if (!c) return;
    if (c->E) (void)hipFree(c->E);
    if (c->stack) (void)hipFree(c->stack);
    if (c->retire) (void)hipFree(c->retire);
    if (c->ctl) (void)hipFree(c->ctl);
    delete c;
}

int chain_clear(ChainMap *c, hipStream_t st) {
    const uint64_t total = c->nb + c->nx;
    k_chain_init<<<grid_for(int64_t(total), kBlock, 8192), kBlock, 0, st>>>(c->E, total, c->stack, c->nb, c->nx,
                                                                             c->ctl);
    VBH_LAUNCHED();
    return VBH_OK;
}

int chain_batch(ChainMap *c, int hash_kind, int opc, const uint8_t *ops, const int32_t *keys, const int32_t *vals,
                int64_t n, int32_t *out, uint32_t *err, hipStream_t st) {
    const int block = opc == 1 ? kBlock : kBatchBlock;  // retrieval needs no workgroup-wide loop
    const unsigned g = grid_for(n, block);
    const uint64_t total = c->nb + c->nx;
#define VBH_CHAIN_LAUNCH(OPC)                                                                                    \
    k_chain_batch<OPC><<<g, block, 0, st>>>(c->E, c->stack, c->retire, c->ctl, c->nb, total, hash_kind, ops, keys, \
                                             vals, n, out, err)
    switch (opc) {
        case 0: VBH_CHAIN_LAUNCH(0); break;
        case 1: VBH_CHAIN_LAUNCH(1); break;
        case 2: VBH_CHAIN_LAUNCH(2); break;
        default: VBH_CHAIN_LAUNCH(-1);
    }
#undef VBH_CHAIN_LAUNCH
    VBH_LAUNCHED();
    if (opc == 1) return VBH_OK;  // retrieval changes nothing
    if (opc != 0) {
        // at most one retirement per operation and per entry
        const int64_t cap = n < int64_t(total) ? n : int64_t(total);
        k_chain_retire<<<grid_for(cap, kBlock), kBlock, 0, st>>>(c->E, c->stack, c->retire, c->ctl, total, c->nx,
                                                                   cap);
        VBH_LAUNCHED();
    }
    k_chain_finish<<<1, 1, 0, st>>>(c->ctl);
    VBH_LAUNCHED();
    return VBH_OK;
}

int chain_count(const ChainMap *c, unsigned long long *cnt, hipStream_t st) {
    const uint64_t total = c->nb + c->nx;
    k_chain_count<<<grid_for(int64_t(total), kBlock, 2048), kBlock, 0, st>>>(c->E, total, cnt);
    VBH_LAUNCHED();
    return VBH_OK;
}

int chain_export(const ChainMap *c, int32_t *keys, int32_t *vals, int64_t cap, unsigned long long *cnt,
                 hipStream_t st) {
    const uint64_t total = c->nb + c->nx;
    k_chain_export<<<grid_for(int64_t(total), kBlock, 4096), kBlock, 0, st>>>(c->E, total, keys, vals, cap, cnt);
    VBH_LAUNCHED();
    return VBH_OK;
}

}  // namespace vbh
