// Device-side building blocks of the voxel-block-hashing path on gfx950 (wave64).
//
// Hash table: open addressing over 16-byte slots {key, value, stamp}.  The key word is
// a 63-bit offset-binary packing of the int3 block coordinate; EMPTY and TOMB have the
// top bit set, which no live key has.  Slots only ever move EMPTY -> key -> TOMB, so a
// key never changes position while the table is in use - the device analogue of the
// invariant of Sec. 5 that entry positions and links are preserved, which makes
// retrieval read-only and lets a single 64-bit CAS decide every race:
//   insert  claims the first EMPTY slot of its probe sequence (never a tombstone), so two
//           concurrent inserts of one key meet at the same slot and the CAS picks one;
//   erase   turns the key into TOMB with a CAS (one eraser wins);
//   find    stops at the key or at the first EMPTY slot.
// A value is published after its key; a reader that sees the key with the PENDING value
// re-reads the slot in the next iteration of its single probe loop (no nested spin, so
// a writer in the same wavefront always makes progress), bounded by kSpinLimit.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#pragma clang fp contract(off)

namespace vbh {

constexpr uint64_t kEmpty = ~0ull;
constexpr uint64_t kTomb = ~0ull - 1ull;
constexpr int32_t kPending = INT32_MIN;  // value not yet published
constexpr int32_t kAbsent = INT32_MIN;   // find() result for a missing key
constexpr int32_t kNoPool = -2;          // block key inserted but no pool block left
constexpr int64_t kKeyOff = int64_t(1) << 20;
constexpr uint32_t kSpinLimit = 1u << 20;

// sticky error bits (host maps them to VBH_E* codes)
enum : uint32_t {
    kErrKeyRange = 1u,
    kErrTableFull = 2u,
    kErrPoolFull = 4u,
    kErrLogFull = 8u,
    kErrSpin = 16u,
};

struct alignas(16) Slot {
    unsigned long long key;
    int32_t val;
    uint32_t stamp;  // last frame that touched this block (scene tables)
};
static_assert(sizeof(Slot) == 16, "slot layout");

__device__ __forceinline__ bool key_ok(int32_t x, int32_t y, int32_t z) {
    return x >= -kKeyOff && x < kKeyOff && y >= -kKeyOff && y < kKeyOff && z >= -kKeyOff && z < kKeyOff;
}

__device__ __forceinline__ uint64_t pack_key(int32_t x, int32_t y, int32_t z) {
    return (uint64_t(int64_t(x) + kKeyOff) << 42) | (uint64_t(int64_t(y) + kKeyOff) << 21) |
           uint64_t(int64_t(z) + kKeyOff);
}

__device__ __forceinline__ void unpack_key(uint64_t k, int32_t &x, int32_t &y, int32_t &z) {
    constexpr uint64_t m = (1ull << 21) - 1;
    x = int32_t(int64_t((k >> 42) & m) - kKeyOff);
    y = int32_t(int64_t((k >> 21) & m) - kKeyOff);
    z = int32_t(int64_t(k & m) - kKeyOff);
}

__device__ __forceinline__ uint64_t mix64(uint64_t x) {
    x ^= x >> 33;
    x *= 0xFF51AFD7ED558CCDull;
    x ^= x >> 33;
    x *= 0xC4CEB9FE1A85EC53ull;
    x ^= x >> 33;
    return x;
}

// Home slot: kind 0 = spatial hash with the primes of Sec. 5 (uint32 wrap-around,
// power-of-two n), kind 1 = 64-bit finalizer of the packed key.
__device__ __forceinline__ uint64_t home_slot(int32_t x, int32_t y, int32_t z, uint64_t key, int kind,
                                              uint64_t mask) {
    if (kind == 0) {
        const uint32_t h = (uint32_t(x) * 73856093u) ^ (uint32_t(y) * 19349669u) ^ (uint32_t(z) * 83492791u);
        return uint64_t(h) & mask;
    }
    return mix64(key) & mask;
}

__device__ __forceinline__ uint64_t ld_key(const Slot *s) {
    return __hip_atomic_load(&s->key, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
// A value word goes from PENDING to its final value once and is the only datum a reader
// takes from it, so device-scope relaxed accesses suffice: they are coherent across the
// XCDs' L2s by themselves.  (Acquire/release would add an L2 invalidate or write-back per
// access to order other memory, which nothing here needs; data published alongside a
// value, such as a pool block's key, is only read by later kernels.)
__device__ __forceinline__ int32_t ld_val(const Slot *s) {
    return __hip_atomic_load(&s->val, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_val(Slot *s, int32_t v) {
    __hip_atomic_store(&s->val, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint64_t cas_key(Slot *s, uint64_t expect, uint64_t desired) {
    return atomicCAS(&s->key, (unsigned long long)expect, (unsigned long long)desired);
}

__device__ __forceinline__ void raise_err(uint32_t *err, uint32_t bit) { atomicOr(err, bit); }

// Claim-or-locate: returns the slot holding `key` (claiming the first EMPTY slot of the
// probe sequence if the key is absent), or -1 if the table has no EMPTY slot on it.
// *claimed is true for the one thread whose CAS inserted the key.
__device__ __forceinline__ int64_t probe_claim(Slot *T, uint64_t mask, uint64_t key, uint64_t home, bool &claimed) {
    claimed = false;
    uint64_t p = home;
    for (uint64_t n = 0; n <= mask; ++n) {
        const uint64_t cur = ld_key(T + p);
        if (cur == key) return int64_t(p);
        if (cur == kEmpty) {
            const uint64_t old = cas_key(T + p, kEmpty, key);
            if (old == kEmpty) {
                claimed = true;
                return int64_t(p);
            }
            if (old == key) return int64_t(p);
        }
        p = (p + 1) & mask;
    }
    return -1;
}

// Locate without modifying (no concurrent inserts of this key may be in flight).
__device__ __forceinline__ int64_t probe_locate(const Slot *T, uint64_t mask, uint64_t key, uint64_t home) {
    uint64_t p = home;
    for (uint64_t n = 0; n <= mask; ++n) {
        const uint64_t cur = ld_key(T + p);
        if (cur == key) return int64_t(p);
        if (cur == kEmpty) return -1;
        p = (p + 1) & mask;
    }
    return -1;
}

// One map operation of a concurrent batch.  op: 0 insert, 1 find, 2 erase.
// Returns the per-op result of the C ABI (status or value); errors set sticky bits.
__device__ __forceinline__ int32_t map_op(Slot *T, uint64_t mask, int kind, int op, int32_t x, int32_t y, int32_t z,
                                          int32_t val, uint32_t *err) {
    if (!key_ok(x, y, z) || (op == 0 && val == kPending)) {
        // a key out of range, or an insert of the reserved value (it marks a slot whose
        // value is not yet published, and readers would wait on it)
        raise_err(err, kErrKeyRange);
        return op == 1 ? kAbsent : -1;
    }
    const uint64_t key = pack_key(x, y, z);
    uint64_t p = home_slot(x, y, z, key, kind, mask);
    uint32_t spins = 0;
    for (uint64_t n = 0; n <= mask;) {
        const uint64_t cur = ld_key(T + p);
        uint64_t step = 1;
        if (cur == key) {
            if (op == 0) return 0;
            if (op == 2) return cas_key(T + p, key, kTomb) == key ? 1 : 0;
            const int32_t v = ld_val(T + p);
            if (v != kPending) return v;
            if (++spins > kSpinLimit) {
                raise_err(err, kErrSpin);
                return kAbsent;
            }
            step = 0;  // value not yet published: read this slot again next iteration
        } else if (cur == kEmpty) {
            if (op != 0) return op == 1 ? kAbsent : 0;
            const uint64_t old = cas_key(T + p, kEmpty, key);
            if (old == kEmpty) {
                st_val(T + p, val);
                return 1;
            }
            if (old == key) return 0;
        }
        p = (p + step) & mask;
        n += step;
    }
    if (op == 0) {
        raise_err(err, kErrTableFull);
        return -4;
    }
    return op == 1 ? kAbsent : 0;
}

// ---------------------------------------------------------------- wave helpers
__device__ __forceinline__ int lane_id() { return int(__lane_id()); }

__device__ __forceinline__ int lanes_below(unsigned long long m) {
    return int(__builtin_amdgcn_mbcnt_hi(uint32_t(m >> 32), __builtin_amdgcn_mbcnt_lo(uint32_t(m), 0u)));
}

// Wave-aggregated append: every active lane must call it; lanes with pred get
// consecutive positions from one atomicAdd on *counter.  Returns -1 for others.
template <typename T>
__device__ __forceinline__ T wave_append(bool pred, T *counter) {
    const unsigned long long m = __ballot(pred);
    if (m == 0) return T(-1);
    const int leader = __builtin_ctzll(m);
    T base = 0;
    if (lane_id() == leader) base = atomicAdd(counter, T(__popcll(m)));
    base = __shfl(base, leader);
    return pred ? base + T(lanes_below(m)) : T(-1);
}

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

}  // namespace vbh
