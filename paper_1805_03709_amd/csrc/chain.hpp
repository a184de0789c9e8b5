// Chained concurrent hash map of Sec. 5 (bucket array + linked-list excess entries +
// free-entry stack + per-entry occupancy flags and locks) - host interface used by the
// C ABI in map.hip.  The device protocol is described in chain.hip.
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace vbh {

// One entry: the key word and the link word, read and written as separate 64-bit atomics.
struct alignas(16) ChainEntry {
    unsigned long long a;  // packed key (bits 0..62) | lifetime bit (63)
    unsigned long long b;  // value (0..31) | next entry (32..59) | dead (60) | lifetime (61) | occupied (62) | lock (63)
};
static_assert(sizeof(ChainEntry) == 16, "entry layout");

// Device-resident bookkeeping of the free-entry stack and the batch's retired entries.
struct ChainCtl {
    unsigned long long top;        // free excess entries on the stack when the batch started
    unsigned long long used;       // stack pops attempted by the running batch
    unsigned long long retired_x;  // list entries emptied by the running batch (log from the front)
    unsigned long long retired_b;  // buckets emptied by the running batch (log from the back)
};

static_assert(offsetof(ChainCtl, retired_x) == offsetof(ChainCtl, used) + 8 &&
                  offsetof(ChainCtl, retired_b) == offsetof(ChainCtl, used) + 16,
              "the batch kernel claims the three counters as consecutive words");

struct ChainMap {
    ChainEntry *E = nullptr;  // [nb buckets][nx excess entries]
    uint32_t *stack = nullptr;  // free excess entries, [nx]
    uint32_t *retire = nullptr; // entries emptied by the running batch, [nb + nx]: list entries
                                // from the front, buckets from the back
    ChainCtl *ctl = nullptr;
    uint64_t nb = 0, nx = 0;
};

constexpr uint64_t kChainMaxEntries = (1ull << 28) - 1;  // the link field holds 28 bits

int chain_create(uint64_t buckets, uint64_t excess, ChainMap **out);
void chain_destroy(ChainMap *c);
int chain_clear(ChainMap *c, hipStream_t st);
// opc 0 insert, 1 find, 2 erase, -1 mixed (kind per op from ops[]).
int chain_batch(ChainMap *c, int hash_kind, int opc, const uint8_t *ops, const int32_t *keys, const int32_t *vals,
                int64_t n, int32_t *out, uint32_t *err, hipStream_t st);
// cnt[0] += occupied entries.
int chain_count(const ChainMap *c, unsigned long long *cnt, hipStream_t st);
// Compacts occupied entries into keys/vals (cap entries at most); cnt[0] = occupied count.
int chain_export(const ChainMap *c, int32_t *keys, int32_t *vals, int64_t cap, unsigned long long *cnt,
                 hipStream_t st);

}  // namespace vbh
