// Host-side helpers of the C ABI: HIP error mapping, launch geometry, sticky errors.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "vbh.h"

namespace vbh {

#define VBH_HIP(expr)                                   \
    do {                                                \
        if ((expr) != hipSuccess) return VBH_EHIP;      \
    } while (0)

#define VBH_LAUNCHED()                                  \
    do {                                                \
        if (hipGetLastError() != hipSuccess) return VBH_EHIP; \
    } while (0)

inline hipStream_t as_stream(void *s) { return static_cast<hipStream_t>(s); }

// First word of every handle struct: its kind, read by vbh_status.
constexpr uint32_t kTagMap = 0x4d415048u, kTagScene = 0x53434e45u;

inline bool is_pow2(uint64_t v) { return v && !(v & (v - 1)); }

inline unsigned grid_for(int64_t n, int per_block, unsigned cap = 1u << 30) {
    int64_t g = (n + per_block - 1) / per_block;
    if (g < 1) g = 1;
    return unsigned(g > cap ? cap : g);
}

// Maps sticky device error bits to the most specific code (first by severity order).
inline int code_from_bits(uint32_t bits) {
    if (!bits) return VBH_OK;
    if (bits & 2u) return VBH_EFULL_TABLE;
    if (bits & 4u) return VBH_EFULL_POOL;
    if (bits & 8u) return VBH_EFULL_LOG;
    if (bits & 16u) return VBH_ESPIN;
    return VBH_EINVAL;
}

// Number of compute units of the current device (for persistent-style grids).
int device_cus();

}  // namespace vbh
