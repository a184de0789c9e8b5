// Self-check of the integration kernel's division on the device: the reciprocal-based
// quotient of fastdiv.hpp against the compiler's correctly rounded division, bit for bit
// (zeros of either sign compare equal), over operands of the range it is used in.
#include <hip/hip_runtime.h>

#include "device.hpp"
#include "fastdiv.hpp"
#include "host.hpp"
#include "vbh.h"

namespace {
using namespace vbh;

__device__ __forceinline__ uint64_t splitmix(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// Operand pair i.  Divisor: exponent in [-32, 31]; significand random (all_ones = 0) or
// all ones (all_ones = 1, where one Newton step on an estimate one ulp off would fall
// short).  Dividend: exponent in [-90, 31], significand i mod 2^23 with all_ones = 1
// (every significand against each divisor), random otherwise; either sign.
__device__ __forceinline__ void operands(uint64_t seed, int64_t i, int all_ones, float &a, float &b) {
    const uint64_t z = splitmix(seed + uint64_t(i) * 0x9E3779B97F4A7C15ull);
    const uint32_t eb = uint32_t(z % 64u), ea = uint32_t((z >> 8) % 122u);
    const uint32_t mb = all_ones ? 0x7FFFFFu : uint32_t(z >> 16) & 0x7FFFFFu;
    const uint32_t ma = all_ones ? uint32_t(i) & 0x7FFFFFu : uint32_t(z >> 39) & 0x7FFFFFu;
    b = __uint_as_float(((eb + 127u - 32u) << 23) | mb);
    a = __uint_as_float((uint32_t(z >> 63) << 31) | ((ea + 127u - 90u) << 23) | ma);
}

constexpr int kBlock = 256;

__global__ void __launch_bounds__(kBlock) k_check_division(int64_t n, uint64_t seed, int all_ones,
                                                           unsigned long long *bad) {
    unsigned long long mine = 0;
    for (int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x; i < n; i += int64_t(gridDim.x) * kBlock) {
        float a, b;
        operands(seed, i, all_ones, a, b);
        const float q = corrected_quotient(a, b, refine_rcp(b, __builtin_amdgcn_rcpf(b)));
        const float want = a / b;
        mine += __float_as_uint(q) != __float_as_uint(want) && !(q == 0.0f && want == 0.0f);
    }
    mine = wave_sum(mine);
    if (lane_id() == 0 && mine) atomicAdd(bad, mine);
}

__global__ void k_zero(unsigned long long *p) { *p = 0; }

}  // namespace

extern "C" int vbh_check_division(int64_t n, uint64_t seed, int32_t all_ones, unsigned long long *d_bad,
                                  void *stream) {
    if (n < 0 || !d_bad || (all_ones != 0 && all_ones != 1)) return VBH_EINVAL;
    hipStream_t st = as_stream(stream);
    k_zero<<<1, 1, 0, st>>>(d_bad);
    if (n > 0) k_check_division<<<grid_for(n, kBlock, 1u << 16), kBlock, 0, st>>>(n, seed, all_ones, d_bad);
    VBH_LAUNCHED();
    return VBH_OK;
}
