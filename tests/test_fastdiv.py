"""Host check of the integration kernel's float32 division (csrc/fastdiv.hpp): the header
is compiled with the host compiler and driven over random operands spread across the
admitted range (divisors in [2^-32, 2^32], dividends in [2^-90, 2^32] in magnitude, both
signs, every exponent), over operands at the range ends and at binade edges, and over tiny
and denormal dividends.
- From the correctly rounded reciprocal, the quotient equals IEEE float32 division bit for
  bit (a zero may differ in sign).
- From an estimate one ulp off, it still does, except for divisors whose significand is all
  ones: there one Newton step can stop half an ulp short of 1/b and the last correction
  can round a quotient that lies just past a midpoint the wrong way (Markstein's known
  exception).  This is what the check expects; the hardware reciprocal is checked against
  the compiler's division on the GPU (test_gpu_fastdiv).
- For dividends below 2^-90 the quotient stays below 2^-56 in magnitude; with a divisor at
  most 1 (so the reciprocal is at least 1 and a nonzero dividend's product cannot vanish)
  its floor equals the floor of the true quotient (0 or -1 by the dividend's sign), which
  is all allocation takes from it."""
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
DRIVER = r'''
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include "fastdiv.hpp"

static float bits(uint32_t u) { float f; std::memcpy(&f, &u, 4); return f; }
static uint32_t ubits(float f) { uint32_t u; std::memcpy(&u, &f, 4); return u; }
static uint64_t s = 0x9E3779B97F4A7C15ull;
static uint64_t next() {  // SplitMix64
    uint64_t z = (s += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}
// a float with a uniformly drawn exponent in [lo, hi] and a random significand
static float draw(int lo, int hi) {
    const uint64_t r = next();
    const int e = lo + int(r % uint64_t(hi - lo + 1));
    const uint32_t m = uint32_t(r >> 32) & 0x7FFFFFu;
    float f = std::ldexp(1.0f + float(m) / 8388608.0f, e);
    return (r >> 63) ? -f : f;
}
static long long checked = 0, bad = 0, bad_tiny = 0, allones_off = 0, bad_floor = 0;
static void check_floor(float a, float b) {  // |a| < 2^-90, 2^-32 <= b <= 1
    const float rb = 1.0f / b;
    for (int k = -1; k <= 1; ++k) {
        const float y = vbh::refine_rcp(b, bits(ubits(rb) + uint32_t(k)));
        const float q = vbh::corrected_quotient(a, b, y);
        ++checked;
        if (!(std::floor(q) == std::floor(a / b))) {
            if (bad_floor < 5) printf("floor mismatch a=%a b=%a q=%a want=%a\n", a, b, q, a / b);
            ++bad_floor;
        }
    }
}
static void check(float a, float b) {
    const float rb = 1.0f / b;
    const bool allones = (ubits(b) & 0x7FFFFFu) == 0x7FFFFFu;
    for (int k = -1; k <= 1; ++k) {
        const float y0 = bits(ubits(rb) + uint32_t(k));
        const float y = vbh::refine_rcp(b, y0);
        const float q = vbh::corrected_quotient(a, b, y);
        ++checked;
        if (a != 0.0f && std::fabs(a) < 0x1p-90f) {
            if (!(std::fabs(q) < 0x1p-56f)) ++bad_tiny;
        } else if (ubits(q) != ubits(a / b) && !(q == 0.0f && a / b == 0.0f)) {
            if (k != 0 && allones) {
                ++allones_off;
                continue;
            }
            if (bad < 5) printf("mismatch a=%a b=%a y0=%a q=%a want=%a\n", a, b, y0, q, a / b);
            ++bad;
        }
    }
}
int main(int argc, char **argv) {
    const long long n = atoll(argv[1]);
    for (long long i = 0; i < n; ++i) {
        float b = std::fabs(draw(-32, 31));
        float a = draw(-90, 31);
        check(a, b);
        check(std::ldexp(b, int(next() % 8)) * (1.0f + 0x1p-23f * float(next() % 4)), b);  // near-integer quotients
    }
    // range ends and binade edges: significands 1, 1 + ulp, 2 - ulp
    const float sig[3] = {1.0f, 1.0f + 0x1p-23f, 2.0f - 0x1p-23f};
    for (int eb = -32; eb <= 31; ++eb)
        for (int ea = -90; ea <= 31; ++ea)
            for (int i = 0; i < 3; ++i)
                for (int j = 0; j < 3; ++j) {
                    const float b = std::ldexp(sig[i], eb), a = std::ldexp(sig[j], ea);
                    if (b > 0x1p32f || a > 0x1p32f) continue;
                    check(a, b);
                    check(-a, b);
                }
    check(0.0f, 1.0f);
    check(-0.0f, 0x1p-32f);
    check(0x1p32f, 0x1p-32f);
    for (int i = 0; i < 100000; ++i) check(draw(-149, -91), std::fabs(draw(-32, 31)));  // tiny dividends
    for (int i = 1; i < 100000; ++i) check(bits(uint32_t(i)), std::fabs(draw(-32, 31)));  // denormal dividends
    for (int i = 0; i < 200000; ++i) {  // floors of tiny and denormal dividends, divisors <= 1
        const float b = (i % 97 == 0) ? 1.0f : std::fabs(draw(-32, -1));
        const float a = (i & 1) ? draw(-149, -91) : bits(uint32_t(1 + next() % 0x7FFFFFu)) * ((next() & 1) ? -1.0f : 1.0f);
        check_floor(a, b);
    }
    check_floor(0.0f, 0x1p-32f);
    check_floor(-0.0f, 1.0f);
    check_floor(-bits(1u), 1.0f);
    check_floor(bits(1u), 0x1p-32f);
    printf("checked %lld bad %lld bad_tiny %lld allones_off %lld bad_floor %lld\n", checked, bad, bad_tiny,
           allones_off, bad_floor);
    return bad || bad_tiny || bad_floor ? 1 : 0;
}
'''


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    d = tmp_path_factory.mktemp("fastdiv")
    src, exe = d / "drv.cpp", d / "drv"
    src.write_text(DRIVER)
    subprocess.run(["g++", "-std=c++17", "-O2", "-mfma", "-ffp-contract=off", "-fno-fast-math",
                    "-I", os.path.join(ROOT, "paper_1805_03709_amd", "csrc"), "-o", str(exe), str(src)],
                   check=True)
    return str(exe)


def test_corrected_quotient_is_correctly_rounded(driver):
    out = subprocess.run([driver, "2000000"], capture_output=True, text=True, timeout=300)
    assert out.returncode == 0, out.stdout + out.stderr
    assert "bad 0 bad_tiny 0" in out.stdout and "bad_floor 0" in out.stdout
