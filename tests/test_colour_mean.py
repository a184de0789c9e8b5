"""The integration kernel's exact colour mean, checked exhaustively on the host.

Each channel becomes floor((W c + c_obs + floor(n/2)) / n), with n = W + 1 observations
(256 once W saturates at 255).  The kernel takes it as the truncation of one float
multiply-add, fma(W c + c_obs, 1/n, (floor(n/2) + 1/2) / n), with 1/n from the hardware
reciprocal (within one ulp).  The driver below restates that arithmetic (the same
float operations and rounding, contraction off) and compares it with the integer
definition for every stored weight W in 0..255, stored colour c and observed colour
c_obs in 0..255, and reciprocals 0, 1 and 2 ulps either side of the correctly rounded
1/n: 16.7M triples times 5 reciprocals.  Dropping the half (a plausible mistake, which
takes away the 1/(2n) margin to the nearest integer) fails."""
import subprocess

import pytest

DRIVER = r'''
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>

static float bits(uint32_t u) { float f; std::memcpy(&f, &u, 4); return f; }
static uint32_t ubits(float f) { uint32_t u; std::memcpy(&u, &f, 4); return u; }

int main(int argc, char **argv) {
    const bool drop_half = argc > 1;
    long long bad = 0, checked = 0;
    for (uint32_t w = 0; w <= 255; ++w) {
        const uint32_t n = w + 1u;  // W = 255 means 256 observations after this one
        const float wf = float(w);
        const float exact_inv = 1.0f / (wf + 1.0f);
        for (int k = -2; k <= 2; ++k) {
            const float inv = bits(ubits(exact_inv) + uint32_t(k));
            const float hinv = drop_half ? float(n >> 1) * inv : (float(n >> 1) + 0.5f) * inv;
            for (uint32_t c = 0; c <= 255; ++c)
                for (uint32_t o = 0; o <= 255; ++o) {
                    const float num = std::fma(wf, float(c), float(o));  // exact: below 2^17
                    const uint32_t got = uint32_t(std::fma(num, inv, hinv));
                    const uint32_t want = (w * c + o + (n >> 1)) / n;
                    ++checked;
                    if (got != want) {
                        if (bad < 3 && !drop_half) printf("W=%u c=%u obs=%u k=%d got %u want %u\n", w, c, o, k, got, want);
                        ++bad;
                    }
                }
        }
    }
    printf("checked %lld bad %lld\n", checked, bad);
    return bad ? 1 : 0;
}
'''


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    d = tmp_path_factory.mktemp("colour")
    src, exe = d / "drv.cpp", d / "drv"
    src.write_text(DRIVER)
    subprocess.run(["g++", "-std=c++17", "-O2", "-mfma", "-ffp-contract=off", "-fno-fast-math", "-o", str(exe),
                    str(src)], check=True)
    return str(exe)


def test_colour_mean_is_exact_for_every_input(driver):
    out = subprocess.run([driver], capture_output=True, text=True, timeout=300)
    assert out.returncode == 0, out.stdout
    assert "bad 0" in out.stdout


def test_dropping_the_half_fails(driver):
    out = subprocess.run([driver, "drop"], capture_output=True, text=True, timeout=300)
    assert out.returncode == 1 and "bad 0" not in out.stdout
