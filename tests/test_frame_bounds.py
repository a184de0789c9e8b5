"""Host logic of the per-frame bounds (vbh::make_frame in csrc/scene.hip), which decide
three shortcuts the kernels take only when they are exact:
- fast_div: integration's reciprocal-based projection quotient (needs |pc| <= 2^32 and
  |fx|, |fy| <= 2^20 for every voxel with block coordinates in the key range);
- fast_bs: allocation's reciprocal-based quotient pw / bs (needs 2^-32 <= bs <= 2^32 and
  |pw| <= 2^32 for every band sample), and with fast_bs == 2 also bs <= 1;
- local_keys: allocation's 32-bit keys (every band sample's block B with 0 <= B - kb <
  1024 per axis, and inside the key range).
A driver linked against the library calls make_frame (host code, no GPU) for random
cameras, volumes and poses, then replays the kernels' float32 arithmetic (contraction
off) by brute force over sampled pixels (image corners included), depths (the range
ends included) and every band step, and over voxels spread across the key range, and
checks each claim the flags make.  It also reports how close the samples came to the
admitted ranges, so that a bound much looser than the arithmetic would show."""
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PKG = os.path.join(ROOT, "paper_1805_03709_amd")
LIB = os.path.join(PKG, "libvbh.so")

DRIVER = r'''
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include "scene.hpp"

static uint64_t st = 0x243F6A8885A308D3ull;
static uint64_t next() {  // SplitMix64
    uint64_t z = (st += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}
static double uni() { return double(next() >> 11) * 0x1p-53; }
static double logu(double lo, double hi) { return std::exp(std::log(lo) + uni() * (std::log(hi) - std::log(lo))); }

int main(int argc, char **argv) {
    st += uint64_t(atoll(argv[1]));
    const int n_cases = atoi(argv[2]);
    long long bad = 0, n_local = 0, n_bs = 0, n_bs2 = 0, n_div = 0, samples = 0;
    int lo_min = 1 << 30, hi_max = -1;
    double pw_frac = 0.0, pc_frac = 0.0;
    for (int cs = 0; cs < n_cases; ++cs) {
        vbh_scene s;
        vbh_params &p = s.p;
        p.width = 1 + int(next() % 640);
        p.height = 1 + int(next() % 480);
        p.fx = float(logu(20.0, 5000.0));
        p.fy = float(p.fx * (0.8 + 0.4 * uni()));
        if (next() % 16 == 0) p.fx = float(logu(0x1p20, 0x1p22));  // beyond the projection's range
        p.cx = float(uni() * p.width);
        p.cy = float(uni() * p.height);
        p.voxel_size = float(logu(1e-4, 0.2));
        if (next() % 16 == 0) p.voxel_size = float(logu(0.2, 40.0));  // blocks above 1 m
        p.trunc = p.voxel_size * float(1 + next() % 8);
        p.depth_min = float(uni() < 0.3 ? 0.0 : logu(0.05, 1.0));
        p.depth_max = float(next() % 8 == 0 ? INFINITY : p.depth_min + logu(0.1, 30.0));
        s.m_band = int(std::floor(p.trunc / p.voxel_size + 0.5f));
        // a random rotation (unit quaternion) and translation, as float32
        double q[4], nq = 0;
        for (double &x : q) { x = uni() * 2 - 1; nq += x * x; }
        nq = std::sqrt(nq);
        for (double &x : q) x /= nq;
        const double a = q[0], b = q[1], c = q[2], d = q[3];
        const double R[9] = {a*a+b*b-c*c-d*d, 2*(b*c-a*d), 2*(b*d+a*c),
                             2*(b*c+a*d), a*a-b*b+c*c-d*d, 2*(c*d-a*b),
                             2*(b*d-a*c), 2*(c*d+a*b), a*a-b*b-c*c+d*d};
        const double T = (next() % 4 == 0) ? 0.0 : logu(0.01, next() % 8 == 0 ? 1e7 : 100.0);
        float P[12];
        for (int r = 0; r < 3; ++r) {
            for (int k = 0; k < 3; ++k) P[4 * r + k] = float(R[3 * r + k]);
            P[4 * r + 3] = float((uni() * 2 - 1) * T);
        }
        const vbh::Frame f = vbh::make_frame(&s, P);
        const float vs = f.vs, bs = 8.0f * f.vs;
        n_local += f.local_keys;
        n_bs += f.fast_bs != 0;
        n_bs2 += f.fast_bs == 2;
        n_div += f.fast_div;
        if (f.fast_bs == 2 && !(bs <= 1.0f)) ++bad;
        if (f.fast_bs && !(bs >= 0x1p-32f && bs <= 0x1p32f)) ++bad;
        // allocation: band samples of sampled pixels and depths
        const float dhi = std::isfinite(f.dmax) ? f.dmax : f.dlo + 50.0f;
        for (int k = 0; k < 64; ++k) {
            int u, v;
            if (k < 4) { u = (k & 1) ? f.W - 1 : 0; v = (k & 2) ? f.H - 1 : 0; }
            else { u = int(next() % uint64_t(f.W)); v = int(next() % uint64_t(f.H)); }
            const float xn = (float(u) - f.cx) / f.fx, yn = (float(v) - f.cy) / f.fy;
            for (int j = 0; j < 4; ++j) {
                float dd = j == 0 ? f.dlo : j == 1 ? dhi : float(f.dlo + (dhi - f.dlo) * uni());
                if (!(dd >= f.dlo && dd <= f.dmax)) continue;
                for (int sm = 0; sm <= 2 * f.m_band; ++sm) {
                    const float lam = (dd - f.mu) + float(sm) * vs;
                    if (!(lam > 0.0f)) continue;
                    const float pc[3] = {lam * xn, lam * yn, lam};
                    for (int cc = 0; cc < 3; ++cc) {
                        volatile float t0 = f.P[cc * 4 + 0] * pc[0];
                        volatile float t1 = f.P[cc * 4 + 1] * pc[1];
                        volatile float t01 = t0 + t1;
                        volatile float t2 = f.P[cc * 4 + 2] * pc[2];
                        volatile float t012 = t01 + t2;
                        const float pw = t012 + f.P[cc * 4 + 3];
                        ++samples;
                        if (f.fast_bs) {
                            if (!(std::fabs(pw) <= 0x1p32f)) ++bad;
                            pw_frac = std::fmax(pw_frac, std::fabs(pw) / 0x1p32);
                        }
                        if (f.local_keys) {
                            const float qq = std::floor(pw / bs);
                            const double off = double(qq) - double(f.kb[cc]);
                            if (!(off >= 0.0 && off < 1024.0) || !(std::fabs(qq) < 1048576.0f)) {
                                if (bad < 5) printf("local key out of range: case %d axis %d off %g\n", cs, cc, off);
                                ++bad;
                            } else {
                                lo_min = std::min(lo_min, int(off));
                                hi_max = std::max(hi_max, int(off));
                            }
                        }
                    }
                }
            }
        }
        // integration: voxels anywhere in the key range
        if (f.fast_div) {
            if (!(std::fabs(f.fx) <= 0x1p20f && std::fabs(f.fy) <= 0x1p20f)) ++bad;
            for (int k = 0; k < 64; ++k) {
                int g[3];
                for (int cc = 0; cc < 3; ++cc) {
                    const int64_t bb = (k < 8) ? ((k >> cc) & 1 ? (1 << 20) - 1 : -(1 << 20))
                                               : int64_t(next() % (1u << 21)) - (1 << 20);
                    g[cc] = int(8 * bb + int64_t(next() % 8));
                }
                const float dl[3] = {float(g[0]) * vs - f.P[3], float(g[1]) * vs - f.P[7], float(g[2]) * vs - f.P[11]};
                for (int cc = 0; cc < 3; ++cc) {
                    volatile float a0 = f.P[cc] * dl[0];
                    volatile float a1 = f.P[4 + cc] * dl[1];
                    volatile float a01 = a0 + a1;
                    volatile float a2 = f.P[8 + cc] * dl[2];
                    const float pcc = a01 + a2;
                    if (!(std::fabs(pcc) <= 0x1p32f)) ++bad;
                    pc_frac = std::fmax(pc_frac, std::fabs(pcc) / 0x1p32);
                }
            }
        }
    }
    printf("cases %d samples %lld local %lld fast_bs %lld fast_bs2 %lld fast_div %lld "
           "offsets [%d, %d] max|pw|/2^32 %.3g max|pc|/2^32 %.3g bad %lld\n",
           n_cases, samples, n_local, n_bs, n_bs2, n_div, lo_min, hi_max, pw_frac, pc_frac, bad);
    return bad ? 1 : 0;
}
'''


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    if not os.path.exists(LIB):
        pytest.skip("libvbh.so not built")
    d = tmp_path_factory.mktemp("bounds")
    src, exe = d / "drv.hip", d / "drv"
    src.write_text(DRIVER)
    subprocess.run(["hipcc", "-std=c++17", "-O1", "-ffp-contract=off", "-fno-fast-math", "--offload-arch=gfx950",
                    "-I", os.path.join(ROOT, "include"), "-I", os.path.join(PKG, "csrc"), "-o", str(exe), str(src),
                    "-L", PKG, "-l:libvbh.so", f"-Wl,-rpath,{PKG}"], check=True)
    return str(exe)


@pytest.mark.parametrize("seed", range(3))
def test_frame_flags_hold_for_every_sample(driver, seed):
    out = subprocess.run([driver, str(seed), "3000"], capture_output=True, text=True, timeout=300)
    assert out.returncode == 0, out.stdout + out.stderr
    fields = out.stdout.split()
    stat = {fields[i]: fields[i + 1] for i in range(0, len(fields) - 1)}
    # every shortcut is exercised, local keys come close to both ends of their range
    assert int(stat["local"]) > 100 and int(stat["fast_bs2"]) > 100 and int(stat["fast_div"]) > 100
    lo, hi = (int(x) for x in out.stdout.split("offsets [")[1].split("]")[0].split(","))
    assert lo < 160 and hi > 860, out.stdout  # about a tenth of the range is the bound's slack
