// Differentiable form of the fusion path: several depth frames are integrated into a
// fresh block-hashed volume (the band allocation kernel of scene.hip, then the voxel
// means in float64 below),
// the loss is L = sum_k F_tri(x_k)^2 over back-projected pixel samples, and the backward
// pass gives dL/d(depth) per pixel and dL/d(xi) per frame, where each camera-to-world
// pose is T_f = Exp(xi_f) T0_f with xi = (rho; phi) and T0_f the caller's base pose.  The
// library composes T_f (float64, then rounded to the float32 pose the fusion kernels use),
// accumulates the left-perturbation gradient g_f = dL/d(delta) of Exp(delta) T_f at
// delta = 0, and returns dL/dxi_f = J_l(xi_f)^T g_f with J_l the SE(3) left Jacobian.
//
// Gradient (discrete decisions fixed at the forward point):
//   samples:  dL/dF_c += 2 F_tri w_c;  g_x = 2 F_tri grad F_tri;
//             dL/dD_f[p] += g_x . (R_f r_c),  dL/drho_f += g_x,  dL/dphi_f += x x g_x
//   voxels:   F_v = mean over observing frames of min(D_f[pix] - z_f, trunc), so for an
//             unclamped observation with c = dL/dF_v / W_v:
//             dL/dD_f[pix] += c,  dL/drho_f += c r3_f,  dL/dphi_f += c (X_v x r3_f)
//             (r3_f: the camera z axis in world coordinates, X_v = g vs).
// The backward recomputes every projection; no per-voxel Jacobian is stored.  The hash
// table and the allocation are not differentiated.
//
// Precision: the float32 volume of the fusion path carries ~1e-7..1e-6 m of rounding in
// F (float32 running means, float32 camera z at metres of range), and the gradients are
// sums of large terms that cancel (moving a depth moves both a sample and the fused
// surface), which would magnify that to ~1e-3 relative.  This path therefore keeps the
// fusion kernels' float32 decisions (allocation, W, pixels, skips, clamps, cells) but
// evaluates its values in float64: F64_v = (1/W_v) sum of float64 TSDFs, float64
// sample points, float64 dL/dF, float64 accumulation (native FP64 atomics).  W_v, the
// count of observations that pass those decisions, is what the float32 integration
// would store (no saturation below 255 frames).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <new>

#include "scene.hpp"

using namespace vbh;

namespace {

constexpr int kMaxFrames = 32;
constexpr int kSampleWG = 256;
constexpr int kMaxWG = 8192;

struct DiffDev {
    Dev S;
    uint32_t *fmask;  // [P] frames whose band touched the block
    double *F64;      // [P][512] float64 mean of the observed TSDFs
    double *dLdF;     // [P][512]
    uint32_t *hot;    // [P] block has a nonzero dL/dF
    double *loss_part;  // [kMaxWG]
    double *xi_part;    // [2 kMaxWG][F][6] per-workgroup pose-gradient partials
    double *gd64;       // [F][H][W] depth gradient accumulator
    int F;
};

struct Cams {
    float P[kMaxFrames][12];
};

// ---------------------------------------------------------------- helpers
__global__ void __launch_bounds__(kBlock) k_zero_u32(uint32_t *p, int64_t n) {
    for (int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x; i < n; i += int64_t(gridDim.x) * kBlock) p[i] = 0u;
}
__global__ void __launch_bounds__(kBlock) k_zero_f64(double *p, int64_t n) {
    for (int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x; i < n; i += int64_t(gridDim.x) * kBlock) p[i] = 0.0;
}
__global__ void __launch_bounds__(kBlock) k_to_f32(const double *src, float *dst, int64_t n) {
    for (int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x; i < n; i += int64_t(gridDim.x) * kBlock)
        dst[i] = float(src[i]);
}

// Zeroes dL/dF and the hot flags of every handed-out block.
__global__ void __launch_bounds__(kBlock) k_zero_grad_blocks(DiffDev D) {
    const unsigned long long pn = D.S.C->pool_next;
    const int64_t n = int64_t(pn) < D.S.pool_cap ? int64_t(pn) : D.S.pool_cap;
    for (int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x; i < n * 512; i += int64_t(gridDim.x) * kBlock) {
        D.dLdF[i] = 0.0;
        if ((i & 511) == 0) D.hot[i >> 9] = 0u;
    }
}

// Marks frame f in the frame mask of every block of update `seq`'s touched list.
__global__ void __launch_bounds__(kBlock) k_touch_mask(DiffDev D, int f, int seq) {
    const int64_t n = D.S.C->fc[seq & (kRing - 1)].n_touched;
    for (int64_t t = int64_t(blockIdx.x) * kBlock + threadIdx.x; t < n; t += int64_t(gridDim.x) * kBlock) {
        const int32_t pool = D.S.T[touched_of(D.S, seq)[t]].val;
        if (pool >= 0) D.fmask[pool] |= 1u << f;  // each block appears once per update
    }
}

__device__ __forceinline__ int32_t find_pool(const Dev &S, int32_t x, int32_t y, int32_t z) {
    if (!key_ok(x, y, z)) return -1;
    const uint64_t k = pack_key(x, y, z);
    const int64_t ps = probe_locate(S.T, S.mask, k, home_slot(x, y, z, k, S.kind, S.mask));
    return ps >= 0 ? S.T[ps].val : -1;
}

// Sample k: its trilinear cell from the float32 point (canonical operation order), the
// float64 point and cell fraction, and the 8 corner voxels (pool*512 + l, or -1 if the
// corner's block is missing or the voxel unobserved) with their float64 F.
struct SamplePt {
    double x[3];
    double fr[3];
    int64_t vox[8];
    double Fc[8];
    bool keep;
};

__device__ __forceinline__ SamplePt sample_point(const DiffDev &D, const Frame &fr, const float *P, float d, int u,
                                                 int v) {
    SamplePt s;
    const float xn = (float(u) - fr.cx) / fr.fx;
    const float yn = (float(v) - fr.cy) / fr.fy;
    const float pc[3] = {d * xn, d * yn, d};
    const double pc64[3] = {double(d) * ((double(u) - fr.cx) / fr.fx), double(d) * ((double(v) - fr.cy) / fr.fy),
                            double(d)};
    int32_t base[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        const float x32 = ((P[i * 4 + 0] * pc[0] + P[i * 4 + 1] * pc[1]) + P[i * 4 + 2] * pc[2]) + P[i * 4 + 3];
        base[i] = int32_t(floorf(x32 / fr.vs));
        s.x[i] = double(P[i * 4 + 0]) * pc64[0] + double(P[i * 4 + 1]) * pc64[1] + double(P[i * 4 + 2]) * pc64[2] +
                 double(P[i * 4 + 3]);
        s.fr[i] = s.x[i] / double(fr.vs) - double(base[i]);
    }
    // corners: c bit 0 -> +x, bit 1 -> +y, bit 2 -> +z; blocks looked up once each
    int32_t bk[8][3];
    int32_t bp[8];
    int nb = 0;
    s.keep = true;
#pragma unroll
    for (int c = 0; c < 8; ++c) {
        const int32_t g[3] = {base[0] + (c & 1), base[1] + ((c >> 1) & 1), base[2] + ((c >> 2) & 1)};
        const int32_t B[3] = {g[0] >> 3, g[1] >> 3, g[2] >> 3};  // arithmetic shift = floor
        int32_t pool = -2;
        for (int i = 0; i < nb; ++i)
            if (bk[i][0] == B[0] && bk[i][1] == B[1] && bk[i][2] == B[2]) pool = bp[i];
        if (pool == -2) {
            pool = find_pool(D.S, B[0], B[1], B[2]);
            bk[nb][0] = B[0];
            bk[nb][1] = B[1];
            bk[nb][2] = B[2];
            bp[nb] = pool;
            ++nb;
        }
        s.vox[c] = -1;
        s.Fc[c] = 0.0;
        if (pool >= 0) {
            const int64_t vx = int64_t(pool) * 512 + (g[0] & 7) + 8 * (g[1] & 7) + 64 * (g[2] & 7);
            if (D.S.WRGB[vx] & 0xFFu) {
                s.vox[c] = vx;
                s.Fc[c] = D.F64[vx];
            }
        }
        if (s.vox[c] < 0) s.keep = false;
    }
    return s;
}

__device__ __forceinline__ void tri_weights(const double *fr, double *w, double (*dw)[3]) {
#pragma unroll
    for (int c = 0; c < 8; ++c) {
        double a[3], da[3];
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            const bool hi = (c >> i) & 1;
            a[i] = hi ? fr[i] : 1.0 - fr[i];
            da[i] = hi ? 1.0 : -1.0;
        }
        w[c] = a[0] * a[1] * a[2];
        if (dw) {
            dw[c][0] = da[0] * a[1] * a[2];
            dw[c][1] = a[0] * da[1] * a[2];
            dw[c][2] = a[0] * a[1] * da[2];
        }
    }
}

// One wave per allocated block: the float64 mean of the observed TSDFs of every voxel and
// its weight W (the number of observations), revisiting each frame whose band touched the
// block with the fusion kernels' float32 decisions (pixel, validity, -trunc skip, +trunc
// clamp).  This is the volume the loss samples; the float32 integration kernel is not run.
__global__ void __launch_bounds__(kBlock) k_mean64(DiffDev D, Frame fr, Cams cams, const float *depth) {
    const Dev &S = D.S;
    const unsigned long long pn = S.C->pool_next;
    const int64_t n = int64_t(pn) < S.pool_cap ? int64_t(pn) : S.pool_cap;
    const int lane = lane_id();
    const int lx = lane & 7, ly = lane >> 3;
    const int64_t gw = int64_t(blockIdx.x) * kWaves + (threadIdx.x >> 6);
    const int64_t nw = int64_t(gridDim.x) * kWaves;
    const int64_t HW = int64_t(fr.W) * fr.H;
    for (int64_t pool = gw; pool < n; pool += nw) {
        int32_t bx, by, bz;
        unpack_key(S.pool_key[pool], bx, by, bz);
        const uint32_t fm = D.fmask[pool];
        const double X = double(8 * bx + lx) * double(fr.vs), Y = double(8 * by + ly) * double(fr.vs);
        double sum[8] = {0, 0, 0, 0, 0, 0, 0, 0};
        int cnt[8] = {0, 0, 0, 0, 0, 0, 0, 0};
        for (int f = 0; f < D.F; ++f) {
            if (!((fm >> f) & 1u)) continue;  // uniform per wave
            const float *P = cams.P[f];
            const float dlx = float(8 * bx + lx) * fr.vs - P[3];
            const float dly = float(8 * by + ly) * fr.vs - P[7];
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                const float dlz = float(8 * bz + j) * fr.vs - P[11];
                const float pcx = (P[0] * dlx + P[4] * dly) + P[8] * dlz;
                const float pcy = (P[1] * dlx + P[5] * dly) + P[9] * dlz;
                const float pcz = (P[2] * dlx + P[6] * dly) + P[10] * dlz;
                if (!(pcz > 0.0f)) continue;
                const float fu = floorf((fr.fx * (pcx / pcz) + fr.cx) + 0.5f);
                const float fv = floorf((fr.fy * (pcy / pcz) + fr.cy) + 0.5f);
                if (!(fu >= 0.0f && fu < float(fr.W) && fv >= 0.0f && fv < float(fr.H))) continue;
                const int64_t pix = int64_t(fv) * fr.W + int64_t(fu);
                const float dd = depth[f * HW + pix];
                if (!depth_valid(dd, fr)) continue;
                const float sdf = dd - pcz;
                if (sdf < -fr.mu) continue;
                double t = double(fr.mu);
                if (sdf < fr.mu) {
                    const double Z = double(8 * bz + j) * double(fr.vs);
                    const double z = double(P[2]) * (X - double(P[3])) + double(P[6]) * (Y - double(P[7])) +
                                     double(P[10]) * (Z - double(P[11]));
                    t = double(dd) - z;
                }
                sum[j] += t;
                ++cnt[j];
            }
        }
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            D.F64[pool * 512 + lane + 64 * j] = cnt[j] ? sum[j] / double(cnt[j]) : 0.0;
            S.WRGB[pool * 512 + lane + 64 * j] = uint32_t(cnt[j]);  // W (at most kMaxFrames observations)
        }
    }
}

// ---------------------------------------------------------------- forward
__global__ void __launch_bounds__(kSampleWG) k_sample_fwd(DiffDev D, Frame fr, Cams cams, const float *depth,
                                                          const int32_t *sf, const int32_t *sp, int64_t K,
                                                          float *f_out) {
    __shared__ double part[kSampleWG / 64];
    const int64_t k = int64_t(blockIdx.x) * kSampleWG + threadIdx.x;
    double l2 = 0.0;
    if (k < K) {
        const int f = sf[k];
        const int32_t pix = sp[k];
        const bool in_range = f >= 0 && f < D.F && pix >= 0 && pix < fr.W * fr.H;
        const float d = in_range ? depth[int64_t(f) * fr.W * fr.H + pix] : 0.0f;
        float val = __builtin_nanf("");
        if (in_range && depth_valid(d, fr)) {
            const SamplePt s = sample_point(D, fr, cams.P[f], d, pix % fr.W, pix / fr.W);
            if (s.keep) {
                double w[8];
                tri_weights(s.fr, w, nullptr);
                double Ft = 0.0;
#pragma unroll
                for (int c = 0; c < 8; ++c) Ft += w[c] * s.Fc[c];
                val = float(Ft);
                l2 = Ft * Ft;
            }
        }
        if (f_out) f_out[k] = val;
    }
    l2 = wave_sum(l2);
    if (lane_id() == 0) part[threadIdx.x >> 6] = l2;
    __syncthreads();
    if (threadIdx.x == 0) {
        double s = 0.0;
        for (int w = 0; w < kSampleWG / 64; ++w) s += part[w];
        D.loss_part[blockIdx.x] = s;
    }
}

__global__ void k_reduce_loss(DiffDev D, int n_part, float *loss) {
    __shared__ double part[4];
    double s = 0.0;
    for (int i = threadIdx.x; i < n_part; i += 256) s += D.loss_part[i];
    s = wave_sum(s);
    if (lane_id() == 0) part[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) *loss = float(part[0] + part[1] + part[2] + part[3]);
}

// ---------------------------------------------------------------- backward
// The gradients are sums of large terms that cancel (moving a depth moves both the sample
// and the fused surface), so the backward evaluates its terms and accumulates in float64
// (native FP64 atomics) and converts to float32 only at the end.
// Per-workgroup pose-gradient accumulator in LDS, written out as a partial.
__device__ __forceinline__ void xi_flush(const DiffDev &D, double (*acc)[6]) {
    __syncthreads();
    for (int i = threadIdx.x; i < D.F * 6; i += blockDim.x)
        D.xi_part[int64_t(blockIdx.x) * D.F * 6 + i] = acc[i / 6][i % 6];
}

__global__ void __launch_bounds__(kSampleWG) k_sample_bwd(DiffDev D, Frame fr, Cams cams, const float *depth,
                                                          const int32_t *sf, const int32_t *sp, int64_t K,
                                                          const float *grad_loss) {
    __shared__ double acc[kMaxFrames][6];
    for (int i = threadIdx.x; i < kMaxFrames * 6; i += kSampleWG) acc[i / 6][i % 6] = 0.0;
    __syncthreads();
    const int64_t k = int64_t(blockIdx.x) * kSampleWG + threadIdx.x;
    if (k < K) {
        const int f = sf[k];
        const int32_t pix = sp[k];
        const bool in_range = f >= 0 && f < D.F && pix >= 0 && pix < fr.W * fr.H;
        const float d = in_range ? depth[int64_t(f) * fr.W * fr.H + pix] : 0.0f;
        if (in_range && depth_valid(d, fr)) {
            const float *P = cams.P[f];
            const SamplePt s = sample_point(D, fr, P, d, pix % fr.W, pix / fr.W);
            if (s.keep) {
                double w[8], dw[8][3];
                tri_weights(s.fr, w, dw);
                double Ft = 0.0, gF[3] = {0.0, 0.0, 0.0};
#pragma unroll
                for (int c = 0; c < 8; ++c) {
                    Ft += w[c] * s.Fc[c];
#pragma unroll
                    for (int i = 0; i < 3; ++i) gF[i] += dw[c][i] * s.Fc[c];
                }
                const double g = 2.0 * Ft * double(*grad_loss);
#pragma unroll
                for (int c = 0; c < 8; ++c) {
                    atomicAdd(&D.dLdF[s.vox[c]], g * w[c]);
                    D.hot[s.vox[c] >> 9] = 1u;
                }
                const double ivs = 1.0 / double(fr.vs);
                const double gx[3] = {g * gF[0] * ivs, g * gF[1] * ivs, g * gF[2] * ivs};
                // dx/dD = R r_c with r_c = ((u-cx)/fx, (v-cy)/fy, 1)
                const double rc[3] = {(double(pix % fr.W) - fr.cx) / fr.fx, (double(pix / fr.W) - fr.cy) / fr.fy, 1.0};
                double gd = 0.0;
#pragma unroll
                for (int i = 0; i < 3; ++i)
                    gd += gx[i] * (double(P[i * 4 + 0]) * rc[0] + double(P[i * 4 + 1]) * rc[1] + double(P[i * 4 + 2]) * rc[2]);
                atomicAdd(&D.gd64[int64_t(f) * fr.W * fr.H + pix], gd);
                const double *x = s.x;
                atomicAdd(&acc[f][0], gx[0]);
                atomicAdd(&acc[f][1], gx[1]);
                atomicAdd(&acc[f][2], gx[2]);
                atomicAdd(&acc[f][3], x[1] * gx[2] - x[2] * gx[1]);
                atomicAdd(&acc[f][4], x[2] * gx[0] - x[0] * gx[2]);
                atomicAdd(&acc[f][5], x[0] * gx[1] - x[1] * gx[0]);
            }
        }
    }
    xi_flush(D, acc);
}

// One wave per block with a nonzero dL/dF; lane = lx + 8 ly handles voxels (lx, ly, 0..7)
// and revisits every frame that integrated the block with the forward's float32 decisions.
__global__ void __launch_bounds__(kBlock) k_integrate_bwd(DiffDev D, Frame fr, Cams cams, const float *depth) {
    __shared__ double acc[kMaxFrames][6];
    for (int i = threadIdx.x; i < kMaxFrames * 6; i += kBlock) acc[i / 6][i % 6] = 0.0;
    __syncthreads();
    const Dev &S = D.S;
    const unsigned long long pn = S.C->pool_next;
    const int64_t n = int64_t(pn) < S.pool_cap ? int64_t(pn) : S.pool_cap;
    const int lane = lane_id();
    const int lx = lane & 7, ly = lane >> 3;
    const int64_t gw = int64_t(blockIdx.x) * kWaves + (threadIdx.x >> 6);
    const int64_t nw = int64_t(gridDim.x) * kWaves;
    const int64_t HW = int64_t(fr.W) * fr.H;
    for (int64_t pool = gw; pool < n; pool += nw) {
        if (!D.hot[pool]) continue;  // uniform per wave
        int32_t bx, by, bz;
        unpack_key(S.pool_key[pool], bx, by, bz);
        double c[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const int64_t idx = pool * 512 + lane + 64 * j;
            const double g = D.dLdF[idx];
            const uint32_t W = S.WRGB[idx] & 0xFFu;
            c[j] = (g != 0.0 && W) ? g / double(W) : 0.0;
        }
        const uint32_t fm = D.fmask[pool];
        const double X = double(8 * bx + lx) * double(fr.vs), Y = double(8 * by + ly) * double(fr.vs);
        for (int f = 0; f < D.F; ++f) {
            if (!((fm >> f) & 1u)) continue;  // uniform per wave
            const float *P = cams.P[f];
            // decisions exactly as in the forward (float32, same operation order)
            const float dlx = float(8 * bx + lx) * fr.vs - P[3];
            const float dly = float(8 * by + ly) * fr.vs - P[7];
            double a[6] = {0, 0, 0, 0, 0, 0};
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                if (c[j] == 0.0) continue;
                const double Z = double(8 * bz + j) * double(fr.vs);
                const float dlz = float(8 * bz + j) * fr.vs - P[11];
                const float pcx = (P[0] * dlx + P[4] * dly) + P[8] * dlz;
                const float pcy = (P[1] * dlx + P[5] * dly) + P[9] * dlz;
                const float pcz = (P[2] * dlx + P[6] * dly) + P[10] * dlz;
                if (!(pcz > 0.0f)) continue;
                const float fu = floorf((fr.fx * (pcx / pcz) + fr.cx) + 0.5f);
                const float fv = floorf((fr.fy * (pcy / pcz) + fr.cy) + 0.5f);
                if (!(fu >= 0.0f && fu < float(fr.W) && fv >= 0.0f && fv < float(fr.H))) continue;
                const int64_t pix = int64_t(fv) * fr.W + int64_t(fu);
                const float dd = depth[f * HW + pix];
                if (!depth_valid(dd, fr)) continue;
                const float sdf = dd - pcz;
                if (sdf < -fr.mu || !(sdf < fr.mu)) continue;  // skipped, or clamped at +trunc
                atomicAdd(&D.gd64[f * HW + pix], c[j]);
                const double r3[3] = {P[2], P[6], P[10]};
                a[0] += c[j] * r3[0];
                a[1] += c[j] * r3[1];
                a[2] += c[j] * r3[2];
                a[3] += c[j] * (Y * r3[2] - Z * r3[1]);
                a[4] += c[j] * (Z * r3[0] - X * r3[2]);
                a[5] += c[j] * (X * r3[1] - Y * r3[0]);
            }
#pragma unroll
            for (int i = 0; i < 6; ++i) {
                const double s = wave_sum(a[i]);
                if (lane == 0 && s != 0.0) atomicAdd(&acc[f][i], s);
            }
        }
    }
    xi_flush(D, acc);
}

// One workgroup per pose-gradient component i: a fixed-order sum of its per-workgroup
// partials (rows), strided over the threads, then across the workgroup.
__global__ void __launch_bounds__(kBlock) k_reduce_xi(DiffDev D, int n_part_a, int n_part_b, double *g_left) {
    // partials of k_sample_bwd occupy rows [0, n_part_a), those of k_integrate_bwd
    // rows [n_part_a, n_part_a + n_part_b) (written at an offset)
    __shared__ double part[kWaves];
    const int i = blockIdx.x;
    const int rows = n_part_a + n_part_b;
    double s = 0.0;
    for (int r = threadIdx.x; r < rows; r += kBlock) s += D.xi_part[int64_t(r) * D.F * 6 + i];
    s = wave_sum(s);
    if (lane_id() == 0) part[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int w = 0; w < kWaves; ++w) t += part[w];
        g_left[i] = t;
    }
}

// 3x3 helpers in float64 for the pose Jacobian.
__device__ __forceinline__ void hat3(const double *w, double M[3][3]) {
    M[0][0] = 0.0;   M[0][1] = -w[2]; M[0][2] = w[1];
    M[1][0] = w[2];  M[1][1] = 0.0;   M[1][2] = -w[0];
    M[2][0] = -w[1]; M[2][1] = w[0];  M[2][2] = 0.0;
}
__device__ __forceinline__ void mul3(const double A[3][3], const double B[3][3], double C[3][3]) {
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) C[i][j] = A[i][0] * B[0][j] + A[i][1] * B[1][j] + A[i][2] * B[2][j];
}

// dL/dxi_f = J_l(xi_f)^T g_f.  J_l = [[J, Q], [0, J]] in (rho; phi) order, with J the SO(3)
// left Jacobian of phi and Q the closed-form coupling block of the SE(3) left Jacobian
// (Barfoot and Furgale, IEEE T-RO 2014); series coefficients below theta = 1e-2.
// xi == nullptr: J_l = I.  One thread per frame.
__global__ void k_pose_grad(const double *g_left, const float *xi, int F, float *grad_xi) {
    const int f = threadIdx.x;
    if (f >= F) return;
    const double *g = g_left + 6 * f;
    if (!xi) {
        for (int i = 0; i < 6; ++i) grad_xi[6 * f + i] = float(g[i]);
        return;
    }
    const double rho[3] = {xi[6 * f + 0], xi[6 * f + 1], xi[6 * f + 2]};
    const double phi[3] = {xi[6 * f + 3], xi[6 * f + 4], xi[6 * f + 5]};
    const double t2 = phi[0] * phi[0] + phi[1] * phi[1] + phi[2] * phi[2];
    const double t = sqrt(t2);
    double a, b, c, d;  // (1-cos)/t^2, (t-sin)/t^3, (t^2+2cos-2)/(2t^4), (2t-3sin+t cos)/(2t^5)
    if (t < 1e-2) {
        a = 0.5 - t2 / 24.0 + t2 * t2 / 720.0;
        b = 1.0 / 6.0 - t2 / 120.0 + t2 * t2 / 5040.0;
        c = 1.0 / 24.0 - t2 / 720.0 + t2 * t2 / 40320.0;
        d = 1.0 / 120.0 - t2 / 2520.0;
    } else {
        const double sn = sin(t), cs = cos(t);
        a = (1.0 - cs) / t2;
        b = (t - sn) / (t2 * t);
        c = (t2 + 2.0 * cs - 2.0) / (2.0 * t2 * t2);
        d = (2.0 * t - 3.0 * sn + t * cs) / (2.0 * t2 * t2 * t);
    }
    double P[3][3], R[3][3], PP[3][3], PR[3][3], RP[3][3], PRP[3][3], PPR[3][3], RPP[3][3], PRPP[3][3], PPRP[3][3];
    hat3(phi, P);
    hat3(rho, R);
    mul3(P, P, PP);
    mul3(P, R, PR);
    mul3(R, P, RP);
    mul3(PR, P, PRP);
    mul3(PP, R, PPR);
    mul3(R, PP, RPP);
    mul3(PRP, P, PRPP);
    mul3(PP, RP, PPRP);
    double J[3][3], Q[3][3];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            J[i][j] = (i == j ? 1.0 : 0.0) + a * P[i][j] + b * PP[i][j];
            Q[i][j] = 0.5 * R[i][j] + b * (PR[i][j] + RP[i][j] + PRP[i][j]) +
                      c * (PPR[i][j] + RPP[i][j] - 3.0 * PRP[i][j]) + d * (PRPP[i][j] + PPRP[i][j]);
        }
    // [J Q; 0 J]^T g = (J^T g_rho ; Q^T g_rho + J^T g_phi)
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        const double top = J[0][j] * g[0] + J[1][j] * g[1] + J[2][j] * g[2];
        const double bot = Q[0][j] * g[0] + Q[1][j] * g[1] + Q[2][j] * g[2] + J[0][j] * g[3] + J[1][j] * g[4] +
                           J[2][j] * g[5];
        grad_xi[6 * f + j] = float(top);
        grad_xi[6 * f + 3 + j] = float(bot);
    }
}

}  // namespace

struct vbh_diff {
    vbh_scene *s = nullptr;
    int F = 0;
    DiffDev d{};
    void *mem[8] = {};
    float *h_xi = nullptr;     // pinned staging of the caller's xi [F][6]
    float base[kMaxFrames][12] = {};  // the forward's base poses T0
    Cams cams{};               // the forward's composed poses Exp(xi) T0 (float32)
    bool have_forward = false;
    bool with_xi = false;
};

namespace {
// Exp(xi) T0 in float64, rounded to float32.  Exp of xi = (rho; phi): rotation
// R = I + (sin t / t) K + ((1 - cos t) / t^2) K^2 (Rodrigues, K = phi^, t = |phi|) and
// translation V rho with V = I + ((1 - cos t) / t^2) K + ((t - sin t) / t^3) K^2.
void compose_pose(const float *T0, const float *xi, float *P) {
    const double rho[3] = {xi[0], xi[1], xi[2]}, phi[3] = {xi[3], xi[4], xi[5]};
    const double t2 = phi[0] * phi[0] + phi[1] * phi[1] + phi[2] * phi[2], t = std::sqrt(t2);
    double A, B, Cc;
    if (t < 1e-4) {
        A = 1.0 - t2 / 6.0;
        B = 0.5 - t2 / 24.0;
        Cc = 1.0 / 6.0 - t2 / 120.0;
    } else {
        A = std::sin(t) / t;
        B = (1.0 - std::cos(t)) / t2;
        Cc = (t - std::sin(t)) / (t2 * t);
    }
    const double K[3][3] = {{0.0, -phi[2], phi[1]}, {phi[2], 0.0, -phi[0]}, {-phi[1], phi[0], 0.0}};
    double R[3][3], V[3][3];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            const double K2 = K[i][0] * K[0][j] + K[i][1] * K[1][j] + K[i][2] * K[2][j];
            R[i][j] = (i == j ? 1.0 : 0.0) + A * K[i][j] + B * K2;
            V[i][j] = (i == j ? 1.0 : 0.0) + B * K[i][j] + Cc * K2;
        }
    for (int i = 0; i < 3; ++i) {
        const double te = V[i][0] * rho[0] + V[i][1] * rho[1] + V[i][2] * rho[2];
        for (int j = 0; j < 3; ++j)
            P[i * 4 + j] = float(R[i][0] * double(T0[0 * 4 + j]) + R[i][1] * double(T0[1 * 4 + j]) +
                                 R[i][2] * double(T0[2 * 4 + j]));
        P[i * 4 + 3] = float(R[i][0] * double(T0[3]) + R[i][1] * double(T0[7]) + R[i][2] * double(T0[11]) + te);
    }
}

bool finite_n(const float *p, int n) {
    for (int i = 0; i < n; ++i)
        if (!std::isfinite(p[i])) return false;
    return true;
}
}  // namespace

extern "C" {

int vbh_diff_create(const vbh_params *p, int32_t n_frames, vbh_diff **out) {
    if (!out || !p || n_frames < 1 || n_frames > kMaxFrames) return VBH_EINVAL;
    *out = nullptr;
    vbh_diff *D = new (std::nothrow) vbh_diff();
    if (!D) return VBH_ENOMEM;
    if (int rc = vbh_scene_create(p, &D->s)) {
        delete D;
        return rc;
    }
    D->F = n_frames;
    const uint64_t P = uint64_t(p->pool_blocks);
    const size_t HW = size_t(p->width) * size_t(p->height);
    const size_t sizes[] = {P * 4, P * 512 * 8, P * 4, size_t(kMaxWG) * 8, size_t(2 * kMaxWG) * kMaxFrames * 6 * 8,
                            HW * size_t(n_frames) * 8, P * 512 * 8, size_t(kMaxFrames) * 6 * 8};
    for (int i = 0; i < 8; ++i) {
        if (hipMalloc(&D->mem[i], sizes[i]) != hipSuccess) {
            vbh_diff_destroy(D);
            return VBH_ENOMEM;
        }
    }
    if (hipHostMalloc(reinterpret_cast<void **>(&D->h_xi), size_t(kMaxFrames) * 6 * sizeof(float), 0) != hipSuccess) {
        D->h_xi = nullptr;
        vbh_diff_destroy(D);
        return VBH_ENOMEM;
    }
    D->d.S = D->s->d;
    D->d.fmask = static_cast<uint32_t *>(D->mem[0]);
    D->d.dLdF = static_cast<double *>(D->mem[1]);
    D->d.F64 = static_cast<double *>(D->mem[6]);
    D->d.hot = static_cast<uint32_t *>(D->mem[2]);
    D->d.loss_part = static_cast<double *>(D->mem[3]);
    D->d.xi_part = static_cast<double *>(D->mem[4]);
    D->d.gd64 = static_cast<double *>(D->mem[5]);
    D->d.F = n_frames;
    *out = D;
    return VBH_OK;
}

void vbh_diff_destroy(vbh_diff *D) {
    if (!D) return;
    for (void *m : D->mem)
        if (m) (void)hipFree(m);
    if (D->h_xi) (void)hipHostFree(D->h_xi);
    vbh_scene_destroy(D->s);
    delete D;
}

int vbh_diff_forward(vbh_diff *D, const float *d_depth, const float *h_poses, const float *d_xi,
                     const int32_t *d_sample_frame, const int32_t *d_sample_pixel, int64_t n_samples,
                     float *d_f_samples, float *d_loss, void *stream) {
    if (!D || !d_depth || !h_poses || n_samples < 0 || (n_samples > 0 && (!d_sample_frame || !d_sample_pixel)) ||
        !d_loss || (n_samples + kSampleWG - 1) / kSampleWG > kMaxWG || !finite_n(h_poses, 12 * D->F))
        return VBH_EINVAL;
    hipStream_t st = as_stream(stream);
    D->have_forward = false;
    if (d_xi) {
        // the composed poses are kernel arguments: xi is read back once, synchronously
        if (hipMemcpyAsync(D->h_xi, d_xi, size_t(D->F) * 6 * sizeof(float), hipMemcpyDeviceToHost, st) !=
                hipSuccess ||
            hipStreamSynchronize(st) != hipSuccess)
            return VBH_EHIP;
        if (!finite_n(D->h_xi, 6 * D->F)) return VBH_EINVAL;
    }
    for (int f = 0; f < D->F; ++f) {
        std::memcpy(D->base[f], h_poses + 12 * f, sizeof(D->base[f]));
        if (d_xi)
            compose_pose(h_poses + 12 * f, D->h_xi + 6 * f, D->cams.P[f]);
        else
            std::memcpy(D->cams.P[f], h_poses + 12 * f, sizeof(D->cams.P[f]));
    }
    D->with_xi = d_xi != nullptr;
    const Cams &cams = D->cams;
    vbh_scene *s = D->s;
    if (int rc = scene_reset(s, st)) return rc;
    const unsigned g = unsigned(s->cus) * 8;
    k_zero_u32<<<g, kBlock, 0, st>>>(D->d.fmask, s->p.pool_blocks);
    VBH_LAUNCHED();
    const int64_t HW = int64_t(s->p.width) * s->p.height;
    for (int f = 0; f < D->F; ++f) {
        const int seq = s->seq;
        if (int rc = scene_alloc_only(s, d_depth + f * HW, cams.P[f], uint32_t(f + 1), st)) return rc;
        k_touch_mask<<<g, kBlock, 0, st>>>(D->d, f, seq);
    }
    const Frame fr = make_frame(s, cams.P[0]);
    k_mean64<<<g, kBlock, 0, st>>>(D->d, fr, cams, d_depth);
    const unsigned gs = unsigned((n_samples + kSampleWG - 1) / kSampleWG);
    if (gs > 0)
        k_sample_fwd<<<gs, kSampleWG, 0, st>>>(D->d, fr, cams, d_depth, d_sample_frame, d_sample_pixel, n_samples,
                                                d_f_samples);
    k_reduce_loss<<<1, 256, 0, st>>>(D->d, int(gs), d_loss);
    VBH_LAUNCHED();
    D->have_forward = true;
    return VBH_OK;
}

int vbh_diff_backward(vbh_diff *D, const float *d_depth, const float *h_poses, const float *d_xi,
                      const int32_t *d_sample_frame, const int32_t *d_sample_pixel, int64_t n_samples,
                      const float *d_grad_loss, float *d_grad_depth, float *d_grad_xi, void *stream) {
    if (!D || !D->have_forward || !d_depth || !h_poses || !d_grad_loss || !d_grad_depth || !d_grad_xi ||
        n_samples < 0 || (n_samples > 0 && (!d_sample_frame || !d_sample_pixel)) ||
        (n_samples + kSampleWG - 1) / kSampleWG > kMaxWG || (d_xi != nullptr) != D->with_xi ||
        std::memcmp(h_poses, D->base, size_t(D->F) * 12 * sizeof(float)) != 0)
        return VBH_EINVAL;
    hipStream_t st = as_stream(stream);
    const Cams &cams = D->cams;
    vbh_scene *s = D->s;
    const int64_t HW = int64_t(s->p.width) * s->p.height;
    const unsigned g = unsigned(s->cus) * 8;
    k_zero_grad_blocks<<<g, kBlock, 0, st>>>(D->d);
    k_zero_f64<<<g, kBlock, 0, st>>>(D->d.gd64, HW * D->F);
    const Frame fr = make_frame(s, cams.P[0]);
    const unsigned gs = unsigned((n_samples + kSampleWG - 1) / kSampleWG);
    if (gs > 0)
        k_sample_bwd<<<gs, kSampleWG, 0, st>>>(D->d, fr, cams, d_depth, d_sample_frame, d_sample_pixel, n_samples,
                                                d_grad_loss);
    DiffDev db = D->d;
    db.xi_part = D->d.xi_part + int64_t(gs) * D->F * 6;  // integration partials follow
    const unsigned gb = g < unsigned(kMaxWG) ? g : unsigned(kMaxWG);
    k_integrate_bwd<<<gb, kBlock, 0, st>>>(db, fr, cams, d_depth);
    double *g_left = static_cast<double *>(D->mem[7]);
    k_reduce_xi<<<unsigned(D->F * 6), kBlock, 0, st>>>(D->d, int(gs), int(gb), g_left);
    k_pose_grad<<<1, 64, 0, st>>>(g_left, d_xi, D->F, d_grad_xi);
    k_to_f32<<<g, kBlock, 0, st>>>(D->d.gd64, d_grad_depth, HW * D->F);
    VBH_LAUNCHED();
    return VBH_OK;
}

}  // extern "C"
