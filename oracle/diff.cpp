// CPU oracle of the differentiable form: TSDF integration of several frames into a fresh
// volume and the loss L = sum_k F_tri(x_k)^2 at back-projected pixel samples, with its
// gradient with respect to per-pixel depth and a left se(3) perturbation of every pose.
//
// TEST INFRASTRUCTURE ONLY (see oracle.h).  Shares no code with the HIP path.
//
// Frozen branches: every discrete decision - the band blocks, each voxel's pixel, its
// validity, the -trunc skip and the +trunc clamp, each sample's trilinear cell and the
// mask of samples with a valid depth whose eight corners are observed - is taken once, in float32 in the
// written operation order, from the unperturbed inputs.  Values are float64:
//   F_v = (1/n_v) sum_{f observes v} tsdf_f(v),  tsdf = D_f[pix] - z_f(v) (or trunc if
//   clamped), z_f(v) = r3_f . (X_v - t_f) with T_f = Exp(xi_f) T0_f (xi = (rho; phi));
//   the reference point is xi_ref (zero by default): its poses Exp(xi_ref) T0, rounded to
//   float32 as the fusion's pose input, take the decisions and are the point where values
//   and gradients are evaluated; a perturbed pose is Exp(xi) T0' with the float64 base
//   T0' = Exp(-xi_ref) P32 that maps exactly onto that rounded reference pose P32;
//   x_k = T_f (D_f[p_k] K^-1 [u, v, 1]);  F_tri = sum_c w_c(frac) F_c.
#include <algorithm>
#include <array>
#include <cmath>
#include <cstring>
#include <unordered_map>
#include <vector>

#include "oracle.h"

namespace {

constexpr int64_t kOff = int64_t(1) << 20;

uint64_t pack(int64_t x, int64_t y, int64_t z) {
    return (uint64_t(x + kOff) << 42) | (uint64_t(y + kOff) << 21) | uint64_t(z + kOff);
}
void unpack(uint64_t k, int64_t *o) {
    const uint64_t m = (uint64_t(1) << 21) - 1;
    o[0] = int64_t((k >> 42) & m) - kOff;
    o[1] = int64_t((k >> 21) & m) - kOff;
    o[2] = int64_t(k & m) - kOff;
}
int64_t fdiv8(int64_t g) { return g >= 0 ? g / 8 : -((-g + 7) / 8); }

bool valid_depth(float d, const orc_params &p) { return d > 0.0f && d >= p.depth_min && d <= p.depth_max; }

// 3x3 and SE(3) helpers in float64
struct Pose {
    double R[3][3];
    double t[3];
};

void hat(const double *w, double M[3][3]) {
    M[0][0] = 0; M[0][1] = -w[2]; M[0][2] = w[1];
    M[1][0] = w[2]; M[1][1] = 0; M[1][2] = -w[0];
    M[2][0] = -w[1]; M[2][1] = w[0]; M[2][2] = 0;
}

// Exp of xi = (rho; phi): rotation by Rodrigues' formula, translation V rho.
Pose se3_exp(const double *xi) {
    const double *rho = xi, *phi = xi + 3;
    const double th2 = phi[0] * phi[0] + phi[1] * phi[1] + phi[2] * phi[2];
    const double th = std::sqrt(th2);
    double A, B, C;  // sin/th, (1-cos)/th^2, (th - sin)/th^3
    if (th < 1e-6) {
        A = 1 - th2 / 6;
        B = 0.5 - th2 / 24;
        C = 1.0 / 6 - th2 / 120;
    } else {
        A = std::sin(th) / th;
        B = (1 - std::cos(th)) / th2;
        C = (th - std::sin(th)) / (th2 * th);
    }
    double K[3][3], K2[3][3];
    hat(phi, K);
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            K2[i][j] = 0;
            for (int k = 0; k < 3; ++k) K2[i][j] += K[i][k] * K[k][j];
        }
    Pose E;
    double V[3][3];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            const double I = i == j ? 1.0 : 0.0;
            E.R[i][j] = I + A * K[i][j] + B * K2[i][j];
            V[i][j] = I + B * K[i][j] + C * K2[i][j];
        }
    for (int i = 0; i < 3; ++i) E.t[i] = V[i][0] * rho[0] + V[i][1] * rho[1] + V[i][2] * rho[2];
    return E;
}

Pose compose(const Pose &a, const Pose &b) {  // a * b
    Pose c;
    for (int i = 0; i < 3; ++i) {
        for (int j = 0; j < 3; ++j) c.R[i][j] = a.R[i][0] * b.R[0][j] + a.R[i][1] * b.R[1][j] + a.R[i][2] * b.R[2][j];
        c.t[i] = a.R[i][0] * b.t[0] + a.R[i][1] * b.t[1] + a.R[i][2] * b.t[2] + a.t[i];
    }
    return c;
}

struct Obs {
    int32_t frame;
    int64_t pix;
    bool unclamped;
};

struct Diff {
    orc_params p{};
    int F = 0;
    int m_band = 0;
    std::vector<float> depth, poses;  // poses: the reference point's, float32 (decisions)
    std::vector<Pose> base_T;         // T0' per frame (float64)
    std::vector<double> xi_ref;       // [F*6], empty = zero
    std::vector<int32_t> sf, sp;
    std::unordered_map<uint64_t, int64_t> index;  // block key -> block id
    std::vector<uint64_t> keys;
    std::vector<uint32_t> fmask;  // frames whose band touched the block
    // voxels that are corners of some kept sample (the only ones the loss reads)
    std::unordered_map<int64_t, int32_t> vid;  // block id * 512 + l -> needed-voxel id
    std::vector<int64_t> vox;
    std::vector<std::vector<Obs>> obs;
    // samples
    std::vector<std::array<int64_t, 3>> base;
    std::vector<std::array<int32_t, 8>> corner;
    std::vector<uint8_t> keep;

    const float *P(int f) const { return &poses[size_t(f) * 12]; }
    const float *D(int f) const { return &depth[size_t(f) * p.width * p.height]; }
};

const int kC[8][3] = {{0, 0, 0}, {1, 0, 0}, {0, 1, 0}, {1, 1, 0}, {0, 0, 1}, {1, 0, 1}, {0, 1, 1}, {1, 1, 1}};

// float32 canonical decisions for voxel g of a block against frame f: pixel index or -1,
// and whether the observation is unclamped (sdf < trunc).
int64_t observe(const Diff &d, int f, const int64_t *g, bool *unclamped) {
    const orc_params &p = d.p;
    const float *P = d.P(f);
    float dl[3], pc[3];
    for (int i = 0; i < 3; ++i) dl[i] = float(g[i]) * p.voxel_size - P[i * 4 + 3];
    for (int j = 0; j < 3; ++j) pc[j] = (P[0 * 4 + j] * dl[0] + P[1 * 4 + j] * dl[1]) + P[2 * 4 + j] * dl[2];
    if (!(pc[2] > 0.0f)) return -1;
    const float fu = std::floor((p.fx * (pc[0] / pc[2]) + p.cx) + 0.5f);
    const float fv = std::floor((p.fy * (pc[1] / pc[2]) + p.cy) + 0.5f);
    if (!(fu >= 0.0f && fu < float(p.width) && fv >= 0.0f && fv < float(p.height))) return -1;
    const int64_t pix = int64_t(fv) * p.width + int64_t(fu);
    const float dd = d.D(f)[pix];
    if (!valid_depth(dd, p)) return -1;
    const float sdf = dd - pc[2];
    if (sdf < -p.trunc) return -1;
    *unclamped = sdf < p.trunc;
    return pix;
}

// float32 canonical sample point x = T0 (d K^-1 [u, v, 1]) and its trilinear cell.
void sample_cell(const Diff &d, int64_t k, int64_t *base) {
    const orc_params &p = d.p;
    const int f = d.sf[size_t(k)];
    const int64_t pix = d.sp[size_t(k)];
    const float u = float(pix % p.width), v = float(pix / p.width);
    const float dd = d.D(f)[pix];
    const float xn = (u - p.cx) / p.fx, yn = (v - p.cy) / p.fy;
    const float pc[3] = {dd * xn, dd * yn, dd};
    const float *P = d.P(f);
    for (int i = 0; i < 3; ++i) {
        const float x = ((P[i * 4 + 0] * pc[0] + P[i * 4 + 1] * pc[1]) + P[i * 4 + 2] * pc[2]) + P[i * 4 + 3];
        base[i] = int64_t(std::floor(x / p.voxel_size));
    }
}

Pose base64(const float *P) {
    Pose T0;
    for (int i = 0; i < 3; ++i) {
        for (int j = 0; j < 3; ++j) T0.R[i][j] = double(P[i * 4 + j]);
        T0.t[i] = double(P[i * 4 + 3]);
    }
    return T0;
}

// Pose of frame f at xi (NULL: the reference point), float64.
Pose pose64(const Diff &d, int f, const double *xi) {
    if (!xi) return base64(d.P(f));  // the reference pose (float32 values)
    return compose(se3_exp(xi + 6 * f), d.base_T[size_t(f)]);
}

// SE(3) left Jacobian of xi = (rho; phi) from its defining series,
// J_l = sum_n ad(xi)^n / (n+1)!,  ad(xi) = [[phi^, rho^], [0, phi^]] (6x6).
void left_jacobian(const double *xi, double J[6][6]) {
    double ad[6][6] = {}, term[6][6] = {}, nxt[6][6];
    double ph[3][3], rh[3][3];
    hat(xi + 3, ph);
    hat(xi, rh);
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            ad[i][j] = ph[i][j];
            ad[i][j + 3] = rh[i][j];
            ad[i + 3][j + 3] = ph[i][j];
        }
    for (int i = 0; i < 6; ++i) {
        term[i][i] = 1.0;  // ad^0 / 1!
        for (int j = 0; j < 6; ++j) J[i][j] = term[i][j];
    }
    for (int n = 1; n <= 40; ++n) {  // term_n = term_{n-1} ad / (n+1)
        for (int i = 0; i < 6; ++i)
            for (int j = 0; j < 6; ++j) {
                double s = 0;
                for (int k = 0; k < 6; ++k) s += term[i][k] * ad[k][j];
                nxt[i][j] = s / double(n + 1);
            }
        for (int i = 0; i < 6; ++i)
            for (int j = 0; j < 6; ++j) {
                term[i][j] = nxt[i][j];
                J[i][j] += term[i][j];
            }
    }
}

void voxel_world(const Diff &d, int64_t gv, double *X, int64_t *g) {
    const int64_t b = gv >> 9;
    const int l = int(gv & 511);
    int64_t B[3];
    unpack(d.keys[size_t(b)], B);
    g[0] = B[0] * 8 + (l & 7);
    g[1] = B[1] * 8 + ((l >> 3) & 7);
    g[2] = B[2] * 8 + (l >> 6);
    for (int i = 0; i < 3; ++i) X[i] = double(g[i]) * double(d.p.voxel_size);
}

// F of every needed voxel at the perturbed point.
std::vector<double> needed_F(const Diff &d, const double *dd, double scale, const double *xi) {
    std::vector<Pose> T(size_t(d.F));
    for (int f = 0; f < d.F; ++f) T[size_t(f)] = pose64(d, f, xi);
    const int64_t HW = int64_t(d.p.width) * d.p.height;
    std::vector<double> Fv(d.vox.size(), 0.0);
#pragma omp parallel for schedule(dynamic, 256)
    for (int64_t i = 0; i < int64_t(d.vox.size()); ++i) {
        const auto &ob = d.obs[size_t(i)];
        if (ob.empty()) continue;
        double X[3];
        int64_t g[3];
        voxel_world(d, d.vox[size_t(i)], X, g);
        double s = 0;
        for (const Obs &o : ob) {
            if (!o.unclamped) {
                s += double(d.p.trunc);
                continue;
            }
            const Pose &Tf = T[size_t(o.frame)];
            const double z = Tf.R[0][2] * (X[0] - Tf.t[0]) + Tf.R[1][2] * (X[1] - Tf.t[1]) + Tf.R[2][2] * (X[2] - Tf.t[2]);
            double D = double(d.D(o.frame)[o.pix]);
            if (dd) D += scale * dd[int64_t(o.frame) * HW + o.pix];
            s += D - z;
        }
        Fv[size_t(i)] = s / double(ob.size());
    }
    return Fv;
}

// x_k at the perturbed point (float64), and the sample's camera ray r_c.
void sample_point(const Diff &d, int64_t k, const Pose &T, const double *dd, double scale, double *x, double *pc) {
    const orc_params &p = d.p;
    const int f = d.sf[size_t(k)];
    const int64_t pix = d.sp[size_t(k)];
    double D = double(d.D(f)[pix]);
    if (dd) D += scale * dd[int64_t(f) * p.width * p.height + pix];
    const double u = double(pix % p.width), v = double(pix / p.width);
    pc[0] = D * (u - double(p.cx)) / double(p.fx);
    pc[1] = D * (v - double(p.cy)) / double(p.fy);
    pc[2] = D;
    for (int i = 0; i < 3; ++i) x[i] = T.R[i][0] * pc[0] + T.R[i][1] * pc[1] + T.R[i][2] * pc[2] + T.t[i];
}

void weights(const double *fr, double *w, double dw[8][3]) {
    for (int c = 0; c < 8; ++c) {
        double a[3], da[3];
        for (int i = 0; i < 3; ++i) {
            a[i] = kC[c][i] ? fr[i] : 1.0 - fr[i];
            da[i] = kC[c][i] ? 1.0 : -1.0;
        }
        w[c] = a[0] * a[1] * a[2];
        if (dw) {
            dw[c][0] = da[0] * a[1] * a[2];
            dw[c][1] = a[0] * da[1] * a[2];
            dw[c][2] = a[0] * a[1] * da[2];
        }
    }
}

}  // namespace

extern "C" {

void *orc_diff_new(const orc_diff_problem *prob) {
    if (!prob || prob->n_frames <= 0 || prob->n_frames > 32 || !prob->depth || !prob->poses) return nullptr;
    Diff *d = new Diff();
    d->p = prob->p;
    d->F = prob->n_frames;
    d->m_band = int(std::floor(d->p.trunc / d->p.voxel_size + 0.5f));
    const int64_t HW = int64_t(d->p.width) * d->p.height;
    d->depth.assign(prob->depth, prob->depth + HW * d->F);
    d->poses.assign(prob->poses, prob->poses + 12 * d->F);
    d->base_T.resize(size_t(d->F));
    for (int f = 0; f < d->F; ++f) d->base_T[size_t(f)] = base64(d->P(f));
    if (prob->xi_ref) {
        d->xi_ref.assign(prob->xi_ref, prob->xi_ref + 6 * d->F);
        for (int f = 0; f < d->F; ++f) {
            // the reference pose Exp(xi_ref) T0, rounded to float32 ...
            const Pose T = compose(se3_exp(&d->xi_ref[size_t(f) * 6]), d->base_T[size_t(f)]);
            for (int i = 0; i < 3; ++i) {
                for (int j = 0; j < 3; ++j) d->poses[size_t(f) * 12 + i * 4 + j] = float(T.R[i][j]);
                d->poses[size_t(f) * 12 + i * 4 + 3] = float(T.t[i]);
            }
            // ... and the base that Exp(xi_ref) maps onto it exactly
            double neg[6];
            for (int a = 0; a < 6; ++a) neg[a] = -d->xi_ref[size_t(f) * 6 + a];
            d->base_T[size_t(f)] = compose(se3_exp(neg), base64(d->P(f)));
        }
    }
    d->sf.assign(prob->sample_frame, prob->sample_frame + prob->n_samples);
    d->sp.assign(prob->sample_pixel, prob->sample_pixel + prob->n_samples);
    const orc_params &p = d->p;
    const float bs = 8.0f * p.voxel_size;
    // band blocks per frame (the same float32 rules as the fusion oracle)
    for (int f = 0; f < d->F; ++f) {
        const float *P = d->P(f);
        for (int v = 0; v < p.height; ++v)
            for (int u = 0; u < p.width; ++u) {
                const float dd = d->D(f)[int64_t(v) * p.width + u];
                if (!valid_depth(dd, p)) continue;
                const float xn = (float(u) - p.cx) / p.fx, yn = (float(v) - p.cy) / p.fy;
                for (int s = 0; s <= 2 * d->m_band; ++s) {
                    const float lam = (dd - p.trunc) + float(s) * p.voxel_size;
                    if (!(lam > 0.0f)) continue;
                    const float pc[3] = {lam * xn, lam * yn, lam};
                    int64_t B[3];
                    for (int i = 0; i < 3; ++i) {
                        const float pw = ((P[i * 4 + 0] * pc[0] + P[i * 4 + 1] * pc[1]) + P[i * 4 + 2] * pc[2]) + P[i * 4 + 3];
                        B[i] = int64_t(std::floor(pw / bs));
                    }
                    const uint64_t key = pack(B[0], B[1], B[2]);
                    auto it = d->index.find(key);
                    if (it == d->index.end()) {
                        it = d->index.emplace(key, int64_t(d->keys.size())).first;
                        d->keys.push_back(key);
                        d->fmask.push_back(0);
                    }
                    d->fmask[size_t(it->second)] |= 1u << f;
                }
            }
    }
    // samples: frozen cell; the corners' observations
    const int64_t K = prob->n_samples;
    d->base.resize(size_t(K));
    d->corner.resize(size_t(K));
    d->keep.assign(size_t(K), 0);
    for (int64_t k = 0; k < K; ++k) {
        const int fk = d->sf[size_t(k)];
        if (fk < 0 || fk >= d->F || !valid_depth(d->D(fk)[d->sp[size_t(k)]], p)) continue;  // dropped
        int64_t b[3];
        sample_cell(*d, k, b);
        d->base[size_t(k)] = {b[0], b[1], b[2]};
        bool ok = true;
        for (int c = 0; c < 8 && ok; ++c) {
            const int64_t g[3] = {b[0] + kC[c][0], b[1] + kC[c][1], b[2] + kC[c][2]};
            const int64_t B[3] = {fdiv8(g[0]), fdiv8(g[1]), fdiv8(g[2])};
            auto it = d->index.find(pack(B[0], B[1], B[2]));
            if (it == d->index.end()) { ok = false; break; }
            const int l = int(g[0] - 8 * B[0]) + 8 * int(g[1] - 8 * B[1]) + 64 * int(g[2] - 8 * B[2]);
            const int64_t gv = it->second * 512 + l;
            auto jt = d->vid.find(gv);
            if (jt == d->vid.end()) {
                jt = d->vid.emplace(gv, int32_t(d->vox.size())).first;
                d->vox.push_back(gv);
                std::vector<Obs> ob;
                for (int f = 0; f < d->F; ++f) {
                    if (!(d->fmask[size_t(it->second)] >> f & 1u)) continue;
                    bool unc = false;
                    const int64_t pix = observe(*d, f, g, &unc);
                    if (pix >= 0) ob.push_back({f, pix, unc});
                }
                d->obs.push_back(std::move(ob));
            }
            d->corner[size_t(k)][size_t(c)] = jt->second;
            if (d->obs[size_t(jt->second)].empty()) ok = false;
        }
        d->keep[size_t(k)] = ok ? 1 : 0;
    }
    return d;
}

void orc_diff_free(void *h) { delete static_cast<Diff *>(h); }

double orc_diff_loss(void *h, const double *dd, double scale, const double *xi) {
    const Diff &d = *static_cast<Diff *>(h);
    const std::vector<double> Fv = needed_F(d, dd, scale, xi);
    std::vector<Pose> T(size_t(d.F));
    for (int f = 0; f < d.F; ++f) T[size_t(f)] = pose64(d, f, xi);
    double L = 0;
    for (int64_t k = 0; k < int64_t(d.keep.size()); ++k) {
        if (!d.keep[size_t(k)]) continue;
        double x[3], pc[3], fr[3], w[8];
        sample_point(d, k, T[size_t(d.sf[size_t(k)])], dd, scale, x, pc);
        for (int i = 0; i < 3; ++i) fr[i] = x[i] / double(d.p.voxel_size) - double(d.base[size_t(k)][size_t(i)]);
        weights(fr, w, nullptr);
        double Ft = 0;
        for (int c = 0; c < 8; ++c) Ft += w[c] * Fv[size_t(d.corner[size_t(k)][size_t(c)])];
        L += Ft * Ft;
    }
    return L;
}

int orc_diff_grad(void *h, double *gD, double *gxi) {
    const Diff &d = *static_cast<Diff *>(h);
    const int64_t HW = int64_t(d.p.width) * d.p.height;
    std::fill(gD, gD + HW * d.F, 0.0);
    std::fill(gxi, gxi + 6 * d.F, 0.0);
    const std::vector<double> Fv = needed_F(d, nullptr, 0.0, nullptr);
    std::vector<double> dLdF(Fv.size(), 0.0);
    const double ivs = 1.0 / double(d.p.voxel_size);
    for (int64_t k = 0; k < int64_t(d.keep.size()); ++k) {
        if (!d.keep[size_t(k)]) continue;
        const int f = d.sf[size_t(k)];
        const Pose T = pose64(d, f, nullptr);
        double x[3], pc[3], fr[3], w[8], dw[8][3];
        sample_point(d, k, T, nullptr, 0.0, x, pc);
        for (int i = 0; i < 3; ++i) fr[i] = x[i] * ivs - double(d.base[size_t(k)][size_t(i)]);
        weights(fr, w, dw);
        double Ft = 0, gF[3] = {0, 0, 0};
        for (int c = 0; c < 8; ++c) {
            const double Fc = Fv[size_t(d.corner[size_t(k)][size_t(c)])];
            Ft += w[c] * Fc;
            for (int i = 0; i < 3; ++i) gF[i] += dw[c][i] * Fc * ivs;
        }
        for (int c = 0; c < 8; ++c) dLdF[size_t(d.corner[size_t(k)][size_t(c)])] += 2 * Ft * w[c];
        const double gx[3] = {2 * Ft * gF[0], 2 * Ft * gF[1], 2 * Ft * gF[2]};
        // x = T (D r_c): dx/dD = R r_c; left perturbation: dx/drho = I, dx/dphi = -[x]_x
        const double rc[3] = {pc[0] / pc[2], pc[1] / pc[2], 1.0};
        double dxdD = 0;
        for (int i = 0; i < 3; ++i) dxdD += gx[i] * (T.R[i][0] * rc[0] + T.R[i][1] * rc[1] + T.R[i][2] * rc[2]);
        gD[int64_t(f) * HW + d.sp[size_t(k)]] += dxdD;
        double *g = gxi + 6 * f;
        for (int i = 0; i < 3; ++i) g[i] += gx[i];
        g[3] += x[1] * gx[2] - x[2] * gx[1];
        g[4] += x[2] * gx[0] - x[0] * gx[2];
        g[5] += x[0] * gx[1] - x[1] * gx[0];
    }
    // through integration: F_v = mean of (D - z); dz/drho = -r3, dz/dphi = r3 x X
    for (size_t i = 0; i < Fv.size(); ++i) {
        if (dLdF[i] == 0.0 || d.obs[i].empty()) continue;
        const double c = dLdF[i] / double(d.obs[i].size());
        double X[3];
        int64_t gg[3];
        voxel_world(d, d.vox[i], X, gg);
        for (const Obs &o : d.obs[i]) {
            if (!o.unclamped) continue;
            const Pose T = pose64(d, o.frame, nullptr);
            const double r3[3] = {T.R[0][2], T.R[1][2], T.R[2][2]};
            gD[int64_t(o.frame) * HW + o.pix] += c;
            double *g = gxi + 6 * o.frame;
            for (int a = 0; a < 3; ++a) g[a] += c * r3[a];
            g[3] += c * (X[1] * r3[2] - X[2] * r3[1]);
            g[4] += c * (X[2] * r3[0] - X[0] * r3[2]);
            g[5] += c * (X[0] * r3[1] - X[1] * r3[0]);
        }
    }
    // dL/dxi = J_l(xi_ref)^T (left-perturbation gradient at the reference poses)
    if (!d.xi_ref.empty()) {
        for (int f = 0; f < d.F; ++f) {
            double J[6][6], g[6];
            left_jacobian(&d.xi_ref[size_t(f) * 6], J);
            for (int j = 0; j < 6; ++j) {
                g[j] = 0;
                for (int i = 0; i < 6; ++i) g[j] += J[i][j] * gxi[6 * f + i];
            }
            for (int j = 0; j < 6; ++j) gxi[6 * f + j] = g[j];
        }
    }
    return ORC_OK;
}

int64_t orc_diff_info(void *h, int64_t *n_kept, int64_t *n_grad_voxels, double *f_samples) {
    const Diff &d = *static_cast<Diff *>(h);
    const std::vector<double> Fv = needed_F(d, nullptr, 0.0, nullptr);
    int64_t kept = 0;
    std::vector<uint8_t> touched(Fv.size(), 0);
    for (int64_t k = 0; k < int64_t(d.keep.size()); ++k) {
        if (!d.keep[size_t(k)]) {
            if (f_samples) f_samples[k] = std::nan("");
            continue;
        }
        ++kept;
        const Pose T = pose64(d, d.sf[size_t(k)], nullptr);
        double x[3], pc[3], fr[3], w[8];
        sample_point(d, k, T, nullptr, 0.0, x, pc);
        for (int i = 0; i < 3; ++i) fr[i] = x[i] / double(d.p.voxel_size) - double(d.base[size_t(k)][size_t(i)]);
        weights(fr, w, nullptr);
        double Ft = 0;
        for (int c = 0; c < 8; ++c) {
            Ft += w[c] * Fv[size_t(d.corner[size_t(k)][size_t(c)])];
            touched[size_t(d.corner[size_t(k)][size_t(c)])] = 1;
        }
        if (f_samples) f_samples[k] = Ft;
    }
    if (n_kept) *n_kept = kept;
    if (n_grad_voxels) *n_grad_voxels = int64_t(std::count(touched.begin(), touched.end(), uint8_t(1)));
    return int64_t(d.keys.size());
}

}  // extern "C"
