// CPU oracle: hash map semantics, block allocation, TSDF integration, MC voxel
// encoding and the update log of SLAMCast's server model (Stotko et al., TVCG 2019).
//
// TEST INFRASTRUCTURE ONLY: loaded by the tests, the smoke check and the CPU-baseline
// leg of the benchmark; never by the product path.  Shares no code with the HIP path.
//
// Build: g++ -std=c++17 -O2 -fopenmp -ffp-contract=off -fno-fast-math -shared -fPIC.
// Every discrete decision (band-sample block keys, voxel->pixel index, validity and
// skip tests) is evaluated in IEEE float32 in the written operation order, so that a
// device implementation that follows the same written formulas takes the same
// decisions; the values (TSDF, running averages) are carried in float64.
#include "oracle.h"

#include <algorithm>
#include <array>
#include <cmath>
#include <cstring>
#include <unordered_map>
#include <vector>

namespace {

constexpr int64_t kOff = int64_t(1) << 20;
constexpr uint64_t kM21 = (uint64_t(1) << 21) - 1;

bool key_in_range(int64_t x, int64_t y, int64_t z) {
    return x >= -kOff && x < kOff && y >= -kOff && y < kOff && z >= -kOff && z < kOff;
}

uint64_t pack(int64_t x, int64_t y, int64_t z) {
    return (uint64_t(x + kOff) << 42) | (uint64_t(y + kOff) << 21) | uint64_t(z + kOff);
}

void unpack(uint64_t k, int32_t *out) {
    out[0] = int32_t(int64_t((k >> 42) & kM21) - kOff);
    out[1] = int32_t(int64_t((k >> 21) & kM21) - kOff);
    out[2] = int32_t(int64_t(k & kM21) - kOff);
}

// floor division for block coordinates (correct for negatives)
int64_t fdiv8(int64_t g) { return g >= 0 ? g / 8 : -((-g + 7) / 8); }

// ------------------------------------------------------------------ hash map (Sec. 5)
struct Map {
    std::unordered_map<uint64_t, int32_t> m;
};

int32_t map_op(Map &M, uint8_t op, const int32_t *k, int32_t v) {
    if (!key_in_range(k[0], k[1], k[2])) return -1;
    uint64_t key = pack(k[0], k[1], k[2]);
    if (op == 0) return M.m.emplace(key, v).second ? 1 : 0;           // insert-if-absent
    if (op == 1) {                                                     // find
        auto it = M.m.find(key);
        return it == M.m.end() ? ORC_ABSENT : it->second;
    }
    return M.m.erase(key) ? 1 : 0;                                     // erase
}

// ------------------------------------------------------------------------ scene
struct Blk {
    double F[512];
    uint8_t W[512];
    uint8_t C[512 * 3];
    uint32_t mc[512];  // stored MC voxel: index | r<<8 | g<<16 | b<<24
    uint32_t mc_stamp;
};

// MC corner offsets in the Lorensen-Cline numbering: bottom face (z=0) counter-clockwise
// from the origin, then the top face (z=1) in the same order.
const int kCorner[8][3] = {{0, 0, 0}, {1, 0, 0}, {1, 1, 0}, {0, 1, 0},
                           {0, 0, 1}, {1, 0, 1}, {1, 1, 1}, {0, 1, 1}};

struct Scene {
    orc_params p;
    int m_band;  // band half-width in voxels
    std::unordered_map<uint64_t, int64_t> index;  // block key -> storage index
    std::vector<Blk> blocks;
    std::vector<uint64_t> block_key;
    std::vector<std::pair<uint32_t, uint64_t>> log;  // (frame, key) in append order
    std::vector<uint64_t> last_touched, last_new, last_mc;
    uint32_t last_frame = 0;
    int error = 0;

    const Blk *get(uint64_t key) const {
        auto it = index.find(key);
        return it == index.end() ? nullptr : &blocks[size_t(it->second)];
    }
    Blk *get(uint64_t key) {
        auto it = index.find(key);
        return it == index.end() ? nullptr : &blocks[size_t(it->second)];
    }
    // Allocate a zeroed block; returns nullptr (and records the error) when full.
    Blk *alloc(uint64_t key) {
        if (int64_t(blocks.size()) >= p.pool_blocks) {
            error = ORC_EFULL_POOL;
            return nullptr;
        }
        index.emplace(key, int64_t(blocks.size()));
        blocks.emplace_back();
        std::memset(&blocks.back(), 0, sizeof(Blk));
        block_key.push_back(key);
        return &blocks.back();
    }
};

// The depth validity rule: positive and inside [depth_min, depth_max] (float32 tests).
bool depth_valid(float d, const orc_params &p) {
    return d > 0.0f && d >= p.depth_min && d <= p.depth_max;
}

// Band allocation for one frame: every valid pixel contributes 2m+1 samples at camera
// depths (d - mu) + s*vs, s = 0..2m; each sample's world point names a block.
std::vector<uint64_t> band_keys(const Scene &S, const float *depth, const float *P, bool *range_err) {
    const orc_params &p = S.p;
    const float bs = 8.0f * p.voxel_size;
    std::vector<uint64_t> keys;
    for (int v = 0; v < p.height; ++v) {
        for (int u = 0; u < p.width; ++u) {
            const float d = depth[int64_t(v) * p.width + u];
            if (!depth_valid(d, p)) continue;
            const float xn = (float(u) - p.cx) / p.fx;
            const float yn = (float(v) - p.cy) / p.fy;
            for (int s = 0; s <= 2 * S.m_band; ++s) {
                const float lam = (d - p.trunc) + float(s) * p.voxel_size;
                if (!(lam > 0.0f)) continue;
                const float pc[3] = {lam * xn, lam * yn, lam};
                int64_t B[3];
                bool ok = true;
                for (int i = 0; i < 3; ++i) {
                    const float pw = ((P[i * 4 + 0] * pc[0] + P[i * 4 + 1] * pc[1]) + P[i * 4 + 2] * pc[2]) + P[i * 4 + 3];
                    const float q = std::floor(pw / bs);
                    if (!(q >= -1048576.0f && q < 1048576.0f)) { ok = false; break; }
                    B[i] = int64_t(q);
                }
                if (!ok) { *range_err = true; continue; }
                keys.push_back(pack(B[0], B[1], B[2]));
            }
        }
    }
    std::sort(keys.begin(), keys.end());
    keys.erase(std::unique(keys.begin(), keys.end()), keys.end());
    return keys;
}

// Running weighted average of one block against one frame (weight 1 per observation,
// weight saturating at 255, TSDF in metres clamped above at mu, integer colour mean
// with round-half-up).  Decisions in float32, values in float64.
void integrate_block(Blk &b, uint64_t key, const orc_params &p, const float *depth,
                     const uint8_t *rgb, const float *P) {
    int32_t Bk[3];
    unpack(key, Bk);
    for (int l = 0; l < 512; ++l) {
        const int64_t g[3] = {int64_t(Bk[0]) * 8 + (l & 7), int64_t(Bk[1]) * 8 + ((l >> 3) & 7),
                              int64_t(Bk[2]) * 8 + (l >> 6)};
        float dl[3];
        for (int i = 0; i < 3; ++i) dl[i] = float(g[i]) * p.voxel_size - P[i * 4 + 3];
        float pc[3];
        for (int j = 0; j < 3; ++j) pc[j] = (P[0 * 4 + j] * dl[0] + P[1 * 4 + j] * dl[1]) + P[2 * 4 + j] * dl[2];
        if (!(pc[2] > 0.0f)) continue;
        const float fu = std::floor((p.fx * (pc[0] / pc[2]) + p.cx) + 0.5f);
        const float fv = std::floor((p.fy * (pc[1] / pc[2]) + p.cy) + 0.5f);
        if (!(fu >= 0.0f && fu < float(p.width) && fv >= 0.0f && fv < float(p.height))) continue;
        const int64_t pix = int64_t(fv) * p.width + int64_t(fu);
        const float d = depth[pix];
        if (!depth_valid(d, p)) continue;
        const float sdf32 = d - pc[2];
        if (sdf32 < -p.trunc) continue;
        // value path in float64 from the same float32 inputs
        double dl64[3];
        for (int i = 0; i < 3; ++i) dl64[i] = double(g[i]) * double(p.voxel_size) - double(P[i * 4 + 3]);
        const double z64 = double(P[0 * 4 + 2]) * dl64[0] + double(P[1 * 4 + 2]) * dl64[1] + double(P[2 * 4 + 2]) * dl64[2];
        const double tsdf = std::min(double(d) - z64, double(p.trunc));
        const int w_old = b.W[l];
        const int n = w_old + 1;
        b.F[l] = (double(w_old) * b.F[l] + tsdf) / double(n);
        b.W[l] = uint8_t(std::min(n, 255));
        if (rgb) {
            for (int c = 0; c < 3; ++c) {
                const int obs = rgb[pix * 3 + c];
                b.C[l * 3 + c] = uint8_t((w_old * int(b.C[l * 3 + c]) + obs + n / 2) / n);
            }
        }
    }
}

// MC voxel of local voxel l of block `key`: bit k of the case index is set iff corner k
// (Lorensen-Cline numbering) has F < 0; a corner in a missing block or with W = 0 makes
// the index 0.  Indices 0 and 255 produce no triangles and are sent as (0, 0,0,0).
uint32_t mc_voxel(const Scene &S, uint64_t key, int l) {
    int32_t Bk[3];
    unpack(key, Bk);
    const int64_t g[3] = {int64_t(Bk[0]) * 8 + (l & 7), int64_t(Bk[1]) * 8 + ((l >> 3) & 7),
                          int64_t(Bk[2]) * 8 + (l >> 6)};
    uint32_t idx = 0;
    for (int k = 0; k < 8; ++k) {
        const int64_t c[3] = {g[0] + kCorner[k][0], g[1] + kCorner[k][1], g[2] + kCorner[k][2]};
        const int64_t cb[3] = {fdiv8(c[0]), fdiv8(c[1]), fdiv8(c[2])};
        if (!key_in_range(cb[0], cb[1], cb[2])) return 0;
        const Blk *b = S.get(pack(cb[0], cb[1], cb[2]));
        if (!b) return 0;
        const int lc = int(c[0] - 8 * cb[0]) + 8 * int(c[1] - 8 * cb[1]) + 64 * int(c[2] - 8 * cb[2]);
        if (b->W[lc] == 0) return 0;
        if (b->F[lc] < 0.0) idx |= 1u << k;
    }
    if (idx == 0 || idx == 255) return 0;
    // the colour is that of the cell's corner-0 voxel, i.e. of g itself (every corner's
    // block was found above)
    const int kc = 0;
    const int64_t cc[3] = {g[0] + kCorner[kc][0], g[1] + kCorner[kc][1], g[2] + kCorner[kc][2]};
    const int64_t ccb[3] = {fdiv8(cc[0]), fdiv8(cc[1]), fdiv8(cc[2])};
    const Blk *cbk = S.get(pack(ccb[0], ccb[1], ccb[2]));
    const int lcol = int(cc[0] - 8 * ccb[0]) + 8 * int(cc[1] - 8 * ccb[1]) + 64 * int(cc[2] - 8 * ccb[2]);
    return idx | uint32_t(cbk->C[lcol * 3 + 0]) << 8 | uint32_t(cbk->C[lcol * 3 + 1]) << 16 |
           uint32_t(cbk->C[lcol * 3 + 2]) << 24;
}

// MC update of the given blocks plus their seven negative-direction neighbours that
// exist (whole blocks are recomputed), followed by stamps and log entries.
void mc_update(Scene &S, const std::vector<uint64_t> &changed, uint32_t frame) {
    std::vector<uint64_t> upd;
    upd.reserve(changed.size() * 8);
    for (uint64_t key : changed) {
        int32_t B[3];
        unpack(key, B);
        for (int e = 0; e < 8; ++e) {
            const int64_t n[3] = {int64_t(B[0]) - (e & 1), int64_t(B[1]) - ((e >> 1) & 1),
                                  int64_t(B[2]) - ((e >> 2) & 1)};
            if (!key_in_range(n[0], n[1], n[2])) continue;
            const uint64_t nk = pack(n[0], n[1], n[2]);
            if (S.get(nk)) upd.push_back(nk);
        }
    }
    std::sort(upd.begin(), upd.end());
    upd.erase(std::unique(upd.begin(), upd.end()), upd.end());
    std::vector<Blk *> ptr(upd.size());
    for (size_t i = 0; i < upd.size(); ++i) ptr[i] = S.get(upd[i]);
    std::vector<std::array<uint32_t, 512>> fresh(upd.size());
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t i = 0; i < int64_t(upd.size()); ++i)
        for (int l = 0; l < 512; ++l) fresh[size_t(i)][size_t(l)] = mc_voxel(S, upd[size_t(i)], l);
    for (size_t i = 0; i < upd.size(); ++i) {
        std::memcpy(ptr[i]->mc, fresh[i].data(), sizeof(ptr[i]->mc));
        ptr[i]->mc_stamp = frame;
        if (int64_t(S.log.size()) >= S.p.log_capacity) {
            S.error = ORC_EFULL_LOG;
        } else {
            S.log.emplace_back(frame, upd[i]);
        }
    }
    S.last_mc = upd;
}

int64_t write_keys(const std::vector<uint64_t> &v, int32_t *keys, int64_t cap) {
    int64_t n = std::min<int64_t>(cap, int64_t(v.size()));
    if (keys)
        for (int64_t i = 0; i < n; ++i) unpack(v[size_t(i)], keys + 3 * i);
    return int64_t(v.size());
}

}  // namespace

// Client geometry from MC voxels (Sec. 4.3; vertices without interpolation, Sec. 6).
// Cube corners k = 0..7 at kCorner[k]; corner k is inside the surface iff bit k of the
// case index is set (F < 0).  A vertex sits at the midpoint of every cube edge whose two
// corners differ.  On each cube face the crossing points are joined in pairs: two
// crossings by one segment; four (inside corners diagonal) by one segment around each
// inside corner, which neighbouring cells sharing the face decide identically.  The
// segments close into loops; each loop is oriented so that its normal points from the
// inside corners to the outside ones, started at its lowest edge and cut into a fan.
namespace mesh {
const int kEdge[12][2] = {{0, 1}, {1, 2}, {2, 3}, {3, 0}, {4, 5}, {5, 6},
                          {6, 7}, {7, 4}, {0, 4}, {1, 5}, {2, 6}, {3, 7}};
const int kFace[6][4] = {{0, 1, 2, 3}, {4, 5, 6, 7}, {0, 1, 5, 4}, {3, 2, 6, 7}, {0, 3, 7, 4}, {1, 2, 6, 5}};

int edge_of(int a, int b) {
    for (int e = 0; e < 12; ++e)
        if ((kEdge[e][0] == a && kEdge[e][1] == b) || (kEdge[e][0] == b && kEdge[e][1] == a)) return e;
    return -1;
}

// Triangles of one case as edge triples, in output order.
std::vector<std::array<int, 3>> cell(uint32_t idx) {
    auto in = [&](int k) { return ((idx >> k) & 1u) != 0; };
    std::vector<int> nb[12];
    for (const auto &f : kFace) {
        int cross[4], nc = 0;
        for (int i = 0; i < 4; ++i) {
            const int a = f[i], b = f[(i + 1) & 3];
            if (in(a) != in(b)) cross[nc++] = edge_of(a, b);
        }
        if (nc == 2) {
            nb[cross[0]].push_back(cross[1]);
            nb[cross[1]].push_back(cross[0]);
        } else if (nc == 4) {
            for (int i = 0; i < 4; ++i) {
                if (!in(f[i])) continue;
                const int e1 = edge_of(f[(i + 3) & 3], f[i]), e2 = edge_of(f[i], f[(i + 1) & 3]);
                nb[e1].push_back(e2);
                nb[e2].push_back(e1);
            }
        }
    }
    std::vector<std::array<int, 3>> tris;
    bool used[12] = {};
    for (int s = 0; s < 12; ++s) {
        if (nb[s].empty() || used[s]) continue;
        std::vector<int> loop{s};
        used[s] = true;
        int prev = s, cur = std::min(nb[s][0], nb[s][1]);
        while (cur != s) {
            loop.push_back(cur);
            used[cur] = true;
            const int nx = nb[cur][0] == prev ? nb[cur][1] : nb[cur][0];
            prev = cur;
            cur = nx;
        }
        // Newell normal of the midpoints (doubled coordinates) against inside -> outside
        long nrm[3] = {0, 0, 0}, dir[3] = {0, 0, 0};
        const size_t L = loop.size();
        for (size_t i = 0; i < L; ++i) {
            const int ea = loop[i], eb = loop[(i + 1) % L];
            long pa[3], pb[3];
            for (int c = 0; c < 3; ++c) {
                pa[c] = kCorner[kEdge[ea][0]][c] + kCorner[kEdge[ea][1]][c];
                pb[c] = kCorner[kEdge[eb][0]][c] + kCorner[kEdge[eb][1]][c];
            }
            nrm[0] += (pa[1] - pb[1]) * (pa[2] + pb[2]);
            nrm[1] += (pa[2] - pb[2]) * (pa[0] + pb[0]);
            nrm[2] += (pa[0] - pb[0]) * (pa[1] + pb[1]);
            const int inside = in(kEdge[ea][0]) ? kEdge[ea][0] : kEdge[ea][1];
            const int outside = kEdge[ea][0] + kEdge[ea][1] - inside;
            for (int c = 0; c < 3; ++c) dir[c] += kCorner[outside][c] - kCorner[inside][c];
        }
        if (nrm[0] * dir[0] + nrm[1] * dir[1] + nrm[2] * dir[2] < 0) std::reverse(loop.begin(), loop.end());
        std::rotate(loop.begin(), std::min_element(loop.begin(), loop.end()), loop.end());
        for (size_t i = 1; i + 1 < L; ++i) tris.push_back({loop[0], loop[i], loop[i + 1]});
    }
    return tris;
}
}  // namespace mesh

extern "C" {

void *orc_map_new(void) { return new Map(); }
void orc_map_free(void *m) { delete static_cast<Map *>(m); }

int orc_map_apply(void *m, const uint8_t *ops, const int32_t *keys, const int32_t *vals, int64_t n,
                  int32_t *out) {
    Map &M = *static_cast<Map *>(m);
    int rc = ORC_OK;
    for (int64_t i = 0; i < n; ++i) {
        if (ops[i] > 2) { out[i] = -1; rc = ORC_EINVAL; continue; }
        out[i] = map_op(M, ops[i], keys + 3 * i, vals ? vals[i] : 0);
        if (ops[i] != 1 && out[i] < 0) rc = ORC_EINVAL;
    }
    return rc;
}

int orc_map_insert(void *m, const int32_t *keys, const int32_t *vals, int64_t n, int32_t *status) {
    std::vector<uint8_t> ops(size_t(n), 0);
    return orc_map_apply(m, ops.data(), keys, vals, n, status);
}
int orc_map_find(void *m, const int32_t *keys, int64_t n, int32_t *vals_out) {
    std::vector<uint8_t> ops(size_t(n), 1);
    return orc_map_apply(m, ops.data(), keys, nullptr, n, vals_out);
}
int orc_map_erase(void *m, const int32_t *keys, int64_t n, int32_t *status) {
    std::vector<uint8_t> ops(size_t(n), 2);
    return orc_map_apply(m, ops.data(), keys, nullptr, n, status);
}
int64_t orc_map_size(void *m) { return int64_t(static_cast<Map *>(m)->m.size()); }

int64_t orc_map_export(void *m, int32_t *keys, int32_t *vals, int64_t cap) {
    Map &M = *static_cast<Map *>(m);
    std::vector<std::pair<uint64_t, int32_t>> kv(M.m.begin(), M.m.end());
    std::sort(kv.begin(), kv.end());
    int64_t n = std::min<int64_t>(cap, int64_t(kv.size()));
    for (int64_t i = 0; i < n; ++i) {
        unpack(kv[size_t(i)].first, keys + 3 * i);
        vals[i] = kv[size_t(i)].second;
    }
    return int64_t(kv.size());
}

void *orc_scene_new(const orc_params *p) {
    if (!p || p->pool_blocks <= 0 || p->voxel_size <= 0 || p->trunc <= 0 || p->width <= 0 || p->height <= 0)
        return nullptr;
    Scene *S = new Scene();
    S->p = *p;
    S->m_band = int(std::floor(p->trunc / p->voxel_size + 0.5f));
    S->blocks.reserve(size_t(std::min<int64_t>(p->pool_blocks, int64_t(1) << 22)));
    return S;
}
void orc_scene_free(void *s) { delete static_cast<Scene *>(s); }

int orc_integrate_frame(void *s, const float *depth, const uint8_t *rgb, const float *P, uint32_t frame_id) {
    Scene &S = *static_cast<Scene *>(s);
    if (!depth || !P || frame_id == 0 || frame_id <= S.last_frame) return ORC_EINVAL;
    S.last_frame = frame_id;
    bool range_err = false;
    std::vector<uint64_t> touched = band_keys(S, depth, P, &range_err);
    if (range_err) S.error = ORC_EINVAL;
    S.last_new.clear();
    std::vector<uint64_t> with_storage;
    with_storage.reserve(touched.size());
    for (uint64_t k : touched) {
        if (!S.get(k)) {
            if (!S.alloc(k)) continue;
            S.last_new.push_back(k);
        }
        with_storage.push_back(k);
    }
    S.last_touched = with_storage;
    std::vector<Blk *> ptr(with_storage.size());
    for (size_t i = 0; i < with_storage.size(); ++i) ptr[i] = S.get(with_storage[i]);
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t i = 0; i < int64_t(with_storage.size()); ++i)
        integrate_block(*ptr[size_t(i)], with_storage[size_t(i)], S.p, depth, rgb, P);
    mc_update(S, with_storage, frame_id);
    return S.error;
}

int orc_integrate_blocks(void *s, const int32_t *keys, int64_t n, const float *depth, const uint8_t *rgb,
                         const float *P, uint32_t frame_id) {
    Scene &S = *static_cast<Scene *>(s);
    if (n < 0 || (n > 0 && !keys) || !depth || !P || frame_id == 0 || frame_id <= S.last_frame) return ORC_EINVAL;
    S.last_frame = frame_id;
    // the listed blocks replace the band blocks as the touched set
    std::vector<uint64_t> touched;
    for (int64_t i = 0; i < n; ++i) {
        const int32_t *k = keys + 3 * i;
        if (!key_in_range(k[0], k[1], k[2])) {
            S.error = ORC_EINVAL;
            continue;
        }
        touched.push_back(pack(k[0], k[1], k[2]));
    }
    std::sort(touched.begin(), touched.end());
    touched.erase(std::unique(touched.begin(), touched.end()), touched.end());
    S.last_new.clear();
    std::vector<uint64_t> with_storage;
    for (uint64_t k : touched) {
        if (!S.get(k)) {
            if (!S.alloc(k)) continue;
            S.last_new.push_back(k);
        }
        with_storage.push_back(k);
    }
    S.last_touched = with_storage;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t i = 0; i < int64_t(with_storage.size()); ++i)
        integrate_block(*S.get(with_storage[size_t(i)]), with_storage[size_t(i)], S.p, depth, rgb, P);
    mc_update(S, with_storage, frame_id);
    return S.error;
}

int64_t orc_last_touched(void *s, int32_t *keys, int64_t cap) {
    return write_keys(static_cast<Scene *>(s)->last_touched, keys, cap);
}
int64_t orc_last_new(void *s, int32_t *keys, int64_t cap) {
    return write_keys(static_cast<Scene *>(s)->last_new, keys, cap);
}
int64_t orc_last_mc_updated(void *s, int32_t *keys, int64_t cap) {
    return write_keys(static_cast<Scene *>(s)->last_mc, keys, cap);
}
int64_t orc_n_blocks(void *s) { return int64_t(static_cast<Scene *>(s)->blocks.size()); }

int64_t orc_export_blocks(void *s, int32_t *keys, int64_t cap) {
    std::vector<uint64_t> k = static_cast<Scene *>(s)->block_key;
    std::sort(k.begin(), k.end());
    return write_keys(k, keys, cap);
}

int orc_read_blocks(void *s, const int32_t *keys, int64_t n, double *F, uint8_t *W, uint8_t *rgb, int32_t *found) {
    Scene &S = *static_cast<Scene *>(s);
    for (int64_t i = 0; i < n; ++i) {
        const int32_t *k = keys + 3 * i;
        const Blk *b = key_in_range(k[0], k[1], k[2]) ? S.get(pack(k[0], k[1], k[2])) : nullptr;
        if (found) found[i] = b ? 1 : 0;
        for (int l = 0; l < 512; ++l) {
            if (F) F[i * 512 + l] = b ? b->F[l] : 0.0;
            if (W) W[i * 512 + l] = b ? b->W[l] : 0;
            if (rgb)
                for (int c = 0; c < 3; ++c) rgb[(i * 512 + l) * 3 + c] = b ? b->C[l * 3 + c] : 0;
        }
    }
    return ORC_OK;
}

int orc_write_blocks(void *s, const int32_t *keys, int64_t n, const float *F, const uint8_t *W, const uint8_t *rgb,
                     uint32_t frame_id) {
    Scene &S = *static_cast<Scene *>(s);
    if (frame_id == 0 || frame_id <= S.last_frame) return ORC_EINVAL;
    S.last_frame = frame_id;
    std::vector<uint64_t> changed;
    for (int64_t i = 0; i < n; ++i) {
        const int32_t *k = keys + 3 * i;
        if (!key_in_range(k[0], k[1], k[2])) { S.error = ORC_EINVAL; continue; }
        const uint64_t key = pack(k[0], k[1], k[2]);
        Blk *b = S.get(key);
        if (!b) b = S.alloc(key);
        if (!b) continue;
        for (int l = 0; l < 512; ++l) {
            b->F[l] = double(F[i * 512 + l]);
            b->W[l] = W[i * 512 + l];
            for (int c = 0; c < 3; ++c) b->C[l * 3 + c] = rgb ? rgb[(i * 512 + l) * 3 + c] : 0;
        }
        changed.push_back(key);
    }
    std::sort(changed.begin(), changed.end());
    changed.erase(std::unique(changed.begin(), changed.end()), changed.end());
    S.last_touched = changed;
    S.last_new.clear();
    mc_update(S, changed, frame_id);
    return S.error;
}

// Scene reset (Sec. 4.1, quasi-static scenes): each listed block that exists loses its
// reconstruction - distance, weight and colour of all its voxels become zero, so it reads
// as never observed - and the MC voxels of the reset blocks and of their seven negative
// neighbours are recomputed and logged as update frame_id, which is how the change
// reaches the clients.  Absent keys are skipped; no block is allocated.
int orc_reset_blocks(void *s, const int32_t *keys, int64_t n, uint32_t frame_id, int64_t *n_reset) {
    Scene &S = *static_cast<Scene *>(s);
    if (frame_id == 0 || frame_id <= S.last_frame) return ORC_EINVAL;
    S.last_frame = frame_id;
    std::vector<uint64_t> changed;
    for (int64_t i = 0; i < n; ++i) {
        const int32_t *k = keys + 3 * i;
        if (!key_in_range(k[0], k[1], k[2])) { S.error = ORC_EINVAL; continue; }
        const uint64_t key = pack(k[0], k[1], k[2]);
        Blk *b = S.get(key);
        if (!b) continue;
        for (int l = 0; l < 512; ++l) b->F[l] = 0.0;
        std::memset(b->W, 0, sizeof(b->W));
        std::memset(b->C, 0, sizeof(b->C));
        changed.push_back(key);
    }
    std::sort(changed.begin(), changed.end());
    changed.erase(std::unique(changed.begin(), changed.end()), changed.end());
    if (n_reset) *n_reset = int64_t(changed.size());
    S.last_touched = changed;
    S.last_new.clear();
    mc_update(S, changed, frame_id);
    return S.error;
}

// Blocks currently visible from camera pose P (row-major camera-to-world [R|t]) under the
// scene's intrinsics and depth range: a block counts when its central voxel, local
// (4, 4, 4), projects to a pixel inside the image at a camera depth that is a valid depth
// measurement.  The projection takes the float32 steps of integration.  Keys in ascending
// packed order; returns the count.
int64_t orc_visible_blocks(void *s, const float *P, int32_t *keys, int64_t cap) {
    const Scene &S = *static_cast<const Scene *>(s);
    const orc_params &p = S.p;
    std::vector<uint64_t> vis;
    for (uint64_t key : S.block_key) {
        int32_t Bk[3];
        unpack(key, Bk);
        float dl[3];
        for (int i = 0; i < 3; ++i) dl[i] = float(int64_t(Bk[i]) * 8 + 4) * p.voxel_size - P[i * 4 + 3];
        float pc[3];
        for (int j = 0; j < 3; ++j) pc[j] = (P[0 * 4 + j] * dl[0] + P[1 * 4 + j] * dl[1]) + P[2 * 4 + j] * dl[2];
        if (!(pc[2] > 0.0f) || !depth_valid(pc[2], p)) continue;
        const float fu = std::floor((p.fx * (pc[0] / pc[2]) + p.cx) + 0.5f);
        const float fv = std::floor((p.fy * (pc[1] / pc[2]) + p.cy) + 0.5f);
        if (fu >= 0.0f && fu < float(p.width) && fv >= 0.0f && fv < float(p.height)) vis.push_back(key);
    }
    std::sort(vis.begin(), vis.end());
    return write_keys(vis, keys, cap);
}

int64_t orc_mc_triangles(const int32_t *keys, const uint32_t *mcv, int64_t n, float voxel_size, float *pos,
                         uint8_t *rgb, int64_t cap) {
    int64_t m = 0;
    const float half = 0.5f * voxel_size;
    for (int64_t b = 0; b < n; ++b) {
        for (int l = 0; l < 512; ++l) {
            const uint32_t v = mcv[b * 512 + l];
            const uint32_t idx = v & 0xFFu;
            if (idx == 0 || idx == 255) continue;
            const int64_t g[3] = {int64_t(keys[3 * b]) * 8 + (l & 7), int64_t(keys[3 * b + 1]) * 8 + ((l >> 3) & 7),
                                  int64_t(keys[3 * b + 2]) * 8 + (l >> 6)};
            for (const auto &t : mesh::cell(idx)) {
                if (m < cap) {
                    for (int k = 0; k < 3; ++k) {
                        const int e = t[size_t(k)];
                        for (int c = 0; c < 3; ++c) {
                            const int64_t h = 2 * g[c] + (kCorner[mesh::kEdge[e][0]][c] + kCorner[mesh::kEdge[e][1]][c]);
                            pos[(m * 3 + k) * 3 + c] = float(h) * half;
                        }
                    }
                    if (rgb)
                        for (int c = 0; c < 3; ++c) rgb[m * 3 + c] = uint8_t(v >> (8 * (c + 1)));
                }
                ++m;
            }
        }
    }
    return m;
}

int orc_extract_mc(void *s, const int32_t *keys, int64_t n, uint8_t *mc, uint8_t *rgb) {
    Scene &S = *static_cast<Scene *>(s);
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t i = 0; i < n; ++i) {
        const int32_t *k = keys + 3 * i;
        const bool ok = key_in_range(k[0], k[1], k[2]) && S.get(pack(k[0], k[1], k[2]));
        for (int l = 0; l < 512; ++l) {
            const uint32_t v = ok ? mc_voxel(S, pack(k[0], k[1], k[2]), l) : 0u;
            mc[i * 512 + l] = uint8_t(v & 0xFF);
            if (rgb)
                for (int c = 0; c < 3; ++c) rgb[(i * 512 + l) * 3 + c] = uint8_t(v >> (8 * (c + 1)));
        }
    }
    return ORC_OK;
}

int orc_stored_mc(void *s, const int32_t *keys, int64_t n, uint8_t *mc, uint8_t *rgb) {
    Scene &S = *static_cast<Scene *>(s);
    for (int64_t i = 0; i < n; ++i) {
        const int32_t *k = keys + 3 * i;
        const Blk *b = key_in_range(k[0], k[1], k[2]) ? S.get(pack(k[0], k[1], k[2])) : nullptr;
        for (int l = 0; l < 512; ++l) {
            const uint32_t v = b ? b->mc[l] : 0u;
            mc[i * 512 + l] = uint8_t(v & 0xFF);
            if (rgb)
                for (int c = 0; c < 3; ++c) rgb[(i * 512 + l) * 3 + c] = uint8_t(v >> (8 * (c + 1)));
        }
    }
    return ORC_OK;
}

int64_t orc_updated_since(void *s, uint64_t cursor, int64_t cap, int32_t *keys, uint64_t *next_cursor) {
    Scene &S = *static_cast<Scene *>(s);
    int64_t cnt = 0;
    uint64_t pos = cursor;
    for (; pos < S.log.size() && cnt < cap; ++pos) {
        const auto &e = S.log[size_t(pos)];
        const Blk *b = S.get(e.second);
        if (b && b->mc_stamp == e.first) {  // live: the block's latest MC update
            if (keys) unpack(e.second, keys + 3 * cnt);
            ++cnt;
        }
    }
    if (next_cursor) *next_cursor = (cnt < cap) ? uint64_t(S.log.size()) : pos;
    return cnt;
}

uint64_t orc_log_length(void *s) { return uint64_t(static_cast<Scene *>(s)->log.size()); }
int orc_scene_error(void *s) { return static_cast<Scene *>(s)->error; }

}  // extern "C"

// ------------------------------------------------ per-client stream sets (Sec. 4.2)
// One set per client of the blocks whose newest MC update it has not been sent yet, with
// that update's frame id.  Updates enter every set; requests take the oldest updates
// first.
namespace {
struct Streams {
    const Scene *S;
    size_t seen = 0;  // update-log entries absorbed so far
    std::vector<std::unordered_map<uint64_t, uint32_t>> set;  // per client: block -> frame

    void fill_all(int32_t c) {
        auto &m = set[size_t(c)];
        m.clear();
        for (size_t i = 0; i < S->blocks.size(); ++i) m[S->block_key[i]] = S->blocks[i].mc_stamp;
    }
    // the client's set ordered by (update frame, packed key)
    std::vector<std::pair<uint32_t, uint64_t>> ordered(int32_t c) const {
        std::vector<std::pair<uint32_t, uint64_t>> v;
        for (const auto &kv : set[size_t(c)]) v.emplace_back(kv.second, kv.first);
        std::sort(v.begin(), v.end());
        return v;
    }
};

bool client_ok(const Streams &T, int32_t c) { return c >= 0 && size_t(c) < T.set.size(); }
}  // namespace

extern "C" {

void *orc_streams_new(void *scene, int32_t n_clients) {
    if (!scene || n_clients <= 0) return nullptr;
    Streams *T = new Streams();
    T->S = static_cast<const Scene *>(scene);
    T->set.resize(size_t(n_clients));
    for (int32_t c = 0; c < n_clients; ++c) T->fill_all(c);
    T->seen = T->S->log.size();
    return T;
}

void orc_streams_free(void *st) { delete static_cast<Streams *>(st); }

int64_t orc_streams_sync(void *st) {
    Streams &T = *static_cast<Streams *>(st);
    const auto &log = T.S->log;
    const int64_t added = int64_t(log.size() - T.seen);
    for (; T.seen < log.size(); ++T.seen) {
        const auto &e = log[T.seen];
        for (auto &m : T.set) m[e.second] = e.first;  // newest update of the block
    }
    return added;
}

int orc_streams_reconnect(void *st, int32_t client) {
    Streams &T = *static_cast<Streams *>(st);
    if (!client_ok(T, client)) return ORC_EINVAL;
    T.fill_all(client);
    return ORC_OK;
}

int64_t orc_streams_pending(void *st, int32_t client, int32_t *keys, uint32_t *frames, int64_t cap) {
    const Streams &T = *static_cast<const Streams *>(st);
    if (!client_ok(T, client)) return ORC_EINVAL;
    const auto v = T.ordered(client);
    const int64_t n = std::min<int64_t>(cap, int64_t(v.size()));
    for (int64_t i = 0; i < n; ++i) {
        if (keys) unpack(v[size_t(i)].second, keys + 3 * i);
        if (frames) frames[i] = v[size_t(i)].first;
    }
    return int64_t(v.size());
}

int64_t orc_streams_serve(void *st, int32_t client, int64_t limit, int32_t *keys) {
    Streams &T = *static_cast<Streams *>(st);
    if (!client_ok(T, client) || limit < 0) return ORC_EINVAL;
    const auto v = T.ordered(client);
    const int64_t n = std::min<int64_t>(limit, int64_t(v.size()));
    for (int64_t i = 0; i < n; ++i) {
        if (keys) unpack(v[size_t(i)].second, keys + 3 * i);
        T.set[size_t(client)].erase(v[size_t(i)].second);
    }
    return n;
}

int orc_streams_take(void *st, int32_t client, int64_t limit, const int32_t *keys, int64_t n) {
    Streams &T = *static_cast<Streams *>(st);
    if (!client_ok(T, client) || limit < 0 || n < 0 || (n > 0 && !keys)) return ORC_EINVAL;
    auto &m = T.set[size_t(client)];
    if (n != std::min<int64_t>(limit, int64_t(m.size()))) return ORC_SERVE_ECOUNT;
    std::vector<uint64_t> sent(static_cast<size_t>(n));
    uint32_t newest = 0;
    for (int64_t i = 0; i < n; ++i) {
        const int32_t *k = keys + 3 * i;
        if (!key_in_range(k[0], k[1], k[2])) return ORC_SERVE_ENOTPENDING;
        sent[size_t(i)] = pack(k[0], k[1], k[2]);
        const auto it = m.find(sent[size_t(i)]);
        if (it == m.end()) return ORC_SERVE_ENOTPENDING;
        newest = std::max(newest, it->second);
    }
    std::vector<uint64_t> uniq = sent;
    std::sort(uniq.begin(), uniq.end());
    if (std::adjacent_find(uniq.begin(), uniq.end()) != uniq.end()) return ORC_SERVE_EDUP;
    // every pending block of an update older than the newest one sent must be sent too
    for (const auto &kv : m)
        if (kv.second < newest && !std::binary_search(uniq.begin(), uniq.end(), kv.first)) return ORC_SERVE_EORDER;
    for (uint64_t k : sent) m.erase(k);
    return ORC_OK;
}

}  // extern "C"
