/* CPU oracle for the voxel-block-hashing hot path of SLAMCast (Stotko et al., TVCG 2019).
 *
 * TEST INFRASTRUCTURE ONLY.  This library is the plain, slow, obviously-correct
 * reference that the HIP path is checked against.  Only the test-suite, the smoke
 * check and the benchmark's CPU-baseline leg may load it; the product path never
 * calls it.  It shares no code, header or table with the HIP path.
 *
 * All pointers are host pointers.  Keys are int32 triples (x,y,z) of block
 * coordinates with each component in [-2^20, 2^20).  Functions return 0 on success or
 * a negative ORC_E* code.
 */
#ifndef VBH_ORACLE_H
#define VBH_ORACLE_H
#include <stdint.h>
#ifdef __cplusplus
extern "C" {
#endif

#define ORC_OK 0
#define ORC_EINVAL (-1)
#define ORC_EFULL_POOL (-5)
#define ORC_EFULL_LOG (-6)
#define ORC_ABSENT INT32_MIN

/* ---- Hash map / set semantics (Sec. 5: retrieval, insertion, removal) ----
 * A std::unordered_map; a batch is applied serially in index order. */
void *orc_map_new(void);
void orc_map_free(void *m);
/* status[i] = 1 inserted, 0 already present (value not overwritten), -1 bad key */
int orc_map_insert(void *m, const int32_t *keys, const int32_t *vals, int64_t n, int32_t *status);
/* vals_out[i] = stored value or ORC_ABSENT */
int orc_map_find(void *m, const int32_t *keys, int64_t n, int32_t *vals_out);
/* status[i] = 1 erased, 0 absent */
int orc_map_erase(void *m, const int32_t *keys, int64_t n, int32_t *status);
/* ops: 0 insert, 1 find, 2 erase; out as for the single-kind calls */
int orc_map_apply(void *m, const uint8_t *ops, const int32_t *keys, const int32_t *vals,
                  int64_t n, int32_t *out);
int64_t orc_map_size(void *m);
/* Writes up to cap (key, value) pairs in ascending packed-key order; returns count. */
int64_t orc_map_export(void *m, int32_t *keys, int32_t *vals, int64_t cap);

/* ---- Scene: allocation, integration, MC index extraction, update log ---- */
typedef struct orc_params {
    int64_t pool_blocks;   /* block capacity */
    int64_t log_capacity;  /* update-log entries */
    float voxel_size;      /* metres */
    float trunc;           /* truncation mu, metres */
    int32_t width, height;
    float fx, fy, cx, cy;
    float depth_min, depth_max;
} orc_params;

void *orc_scene_new(const orc_params *p);
void orc_scene_free(void *s);
/* Fuse one frame: allocation along the truncation band, TSDF/weight/colour update of the
 * touched blocks, MC update of touched blocks and their seven negative neighbours, stamps
 * and log.  depth float32 [H*W] (camera z, metres, 0 = invalid); rgb uint8 [H*W*3] or
 * NULL; pose_c2w float32 row-major 3x4; frame_id strictly increasing and > 0. */
int orc_integrate_frame(void *s, const float *depth, const uint8_t *rgb, const float *pose_c2w,
                        uint32_t frame_id);
/* The same fusion with the allocation step replaced by a list of n block keys
 * (duplicates allowed; absent blocks are allocated; keys out of range record ORC_EINVAL):
 * the listed blocks are the touched set, integrated and MC-updated as update frame_id. */
int orc_integrate_blocks(void *s, const int32_t *keys, int64_t n, const float *depth, const uint8_t *rgb,
                         const float *pose_c2w, uint32_t frame_id);
/* Keys of the last frame's touched / newly allocated / MC-updated blocks (sorted). */
int64_t orc_last_touched(void *s, int32_t *keys, int64_t cap);
int64_t orc_last_new(void *s, int32_t *keys, int64_t cap);
int64_t orc_last_mc_updated(void *s, int32_t *keys, int64_t cap);
int64_t orc_n_blocks(void *s);
int64_t orc_export_blocks(void *s, int32_t *keys, int64_t cap);
/* Voxel state of the given blocks: F float64 [n*512], W [n*512], rgb [n*512*3];
 * found[i] = 0 for absent blocks (their outputs are zero). */
int orc_read_blocks(void *s, const int32_t *keys, int64_t n, double *F, uint8_t *W, uint8_t *rgb,
                    int32_t *found);
/* Load voxel state (allocating absent blocks), then refresh the MC voxels of the loaded
 * blocks and their seven negative neighbours, stamped and logged as frame_id. */
int orc_write_blocks(void *s, const int32_t *keys, int64_t n, const float *F, const uint8_t *W,
                     const uint8_t *rgb, uint32_t frame_id);
/* Scene reset (Sec. 4.1): listed blocks that exist get F = 0, W = 0, colour 0; the MC
 * voxels of those blocks and their seven negative neighbours are recomputed and logged as
 * frame_id.  Absent keys are skipped.  *n_reset (may be NULL) = distinct blocks reset. */
int orc_reset_blocks(void *s, const int32_t *keys, int64_t n, uint32_t frame_id, int64_t *n_reset);
/* Blocks whose central voxel (local 4,4,4) projects into the image at a valid depth under
 * pose P (camera-to-world 3x4); ascending packed-key order, up to cap; returns the count. */
int64_t orc_visible_blocks(void *s, const float *P, int32_t *keys, int64_t cap);
/* Client geometry (Sec. 4.3): triangles of n blocks of MC voxels (keys int32 [n][3], mcv
 * uint32 [n][512] index | RGB << 8), vertices at the midpoints of crossing cube edges.
 * pos float32 [cap][3][3] world positions, rgb uint8 [cap][3] the cell's colour; block,
 * then cell (x fastest), then the cell's loops in order.  Returns the triangle count. */
int64_t orc_mc_triangles(const int32_t *keys, const uint32_t *mcv, int64_t n, float voxel_size, float *pos,
                         uint8_t *rgb, int64_t cap);
/* MC voxels recomputed from the current TSDF: mc [n*512], rgb [n*512*3] (may be NULL). */
int orc_extract_mc(void *s, const int32_t *keys, int64_t n, uint8_t *mc, uint8_t *rgb);
/* MC voxels as stored by the last update of each block (zeros for absent blocks). */
int orc_stored_mc(void *s, const int32_t *keys, int64_t n, uint8_t *mc, uint8_t *rgb);
/* Up to cap live log entries at positions >= cursor, in log order; *next_cursor is the
 * position after the last returned entry (or the log end).  Returns the count. */
int64_t orc_updated_since(void *s, uint64_t cursor, int64_t cap, int32_t *keys, uint64_t *next_cursor);
uint64_t orc_log_length(void *s);
int orc_scene_error(void *s);

/* ---- Serving: per-client stream sets (Sec. 4.2; reconnection Sec. 4.2/4.3) ----
 * Each client has a set of the blocks updated since they were last sent to it.  Every MC
 * update inserts its update set into every client's set (a block already pending keeps
 * one entry, carrying the newest update's frame id).  A request of size limit removes
 * min(limit, |set|) blocks and sends them with their current MC voxels.  The paper takes
 * a random subset; the reading taken here sends the oldest updates first, leaving free only
 * the order among blocks of the same update.  A (re)connecting client's set holds every
 * block of the model.
 * The streams follow a scene's update log: orc_streams_sync absorbs the entries appended
 * since the previous call (the scene must outlive the streams). */
#define ORC_SERVE_ECOUNT (-20)      /* answer size differs from min(limit, |set|) */
#define ORC_SERVE_EDUP (-21)        /* a block sent twice in one answer */
#define ORC_SERVE_ENOTPENDING (-22) /* a block sent that the client's set does not hold */
#define ORC_SERVE_EORDER (-23)      /* an older update left pending while a newer one was sent */
/* Every client starts connected: its set holds every block of the scene. */
void *orc_streams_new(void *scene, int32_t n_clients);
void orc_streams_free(void *st);
/* Absorbs the update-log entries appended since the last sync; returns how many. */
int64_t orc_streams_sync(void *st);
/* The client's set becomes every block of the model (reconnection). */
int orc_streams_reconnect(void *st, int32_t client);
/* The client's set in (update frame, packed key) order, up to cap keys [cap][3] and
 * frames [cap] (either may be NULL); returns its size. */
int64_t orc_streams_pending(void *st, int32_t client, int32_t *keys, uint32_t *frames, int64_t cap);
/* Plain serving: removes and writes the first min(limit, |set|) blocks in (update frame,
 * packed key) order to keys [limit][3]; returns the count. */
int64_t orc_streams_serve(void *st, int32_t client, int64_t limit, int32_t *keys);
/* Checks an answer chosen elsewhere against the rule above: n == min(limit, |set|), no
 * block twice, every block pending, and no pending block of an older update than some
 * sent block left out.  If valid the blocks leave the set and 0 is returned; otherwise the
 * set is unchanged and an ORC_SERVE_E* code is returned. */
int orc_streams_take(void *st, int32_t client, int64_t limit, const int32_t *keys, int64_t n);

/* ---- Differentiable form: frozen-branch FP64 forward and finite differences ----
 * Frames are integrated into a fresh volume (F64), the loss is the sum of squared
 * trilinear F at K back-projected samples.  See oracle/diff.cpp. */
typedef struct orc_diff_problem {
    orc_params p;
    int32_t n_frames;
    const float *depth;      /* [F,H,W] */
    const float *poses;      /* [F,3,4] float32 camera-to-world */
    int64_t n_samples;
    const int32_t *sample_frame;  /* [K] */
    const int32_t *sample_pixel;  /* [K] v*W+u */
    const double *xi_ref;    /* [F,6] or NULL: the reference point is T_f = Exp(xi_ref_f) T0_f */
} orc_diff_problem;

void *orc_diff_new(const orc_diff_problem *prob);
void orc_diff_free(void *d);
/* The poses are T_f = Exp(xi_f) T0_f with T0 the problem's float32 poses.  The reference
 * point is xi = xi_ref (0 if NULL); its poses P32 = Exp(xi_ref) T0 rounded to float32 (the
 * pose input of the fusion) take every discrete decision (band blocks, pixel indices,
 * skips, clamps, trilinear cells, masks) and are where values and gradients are taken.
 * A perturbed pose is Exp(xi) T0' with T0' = Exp(-xi_ref) P32 in float64, the base that
 * maps exactly onto P32 (T0' = T0 when xi_ref is NULL).
 * Loss with depth perturbed by (d_depth, scale) along a full-size direction (may be
 * NULL) at poses Exp(xi_f) T0'_f (xi [F,6] rho;phi; NULL = the reference point), with the
 * branches of the reference point. */
double orc_diff_loss(void *d, const double *d_depth, double scale, const double *xi);
/* Analytic FP64 gradient of the frozen loss at the reference point: grad_depth [F*H*W],
 * grad_xi [F*6] = dL/dxi (the left-perturbation gradient mapped through the transpose of
 * the SE(3) left Jacobian of xi_ref). */
int orc_diff_grad(void *d, double *grad_depth, double *grad_xi);
/* Diagnostics: number of samples kept by the trilinear mask, number of voxels with
 * nonzero dL/dF, forward F at the samples [K] (NaN where masked). */
int64_t orc_diff_info(void *d, int64_t *n_kept, int64_t *n_grad_voxels, double *f_samples);

#ifdef __cplusplus
}
#endif
#endif
