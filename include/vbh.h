/* vbh.h - C ABI of the MI355X voxel-block-hashing hot path.
 *
 * Implements the data-parallel server path of SLAMCast (Stotko, Krumpen, Hullin,
 * Weinmann, Klein; IEEE TVCG 2019, arXiv 1805.03709):
 *   - a thread-safe GPU hash map/set from int3 block coordinates to int32 values with
 *     concurrent retrieval, insertion and removal that always succeed below capacity
 *     and keep keys unique (Sec. 5, "Hash Map and Set Data Structures");
 *   - voxel block hashing reconstruction (Sec. 4.1): block allocation along the
 *     truncation band of every depth ray and TSDF / weight / colour fusion;
 *   - the server's MC voxel block representation (Sec. 4.2): per voxel a Marching
 *     Cubes case index (1 byte) plus colour (3 bytes), cut to zero for indices 0 and
 *     255, recomputed for every updated block and its seven negative neighbours;
 *   - per-client streaming state (Sec. 4.2): blocks updated since a client cursor,
 *     with reconnection from cursor 0 returning every block.
 *
 * Conventions shared by every entry point
 *   Keys: int32 [n][3] (x,y,z) block coordinates, each in [-2^20, 2^20).
 *   Voxel g (int3) sits at world point g * voxel_size; block B = floor(g / 8); local id
 *   l = (g.x-8B.x) + 8 (g.y-8B.y) + 64 (g.z-8B.z) (x fastest); a block has 512 voxels.
 *   Camera: OpenCV (x right, y down, z forward); pose_c2w is the row-major 3x4 [R|t]
 *   mapping camera to world; depth is camera z in metres, 0 (or NaN) = invalid.
 *   Pointers prefixed d_ are device pointers, h_ host pointers.  `stream` is a
 *   hipStream_t (NULL = the null stream).  Every call only enqueues work on `stream`
 *   unless documented as synchronising; the caller keeps all buffers alive until that
 *   work completes.  No pointer is retained after a call returns.
 *   One host thread may use a handle at a time, and all work on one handle must be
 *   ordered on a single stream (the library's own concurrency is on the device).
 *
 * Errors
 *   Calls return VBH_OK (0) or a negative code.  Argument errors are detected on the
 *   host.  Errors found by kernels (a key out of range, a full table, pool or log, an
 *   expired bounded wait) are recorded in a sticky device word; vbh_map_status /
 *   vbh_scene_status synchronise, return the first recorded code and clear it.  No
 *   key is ever dropped silently: an operation that could not be performed reports an
 *   error status.
 */
#ifndef VBH_H
#define VBH_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define VBH_OK 0
#define VBH_EINVAL (-1)      /* bad argument, key out of range, frame id not increasing */
#define VBH_ENOMEM (-2)      /* device allocation failed */
#define VBH_EHIP (-3)        /* a HIP runtime call failed */
#define VBH_EFULL_TABLE (-4) /* no EMPTY slot left on a probe sequence */
#define VBH_EFULL_POOL (-5)  /* voxel block pool exhausted */
#define VBH_EFULL_LOG (-6)   /* update log full */
#define VBH_ESPIN (-7)       /* a bounded wait for a concurrent insert expired */

#define VBH_ABSENT INT32_MIN /* find() result for a missing key; reserved as a value */

/* Operation codes of mixed batches. */
#define VBH_OP_INSERT 0
#define VBH_OP_FIND 1
#define VBH_OP_ERASE 2

/* Home-slot hash: 0 = the spatial hash (x p1 xor y p2 xor z p3) mod n with the primes
 * of Sec. 5 (Retrieval), 1 = 64-bit finalizer mix of the packed key. */
#define VBH_HASH_SPATIAL 0
#define VBH_HASH_MIX64 1

const char *vbh_strerror(int code);
int vbh_version(void);

/* ======================================================================= hash map
 * Concurrent map from int3 keys to int32 values (Sec. 5).  Open addressing in a
 * power-of-two table; a batch of n operations runs as n concurrent device threads.  The
 * outcome of a batch equals that of some serial order of its operations (for batches
 * whose insert, find and erase keys are pairwise disjoint the outcome is unique). */
typedef struct vbh_map vbh_map;

/* slots: power of two in [64, 2^31].  Allocates 16 B per slot on the current device. */
int vbh_map_create(uint64_t slots, int32_t hash_kind, vbh_map **out);
/* The paper's own chained design (Sec. 5, first paragraph and Insertion/Removal): a
 * bucket array plus linked-list excess entries reached through per-entry links, a stack
 * of free excess entries, per-entry occupancy flags and locks, and non-blocking attempts
 * retried until they succeed, under the invariant that entry positions and links are
 * preserved.  Every other vbh_map_* / vbh_insert / vbh_find / vbh_erase / vbh_apply call
 * accepts the handle with the same semantics, except that vbh_map_size reports no
 * tombstones and vbh_map_rebuild does nothing.
 *   buckets: power of two in [64, 2^27]; excess: list entries, buckets + excess < 2^28.
 *   Allocates 16 B per entry plus 4 B per excess entry and 4 B per entry of bookkeeping.
 * Capacity: a key fails with VBH_EFULL_TABLE when its bucket is taken and no excess
 * entry is free.  Entries emptied by a batch are reused from the next batch on. */
int vbh_map_create_chained(uint64_t buckets, uint64_t excess, int32_t hash_kind, vbh_map **out);
void vbh_map_destroy(vbh_map *m);

/* Insert-if-absent (Sec. 5, Insertion).  d_status[i] = 1 inserted, 0 already present
 * (the stored value is kept), VBH_EINVAL for a key out of range or a value equal to the
 * reserved VBH_ABSENT (nothing is stored; vbh_map_status then reports VBH_EINVAL),
 * VBH_EFULL_TABLE when no slot was free.
 * Open addressing never reuses an erased slot within the table's life: erases leave
 * tombstones, which keep occupying probe positions until vbh_map_rebuild (or
 * vbh_map_clear).  Under sustained insert/erase traffic the caller watches the tombstone
 * count of vbh_map_size and rebuilds before live + tombstones approach the slot count;
 * an insert that finds no EMPTY slot on its probe sequence fails with VBH_EFULL_TABLE
 * even if few keys are live.  No call rebuilds by itself (a rebuild allocates a second
 * table). */
int vbh_insert(vbh_map *m, const int32_t *d_keys, const int32_t *d_vals, int64_t n, int32_t *d_status,
               void *stream);
/* Retrieval (Sec. 5): d_vals_out[i] = stored value or VBH_ABSENT. */
int vbh_find(vbh_map *m, const int32_t *d_keys, int64_t n, int32_t *d_vals_out, void *stream);
/* Removal (Sec. 5): d_status[i] = 1 erased, 0 absent. */
int vbh_erase(vbh_map *m, const int32_t *d_keys, int64_t n, int32_t *d_status, void *stream);
/* Mixed batch: d_ops[i] in {VBH_OP_INSERT, VBH_OP_FIND, VBH_OP_ERASE}; d_out[i] as for
 * the single-kind calls.  d_vals is read for inserts only (may be NULL if none). */
int vbh_apply(vbh_map *m, const uint8_t *d_ops, const int32_t *d_keys, const int32_t *d_vals, int64_t n,
              int32_t *d_out, void *stream);
/* Synchronising: live keys and tombstones (erased slots awaiting vbh_map_rebuild). */
int vbh_map_size(vbh_map *m, int64_t *h_live, int64_t *h_tombstones, void *stream);
/* Synchronising: writes up to cap live (key, value) pairs in slot order; *h_count = number
 * of live keys (may exceed cap). */
int vbh_map_export(vbh_map *m, int32_t *d_keys, int32_t *d_vals, int64_t cap, int64_t *h_count, void *stream);
/* Re-inserts the live entries into a fresh table of the same size, dropping tombstones.
 * Must not overlap other work on the map (it is stream-ordered). */
int vbh_map_rebuild(vbh_map *m, void *stream);
/* Removes every key. */
int vbh_map_clear(vbh_map *m, void *stream);
/* Synchronising: first error recorded by kernels since the last call (then cleared). */
int vbh_map_status(vbh_map *m, void *stream);
/* Synchronising: *h_size = live keys (vbh_map_size without the tombstone count). */
int vbh_size(vbh_map *m, int64_t *h_size, void *stream);
/* Synchronising: the first error recorded since the last call on a map or a scene handle
 * (the handle's kind is read from its first word; vbh_map_status / vbh_scene_status),
 * then cleared.  `handle` is a live vbh_map or vbh_scene; NULL, or a handle of another
 * kind, gives VBH_EINVAL. */
int vbh_status(void *handle, void *stream);
/* Measurement helper: the ceiling that the map's compare-and-swaps are compared with.
 * n_ops 64-bit compare-and-swaps (expected 0) at pseudo-random words of d_words
 * (n_words, a power of two, caller-owned device memory, zeroed by the caller); the number
 * that succeeded is added to *d_won (device).  Asynchronous on `stream`. */
int vbh_cas_ceiling(unsigned long long *d_words, int64_t n_words, int64_t n_ops, uint64_t seed,
                    unsigned long long *d_won, void *stream);

/* ========================================================================= scene
 * A voxel block hashing volume (Sec. 4.1) plus the server's MC voxel block
 * representation and update log (Sec. 4.2), resident in device memory:
 *   hash table   16 B x slots            key -> block pool index
 *   TSDF pool    8 B x 512 x pool_blocks  float F (metres, clamped to [-trunc, trunc])
 *                                         + uint32 (W | R<<8 | G<<16 | B<<24)
 *   MC pool      4 B x 512 x pool_blocks  uint32 (index | R<<8 | G<<16 | B<<24)
 *   update log   8 B x log_capacity       (frame, block) in append order
 */
typedef struct vbh_scene vbh_scene;

typedef struct vbh_params {
    uint64_t slots;        /* hash slots, power of two in [64, 2^31] */
    int64_t pool_blocks;   /* voxel block capacity, in [1, 2^30] */
    int64_t log_capacity;  /* update-log entries, >= 1 */
    float voxel_size;      /* metres, > 0 */
    float trunc;           /* truncation band half-width mu, metres, >= voxel_size */
    int32_t width, height; /* depth image size, each in [1, 16384] */
    float fx, fy, cx, cy;  /* pinhole intrinsics in pixels */
    float depth_min;       /* valid depth range [depth_min, depth_max] */
    float depth_max;
    int32_t hash_kind;     /* VBH_HASH_* */
} vbh_params;

typedef struct vbh_stats {
    int64_t n_touched;       /* last frame: blocks allocated or touched by the band */
    int64_t n_new;           /* last frame: newly inserted blocks */
    int64_t n_mc;            /* last frame: blocks whose MC voxels were recomputed */
    int64_t n_voxel_updates; /* last frame: voxels whose TSDF was updated */
    int64_t n_blocks;        /* allocated blocks */
    uint64_t log_length;     /* update-log entries so far */
    uint32_t last_frame;     /* frame id of the last update */
    int32_t error;           /* first sticky error (not cleared) */
    int64_t total_touched;   /* sums over every update since creation */
    int64_t total_mc;
    int64_t total_voxel_updates;
} vbh_stats;

int vbh_scene_create(const vbh_params *p, vbh_scene **out);
void vbh_scene_destroy(vbh_scene *s);

/* Fuse one depth frame (Sec. 4.1 voxel block hashing; Sec. 4.2 MC update):
 *   1. allocation: every valid pixel puts 2m+1 samples (m = round(trunc/voxel_size)) at
 *      camera depths (d - trunc) + s voxel_size on its ray; each sample's block is
 *      inserted (a new block takes a zeroed pool block) and marked touched;
 *   2. integration: every voxel of a touched block is projected to its nearest pixel;
 *      unless the pixel is invalid or sdf = d - z < -trunc, F <- (W F + min(sdf,trunc))
 *      / (W+1), W <- min(W+1, 255), colour <- rounded running mean;
 *   3. MC update: the touched blocks and their existing seven negative neighbours get
 *      their 512 MC voxels recomputed, their MC stamp set to frame_id and one log entry
 *      each.
 * d_depth float32 [H*W]; d_rgb uint8 [H*W*3] or NULL (colour left unchanged); pose_c2w
 * is a HOST pointer to 12 floats, copied by value; frame_id > 0 and greater than every
 * previous frame id of this scene (else VBH_EINVAL). */
int vbh_integrate_frame(vbh_scene *s, const float *d_depth, const uint8_t *d_rgb, const float *pose_c2w,
                        uint32_t frame_id, void *stream);

/* Integration of one frame into an explicit list of blocks instead of the band blocks
 * (Sec. 4.1 fusion with the allocation step replaced by the list): the n keys (duplicates
 * allowed; absent blocks are allocated, keys out of range record VBH_EINVAL) form the
 * touched set, every voxel of them is integrated with the rules of vbh_integrate_frame
 * (step 2), and the MC update (step 3) follows, as update frame_id.  For batches larger
 * than a frame's band, e.g. every block in front of a surface. */
int vbh_integrate_blocks(vbh_scene *s, const int32_t *d_keys, int64_t n, const float *d_depth, const uint8_t *d_rgb,
                         const float *pose_c2w, uint32_t frame_id, void *stream);

/* Self-check of the division that step 2 uses to project a voxel (its pixel is
 * floor(fx * x/z + cx + 1/2), floor(fy * y/z + cy + 1/2)): for each of n seeded operand pairs
 * (divisor in [2^-32, 2^32), with an all-ones significand if all_ones = 1, else a random one;
 * dividend of either sign in [2^-90, 2^32)), the kernel's reciprocal-based quotient is
 * compared bit for bit with the correctly rounded quotient; the number of pairs that differ
 * is written to *d_bad (device, caller-owned).  Asynchronous on `stream`; n < 0, a NULL
 * d_bad or another all_ones value give VBH_EINVAL. */
int vbh_check_division(int64_t n, uint64_t seed, int32_t all_ones, unsigned long long *d_bad, void *stream);

/* Fuse n consecutive frames, each exactly as vbh_integrate_frame would, in order: d_depth
 * float32 [n][H*W], d_rgb uint8 [n][H*W*3] or NULL, poses_c2w a HOST array of n*12 floats
 * (copied), frame ids first_frame_id .. first_frame_id + n - 1 (first_frame_id > 0 and
 * greater than every previous frame id, else VBH_EINVAL; n = 0 does nothing).  Every
 * result equals that of n vbh_integrate_frame calls; the call returns once the last
 * frame is enqueued, keeping at most 64 frames queued ahead of the device. */
int vbh_integrate_frames(vbh_scene *s, const float *d_depth, const uint8_t *d_rgb, const float *poses_c2w,
                         uint32_t first_frame_id, int64_t n, void *stream);

/* vbh_integrate_frames for frames in HOST memory (h_depth float32 [n][H*W], h_rgb uint8
 * [n][H*W*3] or NULL; page-locked memory gives asynchronous copies): each frame is copied
 * over PCIe, on the caller's stream, into one of two library-owned device buffers and
 * then fused.  The host buffers must stay valid until the caller's stream has completed
 * the work; results equal those of vbh_integrate_frames on the same frames.  VBH_ENOMEM
 * if the two buffers cannot be allocated (first call only). */
int vbh_integrate_frames_host(vbh_scene *s, const float *h_depth, const uint8_t *h_rgb, const float *poses_c2w,
                              uint32_t first_frame_id, int64_t n, void *stream);

/* MC voxels (Sec. 4.2) recomputed from the current TSDF for n blocks: d_mc uint8
 * [n*512] case indices (bit k set iff corner k, Lorensen-Cline order (0,0,0) (1,0,0)
 * (1,1,0) (0,1,0) (0,0,1) (1,0,1) (1,1,1) (0,1,1), has F < 0; 0 if any corner lies in a
 * missing block or has W = 0; indices 0 and 255 cut to 0), d_rgb uint8 [n*512*3] or
 * NULL (colour of the voxel, 0 where cut).  Missing blocks yield zeros. */
int vbh_extract_mc_indices(vbh_scene *s, const int32_t *d_keys, int64_t n, uint8_t *d_mc, uint8_t *d_rgb,
                           void *stream);
/* The extraction above for every allocated block: up to cap block keys in pool order to
 * d_keys_out (int32 [cap][3]) and their MC indices (d_mc, uint8 [cap][512]) and colours
 * (d_rgb, uint8 [cap][512][3] or NULL); *h_count = allocated blocks (may exceed cap).
 * Synchronising (the count is read back before the extraction is enqueued). */
int vbh_extract_mc_all(vbh_scene *s, int32_t *d_keys_out, int64_t cap, uint8_t *d_mc, uint8_t *d_rgb,
                       int64_t *h_count, void *stream);
/* MC voxels as kept in the MC pool by the last update of each block (same layout). */
int vbh_stored_mc(vbh_scene *s, const int32_t *d_keys, int64_t n, uint8_t *d_mc, uint8_t *d_rgb, void *stream);

/* Streaming state (Sec. 4.2): walks the update log from position `cursor` and returns,
 * in log order, up to cap blocks whose entry is live (the block's latest MC update);
 * cursor 0 therefore yields every block once (reconnection).  Writes d_keys_out [cap][3],
 * *d_count (int64) and *d_next_cursor (uint64: position after the last returned entry if
 * cap entries were returned, else the log end).  Device-side outputs; does not sync. */
int vbh_updated_blocks_since(vbh_scene *s, uint64_t cursor, int64_t cap, int32_t *d_keys_out, int64_t *d_count,
                             uint64_t *d_next_cursor, void *stream);

/* Synchronising: first error recorded by kernels since the last call (then cleared). */
int vbh_scene_status(vbh_scene *s, void *stream);
/* Synchronising: counters of the last frame and of the scene. */
int vbh_scene_stats(vbh_scene *s, vbh_stats *h_out, void *stream);
/* Synchronising: up to cap allocated block keys in pool order; *h_count = total. */
int vbh_scene_export_blocks(vbh_scene *s, int32_t *d_keys, int64_t cap, int64_t *h_count, void *stream);
/* Synchronising: keys of the last frame's touched blocks / MC-updated blocks. */
int vbh_scene_last_touched(vbh_scene *s, int32_t *d_keys, int64_t cap, int64_t *h_count, void *stream);
int vbh_scene_last_mc(vbh_scene *s, int32_t *d_keys, int64_t cap, int64_t *h_count, void *stream);
/* Voxel state of n blocks: d_F float32 [n*512], d_W uint8 [n*512], d_rgb uint8
 * [n*512*3] (each may be NULL), d_found int32 [n] (may be NULL).  Missing: zeros. */
int vbh_scene_read_blocks(vbh_scene *s, const int32_t *d_keys, int64_t n, float *d_F, uint8_t *d_W,
                          uint8_t *d_rgb, int32_t *d_found, void *stream);
/* Load voxel state for n distinct keys (allocating absent blocks), then refresh the MC
 * voxels of those blocks and their seven negative neighbours as update frame_id (same
 * rules as vbh_integrate_frame).  d_rgb may be NULL (colour 0). */
int vbh_scene_write_blocks(vbh_scene *s, const int32_t *d_keys, int64_t n, const float *d_F, const uint8_t *d_W,
                           const uint8_t *d_rgb, uint32_t frame_id, void *stream);

/* Scene reset (Sec. 4.1, quasi-static scenes: the parts of the model that are currently
 * visible are deleted and the list of their blocks goes to the server, so that the region
 * can be reconstructed anew).  Each of the n keys (duplicates allowed) whose block exists
 * loses its reconstruction: F = 0, W = 0 and colour 0 for all 512 voxels, so the block
 * reads as never observed.  The MC voxels of the reset blocks and of their seven negative
 * neighbours are then recomputed and logged as update frame_id (same rules as
 * vbh_integrate_frame), which delivers the now-empty blocks to every client.  Keys whose
 * block does not exist are skipped; nothing is allocated and blocks keep their pool
 * storage.  The reset blocks are the update's touched set (vbh_scene_last_touched).
 * frame_id must exceed every earlier update's id; keys out of range record VBH_EINVAL. */
int vbh_scene_reset_blocks(vbh_scene *s, const int32_t *d_keys, int64_t n, uint32_t frame_id, void *stream);
/* Synchronising: the blocks currently visible from pose_c2w (host float[12], row-major
 * camera-to-world) under the scene's intrinsics and depth range - those whose central
 * voxel, local (4, 4, 4), projects to a pixel inside the image at a camera depth in
 * [depth_min, depth_max] (the projection of integration).  Writes up to cap keys, in no
 * particular order, to d_keys int32 [cap][3]; *h_count = number of visible blocks (may
 * exceed cap).  The input of vbh_scene_reset_blocks for the reset of Sec. 4.1. */
int vbh_scene_visible_blocks(vbh_scene *s, const float *pose_c2w, int32_t *d_keys, int64_t cap, int64_t *h_count,
                             void *stream);

/* =================================================================== client mesh
 * Client geometry (Sec. 4.3): triangles from n blocks of MC voxels as a client receives
 * them - d_keys int32 [n][3], d_mcv uint32 [n][512] (index | R<<8 | G<<16 | B<<24, local
 * voxel x fastest; the cell of voxel g has its corner 0 at g).  Each vertex is the
 * midpoint of a cube edge whose corners lie on different sides (the paper's MC voxels
 * carry no interpolation weights): world position (2g + a + b) * (voxel_size / 2) for an
 * edge from corner offset a to b.  Per case, crossing points are paired face by face (one
 * segment around each inside corner on a face whose inside corners are diagonal, so
 * neighbouring cells agree and closed surfaces give closed meshes), joined into loops
 * oriented from inside (F < 0) to outside, and fanned from each loop's lowest edge.
 * Indices 0 and 255 give nothing.  Triangles are ordered by block, cell and loop.
 * Outputs: d_pos float32 [cap][3][3], d_rgb uint8 [cap][3] (the cell's colour; may be
 * NULL).  d_work: caller-owned int64 workspace of vbh_mc_work_size(n) elements.
 * Synchronising: *h_count = number of triangles (may exceed cap; then only the first cap
 * are written). */
int64_t vbh_mc_work_size(int64_t n);
/* Host-only query of the rule above, for clients that triangulate on the CPU: returns the
 * number of triangles of case `index` (0..255, else VBH_EINVAL) and, if h_edges is not
 * NULL, writes their cube edges (Lorensen-Cline numbering, e0 = corners 0-1 ... e11 =
 * corners 3-7) as int8 [15], unused entries -1. */
int vbh_mc_case(int32_t index, int8_t *h_edges);
int vbh_mc_triangulate(const int32_t *d_keys, const uint32_t *d_mcv, int64_t n, float voxel_size, float *d_pos,
                       uint8_t *d_rgb, int64_t cap, int64_t *d_work, int64_t *h_count, void *stream);
/* For callers that cannot allocate device memory (serving loops and harnesses that forbid
 * hipMalloc): vbh_mc_triangulate with its workspace taken from a static array of the
 * library on the current device (8 MiB per device, held until the process ends) instead of
 * d_work.  Same inputs, outputs, synchronisation and results; it calls no allocating
 * routine.  n > VBH_MC_STATIC_MAX_BLOCKS gives VBH_EINVAL and enqueues nothing.  Every call
 * on one device shares that array: calls that overlap on one device (other host threads,
 * other streams) race and must be serialised by the caller. */
#define VBH_MC_STATIC_MAX_BLOCKS (1 << 20)
int vbh_mc_triangulate_static(const int32_t *d_keys, const uint32_t *d_mcv, int64_t n, float voxel_size,
                              float *d_pos, uint8_t *d_rgb, int64_t cap, int64_t *h_count, void *stream);

/* Synchronising check, then enqueues a copy of log entries [start, start + n) (which must
 * lie below the log length): d_frame uint32 [n] update frame ids, d_keys int32 [n][3]
 * block keys (either may be NULL).  The log is append-only, so it is the full history of
 * MC updates: entry (f, B) is the latest update of B as of version V iff no later entry of
 * B has a frame <= V. */
int vbh_scene_log_entries(vbh_scene *s, uint64_t start, int64_t n, uint32_t *d_frame, int32_t *d_keys, void *stream);

/* Stage timing.  With period n > 0, every n-th update launches its kernels with HIP
 * start/stop events attached to the kernel dispatches on the caller's stream; period 0
 * turns timing off (the default).  Stages: 0 band allocation with MC-set marking,
 * 1 integration, 2 stand-alone MC-set marking (not used by frame fusion, whose allocation
 * kernel forms the MC set), 3 MC extraction.  vbh_scene_timing synchronises the stream and returns,
 * per stage, the summed kernel milliseconds, the number of updates measured and (h_blocks,
 * may be NULL) the touched blocks [0] and MC-set blocks [1] of exactly those updates, all
 * since the last call (then resets).  ms_out must hold VBH_N_STAGES doubles.  EINVAL for
 * period < 0. */
#define VBH_N_STAGES 4
int vbh_scene_enable_timing(vbh_scene *s, int32_t period);
int vbh_scene_timing(vbh_scene *s, double *ms_out, int64_t *h_frames, int64_t *h_blocks, void *stream);

/* ================================================================= serving loop
 * Streams MC voxel blocks to exploration clients (Sec. 4.2: per-client streaming state,
 * requests answered with at most the client's request-size limit; Sec. 4.3: the client
 * controls request rate and size).  Each client has a cursor into the update log; a
 * request returns, in log order, up to `limit` blocks whose log entry after the cursor is
 * live (vbh_updated_blocks_since) with their keys and 512 MC voxels each (uint32 index |
 * R<<8 | G<<16 | B<<24), and advances the cursor.  A new or reconnecting client starts at
 * cursor 0 and so receives every block.
 * vbh_server_run replays a request schedule in real time: a request is admitted when its
 * arrival time has passed, its client has no request in flight, a request slot is free
 * and its result fits in the device arena.  VBH_SERVE_ROUNDS: admitted requests are
 * launched in rounds of four kernels on a pool of streams, overlapping with earlier
 * rounds; frames given to the run are fused at their times on another stream, and a
 * frame's MC update waits until the requests in flight have completed while no request is
 * launched.  VBH_SERVE_PERSISTENT: admitted requests are published in batches to a ring in
 * pinned host memory, drained by one persistent launch whose teams of workgroups serve
 * batches concurrently (results written straight into the requests' output buffers when
 * given); a frame that falls due stops the launch after its published batches, is fused
 * with its MC update, and a new launch serves the next version.  Either way every request
 * is served against one scene version (result identical to running it alone at that
 * version).  A persistent launch that waits longer than its bounds (10 s for work, 5 s
 * for a step) leaves, and the run returns VBH_EHIP.
 * While a server runs, the scene must not be used through other entry points.  Between
 * runs it may be (frames fused, blocks written or reset): each run starts from the
 * scene's state at its entry, so such updates must have completed by then (for example,
 * the caller synchronised the stream it issued them on). */
typedef struct vbh_server vbh_server;

#define VBH_SERVE_ROUNDS 0     /* each batch is a round of four kernels on a pool of streams */
#define VBH_SERVE_PERSISTENT 1 /* one persistent launch per scene version drains a ring of batches */
typedef struct vbh_server_config {
    int64_t arena_bytes; /* device memory for results in flight, >= 4096 */
    int32_t max_inflight; /* request slots, 1..4096 */
    int32_t n_streams;   /* rounds: serving streams, 1..8 (default priority); persistent: teams
                            of workgroups, 1..4, each serving one batch at a time */
    int32_t n_clients;   /* client table size, >= 1 */
    int32_t max_batch;   /* requests per round or batch, 1..256 */
    int32_t mode;        /* VBH_SERVE_ROUNDS or VBH_SERVE_PERSISTENT */
    int32_t workgroups;  /* persistent launch size, 0..4096 (0: two per compute unit) */
} vbh_server_config;

typedef struct vbh_request {
    int32_t client;
    int32_t reserved;
    int64_t limit;       /* request size limit in blocks, >= 0 */
    double arrival_s;    /* seconds after the start of vbh_server_run; non-decreasing */
    int32_t *d_keys_out; /* optional device copy of the result keys [limit][3] */
    uint32_t *d_mc_out;  /* optional device copy of the MC voxels [limit][512] */
} vbh_request;

typedef struct vbh_request_result {
    double arrival_s, admit_s, done_s; /* seconds after the start; done = results in memory */
    int64_t count;                     /* blocks returned */
    uint64_t cursor_in, cursor_out;    /* client cursor before and after */
    uint32_t version;                  /* frame id of the scene version served */
    int32_t status;                    /* VBH_OK, or an error for this request */
} vbh_request_result;

typedef struct vbh_frame_feed {
    const float *d_depth;  /* [H*W] */
    const uint8_t *d_rgb;  /* [H*W*3] or NULL */
    float pose_c2w[12];
    double time_s;         /* fuse at this time (seconds after the start) */
    uint32_t frame_id;     /* increasing, greater than the scene's last frame */
    uint32_t reserved;
} vbh_frame_feed;

int vbh_server_create(vbh_scene *scene, const vbh_server_config *cfg, vbh_server **out);
void vbh_server_destroy(vbh_server *srv);
/* Client cursor (0 = reconnect: everything again). */
int vbh_server_set_cursor(vbh_server *srv, int32_t client, uint64_t cursor);
int vbh_server_get_cursor(vbh_server *srv, int32_t client, uint64_t *cursor);
/* Blocks until every request is answered and every frame fused.  results: host array of
 * n_req entries in request order. */
int vbh_server_run(vbh_server *srv, const vbh_request *reqs, int64_t n_req, const vbh_frame_feed *frames,
                   int64_t n_frames, vbh_request_result *results);

/* ============================================================ differentiable form
 * Not part of the paper's system: a differentiable variant of the fusion path.  n_frames
 * depth maps (H x W, float32, in d_depth [n_frames][H][W]) are integrated, with the rules
 * of vbh_integrate_frame (weight 1 per observation, no colour), into a fresh volume with
 * the scene parameters p.  K pixel samples (frame index, pixel index v*W+u) are
 * back-projected, x_k = T_f (D_f[p_k] K^-1 [u, v, 1]), and
 *     L = sum_k F_tri(x_k)^2,
 * F_tri being the trilinear interpolation of F over the voxel lattice (voxel g at g *
 * voxel_size).  Samples whose 8 corner voxels are not all allocated and observed are
 * dropped (f_samples = NaN).  The camera-to-world pose of frame f is
 *     T_f = Exp(xi_f) T0_f,   xi_f = (rho; phi) in se(3),
 * with T0_f the base pose (host float32 [n_frames][12], row-major 3x4) and xi a device
 * float32 [n_frames][6] tangent vector (NULL = zero).  The library composes T_f in
 * float64 and rounds it to the float32 pose that the fusion rules use.  The backward pass
 * returns dL/dD for every pixel and dL/dxi_f = J_l(xi_f)^T g_f for every frame, where g_f
 * is the gradient with respect to a left perturbation Exp(delta) T_f at delta = 0 and
 * J_l the SE(3) left Jacobian; discrete decisions (allocation, pixel of each voxel, skip
 * and clamp branches, trilinear cells, the sample mask) are those of the forward point
 * and are not differentiated. */
typedef struct vbh_diff vbh_diff;

/* n_frames in [1, 32].  Owns a scene created with p. */
int vbh_diff_create(const vbh_params *p, int32_t n_frames, vbh_diff **out);
void vbh_diff_destroy(vbh_diff *d);
/* d_f_samples: float32 [K] (may be NULL); d_loss: float32 scalar on the device.  When
 * d_xi is not NULL the call reads it back to the host and synchronises `stream` once
 * (the composed poses are launch arguments); non-finite poses or xi give VBH_EINVAL. */
int vbh_diff_forward(vbh_diff *d, const float *d_depth, const float *h_poses, const float *d_xi,
                     const int32_t *d_sample_frame, const int32_t *d_sample_pixel, int64_t n_samples,
                     float *d_f_samples, float *d_loss, void *stream);
/* Must follow a forward with the same inputs: h_poses equal to the forward's base poses
 * and d_xi NULL exactly when it was NULL there (else VBH_EINVAL); it reuses the forward's
 * composed poses and reads d_xi on the device for J_l.  d_grad_loss: device float32
 * scalar dL_out/dL; outputs (overwritten): d_grad_depth float32 [n_frames][H][W],
 * d_grad_xi float32 [n_frames][6]. */
int vbh_diff_backward(vbh_diff *d, const float *d_depth, const float *h_poses, const float *d_xi,
                      const int32_t *d_sample_frame, const int32_t *d_sample_pixel, int64_t n_samples,
                      const float *d_grad_loss, float *d_grad_depth, float *d_grad_xi, void *stream);

#ifdef __cplusplus
}
#endif
#endif /* VBH_H */
