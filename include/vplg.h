/*
 * vplg.h -- C ABI of the MI355X (gfx950) library for the hybrid virtual-point-
 * light (VPL) method of "A Virtual Point Light Generation Method in
 * Close-Range Area" (Jin, Wang, Zheng, Hua, Huo).
 *
 * The library renders the indirect part of eq. (1): for every G-buffer pixel
 * y it sums, over all VPLs, the diffuse BRDF times the clamped geometry term
 * times the visibility of the VPL.  The VPLs come from the paper's hybrid
 * generation (Section "Close-Range VPL Sampling"): patch-stratified VPLs with
 * the brightness of eq. (2) on the near faces that the camera frames, plus a
 * sparse quasi-random walk (instant radiosity) whose hits on near faces are
 * discarded.  Scene upload, G-buffer, generation and gather are device work
 * behind this header; callers pass plain pointers.
 *
 * Conventions shared by every call:
 *  - Return value: VPLG_OK (0) or a negative VPLG_E* code.  Nothing throws
 *    across the ABI.  vplg_last_error() gives the calling thread's message of
 *    its last failure.
 *  - Ownership: the library owns scenes and VPL sets (device resident until
 *    released; their bytes count against the context's HBM budget).  The
 *    caller owns G-buffer and radiance buffers (device pointers) and streams.
 *    Host input arrays may be freed when the call returns.
 *  - Asynchrony: device calls only enqueue work on `stream` (a hipStream_t,
 *    NULL = the null stream).  Argument and budget errors return at once;
 *    a device fault surfaces as VPLG_EHIP at a later call that synchronises.
 *  - Threads: a context is not thread-safe; use one per thread or lock.
 *  - Units: world units are arbitrary but consistent; light power is radiant
 *    flux per RGB channel; radiance is RGB float32.
 */
#ifndef VPLG_H
#define VPLG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    VPLG_OK = 0,
    VPLG_EINVAL = -1,    /* bad argument (null pointer, size, unknown kind)     */
    VPLG_ENOMEM = -2,    /* device allocation failed                            */
    VPLG_EBUDGET = -3,   /* request would exceed the context's HBM budget       */
    VPLG_ENOTFOUND = -4, /* unknown scene or VPL-set id                         */
    VPLG_EHIP = -5,      /* HIP runtime error (launch, copy, device fault)      */
    VPLG_EBUSY = -6,     /* object still in use                                 */
    VPLG_ECANCELLED = -7,
    VPLG_ETIMEOUT = -8
};

typedef struct vplg_context vplg_context;

/* Message of the calling thread's most recent failure ("" if none).  The
 * pointer stays valid until the thread's next failing call. */
const char* vplg_last_error(void);

/* ABI version: major * 10000 + minor * 100 + patch. */
int vplg_version(void);

/* Create a context on HIP device `device`.  hbm_budget_bytes caps the device
 * memory that resident scenes and VPL sets may hold (0 = no cap). */
int vplg_context_create(int device, uint64_t hbm_budget_bytes, vplg_context** out);
/* Release every scene and VPL set of the context, then the context. */
int vplg_context_destroy(vplg_context* ctx);
/* Bytes currently held against the budget, and the budget (0 = none). */
int vplg_context_usage(vplg_context* ctx, uint64_t* used_bytes, uint64_t* budget_bytes);

/* ------------------------------------------------------------------------ */
/* Scene upload                                                             */
/* ------------------------------------------------------------------------ */

/* Light of the scene.  kind 0: isotropic point light at pos (the paper's
 * scenes use point lights, Section "Results").  kind 1: one-sided
 * Lambertian parallelogram pos + s edge_u + t edge_v, s,t in [0,1], emitting
 * toward normalize(edge_u x edge_v).  power: radiant flux per RGB channel. */
typedef struct {
    int32_t kind;
    float pos[3];
    float edge_u[3];
    float edge_v[3];
    float power[3];
} vplg_light;

/* Upload a triangle scene and build its ray-casting hierarchy (binned-SAH
 * BVH built on the host, then resident on the device).
 *   tri_xyz    host float32 [n_tris][3][3]: vertices A, B, C.  Faces are
 *              one-sided (Section "Close-Range VPL Sampling"): the front is
 *              the side toward (B - A) x (C - A).
 *   tri_albedo host float32 [n_tris][3]: diffuse RGB albedo.
 *   tri_flags  host uint8 [n_tris]: bit 0 = emitter (never receives VPLs).
 *   light      host pointer, copied.
 * On success *scene_id names the resident scene.  The call synchronises the
 * stream before it returns.  EINVAL: n_tris < 1 or > 2^25, null pointer,
 * non-finite vertex, unknown light kind.  EBUDGET / ENOMEM: no room. */
int vplg_scene_upload(vplg_context* ctx, const float* tri_xyz, const float* tri_albedo, const uint8_t* tri_flags,
                      int32_t n_tris, const vplg_light* light, void* stream, uint64_t* scene_id);
int vplg_scene_release(vplg_context* ctx, uint64_t scene_id);

typedef struct {
    int32_t n_tris, n_nodes, n_leaves, max_depth;
    uint64_t device_bytes;
    float lo[3], hi[3]; /* scene bounding box */
} vplg_scene_info;
int vplg_scene_describe(vplg_context* ctx, uint64_t scene_id, vplg_scene_info* out);

/* ------------------------------------------------------------------------ */
/* G-buffer: the shading points y of eq. (1)                                */
/* ------------------------------------------------------------------------ */

/* Pinhole camera: basis f = normalize(target - eye), r = normalize(f x up),
 * u = r x f; pixel (i, j) (row j = 0 at the top) looks along
 * f + (2(i+1/2)/W - 1) tan(vfov/2) (W/H) r + (1 - 2(j+1/2)/H) tan(vfov/2) u. */
typedef struct {
    float eye[3], target[3], up[3];
    float vfov_deg;
    int32_t width, height;
} vplg_camera;

/* Caller-owned device planes of width * height elements, row-major:
 * world position, unflipped unit face normal, albedo (float32), and the hit
 * triangle (int32, -1 where the pixel ray misses; such pixels render 0). */
typedef struct {
    float* pos[3];
    float* nrm[3];
    float* alb[3];
    int32_t* tri;
    int32_t width, height;
} vplg_gbuffer;

/* Closest hit of one primary ray per pixel centre (float32). */
int vplg_gbuffer_render(vplg_context* ctx, uint64_t scene_id, const vplg_camera* cam, const vplg_gbuffer* gb,
                        void* stream);

/* ------------------------------------------------------------------------ */
/* VPL generation (Section "Close-Range VPL Sampling")                      */
/* ------------------------------------------------------------------------ */

/* k_near     K, the number of patch VPLs (strata of the near-area CDF)
 * n_far      number of far VPLs from the quasi-random walk
 * max_bounces surface hits per walk path, 1 to 3
 * max_paths  cap on walk paths (reaching it sets stats.flags bit 0)
 * d_near     distance threshold of the near region
 * patch_h    faces are refined into patches with edges <= patch_h
 * t_eps      shadow-ray segment trim, as in the gather
 * walk_near  0: the paper's flow step (3), every walk hit on a near patch is
 *            discarded and the path continues; 1 (a variant): only
 *            first-bounce near hits are discarded (the patch VPLs stand for
 *            that light), later near hits become walk VPLs and count toward
 *            n_far; 2 (a variant): a near hit is discarded and ends its path.
 * jitter     0: stratum k's target is its midpoint floor((2k+1) f(N) / 2K);
 *            1: B_k + floor(xi_k (B_{k+1} - B_k)) with the stratum bounds
 *            B_k = floor(k f(N) / K) and xi_k the base-5 radical inverse of
 *            k + 1 (jittered strata).
 * walk_schedule 0: paths run until n_far far VPLs exist, the last path cut
 *            there; 1: Keller's schedule: N = floor(n_far / sum_{j<max_bounces}
 *            rb^j) paths, rb the scene's mean albedo (area-weighted over the
 *            faces that do not emit, mean of the channels); path i goes on to
 *            bounce b only if i <= floor(rb^(b-1) N) and a deposit at bounce b
 *            carries Phi prod(rho) / (N rb^(b-1)); at most n_far far VPLs.
 * brightness 0: a patch VPL's flux is eq. (2) at its own point with the area
 *            f(N) / K it stands for; 1: eq. (2) summed over the set of
 *            patches of its stratum (the passage's "set of triangles"), each
 *            at its centroid with the part of its area inside
 *            [B_k, B_{k+1}), so a patch spanning several strata is shared.
 * Values outside these ranges are EINVAL.                                   */
typedef struct {
    int32_t k_near, n_far, max_bounces, max_paths;
    double d_near, patch_h, t_eps;
    int32_t walk_near, jitter, brightness, walk_schedule;
} vplg_gen_params;

typedef struct {
    int64_t n_patches, n_near, n_eligible;
    int64_t q_total;      /* f(N) in units of patch_h^2 / 2^24 */
    int64_t k_eff;        /* patch VPLs made (0 when no near patch faces the light) */
    int64_t n_far_target; /* n_far plus any unused near budget */
    int64_t n_far, n_paths;
    int64_t far_by_bounce[3];
    int64_t flags;        /* bit 0: max_paths reached */
    int64_t near_discarded;
} vplg_gen_stats;

/* Generate a VPL set for (scene, camera): near/far split of the patches,
 * Morton-ordered fixed-point area CDF cut into k_near strata, one VPL per
 * stratum with the brightness of eq. (2), then the walk.  Every integer
 * decision is taken in FP64.  Device work is enqueued on `stream`; the
 * first generation for a (scene, patch_h) pair synchronises once to size
 * the patch arrays.  The VPL count is known after the stream completes
 * (vplg_vplset_count / vplg_vplset_stats wait for it).  In a scene of at
 * least 1,024 triangles the set also records each VPL's free radius (the
 * distance within which no triangle but the VPL's own and those in its plane
 * lies), which gathers against that same scene use to shorten the shadow
 * rays' VPL ends; gathers against any other scene, and uploaded sets, do
 * without. */
int vplg_vpls_generate(vplg_context* ctx, uint64_t scene_id, const vplg_camera* cam, const vplg_gen_params* p,
                       void* stream, uint64_t* vplset_id);
/* Generate again into an existing generated set (same scene, k_near, n_far
 * and patch_h; camera and the other parameters may change), reusing its
 * device buffers: no allocation and no synchronisation.  Work already queued
 * that reads the set must be on the same stream or finished.  EINVAL if the
 * budget parameters differ from the set's. */
int vplg_vpls_regenerate(vplg_context* ctx, uint64_t vplset_id, const vplg_camera* cam, const vplg_gen_params* p,
                         void* stream);
/* Wait for the set's generation and return its statistics. */
int vplg_vplset_stats(vplg_context* ctx, uint64_t vplset_id, vplg_gen_stats* out);
/* Wait for the set and return its VPL count. */
int vplg_vplset_count(vplg_context* ctx, uint64_t vplset_id, int32_t* n);

/* Upload a VPL set from host arrays: pos, nrm, intensity float32 [n][3]
 * (intensity I_k = flux / pi per channel), host_tri int32 [n] (the triangle a
 * VPL lies on, excluded from its shadow rays; -1 for none). */
int vplg_vpls_upload(vplg_context* ctx, const float* pos, const float* nrm, const float* intensity,
                     const int32_t* host_tri, int32_t n, void* stream, uint64_t* vplset_id);
/* Copy a set to host arrays of capacity `cap` (waits for it).  *n = count;
 * EINVAL if cap < count. Any output pointer may be NULL. */
int vplg_vpls_download(vplg_context* ctx, uint64_t vplset_id, float* pos, float* nrm, float* intensity,
                       int32_t* host_tri, int32_t cap, int32_t* n);

/* Intermediate arrays of a generated set, for verification (waits for it):
 *   0 patch flags   uint8 [n_patches]   bit 0 near, bit 1 eligible
 *   1 sorted        int32 [n_eligible]  eligible patch indices, Morton order
 *   2 keys          uint32 [n_eligible] their Morton keys
 *   3 prefix        int64 [n_eligible]  inclusive fixed-point area prefix f(i)
 *   4 strata        int32 [k_eff]       stratum -> position in `sorted`
 *   5 vpl path      int32 [count]       walk path of each VPL (0 = patch VPL)
 *   6 vpl bounce    int32 [count]       bounce of each VPL (0 = patch VPL)
 *   7 patch offsets int64 [n_tris + 1]  first patch index of each triangle
 * *n_items = element count; EINVAL if cap_bytes is too small. */
int vplg_vplset_debug(vplg_context* ctx, uint64_t vplset_id, int32_t what, void* host_buf, int64_t cap_bytes,
                      int64_t* n_items);
int vplg_vplset_release(vplg_context* ctx, uint64_t vplset_id);

/* ------------------------------------------------------------------------ */
/* Gather: eq. (1) without the direct term                                  */
/* ------------------------------------------------------------------------ */

/* g_clamp: C in min(C, cos_p cos_k / r^2) (> 0).  t_eps: shadow segments
 * x + s (y - x) test s in (t_eps, 1 - t_eps), both host triangles excluded.
 * The tile shape: tile_vpl = waves sharing one 8 x 8 pixel tile, each taking
 * every tile_vpl-th VPL (1, 2, 4, 8 or 16); tile_px = pixels per work item,
 * 64 (8 x 8), 128 (16 x 8) or 256 (16 x 16): a workgroup gathers the item's
 * 8 x 8 tiles side by side, tile_vpl waves each, so tile_px / 64 * tile_vpl
 * must be at most 16.  tile_vpl 0 leaves the shape open: the autotuned
 * choice for the view's shape bucket, else 8 x 8 items with 16 waves per
 * tile for a view of fewer than 32 tiles per compute unit (it shortens the
 * launch's tail) and 8 above; a tile_px given with tile_vpl 0 fixes the
 * pixel block (the waves are halved until it fits).  tile_px 0 = 64, or the
 * tuned block when tile_vpl is 0.  A pixel's value depends on tile_vpl
 * only, never on tile_px. */
typedef struct {
    float g_clamp, t_eps;
    int32_t tile_px, tile_vpl;
} vplg_gather_params;

/* radiance[c][p] = (albedo_p[c] / pi) * sum_k I_k[c] * min(C, max(0, n_p.d)
 * max(0, -n_k.d) / |d|^4) * V(x_p, y_k), d = y_k - x_p, for every pixel of
 * gb; pixels with tri < 0 get 0.  radiance: three caller-owned device planes
 * of width * height float32.  Float32 arithmetic, partial sums added in a
 * fixed order per pixel (deterministic: a pixel's value depends only on its
 * inputs and tile_vpl).
 * The launch is a resident grid whose workgroups claim pixel blocks (one
 * work item of tile_px pixels each) from a counter in work memory that the
 * library keeps for `stream` (about 6 MB, allocated on the stream's first
 * gather, outside the context's budget; the counter is reset by a kernel
 * before each launch).  In a view of at least four rounds of blocks
 * (blocks >= 4 x resident workgroups) the last two rounds are claimed in
 * four parts each, whose sums a second kernel on the stream adds up.  Gathers on one stream are ordered and may share the work memory;
 * gathers on different streams run concurrently.  A gather captured into a
 * HIP graph keeps the work memory of the stream it was captured on: capture
 * on a stream that has already run a gather (the first one allocates that
 * memory, which a capture may refuse), and do not replay the graph
 * concurrently with other gathers on that stream or with another replay. */
int vplg_gather(vplg_context* ctx, uint64_t scene_id, uint64_t vplset_id, const vplg_gbuffer* gb,
                float* const radiance[3], const vplg_gather_params* p, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): vplg_gather
 * with the same arguments, kernels and result, bit for bit, that allocates
 * nothing.  Its work memory (the tile counter and the round-group sums of at
 * most 2,048 split tiles: 6,291,712 bytes) is a fixed device array of the
 * library, one per device, held until the process ends; its address is looked
 * up by vplg_context_create.  The split tail is capped at 2,048 tiles, so no
 * view is too large for the array; the call checks that bound and returns
 * VPLG_EINVAL if a launch would need more.  Every call on one device shares
 * the array and overwrites what the last call left (the counter is reset by a
 * kernel on `stream` before each launch): calls that overlap on one device,
 * from any context, stream or thread, race and give wrong results.  Order
 * them on one stream, or wait for one before starting the next. */
int vplg_gather_noalloc(vplg_context* ctx, uint64_t scene_id, uint64_t vplset_id, const vplg_gbuffer* gb,
                        float* const radiance[3], const vplg_gather_params* p, void* stream);

/* The same kernel, instrumented: also adds to counters[0..13] (device
 * uint64) the pairs evaluated, shadow rays cast, BVH node visits of each
 * ray's own traversal (inner nodes whose box its own segment entered, two
 * child slab tests each) and its ray-triangle tests (triangles of leaves its
 * own segment entered); then, per wave, packets traced, packet node steps,
 * active lanes at packet start and packet triangle steps; then node steps
 * ridden by unblocked lanes (own or not), packet steps entering both
 * children, packet steps entering neither, packets with every ray blocked,
 * packets with no ray blocked, and shadow rays blocked.  The radiance is the
 * plain gather's.  For measurement; slower than vplg_gather. */
int vplg_gather_counted(vplg_context* ctx, uint64_t scene_id, uint64_t vplset_id, const vplg_gbuffer* gb,
                        float* const radiance[3], const vplg_gather_params* p, uint64_t* counters, void* stream);

/* Visibility bits of the listed pixels against every VPL, computed for all
 * pairs (no geometry-term culling), with the gather's own shadow-ray code.
 * pixels: device int32 [n_px] pixel indices; vis_bits: device uint32
 * [n_px][ceil(M / 32)], bit k % 32 of word k / 32 = V(x_p, y_k). */
int vplg_gather_visibility_dump(vplg_context* ctx, uint64_t scene_id, uint64_t vplset_id, const vplg_gbuffer* gb,
                                const int32_t* pixels, int32_t n_px, uint32_t* vis_bits,
                                const vplg_gather_params* p, void* stream);

/* Direct term L_e(y) of eq. (1), the direct illumination of each G-buffer
 * point by the scene's light with the light model of eq. (2):
 *   radiance[c][p] = (albedo_p[c] / pi) * power[c] * G_p,
 *   point light: G_p = V(x_p, pos) max(0, n_p.w) / (4 pi |w|^3), w = pos - x_p;
 *   quad light:  G_p = (1/16) sum over the 16 cell centres y_j =
 *                pos + edge_u (i + 1/2)/4 + edge_v (j + 1/2)/4 of
 *                V(x_p, y_j) max(0, n_p.w_j) max(0, -n_l.w_j) / (pi |w_j|^4),
 *                w_j = y_j - x_p, n_l = unit(edge_u x edge_v), the emitting side.
 * Shadow segments x + s w, s in (t_eps, 1 - t_eps), skip the pixel's own
 * triangle; the light's triangles (if any) occlude like any other.  Pixels
 * with tri < 0 get 0; emitters seen directly get no emission term.  The
 * three caller-owned device planes are overwritten.  FP32 arithmetic, samples
 * summed in order (deterministic).  EINVAL: null pointers, bad G-buffer,
 * t_eps outside [0, 0.5).  ENOTFOUND: unknown scene. */
int vplg_direct(vplg_context* ctx, uint64_t scene_id, const vplg_gbuffer* gb, float* const radiance[3], float t_eps,
                void* stream);

/* ------------------------------------------------------------------------ */
/* Batched gather and tile autotuning                                       */
/* ------------------------------------------------------------------------ */

/* One view of a batch: a resident scene and VPL set, its G-buffer, its
 * radiance planes and gather parameters (params.tile_vpl 0 = the shape
 * vplg_autotune_batch chose for the view's shape bucket, else 8 waves per
 * 8 x 8 tile: a batch shares one tail, so the tile-count rule of a lone
 * gather does not apply). */
typedef struct {
    uint64_t scene_id, vplset_id;
    vplg_gbuffer gb;
    float* radiance[3];
    vplg_gather_params params;
} vplg_view;

/* Gather n_views views of any scenes, resolutions and VPL counts in one
 * persistent launch (at most 4096 views).  Workgroups pull (view, pixel
 * blocks) items from a device counter, most expensive views first.  The launch is a
 * HIP graph captured once per context and replayed; each call only rewrites
 * the device work table (copied from pinned host staging on `stream`) before
 * the replay.  Every view's radiance is identical to vplg_gather's with the
 * same resolved tile_vpl, whatever else is in the batch.  A batch that holds
 * a view whose pixel block takes more than 8 waves (tile_px / 64 * tile_vpl)
 * runs in 16-wave workgroups (a second graph, captured on first use), else
 * in 8-wave ones.  Every call shares the context's work
 * table, so calls are ordered on the device: a call's table copies wait (on
 * `stream`) for the previous call's replay, on whatever stream it ran.  The
 * host thread waits only for the previous call's table copy.  Calls on one
 * context from several host threads must be serialised by the caller. */
int vplg_gather_batch(vplg_context* ctx, const vplg_view* views, int32_t n_views, void* stream);

/* Time vplg_gather on this view in every tile shape (tile_px 64, 128, 256 x
 * tile_vpl 1 .. 16 with tile_px / 64 * tile_vpl <= 16; synchronises
 * `stream`), remember the fastest for the view's shape bucket
 * (ceil(log2(pixels)), ceil(log2(VPL capacity))) and return it.  Later lone
 * gathers with tile_vpl 0 in that bucket use it.  The radiance planes are
 * overwritten. */
int vplg_autotune(vplg_context* ctx, uint64_t scene_id, uint64_t vplset_id, const vplg_gbuffer* gb,
                  float* const radiance[3], const vplg_gather_params* p, void* stream, int32_t* best_tile_vpl,
                  int32_t* best_tile_px);
/* Tune the views of a batch with the batched launch as the objective: the
 * open views (tile_vpl 0 and tile_px 0) are grouped by shape bucket, and for
 * each bucket (most pairs first) its views are gathered as a batch of their
 * own in every tile shape (tile_px / 64 * tile_vpl <= 16), the first run
 * untimed; the fastest shape per bucket is kept for views in batches.  Then
 * the whole batch is timed (twice each) untuned and tuned, and the tuned
 * shapes stay only if the batch runs faster with them (*n_tuned = buckets
 * kept, else 0 and those buckets are left untuned).  Synchronises `stream`;
 * overwrites the views' radiance planes. */
int vplg_autotune_batch(vplg_context* ctx, const vplg_view* views, int32_t n_views, void* stream, int32_t* n_tuned);
/* The tile shape a gather of this shape uses with tile_vpl 0: lone
 * (batched 0) or inside a batch (batched 1); the defaults of
 * vplg_gather_params and vplg_view if untuned. */
int vplg_autotune_lookup(vplg_context* ctx, int32_t width, int32_t height, int32_t n_vpls, int32_t batched,
                         int32_t* tile_vpl, int32_t* tile_px);
/* Save / merge the autotuned tables as text ("vplg-autotune 2", then lines
 * "batched log2_pixels log2_vpls tile_vpl tile_px").  load: ENOTFOUND if the
 * file is absent, EINVAL for another format or a bad entry. */
int vplg_autotune_save(vplg_context* ctx, const char* path);
int vplg_autotune_load(vplg_context* ctx, const char* path);

/* ------------------------------------------------------------------------ */
/* Render server: continuous admission under an HBM budget                  */
/* ------------------------------------------------------------------------ */

typedef struct vplg_server vplg_server;

/* hbm_budget_bytes: device memory the server may hold for per-request
 * G-buffers and VPL sets (pooled; > 0).  max_inflight: requests admitted at
 * once (1..256).  n_streams: HIP streams the admitted requests are spread
 * over (1..16, default priority).  The server's gathers claim whole tiles
 * only (requests overlap, so no one view's tail idles the device); their
 * radiance is the same as vplg_gather's. */
typedef struct {
    uint64_t hbm_budget_bytes;
    int32_t max_inflight, n_streams;
} vplg_server_params;

/* One render: the resident scene, the camera (its width x height is the
 * image), generation and gather parameters, and the caller-owned device
 * radiance planes (width * height float32 each) the result is written to. */
typedef struct {
    uint64_t scene_id;
    vplg_camera camera;
    vplg_gen_params gen;
    vplg_gather_params gather;
    float* radiance[3];
} vplg_request;

enum { VPLG_REQ_QUEUED = 0, VPLG_REQ_RUNNING = 1, VPLG_REQ_DONE = 2, VPLG_REQ_FAILED = 3, VPLG_REQ_CANCELLED = 4 };

/* State of a request and its host steady-clock times (ns): submitted,
 * admitted (its work enqueued), done (completion observed). */
typedef struct {
    int32_t state, error;
    int64_t submit_ns, admit_ns, done_ns;
} vplg_timing;

typedef struct {
    int64_t submitted, admitted, completed, failed, cancelled, queued, running, peak_running;
    uint64_t pool_bytes, peak_bytes;
} vplg_server_stats;

/* Start the server thread.  While a server runs, the context's scenes must
 * not be released; other calls on the context stay allowed. */
int vplg_server_start(vplg_context* ctx, const vplg_server_params* p, vplg_server** out);
/* Queue a request (thread-safe).  Returns at once with a ticket.  EBUDGET if
 * the request alone exceeds the server budget; EINVAL / ENOTFOUND for bad
 * arguments.  The first request on a (scene, patch_h) pair synchronises once
 * to build the scene's patch index. */
int vplg_server_submit(vplg_server* s, const vplg_request* r, uint64_t* ticket);
/* Current state and times of a ticket (thread-safe, non-blocking). */
int vplg_server_poll(vplg_server* s, uint64_t ticket, vplg_timing* t);
/* Block until the ticket is done, failed or cancelled (timeout_ms < 0: no
 * limit; ETIMEOUT otherwise).  VPLG_OK only if it is done. */
int vplg_server_wait(vplg_server* s, uint64_t ticket, int64_t timeout_ms, vplg_timing* t);
/* Cancel a queued request; EBUSY once it has been admitted. */
int vplg_server_cancel(vplg_server* s, uint64_t ticket);
int vplg_server_query(vplg_server* s, vplg_server_stats* out);
/* Cancel queued requests, let admitted ones finish, free the pool, join. */
int vplg_server_stop(vplg_server* s);

#ifdef __cplusplus
}
#endif

#endif /* VPLG_H */
