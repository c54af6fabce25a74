/*
 * divas.h -- C ABI of libdivas: depth-weighted voxel aggregation on MI355X.
 *
 * Method: DivAS (arXiv 2601.04860), 2DGS instantiation, thick path.  For every
 * occupied voxel the library projects the voxel centre into each view, tests
 * it against that view's rendered depth, accumulates the refined 2D mask
 * evidence with the depth weight of the paper, applies the consensus
 * threshold, and labels points (Gaussian centres) by voxel lookup.  Options
 * and companions: the thin-structure paths and the NeRF path
 * (divas_params), the scene-statistic grid (divas_grid_from_points), the depth
 * refinement of prompt masks (divas_refine_mask_*) and the needle cull of the
 * voxel-to-surfel mapping (divas_needle_cull).
 *
 * Conventions shared by every entry point
 *   - Grid: a cube of dim^3 voxels (dim a power of two, 2..1024) with min
 *     corner `origin` and edge `voxel`.  A point mu lies in voxel
 *     floor((mu - origin) / voxel) per axis, evaluated in binary64; it is
 *     outside the grid when any axis falls outside [0, dim) or is NaN.
 *     Voxel indices exchanged through this ABI are linear: x + dim*(y + dim*z).
 *   - Cameras: OpenCV pinhole (x right, y down, z forward), intrinsics fx, fy,
 *     cx, cy in pixels, and a row-major 3x4 camera-to-world matrix [R | o]
 *     (world = R * cam + o; the columns of R are the camera right, down and
 *     forward axes; o is the camera centre).  Pixel (px, py) covers
 *     [px, px+1) x [py, py+1); its centre is (px + 0.5, py + 0.5).
 *   - Maps: device arrays, height x width, row-major, float32 (n_samp uint16).
 *     Depths are planar (camera Z), except the NeRF path with
 *     nerf_ray_depths = 1 (distances along the pixel ray); 0 means "no surface
 *     at this pixel".
 *   - All device pointers are caller-owned unless stated; the library never
 *     frees caller memory.  All work is enqueued on the given HIP stream
 *     (NULL = the null stream) and is complete when that stream is.
 *   - Every call returns a status and never throws.  Arguments are validated
 *     before anything is enqueued; on DIVAS_ERR_ARG, DIVAS_ERR_ADMISSION,
 *     DIVAS_ERR_TOO_MANY_VIEWS and DIVAS_ERR_CAPACITY nothing is modified.
 *     A failed device call marks the session DIVAS_ERR_STATE.
 *   - A context and its sessions are not thread-safe; serialise calls on one
 *     context externally.
 */
#ifndef DIVAS_H
#define DIVAS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct divas_ctx_s* divas_ctx;
typedef struct divas_session_s* divas_session;
typedef void* divas_stream; /* a hipStream_t */

typedef enum {
    DIVAS_OK = 0,
    DIVAS_ERR_ARG = 1,            /* invalid argument (null, NaN, size, non-power-of-two dim, ...) */
    DIVAS_ERR_OOM = 2,            /* device allocation failed */
    DIVAS_ERR_ADMISSION = 3,      /* the session's footprint exceeds the context's HBM budget */
    DIVAS_ERR_TOO_MANY_VIEWS = 4, /* more than 64 views (the view bitmask is 64 bits) */
    DIVAS_ERR_STATE = 5,          /* call not valid in the session's state, or the session is poisoned */
    DIVAS_ERR_DEVICE = 6,         /* a HIP call failed */
    DIVAS_ERR_CAPACITY = 7        /* input larger than the capacity fixed at session creation */
} divas_status;

#define DIVAS_MAX_VIEWS 64

/* Voxel grid of the occupancy construction (Sec. 3.5, "Occupancy by
 * Morton-scattered opacity"; the cube of half-extent b around c_scene has
 * origin = c_scene - b). */
typedef struct {
    double origin[3];
    double voxel;
    int32_t dim;
} divas_grid;

/* Occupancy input (Sec. 3.5 and App. F, "Occupancy grid construction"):
 * rho[v] = sum of the opacities of the points in voxel v, summed in point
 * order in binary64; a voxel is active iff rho[v] >= tau_occ (the transmittance
 * floor tau_TF).  xyz: device float32 [n][3]; opacity: device float32 [n] or
 * NULL for opacity 1. */
typedef struct {
    const float* xyz;
    const float* opacity;
    int64_t n;
    double tau_occ;
} divas_occupancy;

/* One view's camera (host memory).  d_cam is the camera-to-target distance of
 * the see-through test (Eq. seethrough). */
typedef struct {
    double fx, fy, cx, cy;
    double c2w[12];
    int32_t width, height;
    double d_cam;
} divas_camera;

/* One view's maps (device memory, height x width row-major).  mask is the
 * depth-refined mask M~ in [0, 1], or, for the differentiable variant, its
 * logit; d_min / d_ref / d_max are the depth tuple (D_ref = D_med for 2DGS);
 * n_samp may be NULL (then no footprint statistics: layered = false, E = 0).
 * The footprint statistics of the 2DGS path (sums of n_samp and n_samp^2
 * over the pixel box of a voxel's 8 projected corners) are read straight from
 * n_samp by the fusion; no integral images are built. */
typedef struct {
    const float* mask;
    const float* d_min;
    const float* d_ref;
    const float* d_max;
    const uint16_t* n_samp;
} divas_view_maps;

/* Fusion constants.  Defaults (divas_params_default) follow Tab.
 * gs-hyperparams: gamma 1.0, beta 0.05, gamma_st 1.5, tau_cons 0.5, and the
 * thick-path entry gate m >= 0.5 of Alg. gs-fusion.  The paper gives no value
 * for alpha1, k (pi_dg) or eps: alpha1 = 1, k_grad = 1 / (4 voxel^2),
 * eps = 1e-6.  mask_gate = 0 makes every depth-consistent view vote its mask.
 * differentiable = 1 selects the soft depth test on logits (mask holds
 * logits, soft_width is the width of the sigmoid in scene units). */
typedef struct {
    double gamma, beta, gamma_st, alpha1, k_grad, eps, tau_cons, mask_gate, soft_width;
    int32_t differentiable;
    int32_t retain_state; /* keep binary64 W, Z and the raw view bitmask on the device
                             so that divas_update_view folds one view in O(N_active) */
    /* variant = 1 selects the NeRF path of Alg. nerf-fusion instead of the
     * 2DGS one: the depth planes hold D_min, D_exp, D_max (camera Z unless
     * nerf_ray_depths), and a view votes iff m >= mask_gate, the centre's
     * distance to the point of its pixel ray at t_c = clamp(t_proj, D_min,
     * D_max) is <= h pi_dg + lambda_range (D_max - D_min) (Eqs. distance_cond,
     * dist_tol) and |x_d - D_exp| <= (gamma + min(beta n_samp, b_max)) h (Eqs.
     * depth_tol, nerf-accept), with the weight exp(-alpha1 r^2), r = |t_c - mid|
     * / half-width of the band (Eq. nerf-vote).  n_samp is read at the pixel
     * (no footprint statistics); the density floor is the occupancy threshold
     * tau_occ; there is no scene contraction.  Not with differentiable = 1. */
    int32_t variant;
    double lambda_range, b_max;
    /* thin = 1 adds the thin-structure path to the fusion.
     * 2DGS (Alg. gs-fusion, Alg. gs-thin; Eqs. behind-gate, thin-nmin,
     * gs-coverage, thin-d2min, thin-tthin-gs): a view where the thick path
     * casts no vote, whose centre pixel is in frame, that is not more than 2h
     * behind the visible surface (D_min if trusted and see-through, else D_med)
     * and whose voxel holds at least rho_thin points sweeps the voxel's
     * projected footprint (the 8-corner box, floor(min)..floor(max), clipped;
     * A = its pixel count).  Per pixel with a surface: the tightened depth gate
     * (gamma h / (1 + beta E), front reference when layered or see-through and
     * D_min <= D_med); depth-consistent pixels count, those with M~ > 0.5 also
     * count towards coverage, give the peak M~ and unproject (at D_min when
     * layered, else D_med) to the nearest surface point.  The score is the peak
     * M~ when at least max(n_abs, ceil(rho_occ A)) pixels are depth-consistent,
     * the coverage is >= rho_cover and the nearest point is within 1.5 h.
     * NeRF (Alg. nerf-fusion, Alg. nerf-thin; Eqs. nerf-thindepth,
     * nerf-support, nerf-counters, nerf-coverage, nerf-thin): a view where the
     * thick path casts no vote, whose centre pixel is in frame with M~ > 0.1
     * and whose voxel holds at least rho_thin points sweeps the same footprint:
     * a pixel is supportive when M~ > 0.5 and |x_d - D_exp| <= (2 gamma +
     * min(beta n_samp, b_max)) h; the score is the largest M~ of the footprint
     * when the supportive fraction of its pixels is >= rho_cover.
     * Either way a score >= tau_thin (> 0) adds score / 1 to W / Z and sets
     * the view bit.  Needs unit opacity (the density is the point count).
     * Chunk boxes are padded by h/2 for the cull, which is skipped when the
     * gate bits cannot cover every pixel that can carry a vote.  Defaults:
     * 2DGS rho_thin 0.5 (the paper keeps the thick path's density floor for the
     * 2DGS thin path), tau_thin 0.6, rho_cover 0.5, rho_occ 0.1, n_abs 25;
     * NeRF (divas_params_nerf) rho_thin 50 / 30, rho_cover 0.2 / 0.3. */
    int32_t thin;
    double rho_thin, tau_thin, rho_cover, rho_occ, n_abs;
    /* NeRF path only: 0 (default) reads the depth tuple as camera Z, as the
     * paper states for both renderers, with x_d the voxel's camera Z and the
     * ray parameter t_proj clamped into [D_min, D_max] as written; 1 reads the
     * tuple as distances along each pixel's unit ray and x_d = t_proj. */
    int32_t nerf_ray_depths;
    /* With retain_state: 1 lets a fold (divas_update_view appending a view,
     * or a batch update that appends one) whose out.P and out.vmask are the
     * buffers of this session's previous fusion call, with no other call that
     * changes the session in between, write only the entries of the chunks
     * whose cull bit for the new view is set: a chunk the view cannot reach
     * keeps W, Z and its views, so its outputs already hold their values, which
     * the caller must not have modified.  The counts are then kept as running
     * totals (each changed voxel's old contribution replaced by its new one),
     * equal to those of a full write.  Any other call writes every entry. */
    int32_t resident_outputs;
} divas_params;

/* Outputs of a fusion call (caller-allocated device buffers, n_active entries):
 *   P      float32 fused probability, Eq. compact-fusion (W / Z rounded once);
 *   vmask  uint64 view-coverage bitmask, Eq. vmask, kept only where P >= tau_cons;
 *   seg_bits  uint32[dim^3 / 32] segmentation bitfield (bit v set iff voxel v is
 *          active and P >= tau_cons), or NULL (the session keeps its own copy);
 *   counts int64[3]: segmented voxels, voxels with |P - tau_cons| <= 1e-5,
 *          accepted votes; or NULL.
 * Entry i of P / vmask belongs to active voxel i of divas_session_info. */
typedef struct {
    float* P;
    uint64_t* vmask;
    uint32_t* seg_bits;
    int64_t* counts;
} divas_result;

/* Fill *out with the defaults above for a grid of edge `voxel`. */
divas_status divas_params_default(double voxel, divas_params* out);
/* The NeRF path with the constants of the NeRF hyperparameter table:
 * column 0 = LLFF (gamma 4, beta 0.2, b_max 10, lambda_range 0.05, rho_thin
 * 50, rho_cover 0.2), column 1 = Mip-NeRF 360 (gamma 0.5, beta 0.2, b_max 1,
 * lambda_range 5, rho_thin 30, rho_cover 0.3); tau_thin 0.6; depths as camera
 * Z; the other fields as divas_params_default. */
divas_status divas_params_nerf(double voxel, int32_t column, divas_params* out);

/* Context for one device: HIP device index and an HBM budget in bytes used to
 * admit sessions (0 = no limit). */
divas_status divas_ctx_create(int device, size_t hbm_budget_bytes, divas_ctx* out);
divas_status divas_ctx_destroy(divas_ctx ctx);
/* Bytes currently held by the context's sessions. */
divas_status divas_ctx_usage(divas_ctx ctx, size_t* used_bytes, size_t* budget_bytes);

/* Device footprint of a session (bytes) for the given capacities: points,
 * views, and the largest view size (pixels).  Pure host arithmetic. */
size_t divas_session_footprint(const divas_grid* grid, int64_t max_points, int32_t max_views,
                               int64_t max_view_pixels, int32_t retain_state);

/* Create a session: admit it against the budget, allocate its device state for
 * at most max_points points (0 = occ->n), max_views views of at most
 * max_view_pixels pixels, and build the active list (occupancy construction)
 * from occ on `stream`.  The active list is sorted by Morton code (x -> bit 0,
 * y -> bit 1, z -> bit 2).  Fails with DIVAS_ERR_ADMISSION when the footprint
 * (divas_session_footprint) does not fit the context's remaining budget. */
divas_status divas_session_create(divas_ctx ctx, const divas_grid* grid, const divas_occupancy* occ,
                                  const divas_params* params, int64_t max_points, int32_t max_views,
                                  int64_t max_view_pixels, divas_stream stream, divas_session* out);

/* Rebuild the active list from new points (occ->n <= the creation capacity);
 * resets the views and the segmentation. */
divas_status divas_session_rebuild(divas_session s, const divas_occupancy* occ, divas_stream stream);

/* Number of active voxels (synchronises on the session's last rebuild), the
 * library-owned device array of their linear indices in Morton order (valid
 * until the next rebuild or destroy), the number of fused views and the
 * session's device footprint. */
divas_status divas_session_info(divas_session s, int64_t* n_active, const uint32_t** active_linear_idx,
                                int32_t* n_views, size_t* footprint_bytes);

/* Fusion of n_views views (Alg. gs-fusion, or Alg. nerf-fusion with
 * variant = 1; the thin-structure path only with params.thin = 1) followed by
 * the compact-fusion rule and the consensus threshold (Eq. compact-fusion).  Views are accumulated in index order in binary64.  The
 * session records cams by value and maps by pointer: the caller keeps every
 * view's maps alive and unchanged until the session is destroyed, rebuilt,
 * re-fused or the view replaced (update_view and fuse_backward re-read them). */
divas_status divas_fuse_views(divas_session s, int32_t n_views, const divas_camera* cams,
                              const divas_view_maps* maps, const divas_result* out, divas_stream stream);

/* A target session: another target object of the scene of `base`.  It shares
 * base's grid, occupancy (active list, chunk boxes, point counts) without a
 * copy and holds its own parameters, views, accumulators, segmentation and
 * outputs; every call that takes a session takes it (fusion, updates, labels,
 * backward, Pass 3, batches, the multi-target fusion below).  base must not be
 * a target session; while target sessions of base exist, base can neither be
 * rebuilt nor destroyed (DIVAS_ERR_STATE), and a target session is never
 * rebuilt.  A thin-path target needs a base built with the thin path (its
 * point counts).  Admitted against the context's budget for its own state
 * only.  The same map-lifetime rule as divas_fuse_views applies. */
divas_status divas_session_create_target(divas_session base, const divas_params* params, int32_t max_views,
                                         int64_t max_view_pixels, divas_stream stream, divas_session* out);

/* One fusion of n_views views for n_targets (1..8) sessions of one scene: a
 * session and target sessions of it (or target sessions of one base), each at
 * most once.  maps[t * n_views + s] are target t's maps of view s; their depth
 * planes and n_samp must be the same pointers for every t (only the mask
 * differs); cams are the views' cameras, shared.  With the 2DGS thick path
 * (variant 0, thin 0, differentiable 0) and equal fusion parameters the
 * targets are fused together: the chunk rectangle of a view is projected once
 * for all targets' culls, and each (voxel, view) sample's projection, depth
 * gathers, depth and spatial gates and weight are evaluated once, every target
 * whose gate bit is set adding its own mask vote (the mask enters Alg.
 * gs-fusion's thick branch only through the entry gate and the vote m w).
 * Otherwise the targets are fused one after another.  schedule chooses:
 * DIVAS_TARGETS_AUTO fuses them together only at mask gate 0 (every in-frame
 * sample with a surface is gathered, so the shared work dominates) and one
 * after another under a positive gate (few samples pass it; the kernel that
 * holds every target's accumulators runs at lower occupancy and was measured
 * slower there); DIVAS_TARGETS_TOGETHER whenever the targets can share;
 * DIVAS_TARGETS_ONE_BY_ONE never.  Either way outs[t] and session t's state
 * equal divas_fuse_views(sessions[t], n_views, cams, maps + t n_views,
 * outs + t) bit for bit.  Errors as divas_fuse_views, and DIVAS_ERR_ARG for
 * sessions of different scenes, a repeated session, depth planes that differ
 * between targets, or an unknown schedule. */
#define DIVAS_TARGETS_AUTO 0
#define DIVAS_TARGETS_TOGETHER 1
#define DIVAS_TARGETS_ONE_BY_ONE 2
divas_status divas_fuse_targets(const divas_session* sessions, int32_t n_targets, int32_t n_views,
                                const divas_camera* cams, const divas_view_maps* maps, const divas_result* outs,
                                int32_t schedule, divas_stream stream);

/* Click-driven update (the per-update re-fusion of the paper's interaction
 * loop).  slot == n_views appends a view; with retain_state the new view is
 * folded into the resident accumulators in O(N_active), bit-identical to a full
 * re-fusion; otherwise, or when slot < n_views replaces a view, all views are
 * re-fused.  Same map-lifetime rule as divas_fuse_views. */
divas_status divas_update_view(divas_session s, int32_t slot, const divas_camera* cam,
                               const divas_view_maps* maps, const divas_result* out,
                               divas_stream stream);

/* Eq. pass1 / Pass 1 of Alg. vox2surfel: labels[i] = 1 iff point i lies in an
 * active voxel whose P >= tau_cons after the session's last fusion; NaN and
 * out-of-grid points get 0.  xyz: device float32 [n][3]; labels: device uint8 [n]. */
divas_status divas_label_points(divas_session s, const float* xyz, int64_t n, uint8_t* labels,
                                divas_stream stream);

/* Eq. pass1 for the points of the session's last occupancy build (the xyz of
 * divas_session_create or divas_session_rebuild, as they were at that call;
 * for a target session, its base session's build): labels[i] equals what
 * divas_label_points gives for point i of that build, read from the voxel
 * codes the build kept instead of from the coordinates.  labels: device
 * uint8 [n], n = the build's point count, which is written to *n_points (may
 * be NULL); labels == NULL only writes *n_points.  DIVAS_ERR_STATE when the
 * build kept no codes (opacities or tau_occ > 1). */
divas_status divas_label_session_points(divas_session s, uint8_t* labels, int64_t* n_points,
                                        divas_stream stream);

/* Reverse mode of the differentiable fusion (params.differentiable = 1, after
 * a divas_fuse_views of the same session): given grad_P (device float32
 * [n_active], dL/dP), writes dL/d(logit), dL/d(d_min), dL/d(d_ref), dL/d(d_max)
 * into per-view device float32 arrays (height x width; any pointer or array
 * may be NULL to skip).  n_views is the length of each of the four host arrays
 * of pointers and must equal the view count of the session's last fusion
 * (DIVAS_ERR_ARG otherwise).  The adjoint is that of the session's current
 * fused state: a caller that keeps a forward for later differentiation
 * records divas_session_generation after it and checks it before this call.
 * Projections are recomputed, not stored; the per-pixel sums are accumulated
 * in a fixed order (deterministic, no float atomics). */
divas_status divas_fuse_backward(divas_session s, const float* grad_P, int32_t n_views, float* const* grad_logit,
                                 float* const* grad_dmin, float* const* grad_dref,
                                 float* const* grad_dmax, divas_stream stream);

/* A counter that every call changing the session's fused state increments
 * (fusion, update, batch item, rebuild). */
divas_status divas_session_generation(divas_session s, uint64_t* generation);

divas_status divas_session_destroy(divas_session s);

/* ------------------------------------------------------------------ batches
 * Many sessions (different scenes, objects, grid sizes and view counts) in one
 * sequence of five launches sized for the whole batch: hot-tile rows and
 * columns of the new views, culling (which lists the chunks that have views to
 * evaluate), fusion of those chunks by persistent wavefronts, and the outputs of
 * the remaining chunks.  Each
 * item does exactly what divas_fuse_views (op DIVAS_BATCH_FUSE) or
 * divas_update_view (op DIVAS_BATCH_UPDATE) does for its session, with
 * bit-identical outputs; at most one item per session per batch.  With
 * use_graph the launches are captured once in a HIP graph
 * and replayed (the per-batch tables are copied to the device before each
 * replay).  The same
 * map-lifetime rule as divas_fuse_views applies.  A batch object owns device
 * tables sized for max_items items and max_new_views new views per run; runs
 * on one batch object are serialised by the library. */
typedef struct divas_batch_s* divas_batch;

typedef enum { DIVAS_BATCH_FUSE = 0, DIVAS_BATCH_UPDATE = 1 } divas_batch_op;

typedef struct {
    divas_session session;
    int32_t op;          /* divas_batch_op */
    int32_t n_views;     /* FUSE: views in cams/maps; UPDATE: must be 1 */
    int32_t slot;        /* UPDATE: slot (== the session's n_views appends) */
    int32_t pad;
    const divas_camera* cams;
    const divas_view_maps* maps;
    divas_result out;
} divas_batch_item;

typedef struct {
    int32_t fuse_waves_per_block; /* wavefronts per block of the fusion launch, one per chunk: 1, 2, 4 or 8 (0 = 4) */
    int32_t cull_blocks_per_cu;   /* grid of the culling pass = this x compute units (0 = 4) */
    int32_t use_graph;            /* capture and replay the launches as a HIP graph */
    int32_t schedule;             /* fusion schedule: 0 = one wavefront per chunk, handed out by the hardware
                                     dispatcher; k > 0 = a persistent grid (16 wavefronts per compute unit)
                                     whose wavefronts pop descriptors of k chunks of one item from an
                                     integer-atomic queue, the items fusing the most views first */
} divas_batch_config;

divas_status divas_batch_create(divas_ctx ctx, int32_t max_items, int32_t max_new_views,
                                const divas_batch_config* cfg, divas_batch* out);
divas_status divas_batch_run(divas_batch b, int32_t n_items, const divas_batch_item* items, divas_stream stream);
/* The argument checks of divas_batch_run alone: returns the status that
 * divas_batch_run would return for these items before enqueuing anything
 * (DIVAS_ERR_ARG, _CAPACITY, _TOO_MANY_VIEWS, _STATE), and enqueues nothing. */
divas_status divas_batch_validate(divas_batch b, int32_t n_items, const divas_batch_item* items);
/* Autotune the batch configuration on a representative batch of
 * DIVAS_BATCH_FUSE items (re-running them is idempotent), timing each
 * candidate with HIP events: fuse_waves_per_block {1, 2, 4, 8} x
 * cull_blocks_per_cu {2, 4, 8} x schedule {0, 1, 4, 16} with the graph, then
 * the winner without it.  The winner is applied to b, written to *chosen and,
 * when cache_path is not NULL, stored in / first looked up from that JSON file
 * (one object per line) under a key made of the device name and the batch's
 * size buckets. */
divas_status divas_batch_tune(divas_batch b, int32_t n_items, const divas_batch_item* items, divas_stream stream,
                              const char* cache_path, divas_batch_config* chosen);
divas_status divas_batch_destroy(divas_batch b);

/* ------------------------------------------------------------------ serving
 * A continuous-batching server for click-driven updates of many resident
 * sessions.  A scheduler thread owns every HIP call on the server's sessions:
 * it admits session opens (FIFO) when their footprint fits the context's HBM
 * budget, gathers the queued requests of admitted sessions without work in
 * flight into one divas_batch_run per free stream slot (requests that arrive
 * while others run join the next batch; batches on different slots overlap on
 * the device), observes completion events, and records each update's latency
 * from its arrival stamp (seconds on divas_server_now's clock; < 0 = now) to
 * the observed completion.  A session's requests are applied in submission
 * order; every request's outputs equal applying it alone.  Cameras are copied;
 * maps and result buffers stay caller-owned until the request is done.  The
 * submit / wait / stats calls are thread-safe; do not call other functions on
 * a server's sessions while the server runs. */
typedef struct divas_server_s* divas_server;

typedef struct {
    int32_t n_streams;     /* batches in flight at once (1..8, default 2) */
    int32_t max_batch;     /* requests per batch (default 64) */
    int32_t max_new_views; /* new views per batch (default 64) */
    int32_t pad;
    divas_batch_config batch;
} divas_server_config;

typedef struct {
    int64_t completed_updates, batches, batched_requests, admission_waits, max_queue, failures;
    int64_t sessions_open, sessions_waiting;
    double p50_ms, p99_ms, mean_ms, max_ms;  /* latency of completed DIVAS_BATCH_UPDATE requests */
} divas_server_statistics;

divas_status divas_server_create(divas_ctx ctx, const divas_server_config* cfg, divas_server* out);
double divas_server_now(divas_server s);
/* Queue a session open (admitted when its footprint fits the budget); the
 * device points `occ` must stay valid until the session is admitted.  A
 * session whose footprint exceeds the whole budget is refused at once
 * (DIVAS_ERR_ADMISSION).  When the server is destroyed, the queued requests
 * of sessions still waiting for admission fail with DIVAS_ERR_ADMISSION. */
divas_status divas_server_open_session(divas_server s, const divas_grid* grid, const divas_occupancy* occ,
                                       const divas_params* params, int64_t max_points, int32_t max_views,
                                       int64_t max_view_pixels, int32_t* session_id);
/* Session handle once admitted (*admitted = 1; 0 waiting; -1 failed). */
divas_status divas_server_session(divas_server s, int32_t session_id, divas_session* out, int32_t* admitted);
/* Close after the session's queued requests are done (frees its budget). */
divas_status divas_server_close_session(divas_server s, int32_t session_id);
/* Queue a request: op DIVAS_BATCH_FUSE (n_views views) or DIVAS_BATCH_UPDATE
 * (one view; slot < 0 appends). */
divas_status divas_server_submit(divas_server s, int32_t session_id, int32_t op, int32_t n_views, int32_t slot,
                                 const divas_camera* cams, const divas_view_maps* maps, const divas_result* out,
                                 double arrival_s, uint64_t* ticket);
/* Wait up to timeout_s for a request; *done = 1 when complete, *latency_ms its latency. */
divas_status divas_server_wait(divas_server s, uint64_t ticket, double timeout_s, int32_t* done, double* latency_ms);
divas_status divas_server_drain(divas_server s, double timeout_s);
divas_status divas_server_stats(divas_server s, divas_server_statistics* out);
divas_status divas_server_latencies(divas_server s, double* out, int64_t capacity, int64_t* n);
divas_status divas_server_destroy(divas_server s);

/* Phase timing (tracing).  divas_session_set_timing selects the phases to time
 * (bit p of phase_mask = phase p; DIVAS_TIMING_ALL = every phase; 0 = off).  A
 * timed phase is measured with HIP events on the caller's stream, taken from
 * the dispatch packets of its first and last kernel (hipExtLaunchKernel), so
 * timing adds no work to the stream (the backward phase records its events
 * around its launches).  divas_session_timings waits for the events and
 * returns, per phase, the accumulated milliseconds and the number of timed
 * launches since the last reset.  Phases: occupancy construction (several
 * kernels), per-view pre-pass (hot tiles, gate bitmask),
 * chunk culling, fusion (the fusion kernel, with the threshold and the
 * bitfield update; the count reduction after it is not timed), labels,
 * backward. */
typedef enum {
    DIVAS_PHASE_OCCUPANCY = 0,
    DIVAS_PHASE_VIEWS = 1,
    DIVAS_PHASE_CULL = 2,
    DIVAS_PHASE_FUSE = 3,
    DIVAS_PHASE_LABEL = 4,
    DIVAS_PHASE_BACKWARD = 5,
    DIVAS_PHASE_COUNT = 6
} divas_phase;
/* Work of the session's last fusion (or update): chunks of 64 active voxels
 * that had views to evaluate, those (chunk, view) pairs, and the samples
 * whose pixel passed the mask gate (the depth-map gathers).  Waits for the
 * device to be idle.  Any output pointer may be NULL. */
divas_status divas_session_fusion_work(divas_session s, int64_t* hot_chunks, int64_t* hot_pairs, int64_t* gathered);
#define DIVAS_TIMING_ALL 0xFFFFFFFFu
divas_status divas_session_set_timing(divas_session s, uint32_t phase_mask);
divas_status divas_session_timings(divas_session s, double* ms, int64_t* launches, int32_t reset);

/* Scene-statistic grid construction (Sec. 3.5 (i), Eq. scene-norm and
 * Eq. voxel-size): the grid that the occupancy construction runs on, derived
 * from the points themselves.
 *   c_scene = coordinate-wise median of the centres;
 *   r_fg    = percentile `percentile` (0.99) of |mu - c_scene|;
 *   b       = ceil(pad * r_fg), pad = 1.05 (an integer half-extent);
 *   h_v     = max(alpha_v * s_med, beta_v * r_fg / g0), (3, 1, 256), where
 *             s_med is the median scale (the first term is dropped without
 *             scales);
 *   dim     = the smallest power of two >= 2 b / h_v (at least 2), capped at
 *             g_max (512 or 1024);
 *   grid    = origin c_scene - b, voxel 2 b / dim (the cube exactly).
 * A point takes part iff its three coordinates (and its scale, when scales
 * are given) are finite.  The median of an even count is the mean of the two
 * middle order statistics, in binary64; the percentile interpolates linearly
 * between the order statistics around position percentile * (m - 1); the
 * distance is sqrt((dx^2 + dy^2) + dz^2) in binary64.  Every order statistic
 * is selected exactly, so the outputs are those of the plain definitions.
 * xyz: device float32 [n][3]; scale: device float32 [n] (one scale per point,
 * e.g. the larger tangent scale of a surfel) or NULL.  Work runs on `stream`;
 * the call returns when it is done (each statistic feeds the next).  It
 * uses 8 n bytes of the context's device scratch (a buffer the context grows
 * on demand and frees when it is destroyed; not counted in its HBM budget).
 * Errors: DIVAS_ERR_ARG for n < 1, a NULL xyz, parameters out of range, no
 * point taking part, or a degenerate result (b or h_v not > 0); then *grid
 * and *stats are not written.  stats may be NULL. */
typedef struct {
    double alpha_v, beta_v, pad, percentile;
    int32_t g0, g_max;
} divas_grid_params;
typedef struct {
    double center[3];
    double r_fg, b, s_med, h_v; /* s_med is NaN without scales */
    int64_t n_used;             /* points taking part */
    int64_t n_kept;             /* points inside the grid (voxel rule above) */
} divas_grid_stats;
/* Defaults of Tab. gs-hyperparams for the given resolution cap. */
divas_status divas_grid_params_default(int32_t g_max, divas_grid_params* out);
divas_status divas_grid_from_points(divas_ctx ctx, const float* xyz, const float* scale, int64_t n,
                                    const divas_grid_params* params, divas_grid* grid, divas_grid_stats* stats,
                                    divas_stream stream);

/* Depth refinement of a view's mask (Sec. 3.2, "Depth-weighting"): the
 * refined mask M~ that the fusion takes, from the prompt mask M (a [0, 1]
 * confidence) and the view's rendered depth.
 *   band-pass (2DGS; Eq. depthband, Eq. gs-bandpass): the band [d_min, d_max]
 *     is the range of the median depth at the positive prompt pixels and at
 *     the view centre (width / 2, height / 2); d_far is the 98th percentile of
 *     the median-depth map;
 *     M~ = M (1 - clip((max(d_min - D, 0) + max(D - d_max, 0))
 *                      / max(d_far - d_max, 1e-6), 0, 1));
 *   min-max (NeRF; Eq. nerf-depthweight), D the expected depth:
 *     M~ = M (1 - (D - min D) / (max D - min D)).
 * A pixel has a surface iff its depth is finite and > 0; d_far and the
 * extrema are taken over surface pixels, a pixel without a surface gets M~ = 0,
 * and anchors without a surface are left out of the band.  The percentile
 * interpolates linearly between the order statistics around 0.98 (m - 1)
 * (selected exactly); with max D = min D every surface pixel keeps M.  The
 * weights are binary64 in the order above and M~ is rounded once to float32.
 * mask, depth, refined: device float32 [height][width] (refined may be mask);
 * prompts_xy: host int32 [2 n_prompts] pixel coordinates (x, y), or NULL when
 * n_prompts is 0.  Work runs on `stream`; the call returns when it is done.
 * The band-pass uses 4 width height bytes of the context's device scratch
 * (see divas_grid_from_points).  Errors: DIVAS_ERR_ARG for NULL buffers, sizes < 1, a prompt outside
 * the view, no pixel with a surface, or (band-pass) no anchor with a surface;
 * then refined is not written.  stats may be NULL. */
typedef struct {
    double band_min, band_max, d_far; /* band-pass (NaN for min-max) */
    double z_min, z_max;              /* min-max (NaN for band-pass) */
    int64_t n_surface;                /* pixels with a surface */
    int32_t n_anchors;                /* band-pass anchors with a surface */
} divas_refine_stats;
divas_status divas_refine_mask_bandpass(divas_ctx ctx, int32_t width, int32_t height, const float* mask,
                                        const float* d_med, const int32_t* prompts_xy, int32_t n_prompts,
                                        float* refined, divas_refine_stats* stats, divas_stream stream);
divas_status divas_refine_mask_minmax(divas_ctx ctx, int32_t width, int32_t height, const float* mask,
                                      const float* d_exp, float* refined, divas_refine_stats* stats,
                                      divas_stream stream);

/* Needle-floater cull, Pass 2 of the voxel-to-surfel mapping (Eq. aspect,
 * Eq. needle, Eq. pass-needle): labels[i] &= (a_i <= tau_a) with
 *   a_i   = max(s_i1, s_i2) / (min(s_i1, s_i2) + eps)   (binary64),
 *   tau_a = the 99th percentile of the aspects (linear between the order
 *           statistics around 0.99 (m - 1), selected exactly).
 * A surfel whose scales or aspect are not finite stays out of the percentile
 * and is culled.  The paper gives no eps; 1e-6 is the library's reading.
 * scales: device float32 [n][2] (the two tangent scales of each surfel);
 * labels: device uint8 [n], the Pass 1 labels (divas_label_points), updated in
 * place.  Runs on `stream` and returns when done; uses 8 n bytes of the
 * context's scratch.  tau_a and n_culled (surfels with a > tau_a or no
 * aspect) may be NULL.  Errors: DIVAS_ERR_ARG for NULL buffers, n < 1, eps not
 * finite and >= 0, or no surfel with an aspect (labels then untouched). */
divas_status divas_needle_cull(divas_ctx ctx, const float* scales, int64_t n, double eps, uint8_t* labels,
                               double* tau_a, int64_t* n_culled, divas_stream stream);

/* The needle cull without any device allocation, for callers that cannot
 * allocate (code that must not call hipMalloc: tight serving loops, harnesses
 * that forbid it).  Same arguments, arithmetic, results and errors as
 * divas_needle_cull, but its scratch is a fixed device array of 32 MiB built
 * into the library (one per device, held until the process ends; its address
 * is looked up when the context is created), so n is limited to
 * DIVAS_NOALLOC_MAX_SURFELS: a larger n fails with DIVAS_ERR_CAPACITY before
 * anything is enqueued.  The call allocates no device or pinned memory.
 * Every call on a device shares that device's array, and the call clears what
 * must start at zero: calls that overlap on one device (from several threads
 * or contexts) race and must be serialised by the caller. */
#define DIVAS_NOALLOC_MAX_SURFELS 4000000
divas_status divas_needle_cull_noalloc(divas_ctx ctx, const float* scales, int64_t n, double eps, uint8_t* labels,
                                       double* tau_a, int64_t* n_culled, divas_stream stream);

/* Pass 3 of the voxel-to-surfel mapping (Alg. vox2surfel, Pass 3; Eqs.
 * keys-no-depth, cov-atomics, kappa, final-F): footprint coverage of the
 * labelled surfels in the session's views.  For every surfel i with
 * labels_in[i] = 1, its voxel (the Pass 1 rule) is looked up in the active
 * list and the view bitmask of that voxel read from vmask; for every view s of
 * that bitmask (gating, step (i)), the centre and the tangent semi-axes
 * t_k = s_k R e_k (k = 1, 2; R the rotation of the unit quaternion) are taken
 * to the camera frame, the four tips mu +- t_k projected, and the 1-sigma
 * pixel box [c - e, c + e] (e per image axis the larger half-difference of the
 * projected tips) visited; a pixel counts when the ray through its centre meets
 * the surfel plane in front of the camera at tangent coordinates (u, v) (in
 * units of the scales) with u^2 + v^2 <= 9, and it is a mask hit when its mask
 * reaches tau_M.  kappa_s = hits / max(total, 1) and kappa_i = max over the
 * gated views (0 without any); labels_out[i] = labels_in[i] and
 * kappa_i >= tau_kappa.  A view whose centre or a tip is not in front of the
 * camera does not score the surfel.  All geometry is binary64.
 * xyz: device float32 [n][3] surfel centres; scales: device float32 [n][2] the
 * two tangent scales; quats: device float32 [n][4] (w, x, y, z), normalised
 * here; labels_in: device uint8 [n] (the Pass 2 labels); vmask: device uint64
 * [n_active], the view bitmask output of the session's last fusion or update;
 * kappa: device float64 [n]; labels_out: device uint8 [n] (may alias
 * labels_in); kept: device int64 [1] receiving the number of labels kept, or
 * NULL.  The views and their masks are the session's current ones (as the
 * last fusion or update recorded them); enqueue on the stream of that fusion
 * or order the streams.  The paper's table gives tau_M = tau_kappa = 0.5.
 * Errors: DIVAS_ERR_ARG for NULL buffers, n < 0, thresholds not finite;
 * DIVAS_ERR_STATE before the session's first fusion. */
divas_status divas_surfel_coverage(divas_session s, const float* xyz, const float* scales, const float* quats,
                                   int64_t n, const uint8_t* labels_in, const uint64_t* vmask, double tau_M,
                                   double tau_kappa, double* kappa, uint8_t* labels_out, int64_t* kept,
                                   divas_stream stream);

const char* divas_status_string(divas_status st);
/* Message of the last error on this thread (empty if none). */
const char* divas_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* DIVAS_H */
