// Internal declarations of libdivas: device-side records and kernel launchers.
// Not part of the public ABI (include/divas.h is).
#pragma once

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace divas {

// Phase timing: the start event is taken from the dispatch of the phase's
// first kernel and the stop event from that of its last kernel
// (hipExtLaunchKernelGGL), so timing adds no packet to the stream.  A launcher
// given events attaches them to its kernels, or records them on the stream
// when it launches none.  Null events: untimed.
struct PhaseEvents {
    hipEvent_t start = nullptr, stop = nullptr;
};

template <typename K, typename... Args>
inline void launch_timed(K kernel, dim3 grid, dim3 block, uint32_t shmem, hipStream_t st, hipEvent_t e0, hipEvent_t e1,
                         Args... args) {
    if (e0 || e1)
        hipExtLaunchKernelGGL(kernel, grid, block, shmem, st, e0, e1, 0u, args...);
    else
        hipLaunchKernelGGL(kernel, grid, block, shmem, st, args...);
}

inline void record_phase_events(const PhaseEvents& ev, hipStream_t st) {
    if (ev.start) (void)hipEventRecord(ev.start, st);
    if (ev.stop) (void)hipEventRecord(ev.stop, st);
}

constexpr int kTile = 8;           // hot-tile edge (pixels) of the per-view mask pre-pass
constexpr int kCullRows = 24;      // tile rows a cull query scans before it keeps the pair
constexpr int kChunk = 64;         // active voxels per chunk = one wavefront
constexpr int kBlock = 256;        // threads per block of the voxel kernels (4 chunks)
constexpr int kMaxViews = 64;
int device_cu_count();

// One view: binary64 camera (for the exact per-voxel evaluation), float32
// copies (for the conservative chunk culling) and device pointers to its maps.
struct DView {
    double R[9];       // R[b * 3 + a] = rotation block of the camera-to-world matrix, row b, col a
    double o[3];       // camera centre
    double fx, fy, cx, cy, d_cam;
    float fR[9], fo[3], ffx, ffy, fcx, fcy;
    int32_t W, H;
    int32_t tw, th;    // hot-tile grid
    int32_t mpitch;    // bytes per row of the gate bitmask (= tw)
    int32_t mpad;
    const float* mask;
    const float* dmin;
    const float* dmed;
    const float* dmax;
    const uint16_t* nsamp; // per-pixel sample counts, or null
    uint64_t* tile_bits;   // hot tiles, th rows of ceil(tw / 64) words: bit tx & 63 of word (ty, tx >> 6)
    uint8_t* mbits;        // gate bitmask, H rows of mpitch bytes: bit k of byte (y, t) = mask(8t + k, y) >= gate
};

// Float bounding box of the voxel centres of a chunk, for the culling: low
// corner, extents (high - low), and p1 = sum over the axes of the larger
// absolute coordinate (the |p|_1 bound of the box's points).
struct alignas(16) ChunkBox {
    float lo[3];
    float p1;
    float ext[3];
    float pad;
};

struct DGrid {
    double origin[3];
    double h;
    int32_t dim;
    int32_t log2dim;
};

struct DParams {
    double gamma, beta, gamma_st, alpha1, k_grad, eps, tau_cons, mask_gate, soft_width;
    int32_t differentiable;
    int32_t variant;            // kVariant2DGS or kVariantNerf
    double lambda_range, b_max;  // NeRF thick path only
    int32_t thin;               // thin-structure path (Alg. gs-thin or Alg. nerf-thin)
    int32_t nerf_ray_depths;    // NeRF depth tuple: 0 camera Z, 1 distances along the pixel ray
    double rho_thin, tau_thin, rho_cover, rho_occ, n_abs;
};
constexpr int32_t kVariant2DGS = 0;
constexpr int32_t kVariantNerf = 1;

struct FuseArgs {
    const uint32_t* act;        // active linear indices, Morton order
    const int64_t* n_act;       // device count
    int64_t cap;                // capacity (grid sizing)
    DGrid g;
    DParams p;
    const DView* views;
    int32_t s_begin, s_end;     // views [s_begin, s_end) are evaluated
    const uint64_t* cull;       // [chunk]: bit s set = some voxel of the chunk may vote in view s
    int32_t cull_all;           // 1: the cull words are not read, every view of the range is evaluated
    int32_t load_acc;           // start from the resident W, Z, vraw
    int32_t store_acc;          // write W, Z, vraw back
    double* W;
    double* Z;
    uint64_t* vraw;
    float* P;
    uint64_t* vout;
    uint32_t* bits;             // session segmentation bitfield (linear index)
    uint32_t* coarse;           // segmented voxels per coarse cell (see coarse_cell)
    uint8_t* segb;              // [n_act] segmentation of the previous fusion (drives the bitfield update)
    int64_t* counts;            // [3]: n_seg, n_flag, n_votes (written by the count reduction)
    int64_t* slots;             // [kCountSlots * kSlotWords] partial counts; zero between fusions
    int64_t* stats;             // [3]: hot chunks, hot (chunk, view) pairs, gathered samples
    const uint32_t* rho;        // [n_act] points per active voxel (thin-structure fallback), or null
    int64_t* tot;               // [3] running totals of counts[0..2], kept by the count reduction, or null
    int32_t delta;              // fold into resident outputs: chunks without a view to evaluate write
                                // nothing, and a fused chunk's slots receive (new - old) counts
};

// Coarse cells of (2^kCoarseShift)^3 voxels (the whole grid for small grids):
// the fusion keeps the number of segmented voxels of every cell, so a label
// lookup in a cell without any skips the bitfield.
constexpr int kCoarseShift = 4;
// floor(fl(d / h)), the voxel coordinate of an offset d from the grid origin,
// with h > 0 and inv_h = fl(1 / h).  The product d * inv_h lies within |q| 2^-51
// of the correctly rounded quotient (the two are within 1.5 ulp and 0.5 ulp of
// the exact one, with the same sign), so their floors agree unless an integer
// lies within |q| 2^-50 of the product; only there is the division evaluated.
// The differences q - f and (f + 1) - q are exact (Sterbenz) where it matters.
__device__ __forceinline__ double voxel_floor(double d, double h, double inv_h) {
    const double q = d * inv_h;
    const double f = floor(q);
    const double margin = fabs(q) * 0x1p-50;
    if (q - f <= margin || (f + 1.0) - q <= margin) return floor(d / h);
    return f;
}

// The same floor for a float32 coordinate x and the origin coordinate o,
// evaluated first in float: with of = fl32(o) and ihf = fl32(inv_h), the
// product qf = fl32(fl32(x - of) * ihf) is within 2^-24 (|o| + 3.01 |x - o|) / h
// of the exact quotient (roundings of o, of the difference, of 1/h to float
// and of the product), so when its fractional part keeps 2^-21 (|of| + |x - of|)
// ihf (at least twice that bound) from both integers its floor is the floor of
// the correctly rounded binary64 quotient; otherwise (and for NaN) the binary64
// evaluation decides.  The fractional part qf - floor(qf) is exact in float for
// |qf| >= 1, and rounds towards 1 (failing the test) for small negative qf.
__device__ __forceinline__ double voxel_floor_f(float x, double o, double h, double inv_h) {
    const float of = (float)o, ihf = (float)inv_h;
    const float s = x - of;
    const float qf = s * ihf;
    const float f = floorf(qf);
    const float fr = qf - f;
    const float m = 0x1p-21f * ((fabsf(of) + fabsf(s)) * ihf);
    if ((fr > m) & (fr < 1.0f - m)) return (double)f;
    return voxel_floor((double)x - o, h, inv_h);
}

__device__ __forceinline__ uint32_t spread3(uint32_t v) {
    // bit b of v -> bit 3b (v < 1024)
    v &= 0x3FFu;
    v = (v | (v << 16)) & 0x030000FFu;
    v = (v | (v << 8)) & 0x0300F00Fu;
    v = (v | (v << 4)) & 0x030C30C3u;
    v = (v | (v << 2)) & 0x09249249u;
    return v;
}

// bit 3b of v -> bit b (the inverse of spread3 on its image)
__device__ __forceinline__ uint32_t compact3(uint32_t v) {
    v &= 0x09249249u;
    v = (v | (v >> 2)) & 0x030C30C3u;
    v = (v | (v >> 4)) & 0x0300F00Fu;
    v = (v | (v >> 8)) & 0x030000FFu;
    v = (v | (v >> 16)) & 0x000003FFu;
    return v;
}

// Morton code of the voxel holding (x, y, z), or 0xFFFFFFFF: same expression as
// point_voxel.
// Voxel index floor((p - origin) / h) per axis (voxel_floor_f: the floor of
// the correctly rounded binary64 quotient), then the Morton code.
__device__ __forceinline__ uint32_t morton_of(float x, float y, float z, const DGrid& g, double inv_h) {
    const float p[3] = {x, y, z};
    uint32_t idx[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const double f = voxel_floor_f(p[k], g.origin[k], g.h, inv_h);
        if (!(f >= 0.0) || !(f < (double)g.dim)) return 0xFFFFFFFFu;
        idx[k] = (uint32_t)f;
    }
    return spread3(idx[0]) | (spread3(idx[1]) << 1) | (spread3(idx[2]) << 2);
}

__host__ __device__ inline int coarse_shift(const DGrid& g) { return g.log2dim < kCoarseShift ? g.log2dim : kCoarseShift; }
__host__ __device__ inline int64_t coarse_cells(const DGrid& g) {
    const int cl = g.log2dim - coarse_shift(g);
    return (int64_t)1 << (3 * cl);
}
__host__ __device__ inline uint32_t coarse_cell(const DGrid& g, uint32_t x, uint32_t y, uint32_t z) {
    const int cs = coarse_shift(g), cl = g.log2dim - cs;
    return (x >> cs) | ((y >> cs) << cl) | ((z >> cs) << (2 * cl));
}

// Sample kinds of the fusion loop: the thick path without / with footprint
// statistics, the differentiable variant, the NeRF path, the thin paths, or a
// per-session runtime choice (batches of mixed sessions).
enum FuseMode { kThick = 0, kThickNsamp = 1, kDiff = 2, kAnyMode = 3, kNerf = 4, kThin = 5, kNerfThin = 6,
                kAnyThin = 7 };  // kAnyMode: per-session choice without thin paths; kAnyThin: with them

// Partial counts are spread over kCountSlots addresses (no single hot atomic),
// two 32-bit fields packed per 64-bit word; launch_count_reduce sums them into
// counts[0..2] and stats[0..2] and clears them.  Slot q takes the chunks
// c = q mod kCountSlots: at most 2^26 chunks, so a slot sees at most 2^18, and
// every field's slot total (at most 2^12 per chunk) stays within 2^31 in
// magnitude, also as a signed change of resident outputs.
constexpr int kCountSlots = 256;
constexpr int kSlotWords = 8;
hipError_t launch_count_reduce(int64_t* slots, int64_t* counts, int64_t* stats, int64_t* tot, int delta,
                               hipStream_t st);

// ---- occupancy (occupancy.hip)
// Partitioning of the Morton range for the unit-opacity build.
struct OccPlan {
    int part_shift;      // log2(voxels per partition)
    int nparts;          // partitions (one workgroup each)
    int part_words;      // bitmap words per partition
    int tiles_per_part;  // compaction tiles (1024 words) per partition
};
OccPlan occupancy_plan(const DGrid& g);
// work: occupancy_work_bytes (partition tables, per-block partition
// histograms, codes, binned codes; no state is kept between builds).
// bitmap: the occupancy bits during the build, all zero on return (ready to
// serve as the empty segmentation bitfield).
// sort_scratch: occupancy_scratch_bytes(..., 1), general path only.
// n_act_host: device-visible pinned host memory receiving the count (or null);
// segb, coarse: the session's segmentation flags (whole chunks) and coarse cell
// counts, cleared for the new list (or null).
hipError_t launch_occupancy(const float* xyz, const float* opacity, int64_t n, double tau_occ,
                            const DGrid& g, uint32_t* bitmap, uint32_t* block_counts,
                            uint32_t* act, ChunkBox* chunk_box, int64_t* n_act_dev, int64_t* n_act_host,
                            uint8_t* segb, uint32_t* coarse, uint32_t* work,
                            void* sort_scratch, size_t sort_scratch_bytes, hipStream_t st, PhaseEvents ev = {},
                            double box_pad = 0.0);
size_t occupancy_work_bytes(const DGrid& g, int64_t max_points);
// The Morton codes of the n points of the last unit-opacity build in work
// (point order; 0xFFFFFFFF for a point outside the grid or with a NaN).
const uint32_t* occupancy_codes(const DGrid& g, const uint32_t* work, int64_t n);
size_t occupancy_scratch_bytes(const DGrid& g, int64_t max_points, int opacity_path);
hipError_t launch_fill_u32(uint32_t* p, uint32_t v, int64_t n, hipStream_t st);
// rho[a] = number of points in active voxel a (counts zeroed first; the list
// in Morton order, every in-grid point's voxel active)
hipError_t launch_voxel_density(const float* xyz, int64_t n, const DGrid& g, const uint32_t* act,
                                const int64_t* n_act, int64_t cap, uint32_t* rho, hipStream_t st);

// ---- per-view pre-pass (views.hip)
hipError_t launch_view_prepass(const DView* dviews, const DView* hviews, int32_t s_begin, int32_t s_end,
                               double mask_gate, int64_t* counters_to_zero, int n_counters, hipStream_t st,
                               PhaseEvents ev = {});

// ---- culling and fusion (fuse.hip)
hipError_t launch_cull(const ChunkBox* chunk_box, const int64_t* n_act, int64_t cap, const DGrid& g,
                       double eps, const DView* views, int32_t s_begin, int32_t s_end, uint64_t* cull,
                       hipStream_t st, PhaseEvents ev = {});
// fusion of every chunk, one wavefront per chunk (any_nsamp: some view of the
// fused range carries n_samp)
hipError_t launch_fuse(const FuseArgs& a, bool any_nsamp, hipStream_t st, PhaseEvents ev = {});
int pow2_at_least(int v);

// ---- labels (label.hip)
hipError_t launch_label(const float* xyz, int64_t n, const DGrid& g, const uint32_t* bits, const uint32_t* coarse,
                        uint8_t* labels, hipStream_t st, PhaseEvents ev = {});
// the same labels from the points' Morton codes (occupancy_codes)
hipError_t launch_label_codes(const uint32_t* codes, int64_t n, const DGrid& g, const uint32_t* bits,
                              const uint32_t* coarse, uint8_t* labels, hipStream_t st, PhaseEvents ev = {});

// ---- backward of the differentiable variant (backward.hip)
struct BwdArgs {
    const uint32_t* act;
    const int64_t* n_act;
    int64_t cap;
    DGrid g;
    DParams p;
    const DView* views;
    int32_t n_views;
    int32_t pad;
    const double* W;
    const double* Z;
    const float* gP;
    int64_t key_base[kMaxViews + 1];  // first (view, pixel) key of each view; key_base[n_views] = n_keys
    uint32_t* key_end;                // [n_keys]: counts, then offsets, then segment ends
    uint32_t* list;                   // voxel ranks grouped by key
    uint32_t* block_sums;
    float* grads[4][kMaxViews];       // d/dlogit, d/dmin, d/dref, d/dmax per view (null = skip)
};
hipError_t launch_backward(const BwdArgs& a, hipStream_t st);
size_t backward_block_sums(int64_t n_keys);

// ---- scene-statistic grid construction (selection.hip), Eq. scene-norm and
// Eq. voxel-size; synchronises the stream (the statistics feed one another)
struct GridStatsParams {
    double alpha_v, beta_v, pad, q;  // 3, 1, 1.05, 0.99
    int32_t g0, g_max;               // 256, 512 or 1024
};
struct GridStatsResult {
    double center[3];
    double r_fg, b, s_med, h_v;
    int32_t dim;  // 0: degenerate (zero extent or zero voxel edge)
    double origin[3];
    double voxel;
    int64_t m;  // points taking part (0: none)
    int64_t n_kept;
};
// scratch: device memory of grid_statistics_scratch(n) bytes
size_t grid_statistics_scratch(int64_t n);
hipError_t grid_statistics(const float* xyz, const float* scale, int64_t n, const GridStatsParams& p,
                           GridStatsResult* out, void* scratch, size_t scratch_bytes, hipStream_t st);

// ---- depth refinement of a view's mask (selection.hip), Eq. gs-bandpass and
// Eq. nerf-depthweight; synchronises the stream.  res->n_surface == 0 or (band
// pass) res->n_anchors == 0: nothing was written.
constexpr int kRefineBandPass = 0;
constexpr int kRefineMinMax = 1;
constexpr double kFarQuantile = 0.98;
struct RefineResult {
    double band_min, band_max, d_far, z_min, z_max;
    int64_t n_surface;
    int32_t n_anchors;
};
// scratch: device memory of refine_mask_scratch(width * height, n_prompts) bytes
size_t refine_mask_scratch(int64_t pixels, int32_t n_prompts);
hipError_t refine_mask(int kind, int32_t width, int32_t height, const float* mask, const float* depth,
                       const int32_t* prompts_xy, int32_t n_prompts, float* out, RefineResult* res, void* scratch,
                       size_t scratch_bytes, hipStream_t st);

// ---- needle cull, Pass 2 of the voxel-to-surfel mapping (selection.hip),
// Eq. aspect, Eq. needle, Eq. pass-needle; synchronises the stream.
// res->m == 0: no surfel has an aspect, nothing was written.
struct NeedleResult {
    double tau;
    int64_t m, n_culled;
};
size_t needle_cull_scratch(int64_t n, bool with_candidates = true);
hipError_t needle_cull(const float* scales, int64_t n, double eps, double q, uint8_t* labels, NeedleResult* res,
                       void* scratch, size_t scratch_bytes, hipStream_t st);

// ---- Pass 3 of the voxel-to-surfel mapping (surfel.hip): coverage kappa and
// labels of the surfels; kept (device int64, or null) receives the labels kept
hipError_t launch_surfel_coverage(const float* xyz, const float* scales, const float* quats, int64_t n,
                                  const uint8_t* labels_in, const DGrid& g, const uint32_t* act,
                                  const int64_t* n_act, const uint64_t* vmask, const DView* views, int32_t n_views,
                                  double tau_M, double tau_kappa, double eps, double* kappa, uint8_t* labels_out,
                                  int64_t* kept, hipStream_t st);

// ---- fixed device scratch (selection.hip) of the allocation-free needle
// cull: kStaticScratchBytes per device.  static_scratch_init (call it with
// `device` current) returns that device's copy's address, looked up once.
constexpr size_t kStaticScratchBytes = (size_t)32 << 20;
hipError_t static_scratch_init(int device, void** out);

// ---- shared scan (occupancy.hip): exclusive scan of uint32 in place
hipError_t launch_scan_u32(uint32_t* a, int64_t n, uint32_t* block_sums, int64_t* total, hipStream_t st);
size_t scan_block_sums(int64_t n);

}  // namespace divas
