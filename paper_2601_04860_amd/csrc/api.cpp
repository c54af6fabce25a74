// Host side of libdivas: the C ABI of include/divas.h.
//
// Validation happens before anything is enqueued; device state lives in
// sessions; every launch goes to the caller's stream.  No exception crosses the
// C boundary.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "../../include/divas.h"
#include "kernels.h"

using namespace divas;

namespace {

thread_local std::string g_last_error;

divas_status fail(divas_status st, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
divas_status fail(divas_status st, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return st;
}

bool is_finite(double x) { return std::isfinite(x); }

struct DeviceGuard {
    int prev = -1;
    explicit DeviceGuard(int dev) {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        if (prev != dev) (void)hipSetDevice(dev);
    }
    ~DeviceGuard() {
        if (prev >= 0) (void)hipSetDevice(prev);
    }
};

int ilog2(int v) {
    int l = 0;
    while ((1 << l) < v) ++l;
    return l;
}

}  // namespace

struct divas_ctx_s {
    int device = 0;
    size_t budget = 0;
    size_t used = 0;
    int sessions = 0;
};

struct divas_session_s {
    divas_ctx ctx = nullptr;
    divas_grid grid{};
    divas_params params{};
    DGrid g{};
    DParams p{};
    int64_t cap_points = 0;
    int64_t cap_act = 0;
    int64_t n_chunks = 0;
    int32_t max_views = 0;
    int64_t max_pix = 0;
    int64_t tile_stride = 0;
    int64_t sat_stride = 0;
    size_t footprint = 0;
    size_t lazy_bytes = 0;
    // device state
    uint32_t* bits = nullptr;          // occupancy bitmap during a rebuild, then the segmentation bitfield
    uint32_t* block_counts = nullptr;
    uint32_t* act = nullptr;
    uint16_t* chunk_box = nullptr;
    int64_t* counters = nullptr;       // [0] n_active, [1..3] scratch counts
    double* W = nullptr;
    double* Z = nullptr;
    uint64_t* vraw = nullptr;
    uint8_t* cull = nullptr;
    uint8_t* tiles = nullptr;
    DView* dviews = nullptr;
    uint64_t* sat = nullptr;           // lazily allocated integral images
    void* occ_scratch = nullptr;       // lazily allocated (general occupancy path)
    size_t occ_scratch_bytes = 0;
    // backward buffers (lazy)
    uint32_t* bw_count = nullptr;
    uint32_t* bw_list = nullptr;
    uint32_t* bw_sums = nullptr;
    int64_t* bw_keybase = nullptr;
    float** bw_ptrs = nullptr;
    int64_t bw_keys_cap = 0;
    int64_t bw_list_cap = 0;
    // host state
    std::vector<DView> hviews;
    int32_t n_views = 0;
    bool acc_valid = false;            // W, Z, vraw hold the fusion of views [0, n_views)
    bool fused = false;
    DView* staging = nullptr;          // pinned
    int64_t* host_counters = nullptr;  // pinned
    hipEvent_t built = nullptr;
    hipEvent_t staged = nullptr;
    bool poisoned = false;
};

namespace {

size_t round_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

struct Layout {
    int64_t cap_act, n_chunks, tile_stride, nwords, nblocks;
    size_t bytes;
};

Layout layout(const divas_grid* grid, int64_t max_points, int32_t max_views, int64_t max_pix, int32_t retain) {
    Layout L{};
    int64_t nvox = (int64_t)grid->dim * grid->dim * grid->dim;
    L.cap_act = std::max<int64_t>(1, std::min<int64_t>(max_points, nvox));
    L.n_chunks = (L.cap_act + kChunk - 1) / kChunk;
    L.tile_stride = max_pix / 8 + 2;
    L.nwords = std::max<int64_t>(1, (nvox + 31) / 32);
    L.nblocks = L.nwords / 1024 + 2;
    size_t b = 0;
    b += round_up((size_t)L.nwords * 4, 256);
    b += round_up((size_t)L.nblocks * 4, 256);
    b += round_up((size_t)L.cap_act * 4, 256);
    b += round_up((size_t)L.n_chunks * 16, 256);
    b += 256;  // counters
    if (retain) b += round_up((size_t)L.cap_act * 24, 256);
    b += round_up((size_t)L.n_chunks * max_views, 256);
    b += round_up((size_t)L.tile_stride * max_views, 256);
    b += round_up(sizeof(DView) * max_views, 256);
    L.bytes = b;
    return L;
}

divas_status check_grid(const divas_grid* g) {
    if (!g) return fail(DIVAS_ERR_ARG, "grid is NULL");
    if (g->dim < 2 || g->dim > 1024 || (g->dim & (g->dim - 1)) != 0)
        return fail(DIVAS_ERR_ARG, "grid dim %d must be a power of two in [2, 1024]", g->dim);
    if (!is_finite(g->voxel) || !(g->voxel > 0.0)) return fail(DIVAS_ERR_ARG, "grid voxel edge must be finite and > 0");
    for (int k = 0; k < 3; ++k)
        if (!is_finite(g->origin[k])) return fail(DIVAS_ERR_ARG, "grid origin must be finite");
    return DIVAS_OK;
}

divas_status check_params(const divas_params* p) {
    if (!p) return fail(DIVAS_ERR_ARG, "params is NULL");
    const double v[] = {p->gamma, p->beta, p->gamma_st, p->alpha1, p->k_grad, p->eps, p->tau_cons, p->mask_gate};
    for (double x : v)
        if (!is_finite(x)) return fail(DIVAS_ERR_ARG, "params must be finite");
    if (!(p->eps > 0.0)) return fail(DIVAS_ERR_ARG, "params.eps must be > 0");
    if (p->differentiable && !(is_finite(p->soft_width) && p->soft_width > 0.0))
        return fail(DIVAS_ERR_ARG, "params.soft_width must be finite and > 0 for the differentiable variant");
    return DIVAS_OK;
}

divas_status check_occ(const divas_occupancy* o) {
    if (!o) return fail(DIVAS_ERR_ARG, "occupancy is NULL");
    if (o->n < 0) return fail(DIVAS_ERR_ARG, "occupancy n < 0");
    if (o->n > 0 && !o->xyz) return fail(DIVAS_ERR_ARG, "occupancy xyz is NULL");
    if (o->n >= ((int64_t)1 << 32)) return fail(DIVAS_ERR_ARG, "occupancy n must be below 2^32");
    if (!is_finite(o->tau_occ) || !(o->tau_occ > 0.0)) return fail(DIVAS_ERR_ARG, "tau_occ must be finite and > 0");
    return DIVAS_OK;
}

divas_status check_view(const divas_session_s* s, const divas_camera* c, const divas_view_maps* m, bool diff) {
    if (!c || !m) return fail(DIVAS_ERR_ARG, "camera or maps is NULL");
    if (c->width <= 0 || c->height <= 0) return fail(DIVAS_ERR_ARG, "view size must be positive");
    if ((int64_t)c->width * c->height > s->max_pix)
        return fail(DIVAS_ERR_CAPACITY, "view %dx%d exceeds the session's max_view_pixels %lld", c->width, c->height,
                    (long long)s->max_pix);
    if (c->width > 65535 || c->height > 65535) return fail(DIVAS_ERR_ARG, "view side above 65535");
    const double v[] = {c->fx, c->fy, c->cx, c->cy, c->d_cam};
    for (double x : v)
        if (!is_finite(x)) return fail(DIVAS_ERR_ARG, "camera intrinsics / d_cam must be finite");
    if (!(c->fx > 0.0) || !(c->fy > 0.0)) return fail(DIVAS_ERR_ARG, "fx and fy must be > 0");
    for (int i = 0; i < 12; ++i)
        if (!is_finite(c->c2w[i])) return fail(DIVAS_ERR_ARG, "camera c2w must be finite");
    // rotation block must be orthonormal (to a loose tolerance)
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) {
            double d = 0;
            for (int r = 0; r < 3; ++r) d += c->c2w[r * 4 + a] * c->c2w[r * 4 + b];
            if (std::fabs(d - (a == b ? 1.0 : 0.0)) > 1e-6)
                return fail(DIVAS_ERR_ARG, "camera rotation block is not orthonormal");
        }
    if (!m->mask || !m->d_min || !m->d_ref || !m->d_max) return fail(DIVAS_ERR_ARG, "mask and depth maps are required");
    (void)diff;
    return DIVAS_OK;
}

void fill_view(divas_session_s* s, int slot, const divas_camera* c, const divas_view_maps* m) {
    DView& v = s->hviews[slot];
    std::memset(&v, 0, sizeof v);
    for (int b = 0; b < 3; ++b)
        for (int a = 0; a < 3; ++a) {
            v.R[b * 3 + a] = c->c2w[b * 4 + a];
            v.fR[b * 3 + a] = (float)c->c2w[b * 4 + a];
        }
    for (int b = 0; b < 3; ++b) {
        v.o[b] = c->c2w[b * 4 + 3];
        v.fo[b] = (float)v.o[b];
    }
    v.fx = c->fx;
    v.fy = c->fy;
    v.cx = c->cx;
    v.cy = c->cy;
    v.d_cam = c->d_cam;
    v.ffx = (float)c->fx;
    v.ffy = (float)c->fy;
    v.fcx = (float)c->cx;
    v.fcy = (float)c->cy;
    v.W = c->width;
    v.H = c->height;
    v.tw = (c->width + kTile - 1) / kTile;
    v.th = (c->height + kTile - 1) / kTile;
    v.mask = m->mask;
    v.dmin = m->d_min;
    v.dmed = m->d_ref;
    v.dmax = m->d_max;
    v.nsamp = s->params.differentiable ? nullptr : m->n_samp;
    v.tiles = s->tiles + (size_t)slot * s->tile_stride;
    if (v.nsamp && s->sat) {
        v.sat1 = s->sat + (size_t)slot * s->sat_stride * 2;
        v.sat2 = v.sat1 + s->sat_stride;
    }
}

#define HIPTRY(sess, expr)                                                                   \
    do {                                                                                     \
        hipError_t _e = (expr);                                                              \
        if (_e != hipSuccess) {                                                              \
            if (sess) (sess)->poisoned = true;                                               \
            return fail(DIVAS_ERR_DEVICE, "%s: %s (%s:%d)", #expr, hipGetErrorString(_e), __FILE__, \
                        __LINE__);                                                           \
        }                                                                                    \
    } while (0)

template <class T>
hipError_t dmalloc(T** p, size_t bytes) {
    return hipMalloc((void**)p, std::max<size_t>(bytes, 16));
}

void free_session(divas_session_s* s) {
    void* ptrs[] = {s->bits, s->block_counts, s->act, s->chunk_box, s->counters, s->W, s->Z, s->vraw, s->cull,
                    s->tiles, s->dviews, s->sat, s->occ_scratch, s->bw_count, s->bw_list, s->bw_sums,
                    s->bw_keybase, s->bw_ptrs};
    for (void* p : ptrs)
        if (p) (void)hipFree(p);
    if (s->staging) (void)hipHostFree(s->staging);
    if (s->host_counters) (void)hipHostFree(s->host_counters);
    if (s->built) (void)hipEventDestroy(s->built);
    if (s->staged) (void)hipEventDestroy(s->staged);
}

// Upload host view records [b, e) to the device through the pinned staging.
divas_status upload_views(divas_session_s* s, int b, int e, hipStream_t st) {
    if (e <= b) return DIVAS_OK;
    // the previous upload must have left the staging buffer
    HIPTRY(s, hipEventSynchronize(s->staged));
    std::memcpy(s->staging + b, s->hviews.data() + b, sizeof(DView) * (e - b));
    HIPTRY(s, hipMemcpyAsync(s->dviews + b, s->staging + b, sizeof(DView) * (e - b), hipMemcpyHostToDevice, st));
    HIPTRY(s, hipEventRecord(s->staged, st));
    return DIVAS_OK;
}

divas_status ensure_sat(divas_session_s* s) {
    if (s->sat) return DIVAS_OK;
    s->sat_stride = 2 * s->max_pix + 2;
    size_t bytes = (size_t)s->max_views * 2 * s->sat_stride * sizeof(uint64_t);
    if (s->ctx->budget && s->ctx->used + bytes > s->ctx->budget)
        return fail(DIVAS_ERR_ADMISSION, "integral images need %zu more bytes than the HBM budget allows", bytes);
    if (dmalloc(&s->sat, bytes) != hipSuccess) {
        s->sat = nullptr;
        return fail(DIVAS_ERR_OOM, "integral images: %zu bytes", bytes);
    }
    s->ctx->used += bytes;
    s->lazy_bytes += bytes;
    return DIVAS_OK;
}

double params_gate(const divas_session_s* s) { return s->params.differentiable ? -INFINITY : s->params.mask_gate; }

// Enqueue the pre-pass of views [b, e), the culling of those views, then the
// fusion of views [fb, fe) (fold = start from the resident accumulators).
divas_status enqueue_fusion(divas_session_s* s, int b, int e, int fb, int fe, bool fold, const divas_result* out,
                            hipStream_t st) {
    int64_t* counts = out && out->counts ? out->counts : s->counters + 1;
    HIPTRY(s, launch_view_prepass(s->dviews, s->hviews.data(), b, e, params_gate(s), counts, 3, st));
    if (s->sat) HIPTRY(s, launch_sat(s->dviews, s->hviews.data(), b, e, s->sat, s->sat_stride, st));
    HIPTRY(s, launch_cull(s->chunk_box, s->counters, s->cap_act, s->g, s->p.eps, s->dviews, b, e, s->cull,
                          s->max_views, st));
    FuseArgs a{};
    a.act = s->act;
    a.n_act = s->counters;
    a.cap = s->cap_act;
    a.g = s->g;
    a.p = s->p;
    a.views = s->dviews;
    a.s_begin = fb;
    a.s_end = fe;
    a.cull = s->cull;
    a.cull_stride = s->max_views;
    a.load_acc = fold ? 1 : 0;
    a.store_acc = s->W ? 1 : 0;
    a.W = s->W;
    a.Z = s->Z;
    a.vraw = s->vraw;
    a.P = out->P;
    a.vout = out->vmask;
    a.bits = s->bits;
    a.counts = counts;
    HIPTRY(s, launch_fuse(a, st));
    if (out->seg_bits) {
        size_t nw = (size_t)std::max<int64_t>(1, ((int64_t)s->grid.dim * s->grid.dim * s->grid.dim + 31) / 32);
        HIPTRY(s, hipMemcpyAsync(out->seg_bits, s->bits, nw * 4, hipMemcpyDeviceToDevice, st));
    }
    return DIVAS_OK;
}

}  // namespace

extern "C" {

const char* divas_status_string(divas_status st) {
    switch (st) {
        case DIVAS_OK: return "ok";
        case DIVAS_ERR_ARG: return "invalid argument";
        case DIVAS_ERR_OOM: return "device out of memory";
        case DIVAS_ERR_ADMISSION: return "HBM budget exceeded (admission denied)";
        case DIVAS_ERR_TOO_MANY_VIEWS: return "too many views (at most 64)";
        case DIVAS_ERR_STATE: return "invalid session state";
        case DIVAS_ERR_DEVICE: return "HIP device error";
        case DIVAS_ERR_CAPACITY: return "input exceeds the session capacity";
    }
    return "unknown status";
}

const char* divas_last_error(void) { return g_last_error.c_str(); }

divas_status divas_params_default(double voxel, divas_params* out) {
    if (!out) return fail(DIVAS_ERR_ARG, "out is NULL");
    if (!is_finite(voxel) || !(voxel > 0.0)) return fail(DIVAS_ERR_ARG, "voxel must be finite and > 0");
    std::memset(out, 0, sizeof *out);
    out->gamma = 1.0;
    out->beta = 0.05;
    out->gamma_st = 1.5;
    out->alpha1 = 1.0;
    out->k_grad = 1.0 / (4.0 * voxel * voxel);
    out->eps = 1e-6;
    out->tau_cons = 0.5;
    out->mask_gate = 0.5;
    out->soft_width = 0.01;
    out->differentiable = 0;
    out->retain_state = 0;
    return DIVAS_OK;
}

divas_status divas_ctx_create(int device, size_t budget, divas_ctx* out) {
    if (!out) return fail(DIVAS_ERR_ARG, "out is NULL");
    *out = nullptr;
    int n = 0;
    hipError_t e = hipGetDeviceCount(&n);
    if (e != hipSuccess || n <= 0) return fail(DIVAS_ERR_DEVICE, "no HIP device available");
    if (device < 0 || device >= n) return fail(DIVAS_ERR_ARG, "device %d out of range [0, %d)", device, n);
    divas_ctx c = new (std::nothrow) divas_ctx_s;
    if (!c) return fail(DIVAS_ERR_OOM, "host allocation failed");
    c->device = device;
    c->budget = budget;
    *out = c;
    return DIVAS_OK;
}

divas_status divas_ctx_destroy(divas_ctx ctx) {
    if (!ctx) return fail(DIVAS_ERR_ARG, "ctx is NULL");
    if (ctx->sessions > 0) return fail(DIVAS_ERR_STATE, "%d sessions still alive", ctx->sessions);
    delete ctx;
    return DIVAS_OK;
}

divas_status divas_ctx_usage(divas_ctx ctx, size_t* used, size_t* budget) {
    if (!ctx) return fail(DIVAS_ERR_ARG, "ctx is NULL");
    if (used) *used = ctx->used;
    if (budget) *budget = ctx->budget;
    return DIVAS_OK;
}

size_t divas_session_footprint(const divas_grid* grid, int64_t max_points, int32_t max_views,
                               int64_t max_view_pixels, int32_t retain_state) {
    if (check_grid(grid) != DIVAS_OK || max_points < 0 || max_views < 1 || max_views > DIVAS_MAX_VIEWS ||
        max_view_pixels < 1)
        return 0;
    return layout(grid, max_points, max_views, max_view_pixels, retain_state).bytes;
}

divas_status divas_session_rebuild(divas_session s, const divas_occupancy* occ, divas_stream stream);

divas_status divas_session_create(divas_ctx ctx, const divas_grid* grid, const divas_occupancy* occ,
                                  const divas_params* params, int64_t max_points, int32_t max_views,
                                  int64_t max_view_pixels, divas_stream stream, divas_session* out) {
    if (!out) return fail(DIVAS_ERR_ARG, "out is NULL");
    *out = nullptr;
    if (!ctx) return fail(DIVAS_ERR_ARG, "ctx is NULL");
    divas_status st;
    if ((st = check_grid(grid)) != DIVAS_OK) return st;
    if ((st = check_occ(occ)) != DIVAS_OK) return st;
    if ((st = check_params(params)) != DIVAS_OK) return st;
    if (max_views > DIVAS_MAX_VIEWS) return fail(DIVAS_ERR_TOO_MANY_VIEWS, "max_views %d > 64", max_views);
    if (max_views < 1) return fail(DIVAS_ERR_ARG, "max_views must be >= 1");
    if (max_view_pixels < 1) return fail(DIVAS_ERR_ARG, "max_view_pixels must be >= 1");
    if (max_points == 0) max_points = occ->n;
    if (max_points < occ->n)
        return fail(DIVAS_ERR_CAPACITY, "%lld points exceed max_points %lld", (long long)occ->n, (long long)max_points);
    if (max_points >= ((int64_t)1 << 32)) return fail(DIVAS_ERR_ARG, "max_points must be below 2^32");
    bool retain = params->retain_state || params->differentiable;
    Layout L = layout(grid, max_points, max_views, max_view_pixels, retain);
    if (ctx->budget && ctx->used + L.bytes > ctx->budget)
        return fail(DIVAS_ERR_ADMISSION, "session needs %zu bytes, %zu of %zu in use", L.bytes, ctx->used,
                    ctx->budget);
    DeviceGuard dg(ctx->device);
    divas_session s = new (std::nothrow) divas_session_s;
    if (!s) return fail(DIVAS_ERR_OOM, "host allocation failed");
    s->ctx = ctx;
    s->grid = *grid;
    s->params = *params;
    s->g.origin[0] = grid->origin[0];
    s->g.origin[1] = grid->origin[1];
    s->g.origin[2] = grid->origin[2];
    s->g.h = grid->voxel;
    s->g.dim = grid->dim;
    s->g.log2dim = ilog2(grid->dim);
    s->p = DParams{params->gamma, params->beta, params->gamma_st, params->alpha1, params->k_grad, params->eps,
                   params->tau_cons, params->mask_gate, params->soft_width, params->differentiable, 0};
    s->cap_points = max_points;
    s->cap_act = L.cap_act;
    s->n_chunks = L.n_chunks;
    s->max_views = max_views;
    s->max_pix = max_view_pixels;
    s->tile_stride = L.tile_stride;
    s->footprint = L.bytes;
    s->hviews.resize(max_views);
    bool ok = dmalloc(&s->bits, (size_t)L.nwords * 4) == hipSuccess &&
              dmalloc(&s->block_counts, (size_t)L.nblocks * 4) == hipSuccess &&
              dmalloc(&s->act, (size_t)L.cap_act * 4) == hipSuccess &&
              dmalloc(&s->chunk_box, (size_t)L.n_chunks * 16) == hipSuccess &&
              dmalloc(&s->counters, 8 * sizeof(int64_t)) == hipSuccess &&
              dmalloc(&s->cull, (size_t)L.n_chunks * max_views) == hipSuccess &&
              dmalloc(&s->tiles, (size_t)L.tile_stride * max_views) == hipSuccess &&
              dmalloc(&s->dviews, sizeof(DView) * max_views) == hipSuccess &&
              hipHostMalloc((void**)&s->staging, sizeof(DView) * max_views, hipHostMallocDefault) == hipSuccess &&
              hipHostMalloc((void**)&s->host_counters, 8 * sizeof(int64_t), hipHostMallocDefault) == hipSuccess &&
              hipEventCreateWithFlags(&s->built, hipEventDisableTiming) == hipSuccess &&
              hipEventCreateWithFlags(&s->staged, hipEventDisableTiming) == hipSuccess;
    if (ok && retain)
        ok = dmalloc(&s->W, (size_t)L.cap_act * 8) == hipSuccess && dmalloc(&s->Z, (size_t)L.cap_act * 8) == hipSuccess &&
             dmalloc(&s->vraw, (size_t)L.cap_act * 8) == hipSuccess;
    if (!ok) {
        (void)hipGetLastError();
        free_session(s);
        delete s;
        return fail(DIVAS_ERR_OOM, "device allocation of %zu bytes failed", L.bytes);
    }
    (void)hipEventRecord(s->staged, (hipStream_t)stream);
    ctx->used += L.bytes;
    ctx->sessions += 1;
    st = divas_session_rebuild(s, occ, stream);
    if (st != DIVAS_OK) {
        std::string msg = g_last_error;
        (void)hipStreamSynchronize((hipStream_t)stream);
        ctx->used -= s->footprint + s->lazy_bytes;
        ctx->sessions -= 1;
        free_session(s);
        delete s;
        g_last_error = msg;
        return st;
    }
    *out = s;
    return DIVAS_OK;
}

divas_status divas_session_rebuild(divas_session s, const divas_occupancy* occ, divas_stream stream) {
    if (!s) return fail(DIVAS_ERR_ARG, "session is NULL");
    if (s->poisoned) return fail(DIVAS_ERR_STATE, "session is poisoned by an earlier device error");
    divas_status st;
    if ((st = check_occ(occ)) != DIVAS_OK) return st;
    if (occ->n > s->cap_points)
        return fail(DIVAS_ERR_CAPACITY, "%lld points exceed the session capacity %lld", (long long)occ->n,
                    (long long)s->cap_points);
    DeviceGuard dg(s->ctx->device);
    hipStream_t hs = (hipStream_t)stream;
    bool general = occ->opacity != nullptr || occ->tau_occ > 1.0;
    if (general && !s->occ_scratch) {
        size_t bytes = occupancy_scratch_bytes(s->g, s->cap_points, 1);
        if (s->ctx->budget && s->ctx->used + bytes > s->ctx->budget)
            return fail(DIVAS_ERR_ADMISSION, "occupancy sort needs %zu more bytes than the budget allows", bytes);
        if (dmalloc(&s->occ_scratch, bytes) != hipSuccess) {
            s->occ_scratch = nullptr;
            (void)hipGetLastError();
            return fail(DIVAS_ERR_OOM, "occupancy sort scratch: %zu bytes", bytes);
        }
        s->occ_scratch_bytes = bytes;
        s->ctx->used += bytes;
        s->lazy_bytes += bytes;
    }
    int64_t nwords = std::max<int64_t>(1, ((int64_t)s->grid.dim * s->grid.dim * s->grid.dim + 31) / 32);
    HIPTRY(s, launch_occupancy(occ->xyz, occ->opacity, occ->n, occ->tau_occ, s->g, s->bits, s->block_counts, s->act,
                               s->chunk_box, s->counters, s->occ_scratch, s->occ_scratch_bytes, hs));
    // the occupancy bitmap becomes the (empty) segmentation bitfield
    HIPTRY(s, launch_fill_u32(s->bits, 0u, nwords, hs));
    HIPTRY(s, hipMemcpyAsync(s->host_counters, s->counters, sizeof(int64_t), hipMemcpyDeviceToHost, hs));
    HIPTRY(s, hipEventRecord(s->built, hs));
    s->n_views = 0;
    s->acc_valid = false;
    s->fused = false;
    return DIVAS_OK;
}

divas_status divas_session_info(divas_session s, int64_t* n_active, const uint32_t** act, int32_t* n_views,
                                size_t* footprint) {
    if (!s) return fail(DIVAS_ERR_ARG, "session is NULL");
    if (n_active) {
        DeviceGuard dg(s->ctx->device);
        HIPTRY(s, hipEventSynchronize(s->built));
        *n_active = s->host_counters[0];
    }
    if (act) *act = s->act;
    if (n_views) *n_views = s->n_views;
    if (footprint) *footprint = s->footprint + s->lazy_bytes;
    return DIVAS_OK;
}

divas_status divas_fuse_views(divas_session s, int32_t n_views, const divas_camera* cams, const divas_view_maps* maps,
                              const divas_result* out, divas_stream stream) {
    if (!s) return fail(DIVAS_ERR_ARG, "session is NULL");
    if (s->poisoned) return fail(DIVAS_ERR_STATE, "session is poisoned by an earlier device error");
    if (n_views > DIVAS_MAX_VIEWS) return fail(DIVAS_ERR_TOO_MANY_VIEWS, "%d views > 64", n_views);
    if (n_views < 0) return fail(DIVAS_ERR_ARG, "n_views < 0");
    if (n_views > s->max_views)
        return fail(DIVAS_ERR_CAPACITY, "%d views exceed the session's max_views %d", n_views, s->max_views);
    if (n_views > 0 && (!cams || !maps)) return fail(DIVAS_ERR_ARG, "cams / maps is NULL");
    if (!out || !out->P || !out->vmask) return fail(DIVAS_ERR_ARG, "result P and vmask are required");
    divas_status st;
    for (int i = 0; i < n_views; ++i)
        if ((st = check_view(s, &cams[i], &maps[i], s->params.differentiable)) != DIVAS_OK) return st;
    bool need_sat = false;
    for (int i = 0; i < n_views; ++i) need_sat |= maps[i].n_samp != nullptr && !s->params.differentiable;
    DeviceGuard dg(s->ctx->device);
    if (need_sat && (st = ensure_sat(s)) != DIVAS_OK) return st;
    hipStream_t hs = (hipStream_t)stream;
    for (int i = 0; i < n_views; ++i) fill_view(s, i, &cams[i], &maps[i]);
    if ((st = upload_views(s, 0, n_views, hs)) != DIVAS_OK) return st;
    if ((st = enqueue_fusion(s, 0, n_views, 0, n_views, false, out, hs)) != DIVAS_OK) return st;
    s->n_views = n_views;
    s->acc_valid = s->W != nullptr;
    s->fused = true;
    return DIVAS_OK;
}

divas_status divas_update_view(divas_session s, int32_t slot, const divas_camera* cam, const divas_view_maps* maps,
                               const divas_result* out, divas_stream stream) {
    if (!s) return fail(DIVAS_ERR_ARG, "session is NULL");
    if (s->poisoned) return fail(DIVAS_ERR_STATE, "session is poisoned by an earlier device error");
    if (slot < 0 || slot > s->n_views) return fail(DIVAS_ERR_ARG, "slot %d outside [0, %d]", slot, s->n_views);
    if (slot >= DIVAS_MAX_VIEWS) return fail(DIVAS_ERR_TOO_MANY_VIEWS, "slot %d: at most 64 views", slot);
    if (slot >= s->max_views)
        return fail(DIVAS_ERR_CAPACITY, "slot %d exceeds the session's max_views %d", slot, s->max_views);
    if (!out || !out->P || !out->vmask) return fail(DIVAS_ERR_ARG, "result P and vmask are required");
    divas_status st;
    if ((st = check_view(s, cam, maps, s->params.differentiable)) != DIVAS_OK) return st;
    DeviceGuard dg(s->ctx->device);
    if (maps->n_samp && !s->params.differentiable && (st = ensure_sat(s)) != DIVAS_OK) return st;
    hipStream_t hs = (hipStream_t)stream;
    bool append = slot == s->n_views;
    bool fold = append && s->acc_valid && s->fused;
    fill_view(s, slot, cam, maps);
    if (s->sat)  // integral-image pointers of earlier views stay valid; refresh all records
        for (int i = 0; i < s->n_views; ++i)
            if (s->hviews[i].nsamp && !s->hviews[i].sat1) {
                s->hviews[i].sat1 = s->sat + (size_t)i * s->sat_stride * 2;
                s->hviews[i].sat2 = s->hviews[i].sat1 + s->sat_stride;
            }
    if ((st = upload_views(s, 0, std::max(slot + 1, s->n_views), hs)) != DIVAS_OK) return st;
    int nv = append ? s->n_views + 1 : s->n_views;
    if (fold)
        st = enqueue_fusion(s, slot, slot + 1, slot, slot + 1, true, out, hs);
    else
        st = enqueue_fusion(s, slot, slot + 1, 0, nv, false, out, hs);
    if (st != DIVAS_OK) return st;
    s->n_views = nv;
    s->acc_valid = s->W != nullptr;
    s->fused = true;
    return DIVAS_OK;
}

divas_status divas_label_points(divas_session s, const float* xyz, int64_t n, uint8_t* labels, divas_stream stream) {
    if (!s) return fail(DIVAS_ERR_ARG, "session is NULL");
    if (s->poisoned) return fail(DIVAS_ERR_STATE, "session is poisoned by an earlier device error");
    if (n < 0) return fail(DIVAS_ERR_ARG, "n < 0");
    if (n > 0 && (!xyz || !labels)) return fail(DIVAS_ERR_ARG, "xyz / labels is NULL");
    DeviceGuard dg(s->ctx->device);
    HIPTRY(s, launch_label(xyz, n, s->g, s->bits, labels, (hipStream_t)stream));
    return DIVAS_OK;
}

divas_status divas_fuse_backward(divas_session s, const float* grad_P, float* const* grad_logit,
                                 float* const* grad_dmin, float* const* grad_dref, float* const* grad_dmax,
                                 divas_stream stream) {
    if (!s) return fail(DIVAS_ERR_ARG, "session is NULL");
    if (s->poisoned) return fail(DIVAS_ERR_STATE, "session is poisoned by an earlier device error");
    if (!s->params.differentiable) return fail(DIVAS_ERR_STATE, "session was not created with differentiable = 1");
    if (!s->fused || !s->acc_valid) return fail(DIVAS_ERR_STATE, "no forward fusion to differentiate");
    if (!grad_P) return fail(DIVAS_ERR_ARG, "grad_P is NULL");
    DeviceGuard dg(s->ctx->device);
    hipStream_t hs = (hipStream_t)stream;
    BwdArgs a{};
    int64_t nk = 0;
    for (int v = 0; v < s->n_views; ++v) {
        a.key_base[v] = nk;
        nk += (int64_t)s->hviews[v].W * s->hviews[v].H;
    }
    a.key_base[s->n_views] = nk;
    if (nk >= ((int64_t)1 << 32)) return fail(DIVAS_ERR_CAPACITY, "too many pixels for the backward pass");
    int64_t keys_cap = (int64_t)s->max_views * s->max_pix;
    int64_t list_cap = s->cap_act * (int64_t)s->max_views;
    if (!s->bw_count) {
        size_t bytes = (size_t)(keys_cap + 1) * 4 + (size_t)list_cap * 4 + backward_block_sums(keys_cap) * 4;
        if (s->ctx->budget && s->ctx->used + bytes > s->ctx->budget)
            return fail(DIVAS_ERR_ADMISSION, "backward buffers need %zu more bytes than the budget allows", bytes);
        if (dmalloc(&s->bw_count, (size_t)(keys_cap + 1) * 4) != hipSuccess ||
            dmalloc(&s->bw_list, (size_t)list_cap * 4) != hipSuccess ||
            dmalloc(&s->bw_sums, backward_block_sums(keys_cap) * 4) != hipSuccess) {
            (void)hipGetLastError();
            if (s->bw_count) (void)hipFree(s->bw_count);
            if (s->bw_list) (void)hipFree(s->bw_list);
            if (s->bw_sums) (void)hipFree(s->bw_sums);
            s->bw_count = s->bw_list = s->bw_sums = nullptr;
            return fail(DIVAS_ERR_OOM, "backward buffers: %zu bytes", bytes);
        }
        s->ctx->used += bytes;
        s->lazy_bytes += bytes;
    }
    a.act = s->act;
    a.n_act = s->counters;
    a.cap = s->cap_act;
    a.g = s->g;
    a.p = s->p;
    a.views = s->dviews;
    a.n_views = s->n_views;
    a.W = s->W;
    a.Z = s->Z;
    a.gP = grad_P;
    a.key_end = s->bw_count;
    a.list = s->bw_list;
    a.block_sums = s->bw_sums;
    float* const* arrs[4] = {grad_logit, grad_dmin, grad_dref, grad_dmax};
    for (int k = 0; k < 4; ++k)
        for (int v = 0; v < s->n_views; ++v) a.grads[k][v] = arrs[k] ? arrs[k][v] : nullptr;
    HIPTRY(s, launch_backward(a, hs));
    return DIVAS_OK;
}

divas_status divas_session_destroy(divas_session s) {
    if (!s) return fail(DIVAS_ERR_ARG, "session is NULL");
    DeviceGuard dg(s->ctx->device);
    (void)hipDeviceSynchronize();
    s->ctx->used -= s->footprint + s->lazy_bytes;
    s->ctx->sessions -= 1;
    free_session(s);
    delete s;
    return DIVAS_OK;
}

}  // extern "C"
