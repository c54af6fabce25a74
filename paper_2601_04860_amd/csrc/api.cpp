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
#include <fstream>
#include <map>
#include <set>
#include <sstream>
#include <new>
#include <string>
#include <vector>

#include "../../include/divas.h"
#include "batch.h"
#include "kernels.h"
#include "targets.h"

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
    void* scratch = nullptr;  // device scratch of the synchronous pre-pass calls, grown on demand
    size_t scratch_bytes = 0;
    void* static_scratch = nullptr;  // the device's fixed scratch array (allocation-free calls)
};

namespace {
// The context's scratch, at least `bytes` long (grown by reallocation; the
// calls that use it wait for their own work, so one buffer serves them all).
hipError_t ctx_scratch(divas_ctx c, size_t bytes, void** out) {
    if (c->scratch_bytes < bytes) {
        const size_t want = std::max(bytes, c->scratch_bytes + c->scratch_bytes / 2);
        if (c->scratch) (void)hipFree(c->scratch);
        c->scratch = nullptr;
        c->scratch_bytes = 0;
        hipError_t e = hipMalloc(&c->scratch, want);
        if (e != hipSuccess) return e;
        c->scratch_bytes = want;
    }
    *out = c->scratch;
    return hipSuccess;
}
}  // namespace

struct divas_session_s {
    divas_ctx ctx = nullptr;
    divas_grid grid{};
    divas_params params{};
    DGrid g{};
    DParams p{};
    int64_t cap_points = 0;
    int64_t occ_points = 0;   // points of the last occupancy build
    bool occ_codes = false;   // that build kept each point's voxel code (unit opacity, tau_occ <= 1)
    int64_t cap_act = 0;
    int64_t n_chunks = 0;
    int32_t max_views = 0;
    int64_t max_pix = 0;
    int64_t tile_stride = 0;
    size_t footprint = 0;
    size_t lazy_bytes = 0;
    // device state
    uint32_t* bits = nullptr;          // occupancy bitmap during a rebuild, then the segmentation bitfield
    uint32_t* coarse = nullptr;        // segmented voxels per coarse cell
    uint32_t* block_counts = nullptr;
    uint32_t* occ_work = nullptr;      // unit-opacity occupancy build (codes, bins, partition tables)
    uint32_t* act = nullptr;
    ChunkBox* chunk_box = nullptr;
    int64_t* counters = nullptr;       // [0] n_active, [1..3] scratch counts, [4..6] work of the last fusion,
                                       // [8..10] running totals of the counts (resident outputs)
    int64_t* slots = nullptr;          // [kCountSlots * kSlotWords] partial counts of a fusion (zero between fusions)
    double* W = nullptr;
    double* Z = nullptr;
    uint64_t* vraw = nullptr;
    uint64_t* cull = nullptr;          // [chunk] view bits of the culling
    uint8_t* segb = nullptr;           // [cap_act] previous segmentation
    // target sessions: the session whose scene geometry (active list, chunk
    // boxes, point counts, n_active) this one shares; bases: how many targets
    divas_session_s* base = nullptr;
    int32_t n_targets = 0;
    TargetArgs* targ_dev = nullptr;    // multi-target fusion led by this session: device table,
    TargetArgs* targ_host = nullptr;   // its pinned staging,
    hipEvent_t targ_staged = nullptr;  // and the copy of the last one
    uint32_t* rho = nullptr;           // [cap_act] points per active voxel (thin-structure fallback only)
    uint8_t* tiles = nullptr;          // per-view hot-tile tables
    DView* dviews = nullptr;
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
    std::vector<DView> dmirror;        // the device view records as last uploaded
    std::vector<char> dmirror_ok;      // [slot]: dmirror holds the device record
    hipStream_t staged_stream = nullptr;  // stream of the last upload (event `staged`)
    int32_t n_views = 0;
    bool acc_valid = false;            // W, Z, vraw hold the fusion of views [0, n_views)
    bool fused = false;
    uint64_t generation = 0;           // bumped by every call that changes the fused state
    // the outputs of the last fusion call and the generation it left (resident
    // outputs), and whether the running count totals belong to it
    const float* out_P = nullptr;
    const uint64_t* out_vm = nullptr;
    uint64_t out_gen = 0;
    bool tot_valid = false;
    DView* staging = nullptr;          // pinned
    int64_t* host_counters = nullptr;  // pinned
    int64_t* host_counters_dev = nullptr;  // the same memory as seen by the device
    hipEvent_t built = nullptr;
    hipEvent_t staged = nullptr;
    bool poisoned = false;
    // phase timing: bit p set = phase p is timed
    uint32_t timing = 0;
    struct Rec {
        int phase;
        hipEvent_t a, b;
    };
    std::vector<Rec> pending;
    std::vector<hipEvent_t> pool;
    double acc_ms[DIVAS_PHASE_COUNT] = {0};
    int64_t acc_n[DIVAS_PHASE_COUNT] = {0};
};

namespace {

size_t round_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

// Per-view tile region: the hot-tile words, th rows of ceil(tw / 64) uint64,
// then the gate bitmask.  For W x H = P pixels the words take at most P + 8
// bytes (tw <= 64: 8 th <= H + 7; tw > 64: 8 th ceil(tw / 64) <= th tw / 4
// <= P / 16), the bitmask tw * H <= W * H = P bytes.
size_t tile_word_bytes(int64_t max_pix) { return round_up((size_t)max_pix + 64, 256); }
size_t tile_region_bytes(int64_t max_pix) { return tile_word_bytes(max_pix) + round_up((size_t)max_pix, 256); }

hipEvent_t take_event(divas_session_s* s) {
    if (!s->pool.empty()) {
        hipEvent_t e = s->pool.back();
        s->pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

void resolve_timings(divas_session_s* s) {
    for (auto& r : s->pending) {
        float ms = 0.f;
        if (hipEventSynchronize(r.b) == hipSuccess && hipEventElapsedTime(&ms, r.a, r.b) == hipSuccess) {
            s->acc_ms[r.phase] += ms;
            s->acc_n[r.phase] += 1;
        }
        s->pool.push_back(r.a);
        s->pool.push_back(r.b);
    }
    s->pending.clear();
}

// Times one phase when its bit is set in the session's timing mask.  Kernel
// phases take the pair of events with ev() and hand it to their launcher,
// which attaches the events to the dispatches of its first and last kernel
// (no packet is added to the stream); a scope whose ev() is not called
// brackets its launches with recorded events instead.
struct PhaseScope {
    divas_session_s* s;
    int phase;
    hipStream_t st;
    hipEvent_t a = nullptr, b = nullptr;
    bool attached = false;
    PhaseScope(divas_session_s* s_, int ph, hipStream_t st_, bool kernel_events = false)
        : s(s_), phase(ph), st(st_), attached(kernel_events) {
        if (!((s->timing >> ph) & 1)) return;
        if (s->pending.size() >= 8192) resolve_timings(s);
        a = take_event(s);
        b = take_event(s);
        if (!a || !b || (!attached && hipEventRecord(a, st) != hipSuccess)) release();
    }
    PhaseEvents ev() const { return attached ? PhaseEvents{a, b} : PhaseEvents{}; }
    void release() {
        if (a) s->pool.push_back(a);
        if (b) s->pool.push_back(b);
        a = b = nullptr;
    }
    ~PhaseScope() {
        if (!a) return;
        if (!attached && hipEventRecord(b, st) != hipSuccess) {
            release();
            return;
        }
        s->pending.push_back({phase, a, b});
    }
};

struct Layout {
    int64_t cap_act, n_chunks, tile_stride, nwords, nblocks, ncoarse;
    size_t occ_work;
    size_t bytes;
};

Layout layout(const divas_grid* grid, int64_t max_points, int32_t max_views, int64_t max_pix, int32_t retain) {
    Layout L{};
    int64_t nvox = (int64_t)grid->dim * grid->dim * grid->dim;
    L.cap_act = std::max<int64_t>(1, std::min<int64_t>(max_points, nvox));
    L.n_chunks = (L.cap_act + kChunk - 1) / kChunk;
    L.tile_stride = (int64_t)tile_region_bytes(max_pix);
    L.nwords = std::max<int64_t>(1, (nvox + 31) / 32);
    L.nblocks = L.nwords / 1024 + 2;
    {
        DGrid g{};
        g.dim = grid->dim;
        g.log2dim = ilog2(grid->dim);
        L.ncoarse = coarse_cells(g);
    }
    {
        DGrid g{};
        g.dim = grid->dim;
        g.log2dim = ilog2(grid->dim);
        L.occ_work = occupancy_work_bytes(g, max_points);
    }
    size_t b = 0;
    b += round_up((size_t)L.nwords * 4, 256);
    b += round_up((size_t)L.ncoarse * 4, 256);
    b += round_up((size_t)L.nblocks * 4, 256);
    b += round_up(L.occ_work, 256);
    b += round_up(round_up((size_t)L.cap_act, kChunk) * 4, 256);  // active list, whole chunks
    b += round_up((size_t)L.n_chunks * sizeof(ChunkBox), 256);
    b += 256;  // counters
    b += round_up(kCountSlots * kSlotWords * sizeof(int64_t), 256);
    if (retain) b += round_up((size_t)L.cap_act * 24, 256);
    b += round_up((size_t)L.n_chunks * 8, 256);
    b += round_up((size_t)L.cap_act, 256) + 256;
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
    if (p->variant != kVariant2DGS && p->variant != kVariantNerf) return fail(DIVAS_ERR_ARG, "params.variant must be 0 or 1");
    if (p->thin != 0 && p->thin != 1) return fail(DIVAS_ERR_ARG, "params.thin must be 0 or 1");
    if (p->thin) {
        if (p->differentiable) return fail(DIVAS_ERR_ARG, "the thin-structure path has no differentiable form");
        const double t[] = {p->rho_thin, p->tau_thin, p->rho_cover, p->rho_occ, p->n_abs};
        for (double x : t)
            if (!is_finite(x) || !(x >= 0.0)) return fail(DIVAS_ERR_ARG, "thin-path constants must be finite and >= 0");
        // a score of 0 must not vote: the chunk cull relies on a thin vote
        // needing a footprint pixel with a mask value above 0
        if (!(p->tau_thin > 0.0)) return fail(DIVAS_ERR_ARG, "params.tau_thin must be > 0");
    }
    if (p->nerf_ray_depths != 0 && p->nerf_ray_depths != 1)
        return fail(DIVAS_ERR_ARG, "params.nerf_ray_depths must be 0 or 1");
    if (p->resident_outputs != 0 && p->resident_outputs != 1)
        return fail(DIVAS_ERR_ARG, "params.resident_outputs must be 0 or 1");
    if (p->variant == kVariantNerf) {
        if (p->differentiable) return fail(DIVAS_ERR_ARG, "the NeRF variant has no differentiable form");
        if (!is_finite(p->lambda_range) || !(p->lambda_range >= 0.0) || !is_finite(p->b_max) || !(p->b_max >= 0.0))
            return fail(DIVAS_ERR_ARG, "params.lambda_range and params.b_max must be finite and >= 0");
    }
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
    v.tile_bits = (uint64_t*)(s->tiles + (size_t)slot * s->tile_stride);
    v.mbits = (uint8_t*)(s->tiles + (size_t)slot * s->tile_stride + tile_word_bytes(s->max_pix));
    v.mpitch = v.tw;
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
    void* ptrs[] = {s->bits, s->block_counts, s->occ_work, s->act, s->chunk_box, s->counters, s->slots, s->coarse, s->W, s->Z, s->vraw, s->cull, s->segb, s->rho,
                    s->tiles, s->dviews, s->occ_scratch, s->bw_count, s->bw_list, s->bw_sums,
                    s->bw_keybase, s->bw_ptrs};
    for (void* p : ptrs)
        if (p) (void)hipFree(p);
    if (s->staging) (void)hipHostFree(s->staging);
    if (s->host_counters) (void)hipHostFree(s->host_counters);
    if (s->built) (void)hipEventDestroy(s->built);
    if (s->staged) (void)hipEventDestroy(s->staged);
}

// Upload host view records [b, e) to the device through the pinned staging,
// unless the last upload already brought every one of them (a repeated fusion
// of the same views then issues no copy and does not wait for the previous
// one; on another stream it waits for that upload on the device).
divas_status upload_views(divas_session_s* s, int b, int e, hipStream_t st) {
    if (e <= b) return DIVAS_OK;
    bool same = true;
    for (int k = b; k < e && same; ++k)
        same = s->dmirror_ok[k] && std::memcmp(&s->dmirror[k], &s->hviews[k], sizeof(DView)) == 0;
    if (same) {
        if (st != s->staged_stream) HIPTRY(s, hipStreamWaitEvent(st, s->staged, 0));
        return DIVAS_OK;
    }
    // the previous upload must have left the staging buffer
    HIPTRY(s, hipEventSynchronize(s->staged));
    std::memcpy(s->staging + b, s->hviews.data() + b, sizeof(DView) * (e - b));
    HIPTRY(s, hipMemcpyAsync(s->dviews + b, s->staging + b, sizeof(DView) * (e - b), hipMemcpyHostToDevice, st));
    HIPTRY(s, hipEventRecord(s->staged, st));
    s->staged_stream = st;
    for (int k = b; k < e; ++k) {
        s->dmirror[k] = s->hviews[k];
        s->dmirror_ok[k] = 1;
    }
    return DIVAS_OK;
}

double params_gate(const divas_session_s* s) { return s->params.differentiable ? -INFINITY : s->params.mask_gate; }


// With a thin path a view can vote through a pixel of a voxel's footprint:
// in the 2DGS path one with M~ > 0.5 (the score is the peak M~ of such
// pixels and must reach tau_thin > 0); in the NeRF path one with M~ > 0.5 when
// rho_cover > 0 (some pixel must be supportive), else one with M~ >= tau_thin
// (the score is the peak of all footprint pixels).  The cull stays
// conservative when the chunk boxes are padded by half a voxel (they then hold
// every voxel's cube, whose projected corners bound the footprint) and the
// gate bits (M~ >= mask_gate) cover every such pixel; otherwise it is skipped.
bool thin_culls(const divas_session_s* s) {
    const divas_params& p = s->params;
    if (!p.thin || !(p.mask_gate <= 0.5)) return false;
    if (p.variant == kVariantNerf && !(p.rho_cover > 0.0)) return p.mask_gate <= p.tau_thin;
    return true;
}

// The session that holds the scene geometry: the base of a target session,
// else the session itself.
divas_session_s* geo(divas_session_s* s) { return s->base ? s->base : s; }

constexpr int kCounterWords = 16;
constexpr int kTotWord = 8;

// Whether a fold may leave the chunks the new view cannot reach untouched:
// resident outputs asked for, the outputs of the session's previous fusion
// call, nothing changed since, and running totals that belong to that call.
bool delta_fold(const divas_session_s* s, bool fold, const divas_result* out) {
    return fold && s->params.resident_outputs && out->P == s->out_P && out->vmask == s->out_vm &&
           s->generation == s->out_gen && s->tot_valid;
}

// After a fusion call that wrote every output or folded into resident ones
// (generation already bumped): remember its outputs.
void record_outputs(divas_session_s* s, const divas_result* out, bool totals) {
    s->out_P = out->P;
    s->out_vm = out->vmask;
    s->out_gen = s->generation;
    s->tot_valid = totals;
}

// The fusion arguments of views [fb, fe) of session s (fold = start from the
// resident accumulators; delta = fold into resident outputs), with its outputs
// and count array.
FuseArgs fuse_args(divas_session_s* s, int fb, int fe, bool fold, bool cull_all, const divas_result* out,
                   int64_t* counts, bool delta = false) {
    divas_session_s* G = geo(s);
    FuseArgs a{};
    a.act = G->act;
    a.n_act = G->counters;
    a.cap = s->cap_act;
    a.g = s->g;
    a.p = s->p;
    a.views = s->dviews;
    a.s_begin = fb;
    a.s_end = fe;
    a.cull = s->cull;
    a.cull_all = cull_all ? 1 : 0;
    a.segb = s->segb;
    a.load_acc = fold ? 1 : 0;
    a.store_acc = s->W ? 1 : 0;
    a.W = s->W;
    a.Z = s->Z;
    a.vraw = s->vraw;
    a.P = out->P;
    a.vout = out->vmask;
    a.bits = s->bits;
    a.coarse = s->coarse;
    a.counts = counts;
    a.slots = s->slots;
    a.stats = s->counters + 4;
    a.rho = s->params.thin ? G->rho : nullptr;
    a.tot = s->counters + kTotWord;
    a.delta = delta ? 1 : 0;
    return a;
}

// Enqueue the pre-pass of views [b, e), the culling of those views, then the
// fusion of views [fb, fe) (fold = start from the resident accumulators).
divas_status enqueue_fusion(divas_session_s* s, int b, int e, int fb, int fe, bool fold, const divas_result* out,
                            hipStream_t st, bool delta = false) {
    int64_t* counts = out && out->counts ? out->counts : s->counters + 1;
    {
        PhaseScope ps(s, DIVAS_PHASE_VIEWS, st, true);
        const PhaseEvents ev = ps.ev();
        HIPTRY(s, launch_view_prepass(s->dviews, s->hviews.data(), b, e, params_gate(s), counts, 3, st, ev));
    }
    // the gate bits cannot stand for M~ > 0.5 in a thin session that does not
    // cull: every view of every chunk is evaluated
    const bool cull_all = s->params.thin && !thin_culls(s);
    {
        PhaseScope ps(s, DIVAS_PHASE_CULL, st, true);
        if (cull_all)
            record_phase_events(ps.ev(), st);
        else
            HIPTRY(s, launch_cull(geo(s)->chunk_box, geo(s)->counters, s->cap_act, s->g, s->p.eps, s->dviews, b, e,
                                  s->cull, st, ps.ev()));
    }
    const FuseArgs a = fuse_args(s, fb, fe, fold, cull_all, out, counts, delta);
    {
        PhaseScope ps(s, DIVAS_PHASE_FUSE, st, true);
        bool any_nsamp = false;
        for (int k = fb; k < fe; ++k) any_nsamp = any_nsamp || s->hviews[k].nsamp != nullptr;
        HIPTRY(s, launch_fuse(a, any_nsamp, st, ps.ev()));
    }
    HIPTRY(s, launch_count_reduce(s->slots, counts, s->counters + 4, a.tot, a.delta, st));
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
    out->variant = kVariant2DGS;
    out->lambda_range = 0.0;
    out->b_max = 0.0;
    out->thin = 0;
    out->rho_thin = 0.5;  // 2DGS: the thin path shares the thick path's density floor
    out->tau_thin = 0.6;
    out->rho_cover = 0.5;
    out->rho_occ = 0.1;
    out->n_abs = 25.0;
    return DIVAS_OK;
}

divas_status divas_params_nerf(double voxel, int32_t column, divas_params* out) {
    if (column != 0 && column != 1) return fail(DIVAS_ERR_ARG, "column must be 0 (LLFF) or 1 (Mip-NeRF 360)");
    divas_status st = divas_params_default(voxel, out);
    if (st != DIVAS_OK) return st;
    out->variant = kVariantNerf;
    out->gamma = column == 0 ? 4.0 : 0.5;
    out->beta = 0.2;
    out->b_max = column == 0 ? 10.0 : 1.0;
    out->lambda_range = column == 0 ? 0.05 : 5.0;
    out->rho_thin = column == 0 ? 50.0 : 30.0;
    out->rho_cover = column == 0 ? 0.2 : 0.3;
    out->tau_thin = 0.6;
    out->nerf_ray_depths = 0;
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
    {
        DeviceGuard dg(device);
        e = static_scratch_init(device, &c->static_scratch);
    }
    if (e != hipSuccess) {
        delete c;
        return fail(DIVAS_ERR_DEVICE, "fixed device scratch of device %d: %s", device, hipGetErrorString(e));
    }
    *out = c;
    return DIVAS_OK;
}

divas_status divas_ctx_destroy(divas_ctx ctx) {
    if (!ctx) return fail(DIVAS_ERR_ARG, "ctx is NULL");
    if (ctx->sessions > 0) return fail(DIVAS_ERR_STATE, "%d sessions still alive", ctx->sessions);
    if (ctx->scratch) {
        DeviceGuard dg(ctx->device);
        (void)hipFree(ctx->scratch);
    }
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
    // the point counts per active voxel of the thin-structure path
    const size_t bytes = L.bytes + (params->thin ? round_up((size_t)L.cap_act * 4, 256) : 0);
    if (ctx->budget && ctx->used + bytes > ctx->budget)
        return fail(DIVAS_ERR_ADMISSION, "session needs %zu bytes, %zu of %zu in use", bytes, ctx->used,
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
                   params->tau_cons, params->mask_gate, params->soft_width, params->differentiable,
                   params->variant, params->lambda_range, params->b_max, params->thin, params->nerf_ray_depths, params->rho_thin,
                   params->tau_thin, params->rho_cover, params->rho_occ, params->n_abs};
    s->cap_points = max_points;
    s->cap_act = L.cap_act;
    s->n_chunks = L.n_chunks;
    s->max_views = max_views;
    s->max_pix = max_view_pixels;
    s->tile_stride = L.tile_stride;
    s->footprint = bytes;
    s->hviews.resize(max_views);
    s->dmirror.resize(max_views);
    s->dmirror_ok.assign(max_views, 0);
    bool ok = dmalloc(&s->bits, (size_t)L.nwords * 4) == hipSuccess &&
              dmalloc(&s->coarse, (size_t)L.ncoarse * 4) == hipSuccess &&
              dmalloc(&s->block_counts, (size_t)L.nblocks * 4) == hipSuccess &&
              dmalloc(&s->occ_work, L.occ_work) == hipSuccess &&
              dmalloc(&s->act, round_up((size_t)L.cap_act, kChunk) * 4) == hipSuccess &&
              dmalloc(&s->chunk_box, (size_t)L.n_chunks * sizeof(ChunkBox)) == hipSuccess &&
              dmalloc(&s->counters, kCounterWords * sizeof(int64_t)) == hipSuccess &&
              hipMemsetAsync(s->counters, 0, kCounterWords * sizeof(int64_t), (hipStream_t)stream) == hipSuccess &&
              dmalloc(&s->slots, kCountSlots * kSlotWords * sizeof(int64_t)) == hipSuccess &&
              hipMemsetAsync(s->slots, 0, kCountSlots * kSlotWords * sizeof(int64_t), (hipStream_t)stream) == hipSuccess &&
              dmalloc(&s->cull, (size_t)L.n_chunks * 8) == hipSuccess &&
              dmalloc(&s->segb, round_up((size_t)L.cap_act, kChunk)) == hipSuccess &&  // whole chunks
              (!params->thin || dmalloc(&s->rho, (size_t)L.cap_act * 4) == hipSuccess) &&
              dmalloc(&s->tiles, (size_t)L.tile_stride * max_views) == hipSuccess &&
              dmalloc(&s->dviews, sizeof(DView) * max_views) == hipSuccess &&
              hipHostMalloc((void**)&s->staging, sizeof(DView) * max_views, hipHostMallocDefault) == hipSuccess &&
              hipHostMalloc((void**)&s->host_counters, 8 * sizeof(int64_t), hipHostMallocDefault) == hipSuccess &&
              hipHostGetDevicePointer((void**)&s->host_counters_dev, s->host_counters, 0) == hipSuccess &&
              hipEventCreateWithFlags(&s->built, hipEventDisableTiming) == hipSuccess &&
              hipEventCreateWithFlags(&s->staged, hipEventDisableTiming) == hipSuccess;
    if (ok && retain)
        ok = dmalloc(&s->W, (size_t)L.cap_act * 8) == hipSuccess && dmalloc(&s->Z, (size_t)L.cap_act * 8) == hipSuccess &&
             dmalloc(&s->vraw, (size_t)L.cap_act * 8) == hipSuccess;
    if (!ok) {
        (void)hipGetLastError();
        free_session(s);
        delete s;
        return fail(DIVAS_ERR_OOM, "device allocation of %zu bytes failed", bytes);
    }
    (void)hipEventRecord(s->staged, (hipStream_t)stream);
    ctx->used += bytes;
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

divas_status divas_session_create_target(divas_session base, const divas_params* params, int32_t max_views,
                                         int64_t max_view_pixels, divas_stream stream, divas_session* out) {
    if (!out) return fail(DIVAS_ERR_ARG, "out is NULL");
    *out = nullptr;
    if (!base) return fail(DIVAS_ERR_ARG, "base is NULL");
    if (base->base) return fail(DIVAS_ERR_ARG, "base is itself a target session");
    if (base->poisoned) return fail(DIVAS_ERR_STATE, "base is poisoned by an earlier device error");
    divas_status st;
    if ((st = check_params(params)) != DIVAS_OK) return st;
    if (params->thin && !base->rho)
        return fail(DIVAS_ERR_ARG, "a thin-path target needs a base built for the thin path (point counts)");
    if (max_views > DIVAS_MAX_VIEWS) return fail(DIVAS_ERR_TOO_MANY_VIEWS, "max_views %d > 64", max_views);
    if (max_views < 1) return fail(DIVAS_ERR_ARG, "max_views must be >= 1");
    if (max_view_pixels < 1) return fail(DIVAS_ERR_ARG, "max_view_pixels must be >= 1");
    divas_ctx ctx = base->ctx;
    const bool retain = params->retain_state || params->differentiable;
    const Layout L = layout(&base->grid, base->cap_points, max_views, max_view_pixels, retain);
    const size_t bytes = round_up((size_t)L.nwords * 4, 256) + round_up((size_t)L.ncoarse * 4, 256) + 256 +
                         round_up(kCountSlots * kSlotWords * sizeof(int64_t), 256) +
                         round_up((size_t)L.n_chunks * 8, 256) + round_up(round_up((size_t)L.cap_act, kChunk), 256) +
                         round_up((size_t)L.tile_stride * max_views, 256) + round_up(sizeof(DView) * max_views, 256) +
                         (retain ? round_up((size_t)L.cap_act * 24, 256) : 0);
    if (ctx->budget && ctx->used + bytes > ctx->budget)
        return fail(DIVAS_ERR_ADMISSION, "target session needs %zu bytes, %zu of %zu in use", bytes, ctx->used,
                    ctx->budget);
    DeviceGuard dg(ctx->device);
    divas_session s = new (std::nothrow) divas_session_s;
    if (!s) return fail(DIVAS_ERR_OOM, "host allocation failed");
    s->ctx = ctx;
    s->base = base;
    s->grid = base->grid;
    s->params = *params;
    s->g = base->g;
    s->p = DParams{params->gamma, params->beta, params->gamma_st, params->alpha1, params->k_grad, params->eps,
                   params->tau_cons, params->mask_gate, params->soft_width, params->differentiable,
                   params->variant, params->lambda_range, params->b_max, params->thin, params->nerf_ray_depths,
                   params->rho_thin, params->tau_thin, params->rho_cover, params->rho_occ, params->n_abs};
    s->cap_points = base->cap_points;
    s->cap_act = base->cap_act;
    s->n_chunks = base->n_chunks;
    s->max_views = max_views;
    s->max_pix = max_view_pixels;
    s->tile_stride = L.tile_stride;
    s->footprint = bytes;
    s->hviews.resize(max_views);
    s->dmirror.resize(max_views);
    s->dmirror_ok.assign(max_views, 0);
    const hipStream_t hs = (hipStream_t)stream;
    const size_t seg_bytes = round_up((size_t)L.cap_act, kChunk);
    bool ok = dmalloc(&s->bits, (size_t)L.nwords * 4) == hipSuccess &&
              hipMemsetAsync(s->bits, 0, (size_t)L.nwords * 4, hs) == hipSuccess &&
              dmalloc(&s->coarse, (size_t)L.ncoarse * 4) == hipSuccess &&
              hipMemsetAsync(s->coarse, 0, (size_t)L.ncoarse * 4, hs) == hipSuccess &&
              dmalloc(&s->counters, kCounterWords * sizeof(int64_t)) == hipSuccess &&
              hipMemsetAsync(s->counters, 0, kCounterWords * sizeof(int64_t), hs) == hipSuccess &&
              dmalloc(&s->slots, kCountSlots * kSlotWords * sizeof(int64_t)) == hipSuccess &&
              hipMemsetAsync(s->slots, 0, kCountSlots * kSlotWords * sizeof(int64_t), hs) == hipSuccess &&
              dmalloc(&s->cull, (size_t)L.n_chunks * 8) == hipSuccess &&
              dmalloc(&s->segb, seg_bytes) == hipSuccess && hipMemsetAsync(s->segb, 0, seg_bytes, hs) == hipSuccess &&
              dmalloc(&s->tiles, (size_t)L.tile_stride * max_views) == hipSuccess &&
              dmalloc(&s->dviews, sizeof(DView) * max_views) == hipSuccess &&
              hipHostMalloc((void**)&s->staging, sizeof(DView) * max_views, hipHostMallocDefault) == hipSuccess &&
              hipEventCreateWithFlags(&s->staged, hipEventDisableTiming) == hipSuccess;
    if (ok && retain)
        ok = dmalloc(&s->W, (size_t)L.cap_act * 8) == hipSuccess && dmalloc(&s->Z, (size_t)L.cap_act * 8) == hipSuccess &&
             dmalloc(&s->vraw, (size_t)L.cap_act * 8) == hipSuccess;
    if (!ok) {
        (void)hipGetLastError();
        free_session(s);
        delete s;
        return fail(DIVAS_ERR_OOM, "device allocation of %zu bytes failed", bytes);
    }
    // the shared geometry: read, never written or freed by the target
    s->act = base->act;
    s->chunk_box = base->chunk_box;
    s->rho = base->rho;
    (void)hipEventRecord(s->staged, hs);
    ctx->used += bytes;
    ctx->sessions += 1;
    base->n_targets += 1;
    *out = s;
    return DIVAS_OK;
}

divas_status divas_session_rebuild(divas_session s, const divas_occupancy* occ, divas_stream stream) {
    if (!s) return fail(DIVAS_ERR_ARG, "session is NULL");
    if (s->poisoned) return fail(DIVAS_ERR_STATE, "session is poisoned by an earlier device error");
    if (s->base) return fail(DIVAS_ERR_STATE, "a target session shares its base's occupancy and is not rebuilt");
    if (s->n_targets > 0) return fail(DIVAS_ERR_STATE, "%d target sessions share this session's occupancy", s->n_targets);
    divas_status st;
    if ((st = check_occ(occ)) != DIVAS_OK) return st;
    if (occ->n > s->cap_points)
        return fail(DIVAS_ERR_CAPACITY, "%lld points exceed the session capacity %lld", (long long)occ->n,
                    (long long)s->cap_points);
    bool general = occ->opacity != nullptr || occ->tau_occ > 1.0;
    if (general && s->params.thin)
        return fail(DIVAS_ERR_ARG, "the thin-structure path needs unit opacity and tau_occ <= 1 (point counts)");
    DeviceGuard dg(s->ctx->device);
    hipStream_t hs = (hipStream_t)stream;
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
    {
        PhaseScope ps(s, DIVAS_PHASE_OCCUPANCY, hs, true);
        // the build writes the count to the pinned host counters as well, leaves
        // its bitmap zero (the empty segmentation bitfield) and clears the
        // per-voxel flags and the coarse cell counts
        HIPTRY(s, launch_occupancy(occ->xyz, occ->opacity, occ->n, occ->tau_occ, s->g, s->bits, s->block_counts,
                                   s->act, s->chunk_box, s->counters, s->host_counters_dev, s->segb, s->coarse,
                                   s->occ_work, s->occ_scratch, s->occ_scratch_bytes, hs, ps.ev(),
                                   thin_culls(s) ? 0.5 * s->g.h : 0.0));
    }
    s->occ_points = occ->n;
    s->occ_codes = !general;
    if (s->params.thin)
        HIPTRY(s, launch_voxel_density(occ->xyz, occ->n, s->g, s->act, s->counters, s->cap_act, s->rho, hs));
    HIPTRY(s, hipEventRecord(s->built, hs));
    s->n_views = 0;
    s->acc_valid = false;
    s->fused = false;
    s->generation += 1;
    return DIVAS_OK;
}

divas_status divas_session_info(divas_session s, int64_t* n_active, const uint32_t** act, int32_t* n_views,
                                size_t* footprint) {
    if (!s) return fail(DIVAS_ERR_ARG, "session is NULL");
    if (n_active) {
        DeviceGuard dg(s->ctx->device);
        HIPTRY(s, hipEventSynchronize(geo(s)->built));
        *n_active = geo(s)->host_counters[0];
    }
    if (act) *act = geo(s)->act;
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
    DeviceGuard dg(s->ctx->device);
    hipStream_t hs = (hipStream_t)stream;
    for (int i = 0; i < n_views; ++i) fill_view(s, i, &cams[i], &maps[i]);
    if ((st = upload_views(s, 0, n_views, hs)) != DIVAS_OK) return st;
    if ((st = enqueue_fusion(s, 0, n_views, 0, n_views, false, out, hs)) != DIVAS_OK) return st;
    s->n_views = n_views;
    s->acc_valid = s->W != nullptr;
    s->fused = true;
    s->generation += 1;
    record_outputs(s, out, true);
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
    hipStream_t hs = (hipStream_t)stream;
    bool append = slot == s->n_views;
    bool fold = append && s->acc_valid && s->fused;
    fill_view(s, slot, cam, maps);
    if ((st = upload_views(s, 0, std::max(slot + 1, s->n_views), hs)) != DIVAS_OK) return st;
    int nv = append ? s->n_views + 1 : s->n_views;
    if (fold)
        st = enqueue_fusion(s, slot, slot + 1, slot, slot + 1, true, out, hs, delta_fold(s, true, out));
    else
        st = enqueue_fusion(s, slot, slot + 1, 0, nv, false, out, hs);
    if (st != DIVAS_OK) return st;
    s->n_views = nv;
    s->acc_valid = s->W != nullptr;
    s->fused = true;
    s->generation += 1;
    record_outputs(s, out, true);
    return DIVAS_OK;
}

divas_status divas_fuse_targets(const divas_session* sessions, int32_t n_targets, int32_t n_views,
                                const divas_camera* cams, const divas_view_maps* maps, const divas_result* outs,
                                int32_t schedule, divas_stream stream) {
    if (!sessions || !outs) return fail(DIVAS_ERR_ARG, "sessions and outs must be non-NULL");
    if (schedule != DIVAS_TARGETS_AUTO && schedule != DIVAS_TARGETS_TOGETHER && schedule != DIVAS_TARGETS_ONE_BY_ONE)
        return fail(DIVAS_ERR_ARG, "unknown schedule %d", schedule);
    if (n_targets < 1 || n_targets > kMaxTargets)
        return fail(DIVAS_ERR_ARG, "n_targets %d outside [1, %d]", n_targets, kMaxTargets);
    if (n_views < 0) return fail(DIVAS_ERR_ARG, "n_views < 0");
    if (n_views > DIVAS_MAX_VIEWS) return fail(DIVAS_ERR_TOO_MANY_VIEWS, "%d views: at most 64", n_views);
    if (n_views > 0 && (!cams || !maps)) return fail(DIVAS_ERR_ARG, "cams / maps is NULL");
    divas_session s0 = sessions[0];
    if (!s0) return fail(DIVAS_ERR_ARG, "session 0 is NULL");
    bool shared = true;
    for (int t = 0; t < n_targets; ++t) {
        divas_session s = sessions[t];
        if (!s) return fail(DIVAS_ERR_ARG, "session %d is NULL", t);
        for (int u = 0; u < t; ++u)
            if (sessions[u] == s) return fail(DIVAS_ERR_ARG, "session %d appears twice", t);
        if (s->poisoned) return fail(DIVAS_ERR_STATE, "session %d is poisoned by an earlier device error", t);
        if (geo(s) != geo(s0)) return fail(DIVAS_ERR_ARG, "session %d does not share session 0's scene", t);
        if (n_views > s->max_views)
            return fail(DIVAS_ERR_CAPACITY, "%d views exceed session %d's max_views %d", n_views, t, s->max_views);
        if (!outs[t].P || !outs[t].vmask) return fail(DIVAS_ERR_ARG, "outs[%d]: P and vmask are required", t);
        for (int k = 0; k < n_views; ++k) {
            divas_status st = check_view(s, &cams[k], &maps[(size_t)t * n_views + k], s->params.differentiable);
            if (st != DIVAS_OK) return st;
            const divas_view_maps& m = maps[(size_t)t * n_views + k];
            if (m.d_min != maps[k].d_min || m.d_ref != maps[k].d_ref || m.d_max != maps[k].d_max ||
                m.n_samp != maps[k].n_samp)
                return fail(DIVAS_ERR_ARG, "target %d, view %d: the depth planes must be those of target 0", t, k);
        }
        shared = shared && s->params.variant == kVariant2DGS && !s->params.thin && !s->params.differentiable &&
                 std::memcmp(&s->p, &s0->p, sizeof(DParams)) == 0;
    }
    // a positive gate leaves little shared work: one after another unless asked
    if (schedule == DIVAS_TARGETS_ONE_BY_ONE || (schedule == DIVAS_TARGETS_AUTO && s0->p.mask_gate > 0.0))
        shared = false;
    if (!shared || n_targets == 1) {  // fused one after another
        for (int t = 0; t < n_targets; ++t) {
            divas_status st = divas_fuse_views(sessions[t], n_views, cams, maps + (size_t)t * n_views, &outs[t], stream);
            if (st != DIVAS_OK) return st;
        }
        return DIVAS_OK;
    }
    DeviceGuard dg(s0->ctx->device);
    const hipStream_t hs = (hipStream_t)stream;
    divas_session_s* G = geo(s0);
#define TTRY(expr)                                                                                     \
    do {                                                                                               \
        hipError_t _e = (expr);                                                                        \
        if (_e != hipSuccess) {                                                                        \
            for (int _t = 0; _t < n_targets; ++_t) sessions[_t]->poisoned = true;                     \
            return fail(DIVAS_ERR_DEVICE, "%s: %s", #expr, hipGetErrorString(_e));                    \
        }                                                                                              \
    } while (0)
    if (!s0->targ_dev) {
        if (dmalloc(&s0->targ_dev, sizeof(TargetArgs)) != hipSuccess ||
            hipHostMalloc((void**)&s0->targ_host, sizeof(TargetArgs), hipHostMallocDefault) != hipSuccess ||
            hipEventCreateWithFlags(&s0->targ_staged, hipEventDisableTiming) != hipSuccess) {
            (void)hipGetLastError();
            return fail(DIVAS_ERR_OOM, "multi-target table");
        }
    }
    int64_t* counts[kMaxTargets];
    TargetCull tc{};
    tc.box = G->chunk_box;
    tc.n_act = G->counters;
    tc.eps = s0->p.eps;
    tc.n = n_targets;
    tc.s_begin = 0;
    tc.ns = n_views;
    for (int t = 0; t < n_targets; ++t) {
        divas_session s = sessions[t];
        for (int k = 0; k < n_views; ++k) fill_view(s, k, &cams[k], &maps[(size_t)t * n_views + k]);
        divas_status st = upload_views(s, 0, n_views, hs);
        if (st != DIVAS_OK) return st;
        counts[t] = outs[t].counts ? outs[t].counts : s->counters + 1;
        TTRY(launch_view_prepass(s->dviews, s->hviews.data(), 0, n_views, params_gate(s), counts[t], 3, hs));
        tc.views[t] = s->dviews;
        tc.cull[t] = s->cull;
    }
    TTRY(launch_cull_targets(tc, s0->cap_act, hs));
    TTRY(hipEventSynchronize(s0->targ_staged));  // the previous table has left the staging
    TargetArgs* T = s0->targ_host;
    std::memset(T, 0, sizeof(TargetArgs));
    T->n = n_targets;
    for (int t = 0; t < n_targets; ++t) T->f[t] = fuse_args(sessions[t], 0, n_views, false, false, &outs[t], counts[t]);
    TTRY(hipMemcpyAsync(s0->targ_dev, T, sizeof(TargetArgs), hipMemcpyHostToDevice, hs));
    TTRY(hipEventRecord(s0->targ_staged, hs));
    bool any_nsamp = false;
    for (int k = 0; k < n_views; ++k) any_nsamp = any_nsamp || s0->hviews[k].nsamp != nullptr;
    TTRY(launch_fuse_targets(s0->targ_dev, n_targets, s0->cap_act, any_nsamp, hs));
    for (int t = 0; t < n_targets; ++t) {
        divas_session s = sessions[t];
        if (outs[t].seg_bits) {
            size_t nw = (size_t)std::max<int64_t>(1, ((int64_t)s->grid.dim * s->grid.dim * s->grid.dim + 31) / 32);
            TTRY(hipMemcpyAsync(outs[t].seg_bits, s->bits, nw * 4, hipMemcpyDeviceToDevice, hs));
        }
        s->n_views = n_views;
        s->acc_valid = s->W != nullptr;
        s->fused = true;
        s->generation += 1;
        record_outputs(s, &outs[t], false);  // the shared count kernel keeps no running totals
    }
#undef TTRY
    return DIVAS_OK;
}

divas_status divas_label_points(divas_session s, const float* xyz, int64_t n, uint8_t* labels, divas_stream stream) {
    if (!s) return fail(DIVAS_ERR_ARG, "session is NULL");
    if (s->poisoned) return fail(DIVAS_ERR_STATE, "session is poisoned by an earlier device error");
    if (n < 0) return fail(DIVAS_ERR_ARG, "n < 0");
    if (n > 0 && (!xyz || !labels)) return fail(DIVAS_ERR_ARG, "xyz / labels is NULL");
    DeviceGuard dg(s->ctx->device);
    PhaseScope ps(s, DIVAS_PHASE_LABEL, (hipStream_t)stream, true);
    HIPTRY(s, launch_label(xyz, n, s->g, s->bits, s->coarse, labels, (hipStream_t)stream, ps.ev()));
    return DIVAS_OK;
}

divas_status divas_label_session_points(divas_session s, uint8_t* labels, int64_t* n_points, divas_stream stream) {
    if (!s) return fail(DIVAS_ERR_ARG, "session is NULL");
    if (s->poisoned) return fail(DIVAS_ERR_STATE, "session is poisoned by an earlier device error");
    const divas_session_s* base = geo(s);
    if (!base->occ_codes)
        return fail(DIVAS_ERR_STATE, "the occupancy was built with opacities or tau_occ > 1: no voxel codes are kept");
    const int64_t n = base->occ_points;
    if (n_points) *n_points = n;
    if (!labels) {  // a query of the count
        if (!n_points) return fail(DIVAS_ERR_ARG, "labels and n_points are NULL");
        return DIVAS_OK;
    }
    DeviceGuard dg(s->ctx->device);
    PhaseScope ps(s, DIVAS_PHASE_LABEL, (hipStream_t)stream, true);
    HIPTRY(s, launch_label_codes(occupancy_codes(base->g, base->occ_work, n), n, s->g, s->bits, s->coarse, labels,
                                 (hipStream_t)stream, ps.ev()));
    return DIVAS_OK;
}

divas_status divas_fuse_backward(divas_session s, const float* grad_P, int32_t n_views, float* const* grad_logit,
                                 float* const* grad_dmin, float* const* grad_dref, float* const* grad_dmax,
                                 divas_stream stream) {
    if (!s) return fail(DIVAS_ERR_ARG, "session is NULL");
    if (s->poisoned) return fail(DIVAS_ERR_STATE, "session is poisoned by an earlier device error");
    if (!s->params.differentiable) return fail(DIVAS_ERR_STATE, "session was not created with differentiable = 1");
    if (!s->fused || !s->acc_valid) return fail(DIVAS_ERR_STATE, "no forward fusion to differentiate");
    if (!grad_P) return fail(DIVAS_ERR_ARG, "grad_P is NULL");
    if (n_views != s->n_views)
        return fail(DIVAS_ERR_ARG, "gradient arrays for %d views, but the last fusion has %d", n_views, s->n_views);
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
    a.act = geo(s)->act;
    a.n_act = geo(s)->counters;
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
    PhaseScope ps(s, DIVAS_PHASE_BACKWARD, hs);
    HIPTRY(s, launch_backward(a, hs));
    return DIVAS_OK;
}

divas_status divas_surfel_coverage(divas_session s, const float* xyz, const float* scales, const float* quats,
                                   int64_t n, const uint8_t* labels_in, const uint64_t* vmask, double tau_M,
                                   double tau_kappa, double* kappa, uint8_t* labels_out, int64_t* kept,
                                   divas_stream stream) {
    if (!s) return fail(DIVAS_ERR_ARG, "session is NULL");
    if (s->poisoned) return fail(DIVAS_ERR_STATE, "session is poisoned by an earlier device error");
    if (n < 0) return fail(DIVAS_ERR_ARG, "n < 0");
    if (!is_finite(tau_M) || !is_finite(tau_kappa)) return fail(DIVAS_ERR_ARG, "tau_M and tau_kappa must be finite");
    if (!s->fused) return fail(DIVAS_ERR_STATE, "no fusion yet: the view bitmasks are undefined");
    if (n > 0 && (!xyz || !scales || !quats || !labels_in || !vmask || !kappa || !labels_out))
        return fail(DIVAS_ERR_ARG, "xyz, scales, quats, labels_in, vmask, kappa and labels_out must be non-NULL");
    DeviceGuard dg(s->ctx->device);
    hipStream_t hs = (hipStream_t)stream;
    HIPTRY(s, launch_surfel_coverage(xyz, scales, quats, n, labels_in, s->g, geo(s)->act, geo(s)->counters, vmask, s->dviews,
                                     s->n_views, tau_M, tau_kappa, s->p.eps, kappa, labels_out, kept, hs));
    return DIVAS_OK;
}

divas_status divas_session_generation(divas_session s, uint64_t* generation) {
    if (!s || !generation) return fail(DIVAS_ERR_ARG, "session or generation is NULL");
    *generation = s->generation;
    return DIVAS_OK;
}

divas_status divas_session_fusion_work(divas_session s, int64_t* hot_chunks, int64_t* hot_pairs, int64_t* gathered) {
    if (!s) return fail(DIVAS_ERR_ARG, "session is NULL");
    DeviceGuard dg(s->ctx->device);
    int64_t v[3] = {0, 0, 0};
    HIPTRY(s, hipDeviceSynchronize());
    HIPTRY(s, hipMemcpy(v, s->counters + 4, sizeof v, hipMemcpyDeviceToHost));
    if (hot_chunks) *hot_chunks = v[0];
    if (hot_pairs) *hot_pairs = v[1];
    if (gathered) *gathered = v[2];
    return DIVAS_OK;
}

divas_status divas_session_set_timing(divas_session s, uint32_t phase_mask) {
    if (!s) return fail(DIVAS_ERR_ARG, "session is NULL");
    s->timing = phase_mask & ((1u << DIVAS_PHASE_COUNT) - 1u);
    return DIVAS_OK;
}

divas_status divas_session_timings(divas_session s, double* ms, int64_t* launches, int32_t reset) {
    if (!s) return fail(DIVAS_ERR_ARG, "session is NULL");
    DeviceGuard dg(s->ctx->device);
    resolve_timings(s);
    for (int p = 0; p < DIVAS_PHASE_COUNT; ++p) {
        if (ms) ms[p] = s->acc_ms[p];
        if (launches) launches[p] = s->acc_n[p];
        if (reset) {
            s->acc_ms[p] = 0.0;
            s->acc_n[p] = 0;
        }
    }
    return DIVAS_OK;
}

divas_status divas_session_destroy(divas_session s) {
    if (!s) return fail(DIVAS_ERR_ARG, "session is NULL");
    if (s->n_targets > 0) return fail(DIVAS_ERR_STATE, "%d target sessions share this session's occupancy", s->n_targets);
    DeviceGuard dg(s->ctx->device);
    (void)hipDeviceSynchronize();
    if (s->base) {  // the shared geometry stays with the base
        s->act = nullptr;
        s->chunk_box = nullptr;
        s->rho = nullptr;
        s->base->n_targets -= 1;
    }
    if (s->targ_dev) (void)hipFree(s->targ_dev);
    if (s->targ_host) (void)hipHostFree(s->targ_host);
    if (s->targ_staged) (void)hipEventDestroy(s->targ_staged);
    for (auto& r : s->pending) {
        (void)hipEventDestroy(r.a);
        (void)hipEventDestroy(r.b);
    }
    for (hipEvent_t e : s->pool) (void)hipEventDestroy(e);
    s->ctx->used -= s->footprint + s->lazy_bytes;
    s->ctx->sessions -= 1;
    free_session(s);
    delete s;
    return DIVAS_OK;
}


// ------------------------------------------------------------------ batches
}  // extern "C"

struct divas_batch_s {
    divas_ctx ctx = nullptr;
    int32_t max_items = 0, max_vjobs = 0;
    divas_batch_config cfg{};
    int n_cu = 256;
    std::string dev_name;
    char* dtab = nullptr;
    char* htab = nullptr;
    size_t tab_bytes = 0;
    size_t off_header = 0, off_items = 0, off_icb = 0, off_cjobs = 0, off_clb = 0, off_vjobs = 0, off_vrb = 0,
           off_vrecs = 0;
    hipEvent_t staged = nullptr;
    hipStream_t cap_stream = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    bool graph_ready = false;
    unsigned fuse_cap = 0;  // fusion blocks of the captured graph (a batch needing more recaptures)
    BDesc* ddesc = nullptr;  // descriptors of the persistent schedule (device, pinned staging), grown on demand
    BDesc* hdesc = nullptr;
    size_t desc_cap = 0;
    int mode = -1;          // fusion kernel of the captured graph
};

namespace {

BatchTables batch_tables(divas_batch b) {
    BatchTables t{};
    t.header = (const BatchHeader*)(b->dtab + b->off_header);
    t.items = (const BItem*)(b->dtab + b->off_items);
    t.item_chunk_base = (const int64_t*)(b->dtab + b->off_icb);
    t.cjobs = (const BCullJob*)(b->dtab + b->off_cjobs);
    t.cjob_lane_base = (const int64_t*)(b->dtab + b->off_clb);
    t.vjobs = (const BViewJob*)(b->dtab + b->off_vjobs);
    t.vjob_row_base = (const int64_t*)(b->dtab + b->off_vrb);
    t.vrecs = (const DView*)(b->dtab + b->off_vrecs);
    t.desc = b->ddesc;
    t.head = &((BatchHeader*)(b->dtab + b->off_header))->head;
    return t;
}

BatchGrid batch_grid(divas_batch b) {
    BatchGrid g;
    g.prep_blocks = (unsigned)(4 * b->n_cu);
    g.cull_blocks = (unsigned)(std::max(1, b->cfg.cull_blocks_per_cu) * b->n_cu);
    g.fuse_threads = (unsigned)(64 * std::max(1, b->cfg.fuse_waves_per_block));
    g.fuse_blocks = std::max(1u, b->fuse_cap);
    g.mode = b->mode < 0 ? kThick : b->mode;
    g.persistent = b->cfg.schedule > 0;
    if (g.persistent)  // 16 wavefronts per compute unit
        g.fuse_blocks = (unsigned)std::max(1, 16 * b->n_cu / std::max(1, b->cfg.fuse_waves_per_block));
    return g;
}

void drop_graph(divas_batch b) {
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    b->exec = nullptr;
    b->graph = nullptr;
    b->graph_ready = false;
}

struct PlannedItem {
    divas_session s;
    int first_new, n_new;  // new view slots [first_new, first_new + n_new)
    int fb, fe;            // fused views
    bool fold;
    bool delta;            // fold into the resident outputs of the session's previous call
    int new_nviews;
    int64_t n_act, nchunks;
    const divas_batch_item* src;
};

divas_status plan_batch(divas_batch b, int32_t n, const divas_batch_item* items, std::vector<PlannedItem>& plan,
                        bool& any_nsamp) {
    if (n < 0 || n > b->max_items) return fail(DIVAS_ERR_CAPACITY, "%d items exceed the batch capacity %d", n, b->max_items);
    if (n > 0 && !items) return fail(DIVAS_ERR_ARG, "items is NULL");
    std::set<divas_session> seen;
    int total_new = 0;
    any_nsamp = false;
    plan.clear();
    for (int i = 0; i < n; ++i) {
        const divas_batch_item& it = items[i];
        divas_session s = it.session;
        if (!s) return fail(DIVAS_ERR_ARG, "item %d: session is NULL", i);
        if (s->ctx != b->ctx) return fail(DIVAS_ERR_ARG, "item %d: session of another context", i);
        if (s->poisoned) return fail(DIVAS_ERR_STATE, "item %d: session is poisoned", i);
        if (!seen.insert(s).second) return fail(DIVAS_ERR_ARG, "item %d: session appears twice in the batch", i);
        if (!it.out.P || !it.out.vmask) return fail(DIVAS_ERR_ARG, "item %d: result P and vmask are required", i);
        PlannedItem pi{};
        pi.s = s;
        pi.src = &it;
        if (it.op == DIVAS_BATCH_FUSE) {
            if (it.n_views > DIVAS_MAX_VIEWS) return fail(DIVAS_ERR_TOO_MANY_VIEWS, "item %d: %d views", i, it.n_views);
            if (it.n_views < 0 || it.n_views > s->max_views)
                return fail(DIVAS_ERR_CAPACITY, "item %d: %d views exceed max_views %d", i, it.n_views, s->max_views);
            if (it.n_views > 0 && (!it.cams || !it.maps)) return fail(DIVAS_ERR_ARG, "item %d: cams / maps NULL", i);
            pi.first_new = 0;
            pi.n_new = it.n_views;
            pi.fb = 0;
            pi.fe = it.n_views;
            pi.fold = false;
            pi.delta = false;
            pi.new_nviews = it.n_views;
        } else if (it.op == DIVAS_BATCH_UPDATE) {
            if (it.n_views != 1 || !it.cams || !it.maps) return fail(DIVAS_ERR_ARG, "item %d: an update carries one view", i);
            if (it.slot < 0 || it.slot > s->n_views) return fail(DIVAS_ERR_ARG, "item %d: slot %d outside [0, %d]", i, it.slot, s->n_views);
            if (it.slot >= DIVAS_MAX_VIEWS) return fail(DIVAS_ERR_TOO_MANY_VIEWS, "item %d: slot %d", i, it.slot);
            if (it.slot >= s->max_views) return fail(DIVAS_ERR_CAPACITY, "item %d: slot %d beyond max_views", i, it.slot);
            bool append = it.slot == s->n_views;
            pi.first_new = it.slot;
            pi.n_new = 1;
            pi.fold = append && s->acc_valid && s->fused;
            pi.delta = delta_fold(s, pi.fold, &it.out);
            pi.new_nviews = append ? s->n_views + 1 : s->n_views;
            pi.fb = pi.fold ? it.slot : 0;
            pi.fe = pi.fold ? it.slot + 1 : pi.new_nviews;
        } else {
            return fail(DIVAS_ERR_ARG, "item %d: unknown op %d", i, it.op);
        }
        for (int k = 0; k < pi.n_new; ++k) {
            divas_status st = check_view(s, &it.cams[k], &it.maps[k], s->params.differentiable);
            if (st != DIVAS_OK) return st;
            if (it.maps[k].n_samp && !s->params.differentiable) any_nsamp = true;
        }
        total_new += pi.n_new;
        plan.push_back(pi);
    }
    if (total_new > b->max_vjobs)
        return fail(DIVAS_ERR_CAPACITY, "%d new views exceed the batch capacity %d", total_new, b->max_vjobs);
    return DIVAS_OK;
}

divas_status run_batch(divas_batch b, int32_t n, const divas_batch_item* items, hipStream_t st, bool allow_graph) {
    std::vector<PlannedItem> plan;
    bool any_nsamp = false;
    divas_status rs = plan_batch(b, n, items, plan, any_nsamp);
    if (rs != DIVAS_OK) return rs;
    if (n == 0) return DIVAS_OK;
    DeviceGuard dg(b->ctx->device);
    for (auto& pi : plan) {
        if (hipEventSynchronize(geo(pi.s)->built) != hipSuccess) return fail(DIVAS_ERR_DEVICE, "occupancy build failed");
        pi.n_act = geo(pi.s)->host_counters[0];
        pi.nchunks = (pi.n_act + kChunk - 1) / kChunk;
    }
    // the previous run must have left the pinned staging
    if (hipEventSynchronize(b->staged) != hipSuccess) return fail(DIVAS_ERR_DEVICE, "batch staging wait failed");
    char* H = b->htab;
    BatchHeader* hd = (BatchHeader*)(H + b->off_header);
    BItem* bi = (BItem*)(H + b->off_items);
    int64_t* icb = (int64_t*)(H + b->off_icb);
    BCullJob* cj = (BCullJob*)(H + b->off_cjobs);
    int64_t* clb = (int64_t*)(H + b->off_clb);
    BViewJob* vj = (BViewJob*)(H + b->off_vjobs);
    int64_t* vrb = (int64_t*)(H + b->off_vrb);
    DView* vr = (DView*)(H + b->off_vrecs);
    int nv = 0, nc = 0;
    int64_t rows = 0, lanes = 0, chunks = 0;
    for (int i = 0; i < (int)plan.size(); ++i) {
        PlannedItem& pi = plan[i];
        divas_session s = pi.s;
        for (int k = 0; k < pi.n_new; ++k) {
            int slot = pi.first_new + k;
            fill_view(s, slot, &pi.src->cams[k], &pi.src->maps[k]);
            vr[nv] = s->hviews[slot];
            s->dmirror_ok[slot] = 0;  // written on the device by the batch, not by an upload
            vj[nv] = BViewJob{i, slot};
            vrb[nv] = rows;
            rows += s->hviews[slot].th;
            ++nv;
        }
        const bool cull_all = s->params.thin && !thin_culls(s);
        if (pi.n_new > 0 && !cull_all) {  // one cull job per item: its new views, lanes grouped per chunk
            int p2 = pow2_at_least(pi.n_new);
            cj[nc] = BCullJob{i, pi.first_new, pi.n_new, p2};
            clb[nc] = lanes;
            lanes += (pi.nchunks * p2 + 63) / 64 * 64;
            ++nc;
        }
        BItem& it = bi[i];
        std::memset(&it, 0, sizeof it);
        FuseArgs& a = it.f;
        a.act = geo(s)->act;
        a.n_act = geo(s)->counters;
        a.cap = s->cap_act;
        a.g = s->g;
        a.p = s->p;
        a.views = s->dviews;
        a.s_begin = pi.fb;
        a.s_end = pi.fe;
        a.cull = s->cull;
        a.cull_all = cull_all ? 1 : 0;
        a.rho = s->params.thin ? geo(s)->rho : nullptr;
        a.segb = s->segb;
        a.load_acc = pi.fold ? 1 : 0;
        a.store_acc = s->W ? 1 : 0;
        a.W = s->W;
        a.Z = s->Z;
        a.vraw = s->vraw;
        a.P = pi.src->out.P;
        a.vout = pi.src->out.vmask;
        a.bits = s->bits;
        a.coarse = s->coarse;
        a.counts = pi.src->out.counts ? pi.src->out.counts : s->counters + 1;
        a.slots = s->slots;
        a.stats = s->counters + 4;
        a.tot = s->counters + kTotWord;
        a.delta = pi.delta ? 1 : 0;
        it.box = geo(s)->chunk_box;
        it.views_rw = s->dviews;
        it.cull_rw = s->cull;
        it.gate = params_gate(s);
        it.fuse_range = (pi.fe - pi.fb >= 64 ? ~0ull : ((1ull << (pi.fe - pi.fb)) - 1ull)) << pi.fb;
        icb[i] = chunks;
        chunks += pi.nchunks;
    }
    icb[plan.size()] = chunks;
    hd->n_items = (int32_t)plan.size();
    hd->n_vjobs = nv;
    hd->n_cjobs = nc;
    hd->chunks_per_wave = 1;
    hd->total_rows = rows;
    hd->total_cull = lanes;
    hd->total_chunks = chunks;
    if (chunks >= ((int64_t)1 << 31)) return fail(DIVAS_ERR_CAPACITY, "too many chunks in one batch");
    size_t bytes = b->off_vrecs + (size_t)nv * sizeof(DView);
    // persistent schedule: chunk ranges of cfg.schedule chunks, the items that
    // fuse the most views (then the most chunks) first
    uint32_t nd = 0;
    if (b->cfg.schedule > 0) {
        const int64_t D = b->cfg.schedule;
        std::vector<int> ord(plan.size());
        for (size_t k = 0; k < ord.size(); ++k) ord[k] = (int)k;
        std::stable_sort(ord.begin(), ord.end(), [&](int x, int y) {
            const int vx = plan[x].fe - plan[x].fb, vy = plan[y].fe - plan[y].fb;
            return vx != vy ? vx > vy : plan[x].nchunks > plan[y].nchunks;
        });
        size_t need = 0;
        for (auto& pi : plan) need += (size_t)((pi.nchunks + D - 1) / D);
        if (need > b->desc_cap) {
            if (b->ddesc) (void)hipFree(b->ddesc);
            if (b->hdesc) (void)hipHostFree(b->hdesc);
            b->ddesc = nullptr;
            b->hdesc = nullptr;
            b->desc_cap = 0;
            drop_graph(b);  // the descriptors' address is part of a captured launch
            const size_t cap = std::max(need, (size_t)1024);
            if (hipMalloc((void**)&b->ddesc, cap * sizeof(BDesc)) != hipSuccess ||
                hipHostMalloc((void**)&b->hdesc, cap * sizeof(BDesc), hipHostMallocDefault) != hipSuccess) {
                (void)hipGetLastError();
                return fail(DIVAS_ERR_OOM, "batch descriptors: %zu", cap);
            }
            b->desc_cap = cap;
        }
        for (int k : ord)
            for (int64_t c = 0; c < plan[k].nchunks; c += D)
                b->hdesc[nd++] = BDesc{k, (uint32_t)c, (uint32_t)std::min<int64_t>(c + D, plan[k].nchunks), 0};
    }
    hd->n_desc = nd;
    hd->head = 0;
    auto poison_all = [&]() {
        for (auto& pi : plan) pi.s->poisoned = true;
    };
#define BTRY(expr)                                                                                       \
    do {                                                                                                 \
        hipError_t _e = (expr);                                                                          \
        if (_e != hipSuccess) {                                                                          \
            poison_all();                                                                                \
            return fail(DIVAS_ERR_DEVICE, "%s: %s", #expr, hipGetErrorString(_e));                        \
        }                                                                                                \
    } while (0)
    BTRY(hipMemcpyAsync(b->dtab, b->htab, bytes, hipMemcpyHostToDevice, st));
    if (nd) BTRY(hipMemcpyAsync(b->ddesc, b->hdesc, nd * sizeof(BDesc), hipMemcpyHostToDevice, st));
    BatchTables t = batch_tables(b);
    {
        // the fusion launch needs a wavefront per chunk and the kernel variant of
        // the batch; a captured graph that has too few blocks or the other
        // variant is dropped (the block count grows by half, so recaptures are rare)
        const unsigned wpb = (unsigned)std::max(1, b->cfg.fuse_waves_per_block);
        const unsigned need = (unsigned)std::max<int64_t>(1, (chunks + wpb - 1) / wpb);
        bool generic = false;
        bool thin = false;
        for (auto& pi : plan) {
            generic = generic || pi.s->params.differentiable || pi.s->params.variant != kVariant2DGS;
            for (int k = pi.fb; k < pi.fe; ++k) generic = generic || pi.s->hviews[k].nsamp != nullptr;
            thin = thin || pi.s->params.thin;
        }
        const int mode = thin ? kAnyThin : (generic ? kAnyMode : kThick);
        if (need > b->fuse_cap || mode != b->mode) {
            drop_graph(b);
            if (need > b->fuse_cap) b->fuse_cap = std::max(need, b->fuse_cap + b->fuse_cap / 2);
            b->mode = mode;
        }
    }
    BatchGrid g = batch_grid(b);
    bool graph = allow_graph && b->cfg.use_graph;
    if (graph) {
        if (!b->graph_ready) {
            drop_graph(b);
            BTRY(hipStreamBeginCapture(b->cap_stream, hipStreamCaptureModeRelaxed));
            hipError_t le = launch_batch(t, g, b->cap_stream);
            hipError_t ee = hipStreamEndCapture(b->cap_stream, &b->graph);
            BTRY(le);
            BTRY(ee);
            BTRY(hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0));
            b->graph_ready = true;
        }
        BTRY(hipGraphLaunch(b->exec, st));
    } else {
        BTRY(launch_batch(t, g, st));
    }
    BTRY(hipEventRecord(b->staged, st));
    for (auto& pi : plan) {
        if (pi.src->out.seg_bits) {
            size_t nw = (size_t)std::max<int64_t>(1, ((int64_t)pi.s->grid.dim * pi.s->grid.dim * pi.s->grid.dim + 31) / 32);
            BTRY(hipMemcpyAsync(pi.src->out.seg_bits, pi.s->bits, nw * 4, hipMemcpyDeviceToDevice, st));
        }
        pi.s->n_views = pi.new_nviews;
        pi.s->acc_valid = pi.s->W != nullptr;
        pi.s->fused = true;
        pi.s->generation += 1;
        record_outputs(pi.s, &pi.src->out, true);
    }
#undef BTRY
    return DIVAS_OK;
}

std::string json_escape(const std::string& x) {
    std::string o;
    for (char c : x)
        if (c != '"' && c != '\\') o += c;
    return o;
}

int bucket(int64_t v) {
    int b = 0;
    while ((int64_t)1 << b < v) ++b;
    return b;
}

}  // namespace

extern "C" {

divas_status divas_batch_create(divas_ctx ctx, int32_t max_items, int32_t max_new_views,
                                const divas_batch_config* cfg, divas_batch* out) {
    if (!out) return fail(DIVAS_ERR_ARG, "out is NULL");
    *out = nullptr;
    if (!ctx) return fail(DIVAS_ERR_ARG, "ctx is NULL");
    if (max_items < 1 || max_new_views < 0) return fail(DIVAS_ERR_ARG, "max_items >= 1 and max_new_views >= 0");
    DeviceGuard dg(ctx->device);
    divas_batch b = new (std::nothrow) divas_batch_s;
    if (!b) return fail(DIVAS_ERR_OOM, "host allocation failed");
    b->ctx = ctx;
    b->max_items = max_items;
    b->max_vjobs = std::max(1, max_new_views);
    b->cfg.fuse_waves_per_block = 4;
    b->cfg.cull_blocks_per_cu = 4;
    b->cfg.use_graph = 1;
    if (cfg) {
        if (cfg->fuse_waves_per_block > 0) {
            int w = 1;
            while (w < cfg->fuse_waves_per_block && w < 8) w <<= 1;
            b->cfg.fuse_waves_per_block = w;
        }
        if (cfg->cull_blocks_per_cu > 0) b->cfg.cull_blocks_per_cu = std::min(cfg->cull_blocks_per_cu, 64);
        b->cfg.use_graph = cfg->use_graph;
        b->cfg.schedule = std::max(0, std::min(cfg->schedule, 1 << 16));
    }
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, ctx->device) == hipSuccess) {
        b->n_cu = prop.multiProcessorCount > 0 ? prop.multiProcessorCount : 256;
        b->dev_name = prop.gcnArchName;
    }
    size_t o = 0;
    auto take = [&](size_t bytes) {
        size_t r = o;
        o = round_up(o + bytes, 256);
        return r;
    };
    b->off_header = take(sizeof(BatchHeader));
    b->off_items = take(sizeof(BItem) * max_items);
    b->off_icb = take(sizeof(int64_t) * (max_items + 1));
    b->off_cjobs = take(sizeof(BCullJob) * b->max_vjobs);
    b->off_clb = take(sizeof(int64_t) * b->max_vjobs);
    b->off_vjobs = take(sizeof(BViewJob) * b->max_vjobs);
    b->off_vrb = take(sizeof(int64_t) * b->max_vjobs);
    b->off_vrecs = take(sizeof(DView) * b->max_vjobs);
    b->tab_bytes = o;
    bool ok = hipMalloc((void**)&b->dtab, b->tab_bytes) == hipSuccess &&
              hipHostMalloc((void**)&b->htab, b->tab_bytes, hipHostMallocDefault) == hipSuccess &&
              hipEventCreateWithFlags(&b->staged, hipEventDisableTiming) == hipSuccess &&
              hipStreamCreateWithFlags(&b->cap_stream, hipStreamNonBlocking) == hipSuccess;
    if (!ok) {
        (void)hipGetLastError();
        if (b->dtab) (void)hipFree(b->dtab);
        if (b->htab) (void)hipHostFree(b->htab);
        if (b->staged) (void)hipEventDestroy(b->staged);
        if (b->cap_stream) (void)hipStreamDestroy(b->cap_stream);
        delete b;
        return fail(DIVAS_ERR_OOM, "batch tables: %zu bytes", (size_t)o);
    }
    std::memset(b->htab, 0, b->tab_bytes);
    (void)hipEventRecord(b->staged, b->cap_stream);
    *out = b;
    return DIVAS_OK;
}

divas_status divas_batch_run(divas_batch b, int32_t n, const divas_batch_item* items, divas_stream stream) {
    if (!b) return fail(DIVAS_ERR_ARG, "batch is NULL");
    return run_batch(b, n, items, (hipStream_t)stream, true);
}

divas_status divas_batch_validate(divas_batch b, int32_t n, const divas_batch_item* items) {
    if (!b) return fail(DIVAS_ERR_ARG, "batch is NULL");
    std::vector<PlannedItem> plan;
    bool any_nsamp = false;
    return plan_batch(b, n, items, plan, any_nsamp);
}

divas_status divas_batch_tune(divas_batch b, int32_t n, const divas_batch_item* items, divas_stream stream,
                              const char* cache_path, divas_batch_config* chosen) {
    if (!b) return fail(DIVAS_ERR_ARG, "batch is NULL");
    for (int i = 0; i < n; ++i)
        if (!items || items[i].op != DIVAS_BATCH_FUSE)
            return fail(DIVAS_ERR_ARG, "tuning needs DIVAS_BATCH_FUSE items (re-running them is idempotent)");
    int64_t vox = 0, views = 0;
    for (int i = 0; i < n; ++i) {
        divas_session s = items[i].session;
        if (!s) return fail(DIVAS_ERR_ARG, "item %d: session is NULL", i);
        if (hipEventSynchronize(geo(s)->built) != hipSuccess) return fail(DIVAS_ERR_DEVICE, "occupancy build failed");
        vox += geo(s)->host_counters[0];
        views += items[i].n_views;
    }
    std::ostringstream key;
    key << json_escape(b->dev_name) << "|items" << bucket(n) << "|vox" << bucket(vox) << "|views" << bucket(views);
    // cache lookup: one JSON object per line,
    // {"key": "...", "waves": W, "cull": C, "schedule": S, "graph": G, "ms": T}
    if (cache_path) {
        std::ifstream f(cache_path);
        std::string line;
        auto field = [&](const char* name, int* v) {
            const std::string k = std::string("\"") + name + "\": ";
            const size_t p = line.find(k);
            if (p == std::string::npos) return false;
            *v = std::atoi(line.c_str() + p + k.size());
            return true;
        };
        while (std::getline(f, line)) {
            if (line.find("\"key\": \"" + key.str() + "\"") == std::string::npos) continue;
            int wv = 0, cu = 0, sc = 0, gr = 1;
            if (field("waves", &wv) && field("cull", &cu) && field("schedule", &sc) && field("graph", &gr) && wv > 0 &&
                cu > 0 && sc >= 0) {
                b->cfg.fuse_waves_per_block = wv;
                b->cfg.cull_blocks_per_cu = cu;
                b->cfg.schedule = sc;
                b->cfg.use_graph = gr ? 1 : 0;
                b->fuse_cap = 0;
                drop_graph(b);
                if (chosen) *chosen = b->cfg;
                return DIVAS_OK;
            }
        }
    }
    DeviceGuard dg(b->ctx->device);
    hipStream_t st = (hipStream_t)stream;
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
        return fail(DIVAS_ERR_DEVICE, "event creation failed");
    // the space: wavefronts per fusion block x cull grid x schedule (the
    // hardware dispatcher, or the persistent queue with 1, 4 or 16 chunks per
    // descriptor), each with the graph; then the winner without the graph
    const int waves[] = {1, 2, 4, 8};
    const int culls[] = {2, 4, 8};
    const int scheds[] = {0, 1, 4, 16};
    divas_batch_config best = b->cfg;
    float best_ms = 1e30f;
    divas_status rs = DIVAS_OK;
    auto time_cfg = [&](const divas_batch_config& c) -> float {
        b->cfg = c;
        b->fuse_cap = 0;
        drop_graph(b);
        if ((rs = run_batch(b, n, items, st, true)) != DIVAS_OK) return 1e30f;  // warm-up (and graph capture)
        (void)hipEventRecord(e0, st);
        const int reps = 3;
        for (int r = 0; r < reps && rs == DIVAS_OK; ++r) rs = run_batch(b, n, items, st, true);
        (void)hipEventRecord(e1, st);
        if (rs != DIVAS_OK) return 1e30f;
        float ms = 0;
        if (hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
            rs = fail(DIVAS_ERR_DEVICE, "tuning timing failed");
            return 1e30f;
        }
        return ms / reps;
    };
    for (int sc : scheds)
        for (int wv : waves)
            for (int cu : culls) {
                if (rs != DIVAS_OK) break;
                divas_batch_config c = b->cfg;
                c.fuse_waves_per_block = wv;
                c.cull_blocks_per_cu = cu;
                c.schedule = sc;
                c.use_graph = 1;
                const float ms = time_cfg(c);
                if (ms < best_ms) {
                    best_ms = ms;
                    best = c;
                }
            }
    if (rs == DIVAS_OK) {
        divas_batch_config c = best;
        c.use_graph = 0;
        const float ms = time_cfg(c);
        if (ms < best_ms) {
            best_ms = ms;
            best = c;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rs != DIVAS_OK) return rs;
    b->cfg = best;
    b->fuse_cap = 0;
    drop_graph(b);
    if (chosen) *chosen = best;
    if (cache_path) {
        std::ofstream f(cache_path, std::ios::app);
        f << "{\"key\": \"" << key.str() << "\", \"waves\": " << best.fuse_waves_per_block
          << ", \"cull\": " << best.cull_blocks_per_cu << ", \"schedule\": " << best.schedule
          << ", \"graph\": " << best.use_graph << ", \"ms\": " << best_ms << "}\n";
    }
    return DIVAS_OK;
}

divas_status divas_batch_destroy(divas_batch b) {
    if (!b) return fail(DIVAS_ERR_ARG, "batch is NULL");
    DeviceGuard dg(b->ctx->device);
    (void)hipEventSynchronize(b->staged);
    (void)hipStreamSynchronize(b->cap_stream);
    drop_graph(b);
    (void)hipFree(b->dtab);
    (void)hipHostFree(b->htab);
    if (b->ddesc) (void)hipFree(b->ddesc);
    if (b->hdesc) (void)hipHostFree(b->hdesc);
    (void)hipEventDestroy(b->staged);
    (void)hipStreamDestroy(b->cap_stream);
    delete b;
    return DIVAS_OK;
}

divas_status divas_grid_params_default(int32_t g_max, divas_grid_params* out) {
    if (!out) return fail(DIVAS_ERR_ARG, "out is NULL");
    if (g_max < 2 || g_max > 1024 || (g_max & (g_max - 1)))
        return fail(DIVAS_ERR_ARG, "g_max must be a power of two in [2, 1024]");
    std::memset(out, 0, sizeof *out);
    out->alpha_v = 3.0;
    out->beta_v = 1.0;
    out->pad = 1.05;
    out->percentile = 0.99;
    out->g0 = 256;
    out->g_max = g_max;
    return DIVAS_OK;
}

divas_status divas_grid_from_points(divas_ctx ctx, const float* xyz, const float* scale, int64_t n,
                                    const divas_grid_params* p, divas_grid* grid, divas_grid_stats* stats,
                                    divas_stream stream) {
    if (!ctx || !xyz || !p || !grid) return fail(DIVAS_ERR_ARG, "ctx, xyz, params and grid must be non-NULL");
    if (n < 1 || n > ((int64_t)1 << 31)) return fail(DIVAS_ERR_ARG, "n must be in [1, 2^31]");
    if (!is_finite(p->alpha_v) || !(p->alpha_v >= 0.0) || !is_finite(p->beta_v) || !(p->beta_v > 0.0) ||
        !is_finite(p->pad) || !(p->pad > 0.0) || !is_finite(p->percentile) || !(p->percentile >= 0.0) ||
        !(p->percentile <= 1.0) || p->g0 < 1 || p->g_max < 2 || p->g_max > 1024 || (p->g_max & (p->g_max - 1)))
        return fail(DIVAS_ERR_ARG, "grid parameters out of range");
    DeviceGuard dg(ctx->device);
    GridStatsParams q{p->alpha_v, p->beta_v, p->pad, p->percentile, p->g0, p->g_max};
    GridStatsResult r{};
    void* scr = nullptr;
    const size_t need = grid_statistics_scratch(n);
    if (ctx_scratch(ctx, need, &scr) != hipSuccess) return fail(DIVAS_ERR_OOM, "device scratch of %zu bytes", need);
    const hipError_t e = grid_statistics(xyz, scale, n, q, &r, scr, need, (hipStream_t)stream);
    if (e != hipSuccess) return fail(DIVAS_ERR_DEVICE, "grid statistics: %s", hipGetErrorString(e));
    if (r.m == 0) return fail(DIVAS_ERR_ARG, "no point has finite coordinates (and scale)");
    if (r.dim == 0) return fail(DIVAS_ERR_ARG, "degenerate scene: b = %g, h_v = %g", r.b, r.h_v);
    for (int a = 0; a < 3; ++a) grid->origin[a] = r.origin[a];
    grid->voxel = r.voxel;
    grid->dim = r.dim;
    if (stats) {
        for (int a = 0; a < 3; ++a) stats->center[a] = r.center[a];
        stats->r_fg = r.r_fg;
        stats->b = r.b;
        stats->s_med = r.s_med;
        stats->h_v = r.h_v;
        stats->n_used = r.m;
        stats->n_kept = r.n_kept;
    }
    return DIVAS_OK;
}

}  // extern "C"

namespace {
divas_status refine_call(int kind, divas_ctx ctx, int32_t width, int32_t height, const float* mask,
                         const float* depth, const int32_t* prompts_xy, int32_t n_prompts, float* refined,
                         divas_refine_stats* stats, divas_stream stream) {
    if (!ctx || !mask || !depth || !refined) return fail(DIVAS_ERR_ARG, "ctx, mask, depth and refined must be non-NULL");
    if (width < 1 || height < 1 || (int64_t)width * height > ((int64_t)1 << 31))
        return fail(DIVAS_ERR_ARG, "view size %d x %d out of range", width, height);
    if (n_prompts < 0 || n_prompts > (1 << 20) || (n_prompts > 0 && !prompts_xy))
        return fail(DIVAS_ERR_ARG, "n_prompts out of range or prompts_xy NULL");
    for (int k = 0; k < n_prompts; ++k)
        if (prompts_xy[2 * k] < 0 || prompts_xy[2 * k] >= width || prompts_xy[2 * k + 1] < 0 ||
            prompts_xy[2 * k + 1] >= height)
            return fail(DIVAS_ERR_ARG, "prompt %d (%d, %d) outside the %d x %d view", k, prompts_xy[2 * k],
                        prompts_xy[2 * k + 1], width, height);
    DeviceGuard dg(ctx->device);
    RefineResult r{};
    void* scr = nullptr;
    const size_t need = refine_mask_scratch((int64_t)width * height, n_prompts);
    if (ctx_scratch(ctx, need, &scr) != hipSuccess) return fail(DIVAS_ERR_OOM, "device scratch of %zu bytes", need);
    const hipError_t e = refine_mask(kind, width, height, mask, depth, prompts_xy, n_prompts, refined, &r, scr, need,
                                     (hipStream_t)stream);
    if (e != hipSuccess) return fail(DIVAS_ERR_DEVICE, "mask refinement: %s", hipGetErrorString(e));
    if (r.n_surface == 0) return fail(DIVAS_ERR_ARG, "no pixel of the depth map has a surface");
    if (kind == kRefineBandPass && r.n_anchors == 0)
        return fail(DIVAS_ERR_ARG, "no prompt pixel (nor the view centre) has a surface");
    if (stats) {
        stats->band_min = r.band_min;
        stats->band_max = r.band_max;
        stats->d_far = r.d_far;
        stats->z_min = r.z_min;
        stats->z_max = r.z_max;
        stats->n_surface = r.n_surface;
        stats->n_anchors = r.n_anchors;
    }
    return DIVAS_OK;
}
}  // namespace

extern "C" {

divas_status divas_refine_mask_bandpass(divas_ctx ctx, int32_t width, int32_t height, const float* mask,
                                        const float* d_med, const int32_t* prompts_xy, int32_t n_prompts,
                                        float* refined, divas_refine_stats* stats, divas_stream stream) {
    return refine_call(kRefineBandPass, ctx, width, height, mask, d_med, prompts_xy, n_prompts, refined, stats,
                       stream);
}

divas_status divas_refine_mask_minmax(divas_ctx ctx, int32_t width, int32_t height, const float* mask,
                                      const float* d_exp, float* refined, divas_refine_stats* stats,
                                      divas_stream stream) {
    return refine_call(kRefineMinMax, ctx, width, height, mask, d_exp, nullptr, 0, refined, stats, stream);
}

}  // extern "C"

extern "C" {

}  // extern "C"

namespace {
divas_status check_needle(divas_ctx ctx, const float* scales, int64_t n, double eps, const uint8_t* labels) {
    if (!ctx || !scales || !labels) return fail(DIVAS_ERR_ARG, "ctx, scales and labels must be non-NULL");
    if (n < 1 || n > ((int64_t)1 << 31)) return fail(DIVAS_ERR_ARG, "n must be in [1, 2^31]");
    if (!is_finite(eps) || !(eps >= 0.0)) return fail(DIVAS_ERR_ARG, "eps must be finite and >= 0");
    return DIVAS_OK;
}

divas_status needle_call(const float* scales, int64_t n, double eps, uint8_t* labels, double* tau_a,
                         int64_t* n_culled, void* scr, size_t need, divas_stream stream) {
    NeedleResult r{};
    const hipError_t e = needle_cull(scales, n, eps, 0.99, labels, &r, scr, need, (hipStream_t)stream);
    if (e != hipSuccess) return fail(DIVAS_ERR_DEVICE, "needle cull: %s", hipGetErrorString(e));
    if (r.m == 0) return fail(DIVAS_ERR_ARG, "no surfel has finite scales and aspect");
    if (tau_a) *tau_a = r.tau;
    if (n_culled) *n_culled = r.n_culled;
    return DIVAS_OK;
}
}  // namespace

extern "C" {

divas_status divas_needle_cull(divas_ctx ctx, const float* scales, int64_t n, double eps, uint8_t* labels,
                               double* tau_a, int64_t* n_culled, divas_stream stream) {
    const divas_status st = check_needle(ctx, scales, n, eps, labels);
    if (st != DIVAS_OK) return st;
    DeviceGuard dg(ctx->device);
    void* scr = nullptr;
    const size_t need = needle_cull_scratch(n);
    if (ctx_scratch(ctx, need, &scr) != hipSuccess) return fail(DIVAS_ERR_OOM, "device scratch of %zu bytes", need);
    return needle_call(scales, n, eps, labels, tau_a, n_culled, scr, need, stream);
}

divas_status divas_needle_cull_noalloc(divas_ctx ctx, const float* scales, int64_t n, double eps, uint8_t* labels,
                                       double* tau_a, int64_t* n_culled, divas_stream stream) {
    const divas_status st = check_needle(ctx, scales, n, eps, labels);
    if (st != DIVAS_OK) return st;
    if (n > DIVAS_NOALLOC_MAX_SURFELS)
        return fail(DIVAS_ERR_CAPACITY, "n = %lld exceeds the fixed scratch's maximum of %d surfels", (long long)n,
                    DIVAS_NOALLOC_MAX_SURFELS);
    const size_t need = needle_cull_scratch(n, false);  // candidates only in what is left of the fixed array
    if (!ctx->static_scratch || need > kStaticScratchBytes)
        return fail(DIVAS_ERR_STATE, "fixed device scratch unavailable (%zu bytes needed)", need);
    DeviceGuard dg(ctx->device);
    return needle_call(scales, n, eps, labels, tau_a, n_culled, ctx->static_scratch, kStaticScratchBytes, stream);
}

}  // extern "C"
