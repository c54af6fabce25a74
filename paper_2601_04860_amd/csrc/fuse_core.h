// Per-chunk device code of the culling and of the fusion, shared by the
// single-session kernels (fuse.hip) and the batched persistent kernels
// (batch.hip): a voxel's result is computed by the same instructions in both.
#pragma once

#include "kernels.h"
#include "sample.h"

namespace divas {

// Per-wavefront values made scalar for the compiler (v_readfirstlane): loads
// addressed by them go through the scalar cache and branches on them stay
// uniform.  Only for values that are equal on every lane of the wavefront.
__device__ __forceinline__ int wave_uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ int wave_in_block() { return wave_uniform((int)(threadIdx.x >> 6)); }

// The conservative pixel rectangle of a chunk in a view, in hot tiles, and
// the decisions that do not need the tiles.
struct CullRect {
    int tx0, tx1, ty0, ty1;
    bool behind, nearp, empty;
};

// Can any voxel of the chunk whose voxel-index bounding box is `b` vote in view
// v?  Conservative: 0 only when no voxel centre of the box projects onto a hot
// tile (or every centre is behind the camera).  cull_rect projects the box,
// cull_tiles tests the view's hot-tile words; the rectangle depends only on
// the camera, so views that share a camera (several targets of one scene)
// share it.
//
// The box of voxel centres is projected through its 8 corners in float: the
// camera coordinates of the low corner plus the box's three edge vectors
// (columns of the rotation scaled by the extents), so a corner costs at most
// three additions.  Every float camera coordinate is within
// qerr = 2^-20 (|p|_1 + |o|_1 + |p - o|_1) of the binary64 one (the rounding
// of p, o, R and of at most eight operations, each below 2^-24 of these
// magnitudes), which bounds the pixel error by
// f (1 + |u_n| + |v_n|) qerr / z_min; the rectangle is widened by twice that
// plus one pixel (which also covers the rounding of the pixel mapping and of
// the hardware reciprocal).  Boxes reaching the camera plane are kept.
__device__ __forceinline__ CullRect cull_rect(const ChunkBox* __restrict__ b, double eps, const DView& v) {
    const float4 b0 = ldg4(&b->lo[0]), b1 = ldg4(&b->ext[0]);
    const float lo[3] = {b0.x, b0.y, b0.z}, ext[3] = {b1.x, b1.y, b1.z};
    const float P1 = b0.w;
    float D1 = 0.f;
#pragma unroll
    for (int k = 0; k < 3; ++k) D1 += fmaxf(fabsf(lo[k] - v.fo[k]), fabsf(lo[k] + ext[k] - v.fo[k]));
    const float O1 = fabsf(v.fo[0]) + fabsf(v.fo[1]) + fabsf(v.fo[2]);
    const float qerr = 0x1p-20f * (P1 + O1 + D1);
    const float d0 = lo[0] - v.fo[0], d1 = lo[1] - v.fo[1], d2 = lo[2] - v.fo[2];
    float cx[8], cy[8], cz[8];
    cx[0] = v.fR[0] * d0 + v.fR[3] * d1 + v.fR[6] * d2;
    cy[0] = v.fR[1] * d0 + v.fR[4] * d1 + v.fR[7] * d2;
    cz[0] = v.fR[2] * d0 + v.fR[5] * d1 + v.fR[8] * d2;
#pragma unroll
    for (int k = 0; k < 3; ++k) {  // corners with bit k set = corners without it + edge vector k
        const float ex = v.fR[3 * k] * ext[k], ey = v.fR[3 * k + 1] * ext[k], ez = v.fR[3 * k + 2] * ext[k];
#pragma unroll
        for (int j = 0; j < (1 << k); ++j) {
            cx[j + (1 << k)] = cx[j] + ex;
            cy[j + (1 << k)] = cy[j] + ey;
            cz[j + (1 << k)] = cz[j] + ez;
        }
    }
    float zmin = cz[0], zmax = cz[0];
#pragma unroll
    for (int j = 1; j < 8; ++j) {
        zmin = fminf(zmin, cz[j]);
        zmax = fmaxf(zmax, cz[j]);
    }
    CullRect r;
    r.behind = zmax < (float)eps - qerr;     // every voxel centre is behind the camera
    r.nearp = zmin < 16.0f * qerr + 1e-3f;  // the box reaches the camera plane: no bound
    float umin = INFINITY, umax = -INFINITY, vmin = INFINITY, vmax = -INFINITY, rmax = 0.f;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        const float iz = __builtin_amdgcn_rcpf(cz[j]);
        const float un = cx[j] * iz, vn = cy[j] * iz;
        rmax = fmaxf(rmax, fabsf(un) + fabsf(vn));
        const float u = v.ffx * un + v.fcx, vv = v.ffy * vn + v.fcy;
        umin = fminf(umin, u);
        umax = fmaxf(umax, u);
        vmin = fminf(vmin, vv);
        vmax = fmaxf(vmax, vv);
    }
    const float pad = 1.0f + fmaxf(v.ffx, v.ffy) * (1.0f + rmax) * 2.0f * qerr / (r.nearp ? 1.0f : zmin);
    // pixel rectangle; the bounds are kept finite (and every value below in
    // range) also where the projection is not used (behind, nearp)
    const float lim = 1e9f;
    int x0 = (int)fminf(fmaxf(floorf(umin - pad), -lim), lim), x1 = (int)fminf(fmaxf(floorf(umax + pad), -lim), lim);
    int y0 = (int)fminf(fmaxf(floorf(vmin - pad), -lim), lim), y1 = (int)fminf(fmaxf(floorf(vmax + pad), -lim), lim);
    x0 = max(x0, 0);
    y0 = max(y0, 0);
    x1 = min(x1, v.W - 1);
    y1 = min(y1, v.H - 1);
    r.empty = (x0 > x1) | (y0 > y1);
    r.tx0 = r.empty ? 0 : x0 / kTile;
    r.tx1 = r.empty ? 0 : x1 / kTile;
    r.ty0 = r.empty ? 0 : y0 / kTile;
    r.ty1 = r.empty ? 0 : y1 / kTile;
    return r;
}

// The decisions of the cull are combined at the end rather than taken as early
// exits, so the hot-tile words of a small rectangle are loaded in one round
// (early exits let the compiler defer loads past the tests).
__device__ __forceinline__ uint8_t cull_tiles(const CullRect& r, const DView& v) {
    const uint64_t* __restrict__ T = v.tile_bits;
    const int nw = (v.tw + 63) >> 6, w0 = r.tx0 >> 6, w1 = r.tx1 >> 6;
    const uint64_t mlo = ~0ull << (r.tx0 & 63), mhi = ~0ull >> (63 - (r.tx1 & 63));
    // the common small box (up to 4 tile rows, 2 words): eight loads with
    // clamped, always valid rows, issued together
    const bool small = (r.ty1 - r.ty0 < 4) & (w1 - w0 <= 1);
    const uint64_t m0 = w0 == w1 ? (mlo & mhi) : mlo, m1 = w0 == w1 ? 0ull : mhi;
    uint64_t any = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const uint64_t* row = T + (size_t)min(r.ty0 + k, r.ty1) * nw;
        any |= (ldg(row + w0) & m0) | (ldg(row + w1) & m1);
    }
    if (r.behind) return 0;
    if (r.nearp) return 1;
    if (r.empty) return 0;
    if (small) return any != 0;
    if (r.ty1 - r.ty0 >= kCullRows) return 1;  // a tall box: no bound (the fusion tests every sample)
    any = 0;
    for (int ty = r.ty0; ty <= r.ty1; ++ty) {
        const uint64_t* row = T + (size_t)ty * nw;
        if (w0 == w1) {
            any |= ldg(row + w0) & mlo & mhi;
        } else {
            any |= (ldg(row + w0) & mlo) | (ldg(row + w1) & mhi);
            for (int w = w0 + 1; w < w1; ++w) any |= ldg(row + w);
        }
    }
    return any != 0;
}

__device__ __forceinline__ uint8_t cull_chunk(const ChunkBox* __restrict__ b, double eps, const DView& v) {
    return cull_tiles(cull_rect(b, eps, v), v);
}

// Hot-tile flag of tile (tx, ty) of view v: some pixel has mask >= gate.  The
// tile's rows of the gate bitmask are written on the way.
__device__ __forceinline__ uint32_t tile_flag(const DView& v, int tx, int ty, double gate) {
    const int W = v.W, H = v.H;
    int x0 = tx * kTile, y0 = ty * kTile;
    int x1 = min(x0 + kTile, W), y1 = min(y0 + kTile, H);
    const float* __restrict__ m = v.mask;
    uint32_t hot = 0;
    bool vec = (x1 - x0 == kTile) && ((W & 3) == 0) && ((((uintptr_t)m) & 15u) == 0);
    for (int y = y0; y < y1; ++y) {
        uint32_t b = 0;
        if (vec) {
            const float* row = m + (size_t)y * W + x0;
            float4 q0 = ldg4(row), q1 = ldg4(row + 4);
            b = ((double)q0.x >= gate ? 1u : 0u) | ((double)q0.y >= gate ? 2u : 0u) |
                ((double)q0.z >= gate ? 4u : 0u) | ((double)q0.w >= gate ? 8u : 0u) |
                ((double)q1.x >= gate ? 16u : 0u) | ((double)q1.y >= gate ? 32u : 0u) |
                ((double)q1.z >= gate ? 64u : 0u) | ((double)q1.w >= gate ? 128u : 0u);
        } else {
            for (int x = x0; x < x1; ++x) b |= (double)ldg(m + (size_t)y * W + x) >= gate ? 1u << (x - x0) : 0u;
        }
        v.mbits[(size_t)y * v.mpitch + (size_t)tx] = (uint8_t)b;
        hot |= b;
    }
    return hot ? 1u : 0u;
}

// Hot-tile words of tile row ty of a view, one wavefront: every lane computes
// the flag of one tile (and the tile's bytes of the gate bitmask), a ballot
// packs 64 flags into a word.
__device__ __forceinline__ void tile_row_words(const DView& v, int ty, double gate) {
    const int lane = threadIdx.x & 63;
    const int tw = v.tw, nw = (tw + 63) >> 6;
    for (int w = 0; w < nw; ++w) {
        const int tx = w * 64 + lane;
        const uint32_t f = tx < tw ? tile_flag(v, tx, ty, gate) : 0u;
        const uint64_t word = __ballot(f != 0u);
        if (lane == 0) v.tile_bits[(size_t)ty * nw + w] = word;
    }
}

// Cull of the chunks of a job for views [s_begin, s_begin + ns): lanes are
// grouped per chunk (p2 = next power of two >= ns lanes, lane k of a group
// tests view s_begin + k); a ballot gathers the group's bits and the group's
// first lane writes the chunk's view bitmask (bits outside the range kept).
// `lane_in_job` counts lanes from the job's first chunk; groups never straddle
// a wavefront because p2 divides 64 and jobs start at a multiple of 64 lanes.
__device__ __forceinline__ void cull_group(const ChunkBox* __restrict__ box, int64_t n_act, double eps, const DView* __restrict__ views, int32_t s_begin,
                                           int32_t ns, int32_t p2, int64_t lane_in_job, uint64_t* __restrict__ cull,
                                           bool lane_live) {
    const int64_t chunk = lane_in_job / p2;
    const int k = (int)(lane_in_job - chunk * p2);
    const bool in = lane_live && chunk * kChunk < n_act;
    uint8_t hot = 0;
    if (in && k < ns) hot = cull_chunk(box + chunk, eps, views[s_begin + k]);
    const uint64_t bal = __ballot(hot != 0);
    if (in && k == 0) {
        const int base = (threadIdx.x & 63) - k;
        const uint64_t grp = p2 == 64 ? bal : ((bal >> base) & ((1ull << p2) - 1ull));
        const uint64_t range = (ns >= 64 ? ~0ull : ((1ull << ns) - 1ull)) << s_begin;
        cull[chunk] = (cull[chunk] & ~range) | ((grp << s_begin) & range);
    }
}

__device__ __forceinline__ uint64_t view_range(int s_begin, int s_end) {
    const int n = s_end - s_begin;
    return (n >= 64 ? ~0ull : ((1ull << n) - 1ull)) << s_begin;
}

__device__ __forceinline__ void voxel_centre(const DGrid& g, uint32_t lin, uint32_t* iv, double* c) {
    const uint32_t msk = (uint32_t)g.dim - 1u;
    iv[0] = lin & msk;
    iv[1] = (lin >> g.log2dim) & msk;
    iv[2] = lin >> (2 * g.log2dim);
    for (int k = 0; k < 3; ++k) c[k] = g.origin[k] + ((double)iv[k] + 0.5) * g.h;
}

// Counts of one or more chunks (wave-uniform values): the result counts, and
// the work done by the hot path (chunks fused with views to evaluate, those
// (chunk, view) pairs, and the samples whose pixel passed the mask gate and so
// gathered the depth maps).
struct Counts3 {
    uint64_t seg, flag, votes, hot_chunks, hot_pairs, gathered;
};

__device__ __forceinline__ void add_counts(Counts3& acc, const Counts3& c) {
    acc.seg += c.seg;
    acc.flag += c.flag;
    acc.votes += c.votes;
    acc.hot_chunks += c.hot_chunks;
    acc.hot_pairs += c.hot_pairs;
    acc.gathered += c.gathered;
}

// Adds a wave's counts to one of the kCountSlots partial slots (lane 0): the
// six fields as three 64-bit words of two 32-bit halves (field 2w low, 2w + 1
// high), so at most three atomics.  The fields may be changes modulo 2^64
// (resident outputs); a slot's word is then (low total) + 2^32 (high total)
// modulo 2^64, both totals signed and below 2^31 in magnitude.
__device__ __forceinline__ void flush_counts(int64_t* __restrict__ slots, int64_t slot, const Counts3& c, int lane) {
    if (lane != 0) return;
    unsigned long long* p = (unsigned long long*)(slots + (slot & (kCountSlots - 1)) * kSlotWords);
    const uint64_t w[3] = {c.seg + (c.flag << 32), c.votes + (c.hot_chunks << 32), c.hot_pairs + (c.gathered << 32)};
#pragma unroll
    for (int k = 0; k < 3; ++k)
        if (w[k]) atomicAdd(p + k, (unsigned long long)w[k]);
}

// The lane's share of the slots (slots lane, lane + 64, ...), unpacked into
// the six fields and cleared for the next fusion; the caller sums the lanes.
__device__ __forceinline__ void take_slots(int64_t* __restrict__ slots, int lane, uint64_t (&v)[6]) {
#pragma unroll
    for (int k = 0; k < 6; ++k) v[k] = 0;
    for (int q = lane; q < kCountSlots; q += 64) {
#pragma unroll
        for (int w = 0; w < 3; ++w) {
            const int64_t s = slots[q * kSlotWords + w];
            slots[q * kSlotWords + w] = 0;
            const int64_t lo = (int32_t)(uint32_t)((uint64_t)s & 0xFFFFFFFFull);  // signed low half
            const int64_t hi = (int64_t)((uint64_t)s - (uint64_t)lo) >> 32;
            v[2 * w] += (uint64_t)lo;
            v[2 * w + 1] += (uint64_t)hi;
        }
    }
}

// Compact fusion, consensus threshold, outputs and bitfield update of the
// wavefront's chunk, from the lanes' accumulators; returns the chunk's counts.
// lin == kNoLin: the voxel index is loaded only if the segmentation changes.
// NOVOTE: the chunk has no vote at all (W = Z = 0, no view bit), so P = 0
// without a division and the vote count is zero without a reduction.
constexpr uint32_t kNoLin = 0xFFFFFFFFu;
template <bool NOVOTE = false>
__device__ __forceinline__ Counts3 finalize_chunk(const FuseArgs& a, int64_t i, bool live, uint32_t lin, double Wx,
                                                  double Zx, uint64_t vm, bool store, uint8_t old_seg) {
    double P64 = 0.0;
    if constexpr (!NOVOTE) P64 = Zx > a.p.eps ? Wx / Zx : 0.0;
    bool seg = live && (P64 >= a.p.tau_cons);
    bool flag = live && (fabs(P64 - a.p.tau_cons) <= 1e-5);
    if (live) {
        a.P[i] = (float)P64;
        a.vout[i] = seg ? vm : 0;
        if (store) {
            a.W[i] = Wx;
            a.Z[i] = Zx;
            a.vraw[i] = vm;
        }
        const bool old = old_seg != 0;
        if (seg != old) {
            if (lin == kNoLin) lin = a.act[i];  // cold chunks read the index only here
            a.segb[i] = seg ? 1 : 0;
            const uint32_t bit = 1u << (lin & 31u);
            if (seg)
                atomicOr(&a.bits[lin >> 5], bit);
            else
                atomicAnd(&a.bits[lin >> 5], ~bit);
            const uint32_t msk = (uint32_t)a.g.dim - 1u;
            const uint32_t cell =
                coarse_cell(a.g, lin & msk, (lin >> a.g.log2dim) & msk, lin >> (2 * a.g.log2dim));
            atomicAdd(&a.coarse[cell], seg ? 1u : 0xFFFFFFFFu);  // +1 / -1
        }
    }
    uint64_t votes = 0;
    if constexpr (!NOVOTE) {
        votes = live ? (uint64_t)__popcll(vm) : 0;
        for (int off = 32; off > 0; off >>= 1) votes += __shfl_xor(votes, off);
    }
    return Counts3{(uint64_t)__popcll(__ballot(seg)), (uint64_t)__popcll(__ballot(flag)), votes, 0, 0, 0};
}

// One wavefront fuses one chunk of 64 active voxels over the views of
// [a.s_begin, a.s_end) whose cull bit is set: binary64 accumulation in view
// order, then finalize_chunk.  lin_in and seg_in are the lane's active-list
// entry and segmentation flag, loaded by the caller (entries past n ignored).
//
// COOP (thin paths only): every wavefront of the block runs this for the same
// chunk; the thick samples, the eligibility and the accumulation are computed
// identically by each, and the footprints eligible for the thin sweep are
// shared out among them (footprint k to wavefront k mod waves), their scores
// passed through LDS.  A footprint's score is the same whichever wavefront
// sweeps it, so the results equal the one-wavefront ones.  Only wavefront 0
// finalizes; the others return zero counts.
template <int MODE, bool COOP = false>
__device__ __forceinline__ Counts3 fuse_chunk(const FuseArgs& a, int64_t n, int64_t chunk, int lane, uint32_t lin_in,
                                              uint8_t seg_in) {
    const int64_t i = chunk * kChunk + lane;
    const bool live = i < n;
    const uint32_t lin = live ? lin_in : 0u;
    const uint8_t old_seg = live ? seg_in : (uint8_t)0;
    uint32_t iv[3];
    double c[3];
    voxel_centre(a.g, lin, iv, c);
    double Wx = 0.0, Zx = 0.0;
    uint64_t vm = 0;
    if (a.load_acc && live) {
        Wx = a.W[i];
        Zx = a.Z[i];
        vm = a.vraw[i];
    }
    // resident outputs: the chunk's counts as the previous fusion counted them
    // (same arithmetic as finalize_chunk), to be replaced by the new ones
    Counts3 old{};
    if (a.delta) {  // uniform
        const double P0 = Zx > a.p.eps ? Wx / Zx : 0.0;
        old.seg = (uint64_t)__popcll(__ballot(old_seg != 0));
        old.flag = (uint64_t)__popcll(__ballot(live && fabs(P0 - a.p.tau_cons) <= 1e-5));
        uint64_t v0 = live ? (uint64_t)__popcll(vm) : 0;
        for (int off = 32; off > 0; off >>= 1) v0 += __shfl_xor(v0, off);
        old.votes = v0;
    }
    constexpr bool ANY = MODE == kAnyMode || MODE == kAnyThin;  // per-session choice at run time
    const bool diff = MODE == kDiff || (ANY && a.p.differentiable);
    uint64_t todo = (a.cull_all ? ~0ull : a.cull[chunk]) & view_range(a.s_begin, a.s_end);  // uniform
    const uint64_t pairs = (uint64_t)__popcll(todo);
    uint64_t gathered = 0;
    if constexpr (MODE == kThick || MODE == kThickNsamp) {
        // two-stage pipeline over the views: the projection and mask load of the
        // next view are issued before the current view's gathers and arithmetic;
        // votes are still added in view order
        constexpr bool NS = MODE == kThickNsamp;
        int s = -1;
        SampleHead h{};
        if (todo) {
            s = __ffsll((unsigned long long)todo) - 1;
            todo &= todo - 1;
            h = sample_head(a.views[s], c, a.p.eps);  // every lane (branch-free)
        }
        while (s >= 0) {
            int sn = -1;
            SampleHead hn{};
            if (todo) {
                sn = __ffsll((unsigned long long)todo) - 1;
                todo &= todo - 1;
                hn = sample_head(a.views[sn], c, a.p.eps);
            }
            double w = 0.0, m = 0.0;
            bool gath = false;
            const bool vote = thick_sample_wave<NS>(a.views[s], a.g, a.p, iv, c, h, live, lane, &w, &m, &gath);
            gathered += (uint64_t)__popcll(__ballot(gath));
            if (vote) {
                Wx += m * w;
                Zx += w;
                vm |= (uint64_t)1 << s;
            }
            s = sn;
            h = hn;
        }
    } else {
        __shared__ double coop_score[kChunk];  // COOP: the thin scores of the chunk's lanes
        (void)coop_score;
        // points of the lane's voxel, for the density floor of the thin fallback
        uint32_t rho = 0;
        if constexpr (MODE == kThin || MODE == kNerfThin || MODE == kAnyThin)
            if (a.rho && live) rho = a.rho[i];
        // thin paths: fixed by the kernel, or (generic batch kernel) per session
        const bool thin_gs = MODE == kThin || (MODE == kAnyThin && a.p.thin && a.p.variant != kVariantNerf);
        const bool thin_nerf = MODE == kNerfThin || (MODE == kAnyThin && a.p.thin && a.p.variant == kVariantNerf);
        while (todo) {
            const int s = __ffsll((unsigned long long)todo) - 1;
            todo &= todo - 1;
            double w = 0.0, m = 0.0;
            bool vote = false, gath = false;
            const DView& v = a.views[s];
            // the 2DGS thick path (uniform per wavefront): head, footprint
            // statistics of the lanes past the gate, tail
            const bool thick = MODE == kThin || (ANY && a.p.variant != kVariantNerf && !diff);
            if (thick) {
                vote = thick_sample_wave<true>(v, a.g, a.p, iv, c, sample_head(v, c, a.p.eps), live, lane, &w, &m,
                                               &gath);
            } else if (live) {
                if constexpr (MODE == kDiff)
                    vote = diff_sample(v, a.g, a.p, c, &w, &m, &gath);
                else if constexpr (MODE == kNerf || MODE == kNerfThin)
                    vote = nerf_sample(v, a.g, a.p, c, &w, &m, &gath);
                else
                    vote = a.p.variant == kVariantNerf ? nerf_sample(v, a.g, a.p, c, &w, &m, &gath)
                                                       : diff_sample(v, a.g, a.p, c, &w, &m, &gath);
            }
            if (MODE == kThin || (MODE == kAnyThin && thin_gs)) {  // uniform
                // thin fallback: the lanes whose sample the thick path rejected
                // and that pass its entry gates, one footprint at a time, swept
                // by the whole wavefront
                double xd = 0.0;
                const bool elig = live && !vote && thin_eligible(a.views[s], a.g, a.p, c, rho, &xd);
                uint64_t todo_t = __ballot(elig);
                const bool any_t = todo_t != 0;  // uniform across the block under COOP
                for (int k = 0; todo_t; ++k) {  // uniform
                    const int l = __ffsll((unsigned long long)todo_t) - 1;
                    todo_t &= todo_t - 1;
                    if (COOP && k % (int)(blockDim.x >> 6) != wave_in_block()) continue;
                    uint32_t ivl[3];
                    double cl[3];
                    for (int q = 0; q < 3; ++q) {
                        ivl[q] = (uint32_t)__shfl((int)iv[q], l);
                        cl[q] = __shfl(c[q], l);
                    }
                    const double t = thin_score_wave(a.views[s], a.g, a.p, ivl, cl, __shfl(xd, l), lane);
                    if constexpr (COOP) {
                        if (lane == 0) coop_score[l] = t;
                    } else if (lane == l && t >= a.p.tau_thin) {
                        vote = true;
                        w = 1.0;
                        m = t;
                    }
                }
                if constexpr (COOP) {
                    if (any_t) {
                        __syncthreads();
                        const double t = coop_score[lane];
                        if (elig && t >= a.p.tau_thin) {
                            vote = true;
                            w = 1.0;
                            m = t;
                        }
                        __syncthreads();  // the scores are read before the next view writes them
                    }
                }
            }
            if (MODE == kNerfThin || (MODE == kAnyThin && thin_nerf)) {  // uniform
                // NeRF thin path (Alg. nerf-fusion): the lanes whose sample the
                // thick path did not accept and that pass the entry tests, one
                // footprint at a time, swept by the whole wavefront
                double xd = 0.0;
                const bool elig = live && !vote && nerf_thin_eligible(a.views[s], a.g, a.p, c, rho, &xd);
                uint64_t todo_t = __ballot(elig);
                const bool any_t = todo_t != 0;  // uniform across the block under COOP
                for (int k = 0; todo_t; ++k) {  // uniform
                    const int l = __ffsll((unsigned long long)todo_t) - 1;
                    todo_t &= todo_t - 1;
                    if (COOP && k % (int)(blockDim.x >> 6) != wave_in_block()) continue;
                    uint32_t ivl[3];
                    for (int q = 0; q < 3; ++q) ivl[q] = (uint32_t)__shfl((int)iv[q], l);
                    const double t = nerf_thin_score_wave(a.views[s], a.g, a.p, ivl, __shfl(xd, l), lane);
                    if constexpr (COOP) {
                        if (lane == 0) coop_score[l] = t;
                    } else if (lane == l && t >= a.p.tau_thin) {
                        vote = true;
                        w = 1.0;
                        m = t;
                    }
                }
                if constexpr (COOP) {
                    if (any_t) {
                        __syncthreads();
                        const double t = coop_score[lane];
                        if (elig && t >= a.p.tau_thin) {
                            vote = true;
                            w = 1.0;
                            m = t;
                        }
                        __syncthreads();
                    }
                }
            }
            gathered += (uint64_t)__popcll(__ballot(gath));
            if (vote) {
                Wx += m * w;
                Zx += w;
                vm |= (uint64_t)1 << s;
            }
        }
    }
    if (COOP && wave_in_block() != 0) return Counts3{};  // wavefront 0 finalizes
    Counts3 cn = finalize_chunk(a, i, live, lin, Wx, Zx, vm, a.store_acc != 0, old_seg);
    cn.seg -= old.seg;  // modulo 2^64: the slots sum to the signed change
    cn.flag -= old.flag;
    cn.votes -= old.votes;
    cn.hot_chunks = 1;
    cn.hot_pairs = pairs;
    cn.gathered = gathered;
    return cn;
}

// A chunk with no cull bit in the fused range: no new vote, so its outputs
// follow from the resident accumulators (fold) or from zero (fresh fusion);
// unchanged accumulators are not written back.  lin_in (kNoLin: read when
// needed) and seg_in as for fuse_chunk.
__device__ __forceinline__ Counts3 cold_chunk(const FuseArgs& a, int64_t n, int64_t chunk, int lane, uint32_t lin_in,
                                              uint8_t seg_in) {
    const int64_t i = chunk * kChunk + lane;
    const bool live = i < n;
    const uint32_t lin = lin_in;
    if (!a.load_acc)  // fresh fusion: nothing to accumulate (uniform)
        return finalize_chunk<true>(a, i, live, lin, 0.0, 0.0, 0ull, a.store_acc != 0, live ? seg_in : (uint8_t)0);
    double Wx = 0.0, Zx = 0.0;
    uint64_t vm = 0;
    if (live) {
        Wx = a.W[i];
        Zx = a.Z[i];
        vm = a.vraw[i];
    }
    (void)lane;
    return finalize_chunk(a, i, live, lin, Wx, Zx, vm, a.store_acc != 0 && !a.load_acc, live ? seg_in : (uint8_t)0);
}

}  // namespace divas
