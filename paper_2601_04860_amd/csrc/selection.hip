// Exact order-statistic selection and the two pre-passes built on it:
//   - scene-statistic grid construction: Sec. 3.5 (i), Eq. scene-norm and
//     Eq. voxel-size;
//   - depth refinement of a view's mask: Sec. 3.2 "Depth-weighting",
//     Eq. depthband with Eq. gs-bandpass (2DGS) and Eq. nerf-depthweight.
//
// The grid statistics are order statistics of the points: the coordinate-wise
// median of the centres, the 99th percentile of their distance to that median,
// and the median scale.  Each is found exactly by a most-significant-digit
// radix selection over order-preserving integer keys: float32 values map to
// 32-bit keys, the non-negative binary64 distances to their 64-bit patterns.
// A pass histograms one 8-bit digit of the keys that share the digits found
// so far (a block histogram in LDS, merged with one atomic per bin); the
// digit that holds the wanted rank is picked from that histogram by every
// block of the next pass (one wavefront's scan of 256 bins, cheaper than a
// launch of its own) and, after the last pass, by a one-wavefront launch that
// also turns the selected keys into the statistic.  Two ranks are selected
// together (the two middle elements of an even count, or the two neighbours
// of the percentile position).  Everything between the statistics runs on
// the device as well: one-thread launches set the ranks from the count of
// keys and evaluate the closed forms in binary64, and the launches that
// depend on a statistic (the distances need the centre) read it from device
// memory.  The host waits once per call, for the results.  The keys of the
// three coordinates and the scales are written by one pass over the points.
//
// A point takes part iff its coordinates (and its scale, when scales are
// given) are finite; the others get the largest key, which no selected rank
// reaches.  Distances are sqrt((dx^2 + dy^2) + dz^2) in binary64, in that
// order, and the kept count uses the library's voxel rule.
//
// The band-pass refinement selects d_far, the 98th percentile of the
// median-depth map over pixels with a surface (finite depth > 0), the same
// way; the band is the range of the median depths at the prompt pixels and at
// the view centre (gathered by one small launch).  The min-max refinement
// needs the extreme depths only (order-preserving keys, one atomic min and
// max per wavefront).  The per-pixel weights are binary64 in the order of the
// equations, and the refined value M * (1 - weight) is rounded once to
// float32; a pixel without a surface gets weight 0.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <vector>

#include "kernels.h"

namespace divas {

namespace {

constexpr int kSelThreads = 256;
constexpr int kSelBins = 256;
constexpr int kSelTargets = 2;

__device__ __forceinline__ uint32_t float_key(float x) {
    const uint32_t u = __float_as_uint(x);
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}

__host__ __device__ __forceinline__ float key_float(uint32_t k) {
    const uint32_t u = (k & 0x80000000u) ? (k & 0x7FFFFFFFu) : ~k;
    float f;
    __builtin_memcpy(&f, &u, 4);
    return f;
}

// Counting launches stride over their input with a bounded grid and add one
// block total to the global counter: one atomic per wavefront on a single
// address would serialise tens of thousands of atomics.
constexpr int kCountThreads = 256;
constexpr unsigned kCountBlocks = 512;

// Sum of v over the block, valid in thread 0.
__device__ __forceinline__ unsigned block_total(unsigned v) {
    __shared__ unsigned part[kCountThreads / 64];
    for (int off = 32; off > 0; off >>= 1) v += (unsigned)__shfl_xor((int)v, off);
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = v;
    __syncthreads();
    unsigned t = 0;
    if (threadIdx.x == 0)
        for (int k = 0; k < kCountThreads / 64; ++k) t += part[k];
    return t;
}

__device__ __forceinline__ bool point_takes_part(const float* __restrict__ xyz, const float* __restrict__ scale,
                                                 int64_t i) {
    bool ok = isfinite(xyz[3 * i]) && isfinite(xyz[3 * i + 1]) && isfinite(xyz[3 * i + 2]);
    if (scale) ok = ok && isfinite(scale[i]);
    return ok;
}

// The coordinates of points 4q .. 4q + 3 from three 16-byte loads (xyz
// 16-byte aligned), and their scales from one (scale 16-byte aligned).
__device__ __forceinline__ void load_quad(const float* __restrict__ xyz, int64_t q, float (&x)[4], float (&y)[4],
                                          float (&z)[4]) {
    const float4* p = (const float4*)(xyz + 12 * q);
    const float4 a = p[0], b = p[1], c = p[2];
    x[0] = a.x, y[0] = a.y, z[0] = a.z;
    x[1] = a.w, y[1] = b.x, z[1] = b.y;
    x[2] = b.z, y[2] = b.w, z[2] = c.x;
    x[3] = c.y, y[3] = c.z, z[3] = c.w;
}
__device__ __forceinline__ void load_quad_scale(const float* __restrict__ scale, int64_t q, float (&s)[4]) {
    const float4 v = ((const float4*)scale)[q];
    s[0] = v.x, s[1] = v.y, s[2] = v.z, s[3] = v.w;
}

// The keys of the points, one array per statistic: keys[a n + i] = key of
// xyz[i][a] (a = 0..2) and, with scales, keys[3 n + i] = key of scale[i];
// counts the points that take part into *m.  QUAD: four points per step of a
// lane, 16-byte loads and stores (xyz, scale and keys 16-byte aligned, n a
// multiple of 4).
template <bool QUAD>
__global__ __launch_bounds__(kCountThreads) void k_keys_points(const float* __restrict__ xyz,
                                                                const float* __restrict__ scale, int64_t n,
                                                                uint32_t* __restrict__ keys,
                                                                unsigned long long* __restrict__ m) {
    unsigned cnt = 0;
    const int64_t stride = (int64_t)gridDim.x * kCountThreads;
    if constexpr (QUAD) {
        const int64_t n4 = n / 4;
        for (int64_t q = blockIdx.x * (int64_t)kCountThreads + threadIdx.x; q < n4; q += stride) {
            float x[4], y[4], z[4], sc[4] = {0.0f, 0.0f, 0.0f, 0.0f};
            load_quad(xyz, q, x, y, z);
            if (scale) load_quad_scale(scale, q, sc);
            uint32_t kx[4], ky[4], kz[4], ks[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const bool part = isfinite(x[k]) && isfinite(y[k]) && isfinite(z[k]) && (!scale || isfinite(sc[k]));
                kx[k] = part ? float_key(x[k]) : 0xFFFFFFFFu;
                ky[k] = part ? float_key(y[k]) : 0xFFFFFFFFu;
                kz[k] = part ? float_key(z[k]) : 0xFFFFFFFFu;
                ks[k] = part ? float_key(sc[k]) : 0xFFFFFFFFu;
                cnt += part ? 1u : 0u;
            }
            ((uint4*)keys)[q] = make_uint4(kx[0], kx[1], kx[2], kx[3]);
            ((uint4*)(keys + n))[q] = make_uint4(ky[0], ky[1], ky[2], ky[3]);
            ((uint4*)(keys + 2 * n))[q] = make_uint4(kz[0], kz[1], kz[2], kz[3]);
            if (scale) ((uint4*)(keys + 3 * n))[q] = make_uint4(ks[0], ks[1], ks[2], ks[3]);
        }
    } else {
        for (int64_t i = blockIdx.x * (int64_t)kCountThreads + threadIdx.x; i < n; i += stride) {
            const bool part = point_takes_part(xyz, scale, i);
#pragma unroll
            for (int a = 0; a < 3; ++a) keys[a * n + i] = part ? float_key(xyz[3 * i + a]) : 0xFFFFFFFFu;
            if (scale) keys[3 * n + i] = part ? float_key(scale[i]) : 0xFFFFFFFFu;
            cnt += part ? 1u : 0u;
        }
    }
    const unsigned t = block_total(cnt);
    if (threadIdx.x == 0 && t) atomicAdd(m, (unsigned long long)t);
}

// The bit pattern of the binary64 distance of (x, y, z) to the centre, or the
// largest key for a point that takes no part.
__device__ __forceinline__ uint64_t distance_key(bool part, float x, float y, float z, double cx, double cy,
                                                 double cz) {
    if (!part) return ~0ull;
    const double dx = (double)x - cx;
    const double dy = (double)y - cy;
    const double dz = (double)z - cz;
    const double d = sqrt((dx * dx + dy * dy) + dz * dz);
    return (uint64_t)__double_as_longlong(d);
}

// keys[i] = bit pattern of the binary64 distance of point i to the centre c;
// one point per thread, or (QUAD, as for k_keys_points) four.
template <bool QUAD>
__global__ void k_keys_distance(const float* __restrict__ xyz, const float* __restrict__ scale, int64_t n,
                                const double* __restrict__ c, uint64_t* __restrict__ keys) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const double cx = c[0], cy = c[1], cz = c[2];
    if constexpr (QUAD) {
        if (i >= n / 4) return;
        float x[4], y[4], z[4], sc[4] = {0.0f, 0.0f, 0.0f, 0.0f};
        load_quad(xyz, i, x, y, z);
        if (scale) load_quad_scale(scale, i, sc);
        uint64_t k4[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const bool part = isfinite(x[k]) && isfinite(y[k]) && isfinite(z[k]) && (!scale || isfinite(sc[k]));
            k4[k] = distance_key(part, x[k], y[k], z[k], cx, cy, cz);
        }
        ((ulonglong2*)keys)[2 * i] = make_ulonglong2(k4[0], k4[1]);
        ((ulonglong2*)keys)[2 * i + 1] = make_ulonglong2(k4[2], k4[3]);
    } else {
        if (i >= n) return;
        keys[i] = distance_key(point_takes_part(xyz, scale, i), xyz[3 * i], xyz[3 * i + 1], xyz[3 * i + 2], cx, cy,
                               cz);
    }
}

// Selection state: for each target rank, the key digits found so far (the
// bits above the digit of the next pass; the bits below are zero) and the
// rank left among the keys that share them.
struct SelState {
    unsigned long long prefix[kSelTargets];
    unsigned long long rank[kSelTargets];
};

// Most passes of one selection (8-bit digits of 64-bit keys).
constexpr int kSelMaxPasses = 8;
constexpr int kSelHistWords = kSelTargets * kSelBins;

// The device buffers of a selection: two state slots (the state before pass
// j is in slot j % 2, the ranks kernel writes slot 0) and one histogram per
// pass.  Every histogram is zero before a selection and after it.
struct SelBuffers {
    SelState* slots;      // [2]
    unsigned int* hists;  // [kSelMaxPasses][kSelTargets][kSelBins]
    void* cand;           // room for cand_cap keys (may be null)
    int64_t cand_cap;
    unsigned long long* n_cand;  // zero before a selection that gathers candidates
};

// How a pass finds its keys: all of them; all of them, gathering those that
// match a target's prefix into the candidate buffer; or the candidates
// gathered by an earlier pass when they all fit (else all keys again).
constexpr int kPassAll = 0;
constexpr int kPassGather = 1;
constexpr int kPassCand = 2;
// The pass of a 64-bit selection that gathers candidates: two digits are
// known by then, and the keys that share them are usually few.
constexpr int kGatherPass = 2;

// The pick after a pass, by one wavefront (lane l holds bins 4l .. 4l + 3):
// for each target, the digit whose bin holds the remaining rank joins the
// prefix, and the keys of the lower bins leave the rank.  A pass that found
// the two prefixes equal counted its keys once, in the first histogram.  A
// rank beyond the keys (no bin holds it) leaves the state as it is.
__device__ SelState sel_pick_wave(const SelState in, const unsigned int* __restrict__ hist, int shift, int lane) {
    SelState out = in;
    const bool one = in.prefix[0] == in.prefix[1];
#pragma unroll
    for (int t = 0; t < kSelTargets; ++t) {
        const uint4 v = *(const uint4*)(hist + (one ? 0 : t) * kSelBins + 4 * lane);
        const unsigned own = v.x + v.y + v.z + v.w;
        unsigned incl = own;
        for (int off = 1; off < 64; off <<= 1) {  // inclusive scan over the lanes
            const unsigned x = (unsigned)__shfl_up((int)incl, off);
            if (lane >= off) incl += x;
        }
        const unsigned long long r = in.rank[t];
        unsigned long long below = incl - own;
        const unsigned vb[4] = {v.x, v.y, v.z, v.w};
        int bin = -1;
        unsigned long long rest = 0;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            if (bin < 0 && vb[k] && r >= below && r < below + vb[k]) {
                bin = 4 * lane + k;
                rest = r - below;
            }
            below += vb[k];
        }
        const unsigned long long hit = __ballot(bin >= 0);  // one lane at most
        if (hit) {
            const int src = __ffsll((long long)hit) - 1;
            out.prefix[t] = in.prefix[t] | ((unsigned long long)__shfl(bin, src) << shift);
            out.rank[t] = __shfl(rest, src);
        }
    }
    return out;
}

// Pass `pass` of a selection over keys[0, n): every block first takes the
// pick of the previous pass (from its histogram and state; block 0 stores the
// new state for the next pass and clears the histogram of the pass before),
// then histograms the digit of this pass over the keys whose bits above it
// equal a target's prefix (a block histogram in LDS, merged with one atomic
// per nonzero bin).  When the two targets share their prefix (always in the
// first pass, and for adjacent ranks mostly after it) the keys are counted
// once, for both.
//
// A gathering pass counts its block's matching keys in LDS, reserves their
// room with one global atomic per block, and reads its keys a second time to
// write them; keys past the buffer's capacity are not written, and the later
// passes then read all keys.
template <class K, int SRC>
__global__ __launch_bounds__(kSelThreads) void k_sel_pass(const K* __restrict__ keys, int64_t n, int pass,
                                                          SelBuffers sb) {
    static_assert(kSelTargets == 2 && kSelThreads == kSelBins && kSelBins == 4 * 64, "two targets, 4 bins a lane");
    constexpr int kBits = 8 * (int)sizeof(K);
    const int shift = kBits - 8 * (pass + 1);
    __shared__ unsigned int h[kSelTargets][kSelBins];
    __shared__ SelState cur;
    for (int b = threadIdx.x; b < kSelHistWords; b += kSelThreads) (&h[0][0])[b] = 0u;
    if (threadIdx.x < 64) {
        SelState st = sb.slots[pass == 0 ? 0 : (pass - 1) % 2];
        if (pass > 0) st = sel_pick_wave(st, sb.hists + (pass - 1) * kSelHistWords, shift + 8, threadIdx.x);
        if (threadIdx.x == 0) {
            cur = st;
            if (pass > 0 && blockIdx.x == 0) sb.slots[pass % 2] = st;
        }
    }
    if (pass >= 2 && blockIdx.x == 0)
        for (int b = threadIdx.x; b < kSelHistWords; b += kSelThreads) sb.hists[(pass - 2) * kSelHistWords + b] = 0u;
    __syncthreads();
    const int hi = shift + 8;  // bits at and above hi are known
    K want[kSelTargets];
#pragma unroll
    for (int t = 0; t < kSelTargets; ++t) want[t] = hi < kBits ? (K)(cur.prefix[t] >> hi) : (K)0;
    const bool shared_prefix = want[0] == want[1];
    const K* src = keys;
    int64_t len = n;
    if (SRC == kPassCand) {
        const unsigned long long nc = *sb.n_cand;
        if (nc <= (unsigned long long)sb.cand_cap) {
            src = (const K*)sb.cand;
            len = (int64_t)nc;
        }
    }
    __shared__ unsigned int matched, base_room;
    if (SRC == kPassGather && threadIdx.x == 0) matched = 0u;
    if (SRC == kPassGather) __syncthreads();
    const int64_t stride = (int64_t)gridDim.x * kSelThreads;
    for (int64_t i = blockIdx.x * (int64_t)kSelThreads + threadIdx.x; i < len; i += stride) {
        const K k = src[i];
        const unsigned d = (unsigned)(k >> shift) & (kSelBins - 1);
        const K top = hi < kBits ? (K)(k >> hi) : (K)0;
        if (top == want[0]) atomicAdd(&h[0][d], 1u);
        if (!shared_prefix && top == want[1]) atomicAdd(&h[1][d], 1u);
        if (SRC == kPassGather && (top == want[0] || top == want[1])) atomicAdd(&matched, 1u);
    }
    if (SRC == kPassGather) {
        __syncthreads();
        if (threadIdx.x == 0) {
            base_room = matched ? (unsigned)atomicAdd(sb.n_cand, (unsigned long long)matched) : 0u;
            matched = 0u;
        }
        __syncthreads();
        K* cand = (K*)sb.cand;
        for (int64_t i = blockIdx.x * (int64_t)kSelThreads + threadIdx.x; i < n; i += stride) {
            const K k = keys[i];
            const K top = hi < kBits ? (K)(k >> hi) : (K)0;
            if (top == want[0] || top == want[1]) {
                const int64_t at = (int64_t)base_room + atomicAdd(&matched, 1u);
                if (at < sb.cand_cap) cand[at] = k;
            }
        }
    }
    __syncthreads();
    unsigned int* out = sb.hists + pass * kSelHistWords;
    for (int b = threadIdx.x; b < (shared_prefix ? kSelBins : kSelHistWords); b += kSelThreads) {
        const unsigned v = (&h[0][0])[b];
        if (v) atomicAdd(out + b, v);
    }
}

// Points inside the grid g by the voxel rule (nothing without a grid); QUAD
// as for k_keys_points.
template <bool QUAD>
__global__ __launch_bounds__(kCountThreads) void k_count_kept(const float* __restrict__ xyz, int64_t n,
                                                               const GridStatsResult* __restrict__ g,
                                                               unsigned long long* __restrict__ kept) {
    if (g->m == 0 || g->dim == 0) return;
    const double o[3] = {g->origin[0], g->origin[1], g->origin[2]};
    const double h = g->voxel, inv_h = 1.0 / h;
    const int32_t dim = g->dim;
    auto inside = [&](float x, float y, float z) {
        const float p[3] = {x, y, z};
        bool in = true;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const double f = voxel_floor((double)p[k] - o[k], h, inv_h);
            in = in && (f >= 0.0) && (f < (double)dim);  // NaN fails
        }
        return in;
    };
    unsigned cnt = 0;
    const int64_t stride = (int64_t)gridDim.x * kCountThreads;
    if constexpr (QUAD) {
        for (int64_t q = blockIdx.x * (int64_t)kCountThreads + threadIdx.x; q < n / 4; q += stride) {
            float x[4], y[4], z[4];
            load_quad(xyz, q, x, y, z);
#pragma unroll
            for (int k = 0; k < 4; ++k) cnt += inside(x[k], y[k], z[k]) ? 1u : 0u;
        }
    } else {
        for (int64_t i = blockIdx.x * (int64_t)kCountThreads + threadIdx.x; i < n; i += stride)
            cnt += inside(xyz[3 * i], xyz[3 * i + 1], xyz[3 * i + 2]) ? 1u : 0u;
    }
    const unsigned t = block_total(cnt);
    if (threadIdx.x == 0 && t) atomicAdd(kept, (unsigned long long)t);
}

// ---- the statistics between the selections (one thread each)

// The quantile position q (m - 1) of m keys: the lower rank i and the
// fraction f towards rank i + 1.
struct QuantPos {
    unsigned long long i;
    double f;
};

// How a selected key turns back into its value.
constexpr int kKeyF32 = 0;     // float_key of a float32
constexpr int kKeyF64Bits = 1; // the bit pattern of a non-negative binary64
constexpr int kKeyF64 = 2;     // double_key of a binary64

template <int KIND>
__device__ __forceinline__ double key_value(unsigned long long k) {
    if (KIND == kKeyF32) return (double)key_float((uint32_t)k);
    const unsigned long long u =
        KIND == kKeyF64Bits ? k : ((k & 0x8000000000000000ull) ? (k & 0x7FFFFFFFFFFFFFFFull) : ~k);
    return __longlong_as_double((long long)u);
}

// Ranks of the median of the *m keys that take part: the two middle ones,
// equal when *m is odd.
__global__ void k_ranks_median(const unsigned long long* __restrict__ m, SelState* __restrict__ st) {
    const unsigned long long c = *m;
    for (int t = 0; t < kSelTargets; ++t) st->prefix[t] = 0ull;
    st->rank[0] = c ? (c - 1) / 2 : 0ull;
    st->rank[1] = c / 2;
}

// Ranks of the q-quantile of the *m keys, linear between the order statistics
// i and i + 1 around the position q (m - 1); the position goes to *qp.
__global__ void k_ranks_quantile(const unsigned long long* __restrict__ m, double q, SelState* __restrict__ st,
                                 QuantPos* __restrict__ qp) {
    const unsigned long long c = *m;
    unsigned long long i = 0;
    double f = 0.0;
    if (c) {
        const double pos = q * (double)(c - 1);
        const double fl = floor(pos);
        i = (unsigned long long)fl;
        f = pos - fl;
    }
    for (int t = 0; t < kSelTargets; ++t) st->prefix[t] = 0ull;
    st->rank[0] = i;
    st->rank[1] = i + 1 < c ? i + 1 : i;
    qp->i = i;
    qp->f = f;
}

// The pick of the last pass of a selection of KIND keys (one wavefront),
// which leaves the two selected keys in the prefixes; clears the histograms
// of the last two passes (the earlier ones were cleared by the passes).
template <int KIND>
__device__ SelState sel_finish(SelBuffers sb, int lane) {
    constexpr int kPasses = KIND == kKeyF32 ? 4 : 8;
    const SelState st =
        sel_pick_wave(sb.slots[(kPasses - 1) % 2], sb.hists + (kPasses - 1) * kSelHistWords, 0, lane);
    for (int w = lane; w < 2 * kSelHistWords; w += 64) sb.hists[(kPasses - 2) * kSelHistWords + w] = 0u;
    return st;
}

// The median from the two selected keys: the middle value for an odd count,
// the mean of the two middle ones for an even count (nothing without keys).
template <int KIND>
__global__ __launch_bounds__(64) void k_take_median(const unsigned long long* __restrict__ m, SelBuffers sb,
                                                    double* __restrict__ dst) {
    const SelState st = sel_finish<KIND>(sb, threadIdx.x);
    const unsigned long long c = *m;
    if (threadIdx.x != 0 || !c) return;
    const double lo = key_value<KIND>(st.prefix[0]), hi = key_value<KIND>(st.prefix[1]);
    *dst = (c % 2) ? lo : (lo + hi) / 2.0;
}

// The quantile from the two selected keys, linear between them.
template <int KIND>
__global__ __launch_bounds__(64) void k_take_quantile(const unsigned long long* __restrict__ m, SelBuffers sb,
                                                      const QuantPos* __restrict__ qp, double* __restrict__ dst) {
    const SelState st = sel_finish<KIND>(sb, threadIdx.x);
    const unsigned long long c = *m;
    if (threadIdx.x != 0 || !c) return;
    const double lo = key_value<KIND>(st.prefix[0]), hi = key_value<KIND>(st.prefix[1]);
    *dst = qp->i + 1 < c ? lo + (hi - lo) * qp->f : lo;
}

// Eq. scene-norm and Eq. voxel-size from the statistics in g: the padded
// half-extent b, the voxel edge h_v (the scale term only with scales), the
// power-of-two resolution and the grid.  A zero extent or voxel edge leaves
// dim 0.
__global__ void k_grid_finish(const unsigned long long* __restrict__ m, GridStatsParams p, int with_scale,
                              GridStatsResult* __restrict__ g) {
    g->m = (int64_t)*m;
    if (g->m == 0) return;
    if (!with_scale) g->s_med = NAN;
    g->b = ceil(p.pad * g->r_fg);
    double h_v = p.beta_v * g->r_fg / (double)p.g0;
    if (with_scale) {
        const double hs = p.alpha_v * g->s_med;
        h_v = hs < h_v ? h_v : hs;
    }
    g->h_v = h_v;
    if (!(g->b > 0.0) || !(h_v > 0.0)) {
        g->dim = 0;
        return;
    }
    const double need = 2.0 * g->b / h_v;
    int32_t d = 2;
    while (d < need && d < p.g_max) d *= 2;
    g->dim = p.g_max < d ? p.g_max : d;
    for (int a = 0; a < 3; ++a) g->origin[a] = g->center[a] - g->b;
    g->voxel = 2.0 * g->b / (double)g->dim;
}

unsigned blocks_of(int64_t n, int t) { return (unsigned)((n + t - 1) / t); }

// Launches the passes that select the keys of the two ranks in slot 0 (set
// by a launch before) among keys[0, n); a k_take_* launch takes the last pick.
// A bounded grid: each block adds its nonzero bins to the pass's histogram.
// A 64-bit selection with a candidate buffer (sb.cand, *sb.n_cand zero)
// gathers the keys that share its first two digits and reads only those in
// its last passes when they fit.
template <class K>
void enqueue_select(const K* keys, int64_t n, SelBuffers sb, hipStream_t st) {
    const unsigned grid = std::min<unsigned>(blocks_of(n, kSelThreads * 16), 512u);
    const bool gather = sizeof(K) == 8 && sb.cand && sb.cand_cap > 0;
    for (int pass = 0; pass < (int)sizeof(K); ++pass) {
        if (gather && pass == kGatherPass)
            hipLaunchKernelGGL((k_sel_pass<K, kPassGather>), dim3(grid), dim3(kSelThreads), 0, st, keys, n, pass, sb);
        else if (gather && pass > kGatherPass)
            hipLaunchKernelGGL((k_sel_pass<K, kPassCand>), dim3(grid), dim3(kSelThreads), 0, st, keys, n, pass, sb);
        else
            hipLaunchKernelGGL((k_sel_pass<K, kPassAll>), dim3(grid), dim3(kSelThreads), 0, st, keys, n, pass, sb);
    }
}

double as_double(unsigned long long k) {
    double d;
    std::memcpy(&d, &k, 8);
    return d;
}

// ---- needle cull (Pass 2 of the voxel-to-surfel mapping)

// Order-preserving 64-bit key of a binary64 value.
__device__ __forceinline__ uint64_t double_key(double x) {
    const uint64_t u = (uint64_t)__double_as_longlong(x);
    return (u & 0x8000000000000000ull) ? ~u : (u | 0x8000000000000000ull);
}

// Eq. aspect of surfel i; false when a scale or the aspect is not finite.
__device__ __forceinline__ bool surfel_aspect(const float* __restrict__ scales, int64_t i, double eps, double* a) {
    const double s0 = (double)scales[2 * i], s1 = (double)scales[2 * i + 1];
    const double hi = s0 > s1 ? s0 : s1;
    const double lo = s0 > s1 ? s1 : s0;
    *a = hi / (lo + eps);
    return isfinite(s0) && isfinite(s1) && isfinite(*a);
}

// keys[i] = key of the aspect of surfel i (the largest key without one);
// counts the surfels with an aspect into *m.
__global__ __launch_bounds__(kCountThreads) void k_keys_aspect(const float* __restrict__ scales, int64_t n, double eps,
                                                                uint64_t* __restrict__ keys,
                                                                unsigned long long* __restrict__ m) {
    unsigned cnt = 0;
    const int64_t stride = (int64_t)gridDim.x * kCountThreads;
    for (int64_t i = blockIdx.x * (int64_t)kCountThreads + threadIdx.x; i < n; i += stride) {
        double a;
        const bool ok = surfel_aspect(scales, i, eps, &a);
        keys[i] = ok ? double_key(a) : ~0ull;
        cnt += ok ? 1u : 0u;
    }
    const unsigned t = block_total(cnt);
    if (threadIdx.x == 0 && t) atomicAdd(m, (unsigned long long)t);
}

// Eq. pass-needle: labels[i] &= (aspect <= *tau); counts the culled surfels
// (nothing without an aspect, *m == 0).
__global__ __launch_bounds__(kCountThreads) void k_needle_apply(const float* __restrict__ scales, int64_t n,
                                                                 double eps, const unsigned long long* __restrict__ m,
                                                                 const double* __restrict__ tau_p,
                                                                 uint8_t* __restrict__ labels,
                                                                 unsigned long long* __restrict__ culled) {
    if (*m == 0) return;
    const double tau = *tau_p;
    unsigned cnt = 0;
    const int64_t stride = (int64_t)gridDim.x * kCountThreads;
    for (int64_t i = blockIdx.x * (int64_t)kCountThreads + threadIdx.x; i < n; i += stride) {
        double a;
        const bool keep = surfel_aspect(scales, i, eps, &a) && a <= tau;
        if (!keep) labels[i] = 0;
        cnt += keep ? 0u : 1u;
    }
    const unsigned t = block_total(cnt);
    if (threadIdx.x == 0 && t) atomicAdd(culled, (unsigned long long)t);
}

// ---- mask refinement

__device__ __forceinline__ bool has_surface(float d) { return isfinite(d) && d > 0.0f; }

// keys[i] = key of depth i, or the largest key for a pixel without a surface;
// counts the surface pixels into *m.
__global__ __launch_bounds__(kCountThreads) void k_keys_depth(const float* __restrict__ d, int64_t n,
                                                               uint32_t* __restrict__ keys,
                                                               unsigned long long* __restrict__ m) {
    unsigned cnt = 0;
    const int64_t stride = (int64_t)gridDim.x * kCountThreads;
    for (int64_t i = blockIdx.x * (int64_t)kCountThreads + threadIdx.x; i < n; i += stride) {
        const float v = d[i];
        const bool s = has_surface(v);
        keys[i] = s ? float_key(v) : 0xFFFFFFFFu;
        cnt += s ? 1u : 0u;
    }
    const unsigned t = block_total(cnt);
    if (threadIdx.x == 0 && t) atomicAdd(m, (unsigned long long)t);
}

// out[k] = d[idx[k]] for the anchor pixels.
__global__ void k_gather_depth(const float* __restrict__ d, const int64_t* __restrict__ idx, int n,
                               float* __restrict__ out) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < n) out[k] = d[idx[k]];
}

// ext[0] = min key, ext[1] = max key over the surface pixels (ext preset to
// all ones and zero); counts the surface pixels into *m.
__global__ __launch_bounds__(kCountThreads) void k_depth_extrema(const float* __restrict__ d, int64_t n,
                                                                  unsigned int* __restrict__ ext,
                                                                  unsigned long long* __restrict__ m) {
    __shared__ uint32_t wlo[kCountThreads / 64], whi[kCountThreads / 64];
    uint32_t lo = 0xFFFFFFFFu, hi = 0u;
    unsigned cnt = 0;
    const int64_t stride = (int64_t)gridDim.x * kCountThreads;
    for (int64_t i = blockIdx.x * (int64_t)kCountThreads + threadIdx.x; i < n; i += stride) {
        const float v = d[i];
        if (has_surface(v)) {
            const uint32_t k = float_key(v);
            lo = k < lo ? k : lo;
            hi = k > hi ? k : hi;
            ++cnt;
        }
    }
    for (int off = 32; off > 0; off >>= 1) {
        const uint32_t a = (uint32_t)__shfl_xor((int)lo, off), b = (uint32_t)__shfl_xor((int)hi, off);
        lo = a < lo ? a : lo;
        hi = b > hi ? b : hi;
    }
    if ((threadIdx.x & 63) == 0) {
        wlo[threadIdx.x >> 6] = lo;
        whi[threadIdx.x >> 6] = hi;
    }
    const unsigned t = block_total(cnt);  // synchronises the block
    if (threadIdx.x == 0) {
        for (int k = 0; k < kCountThreads / 64; ++k) {
            lo = wlo[k] < lo ? wlo[k] : lo;
            hi = whi[k] > hi ? whi[k] : hi;
        }
        if (t) {
            atomicAdd(m, (unsigned long long)t);
            atomicMin(ext, lo);
            atomicMax(ext + 1, hi);
        }
    }
}

// The band of Eq. depthband (one thread): the range of the anchors' median
// depths (the anchors with a surface).  par[0..1] the band, par[3] the anchor
// count, par[4] 1 when the view is refined (a surface pixel and an anchor);
// par[2] receives d_far from the selection.
__global__ void k_band_anchors(const unsigned long long* __restrict__ m, const float* __restrict__ anchors, int na,
                               double* __restrict__ par) {
    double bmin = NAN, bmax = NAN;
    int cnt = 0;
    for (int k = 0; k < na; ++k) {
        const float v = anchors[k];
        if (!has_surface(v)) continue;
        const double dd = (double)v;
        if (cnt == 0 || dd < bmin) bmin = dd;
        if (cnt == 0 || dd > bmax) bmax = dd;
        ++cnt;
    }
    par[0] = bmin;
    par[1] = bmax;
    par[3] = (double)cnt;
    par[4] = *m > 0 && cnt > 0 ? 1.0 : 0.0;
}

// Eq. gs-bandpass per pixel, with the band and d_far in par (nothing is
// written when the view is not refined).
__global__ void k_refine_band(const float* mask, const float* __restrict__ d, int64_t n,
                              const double* __restrict__ par, float* out) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n || par[4] == 0.0) return;
    const double lo = par[0], hi = par[1], reach = par[2] - hi;
    const double den = reach < 1e-6 ? 1e-6 : reach;
    const float df = d[i];
    double band = 1.0;
    if (has_surface(df)) {
        const double D = (double)df;
        const double dneg = fmax(lo - D, 0.0);
        const double dpos = fmax(D - hi, 0.0);
        band = fmin(fmax((dneg + dpos) / den, 0.0), 1.0);
    }
    out[i] = (float)((double)mask[i] * (1.0 - band));
}

// Eq. nerf-depthweight per pixel (flat: every surface pixel keeps weight 1),
// with the extreme depths of k_depth_extrema (keys in ext, the surface count
// in *m; nothing is written without a surface pixel).
__global__ void k_refine_minmax(const float* mask, const float* __restrict__ d, int64_t n,
                                const unsigned int* __restrict__ ext, const unsigned long long* __restrict__ m,
                                float* out) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n || *m == 0) return;
    const double zmin = (double)key_float(ext[0]), zmax = (double)key_float(ext[1]);
    const float df = d[i];
    double z = 1.0;
    if (has_surface(df)) z = zmax > zmin ? ((double)df - zmin) / (zmax - zmin) : 0.0;
    out[i] = (float)((double)mask[i] * (1.0 - z));
}

}  // namespace

// The buffers of one run, carved from the caller's scratch (256-byte aligned
// pieces): the keys, the selection's state slots and histograms, eight
// counter words and a small region (the anchor tables, the grid statistics).
// Counter words: [0] the count of keys that take part, [1] and [2] other
// counts (or the extreme depth keys), [4] the gathered candidates of a 64-bit
// selection, [5..6] the quantile position, [7] a statistic for the host.
struct Scratch {
    void* keys = nullptr;
    SelBuffers sel{};
    unsigned long long* counters = nullptr;
    QuantPos* qpos = nullptr;
    double* stat = nullptr;
    void* small = nullptr;
};
constexpr size_t kAlign = 256;
constexpr size_t kCounterBytes = 8 * 8;
size_t up(size_t b) { return (b + kAlign - 1) / kAlign * kAlign; }
constexpr size_t kHistBytes = sizeof(unsigned) * kSelMaxPasses * kSelHistWords;
size_t fixed_bytes(size_t small) {
    return up(2 * sizeof(SelState)) + up(kHistBytes) + up(kCounterBytes) + up(small);
}
bool carve(void* base, size_t bytes, size_t key_bytes, size_t small, Scratch* sc) {
    if (bytes < up(key_bytes) + fixed_bytes(small)) return false;
    char* p = (char*)base;
    sc->keys = p;
    p += up(key_bytes);
    sc->sel.slots = (SelState*)p;
    p += up(2 * sizeof(SelState));
    sc->sel.hists = (unsigned int*)p;
    p += up(kHistBytes);
    sc->counters = (unsigned long long*)p;
    sc->sel.n_cand = sc->counters + 4;
    sc->qpos = (QuantPos*)(sc->counters + 5);
    sc->stat = (double*)(sc->counters + 7);
    p += up(kCounterBytes);
    sc->small = p;
    return true;
}

// Clears the histograms and the counters: a selection leaves its histograms
// at zero, but a run that failed half way may not have.
hipError_t clear_scratch(const Scratch& sc, hipStream_t st) {
    hipError_t e = hipMemsetAsync(sc.sel.hists, 0, kHistBytes, st);
    if (e != hipSuccess) return e;
    return hipMemsetAsync(sc.counters, 0, kCounterBytes, st);
}

// keys: four 32-bit arrays (the coordinates and the scales), the 64-bit
// distances over the first two once their medians are taken
size_t grid_statistics_scratch(int64_t n) { return up((size_t)n * 16) + fixed_bytes(sizeof(GridStatsResult)); }

// the anchor indices and values, padding, and the band parameters
size_t refine_small_bytes(int32_t n_prompts) { return (size_t)(n_prompts + 1) * 12 + 8 + 5 * 8; }

size_t refine_mask_scratch(int64_t pixels, int32_t n_prompts) {
    return up((size_t)pixels * 4) + fixed_bytes(refine_small_bytes(n_prompts));
}

hipError_t grid_statistics(const float* xyz, const float* scale, int64_t n, const GridStatsParams& p,
                           GridStatsResult* out, void* scratch, size_t scratch_bytes, hipStream_t st) {
    Scratch sc;
    hipError_t e;
    if (!carve(scratch, scratch_bytes, (size_t)n * 16, sizeof(GridStatsResult), &sc)) return hipErrorInvalidValue;
    if ((e = clear_scratch(sc, st)) != hipSuccess) return e;
    GridStatsResult* g = (GridStatsResult*)sc.small;  // the statistics, on the device
    if ((e = hipMemcpyAsync(g, out, sizeof *g, hipMemcpyHostToDevice, st)) != hipSuccess) return e;
    uint32_t* k32 = (uint32_t*)sc.keys;
    uint64_t* k64 = (uint64_t*)sc.keys;
    const unsigned gb = blocks_of(n, 256);
    const unsigned cb = std::min(blocks_of(n, kCountThreads), kCountBlocks);
    const unsigned long long* m = sc.counters;  // points that take part, counted with the first axis

    // medians of the three coordinates (and of the scales)
    // four points per step of a lane where the buffers allow 16-byte accesses
    const bool quad = ((uintptr_t)xyz & 15u) == 0 && ((uintptr_t)scale & 15u) == 0 && n % 4 == 0;
    if (quad)
        hipLaunchKernelGGL(k_keys_points<true>, dim3(std::min(blocks_of(n / 4, kCountThreads), kCountBlocks)),
                           dim3(kCountThreads), 0, st, xyz, scale, n, k32, sc.counters);
    else
        hipLaunchKernelGGL(k_keys_points<false>, dim3(cb), dim3(kCountThreads), 0, st, xyz, scale, n, k32,
                           sc.counters);
    auto median_of = [&](int axis, double* med) {
        hipLaunchKernelGGL(k_ranks_median, dim3(1), dim3(1), 0, st, m, sc.sel.slots);
        enqueue_select<uint32_t>(k32 + axis * n, n, sc.sel, st);
        hipLaunchKernelGGL(k_take_median<kKeyF32>, dim3(1), dim3(64), 0, st, m, sc.sel, med);
    };
    for (int a = 0; a < 3; ++a) median_of(a, &g->center[a]);

    // 99th percentile of the distances, linear between order statistics (the
    // distance keys overwrite the keys of the first two coordinates)
    if (quad)
        hipLaunchKernelGGL(k_keys_distance<true>, dim3(blocks_of(n / 4, 256)), dim3(256), 0, st, xyz, scale, n,
                           g->center, k64);
    else
        hipLaunchKernelGGL(k_keys_distance<false>, dim3(gb), dim3(256), 0, st, xyz, scale, n, g->center, k64);
    // candidates over the third coordinate's keys, whose median is taken
    sc.sel.cand = (char*)sc.keys + (size_t)n * 8;
    sc.sel.cand_cap = n / 2;
    hipLaunchKernelGGL(k_ranks_quantile, dim3(1), dim3(1), 0, st, m, p.q, sc.sel.slots, sc.qpos);
    enqueue_select<uint64_t>(k64, n, sc.sel, st);
    hipLaunchKernelGGL(k_take_quantile<kKeyF64Bits>, dim3(1), dim3(64), 0, st, m, sc.sel, sc.qpos, &g->r_fg);
    sc.sel.cand = nullptr;
    sc.sel.cand_cap = 0;

    if (scale) median_of(3, &g->s_med);

    // Eq. scene-norm / Eq. voxel-size, and the points inside the grid
    hipLaunchKernelGGL(k_grid_finish, dim3(1), dim3(1), 0, st, m, p, scale ? 1 : 0, g);
    if (quad)
        hipLaunchKernelGGL(k_count_kept<true>, dim3(std::min(blocks_of(n / 4, kCountThreads), kCountBlocks)),
                           dim3(kCountThreads), 0, st, xyz, n, g, sc.counters + 2);
    else
        hipLaunchKernelGGL(k_count_kept<false>, dim3(cb), dim3(kCountThreads), 0, st, xyz, n, g, sc.counters + 2);
    unsigned long long kept = 0;
    if ((e = hipMemcpyAsync(out, g, sizeof *out, hipMemcpyDeviceToHost, st)) != hipSuccess) return e;
    if ((e = hipMemcpyAsync(&kept, sc.counters + 2, 8, hipMemcpyDeviceToHost, st)) != hipSuccess) return e;
    if ((e = hipStreamSynchronize(st)) != hipSuccess) return e;
    if (out->m > 0 && out->dim > 0) out->n_kept = (int64_t)kept;
    return hipGetLastError();
}

hipError_t refine_mask(int kind, int32_t width, int32_t height, const float* mask, const float* depth,
                       const int32_t* prompts_xy, int32_t n_prompts, float* out, RefineResult* res,
                       void* scratch, size_t scratch_bytes, hipStream_t st) {
    const int64_t n = (int64_t)width * height;
    const unsigned gb = blocks_of(n, 256);
    const unsigned cb = std::min(blocks_of(n, kCountThreads), kCountBlocks);
    Scratch sc;
    hipError_t e;
    *res = RefineResult{};
    res->band_min = res->band_max = res->d_far = res->z_min = res->z_max = NAN;
    if (!carve(scratch, scratch_bytes, kind == kRefineMinMax ? 0 : (size_t)n * 4, refine_small_bytes(n_prompts), &sc))
        return hipErrorInvalidValue;
    if ((e = clear_scratch(sc, st)) != hipSuccess) return e;
    if (kind == kRefineMinMax) {
        unsigned int* ext = (unsigned int*)(sc.counters + 1);  // [min key, max key]
        if ((e = hipMemsetAsync(ext, 0xFF, 4, st)) != hipSuccess) return e;
        hipLaunchKernelGGL(k_depth_extrema, dim3(cb), dim3(kCountThreads), 0, st, depth, n, ext, sc.counters);
        hipLaunchKernelGGL(k_refine_minmax, dim3(gb), dim3(256), 0, st, mask, depth, n, ext, sc.counters, out);
        unsigned long long h[2];
        if ((e = hipMemcpyAsync(h, sc.counters, 16, hipMemcpyDeviceToHost, st)) != hipSuccess) return e;
        if ((e = hipStreamSynchronize(st)) != hipSuccess) return e;
        res->n_surface = (int64_t)h[0];
        if (h[0] == 0) return hipGetLastError();
        const uint32_t kmin = (uint32_t)(h[1] & 0xFFFFFFFFull), kmax = (uint32_t)(h[1] >> 32);
        res->z_min = (double)key_float(kmin);
        res->z_max = (double)key_float(kmax);
        return hipGetLastError();
    }

    // band-pass: surface count and depth keys, the anchors and their band,
    // d_far by selection, the weights; the host reads the statistics at the end
    const int na = n_prompts + 1;
    int64_t* didx = (int64_t*)sc.small;
    float* dval = (float*)(didx + na);
    double* par = (double*)(dval + na + (na & 1));  // 8-byte aligned after the anchor values
    std::vector<int64_t> idx((size_t)na);
    for (int k = 0; k < n_prompts; ++k) idx[k] = (int64_t)prompts_xy[2 * k + 1] * width + prompts_xy[2 * k];
    idx[n_prompts] = (int64_t)(height / 2) * width + width / 2;
    uint32_t* k32 = (uint32_t*)sc.keys;
    const unsigned long long* m = sc.counters;
    hipLaunchKernelGGL(k_keys_depth, dim3(cb), dim3(kCountThreads), 0, st, depth, n, k32, sc.counters);
    if ((e = hipMemcpyAsync(didx, idx.data(), (size_t)na * 8, hipMemcpyHostToDevice, st)) != hipSuccess) return e;
    hipLaunchKernelGGL(k_gather_depth, dim3(blocks_of(na, 64)), dim3(64), 0, st, depth, didx, na, dval);
    hipLaunchKernelGGL(k_band_anchors, dim3(1), dim3(1), 0, st, m, dval, na, par);
    hipLaunchKernelGGL(k_ranks_quantile, dim3(1), dim3(1), 0, st, m, kFarQuantile, sc.sel.slots, sc.qpos);
    enqueue_select<uint32_t>(k32, n, sc.sel, st);
    hipLaunchKernelGGL(k_take_quantile<kKeyF32>, dim3(1), dim3(64), 0, st, m, sc.sel, sc.qpos, par + 2);
    hipLaunchKernelGGL(k_refine_band, dim3(gb), dim3(256), 0, st, mask, depth, n, par, out);
    double hp[5];
    unsigned long long surf = 0;
    if ((e = hipMemcpyAsync(hp, par, sizeof hp, hipMemcpyDeviceToHost, st)) != hipSuccess) return e;
    if ((e = hipMemcpyAsync(&surf, m, 8, hipMemcpyDeviceToHost, st)) != hipSuccess) return e;
    if ((e = hipStreamSynchronize(st)) != hipSuccess) return e;
    res->n_surface = (int64_t)surf;
    res->n_anchors = (int32_t)hp[3];
    if (res->n_anchors > 0) {
        res->band_min = hp[0];
        res->band_max = hp[1];
    }
    if (hp[4] != 0.0) res->d_far = hp[2];
    return hipGetLastError();
}

// the aspect keys, the fixed part, and (with_candidates) room for n / 2
// gathered candidates; without that room the selection reads all keys in
// every pass
size_t needle_cull_scratch(int64_t n, bool with_candidates) {
    return up((size_t)n * 8) + fixed_bytes(0) + (with_candidates ? up((size_t)(n / 2) * 8) : 0);
}

hipError_t needle_cull(const float* scales, int64_t n, double eps, double q, uint8_t* labels, NeedleResult* res,
                       void* scratch, size_t scratch_bytes, hipStream_t st) {
    Scratch sc;
    hipError_t e;
    *res = NeedleResult{};
    res->tau = NAN;
    if (!carve(scratch, scratch_bytes, (size_t)n * 8, 0, &sc)) return hipErrorInvalidValue;
    if ((e = clear_scratch(sc, st)) != hipSuccess) return e;
    // candidates in what the scratch holds past the fixed part (none when it
    // holds nothing more: then every pass reads all keys)
    const size_t used = up((size_t)n * 8) + fixed_bytes(0);
    sc.sel.cand = (char*)scratch + used;
    sc.sel.cand_cap = std::min<int64_t>((int64_t)((scratch_bytes - used) / 8), n);
    const unsigned cb = std::min(blocks_of(n, kCountThreads), kCountBlocks);
    uint64_t* k64 = (uint64_t*)sc.keys;
    const unsigned long long* m = sc.counters;
    // the aspects' keys, tau by selection, the cull; the host reads the counts
    // and tau at the end
    hipLaunchKernelGGL(k_keys_aspect, dim3(cb), dim3(kCountThreads), 0, st, scales, n, eps, k64, sc.counters);
    hipLaunchKernelGGL(k_ranks_quantile, dim3(1), dim3(1), 0, st, m, q, sc.sel.slots, sc.qpos);
    enqueue_select<uint64_t>(k64, n, sc.sel, st);
    hipLaunchKernelGGL(k_take_quantile<kKeyF64>, dim3(1), dim3(64), 0, st, m, sc.sel, sc.qpos, sc.stat);
    hipLaunchKernelGGL(k_needle_apply, dim3(cb), dim3(kCountThreads), 0, st, scales, n, eps, m, sc.stat, labels,
                       sc.counters + 1);
    unsigned long long c[8];
    if ((e = hipMemcpyAsync(c, sc.counters, sizeof c, hipMemcpyDeviceToHost, st)) != hipSuccess) return e;
    if ((e = hipStreamSynchronize(st)) != hipSuccess) return e;
    res->m = (int64_t)c[0];
    if (c[0] == 0) return hipGetLastError();
    res->tau = as_double(c[7]);
    res->n_culled = (int64_t)c[1];
    return hipGetLastError();
}

// ---- fixed device scratch of the allocation-free needle cull
//
// One array per device, held until the process ends.  Host code never passes
// the array's name to a kernel or a copy: in host code that name is a
// host-side stand-in, not a device address.  The device address is looked up
// once per device with hipGetSymbolAddress (with that device current) and
// kept in g_static_scratch.
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_static_mu;
void* g_static_scratch[kMaxDevices] = {};
}  // namespace

hipError_t static_scratch_init(int device, void** out) {
    *out = nullptr;
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_static_mu);
    if (!g_static_scratch[device]) {
        void* ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!ptr) return hipErrorInvalidSymbol;
        g_static_scratch[device] = ptr;
    }
    *out = g_static_scratch[device];
    return hipSuccess;
}

}  // namespace divas
