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
// so far (a block histogram in LDS, merged with one atomic per bin), and a
// one-block launch picks the digit that holds the wanted rank.  Two ranks are
// selected together (the two middle elements of an even count, or the two
// neighbours of the percentile position).  The host reads the selected keys
// back after each statistic, since the next one depends on it (distances need
// the centre), and evaluates the closed forms in binary64.
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

float key_float(uint32_t k) {
    const uint32_t u = (k & 0x80000000u) ? (k & 0x7FFFFFFFu) : ~k;
    float f;
    std::memcpy(&f, &u, 4);
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

// keys[i] = key of xyz[i][axis] (axis 0..2) or of scale[i] (axis 3); counts
// the points that take part into *m.
__global__ __launch_bounds__(kCountThreads) void k_keys_value(const float* __restrict__ xyz,
                                                               const float* __restrict__ scale, int64_t n, int axis,
                                                               uint32_t* __restrict__ keys,
                                                               unsigned long long* __restrict__ m) {
    unsigned cnt = 0;
    const int64_t stride = (int64_t)gridDim.x * kCountThreads;
    for (int64_t i = blockIdx.x * (int64_t)kCountThreads + threadIdx.x; i < n; i += stride) {
        const bool part = point_takes_part(xyz, scale, i);
        const float v = axis < 3 ? xyz[3 * i + axis] : scale[i];
        keys[i] = part ? float_key(v) : 0xFFFFFFFFu;
        cnt += part ? 1u : 0u;
    }
    const unsigned t = block_total(cnt);
    if (threadIdx.x == 0 && t) atomicAdd(m, (unsigned long long)t);
}

// keys[i] = bit pattern of the binary64 distance of point i to the centre.
__global__ void k_keys_distance(const float* __restrict__ xyz, const float* __restrict__ scale, int64_t n, double cx,
                                double cy, double cz, uint64_t* __restrict__ keys) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    if (!point_takes_part(xyz, scale, i)) {
        keys[i] = ~0ull;
        return;
    }
    const double dx = (double)xyz[3 * i] - cx;
    const double dy = (double)xyz[3 * i + 1] - cy;
    const double dz = (double)xyz[3 * i + 2] - cz;
    const double d = sqrt((dx * dx + dy * dy) + dz * dz);
    keys[i] = (uint64_t)__double_as_longlong(d);
}

// Selection state: for each target rank, the key digits found so far (the
// top `known` bits of prefix) and the rank left inside them.
struct SelState {
    unsigned long long prefix[kSelTargets];
    unsigned long long rank[kSelTargets];
};

// One pass: histogram of the digit at bit `shift` of the keys whose bits
// above shift + 8 equal the target's prefix.
template <class K>
__global__ __launch_bounds__(kSelThreads) void k_sel_hist(const K* __restrict__ keys, int64_t n, int shift,
                                                          const SelState* __restrict__ st,
                                                          unsigned int* __restrict__ hist) {
    __shared__ unsigned int h[kSelTargets][kSelBins];
    for (int b = threadIdx.x; b < kSelTargets * kSelBins; b += kSelThreads) (&h[0][0])[b] = 0u;
    __syncthreads();
    const int hi = shift + 8;  // bits at and above hi are known
    constexpr int kBits = 8 * (int)sizeof(K);
    K want[kSelTargets];
#pragma unroll
    for (int t = 0; t < kSelTargets; ++t) want[t] = hi < kBits ? (K)(st->prefix[t] >> hi) : (K)0;
    const int64_t stride = (int64_t)gridDim.x * kSelThreads;
    for (int64_t i = blockIdx.x * (int64_t)kSelThreads + threadIdx.x; i < n; i += stride) {
        const K k = keys[i];
        const unsigned d = (unsigned)(k >> shift) & (kSelBins - 1);
        const K top = hi < kBits ? (K)(k >> hi) : (K)0;
#pragma unroll
        for (int t = 0; t < kSelTargets; ++t)
            if (top == want[t]) atomicAdd(&h[t][d], 1u);
    }
    __syncthreads();
    for (int b = threadIdx.x; b < kSelTargets * kSelBins; b += kSelThreads) {
        const unsigned v = (&h[0][0])[b];
        if (v) atomicAdd(hist + b, v);
    }
}

// One block of kSelBins threads: for each target, the digit whose bin holds
// the remaining rank; appends it to the prefix, and clears the histogram.
__global__ __launch_bounds__(kSelBins) void k_sel_pick(int shift, SelState* __restrict__ st,
                                                       unsigned int* __restrict__ hist) {
    __shared__ unsigned int cum[kSelBins];
    const int b = threadIdx.x;
    for (int t = 0; t < kSelTargets; ++t) {
        const unsigned v = hist[t * kSelBins + b];
        cum[b] = v;
        __syncthreads();
        for (int off = 1; off < kSelBins; off <<= 1) {  // inclusive scan
            const unsigned x = b >= off ? cum[b - off] : 0u;
            __syncthreads();
            cum[b] += x;
            __syncthreads();
        }
        const unsigned long long r = st->rank[t];
        const unsigned long long below = (unsigned long long)(cum[b] - v);
        if (v && r >= below && r < below + v) {  // exactly one bin when the rank exists
            st->prefix[t] |= (unsigned long long)b << shift;
            st->rank[t] = r - below;
        }
        __syncthreads();
        hist[t * kSelBins + b] = 0u;
        __syncthreads();
    }
}

// Points inside the grid by the voxel rule.
__global__ __launch_bounds__(kCountThreads) void k_count_kept(const float* __restrict__ xyz, int64_t n, double ox,
                                                               double oy, double oz, double h, double inv_h,
                                                               int32_t dim, unsigned long long* __restrict__ kept) {
    const double o[3] = {ox, oy, oz};
    unsigned cnt = 0;
    const int64_t stride = (int64_t)gridDim.x * kCountThreads;
    for (int64_t i = blockIdx.x * (int64_t)kCountThreads + threadIdx.x; i < n; i += stride) {
        bool in = true;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const double f = voxel_floor((double)xyz[3 * i + k] - o[k], h, inv_h);
            in = in && (f >= 0.0) && (f < (double)dim);  // NaN fails
        }
        cnt += in ? 1u : 0u;
    }
    const unsigned t = block_total(cnt);
    if (threadIdx.x == 0 && t) atomicAdd(kept, (unsigned long long)t);
}

unsigned blocks_of(int64_t n, int t) { return (unsigned)((n + t - 1) / t); }

// Selects the keys of ranks r[0], r[1] (0-based, < n) of keys[0, n).
template <class K>
hipError_t select2(const K* keys, int64_t n, const unsigned long long r[2], SelState* dst, unsigned int* dhist,
                   unsigned long long out[2], hipStream_t st) {
    SelState s0{};
    s0.rank[0] = r[0];
    s0.rank[1] = r[1];
    hipError_t e = hipMemcpyAsync(dst, &s0, sizeof s0, hipMemcpyHostToDevice, st);
    if (e != hipSuccess) return e;
    // a bounded grid: each block adds its nonzero bins to the shared histogram
    const unsigned grid = std::min<unsigned>(blocks_of(n, kSelThreads * 8), 256u);
    for (int shift = 8 * (int)sizeof(K) - 8; shift >= 0; shift -= 8) {
        hipLaunchKernelGGL(k_sel_hist<K>, dim3(grid), dim3(kSelThreads), 0, st, keys, n, shift, dst, dhist);
        hipLaunchKernelGGL(k_sel_pick, dim3(1), dim3(kSelBins), 0, st, shift, dst, dhist);
    }
    SelState s1{};
    if ((e = hipMemcpyAsync(&s1, dst, sizeof s1, hipMemcpyDeviceToHost, st)) != hipSuccess) return e;
    if ((e = hipStreamSynchronize(st)) != hipSuccess) return e;
    out[0] = s1.prefix[0];
    out[1] = s1.prefix[1];
    return hipGetLastError();
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

// Eq. pass-needle: labels[i] &= (aspect <= tau); counts the culled surfels.
__global__ __launch_bounds__(kCountThreads) void k_needle_apply(const float* __restrict__ scales, int64_t n,
                                                                 double eps, double tau, uint8_t* __restrict__ labels,
                                                                 unsigned long long* __restrict__ culled) {
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

// Eq. gs-bandpass per pixel.
__global__ void k_refine_band(const float* mask, const float* __restrict__ d, int64_t n, double lo, double hi,
                              double den, float* out) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
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

// Eq. nerf-depthweight per pixel (flat: every surface pixel keeps weight 1).
__global__ void k_refine_minmax(const float* mask, const float* __restrict__ d, int64_t n, double zmin, double zmax,
                                float* out) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float df = d[i];
    double z = 1.0;
    if (has_surface(df)) z = zmax > zmin ? ((double)df - zmin) / (zmax - zmin) : 0.0;
    out[i] = (float)((double)mask[i] * (1.0 - z));
}

}  // namespace

// The buffers of one run, carved from the caller's scratch (256-byte aligned
// pieces): the keys, the selection state and histogram, four counters and the
// anchor tables.
struct Scratch {
    void* keys = nullptr;
    SelState* state = nullptr;
    unsigned int* hist = nullptr;
    unsigned long long* counters = nullptr;
    void* small = nullptr;
};
constexpr size_t kAlign = 256;
size_t up(size_t b) { return (b + kAlign - 1) / kAlign * kAlign; }
size_t fixed_bytes(size_t small) {
    return up(sizeof(SelState)) + up(sizeof(unsigned) * kSelTargets * kSelBins) + up(8 * 4) + up(small);
}
bool carve(void* base, size_t bytes, size_t key_bytes, size_t small, Scratch* sc) {
    if (bytes < up(key_bytes) + fixed_bytes(small)) return false;
    char* p = (char*)base;
    sc->keys = p;
    p += up(key_bytes);
    sc->state = (SelState*)p;
    p += up(sizeof(SelState));
    sc->hist = (unsigned int*)p;
    p += up(sizeof(unsigned) * kSelTargets * kSelBins);
    sc->counters = (unsigned long long*)p;
    p += up(8 * 4);
    sc->small = p;
    return true;
}

size_t grid_statistics_scratch(int64_t n) { return up((size_t)n * 8) + fixed_bytes(0); }

size_t refine_mask_scratch(int64_t pixels, int32_t n_prompts) {
    return up((size_t)pixels * 4) + fixed_bytes((size_t)(n_prompts + 1) * 12 + 16);
}

hipError_t grid_statistics(const float* xyz, const float* scale, int64_t n, const GridStatsParams& p,
                           GridStatsResult* out, void* scratch, size_t scratch_bytes, hipStream_t st) {
    Scratch sc;
    hipError_t e;
    if (!carve(scratch, scratch_bytes, (size_t)n * 8, 0, &sc)) return hipErrorInvalidValue;
    if ((e = hipMemsetAsync(sc.hist, 0, sizeof(unsigned) * kSelTargets * kSelBins, st)) != hipSuccess) return e;
    if ((e = hipMemsetAsync(sc.counters, 0, 8 * 4, st)) != hipSuccess) return e;
    uint32_t* k32 = (uint32_t*)sc.keys;
    uint64_t* k64 = (uint64_t*)sc.keys;
    const unsigned gb = blocks_of(n, 256);
    const unsigned cb = std::min(blocks_of(n, kCountThreads), kCountBlocks);

    // medians of the three coordinates (and of the scales)
    unsigned long long m = 0;
    auto median_of = [&](int axis, double* med) -> hipError_t {
        hipLaunchKernelGGL(k_keys_value, dim3(cb), dim3(kCountThreads), 0, st, xyz, scale, n, axis, k32,
                           sc.counters + (axis == 0 ? 0 : 1));
        if (axis == 0) {
            hipError_t e2 = hipMemcpyAsync(&m, sc.counters, 8, hipMemcpyDeviceToHost, st);
            if (e2 != hipSuccess) return e2;
            if ((e2 = hipStreamSynchronize(st)) != hipSuccess) return e2;
            if (m == 0) return hipSuccess;
        }
        const unsigned long long r[2] = {(m - 1) / 2, m / 2};  // equal when m is odd
        unsigned long long kk[2];
        hipError_t e2 = select2<uint32_t>(k32, n, r, sc.state, sc.hist, kk, st);
        if (e2 != hipSuccess) return e2;
        const double lo = (double)key_float((uint32_t)kk[0]), hi = (double)key_float((uint32_t)kk[1]);
        *med = (m % 2) ? lo : (lo + hi) / 2.0;
        return hipSuccess;
    };
    for (int a = 0; a < 3; ++a) {
        if ((e = median_of(a, &out->center[a])) != hipSuccess) return e;
        if (m == 0) {
            out->m = 0;
            return hipSuccess;
        }
    }
    out->m = (int64_t)m;

    // 99th percentile of the distances, linear between order statistics
    hipLaunchKernelGGL(k_keys_distance, dim3(gb), dim3(256), 0, st, xyz, scale, n, out->center[0], out->center[1],
                       out->center[2], k64);
    {
        const double pos = p.q * (double)(m - 1);
        const double fi = std::floor(pos);
        const unsigned long long i = (unsigned long long)fi;
        const double f = pos - fi;
        const unsigned long long r[2] = {i, i + 1 < m ? i + 1 : i};
        unsigned long long kk[2];
        if ((e = select2<uint64_t>(k64, n, r, sc.state, sc.hist, kk, st)) != hipSuccess) return e;
        const double lo = as_double(kk[0]), hi = as_double(kk[1]);
        out->r_fg = i + 1 < m ? lo + (hi - lo) * f : lo;
    }

    out->s_med = NAN;
    if (scale)
        if ((e = median_of(3, &out->s_med)) != hipSuccess) return e;

    // Eq. scene-norm / Eq. voxel-size
    out->b = std::ceil(p.pad * out->r_fg);
    double h_v = p.beta_v * out->r_fg / (double)p.g0;
    if (scale) h_v = std::max(p.alpha_v * out->s_med, h_v);
    out->h_v = h_v;
    if (!(out->b > 0.0) || !(h_v > 0.0)) {
        out->dim = 0;
        return hipSuccess;
    }
    const double need = 2.0 * out->b / h_v;
    int32_t g = 2;
    while (g < need && g < p.g_max) g *= 2;
    out->dim = std::min(g, p.g_max);
    for (int a = 0; a < 3; ++a) out->origin[a] = out->center[a] - out->b;
    out->voxel = 2.0 * out->b / (double)out->dim;

    hipLaunchKernelGGL(k_count_kept, dim3(cb), dim3(kCountThreads), 0, st, xyz, n, out->origin[0], out->origin[1],
                       out->origin[2], out->voxel, 1.0 / out->voxel, out->dim, sc.counters + 2);
    unsigned long long kept = 0;
    if ((e = hipMemcpyAsync(&kept, sc.counters + 2, 8, hipMemcpyDeviceToHost, st)) != hipSuccess) return e;
    if ((e = hipStreamSynchronize(st)) != hipSuccess) return e;
    out->n_kept = (int64_t)kept;
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
    if (!carve(scratch, scratch_bytes, kind == kRefineMinMax ? 0 : (size_t)n * 4, (size_t)(n_prompts + 1) * 12 + 16,
               &sc))
        return hipErrorInvalidValue;
    if ((e = hipMemsetAsync(sc.counters, 0, 8 * 4, st)) != hipSuccess) return e;
    if (kind == kRefineMinMax) {
        unsigned int* ext = (unsigned int*)(sc.counters + 1);  // [min key, max key]
        if ((e = hipMemsetAsync(ext, 0xFF, 4, st)) != hipSuccess) return e;
        hipLaunchKernelGGL(k_depth_extrema, dim3(cb), dim3(kCountThreads), 0, st, depth, n, ext, sc.counters);
        unsigned long long h[2];
        if ((e = hipMemcpyAsync(h, sc.counters, 16, hipMemcpyDeviceToHost, st)) != hipSuccess) return e;
        if ((e = hipStreamSynchronize(st)) != hipSuccess) return e;
        res->n_surface = (int64_t)h[0];
        if (h[0] == 0) return hipSuccess;
        const uint32_t kmin = (uint32_t)(h[1] & 0xFFFFFFFFull), kmax = (uint32_t)(h[1] >> 32);
        res->z_min = (double)key_float(kmin);
        res->z_max = (double)key_float(kmax);
        hipLaunchKernelGGL(k_refine_minmax, dim3(gb), dim3(256), 0, st, mask, depth, n, res->z_min, res->z_max, out);
        if ((e = hipStreamSynchronize(st)) != hipSuccess) return e;
        return hipGetLastError();
    }

    // band-pass: surface count and depth keys, then the anchors
    if ((e = hipMemsetAsync(sc.hist, 0, sizeof(unsigned) * kSelTargets * kSelBins, st)) != hipSuccess) return e;
    const int na = n_prompts + 1;
    int64_t* didx = (int64_t*)sc.small;
    float* dval = (float*)(didx + na);
    std::vector<int64_t> idx((size_t)na);
    for (int k = 0; k < n_prompts; ++k) idx[k] = (int64_t)prompts_xy[2 * k + 1] * width + prompts_xy[2 * k];
    idx[n_prompts] = (int64_t)(height / 2) * width + width / 2;
    uint32_t* k32 = (uint32_t*)sc.keys;
    hipLaunchKernelGGL(k_keys_depth, dim3(cb), dim3(kCountThreads), 0, st, depth, n, k32, sc.counters);
    if ((e = hipMemcpyAsync(didx, idx.data(), (size_t)na * 8, hipMemcpyHostToDevice, st)) != hipSuccess) return e;
    hipLaunchKernelGGL(k_gather_depth, dim3(blocks_of(na, 64)), dim3(64), 0, st, depth, didx, na, dval);
    std::vector<float> av((size_t)na);
    unsigned long long m = 0;
    if ((e = hipMemcpyAsync(av.data(), dval, (size_t)na * 4, hipMemcpyDeviceToHost, st)) != hipSuccess) return e;
    if ((e = hipMemcpyAsync(&m, sc.counters, 8, hipMemcpyDeviceToHost, st)) != hipSuccess) return e;
    if ((e = hipStreamSynchronize(st)) != hipSuccess) return e;
    res->n_surface = (int64_t)m;
    for (float v : av) {
        if (!(std::isfinite(v) && v > 0.0f)) continue;
        const double d = (double)v;
        if (res->n_anchors == 0 || d < res->band_min) res->band_min = d;
        if (res->n_anchors == 0 || d > res->band_max) res->band_max = d;
        ++res->n_anchors;
    }
    if (m == 0 || res->n_anchors == 0) return hipSuccess;

    // d_far: 98th percentile of the surface depths, linear between order statistics
    const double pos = kFarQuantile * (double)(m - 1);
    const double fi = std::floor(pos);
    const unsigned long long i = (unsigned long long)fi;
    const double f = pos - fi;
    const unsigned long long r[2] = {i, i + 1 < m ? i + 1 : i};
    unsigned long long kk[2];
    if ((e = select2<uint32_t>(k32, n, r, sc.state, sc.hist, kk, st)) != hipSuccess) return e;
    const double lo = (double)key_float((uint32_t)kk[0]), hi = (double)key_float((uint32_t)kk[1]);
    res->d_far = i + 1 < m ? lo + (hi - lo) * f : lo;
    const double den = std::max(res->d_far - res->band_max, 1e-6);
    hipLaunchKernelGGL(k_refine_band, dim3(gb), dim3(256), 0, st, mask, depth, n, res->band_min, res->band_max, den,
                       out);
    if ((e = hipStreamSynchronize(st)) != hipSuccess) return e;
    return hipGetLastError();
}

size_t needle_cull_scratch(int64_t n) { return up((size_t)n * 8) + fixed_bytes(0); }

static double key_double(unsigned long long k) {
    const unsigned long long u = (k & 0x8000000000000000ull) ? (k & 0x7FFFFFFFFFFFFFFFull) : ~k;
    return as_double(u);
}

hipError_t needle_cull(const float* scales, int64_t n, double eps, double q, uint8_t* labels, NeedleResult* res,
                       void* scratch, size_t scratch_bytes, hipStream_t st) {
    Scratch sc;
    hipError_t e;
    *res = NeedleResult{};
    res->tau = NAN;
    if (!carve(scratch, scratch_bytes, (size_t)n * 8, 0, &sc)) return hipErrorInvalidValue;
    if ((e = hipMemsetAsync(sc.hist, 0, sizeof(unsigned) * kSelTargets * kSelBins, st)) != hipSuccess) return e;
    if ((e = hipMemsetAsync(sc.counters, 0, 8 * 4, st)) != hipSuccess) return e;
    const unsigned cb = std::min(blocks_of(n, kCountThreads), kCountBlocks);
    uint64_t* k64 = (uint64_t*)sc.keys;
    hipLaunchKernelGGL(k_keys_aspect, dim3(cb), dim3(kCountThreads), 0, st, scales, n, eps, k64, sc.counters);
    unsigned long long m = 0;
    if ((e = hipMemcpyAsync(&m, sc.counters, 8, hipMemcpyDeviceToHost, st)) != hipSuccess) return e;
    if ((e = hipStreamSynchronize(st)) != hipSuccess) return e;
    res->m = (int64_t)m;
    if (m == 0) return hipSuccess;
    const double pos = q * (double)(m - 1);
    const double fi = std::floor(pos);
    const unsigned long long i = (unsigned long long)fi;
    const double f = pos - fi;
    const unsigned long long r[2] = {i, i + 1 < m ? i + 1 : i};
    unsigned long long kk[2];
    if ((e = select2<uint64_t>(k64, n, r, sc.state, sc.hist, kk, st)) != hipSuccess) return e;
    const double lo = key_double(kk[0]), hi = key_double(kk[1]);
    res->tau = i + 1 < m ? lo + (hi - lo) * f : lo;
    hipLaunchKernelGGL(k_needle_apply, dim3(cb), dim3(kCountThreads), 0, st, scales, n, eps, res->tau, labels,
                       sc.counters + 1);
    unsigned long long cut = 0;
    if ((e = hipMemcpyAsync(&cut, sc.counters + 1, 8, hipMemcpyDeviceToHost, st)) != hipSuccess) return e;
    if ((e = hipStreamSynchronize(st)) != hipSuccess) return e;
    res->n_culled = (int64_t)cut;
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
