// Scene-statistic grid construction: Sec. 3.5 (i), Eq. scene-norm and
// Eq. voxel-size.
//
// The statistics are order statistics of the points: the coordinate-wise
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
#include <algorithm>
#include <cmath>
#include <cstring>

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

__device__ __forceinline__ bool point_takes_part(const float* __restrict__ xyz, const float* __restrict__ scale,
                                                 int64_t i) {
    bool ok = isfinite(xyz[3 * i]) && isfinite(xyz[3 * i + 1]) && isfinite(xyz[3 * i + 2]);
    if (scale) ok = ok && isfinite(scale[i]);
    return ok;
}

// keys[i] = key of xyz[i][axis] (axis 0..2) or of scale[i] (axis 3); counts
// the points that take part into *m.
__global__ void k_keys_value(const float* __restrict__ xyz, const float* __restrict__ scale, int64_t n, int axis,
                             uint32_t* __restrict__ keys, unsigned long long* __restrict__ m) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    bool part = false;
    if (i < n) {
        part = point_takes_part(xyz, scale, i);
        const float v = axis < 3 ? xyz[3 * i + axis] : scale[i];
        keys[i] = part ? float_key(v) : 0xFFFFFFFFu;
    }
    const uint64_t c = (uint64_t)__popcll(__ballot(part));
    if ((threadIdx.x & 63) == 0 && c) atomicAdd(m, (unsigned long long)c);
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
__global__ void k_count_kept(const float* __restrict__ xyz, int64_t n, double ox, double oy, double oz, double h,
                             double inv_h, int32_t dim, unsigned long long* __restrict__ kept) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    bool in = false;
    if (i < n) {
        const double o[3] = {ox, oy, oz};
        in = true;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const double f = voxel_floor((double)xyz[3 * i + k] - o[k], h, inv_h);
            in = in && (f >= 0.0) && (f < (double)dim);  // NaN fails
        }
    }
    const uint64_t c = (uint64_t)__popcll(__ballot(in));
    if ((threadIdx.x & 63) == 0 && c) atomicAdd(kept, (unsigned long long)c);
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
    const unsigned grid = std::min<unsigned>(blocks_of(n, kSelThreads * 8), 2048u);
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

}  // namespace

// Device buffers of one run, freed on every exit.
struct GridScratch {
    void* keys = nullptr;
    SelState* state = nullptr;
    unsigned int* hist = nullptr;
    unsigned long long* counters = nullptr;
    ~GridScratch() {
        if (keys) (void)hipFree(keys);
        if (state) (void)hipFree(state);
        if (hist) (void)hipFree(hist);
        if (counters) (void)hipFree(counters);
    }
};

hipError_t grid_statistics(const float* xyz, const float* scale, int64_t n, const GridStatsParams& p,
                           GridStatsResult* out, hipStream_t st) {
    GridScratch sc;
    hipError_t e;
    if ((e = hipMalloc(&sc.keys, (size_t)n * 8)) != hipSuccess) return e;
    if ((e = hipMalloc((void**)&sc.state, sizeof(SelState))) != hipSuccess) return e;
    if ((e = hipMalloc((void**)&sc.hist, sizeof(unsigned) * kSelTargets * kSelBins)) != hipSuccess) return e;
    if ((e = hipMalloc((void**)&sc.counters, 8 * 4)) != hipSuccess) return e;
    if ((e = hipMemsetAsync(sc.hist, 0, sizeof(unsigned) * kSelTargets * kSelBins, st)) != hipSuccess) return e;
    if ((e = hipMemsetAsync(sc.counters, 0, 8 * 4, st)) != hipSuccess) return e;
    uint32_t* k32 = (uint32_t*)sc.keys;
    uint64_t* k64 = (uint64_t*)sc.keys;
    const unsigned gb = blocks_of(n, 256);

    // medians of the three coordinates (and of the scales)
    unsigned long long m = 0;
    auto median_of = [&](int axis, double* med) -> hipError_t {
        hipLaunchKernelGGL(k_keys_value, dim3(gb), dim3(256), 0, st, xyz, scale, n, axis, k32,
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

    hipLaunchKernelGGL(k_count_kept, dim3(gb), dim3(256), 0, st, xyz, n, out->origin[0], out->origin[1],
                       out->origin[2], out->voxel, 1.0 / out->voxel, out->dim, sc.counters + 2);
    unsigned long long kept = 0;
    if ((e = hipMemcpyAsync(&kept, sc.counters + 2, 8, hipMemcpyDeviceToHost, st)) != hipSuccess) return e;
    if ((e = hipStreamSynchronize(st)) != hipSuccess) return e;
    out->n_kept = (int64_t)kept;
    return hipGetLastError();
}

}  // namespace divas
