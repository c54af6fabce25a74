// Per-view pre-pass of the fusion.
//
//  * Hot tiles: for every kTile x kTile pixel tile, a flag "some pixel has
//    mask >= mask_gate".  A voxel can only vote in a view through a pixel that
//    passes the thick-path entry gate of Alg. gs-fusion, so a chunk of voxels
//    whose projection touches no hot tile cannot vote in that view; the culling
//    kernel uses the flags to skip such (chunk, view) pairs exactly.  One fully
//    parallel pass over the mask planes (one lane per tile row segment of 8
//    pixels) packs the flags of 64 tiles of a tile row into a word.  The same
//    pass writes the gate bitmask, one bit per pixel: the fusion tests a
//    sample's bit (an L2-resident byte) before it reads any float map.
//  * Integral images of n_samp and n_samp^2 ("Footprint statistics via
//    integral images", Sec. 3.5 and App. F), (W+1) x (H+1) uint64 with a zero
//    first row and column, when the view carries n_samp.
#include "fuse_core.h"

#include <algorithm>

namespace divas {

namespace {

// Hot-tile flags: block (word, tile row, view) of 8 waves; wave r reads pixel
// row 8 ty + r, each lane the 8 pixels of one tile (two 16-byte loads when
// aligned) and writes their byte of the gate bitmask, so a block covers the 64
// tiles of one hot-tile word and the pass reads every mask plane once with
// coalesced loads.  Block (0, 0, 0) also zeroes the fusion counters.
constexpr int kFlagThreads = kTile * 64;
__global__ __launch_bounds__(kFlagThreads) void k_tile_flags(const DView* __restrict__ views, int32_t s_begin,
                                                             double gate, int64_t* __restrict__ counters,
                                                             int n_counters) {
    if (blockIdx.x == 0 && blockIdx.y == 0 && blockIdx.z == 0 && counters && (int)threadIdx.x < n_counters)
        counters[threadIdx.x] = 0;
    const DView& v = views[s_begin + blockIdx.z];
    const int ty = blockIdx.y;
    const int tx0 = blockIdx.x * 64;
    if (ty >= v.th || tx0 >= v.tw) return;  // uniform per block
    __shared__ uint32_t tf[64];
    const int lane = threadIdx.x & 63;
    if (threadIdx.x < 64) tf[threadIdx.x] = 0u;
    __syncthreads();
    const int y = ty * kTile + (int)(threadIdx.x >> 6);
    const int x = (tx0 + lane) * kTile;
    uint32_t hot = 0;
    if (y < v.H && x < v.W) {
        const float* __restrict__ row = v.mask + (size_t)y * v.W;
        if (x + kTile <= v.W && (((uintptr_t)(row + x)) & 15u) == 0) {
            const float4 q0 = ldg4(row + x), q1 = ldg4(row + x + 4);
            hot = ((double)q0.x >= gate ? 1u : 0u) | ((double)q0.y >= gate ? 2u : 0u) |
                  ((double)q0.z >= gate ? 4u : 0u) | ((double)q0.w >= gate ? 8u : 0u) |
                  ((double)q1.x >= gate ? 16u : 0u) | ((double)q1.y >= gate ? 32u : 0u) |
                  ((double)q1.z >= gate ? 64u : 0u) | ((double)q1.w >= gate ? 128u : 0u);
        } else {
            for (int k = 0; k < kTile && x + k < v.W; ++k) hot |= (double)ldg(row + x + k) >= gate ? 1u << k : 0u;
        }
        v.mbits[(size_t)y * v.mpitch + (size_t)(tx0 + lane)] = (uint8_t)hot;
    }
    if (hot) atomicOr(&tf[lane], 1u);
    __syncthreads();
    if (threadIdx.x < 64) {  // wave 0: tiles past tw hold no pixel, so their flags are 0
        const uint64_t word = __ballot(tf[threadIdx.x] != 0u);
        if (threadIdx.x == 0) v.tile_bits[(size_t)ty * ((v.tw + 63) >> 6) + blockIdx.x] = word;
    }
}

// Row pass of the integral images: block per (row, view); each thread sums a
// contiguous segment, a block scan turns segment sums into offsets.
__global__ void k_sat_rows(const DView* __restrict__ views, int32_t s_begin, uint64_t* __restrict__ sat_base,
                           int64_t sat_stride) {
    const DView& v = views[s_begin + blockIdx.y];
    if (!v.nsamp) return;
    const int W = v.W, H = v.H;
    int y = blockIdx.x;
    if (y > H) return;
    uint64_t* s1 = sat_base + (size_t)(s_begin + blockIdx.y) * sat_stride * 2;
    uint64_t* s2 = s1 + sat_stride;
    const int W1 = W + 1;
    if (y == 0) {
        for (int x = threadIdx.x; x < W1; x += blockDim.x) s1[x] = s2[x] = 0;
        return;
    }
    const uint16_t* row = v.nsamp + (size_t)(y - 1) * W;
    int T = blockDim.x;
    int seg = (W + T - 1) / T;
    int a = threadIdx.x * seg, b = min(a + seg, W);
    uint64_t t1 = 0, t2 = 0;
    for (int x = a; x < b; ++x) {
        uint64_t n = row[x];
        t1 += n;
        t2 += n * n;
    }
    __shared__ uint64_t sh1[256], sh2[256];
    sh1[threadIdx.x] = t1;
    sh2[threadIdx.x] = t2;
    __syncthreads();
    for (int off = 1; off < T; off <<= 1) {
        uint64_t u1 = threadIdx.x >= (unsigned)off ? sh1[threadIdx.x - off] : 0;
        uint64_t u2 = threadIdx.x >= (unsigned)off ? sh2[threadIdx.x - off] : 0;
        __syncthreads();
        sh1[threadIdx.x] += u1;
        sh2[threadIdx.x] += u2;
        __syncthreads();
    }
    uint64_t c1 = sh1[threadIdx.x] - t1, c2 = sh2[threadIdx.x] - t2;
    uint64_t* o1 = s1 + (size_t)y * W1;
    uint64_t* o2 = s2 + (size_t)y * W1;
    if (threadIdx.x == 0) o1[0] = o2[0] = 0;
    for (int x = a; x < b; ++x) {
        uint64_t n = row[x];
        c1 += n;
        c2 += n * n;
        o1[x + 1] = c1;
        o2[x + 1] = c2;
    }
}

// Column pass: thread per (column, view), walking down the rows (coalesced).
__global__ void k_sat_cols(const DView* __restrict__ views, int32_t s_begin, uint64_t* __restrict__ sat_base,
                           int64_t sat_stride) {
    const DView& v = views[s_begin + blockIdx.y];
    if (!v.nsamp) return;
    const int W1 = v.W + 1, H = v.H;
    int x = blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= W1) return;
    uint64_t* s1 = sat_base + (size_t)(s_begin + blockIdx.y) * sat_stride * 2;
    uint64_t* s2 = s1 + sat_stride;
    uint64_t a1 = 0, a2 = 0;
    for (int y = 1; y <= H; ++y) {
        a1 += s1[(size_t)y * W1 + x];
        a2 += s2[(size_t)y * W1 + x];
        s1[(size_t)y * W1 + x] = a1;
        s2[(size_t)y * W1 + x] = a2;
    }
}

}  // namespace

hipError_t launch_view_prepass(const DView* dviews, const DView* hviews, int32_t s_begin, int32_t s_end,
                               double mask_gate, int64_t* counters, int n_counters, hipStream_t st, PhaseEvents ev) {
    int ns = s_end - s_begin;
    if (ns <= 0) {
        record_phase_events(ev, st);
        if (counters && n_counters > 0) return launch_fill_u32((uint32_t*)counters, 0u, 2 * n_counters, st);
        return hipSuccess;
    }
    int max_tw = 0, max_th = 0;
    for (int s = s_begin; s < s_end; ++s) {
        max_tw = std::max(max_tw, hviews[s].tw);
        max_th = std::max(max_th, hviews[s].th);
    }
    launch_timed(k_tile_flags, dim3((unsigned)((max_tw + 63) / 64), (unsigned)max_th, (unsigned)ns),
                 dim3(kFlagThreads), 0, st, ev.start, ev.stop, dviews, s_begin, mask_gate, counters, n_counters);
    return hipGetLastError();
}

hipError_t launch_sat(const DView* dviews, const DView* hviews, int32_t s_begin, int32_t s_end, uint64_t* sat_base,
                      int64_t sat_stride, hipStream_t st, PhaseEvents ev) {
    int ns = s_end - s_begin;
    int max_W1 = 0, max_H = 0;
    bool any = false;
    for (int s = s_begin; s < s_end; ++s) {
        if (!hviews[s].nsamp) continue;
        any = true;
        max_W1 = std::max(max_W1, hviews[s].W + 1);
        max_H = std::max(max_H, hviews[s].H);
    }
    if (!any || ns <= 0) {
        record_phase_events(ev, st);
        return hipSuccess;
    }
    launch_timed(k_sat_rows, dim3((unsigned)(max_H + 1), (unsigned)ns), dim3(256), 0, st, ev.start, nullptr, dviews,
                 s_begin, sat_base, sat_stride);
    launch_timed(k_sat_cols, dim3((unsigned)((max_W1 + 255) / 256), (unsigned)ns), dim3(256), 0, st, nullptr, ev.stop,
                 dviews, s_begin, sat_base, sat_stride);
    return hipGetLastError();
}

}  // namespace divas
