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
//  * The footprint statistics of n_samp (Sec. 3.5, App. F) need no pre-pass
//    here: the fusion sums the counts of a voxel's few footprint pixels
//    directly, where the paper builds integral images of every pixel.
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

}  // namespace divas
