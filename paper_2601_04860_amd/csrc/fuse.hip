// Thick-path depth-weighted voxel fusion on CDNA4 (gfx950).
//
// Alg. gs-fusion (thick branch; the thin-structure call is not part of this
// path) with Eqs. planar-to-ray, seethrough, asym-gate, tightening,
// gs-spatial, gs-depthweight and vmask, followed by Eq. compact-fusion and the
// consensus threshold.
//
// Layout and schedule
//   * One wavefront owns a chunk of 64 consecutive entries of the Morton-ordered
//     active list (a compact 3D cluster).  Each lane owns one voxel and walks the
//     views in increasing order, accumulating W and Z in binary64 registers, so
//     the result is deterministic and independent of the launch shape (no float
//     atomics anywhere).
//   * A culling kernel first decides, per (chunk, view), whether any voxel of
//     the chunk can vote: the chunk's voxel-centre bounding box is projected
//     conservatively and tested against the view's hot-tile flags (tiles that
//     hold a pixel passing the mask gate).  Skipped pairs cost the fusion kernel
//     one scalar byte load; the per-lane evaluation runs only where a vote is
//     possible.
//   * The per-lane evaluation is the exact fp64 sequence of the arithmetic
//     convention (same operation order as the reference; compiled without FMA
//     contraction), so pixel choices and gate decisions are reproducible.
//   * View records are read through uniform (scalar) loads; maps are gathered at
//     the projected pixel; the compact-fusion rule, the threshold, the
//     segmentation bitfield update and the counts are fused into the same pass.
//   * Blocks are remapped so that each XCD receives a contiguous range of chunks
//     (spatially coherent view reads stay in that XCD's L2).
#include "fuse_core.h"

#include <algorithm>

namespace divas {

namespace {

constexpr int kWaves = kBlock / 64;

// ------------------------------------------------------------ culling
__global__ void k_cull(const uint16_t* __restrict__ box, const int64_t* __restrict__ n_act, DGrid g, double eps,
                       const DView* __restrict__ views, int32_t s_begin, int32_t ns, int32_t p2,
                       uint64_t* __restrict__ cull, int64_t lanes, uint64_t fuse_range, uint64_t* __restrict__ hot_list,
                       uint32_t* __restrict__ hot_count) {
    int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    cull_group(box, *n_act, g, eps, views, s_begin, ns, p2, t, cull, t < lanes, fuse_range, 0ull, hot_list,
               hot_count);
}

// ------------------------------------------------------------ fusion kernels
// Hot chunks: persistent wavefronts walk the hot list (every wave exits when
// the list is exhausted).
__global__ __launch_bounds__(kBlock) void k_fuse_hot(FuseArgs a, const uint64_t* __restrict__ hot_list,
                                                     const uint32_t* __restrict__ hot_count) {
    const int lane = threadIdx.x & 63;
    const int64_t n = *a.n_act;
    const uint32_t nh = *hot_count;
    const uint32_t waves = gridDim.x * (kBlock / 64);
    for (uint32_t e = blockIdx.x * (kBlock / 64) + (threadIdx.x >> 6); e < nh; e += waves)
        fuse_chunk(a, n, (int64_t)(hot_list[e] & 0xFFFFFFFFFFull), lane);
}

// Cold chunks: one wavefront per chunk, XCD-aware block order (each XCD gets a
// contiguous range of chunks); hot chunks are left to k_fuse_hot.
__global__ __launch_bounds__(kBlock) void k_fuse_cold(FuseArgs a) {
    const unsigned G = gridDim.x;
    const unsigned b = blockIdx.x;
    const unsigned per = G / 8u;
    const unsigned lb = (b % 8u) * per + b / 8u;
    const int lane = threadIdx.x & 63;
    const int64_t n = *a.n_act;
    const int64_t chunk = (int64_t)lb * kWaves + (threadIdx.x >> 6);
    if (chunk * kChunk >= n) return;
    if (a.cull[chunk] & view_range(a.s_begin, a.s_end)) return;  // hot
    cold_chunk(a, n, chunk, lane);
}

}  // namespace

int pow2_at_least(int v) {
    int p = 1;
    while (p < v) p <<= 1;
    return p;
}

int device_cu_count() {
    static int n = 0;
    if (n == 0) {
        int dev = 0;
        hipDeviceProp_t prop;
        if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess)
            n = prop.multiProcessorCount;
        if (n <= 0) n = 256;
    }
    return n;
}

hipError_t launch_cull(const uint16_t* chunk_box, const int64_t* n_act, int64_t cap, const DGrid& g, double eps,
                       const DView* views, int32_t s_begin, int32_t s_end, uint64_t* cull, uint64_t fuse_range,
                       uint64_t* hot_list, uint32_t* hot_count, hipStream_t st) {
    int ns = s_end - s_begin;
    if (ns <= 0 || cap <= 0) return hipSuccess;
    int p2 = pow2_at_least(ns);
    int64_t nchunks = (cap + kChunk - 1) / kChunk;
    int64_t lanes = nchunks * p2;
    hipLaunchKernelGGL(k_cull, dim3((unsigned)((lanes + 255) / 256)), dim3(256), 0, st, chunk_box, n_act, g, eps, views,
                       s_begin, ns, p2, cull, lanes, fuse_range, hot_list, hot_count);
    return hipGetLastError();
}

hipError_t launch_fuse(const FuseArgs& a, const uint64_t* hot_list, const uint32_t* hot_count, int blocks_per_cu,
                       hipStream_t st) {
    if (a.cap <= 0) return hipSuccess;
    int64_t nchunks = (a.cap + kChunk - 1) / kChunk;
    int64_t hot_blocks = std::min<int64_t>((nchunks + kWaves - 1) / kWaves,
                                           (int64_t)std::max(1, blocks_per_cu) * device_cu_count());
    hipLaunchKernelGGL(k_fuse_hot, dim3((unsigned)hot_blocks), dim3(kBlock), 0, st, a, hot_list, hot_count);
    int64_t nblocks = (nchunks + kWaves - 1) / kWaves;
    nblocks = (nblocks + 7) / 8 * 8;  // whole XCD groups for the remap
    hipLaunchKernelGGL(k_fuse_cold, dim3((unsigned)nblocks), dim3(kBlock), 0, st, a);
    return hipGetLastError();
}

}  // namespace divas
