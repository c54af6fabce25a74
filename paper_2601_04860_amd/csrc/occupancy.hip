// Occupancy construction: points -> voxel density -> Morton-ordered active list.
//
// Sec. 3.5 ("Occupancy by Morton-scattered opacity") and App. F ("Occupancy
// grid construction"): points are filtered against the grid, mapped to an
// integer voxel and its Morton index, their opacities summed per voxel, and the
// voxels with rho >= tau (the transmittance floor tau_TF) form the compact
// active list.
//
// Two deterministic device paths, both ending in the same compaction:
//   * unit opacity with tau <= 1: rho >= tau  <=>  the voxel holds a point, so
//     only the set of occupied voxels is needed.  Points are binned by the top
//     bits of their Morton code (partitions of 2^18 voxels), and one workgroup
//     per partition builds that partition's bitmap in LDS with LDS atomics, so
//     no random device-scope atomic reaches memory;
//   * general opacity (or tau > 1): a counting sort by Morton code; each voxel
//     then sorts its own point indices and sums the opacities in point order in
//     binary64 (the order the definition is written in), no float atomics.
// Compaction walks the Morton bitmap tile by tile (1024 words): empty tiles are
// skipped, and the active voxels of a tile are written out in Morton order with
// coalesced stores (each output slot finds its word by a search over the tile's
// popcount prefix).  Per chunk of 64 consecutive active voxels
// the voxel-index bounding box is recorded for the culling of the fusion.
#include "kernels.h"

#include <algorithm>

namespace divas {

namespace {

constexpr int kScanThreads = 256;
constexpr int kWordsPerThread = 4;
constexpr int kWordsPerBlock = kScanThreads * kWordsPerThread;  // 1024 words = 32768 voxels
constexpr int kPartShiftMax = 18;    // voxels per partition: 2^18 (32 KB LDS bitmap)
constexpr int kMaxTilesPerPart = 8;  // 2^18 / 32 words / kWordsPerBlock
static_assert((1 << kPartShiftMax) / 32 / kWordsPerBlock == kMaxTilesPerPart, "tiles per partition");
constexpr int kMaxParts = 4096;      // 1024^3 grid / 2^18
constexpr int kCodeThreads = 1024;
constexpr int kCodesPerThread = 16;
constexpr int kCodesPerBlock = kCodeThreads * kCodesPerThread;
constexpr int kPartThreads = 1024;
constexpr uint32_t kNoVoxel = 0xFFFFFFFFu;  // Morton codes stay below 2^30

// Voxel of a point in binary64: floor((x - origin) / h) per axis; 0 when any
// coordinate is NaN or outside [0, dim).  Same expression as the label lookup.
__device__ __forceinline__ bool point_voxel(const float* __restrict__ xyz, int64_t i, const DGrid& g,
                                            uint32_t* ix, uint32_t* iy, uint32_t* iz) {
    uint32_t idx[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        double x = (double)xyz[3 * i + k];
        double f = floor((x - g.origin[k]) / g.h);
        if (!(f >= 0.0) || !(f < (double)g.dim)) return false;  // also rejects NaN
        idx[k] = (uint32_t)f;
    }
    *ix = idx[0];
    *iy = idx[1];
    *iz = idx[2];
    return true;
}

__global__ void k_fill_u32(uint32_t* __restrict__ p, uint32_t v, int64_t n) {
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    int64_t st = (int64_t)gridDim.x * blockDim.x;
    for (; i < n; i += st) p[i] = v;
}

// 16-byte stores over p[0, 4 * n4) (p 16-byte aligned).
__global__ void k_fill_u32x4(uint4* __restrict__ p, uint32_t v, int64_t n4) {
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    int64_t st = (int64_t)gridDim.x * blockDim.x;
    const uint4 q = make_uint4(v, v, v, v);
    for (; i < n4; i += st) p[i] = q;
}

__device__ __forceinline__ uint32_t wave_scan_incl(uint32_t v, int lane) {
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        uint32_t t = __shfl_up(v, off);
        if (lane >= off) v += t;
    }
    return v;
}

__device__ __forceinline__ uint32_t wave_sum(uint32_t v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    return v;
}

// Exclusive scan over a block of kThreads threads (a multiple of 64); the
// block total goes to *total.  Every thread of the block must call it.
template <int kThreads>
__device__ __forceinline__ uint32_t block_scan_excl(uint32_t v, uint32_t* total) {
    constexpr int kW = kThreads / 64;
    __shared__ uint32_t wsum[kW];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const uint32_t inc = wave_scan_incl(v, lane);
    if (lane == 63) wsum[w] = inc;
    __syncthreads();
    if (w == 0) {
        uint32_t x = lane < kW ? wsum[lane] : 0u;
        x = wave_scan_incl(x, lane);
        if (lane < kW) wsum[lane] = x;
    }
    __syncthreads();
    const uint32_t before = w ? wsum[w - 1] : 0u;
    *total = wsum[kW - 1];
    __syncthreads();
    return before + inc - v;
}

template <int kThreads>
__device__ __forceinline__ uint32_t block_sum(uint32_t v) {
    constexpr int kW = kThreads / 64;
    __shared__ uint32_t wsum[kW];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    v = wave_sum(v);
    if (lane == 0) wsum[w] = v;
    __syncthreads();
    uint32_t t = 0;
#pragma unroll
    for (int k = 0; k < kW; ++k) t += wsum[k];
    __syncthreads();
    return t;
}

// Position of the set bit of rank r (0-based, from bit 0) in w; r < popc(w).
__device__ __forceinline__ int select_bit(uint32_t w, uint32_t r) {
    int pos = 0;
#pragma unroll
    for (int width = 16; width > 0; width >>= 1) {
        const uint32_t c = __popc((w >> pos) & ((1u << width) - 1u));
        if (r >= c) {
            r -= c;
            pos += width;
        }
    }
    return pos;
}

// ---- unit-opacity path: bin by partition, then one LDS bitmap per partition
// Block b covers points [b * kCodesPerBlock, (b + 1) * kCodesPerBlock): the
// Morton code of each point (kNoVoxel outside the grid) and the block's
// partition histogram, written as row b of block_hist (nparts entries).  VEC:
// four consecutive points per step of a lane, three 16-byte xyz loads and one
// 16-byte code store (xyz and codes 16-byte aligned); a ragged last group is
// done point by point.
template <bool VEC>
__global__ __launch_bounds__(kCodeThreads) void k_occ_codes(const float* __restrict__ xyz, int64_t n, DGrid g,
                                                            int part_shift, int nparts, uint32_t* __restrict__ codes,
                                                            uint32_t* __restrict__ block_hist) {
    __shared__ uint32_t hist[kMaxParts];
    const int t = threadIdx.x;
    for (int b = t; b < nparts; b += kCodeThreads) hist[b] = 0u;
    __syncthreads();
    const double inv_h = 1.0 / g.h;
    const int64_t p0 = (int64_t)blockIdx.x * kCodesPerBlock;
    if constexpr (VEC) {
        constexpr int kSteps = kCodesPerThread / 4;
        float4 q[kSteps][3];
#pragma unroll
        for (int k = 0; k < kSteps; ++k) {
            const int64_t pt = p0 + 4 * ((int64_t)k * kCodeThreads + t);
            if (pt + 4 <= n) {
                const float4* x4 = (const float4*)(xyz + 3 * pt);
                q[k][0] = x4[0];
                q[k][1] = x4[1];
                q[k][2] = x4[2];
            }
        }
#pragma unroll
        for (int k = 0; k < kSteps; ++k) {
            const int64_t pt = p0 + 4 * ((int64_t)k * kCodeThreads + t);
            if (pt + 4 <= n) {
                const float4 a = q[k][0], b = q[k][1], c = q[k][2];
                uint4 m;
                m.x = morton_of(a.x, a.y, a.z, g, inv_h);
                m.y = morton_of(a.w, b.x, b.y, g, inv_h);
                m.z = morton_of(b.z, b.w, c.x, g, inv_h);
                m.w = morton_of(c.y, c.z, c.w, g, inv_h);
                if (m.x != kNoVoxel) atomicAdd(&hist[m.x >> part_shift], 1u);
                if (m.y != kNoVoxel) atomicAdd(&hist[m.y >> part_shift], 1u);
                if (m.z != kNoVoxel) atomicAdd(&hist[m.z >> part_shift], 1u);
                if (m.w != kNoVoxel) atomicAdd(&hist[m.w >> part_shift], 1u);
                *(uint4*)(codes + pt) = m;
            } else {
                for (int64_t i = pt; i < n; ++i) {
                    const uint32_t m = morton_of(xyz[3 * i], xyz[3 * i + 1], xyz[3 * i + 2], g, inv_h);
                    if (m != kNoVoxel) atomicAdd(&hist[m >> part_shift], 1u);
                    codes[i] = m;
                }
            }
        }
    } else {
        float p[kCodesPerThread][3];
#pragma unroll
        for (int k = 0; k < kCodesPerThread; ++k) {
            const int64_t i = p0 + (int64_t)k * kCodeThreads + t;
            if (i < n) {
                p[k][0] = xyz[3 * i];
                p[k][1] = xyz[3 * i + 1];
                p[k][2] = xyz[3 * i + 2];
            }
        }
#pragma unroll
        for (int k = 0; k < kCodesPerThread; ++k) {
            const int64_t i = p0 + (int64_t)k * kCodeThreads + t;
            if (i < n) {
                const uint32_t m = morton_of(p[k][0], p[k][1], p[k][2], g, inv_h);
                if (m != kNoVoxel) atomicAdd(&hist[m >> part_shift], 1u);
                codes[i] = m;
            }
        }
    }
    __syncthreads();
    uint32_t* row = block_hist + (int64_t)blockIdx.x * nparts;
    for (int b = t; b < nparts; b += kCodeThreads) row[b] = hist[b];
}

// One wavefront per partition p: exclusive scan of column p of block_hist over
// the nblk code blocks, in place (the offset of block b's run inside partition
// p), and the partition's total.  Lane l owns blocks [l * per, l * per + per);
// up to kOffRegs of them are kept in registers between the sum and the write
// (one memory round trip), more are read twice.  No atomics: the bin layout is
// deterministic.
constexpr int kOffRegs = 16;
__global__ __launch_bounds__(kScanThreads) void k_occ_offsets(uint32_t* __restrict__ block_hist, int64_t nblk,
                                                              int nparts, uint32_t* __restrict__ part_total) {
    const int lane = threadIdx.x & 63;
    const int p = blockIdx.x * (kScanThreads / 64) + (threadIdx.x >> 6);
    if (p >= nparts) return;  // uniform per wavefront
    const int64_t per = (nblk + 63) / 64;
    const int64_t b0 = lane * per;
    const int64_t b1 = b0 + per < nblk ? b0 + per : nblk;
    uint32_t s = 0;
    if (per <= kOffRegs) {
        uint32_t v[kOffRegs];
#pragma unroll
        for (int k = 0; k < kOffRegs; ++k) {
            v[k] = b0 + k < b1 ? block_hist[(b0 + k) * nparts + p] : 0u;
            s += v[k];
        }
        const uint32_t incl = wave_scan_incl(s, lane);
        uint32_t ex = incl - s;
#pragma unroll
        for (int k = 0; k < kOffRegs; ++k) {
            if (b0 + k < b1) block_hist[(b0 + k) * nparts + p] = ex;
            ex += v[k];
        }
        if (lane == 63) part_total[p] = incl;
        return;
    }
    for (int64_t b = b0; b < b1; ++b) s += block_hist[b * nparts + p];
    const uint32_t incl = wave_scan_incl(s, lane);
    uint32_t ex = incl - s;
    for (int64_t b = b0; b < b1; ++b) {
        const uint32_t v = block_hist[b * nparts + p];
        block_hist[b * nparts + p] = ex;
        ex += v;
    }
    if (lane == 63) part_total[p] = incl;
}

// Scatter of the codes into their partitions.  Same block ranges as
// k_occ_codes; the block's run of partition p starts at (sum of the totals of
// partitions before p) + block_hist[b][p].  The block first sorts its codes by partition in LDS (ranks
// from LDS atomics, run offsets from a block scan), then writes the runs with
// consecutive lanes on consecutive addresses.  The order inside a partition
// does not matter (the partition only ORs bits).
__global__ __launch_bounds__(kCodeThreads) void k_occ_scatter(const uint32_t* __restrict__ codes, int64_t n,
                                                              int part_shift, int nparts,
                                                              const uint32_t* __restrict__ block_hist,
                                                              const uint32_t* __restrict__ part_total,
                                                              uint32_t* __restrict__ binned) {
    __shared__ uint32_t hist[kMaxParts];  // run lengths, then (global base - local offset)
    __shared__ uint32_t loff[kMaxParts];  // local run offsets
    __shared__ uint32_t stage[kCodesPerBlock];
    const int t = threadIdx.x;
    for (int b = t; b < nparts; b += kCodeThreads) hist[b] = 0u;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * kCodesPerBlock + t;
    uint32_t code[kCodesPerThread], rank[kCodesPerThread];
#pragma unroll
    for (int k = 0; k < kCodesPerThread; ++k) {
        const int64_t i = base + (int64_t)k * kCodeThreads;
        code[k] = i < n ? codes[i] : kNoVoxel;
    }
#pragma unroll
    for (int k = 0; k < kCodesPerThread; ++k)
        rank[k] = code[k] != kNoVoxel ? atomicAdd(&hist[code[k] >> part_shift], 1u) : 0u;
    __syncthreads();
    // thread t owns partitions [t * per, t * per + per); the partition starts
    // are the exclusive scan of the partition totals, done here by every block
    const int per = (nparts + kCodeThreads - 1) / kCodeThreads;
    const int b0 = t * per;
    const int b1 = b0 + per < nparts ? b0 + per : nparts;
    uint32_t own = 0, own_pts = 0;
    for (int b = b0; b < b1; ++b) {
        own += hist[b];
        own_pts += part_total[b];
    }
    uint32_t total, all_pts;
    uint32_t run = block_scan_excl<kCodeThreads>(own, &total);
    uint32_t start = block_scan_excl<kCodeThreads>(own_pts, &all_pts);
    const uint32_t* row = block_hist + (int64_t)blockIdx.x * nparts;
    for (int b = b0; b < b1; ++b) {
        const uint32_t c = hist[b];
        loff[b] = run;
        hist[b] = start + row[b] - run;
        run += c;
        start += part_total[b];
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kCodesPerThread; ++k)
        if (code[k] != kNoVoxel) stage[loff[code[k] >> part_shift] + rank[k]] = code[k];
    __syncthreads();
    for (uint32_t j = t; j < total; j += kCodeThreads) {
        const uint32_t c = stage[j];
        binned[hist[c >> part_shift] + j] = c;
    }
}

// One block per partition: the partition's bitmap (part_words words) is built
// in LDS, then written out tile by tile (1024 words) with the tile's popcount;
// the partition's active-voxel total goes to part_unique[p].  Tiles without a
// set bit are not written (the compaction skips them).  The partition's run
// of binned codes starts at the sum of the earlier partitions' totals,
// reduced here by the block.
__global__ __launch_bounds__(kPartThreads) void k_occ_part_bits(const uint32_t* __restrict__ binned,
                                                                const uint32_t* __restrict__ part_total,
                                                                int part_shift, int part_words, int tiles_per_part,
                                                                uint32_t* __restrict__ bitmap,
                                                                uint32_t* __restrict__ tile_counts,
                                                                uint32_t* __restrict__ part_unique) {
    extern __shared__ uint32_t lbm[];
    const int p = blockIdx.x;
    const int t = threadIdx.x;
    uint32_t before = 0;
    for (int q = t; q < p; q += kPartThreads) before += part_total[q];
    const uint32_t b0 = block_sum<kPartThreads>(before), b1 = b0 + part_total[p];
    if (b0 == b1) {
        for (int k = t; k < tiles_per_part; k += kPartThreads) tile_counts[(int64_t)p * tiles_per_part + k] = 0u;
        if (t == 0) part_unique[p] = 0u;
        return;
    }
    const uint32_t local = (1u << part_shift) - 1u;
    for (int w = t; w < part_words; w += kPartThreads) lbm[w] = 0u;
    __syncthreads();
    uint32_t i = b0 + t;
    constexpr int kU = 8;  // loads in flight per thread
    for (; i + (kU - 1) * kPartThreads < b1; i += kU * kPartThreads) {
        uint32_t c[kU];
#pragma unroll
        for (int u = 0; u < kU; ++u) c[u] = binned[i + u * kPartThreads] & local;
#pragma unroll
        for (int u = 0; u < kU; ++u) atomicOr(&lbm[c[u] >> 5], 1u << (c[u] & 31u));
    }
    for (; i < b1; i += kPartThreads) {
        const uint32_t c = binned[i] & local;
        atomicOr(&lbm[c >> 5], 1u << (c & 31u));
    }
    __syncthreads();
    // tile totals: one wave reduction per tile, then thread k sums tile k over
    // the wavefronts (two barriers for all the partition's tiles)
    __shared__ uint32_t wtot[kPartThreads / 64][kMaxTilesPerPart];
    __shared__ uint32_t ttot[kMaxTilesPerPart];
    const int lane = t & 63, wv = t >> 6;
    uint32_t v[kMaxTilesPerPart];
#pragma unroll
    for (int k = 0; k < kMaxTilesPerPart; ++k) {
        const int w = k * kWordsPerBlock + t;
        v[k] = k < tiles_per_part && w < part_words ? lbm[w] : 0u;
        const uint32_t c = wave_sum((uint32_t)__popc(v[k]));
        if (lane == 0) wtot[wv][k] = c;
    }
    __syncthreads();
    if (t < kMaxTilesPerPart) {
        uint32_t s = 0;
#pragma unroll
        for (int j = 0; j < kPartThreads / 64; ++j) s += wtot[j][t];
        ttot[t] = s;
        if (t < tiles_per_part) tile_counts[(int64_t)p * tiles_per_part + t] = s;
    }
    __syncthreads();
    uint32_t unique = 0;
#pragma unroll
    for (int k = 0; k < kMaxTilesPerPart; ++k) {
        const int w = k * kWordsPerBlock + t;
        const uint32_t tot = ttot[k];
        if (tot && k < tiles_per_part && w < part_words) bitmap[(int64_t)p * part_words + w] = v[k];
        unique += k < tiles_per_part ? tot : 0u;
    }
    if (t == 0) part_unique[p] = unique;
}

// ---- general path: counting sort by Morton code
__global__ void k_count_points(const float* __restrict__ xyz, int64_t n, DGrid g, uint32_t* __restrict__ cnt) {
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    uint32_t x, y, z;
    if (!point_voxel(xyz, i, g, &x, &y, &z)) return;
    uint32_t m = spread3(x) | (spread3(y) << 1) | (spread3(z) << 2);
    atomicAdd(&cnt[m], 1u);
}

__global__ void k_scatter_points(const float* __restrict__ xyz, int64_t n, DGrid g, uint32_t* __restrict__ cur,
                                 uint32_t* __restrict__ list) {
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    uint32_t x, y, z;
    if (!point_voxel(xyz, i, g, &x, &y, &z)) return;
    uint32_t m = spread3(x) | (spread3(y) << 1) | (spread3(z) << 2);
    uint32_t slot = atomicAdd(&cur[m], 1u);
    list[slot] = (uint32_t)i;
}

// One thread per 32 voxels (one bitmap word).  After the scatter, end[m] is the
// end of voxel m's segment and end[m - 1] its start.  Each segment is sorted by
// point index (insertion sort; segments are short) and its opacities summed in
// that order in binary64.
__global__ void k_reduce_voxels(const uint32_t* __restrict__ end, uint32_t* __restrict__ list,
                                const float* __restrict__ opacity, double tau, int64_t nwords,
                                uint32_t* __restrict__ bitmap) {
    int64_t w = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (w >= nwords) return;
    uint32_t word = 0;
    for (int b = 0; b < 32; ++b) {
        int64_t m = w * 32 + b;
        uint32_t e = end[m];
        uint32_t s = m > 0 ? end[m - 1] : 0u;
        if (e == s) continue;
        for (uint32_t i = s + 1; i < e; ++i) {
            uint32_t key = list[i];
            uint32_t j = i;
            while (j > s && list[j - 1] > key) {
                list[j] = list[j - 1];
                --j;
            }
            list[j] = key;
        }
        double rho = 0.0;
        for (uint32_t i = s; i < e; ++i) rho += opacity ? (double)opacity[list[i]] : 1.0;
        if (rho >= tau) word |= 1u << b;
    }
    bitmap[w] = word;
}

// ---- generic in-place exclusive scan of uint32 (tiles of kWordsPerBlock)
__device__ __forceinline__ uint32_t block_exclusive_scan(uint32_t v, uint32_t* total) {
    __shared__ uint32_t sh[kScanThreads];
    int t = threadIdx.x;
    sh[t] = v;
    __syncthreads();
    for (int off = 1; off < kScanThreads; off <<= 1) {
        uint32_t add = t >= off ? sh[t - off] : 0u;
        __syncthreads();
        sh[t] += add;
        __syncthreads();
    }
    uint32_t incl = sh[t];
    *total = sh[kScanThreads - 1];
    __syncthreads();
    return incl - v;
}

__global__ void k_scan_tiles(const uint32_t* __restrict__ a, int64_t n, uint32_t* __restrict__ block_sums) {
    int64_t base = blockIdx.x * (int64_t)kWordsPerBlock + threadIdx.x * kWordsPerThread;
    uint32_t s = 0;
#pragma unroll
    for (int k = 0; k < kWordsPerThread; ++k)
        if (base + k < n) s += a[base + k];
    uint32_t tot;
    block_exclusive_scan(s, &tot);
    if (threadIdx.x == 0) block_sums[blockIdx.x] = tot;
}

// Single block: exclusive scan of the block sums in place; total -> *total (int64).
__global__ void k_scan_top(uint32_t* __restrict__ bs, int64_t nb, int64_t* __restrict__ total) {
    __shared__ uint32_t carry;
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    for (int64_t base = 0; base < nb; base += kScanThreads) {
        int64_t i = base + threadIdx.x;
        uint32_t v = i < nb ? bs[i] : 0u;
        uint32_t tot;
        uint32_t ex = block_exclusive_scan(v, &tot);
        if (i < nb) bs[i] = carry + ex;
        __syncthreads();
        if (threadIdx.x == 0) carry += tot;
        __syncthreads();
    }
    if (threadIdx.x == 0 && total) *total = (int64_t)carry;
}

__global__ void k_scan_apply(uint32_t* __restrict__ a, int64_t n, const uint32_t* __restrict__ block_off) {
    int64_t base = blockIdx.x * (int64_t)kWordsPerBlock + threadIdx.x * kWordsPerThread;
    uint32_t v[kWordsPerThread];
    uint32_t s = 0;
#pragma unroll
    for (int k = 0; k < kWordsPerThread; ++k) {
        v[k] = base + k < n ? a[base + k] : 0u;
        s += v[k];
    }
    uint32_t tot;
    uint32_t ex = block_exclusive_scan(s, &tot) + block_off[blockIdx.x];
#pragma unroll
    for (int k = 0; k < kWordsPerThread; ++k) {
        if (base + k < n) a[base + k] = ex;
        ex += v[k];
    }
}

// ---- compaction of the Morton bitmap
__global__ void k_bitmap_count(const uint32_t* __restrict__ bm, int64_t nwords, uint32_t* __restrict__ block_sums) {
    int64_t base = blockIdx.x * (int64_t)kWordsPerBlock + threadIdx.x * kWordsPerThread;
    uint32_t s = 0;
#pragma unroll
    for (int k = 0; k < kWordsPerThread; ++k)
        if (base + k < nwords) s += __popc(bm[base + k]);
    uint32_t tot;
    block_exclusive_scan(s, &tot);
    if (threadIdx.x == 0) block_sums[blockIdx.x] = tot;
}

// One block of 1024 threads: exclusive scan of the nb tile counts in place,
// c[nb] = total (c holds nb + 1 entries); the total also goes to *total.
// Thread t owns a contiguous run of ceil(nb / 1024) entries.
__global__ __launch_bounds__(1024) void k_scan_counts(uint32_t* __restrict__ c, int64_t nb,
                                                      int64_t* __restrict__ total, int64_t* __restrict__ total_host) {
    const int64_t per = (nb + 1023) / 1024;
    const int64_t b = threadIdx.x * per;
    const int64_t e = b + per < nb ? b + per : nb;
    uint32_t s = 0;
    for (int64_t i = b; i < e; ++i) s += c[i];
    uint32_t tot;
    uint32_t ex = block_scan_excl<1024>(s, &tot);
    for (int64_t i = b; i < e; ++i) {
        const uint32_t v = c[i];
        c[i] = ex;
        ex += v;
    }
    if (threadIdx.x == 0) {
        c[nb] = tot;
        if (total) *total = (int64_t)tot;
        if (total_host) *total_host = (int64_t)tot;  // pinned host memory: no copy operation needed
    }
}

// One block of 256 threads per tile of 1024 bitmap words (tile_off: the
// exclusive tile offsets, nb + 1 entries).  Thread t owns words 4t .. 4t + 3
// (one 16-byte load, issued together with the offset loads: a launch like this
// one is bound by dependent memory round trips, not by bandwidth); a word
// covers 32 consecutive Morton codes, i.e. a 4 x 4 x 2 brick (bits 0..4 of the
// code interleave x0 y0 z0 x1 y1), so the thread decodes each brick corner
// once and each set bit adds a small offset.  The voxels go, in order, to the
// LDS staging array at the thread's popcount prefix (a tile holds about 1.4k
// active voxels on average, rarely more than kStage), and the block copies them
// out with consecutive lanes on consecutive addresses; a tile with more than
// kStage voxels writes them straight to the list from the same loop.
// Every tile is left zero (the words of an empty tile are stale), so the
// bitmap is ready to serve as the empty segmentation bitfield.
//
// The tile's offset comes either from an exclusive scan of the tile counts
// (TileOffsets.part_total null: counts holds nb + 1 offsets) or, when the
// bitmap was built partition by partition, from the per-tile counts and the
// per-partition totals: the block sums the totals of the earlier partitions and
// the counts of the earlier tiles of its own partition, and the block of the
// last tile writes the active count.
struct TileOffsets {
    const uint32_t* counts;
    const uint32_t* part_total;
    int tiles_per_part;
    int64_t* n_act_dev;
    int64_t* n_act_host;
};
constexpr int kEmitThreads = 256;
constexpr int kEmitWords = 4;  // words per thread: 2, 4 or 8
constexpr int kEmitTiles = kEmitWords * kEmitThreads / kWordsPerBlock;
static_assert((kEmitWords == 2 || kEmitWords % 4 == 0) && kEmitTiles >= 1 &&
                  kEmitTiles * kWordsPerBlock == kEmitWords * kEmitThreads, "emit layout");
constexpr uint32_t kStage = 4096;
constexpr int kEmitMaxParts = 1024;  // partition totals read by each block (4 per thread at most)

// Writes the voxels of the thread's words, in order, to dst[pos ...]: the
// words as 64-bit halves, two set bits per step.  dst is the LDS
// staging array or the list itself (the compiler keeps the address space of
// each inlined call).
__device__ __forceinline__ void emit_words(const uint32_t (&q)[kEmitWords], const uint32_t (&base)[kEmitWords],
                                           const uint32_t* lut, uint32_t pos, uint32_t* dst) {
#pragma unroll
    for (int h = 0; h < kEmitWords / 2; ++h) {
        uint64_t w = (uint64_t)q[2 * h] | ((uint64_t)q[2 * h + 1] << 32);
        const uint32_t b0 = base[2 * h], b1 = base[2 * h + 1];
        while (w) {
            const uint32_t i1 = (uint32_t)(__ffsll((unsigned long long)w) - 1);
            w &= w - 1;
            dst[pos] = (i1 < 32 ? b0 : b1) + lut[i1 & 31u];  // bit 0..31: x0 y0 z0 x1 y1
            const bool two = w != 0;
            if (two) {
                const uint32_t i2 = (uint32_t)(__ffsll((unsigned long long)w) - 1);
                w &= w - 1;
                dst[pos + 1] = (i2 < 32 ? b0 : b1) + lut[i2 & 31u];
            }
            pos += two ? 2u : 1u;
        }
    }
}

__global__ __launch_bounds__(kEmitThreads) void k_bitmap_emit(uint32_t* __restrict__ bm, int64_t nwords,
                                                              int64_t ntiles, TileOffsets to, int log2dim,
                                                              uint32_t* __restrict__ act) {
    __shared__ uint32_t stage[kStage];
    __shared__ uint32_t lut[32];  // linear offset of bit b of a word from the word's brick corner
    const int64_t tile = blockIdx.x * (int64_t)kEmitTiles;  // the block's first tile
    const int t = threadIdx.x;
    if (t < 32) {
        const uint32_t dx = (t & 1u) | ((t >> 2) & 2u);
        const uint32_t dy = ((t >> 1) & 1u) | ((t >> 3) & 2u);
        const uint32_t dz = (t >> 2) & 1u;
        lut[t] = dx + (dy << log2dim) + (dz << (2 * log2dim));
    }
    const int64_t w0 = tile * (int64_t)kWordsPerBlock + (int64_t)t * kEmitWords;
    const bool whole = w0 + kEmitWords <= nwords;
    uint32_t q[kEmitWords];
    if (whole) {
        if constexpr (kEmitWords == 2) {
            const uint2 v = *(const uint2*)(bm + w0);
            q[0] = v.x;
            q[1] = v.y;
        } else {
#pragma unroll
            for (int j = 0; j < kEmitWords / 4; ++j) {
                const uint4 v = *(const uint4*)(bm + w0 + 4 * j);
                q[4 * j] = v.x;
                q[4 * j + 1] = v.y;
                q[4 * j + 2] = v.z;
                q[4 * j + 3] = v.w;
            }
        }
    } else {
#pragma unroll
        for (int k = 0; k < kEmitWords; ++k) q[k] = w0 + k < nwords ? bm[w0 + k] : 0u;
    }
    uint32_t off, cnt;
    if (to.part_total) {  // uniform
        const int tpp = to.tiles_per_part;
        const int p = (int)(tile / tpp);
        uint32_t s = 0;
        for (int i = t; i < p; i += kEmitThreads) s += to.part_total[i];
        for (int64_t i = (int64_t)p * tpp + t; i < tile; i += kEmitThreads) s += to.counts[i];
        cnt = 0;
#pragma unroll
        for (int j = 0; j < kEmitTiles; ++j) cnt += tile + j < ntiles ? to.counts[tile + j] : 0u;
        off = block_sum<kEmitThreads>(s);
        if (t == 0 && blockIdx.x + 1 == gridDim.x) {
            if (to.n_act_dev) *to.n_act_dev = (int64_t)(off + cnt);
            if (to.n_act_host) *to.n_act_host = (int64_t)(off + cnt);  // pinned host memory
        }
    } else {
        off = to.counts[tile];
        cnt = to.counts[tile + kEmitTiles < ntiles ? tile + kEmitTiles : ntiles] - off;
    }
    if (cnt != 0) {  // uniform
        uint32_t own = 0;
#pragma unroll
        for (int k = 0; k < kEmitWords; ++k) own += (uint32_t)__popc(q[k]);
        uint32_t tot;
        const uint32_t ex = block_scan_excl<kEmitThreads>(own, &tot);
        uint32_t base[kEmitWords];
#pragma unroll
        for (int k = 0; k < kEmitWords; ++k) {
            const uint32_t m0 = (uint32_t)((w0 + k) * 32);
            base[k] = compact3(m0) | (compact3(m0 >> 1) << log2dim) | (compact3(m0 >> 2) << (2 * log2dim));
        }
        if (cnt <= kStage) {  // uniform: staged, the usual case
            emit_words(q, base, lut, ex, stage);
            __syncthreads();
            for (uint32_t j = t; j < cnt; j += kEmitThreads) act[off + j] = stage[j];
        } else {
            emit_words(q, base, lut, ex, act + off);
        }
    }
    if (whole) {
        if constexpr (kEmitWords == 2) {
            *(uint2*)(bm + w0) = make_uint2(0u, 0u);
        } else {
#pragma unroll
            for (int j = 0; j < kEmitWords / 4; ++j) *(uint4*)(bm + w0 + 4 * j) = make_uint4(0u, 0u, 0u, 0u);
        }
    } else {
        for (int k = 0; k < kEmitWords; ++k)
            if (w0 + k < nwords) bm[w0 + k] = 0u;
    }
}

// Sixteen lanes per chunk of 64 consecutive active voxels: each lane loads
// four entries (one 16-byte load, so a chunk is one coalesced 256-byte read),
// decodes them, and a 16-lane shuffle reduction gives the chunk's voxel-index
// bounding box; the first lane turns it into the float box of the voxel
// centres (corners evaluated in binary64, then rounded) used by the culling.
// The active list is allocated in whole chunks, so the loads stay inside it;
// entries past n_act are ignored.  The same launch clears the session's
// per-voxel segmentation flags of the chunk (one 4-byte store per lane; the
// flags are allocated in whole chunks) and, striding over the grid, the coarse
// cell counts: a new active list starts with an empty segmentation.
constexpr int kBoxLanes = kChunk / 4;
__global__ void k_chunk_boxes(const uint32_t* __restrict__ act, const int64_t* __restrict__ n_act, DGrid g,
                              double pad, ChunkBox* __restrict__ box, uint32_t* __restrict__ segb4,
                              uint32_t* __restrict__ coarse, int64_t ncoarse) {
    const int64_t n = *n_act;
    const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    for (int64_t c = t; c < ncoarse; c += (int64_t)gridDim.x * blockDim.x) coarse[c] = 0u;
    const int64_t chunk = t / kBoxLanes;
    const int q = (int)(t % kBoxLanes);
    const bool in = chunk * kChunk < n;  // uniform over the 16 lanes of a chunk
    if (in && segb4) segb4[chunk * kBoxLanes + q] = 0u;
    const int log2dim = g.log2dim;
    const uint32_t mask = (1u << log2dim) - 1u;
    uint32_t lo[3] = {0xFFFFu, 0xFFFFu, 0xFFFFu}, hi[3] = {0u, 0u, 0u};
    if (in) {
        const uint4 v = *(const uint4*)(act + chunk * kChunk + 4 * q);
        const uint32_t e[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            if (chunk * kChunk + 4 * q + r < n) {
                const uint32_t c[3] = {e[r] & mask, (e[r] >> log2dim) & mask, e[r] >> (2 * log2dim)};
#pragma unroll
                for (int k = 0; k < 3; ++k) {
                    lo[k] = c[k] < lo[k] ? c[k] : lo[k];
                    hi[k] = c[k] > hi[k] ? c[k] : hi[k];
                }
            }
        }
    }
#pragma unroll
    for (int off = kBoxLanes / 2; off > 0; off >>= 1) {
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const uint32_t l = (uint32_t)__shfl_xor((int)lo[k], off), h = (uint32_t)__shfl_xor((int)hi[k], off);
            lo[k] = l < lo[k] ? l : lo[k];
            hi[k] = h > hi[k] ? h : hi[k];
        }
    }
    if (in && q == 0) {
        ChunkBox cb;
        float p1 = 0.f;
        for (int k = 0; k < 3; ++k) {
            const float l = (float)(g.origin[k] + ((double)lo[k] + 0.5) * g.h - pad);
            const float h = (float)(g.origin[k] + ((double)hi[k] + 0.5) * g.h + pad);
            cb.lo[k] = l;
            cb.ext[k] = h - l;
            p1 += fmaxf(fabsf(l), fabsf(h));
        }
        cb.p1 = p1;
        cb.pad = 0.f;
        box[chunk] = cb;
    }
}

inline unsigned blocks_for(int64_t n, int t) { return (unsigned)((n + t - 1) / t); }

hipError_t scan_in_place(uint32_t* a, int64_t n, uint32_t* block_sums, int64_t* total, hipStream_t st) {
    int64_t nb = (n + kWordsPerBlock - 1) / kWordsPerBlock;
    if (nb == 0) nb = 1;
    hipLaunchKernelGGL(k_scan_tiles, dim3((unsigned)nb), dim3(kScanThreads), 0, st, a, n, block_sums);
    hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(kScanThreads), 0, st, block_sums, nb, total);
    hipLaunchKernelGGL(k_scan_apply, dim3((unsigned)nb), dim3(kScanThreads), 0, st, a, n, block_sums);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_scan_u32(uint32_t* a, int64_t n, uint32_t* block_sums, int64_t* total, hipStream_t st) {
    return scan_in_place(a, n, block_sums, total, st);
}

size_t scan_block_sums(int64_t n) { return (size_t)(n / kWordsPerBlock + 2); }

hipError_t launch_fill_u32(uint32_t* p, uint32_t v, int64_t n, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    int64_t head = 0;
    if (((uintptr_t)p & 15u) == 0) {
        const int64_t n4 = n / 4;
        if (n4 > 0) {
            unsigned nb = (unsigned)std::min<int64_t>((n4 + 255) / 256, 8192);
            hipLaunchKernelGGL(k_fill_u32x4, dim3(nb), dim3(256), 0, st, (uint4*)p, v, n4);
        }
        head = n4 * 4;
    }
    if (head < n) {
        unsigned nb = (unsigned)std::min<int64_t>((n - head + 255) / 256, 65536);
        hipLaunchKernelGGL(k_fill_u32, dim3(nb), dim3(256), 0, st, p + head, v, n - head);
    }
    return hipGetLastError();
}


OccPlan occupancy_plan(const DGrid& g) {
    OccPlan q{};
    const int mbits = 3 * g.log2dim;
    q.part_shift = std::min(kPartShiftMax, mbits);
    q.nparts = 1 << (mbits - q.part_shift);
    q.part_words = std::max(1, (1 << q.part_shift) / 32);
    q.tiles_per_part = std::max(1, q.part_words / kWordsPerBlock);
    return q;
}

size_t occupancy_work_bytes(const DGrid& g, int64_t max_points) {
    const int64_t np = max_points > 0 ? max_points : 1;
    const int64_t nblk = (np + kCodesPerBlock - 1) / kCodesPerBlock;
    const OccPlan q = occupancy_plan(g);
    return (size_t)(2 * np + (int64_t)q.nparts * nblk + 2 * kMaxParts + 1) * 4 + 16;
}

// The layout of launch_occupancy's work buffer: partition totals and unique
// counts, the code blocks' partition histograms, then the codes (16-byte
// aligned) and the binned codes.
static uint32_t* occupancy_codes_in(const DGrid& g, uint32_t* work, int64_t n) {
    const OccPlan q = occupancy_plan(g);
    const int64_t np = n > 0 ? n : 1;
    const int64_t nblk = (np + kCodesPerBlock - 1) / kCodesPerBlock;
    uint32_t* codes = work + 2 * kMaxParts + 1 + (int64_t)q.nparts * nblk;
    return codes + (16 - ((uintptr_t)codes & 15u)) / 4 % 4;  // the buffer holds 16 spare bytes
}

const uint32_t* occupancy_codes(const DGrid& g, const uint32_t* work, int64_t n) {
    return occupancy_codes_in(g, const_cast<uint32_t*>(work), n);
}

size_t occupancy_scratch_bytes(const DGrid& g, int64_t max_points, int opacity_path) {
    if (!opacity_path) return 0;
    int64_t nvox = (int64_t)g.dim * g.dim * g.dim;
    int64_t nb = nvox / kWordsPerBlock + 1;
    return (size_t)nvox * 4 + (size_t)(max_points > 0 ? max_points : 1) * 4 + (size_t)nb * 4;
}

// act: room for whole chunks (a multiple of 64 entries >= min(n, dim^3)).
// bitmap: dim^3 / 32 words in Morton order, the occupancy bits while the
// active list is emitted; on return it is all zero.  n_act_host: pinned host
// memory that receives the count as well (or null).  segb (whole chunks, 4-byte
// aligned) and coarse (coarse_cells(g) words): cleared for the new list (or
// null).
// block_counts: >= ceil(words / 1024) + 1 entries.  work: occupancy_work_bytes
// (partition counts zero on entry; they are left zero).
hipError_t launch_occupancy(const float* xyz, const float* opacity, int64_t n, double tau_occ, const DGrid& g,
                            uint32_t* bitmap, uint32_t* block_counts, uint32_t* act, ChunkBox* chunk_box,
                            int64_t* n_act_dev, int64_t* n_act_host, uint8_t* segb, uint32_t* coarse,
                            uint32_t* work, void* scratch, size_t scratch_bytes, hipStream_t st, PhaseEvents ev,
                            double box_pad) {
    int64_t nvox = (int64_t)g.dim * g.dim * g.dim;
    int64_t nwords = (nvox + 31) / 32;
    int64_t nb = (nwords + kWordsPerBlock - 1) / kWordsPerBlock;
    hipError_t e;
    bool general = opacity != nullptr || tau_occ > 1.0;
    bool emitted = false;
    if (!general) {
        const OccPlan q = occupancy_plan(g);
        if (q.nparts > kMaxParts || (int64_t)q.nparts * q.tiles_per_part != nb) return hipErrorInvalidValue;
        const int64_t np = n > 0 ? n : 1;
        const int64_t nblk = (np + kCodesPerBlock - 1) / kCodesPerBlock;
        uint32_t* part_total = work;
        uint32_t* part_unique = part_total + kMaxParts;
        uint32_t* block_hist = part_unique + kMaxParts + 1;
        uint32_t* codes = occupancy_codes_in(g, work, n);  // 16-byte aligned
        uint32_t* binned = codes + np;
        if (n > 0) {
            if (((uintptr_t)xyz & 15u) == 0)
                launch_timed(k_occ_codes<true>, dim3((unsigned)nblk), dim3(kCodeThreads), 0, st, ev.start, nullptr,
                             xyz, n, g, q.part_shift, q.nparts, codes, block_hist);
            else
                launch_timed(k_occ_codes<false>, dim3((unsigned)nblk), dim3(kCodeThreads), 0, st, ev.start, nullptr,
                             xyz, n, g, q.part_shift, q.nparts, codes, block_hist);
            hipLaunchKernelGGL(k_occ_offsets, dim3((unsigned)((q.nparts + 3) / 4)), dim3(kScanThreads), 0, st,
                               block_hist, nblk, q.nparts, part_total);
        } else {
            launch_timed(k_fill_u32, dim3(1), dim3(256), 0, st, ev.start, nullptr, part_total, 0u, (int64_t)q.nparts);
        }
        if (n > 0)
            hipLaunchKernelGGL(k_occ_scatter, dim3((unsigned)nblk), dim3(kCodeThreads), 0, st, codes, n, q.part_shift,
                               q.nparts, block_hist, part_total, binned);
        hipLaunchKernelGGL(k_occ_part_bits, dim3((unsigned)q.nparts), dim3(kPartThreads),
                           (size_t)q.part_words * 4, st, binned, part_total, q.part_shift, q.part_words,
                           q.tiles_per_part, bitmap, block_counts, part_unique);
        if (q.nparts <= kEmitMaxParts) {
            const TileOffsets to{block_counts, part_unique, q.tiles_per_part, n_act_dev, n_act_host};
            hipLaunchKernelGGL(k_bitmap_emit, dim3((unsigned)((nb + kEmitTiles - 1) / kEmitTiles)),
                               dim3(kEmitThreads), 0, st, bitmap, nwords, nb, to, g.log2dim, act);
            emitted = true;
        }
    } else {
        if (scratch_bytes < occupancy_scratch_bytes(g, n, 1)) return hipErrorInvalidValue;
        if (ev.start) (void)hipEventRecord(ev.start, st);  // several helper launches follow
        uint32_t* cnt = (uint32_t*)scratch;
        uint32_t* list = cnt + nvox;
        uint32_t* sums = list + (n > 0 ? n : 1);
        if ((e = launch_fill_u32(cnt, 0u, nvox, st)) != hipSuccess) return e;
        if (n > 0) hipLaunchKernelGGL(k_count_points, dim3(blocks_for(n, 256)), dim3(256), 0, st, xyz, n, g, cnt);
        if ((e = scan_in_place(cnt, nvox, sums, nullptr, st)) != hipSuccess) return e;
        if (n > 0) hipLaunchKernelGGL(k_scatter_points, dim3(blocks_for(n, 256)), dim3(256), 0, st, xyz, n, g, cnt, list);
        hipLaunchKernelGGL(k_reduce_voxels, dim3(blocks_for(nwords, 256)), dim3(256), 0, st, cnt, list, opacity,
                           tau_occ, nwords, bitmap);
        hipLaunchKernelGGL(k_bitmap_count, dim3((unsigned)nb), dim3(kScanThreads), 0, st, bitmap, nwords,
                           block_counts);
    }
    if (!emitted) {
        hipLaunchKernelGGL(k_scan_counts, dim3(1), dim3(1024), 0, st, block_counts, nb, n_act_dev, n_act_host);
        const TileOffsets to{block_counts, nullptr, 1, nullptr, nullptr};
        hipLaunchKernelGGL(k_bitmap_emit, dim3((unsigned)((nb + kEmitTiles - 1) / kEmitTiles)), dim3(kEmitThreads),
                           0, st, bitmap, nwords, nb, to, g.log2dim, act);
    }
    int64_t cap = std::max<int64_t>(std::min<int64_t>(n, nvox), 1);
    int64_t nchunks = (cap + kChunk - 1) / kChunk;
    launch_timed(k_chunk_boxes, dim3(blocks_for(nchunks * kBoxLanes, 256)), dim3(256), 0, st, nullptr, ev.stop, act,
                 (const int64_t*)n_act_dev, g, box_pad, chunk_box, (uint32_t*)segb, coarse,
                 coarse ? coarse_cells(g) : (int64_t)0);
    return hipGetLastError();
}

namespace {
// Points per active voxel: each point finds its voxel in the Morton-ordered
// list by binary search on the Morton codes and adds one (integer atomics:
// the count does not depend on their order).
__global__ void k_voxel_density(const float* __restrict__ xyz, int64_t n, DGrid g, double inv_h,
                                const uint32_t* __restrict__ act, const int64_t* __restrict__ n_act,
                                uint32_t* __restrict__ rho) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint32_t m = morton_of(xyz[3 * i], xyz[3 * i + 1], xyz[3 * i + 2], g, inv_h);
    if (m == 0xFFFFFFFFu) return;
    const uint32_t msk = (uint32_t)g.dim - 1u;
    const auto code = [&](uint32_t l) {
        return spread3(l & msk) | (spread3((l >> g.log2dim) & msk) << 1) | (spread3(l >> (2 * g.log2dim)) << 2);
    };
    const int64_t na = *n_act;
    int64_t lo = 0, hi = na;  // first entry whose code is >= m
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (code(act[mid]) < m)
            lo = mid + 1;
        else
            hi = mid;
    }
    if (lo < na && code(act[lo]) == m) atomicAdd(&rho[lo], 1u);
}
}  // namespace

hipError_t launch_voxel_density(const float* xyz, int64_t n, const DGrid& g, const uint32_t* act,
                                const int64_t* n_act, int64_t cap, uint32_t* rho, hipStream_t st) {
    hipError_t e = launch_fill_u32(rho, 0u, cap > 0 ? cap : 1, st);
    if (e != hipSuccess || n <= 0) return e;
    hipLaunchKernelGGL(k_voxel_density, dim3(blocks_for(n, 256)), dim3(256), 0, st, xyz, n, g, 1.0 / g.h, act, n_act,
                       rho);
    return hipGetLastError();
}

}  // namespace divas
