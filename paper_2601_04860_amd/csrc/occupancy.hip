// Occupancy construction: points -> voxel density -> Morton-ordered active list.
//
// Sec. 3.5 ("Occupancy by Morton-scattered opacity") and App. F ("Occupancy
// grid construction"): points are filtered against the grid, mapped to an
// integer voxel and its Morton index, their opacities summed per voxel, and the
// voxels with rho >= tau (the transmittance floor tau_TF) form the compact
// active list.
//
// Two deterministic device paths, both ending in the same compaction:
//   * unit opacity with tau <= 1: rho >= tau  <=>  the voxel holds a point, so a
//     Morton-ordered occupancy bitmap is built with integer atomicOr;
//   * general opacity (or tau > 1): a counting sort by Morton code; each voxel
//     then sorts its own point indices and sums the opacities in point order in
//     binary64 (the order the definition is written in), no float atomics.
// Compaction walks the Morton bitmap with popcounts and a block scan, so the
// list comes out in Morton order.  Per chunk of 64 consecutive active voxels
// the voxel-index bounding box is recorded for the culling of the fusion.
#include "kernels.h"

#include <algorithm>

namespace divas {

namespace {

constexpr int kScanThreads = 256;
constexpr int kWordsPerThread = 4;
constexpr int kWordsPerBlock = kScanThreads * kWordsPerThread;  // 1024 words = 32768 voxels

__device__ __forceinline__ uint32_t spread3(uint32_t v) {
    // bit b of v -> bit 3b (v < 1024)
    v &= 0x3FFu;
    v = (v | (v << 16)) & 0x030000FFu;
    v = (v | (v << 8)) & 0x0300F00Fu;
    v = (v | (v << 4)) & 0x030C30C3u;
    v = (v | (v << 2)) & 0x09249249u;
    return v;
}

__device__ __forceinline__ uint32_t compact3(uint32_t v) {
    v &= 0x09249249u;
    v = (v | (v >> 2)) & 0x030C30C3u;
    v = (v | (v >> 4)) & 0x0300F00Fu;
    v = (v | (v >> 8)) & 0x030000FFu;
    v = (v | (v >> 16)) & 0x000003FFu;
    return v;
}

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

__global__ void k_mark_points(const float* __restrict__ xyz, int64_t n, DGrid g, uint32_t* __restrict__ bitmap) {
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    uint32_t x, y, z;
    if (!point_voxel(xyz, i, g, &x, &y, &z)) return;
    uint32_t m = spread3(x) | (spread3(y) << 1) | (spread3(z) << 2);
    atomicOr(&bitmap[m >> 5], 1u << (m & 31u));
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

__global__ void k_bitmap_write(const uint32_t* __restrict__ bm, int64_t nwords, const uint32_t* __restrict__ block_off,
                               int log2dim, uint32_t* __restrict__ act) {
    int64_t base = blockIdx.x * (int64_t)kWordsPerBlock + threadIdx.x * kWordsPerThread;
    uint32_t w[kWordsPerThread];
    uint32_t s = 0;
#pragma unroll
    for (int k = 0; k < kWordsPerThread; ++k) {
        w[k] = base + k < nwords ? bm[base + k] : 0u;
        s += __popc(w[k]);
    }
    uint32_t tot;
    uint32_t pos = block_exclusive_scan(s, &tot) + block_off[blockIdx.x];
#pragma unroll
    for (int k = 0; k < kWordsPerThread; ++k) {
        uint32_t word = w[k];
        while (word) {
            int b = __ffs(word) - 1;
            word &= word - 1;
            uint32_t m = (uint32_t)((base + k) * 32 + b);
            uint32_t x = compact3(m), y = compact3(m >> 1), z = compact3(m >> 2);
            act[pos++] = x | (y << log2dim) | (z << (2 * log2dim));
        }
    }
}

// One wavefront per chunk of 64 consecutive active voxels: voxel-index bounding box.
__global__ void k_chunk_boxes(const uint32_t* __restrict__ act, const int64_t* __restrict__ n_act, int64_t cap,
                              int log2dim, uint16_t* __restrict__ box) {
    int64_t n = *n_act;
    int lane = threadIdx.x & 63;
    int64_t chunk = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> 6;
    if (chunk * kChunk >= n) return;
    int64_t i = chunk * kChunk + lane;
    uint32_t mask = (1u << log2dim) - 1u;
    int lo[3] = {65535, 65535, 65535}, hi[3] = {0, 0, 0};
    if (i < n) {
        uint32_t l = act[i];
        int c[3] = {(int)(l & mask), (int)((l >> log2dim) & mask), (int)(l >> (2 * log2dim))};
        for (int k = 0; k < 3; ++k) lo[k] = hi[k] = c[k];
    }
    for (int off = 32; off > 0; off >>= 1) {
        for (int k = 0; k < 3; ++k) {
            lo[k] = min(lo[k], __shfl_xor(lo[k], off));
            hi[k] = max(hi[k], __shfl_xor(hi[k], off));
        }
    }
    if (lane == 0) {
        uint16_t* b = box + chunk * 8;
        for (int k = 0; k < 3; ++k) {
            b[k] = (uint16_t)lo[k];
            b[3 + k] = (uint16_t)hi[k];
        }
        b[6] = b[7] = 0;
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
    unsigned nb = (unsigned)std::min<int64_t>((n + 255) / 256, 65536);
    hipLaunchKernelGGL(k_fill_u32, dim3(nb), dim3(256), 0, st, p, v, n);
    return hipGetLastError();
}

size_t occupancy_scratch_bytes(const DGrid& g, int64_t max_points, int opacity_path) {
    if (!opacity_path) return 0;
    int64_t nvox = (int64_t)g.dim * g.dim * g.dim;
    int64_t nb = nvox / kWordsPerBlock + 1;
    return (size_t)nvox * 4 + (size_t)(max_points > 0 ? max_points : 1) * 4 + (size_t)nb * 4;
}

// bitmap: dim^3 / 32 words (Morton order; left zeroed on return is NOT promised:
// it holds the occupancy bits).  block_counts: >= ceil(words / 1024) entries.
hipError_t launch_occupancy(const float* xyz, const float* opacity, int64_t n, double tau_occ, const DGrid& g,
                            uint32_t* bitmap, uint32_t* block_counts, uint32_t* act, uint16_t* chunk_box,
                            int64_t* n_act_dev, void* scratch, size_t scratch_bytes, hipStream_t st) {
    int64_t nvox = (int64_t)g.dim * g.dim * g.dim;
    int64_t nwords = (nvox + 31) / 32;
    hipError_t e;
    bool general = opacity != nullptr || tau_occ > 1.0;
    if (!general) {
        if ((e = launch_fill_u32(bitmap, 0u, nwords, st)) != hipSuccess) return e;
        if (n > 0) hipLaunchKernelGGL(k_mark_points, dim3(blocks_for(n, 256)), dim3(256), 0, st, xyz, n, g, bitmap);
    } else {
        if (scratch_bytes < occupancy_scratch_bytes(g, n, 1)) return hipErrorInvalidValue;
        uint32_t* cnt = (uint32_t*)scratch;
        uint32_t* list = cnt + nvox;
        uint32_t* sums = list + (n > 0 ? n : 1);
        if ((e = launch_fill_u32(cnt, 0u, nvox, st)) != hipSuccess) return e;
        if (n > 0) hipLaunchKernelGGL(k_count_points, dim3(blocks_for(n, 256)), dim3(256), 0, st, xyz, n, g, cnt);
        if ((e = scan_in_place(cnt, nvox, sums, nullptr, st)) != hipSuccess) return e;
        if (n > 0) hipLaunchKernelGGL(k_scatter_points, dim3(blocks_for(n, 256)), dim3(256), 0, st, xyz, n, g, cnt, list);
        hipLaunchKernelGGL(k_reduce_voxels, dim3(blocks_for(nwords, 256)), dim3(256), 0, st, cnt, list, opacity,
                           tau_occ, nwords, bitmap);
    }
    int64_t nb = (nwords + kWordsPerBlock - 1) / kWordsPerBlock;
    hipLaunchKernelGGL(k_bitmap_count, dim3((unsigned)nb), dim3(kScanThreads), 0, st, bitmap, nwords, block_counts);
    hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(kScanThreads), 0, st, block_counts, nb, n_act_dev);
    hipLaunchKernelGGL(k_bitmap_write, dim3((unsigned)nb), dim3(kScanThreads), 0, st, bitmap, nwords, block_counts,
                       g.log2dim, act);
    int64_t cap = std::max<int64_t>(std::min<int64_t>(n, nvox), 1);
    int64_t nchunks = (cap + kChunk - 1) / kChunk;
    hipLaunchKernelGGL(k_chunk_boxes, dim3(blocks_for(nchunks * 64, 256)), dim3(256), 0, st, act, n_act_dev, cap,
                       g.log2dim, chunk_box);
    return hipGetLastError();
}

}  // namespace divas
