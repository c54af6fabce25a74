// Batched fusion: many sessions (scenes, objects, grids and view counts of
// uneven size) in one sequence of five launches, every one sized for the whole
// batch:
//   k_batch_prep   scatters the new view records into their sessions, zeroes
//                  the items' counters and the hot-list counter, and computes
//                  the hot-tile rows of every new view (wavefront per row);
//   k_batch_cols   the column pass of those tile tables (wavefront per column);
//   k_batch_cull   culls every (item, chunk, new view) triple and appends the
//                  chunks with views to evaluate to one batch-wide hot list;
//   k_batch_hot    persistent wavefronts walk the hot list and fuse its chunks
//                  (every wave exits when the list is exhausted);
//   k_batch_cold   the remaining chunks of every item (no new vote).
// A voxel is still accumulated by one lane, in view order, with the same device
// code as the single-session kernels, so every item's outputs are bit-identical
// to running it alone.  The grids are fixed per batch object, so the launch
// sequence can be captured once in a HIP graph and replayed with new tables.
#include "batch.h"
#include "fuse_core.h"

namespace divas {

namespace {

__device__ __forceinline__ int find_job(const int64_t* __restrict__ base, int n, int64_t t) {
    int lo = 0, hi = n - 1;
    while (lo < hi) {  // last job whose base <= t
        int mid = (lo + hi + 1) >> 1;
        if (base[mid] <= t)
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo;
}

__global__ void k_batch_prep(BatchTables t) {
    const BatchHeader& h = *t.header;
    const int64_t gid = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const int64_t gsz = (int64_t)gridDim.x * blockDim.x;
    for (int64_t j = gid; j < h.n_vjobs; j += gsz) {
        const BViewJob& vj = t.vjobs[j];
        t.items[vj.item].views_rw[vj.slot] = t.vrecs[j];
    }
    for (int64_t j = gid; j < (int64_t)h.n_items * 3; j += gsz) t.items[j / 3].f.counts[j % 3] = 0;
    if (gid == 0) *t.hot_count = 0u;
    // tile rows of the new views, from the batch's own copy of the records
    const int64_t wave = gid >> 6, nwaves = gsz >> 6;
    for (int64_t r = wave; r < h.total_rows; r += nwaves) {
        int j = find_job(t.vjob_row_base, h.n_vjobs, r);
        tile_row_scan(t.vrecs[j], (int)(r - t.vjob_row_base[j]), t.items[t.vjobs[j].item].gate);
    }
}

__global__ void k_batch_cols(BatchTables t) {
    const BatchHeader& h = *t.header;
    const int64_t wave = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> 6;
    const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
    for (int64_t c = wave; c < h.total_cols; c += nwaves) {
        int j = find_job(t.vjob_col_base, h.n_vjobs, c);
        tile_col_scan(t.vrecs[j], 1 + (int)(c - t.vjob_col_base[j]));
    }
}

// Lanes are laid out per job in whole wavefronts (job bases are multiples of
// 64 and every wave runs the same number of iterations), as cull_group needs.
__global__ void k_batch_cull(BatchTables t) {
    const BatchHeader& h = *t.header;
    const int64_t gsz = (int64_t)gridDim.x * blockDim.x;
    for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < h.total_cull; k += gsz) {
        int j = find_job(t.cjob_lane_base, h.n_cjobs, k);
        const BCullJob& cj = t.cjobs[j];
        const BItem& it = t.items[cj.item];
        const int64_t n = *it.f.n_act;
        const int64_t local = k - t.cjob_lane_base[j];
        const int64_t nch = (n + kChunk - 1) / kChunk;
        cull_group(it.box, n, it.f.g, it.f.p.eps, it.f.views, cj.s_begin, cj.ns, cj.p2, local, it.cull_rw,
                   local < nch * cj.p2, it.fuse_range, (uint64_t)cj.item << 40, t.hot_list, t.hot_count);
    }
}

__global__ __launch_bounds__(kBlock) void k_batch_hot(BatchTables t) {
    const int lane = threadIdx.x & 63;
    const uint32_t nh = *t.hot_count;
    const uint32_t waves = gridDim.x * (kBlock / 64);
    for (uint32_t e = blockIdx.x * (kBlock / 64) + (threadIdx.x >> 6); e < nh; e += waves) {
        const uint64_t tag = t.hot_list[e];
        const BItem& it = t.items[(int)(tag >> 40)];
        fuse_chunk(it.f, *it.f.n_act, (int64_t)(tag & 0xFFFFFFFFFFull), lane);
    }
}

__global__ __launch_bounds__(kBlock) void k_batch_cold(BatchTables t) {
    const BatchHeader& h = *t.header;
    const int lane = threadIdx.x & 63;
    const int64_t wave = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> 6;
    const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
    for (int64_t c = wave; c < h.total_chunks; c += nwaves) {
        int j = find_job(t.item_chunk_base, h.n_items, c);
        const BItem& it = t.items[j];
        const int64_t n = *it.f.n_act;
        const int64_t chunk = c - t.item_chunk_base[j];
        if (chunk * kChunk >= n) continue;
        if (it.f.cull[chunk] & it.fuse_range) continue;  // hot
        cold_chunk(it.f, n, chunk, lane);
    }
}

}  // namespace

hipError_t launch_batch_phase(const BatchTables& t, const BatchGrid& g, int phase, hipStream_t st) {
    if (phase == 0) hipLaunchKernelGGL(k_batch_prep, dim3(g.prep_blocks), dim3(256), 0, st, t);
    if (phase == 1) hipLaunchKernelGGL(k_batch_cols, dim3(g.sat_blocks), dim3(256), 0, st, t);
    if (phase == 2) hipLaunchKernelGGL(k_batch_cull, dim3(g.cull_blocks), dim3(256), 0, st, t);
    if (phase == 3) hipLaunchKernelGGL(k_batch_hot, dim3(g.fuse_blocks), dim3(kBlock), 0, st, t);
    if (phase == 4) hipLaunchKernelGGL(k_batch_cold, dim3(g.cold_blocks), dim3(kBlock), 0, st, t);
    return hipGetLastError();
}

hipError_t launch_batch(const BatchTables& t, const BatchGrid& g, hipStream_t st) {
    for (int ph = 0; ph < kBatchPhases; ++ph) {
        hipError_t e = launch_batch_phase(t, g, ph, st);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace divas
