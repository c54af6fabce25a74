// Batched fusion: many sessions (scenes, objects, grids and view counts of
// uneven size) in one sequence of four launches, every one sized for the whole
// batch:
//   k_batch_prep   scatters the new view records into their sessions and
//                  computes the hot-tile words and the gate bitmask of every
//                  new view (wavefront per tile row);
//   k_batch_cull   culls every (item, chunk, new view) triple into the items'
//                  cull words;
//   k_batch_fuse   one wavefront per chunk of every item: the thick path for
//                  chunks with a view bit in their item's fused range, the
//                  outputs only for the others (or k_batch_fuse_queue, the
//                  persistent schedule: a fixed grid pulling chunk-range
//                  descriptors, costliest items first, from an atomic queue);
//   k_batch_counts sums every item's partial count slots into its counts.
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

// Job tables of up to kLdsJobs entries are copied to LDS so that the searches
// above cost LDS reads, not dependent global loads.  Uniform per block.
constexpr int kLdsJobs = 1024;
__device__ __forceinline__ const int64_t* stage_table(int64_t* sh, const int64_t* __restrict__ g, int n) {
    if (n > kLdsJobs) return g;
    for (int k = threadIdx.x; k < n; k += blockDim.x) sh[k] = g[k];
    __syncthreads();
    return sh;
}

__global__ void k_batch_prep(BatchTables t) {
    const BatchHeader& h = *t.header;
    const int64_t gid = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const int64_t gsz = (int64_t)gridDim.x * blockDim.x;
    for (int64_t j = gid; j < h.n_vjobs; j += gsz) {
        const BViewJob& vj = t.vjobs[j];
        t.items[vj.item].views_rw[vj.slot] = t.vrecs[j];
    }
    // tile rows of the new views, from the batch's own copy of the records
    const int64_t wave = gid >> 6, nwaves = gsz >> 6;
    __shared__ int64_t sh[kLdsJobs];
    const int64_t* rb = stage_table(sh, t.vjob_row_base, h.n_vjobs);
    for (int64_t r = wave; r < h.total_rows; r += nwaves) {
        int j = find_job(rb, h.n_vjobs, r);
        tile_row_words(t.vrecs[j], (int)(r - rb[j]), t.items[t.vjobs[j].item].gate);
    }
}

// Lanes are laid out per job in whole wavefronts (job bases are multiples of
// 64 and every wave runs the same number of iterations), as cull_group needs.
__global__ void k_batch_cull(BatchTables t) {
    const BatchHeader& h = *t.header;
    const int64_t gsz = (int64_t)gridDim.x * blockDim.x;
    __shared__ int64_t sh[kLdsJobs];
    const int64_t* lb = stage_table(sh, t.cjob_lane_base, h.n_cjobs);
    for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < h.total_cull; k += gsz) {
        int j = find_job(lb, h.n_cjobs, k);
        const BCullJob& cj = t.cjobs[j];
        const BItem& it = t.items[cj.item];
        const int64_t n = *it.f.n_act;
        const int64_t local = k - lb[j];
        const int64_t nch = (n + kChunk - 1) / kChunk;
        cull_group(it.box, n, it.f.p.eps, it.f.views, cj.s_begin, cj.ns, cj.p2, local, it.cull_rw,
                   local < nch * cj.p2);
    }
}

// One wavefront per flattened chunk (the item by a search in the LDS copy of
// the item chunk bases): chunks with a view bit in their item's fused range
// take the binary64 thick path, the others only write their outputs.  The
// hardware dispatcher hands chunks to free wavefronts, which balances the very
// uneven hot chunks; waves past the last chunk leave at once.
// Chunk `chunk` of item it (wave-uniform), below the item's active count n.
template <int MODE>
__device__ __forceinline__ void batch_chunk(const BItem& it, int64_t n, int64_t chunk, int lane) {
    // resident outputs: a chunk without a view to evaluate keeps its outputs
    if (it.f.delta && !((it.f.cull[chunk] | (it.f.cull_all ? ~0ull : 0ull)) & it.fuse_range)) return;
    const int64_t i = chunk * kChunk + lane;  // whole chunks: in bounds
    const uint32_t lin = it.f.act[i];
    const uint8_t seg = it.f.segb[i];
    if ((it.f.cull[chunk] | (it.f.cull_all ? ~0ull : 0ull)) & it.fuse_range)
        flush_counts(it.f.slots, chunk, fuse_chunk<MODE>(it.f, n, chunk, lane, lin, seg), lane);
    else
        flush_counts(it.f.slots, chunk, cold_chunk(it.f, n, chunk, lane, lin, seg), lane);
}

template <int MODE>
__global__ __launch_bounds__(512, 4) void k_batch_fuse(BatchTables t) {
    const BatchHeader& h = *t.header;
    __shared__ int64_t sh[kLdsJobs];
    const int64_t* ib = stage_table(sh, t.item_chunk_base, h.n_items + 1);
    const int lane = threadIdx.x & 63;
    const int64_t c = (int64_t)blockIdx.x * (blockDim.x >> 6) + wave_in_block();
    if (c >= h.total_chunks) return;
    const int j = wave_uniform(find_job(ib, h.n_items, c));
    const BItem& it = t.items[j];
    const int64_t n = *it.f.n_act;
    const int64_t chunk = wave_uniform((int)(c - ib[j]));  // chunks of a batch < 2^31
    if (chunk * kChunk >= n) return;
    batch_chunk<MODE>(it, n, chunk, lane);
}

// Persistent schedule: a fixed grid whose wavefronts pop descriptors (chunk
// ranges of one item, costliest items first) from an integer-atomic queue
// until it is empty; every wavefront leaves when a pop finds the queue
// exhausted, so the grid drains.  Each chunk is still done by one wavefront
// with the same device code, so the outputs are those of the other schedule.
template <int MODE>
__global__ __launch_bounds__(512, 4) void k_batch_fuse_queue(BatchTables t) {
    const BatchHeader& h = *t.header;
    const int lane = threadIdx.x & 63;
    const uint32_t nd = h.n_desc;
    for (;;) {
        uint32_t d = 0;
        if (lane == 0) d = atomicAdd(t.head, 1u);
        d = (uint32_t)wave_uniform((int)__shfl((int)d, 0));
        if (d >= nd) break;
        const BDesc ds = t.desc[d];
        const BItem& it = t.items[wave_uniform(ds.item)];
        const int64_t n = *it.f.n_act;
        for (int64_t chunk = ds.c0; chunk < (int64_t)ds.c1 && chunk * kChunk < n; ++chunk)
            batch_chunk<MODE>(it, n, wave_uniform((int)chunk), lane);
    }
}

// One wavefront per item: its partial count slots summed into its counts and
// statistics, and cleared.
__global__ void k_batch_counts(BatchTables t) {
    const BatchHeader& h = *t.header;
    const int lane = threadIdx.x & 63;
    const int64_t wave = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> 6;
    const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
    for (int64_t j = wave; j < h.n_items; j += nwaves) {
        const FuseArgs& f = t.items[j].f;
        uint64_t v[6];
        take_slots(f.slots, lane, v);
#pragma unroll
        for (int off = 32; off > 0; off >>= 1)
#pragma unroll
            for (int k = 0; k < 6; ++k) v[k] += __shfl_xor(v[k], off);
        if (lane == 0) {
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                const int64_t c = (int64_t)(v[k] + (f.delta ? (uint64_t)f.tot[k] : 0ull));
                f.counts[k] = c;
                if (f.tot) f.tot[k] = c;
            }
            f.stats[0] = (int64_t)v[3];
            f.stats[1] = (int64_t)v[4];
            f.stats[2] = (int64_t)v[5];
        }
    }
}

}  // namespace

hipError_t launch_batch_phase(const BatchTables& t, const BatchGrid& g, int phase, hipStream_t st) {
    if (phase == 0) hipLaunchKernelGGL(k_batch_prep, dim3(g.prep_blocks), dim3(256), 0, st, t);
    if (phase == 1) hipLaunchKernelGGL(k_batch_cull, dim3(g.cull_blocks), dim3(256), 0, st, t);
    if (phase == 2) {
        const dim3 gb(g.fuse_blocks), tb(g.fuse_threads);
        if (g.persistent) {
            if (g.mode == kThick)
                hipLaunchKernelGGL(k_batch_fuse_queue<kThick>, gb, tb, 0, st, t);
            else if (g.mode == kAnyThin)
                hipLaunchKernelGGL(k_batch_fuse_queue<kAnyThin>, gb, tb, 0, st, t);
            else
                hipLaunchKernelGGL(k_batch_fuse_queue<kAnyMode>, gb, tb, 0, st, t);
        } else if (g.mode == kThick) {
            hipLaunchKernelGGL(k_batch_fuse<kThick>, gb, tb, 0, st, t);
        } else if (g.mode == kAnyThin) {
            hipLaunchKernelGGL(k_batch_fuse<kAnyThin>, gb, tb, 0, st, t);
        } else {
            hipLaunchKernelGGL(k_batch_fuse<kAnyMode>, gb, tb, 0, st, t);
        }
    }
    if (phase == 3) hipLaunchKernelGGL(k_batch_counts, dim3(g.prep_blocks), dim3(256), 0, st, t);
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
