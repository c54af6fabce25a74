// Depth-weighted voxel fusion on CDNA4 (gfx950).
//
// Alg. gs-fusion with Eqs. planar-to-ray, seethrough, asym-gate, tightening,
// gs-spatial, gs-depthweight and vmask, followed by Eq. compact-fusion and the
// consensus threshold (k_fuse_all); with the thin-structure call of Alg.
// gs-thin or Alg. nerf-thin, k_fuse_coop.
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
//   * Blocks are remapped so that each XCD takes runs of consecutive chunks
//     (spatially coherent view reads share that XCD's L2).
#include "fuse_core.h"

#include <algorithm>

namespace divas {

namespace {

constexpr int kWaves = kBlock / 64;
constexpr int kXcdRun = 16;  // blocks per XCD run of the fusion launch

// ------------------------------------------------------------ culling
// A block covers 64 chunks (a lane each); its wavefronts take the views of
// [s_begin, s_begin + ns) in turn, so the view is wave-uniform: its record is
// read through the scalar cache and each lane loads only its chunk's box and
// the hot-tile words.  The view bits meet in LDS and the first wavefront
// writes the chunks' cull words (bits outside the range kept).
constexpr int kCullWaves = 16;
__global__ __launch_bounds__(64 * kCullWaves) void k_cull(const ChunkBox* __restrict__ box,
                                                          const int64_t* __restrict__ n_act, double eps,
                                                          const DView* __restrict__ views, int32_t s_begin, int32_t ns,
                                                          uint64_t* __restrict__ cull) {
    __shared__ unsigned long long bits[64];
    const int lane = threadIdx.x & 63;
    const int w = wave_in_block(), nw = (int)(blockDim.x >> 6);
    const int64_t chunk = (int64_t)blockIdx.x * 64 + lane;
    const int64_t n = *n_act;
    const bool in = chunk * kChunk < n;
    if (w == 0) bits[lane] = 0ull;
    __syncthreads();
    for (int k = w; k < ns; k += nw) {  // uniform per wavefront
        const int s = s_begin + k;
        if (in && cull_chunk(box + chunk, eps, views[s])) atomicOr(&bits[lane], 1ull << s);
    }
    __syncthreads();
    if (w == 0 && in) {
        const uint64_t range = (ns >= 64 ? ~0ull : ((1ull << ns) - 1ull)) << s_begin;
        cull[chunk] = (cull[chunk] & ~range) | ((uint64_t)bits[lane] & range);
    }
}

// ------------------------------------------------------------ fusion kernels
// All chunks in one launch, one wavefront per chunk: a chunk with a view bit
// in the fused range takes the binary64 thick path over those views, the
// others only write their outputs (from the resident accumulators or from
// zero).  The hardware dispatcher hands chunks to free wavefronts as earlier
// ones finish, which balances the very uneven cost of hot chunks (1 to 64
// views, most without a sample past the mask gate).
//
// The lane's active-list entry and segmentation flag are loaded together with
// the count and the cull word (the active list and the flags are allocated in
// whole chunks): the launch is bound by dependent memory round trips, and
// this removes one from every hot chunk.
//
// Blocks are spread over the XCDs in runs: the hardware hands consecutive
// blocks to the 8 XCDs in turn, and block b is remapped so that each XCD
// takes runs of kXcdRun consecutive blocks (4 kXcdRun chunks).  A run is a
// compact region of the scene whose views' pixels share that XCD's L2, while
// the runs of one object still spread over every XCD.
template <int MODE>
__global__ __launch_bounds__(kBlock, 4) void k_fuse_all(FuseArgs a) {
    const int lane = threadIdx.x & 63;
    const int64_t bq = blockIdx.x >> 3, bx = blockIdx.x & 7;
    const int64_t lb = ((bq / kXcdRun) * 8 + bx) * kXcdRun + (bq % kXcdRun);
    const int64_t chunk = lb * kWaves + wave_in_block();
    if (chunk * kChunk >= a.cap) return;  // past the allocation (uniform)
    // resident outputs: a chunk without a view to evaluate keeps its outputs
    if (a.delta && !((a.cull[chunk] | (a.cull_all ? ~0ull : 0ull)) & view_range(a.s_begin, a.s_end))) return;
    const int64_t i = chunk * kChunk + lane;
    const uint32_t lin = a.act[i];
    const uint8_t seg = a.segb[i];
    const uint64_t word = a.cull[chunk] | (a.cull_all ? ~0ull : 0ull);
    const int64_t n = *a.n_act;
    if (chunk * kChunk >= n) return;
    if (word & view_range(a.s_begin, a.s_end))
        flush_counts(a.slots, chunk, fuse_chunk<MODE>(a, n, chunk, lane, lin, seg), lane);
    else
        flush_counts(a.slots, chunk, cold_chunk(a, n, chunk, lane, lin, seg), lane);
}

// Thin paths: one block per chunk, its wavefronts sharing out the footprints
// eligible for the thin sweep (fuse_chunk with COOP); wavefront 0 writes the
// outputs and counts.  The block size is chosen per launch so that a small
// scene still fills the chip (a footprint of a zoomed view holds about a
// thousand pixels, and a whole wavefront sweeps it).
constexpr int kThinMaxWaves = 8;
template <int MODE>
__global__ __launch_bounds__(64 * kThinMaxWaves) void k_fuse_coop(FuseArgs a) {
    const int lane = threadIdx.x & 63;
    const int64_t chunk = blockIdx.x;
    if (chunk * kChunk >= a.cap) return;  // uniform across the block
    const uint64_t word = a.cull[chunk] | (a.cull_all ? ~0ull : 0ull);
    const bool hot = (word & view_range(a.s_begin, a.s_end)) != 0;
    if (a.delta && !hot) return;  // resident outputs: nothing changes
    const int64_t i = chunk * kChunk + lane;
    const uint32_t lin = a.act[i];
    const uint8_t seg = a.segb[i];
    const int64_t n = *a.n_act;
    if (chunk * kChunk >= n) return;
    if (hot) {
        const Counts3 c = fuse_chunk<MODE, true>(a, n, chunk, lane, lin, seg);
        if (wave_in_block() == 0) flush_counts(a.slots, chunk, c, lane);
    } else if (wave_in_block() == 0) {
        flush_counts(a.slots, chunk, cold_chunk(a, n, chunk, lane, lin, seg), lane);
    }
}

// One wavefront: sums the partial count slots into counts[0..2] and
// stats[0..2], clears them; with tot, keeps the running totals (delta: the
// slots hold changes, added to the totals).
__global__ void k_count_reduce(int64_t* __restrict__ slots, int64_t* __restrict__ counts,
                               int64_t* __restrict__ stats, int64_t* __restrict__ tot, int delta) {
    const int lane = threadIdx.x & 63;
    uint64_t v[6];
    take_slots(slots, lane, v);
#pragma unroll
    for (int off = 32; off > 0; off >>= 1)
#pragma unroll
        for (int k = 0; k < 6; ++k) v[k] += __shfl_xor(v[k], off);
    if (lane == 0) {
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const int64_t c = (int64_t)(v[k] + (delta ? (uint64_t)tot[k] : 0ull));
            counts[k] = c;
            if (tot) tot[k] = c;
        }
        stats[0] = (int64_t)v[3];
        stats[1] = (int64_t)v[4];
        stats[2] = (int64_t)v[5];
    }
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

hipError_t launch_cull(const ChunkBox* chunk_box, const int64_t* n_act, int64_t cap, const DGrid& g, double eps,
                       const DView* views, int32_t s_begin, int32_t s_end, uint64_t* cull, hipStream_t st,
                       PhaseEvents ev) {
    int ns = s_end - s_begin;
    if (ns <= 0 || cap <= 0) {
        record_phase_events(ev, st);
        return hipSuccess;
    }
    const int64_t nchunks = (cap + kChunk - 1) / kChunk;
    const unsigned waves = (unsigned)std::min(ns, kCullWaves);
    launch_timed(k_cull, dim3((unsigned)((nchunks + 63) / 64)), dim3(64 * waves), 0, st, ev.start, ev.stop, chunk_box,
                 n_act, eps, views, s_begin, ns, cull);
    return hipGetLastError();
}

hipError_t launch_fuse(const FuseArgs& a, bool any_nsamp, hipStream_t st, PhaseEvents ev) {
    if (a.cap <= 0) {
        record_phase_events(ev, st);
        return hipSuccess;
    }
    const int64_t nchunks = (a.cap + kChunk - 1) / kChunk;
    const int64_t nblocks = (nchunks + kWaves - 1) / kWaves;
    constexpr int64_t kRuns = 8 * kXcdRun;  // whole runs on every XCD; the extra blocks leave at once
    const dim3 grid((unsigned)((nblocks + kRuns - 1) / kRuns * kRuns)), block(kBlock);
    if (a.p.thin && !a.p.differentiable) {
        // wavefronts per chunk: enough blocks x waves to fill the chip
        int waves = 1;
        while (waves < kThinMaxWaves && nchunks * waves < 4096) waves <<= 1;
        const dim3 tgrid((unsigned)nchunks), tblock(64 * waves);
        if (a.p.variant == kVariantNerf)
            launch_timed(k_fuse_coop<kNerfThin>, tgrid, tblock, 0, st, ev.start, ev.stop, a);
        else
            launch_timed(k_fuse_coop<kThin>, tgrid, tblock, 0, st, ev.start, ev.stop, a);
        return hipGetLastError();
    }
    if (a.p.differentiable)
        launch_timed(k_fuse_all<kDiff>, grid, block, 0, st, ev.start, ev.stop, a);
    else if (a.p.variant == kVariantNerf)
        launch_timed(k_fuse_all<kNerf>, grid, block, 0, st, ev.start, ev.stop, a);
    else if (any_nsamp)
        launch_timed(k_fuse_all<kThickNsamp>, grid, block, 0, st, ev.start, ev.stop, a);
    else
        launch_timed(k_fuse_all<kThick>, grid, block, 0, st, ev.start, ev.stop, a);
    return hipGetLastError();
}

hipError_t launch_count_reduce(int64_t* slots, int64_t* counts, int64_t* stats, int64_t* tot, int delta,
                               hipStream_t st) {
    hipLaunchKernelGGL(k_count_reduce, dim3(1), dim3(64), 0, st, slots, counts, stats, tot, delta);
    return hipGetLastError();
}

}  // namespace divas
