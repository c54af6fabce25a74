// Several target objects of one scene fused together (the multi-object form of
// the batched path).  The targets share the scene's active list and chunk
// boxes, the views' cameras and depth planes; only the mask planes differ.
// The 2DGS thick path decides everything but the mask vote from the camera
// and the depths: the entry gate reads the mask, the vote adds m w.  So per
// (voxel, view) sample the projection, the depth gathers, the depth and
// spatial gates and the weight are evaluated once, and every target whose gate
// bit is set adds its own mask value.  Each target keeps its own accumulators
// (registers of the lane), threshold, segmentation and outputs, computed by
// the same operations in the same view order as a fusion of that target
// alone, so its results are bit-identical to it.
//
//   k_cull_targets    the chunk rectangle of a view is projected once and
//                     tested against every target's hot tiles;
//   k_fuse_targets    one wavefront per chunk of the shared active list;
//   k_counts_targets  one wavefront per target sums its count slots.
#include "targets.h"

#include <algorithm>

#include "fuse_core.h"

namespace divas {

namespace {

constexpr int kWaves = kBlock / 64;
constexpr int kXcdRun = 16;  // blocks per XCD run (as the single-target fusion)
constexpr int kCullWaves = 16;

__global__ __launch_bounds__(64 * kCullWaves) void k_cull_targets(TargetCull tc) {
    __shared__ unsigned long long bits[kMaxTargets][64];
    const int lane = threadIdx.x & 63;
    const int w = wave_in_block(), nw = (int)(blockDim.x >> 6);
    const int64_t chunk = (int64_t)blockIdx.x * 64 + lane;
    const int64_t n = *tc.n_act;
    const bool in = chunk * kChunk < n;
    if (w == 0)
        for (int t = 0; t < kMaxTargets; ++t) bits[t][lane] = 0ull;
    __syncthreads();
    for (int k = w; k < tc.ns; k += nw) {  // uniform per wavefront
        const int s = tc.s_begin + k;
        if (in) {
            const CullRect r = cull_rect(tc.box + chunk, tc.eps, tc.views[0][s]);
            for (int t = 0; t < tc.n; ++t)
                if (cull_tiles(r, tc.views[t][s])) atomicOr(&bits[t][lane], 1ull << s);
        }
    }
    __syncthreads();
    if (w == 0 && in) {
        const uint64_t range = (tc.ns >= 64 ? ~0ull : ((1ull << tc.ns) - 1ull)) << tc.s_begin;
        for (int t = 0; t < tc.n; ++t)
            tc.cull[t][chunk] = (tc.cull[t][chunk] & ~range) | ((uint64_t)bits[t][lane] & range);
    }
}

// One wavefront per chunk (XCD runs as in the single-target fusion).  Chunks
// without a view bit of any target write every target's outputs from zero.
template <int NT, bool NS>
__global__ __launch_bounds__(kBlock, 2) void k_fuse_targets(const TargetArgs* __restrict__ tap) {
    const TargetArgs& ta = *tap;
    const int lane = threadIdx.x & 63;
    const int64_t bq = blockIdx.x >> 3, bx = blockIdx.x & 7;
    const int64_t lb = ((bq / kXcdRun) * 8 + bx) * kXcdRun + (bq % kXcdRun);
    const int64_t chunk = lb * kWaves + wave_in_block();
    const FuseArgs& a0 = ta.f[0];
    if (chunk * kChunk >= a0.cap) return;  // past the allocation (uniform)
    const int64_t i = chunk * kChunk + lane;
    const uint32_t lin_in = a0.act[i];
    const int64_t n = *a0.n_act;
    if (chunk * kChunk >= n) return;
    const uint64_t range = view_range(a0.s_begin, a0.s_end);
    uint64_t word[NT], any = 0;
    uint8_t seg[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) {
        word[t] = t < ta.n ? ta.f[t].cull[chunk] & range : 0ull;
        seg[t] = t < ta.n ? ta.f[t].segb[i] : (uint8_t)0;
        any |= word[t];
    }
    if (!any) {
        for (int t = 0; t < ta.n; ++t)
            flush_counts(ta.f[t].slots, chunk, cold_chunk(ta.f[t], n, chunk, lane, lin_in, seg[t]), lane);
        return;
    }
    const bool live = i < n;
    const uint32_t lin = live ? lin_in : 0u;
    uint32_t iv[3];
    double c[3];
    voxel_centre(a0.g, lin, iv, c);
    double Wx[NT], Zx[NT];
    uint64_t vm[NT], gathered[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) {
        Wx[t] = 0.0;
        Zx[t] = 0.0;
        vm[t] = 0;
        gathered[t] = 0;
    }
    uint64_t todo = any;
    while (todo) {  // uniform, views in increasing order
        const int s = __ffsll((unsigned long long)todo) - 1;
        todo &= todo - 1;
        const DView& v = a0.views[s];  // camera and depth planes shared by the targets
        const SampleHead hd = sample_proj(v, c, a0.p.eps);
        // the gate bytes of the targets with the view bit, all issued before
        // the first is used
        uint32_t byte[NT];
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            byte[t] = 0u;
            if (t < ta.n && ((word[t] >> s) & 1ull)) byte[t] = gate_byte(ta.f[t].views[s], hd);  // uniform
        }
        bool gate[NT];
        bool pass = false;
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            gate[t] = live && hd.in && ((byte[t] >> (hd.px & 7)) & 1u);
            pass |= gate[t];
        }
        PixelSample ps{};
        if (pass) ps = sample_load(v, hd);
        const bool ns = NS && v.nsamp != nullptr;  // uniform
        const bool cand = pass && depth_candidate(v, a0.g, a0.p, hd.qz, ps, ns);
        bool layered = false;
        double E = 0.0;
        if (ns) footprint_stats_wave(v, a0.g, iv, a0.p.eps, cand, hd.px, hd.py, lane, &layered, &E);
        double w = 0.0, m0 = 0.0;
        bool ok = false;
        if (cand) ok = sample_decide(v, a0.g, a0.p, c, hd, ps, layered, E, &w, &m0);
        const size_t pix = (size_t)hd.py * (size_t)v.W + (size_t)hd.px;  // (0, 0) out of frame
        // every target's mask value at the pixel, loaded together by the
        // lanes that vote for some target
        float mt[NT];
#pragma unroll
        for (int t = 0; t < NT; ++t) mt[t] = 0.0f;
        if (ok) {
#pragma unroll
            for (int t = 0; t < NT; ++t) mt[t] = ldg(ta.f[t < ta.n ? t : 0].views[s].mask + pix);
        }
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            if (t < ta.n) gathered[t] += (uint64_t)__popcll(__ballot(gate[t]));
            if (ok && gate[t]) {
                Wx[t] += (double)mt[t] * w;
                Zx[t] += w;
                vm[t] |= (uint64_t)1 << s;
            }
        }
    }
#pragma unroll
    for (int t = 0; t < NT; ++t) {
        if (t >= ta.n) break;
        const FuseArgs& a = ta.f[t];
        Counts3 cn;
        if (word[t]) {
            cn = finalize_chunk(a, i, live, lin, Wx[t], Zx[t], vm[t], a.store_acc != 0, live ? seg[t] : (uint8_t)0);
            cn.hot_chunks = 1;
            cn.hot_pairs = (uint64_t)__popcll(word[t]);
            cn.gathered = gathered[t];
        } else {
            cn = cold_chunk(a, n, chunk, lane, lin_in, seg[t]);
        }
        flush_counts(a.slots, chunk, cn, lane);
    }
}

// Wavefront t sums target t's partial count slots into its counts and
// statistics, and clears them.
__global__ void k_counts_targets(const TargetArgs* __restrict__ tap) {
    const TargetArgs& ta = *tap;
    const int lane = threadIdx.x & 63;
    const int t = wave_in_block();
    if (t >= ta.n) return;
    const FuseArgs& f = ta.f[t];
    uint64_t v[6];
    take_slots(f.slots, lane, v);
#pragma unroll
    for (int off = 32; off > 0; off >>= 1)
#pragma unroll
        for (int k = 0; k < 6; ++k) v[k] += __shfl_xor(v[k], off);
    if (lane == 0) {
        f.counts[0] = (int64_t)v[0];
        f.counts[1] = (int64_t)v[1];
        f.counts[2] = (int64_t)v[2];
        f.stats[0] = (int64_t)v[3];
        f.stats[1] = (int64_t)v[4];
        f.stats[2] = (int64_t)v[5];
    }
}

template <bool NS>
void launch_fuse_nt(const TargetArgs* ta, int n, dim3 grid, hipStream_t st) {
    if (n <= 2)
        hipLaunchKernelGGL((k_fuse_targets<2, NS>), grid, dim3(kBlock), 0, st, ta);
    else if (n <= 4)
        hipLaunchKernelGGL((k_fuse_targets<4, NS>), grid, dim3(kBlock), 0, st, ta);
    else
        hipLaunchKernelGGL((k_fuse_targets<8, NS>), grid, dim3(kBlock), 0, st, ta);
}

}  // namespace

hipError_t launch_cull_targets(const TargetCull& tc, int64_t cap, hipStream_t st) {
    if (tc.ns <= 0 || cap <= 0) return hipSuccess;
    const int64_t nchunks = (cap + kChunk - 1) / kChunk;
    const unsigned waves = (unsigned)std::min(tc.ns, kCullWaves);
    hipLaunchKernelGGL(k_cull_targets, dim3((unsigned)((nchunks + 63) / 64)), dim3(64 * waves), 0, st, tc);
    return hipGetLastError();
}

hipError_t launch_fuse_targets(const TargetArgs* ta_dev, int n_targets, int64_t cap, bool any_nsamp,
                               hipStream_t st) {
    if (cap > 0) {
        const int64_t nchunks = (cap + kChunk - 1) / kChunk;
        const int64_t nblocks = (nchunks + kWaves - 1) / kWaves;
        constexpr int64_t kRuns = 8 * kXcdRun;
        const dim3 grid((unsigned)((nblocks + kRuns - 1) / kRuns * kRuns));
        if (any_nsamp)
            launch_fuse_nt<true>(ta_dev, n_targets, grid, st);
        else
            launch_fuse_nt<false>(ta_dev, n_targets, grid, st);
    }
    hipLaunchKernelGGL(k_counts_targets, dim3(1), dim3(64 * kMaxTargets), 0, st, ta_dev);
    return hipGetLastError();
}

}  // namespace divas
