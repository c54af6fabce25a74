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
#include "kernels.h"
#include "sample.h"

namespace divas {

namespace {

constexpr int kWaves = kBlock / 64;

// ------------------------------------------------------------ culling
__global__ void k_cull(const uint16_t* __restrict__ box, const int64_t* __restrict__ n_act, DGrid g, double eps,
                       const DView* __restrict__ views, int32_t s_begin, int32_t ns, uint8_t* __restrict__ cull,
                       int32_t stride) {
    int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    int64_t chunk = t / ns;
    int s = s_begin + (int)(t - chunk * ns);
    int64_t n = *n_act;
    if (chunk * kChunk >= n) return;
    const DView& v = views[s];
    const uint16_t* b = box + chunk * 8;
    float lo[3], hi[3];
    for (int k = 0; k < 3; ++k) {
        lo[k] = (float)(g.origin[k] + ((double)b[k] + 0.5) * g.h);
        hi[k] = (float)(g.origin[k] + ((double)b[3 + k] + 0.5) * g.h);
    }
    float umin = INFINITY, umax = -INFINITY, vmin = INFINITY, vmax = -INFINITY;
    float zmin = INFINITY, zmax = -INFINITY, rmax = 0.f, dist = 0.f;
    for (int j = 0; j < 8; ++j) {
        float p0 = (j & 1) ? hi[0] : lo[0], p1 = (j & 2) ? hi[1] : lo[1], p2 = (j & 4) ? hi[2] : lo[2];
        float d0 = p0 - v.fo[0], d1 = p1 - v.fo[1], d2 = p2 - v.fo[2];
        float qx = v.fR[0] * d0 + v.fR[3] * d1 + v.fR[6] * d2;
        float qy = v.fR[1] * d0 + v.fR[4] * d1 + v.fR[7] * d2;
        float qz = v.fR[2] * d0 + v.fR[5] * d1 + v.fR[8] * d2;
        zmin = fminf(zmin, qz);
        zmax = fmaxf(zmax, qz);
        dist = fmaxf(dist, fabsf(d0) + fabsf(d1) + fabsf(d2));
        if (qz > 0.f) {
            float iz = 1.0f / qz;
            float un = qx * iz, vn = qy * iz;
            rmax = fmaxf(rmax, fabsf(un) + fabsf(vn));
            float u = v.ffx * un + v.fcx, vv = v.ffy * vn + v.fcy;
            umin = fminf(umin, u);
            umax = fmaxf(umax, u);
            vmin = fminf(vmin, vv);
            vmax = fmaxf(vmax, vv);
        }
    }
    uint8_t hot;
    // float error of a camera coordinate is below 8 ulp of |p - o|_1
    float qerr = 8.0f * 1.2e-7f * dist + 1e-6f;
    if (zmax < (float)eps - qerr) {
        hot = 0;  // every voxel centre of the chunk is behind the camera
    } else if (zmin < 16.0f * qerr + 1e-3f) {
        hot = 1;  // the box reaches the camera plane: no bound on the projection
    } else {
        // conservative pixel rectangle: f32 rounding of u is below
        // f * (1 + |u_n| + |v_n|) * qerr / z_min, padded by one whole pixel
        float pad = 1.0f + fmaxf(v.ffx, v.ffy) * (1.0f + rmax) * 2.0f * qerr / zmin;
        int x0 = (int)floorf(umin - pad), x1 = (int)floorf(umax + pad);
        int y0 = (int)floorf(vmin - pad), y1 = (int)floorf(vmax + pad);
        x0 = max(x0, 0);
        y0 = max(y0, 0);
        x1 = min(x1, v.W - 1);
        y1 = min(y1, v.H - 1);
        if (x0 > x1 || y0 > y1) {
            hot = 0;
        } else {
            int tx0 = x0 / kTile, tx1 = x1 / kTile, ty0 = y0 / kTile, ty1 = y1 / kTile;
            if ((int64_t)(tx1 - tx0 + 1) * (ty1 - ty0 + 1) > 1024) {
                hot = 1;
            } else {
                hot = 0;
                for (int ty = ty0; ty <= ty1 && !hot; ++ty)
                    for (int tx = tx0; tx <= tx1; ++tx)
                        if (v.tiles[(size_t)ty * v.tw + tx]) {
                            hot = 1;
                            break;
                        }
            }
        }
    }
    cull[chunk * stride + s] = hot;
}

// ------------------------------------------------------------ fusion kernel
__global__ __launch_bounds__(kBlock) void k_fuse(FuseArgs a) {
    // XCD-aware remap: hardware block b runs on XCD (b mod 8); give each XCD a
    // contiguous range of logical blocks.
    const unsigned G = gridDim.x;
    const unsigned b = blockIdx.x;
    const unsigned per = G / 8u;
    const unsigned lb = (b % 8u) * per + b / 8u;
    const int wave = threadIdx.x >> 6;
    const int lane = threadIdx.x & 63;
    const int64_t n = *a.n_act;
    const int64_t chunk = (int64_t)lb * kWaves + wave;
    if (chunk * kChunk >= n) return;
    const int64_t i = chunk * kChunk + lane;
    const bool live = i < n;
    const uint32_t lin = live ? a.act[i] : 0u;
    const uint32_t msk = (uint32_t)a.g.dim - 1u;
    uint32_t iv[3] = {lin & msk, (lin >> a.g.log2dim) & msk, lin >> (2 * a.g.log2dim)};
    double c[3];
    for (int k = 0; k < 3; ++k) c[k] = a.g.origin[k] + ((double)iv[k] + 0.5) * a.g.h;
    double Wx = 0.0, Zx = 0.0;
    uint64_t vm = 0;
    if (a.load_acc && live) {
        Wx = a.W[i];
        Zx = a.Z[i];
        vm = a.vraw[i];
    }
    const uint8_t* cullrow = a.cull + chunk * a.cull_stride;
    for (int s = a.s_begin; s < a.s_end; ++s) {
        if (!cullrow[s]) continue;  // uniform: no voxel of this chunk can vote in view s
        if (!live) continue;
        const DView& v = a.views[s];
        if (a.p.differentiable) {
            double sw, m;
            if (diff_sample(v, a.g, a.p, c, &sw, &m)) {
                Wx += m * sw;
                Zx += sw;
                vm |= (uint64_t)1 << s;
            }
        } else {
            double w, m;
            if (thick_sample(v, a.g, a.p, iv, c, &w, &m)) {
                Wx += m * w;
                Zx += w;
                vm |= (uint64_t)1 << s;
            }
        }
    }
    // compact fusion, consensus threshold, outputs
    double P64 = Zx > a.p.eps ? Wx / Zx : 0.0;
    bool seg = live && (P64 >= a.p.tau_cons);
    bool flag = live && (fabs(P64 - a.p.tau_cons) <= 1e-5);
    if (live) {
        a.P[i] = (float)P64;
        a.vout[i] = seg ? vm : 0;
        if (a.store_acc) {
            a.W[i] = Wx;
            a.Z[i] = Zx;
            a.vraw[i] = vm;
        }
        uint32_t word = a.bits[lin >> 5];
        uint32_t bit = 1u << (lin & 31u);
        bool old = (word & bit) != 0;
        if (seg && !old) atomicOr(&a.bits[lin >> 5], bit);
        if (!seg && old) atomicAnd(&a.bits[lin >> 5], ~bit);
    }
    uint64_t bseg = __ballot(seg);
    uint64_t bflag = __ballot(flag);
    uint64_t votes = live ? (uint64_t)__popcll(vm) : 0;
    for (int off = 32; off > 0; off >>= 1) votes += __shfl_xor(votes, off);
    if (lane == 0) {
        if (bseg) atomicAdd((unsigned long long*)&a.counts[0], (unsigned long long)__popcll(bseg));
        if (bflag) atomicAdd((unsigned long long*)&a.counts[1], (unsigned long long)__popcll(bflag));
        if (votes) atomicAdd((unsigned long long*)&a.counts[2], (unsigned long long)votes);
    }
}

}  // namespace

hipError_t launch_cull(const uint16_t* chunk_box, const int64_t* n_act, int64_t cap, const DGrid& g, double eps,
                       const DView* views, int32_t s_begin, int32_t s_end, uint8_t* cull, int32_t cull_stride,
                       hipStream_t st) {
    int ns = s_end - s_begin;
    if (ns <= 0 || cap <= 0) return hipSuccess;
    int64_t nchunks = (cap + kChunk - 1) / kChunk;
    int64_t lanes = nchunks * ns;
    hipLaunchKernelGGL(k_cull, dim3((unsigned)((lanes + 255) / 256)), dim3(256), 0, st, chunk_box, n_act, g, eps, views,
                       s_begin, ns, cull, cull_stride);
    return hipGetLastError();
}

hipError_t launch_fuse(const FuseArgs& a, hipStream_t st) {
    if (a.cap <= 0) return hipSuccess;
    int64_t nchunks = (a.cap + kChunk - 1) / kChunk;
    int64_t nblocks = (nchunks + kWaves - 1) / kWaves;
    nblocks = (nblocks + 7) / 8 * 8;  // whole XCD groups for the remap
    hipLaunchKernelGGL(k_fuse, dim3((unsigned)nblocks), dim3(kBlock), 0, st, a);
    return hipGetLastError();
}

}  // namespace divas
