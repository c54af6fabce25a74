// Voxel-lookup labels: Eq. pass1 (Pass 1 of Alg. vox2surfel).
//
// Each point is mapped to its voxel with the same binary64 expression as the
// occupancy construction (so a point is never looked up in a voxel it was not
// voxelised into), and its label is the voxel's bit of the segmentation
// bitfield; a point whose coarse cell holds no segmented voxel is answered
// from the small per-cell count table without touching the bitfield.  NaN and
// out-of-grid points get 0.  Four consecutive points per lane
// (three 16-byte xyz loads, four lookups in flight, one 4-byte store) when the
// buffers are aligned for it, else one lane per point; the bitfield (dim^3 / 8
// bytes) stays in L2 / the Infinity Cache.
#include "kernels.h"

namespace divas {

namespace {

__device__ __forceinline__ uint8_t label_of(float x, float y, float z, const DGrid& g, double inv_h,
                                            const uint32_t* __restrict__ bits, const uint32_t* __restrict__ coarse) {
    const double p[3] = {(double)x, (double)y, (double)z};
    uint32_t idx[3];
    bool ok = true;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const double f = voxel_floor(p[k] - g.origin[k], g.h, inv_h);
        ok = ok && (f >= 0.0) && (f < (double)g.dim);
        idx[k] = ok ? (uint32_t)f : 0u;
    }
    if (!ok) return 0;
    if (coarse[coarse_cell(g, idx[0], idx[1], idx[2])] == 0u) return 0;  // no segmented voxel in the cell
    uint32_t lin = idx[0] | (idx[1] << g.log2dim) | (idx[2] << (2 * g.log2dim));
    return (uint8_t)((bits[lin >> 5] >> (lin & 31u)) & 1u);
}

// One lane per point (any alignment).
__global__ void k_label(const float* __restrict__ xyz, int64_t n, DGrid g, double inv_h, const uint32_t* __restrict__ bits,
                        const uint32_t* __restrict__ coarse, uint8_t* __restrict__ labels) {
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    labels[i] = label_of(xyz[3 * i], xyz[3 * i + 1], xyz[3 * i + 2], g, inv_h, bits, coarse);
}

// Four consecutive points per lane: three 16-byte loads of xyz, four bitfield
// lookups in flight, one 4-byte label store (xyz 16-byte and labels 4-byte
// aligned; points [0, 4 * n4)).
__global__ void k_label4(const float4* __restrict__ xyz4, int64_t n4, DGrid g, double inv_h,
                         const uint32_t* __restrict__ bits,
                         const uint32_t* __restrict__ coarse, uchar4* __restrict__ labels4) {
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n4) return;
    const float4 a = xyz4[3 * i], b = xyz4[3 * i + 1], c = xyz4[3 * i + 2];
    uchar4 l;
    l.x = label_of(a.x, a.y, a.z, g, inv_h, bits, coarse);
    l.y = label_of(a.w, b.x, b.y, g, inv_h, bits, coarse);
    l.z = label_of(b.z, b.w, c.x, g, inv_h, bits, coarse);
    l.w = label_of(c.y, c.z, c.w, g, inv_h, bits, coarse);
    labels4[i] = l;
}

}  // namespace

hipError_t launch_label(const float* xyz, int64_t n, const DGrid& g, const uint32_t* bits, const uint32_t* coarse,
                        uint8_t* labels, hipStream_t st, PhaseEvents ev) {
    if (n <= 0) {
        record_phase_events(ev, st);
        return hipSuccess;
    }
    const double inv_h = 1.0 / g.h;  // correctly rounded on the host as on the device
    int64_t head = 0;
    if (((uintptr_t)xyz & 15u) == 0 && ((uintptr_t)labels & 3u) == 0) {
        const int64_t n4 = n / 4;
        head = n4 * 4;
        if (n4 > 0) {
            launch_timed(k_label4, dim3((unsigned)((n4 + 255) / 256)), dim3(256), 0, st, ev.start,
                         head < n ? nullptr : ev.stop, (const float4*)xyz, n4, g, inv_h, bits, coarse,
                         (uchar4*)labels);
            ev.start = nullptr;
        }
    }
    if (head < n)
        launch_timed(k_label, dim3((unsigned)((n - head + 255) / 256)), dim3(256), 0, st, ev.start, ev.stop,
                     xyz + 3 * head, n - head, g, inv_h, bits, coarse, labels + head);
    return hipGetLastError();
}

}  // namespace divas
