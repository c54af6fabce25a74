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
//
// The points of the session's own occupancy build can instead be labelled
// from the Morton codes that build kept (the same voxel rule, evaluated once):
// four codes per lane in one 16-byte load instead of twelve coordinates.
#include "kernels.h"

namespace divas {

namespace {

// The voxel of a point (ok = inside the grid and not NaN), its linear index
// and its coarse cell.
struct PointVoxel {
    bool ok;
    uint32_t lin, cell;
};

__device__ __forceinline__ PointVoxel point_voxel_of(float x, float y, float z, const DGrid& g, double inv_h) {
    const float p[3] = {x, y, z};
    uint32_t idx[3];
    bool ok = true;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const double f = voxel_floor_f(p[k], g.origin[k], g.h, inv_h);
        ok = ok & (f >= 0.0) & (f < (double)g.dim);  // NaN fails both
        idx[k] = ok ? (uint32_t)f : 0u;
    }
    PointVoxel v;
    v.ok = ok;
    v.lin = idx[0] | (idx[1] << g.log2dim) | (idx[2] << (2 * g.log2dim));
    v.cell = coarse_cell(g, idx[0], idx[1], idx[2]);
    return v;
}

// Labels of N points of one lane in two rounds of loads: the coarse counts of
// all of them together, then the bitfield words of those in a cell with a
// segmented voxel (the others read word 0, which stays cached), so a lane
// waits for two memory round trips whatever N is.
template <int N>
__device__ __forceinline__ void labels_of(const float (&x)[N], const float (&y)[N], const float (&z)[N], const DGrid& g,
                                          double inv_h, const uint32_t* __restrict__ bits,
                                          const uint32_t* __restrict__ coarse, uint8_t (&out)[N]) {
    PointVoxel v[N];
    uint32_t cc[N], w[N];
#pragma unroll
    for (int k = 0; k < N; ++k) v[k] = point_voxel_of(x[k], y[k], z[k], g, inv_h);
#pragma unroll
    for (int k = 0; k < N; ++k) cc[k] = coarse[v[k].ok ? v[k].cell : 0u];
#pragma unroll
    for (int k = 0; k < N; ++k) {
        v[k].ok = v[k].ok & (cc[k] != 0u);  // no segmented voxel in the cell: label 0
        w[k] = bits[v[k].ok ? v[k].lin >> 5 : 0u];
    }
#pragma unroll
    for (int k = 0; k < N; ++k) out[k] = v[k].ok ? (uint8_t)((w[k] >> (v[k].lin & 31u)) & 1u) : (uint8_t)0;
}

// Labels of N points of one lane from their Morton codes (0xFFFFFFFF: no
// voxel), in the same two rounds of loads.
template <int N>
__device__ __forceinline__ void labels_of_codes(const uint32_t (&code)[N], const DGrid& g,
                                                const uint32_t* __restrict__ bits,
                                                const uint32_t* __restrict__ coarse, uint8_t (&out)[N]) {
    bool ok[N];
    uint32_t lin[N], cc[N], w[N];
#pragma unroll
    for (int k = 0; k < N; ++k) {
        ok[k] = code[k] != 0xFFFFFFFFu;
        const uint32_t c = ok[k] ? code[k] : 0u;
        const uint32_t x = compact3(c), y = compact3(c >> 1), z = compact3(c >> 2);
        lin[k] = x | (y << g.log2dim) | (z << (2 * g.log2dim));
        cc[k] = coarse[ok[k] ? coarse_cell(g, x, y, z) : 0u];
    }
#pragma unroll
    for (int k = 0; k < N; ++k) {
        ok[k] = ok[k] & (cc[k] != 0u);
        w[k] = bits[ok[k] ? lin[k] >> 5 : 0u];
    }
#pragma unroll
    for (int k = 0; k < N; ++k) out[k] = ok[k] ? (uint8_t)((w[k] >> (lin[k] & 31u)) & 1u) : (uint8_t)0;
}

// Four points per lane from their codes (codes 16-byte, labels 4-byte aligned).
__global__ void k_label_codes4(const uint4* __restrict__ codes4, int64_t n4, DGrid g,
                               const uint32_t* __restrict__ bits, const uint32_t* __restrict__ coarse,
                               uchar4* __restrict__ labels4) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n4) return;
    const uint4 c = codes4[i];
    const uint32_t code[4] = {c.x, c.y, c.z, c.w};
    uint8_t l[4];
    labels_of_codes<4>(code, g, bits, coarse, l);
    labels4[i] = make_uchar4(l[0], l[1], l[2], l[3]);
}

// One point per lane from its code (any alignment).
__global__ void k_label_codes(const uint32_t* __restrict__ codes, int64_t n, DGrid g,
                              const uint32_t* __restrict__ bits, const uint32_t* __restrict__ coarse,
                              uint8_t* __restrict__ labels) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint32_t code[1] = {codes[i]};
    uint8_t l[1];
    labels_of_codes<1>(code, g, bits, coarse, l);
    labels[i] = l[0];
}

// One lane per point (any alignment).
__global__ void k_label(const float* __restrict__ xyz, int64_t n, DGrid g, double inv_h, const uint32_t* __restrict__ bits,
                        const uint32_t* __restrict__ coarse, uint8_t* __restrict__ labels) {
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float x[1] = {xyz[3 * i]}, y[1] = {xyz[3 * i + 1]}, z[1] = {xyz[3 * i + 2]};
    uint8_t l[1];
    labels_of<1>(x, y, z, g, inv_h, bits, coarse, l);
    labels[i] = l[0];
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
    const float x[4] = {a.x, a.w, b.z, c.y}, y[4] = {a.y, b.x, b.w, c.z}, z[4] = {a.z, b.y, c.x, c.w};
    uint8_t l[4];
    labels_of<4>(x, y, z, g, inv_h, bits, coarse, l);
    labels4[i] = make_uchar4(l[0], l[1], l[2], l[3]);
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

hipError_t launch_label_codes(const uint32_t* codes, int64_t n, const DGrid& g, const uint32_t* bits,
                              const uint32_t* coarse, uint8_t* labels, hipStream_t st, PhaseEvents ev) {
    if (n <= 0) {
        record_phase_events(ev, st);
        return hipSuccess;
    }
    int64_t head = 0;
    if (((uintptr_t)codes & 15u) == 0 && ((uintptr_t)labels & 3u) == 0) {
        const int64_t n4 = n / 4;
        head = n4 * 4;
        if (n4 > 0) {
            launch_timed(k_label_codes4, dim3((unsigned)((n4 + 255) / 256)), dim3(256), 0, st, ev.start,
                         head < n ? nullptr : ev.stop, (const uint4*)codes, n4, g, bits, coarse, (uchar4*)labels);
            ev.start = nullptr;
        }
    }
    if (head < n)
        launch_timed(k_label_codes, dim3((unsigned)((n - head + 255) / 256)), dim3(256), 0, st, ev.start, ev.stop,
                     codes + head, n - head, g, bits, coarse, labels + head);
    return hipGetLastError();
}

}  // namespace divas
