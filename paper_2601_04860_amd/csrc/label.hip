// Voxel-lookup labels: Eq. pass1 (Pass 1 of Alg. vox2surfel).
//
// Each point is mapped to its voxel with the same binary64 expression as the
// occupancy construction (so a point is never looked up in a voxel it was not
// voxelised into), and its label is the voxel's bit of the segmentation
// bitfield.  NaN and out-of-grid points get 0.  One lane per point; xyz is read
// as three consecutive floats per lane (a wavefront reads 768 contiguous bytes),
// the bitfield (dim^3 / 8 bytes) stays in L2 / the Infinity Cache.
#include "kernels.h"

namespace divas {

namespace {

__global__ void k_label(const float* __restrict__ xyz, int64_t n, DGrid g, const uint32_t* __restrict__ bits,
                        uint8_t* __restrict__ labels) {
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    uint32_t idx[3];
    bool ok = true;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        double x = (double)xyz[3 * i + k];
        double f = floor((x - g.origin[k]) / g.h);
        ok = ok && (f >= 0.0) && (f < (double)g.dim);
        idx[k] = ok ? (uint32_t)f : 0u;
    }
    uint8_t lab = 0;
    if (ok) {
        uint32_t lin = idx[0] | (idx[1] << g.log2dim) | (idx[2] << (2 * g.log2dim));
        lab = (uint8_t)((bits[lin >> 5] >> (lin & 31u)) & 1u);
    }
    labels[i] = lab;
}

}  // namespace

hipError_t launch_label(const float* xyz, int64_t n, const DGrid& g, const uint32_t* bits, uint8_t* labels,
                        hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_label, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, xyz, n, g, bits, labels);
    return hipGetLastError();
}

}  // namespace divas
