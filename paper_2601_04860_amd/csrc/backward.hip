// Reverse mode of the differentiable fusion (soft depth test on mask logits).
//
// With P = W / Z and one vote of voxel x in view i contributing m s w to W and
// s w to Z:  dP/dm = s w / Z  and  dP/d(s w) = (m - P) / Z.  Every vote maps to
// exactly one pixel of one view, so the gradient of a pixel is a sum over the
// voxels that vote through it.  That sum is formed without float atomics and in
// a fixed order:
//   1. count the votes of every (view, pixel) key  (integer atomics)
//   2. exclusive scan of the counts                 (offsets)
//   3. scatter voxel ranks into their key segment   (integer cursor atomics)
//   4. one lane per key: sort its (short) segment by voxel rank, recompute each
//      vote's projection and partial derivatives, accumulate in binary64 in that
//      order, and write the pixel's gradients (zero for pixels without votes).
// Projections are recomputed in steps 1, 3 and 4; only W and Z per voxel are
// kept from the forward pass.
#include "kernels.h"
#include "sample.h"

#include <algorithm>

namespace divas {

namespace {

__device__ __forceinline__ void voxel_center(const DGrid& g, uint32_t lin, double* c) {
    const uint32_t msk = (uint32_t)g.dim - 1u;
    uint32_t iv[3] = {lin & msk, (lin >> g.log2dim) & msk, lin >> (2 * g.log2dim)};
    for (int k = 0; k < 3; ++k) c[k] = g.origin[k] + ((double)iv[k] + 0.5) * g.h;
}

// Steps 1 and 3: one lane per voxel, views in order.
template <bool SCATTER>
__global__ void k_bw_votes(BwdArgs a) {
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= *a.n_act) return;
    if (!(a.Z[i] > a.p.eps) || a.gP[i] == 0.0f) return;  // P is locally constant
    double c[3];
    voxel_center(a.g, a.act[i], c);
    for (int s = 0; s < a.n_views; ++s) {
        DiffVote dv;
        if (!diff_vote_grad(a.views[s], a.g, a.p, c, &dv)) continue;
        int64_t key = a.key_base[s] + dv.pix;
        if (SCATTER) {
            uint32_t slot = atomicAdd(&a.key_end[key], 1u);
            a.list[slot] = (uint32_t)i;
        } else {
            atomicAdd(&a.key_end[key], 1u);
        }
    }
}

// Step 4: one lane per (view, pixel) key.
__global__ void k_bw_gather(BwdArgs a) {
    int64_t key = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (key >= a.key_base[a.n_views]) return;
    int s = 0;
    while (key >= a.key_base[s + 1]) ++s;
    int64_t pix = key - a.key_base[s];
    uint32_t e = a.key_end[key];
    uint32_t b = key > 0 ? a.key_end[key - 1] : 0u;
    for (uint32_t k = b + 1; k < e; ++k) {  // insertion sort by voxel rank
        uint32_t v = a.list[k];
        uint32_t j = k;
        while (j > b && a.list[j - 1] > v) {
            a.list[j] = a.list[j - 1];
            --j;
        }
        a.list[j] = v;
    }
    double gl = 0.0, gmin = 0.0, gmed = 0.0, gmax = 0.0;
    const DView& v = a.views[s];
    for (uint32_t k = b; k < e; ++k) {
        uint32_t i = a.list[k];
        double c[3];
        voxel_center(a.g, a.act[i], c);
        DiffVote dv;
        if (!diff_vote_grad(v, a.g, a.p, c, &dv)) continue;  // cannot happen: same decisions as step 1
        double Zx = a.Z[i];
        double P = a.W[i] / Zx;
        double g = (double)a.gP[i] / Zx;
        double gsw = g * (dv.m - P);
        gl += g * dv.sw * dv.dm_dl;
        gmin += gsw * dv.dsw_dmin;
        gmed += gsw * dv.dsw_dmed;
        gmax += gsw * dv.dsw_dmax;
    }
    if (a.grads[0][s]) a.grads[0][s][pix] = (float)gl;
    if (a.grads[1][s]) a.grads[1][s][pix] = (float)gmin;
    if (a.grads[2][s]) a.grads[2][s][pix] = (float)gmed;
    if (a.grads[3][s]) a.grads[3][s][pix] = (float)gmax;
}

}  // namespace

size_t backward_block_sums(int64_t n_keys) { return scan_block_sums(n_keys); }

hipError_t launch_backward(const BwdArgs& a, hipStream_t st) {
    int64_t n_keys = a.key_base[a.n_views];
    if (n_keys <= 0) return hipSuccess;
    hipError_t e;
    if ((e = launch_fill_u32(a.key_end, 0u, n_keys, st)) != hipSuccess) return e;
    unsigned vb = (unsigned)std::max<int64_t>(1, (a.cap + 255) / 256);
    hipLaunchKernelGGL(k_bw_votes<false>, dim3(vb), dim3(256), 0, st, a);
    if ((e = launch_scan_u32(a.key_end, n_keys, a.block_sums, nullptr, st)) != hipSuccess) return e;
    hipLaunchKernelGGL(k_bw_votes<true>, dim3(vb), dim3(256), 0, st, a);
    hipLaunchKernelGGL(k_bw_gather, dim3((unsigned)((n_keys + 255) / 256)), dim3(256), 0, st, a);
    return hipGetLastError();
}

}  // namespace divas
