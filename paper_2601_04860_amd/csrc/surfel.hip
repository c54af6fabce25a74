// Pass 3 of the voxel-to-surfel mapping on CDNA4 (gfx950): footprint coverage
// of every labelled surfel in the views that cover its voxel (Alg. vox2surfel,
// Pass 3; Eqs. keys-no-depth, cov-atomics, kappa, final-F).
//
// The paper bins surfel footprints into screen tiles (keys without depth),
// sorts the keys and lets tiles count covered pixels with integer atomics.
// Here a lane owns a surfel and gathers its own footprint: the counts are the
// lane's private integers, so no key sort, no atomics and no tile lists are
// needed, and the result does not depend on the schedule.  Footprints are a
// few pixels across for surfels of about a third of a voxel; a footprint of
// more than kSerialPixels pixels (a large surfel close to the camera) is swept
// by the whole wavefront with integer sums across the lanes, as the
// thin-structure fallback sweeps a voxel footprint.
//
// Per surfel (labels_in set): its voxel in binary64 (the Pass 1 rule), the
// voxel's position in the Morton-ordered active list by binary search, the
// view bitmask of that voxel from the fusion's output; then, for every view of
// the bitmask, the centre and the two tangent semi-axes in camera coordinates,
// the four projected tips, the 1-sigma pixel box and the 3-sigma ellipse test
// of every pixel of the box (ray-plane intersection in tangent coordinates,
// Cramer's rule), counting accepted pixels and those whose mask reaches tau_M.
// kappa is the largest mask_hit / max(total, 1) over the views; the label is
// kept when kappa >= tau_kappa.  Every expression is binary64 in the order of
// the arithmetic convention (no FMA contraction), so each pixel decision is
// reproducible.
#include "fuse_core.h"

namespace divas {

namespace {

constexpr int kSerialPixels = 64;

// Rotation of the unit quaternion (w, x, y, z), normalised in binary64;
// column k is the surfel's k-th local axis in world coordinates.  false when
// the quaternion has no finite non-zero norm.
__device__ __forceinline__ bool quat_axes(const float* __restrict__ q4, double* Rm) {
    double w = q4[0], x = q4[1], y = q4[2], z = q4[3];
    const double n = sqrt(((w * w + x * x) + y * y) + z * z);
    if (!(n > 0.0) || !isfinite(n)) return false;
    w /= n;
    x /= n;
    y /= n;
    z /= n;
    Rm[0] = 1.0 - 2.0 * (y * y + z * z);
    Rm[1] = 2.0 * (x * y - w * z);
    Rm[3] = 2.0 * (x * y + w * z);
    Rm[4] = 1.0 - 2.0 * (x * x + z * z);
    Rm[6] = 2.0 * (x * z - w * y);
    Rm[7] = 2.0 * (y * z + w * x);
    return true;
}

// A surfel in one view's camera frame: centre a, tangent semi-axes A and B,
// and the pixel box of its 1-sigma extent.
struct SurfelView {
    double a[3], A[3], B[3];
    int x0, x1, y0, y1;
    bool scored;  // centre and the four tips in front of the camera
};

__device__ __forceinline__ SurfelView surfel_in_view(const DView& v, const double* mu, const double* t0,
                                                     const double* t1, double eps) {
    SurfelView s;
    const double d0 = mu[0] - v.o[0], d1 = mu[1] - v.o[1], d2 = mu[2] - v.o[2];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        s.a[k] = (v.R[k] * d0 + v.R[3 + k] * d1) + v.R[6 + k] * d2;
        s.A[k] = (v.R[k] * t0[0] + v.R[3 + k] * t0[1]) + v.R[6 + k] * t0[2];
        s.B[k] = (v.R[k] * t1[0] + v.R[3 + k] * t1[1]) + v.R[6 + k] * t1[2];
    }
    s.x0 = 0;
    s.x1 = -1;
    s.y0 = 0;
    s.y1 = -1;
    s.scored = s.a[2] > eps;
    if (!s.scored) return s;
    double pu[4], pv[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const double* T = j < 2 ? s.A : s.B;  // tips a + A, a - A, a + B, a - B
        double tip[3];
        for (int k = 0; k < 3; ++k) tip[k] = j & 1 ? s.a[k] - T[k] : s.a[k] + T[k];
        s.scored &= tip[2] > eps;
        pu[j] = (v.fx * tip[0]) / tip[2] + v.cx;
        pv[j] = (v.fy * tip[1]) / tip[2] + v.cy;
    }
    if (!s.scored) return s;
    const double cu = (v.fx * s.a[0]) / s.a[2] + v.cx;
    const double cv = (v.fy * s.a[1]) / s.a[2] + v.cy;
    const double ax0 = (pu[0] - pu[1]) / 2.0, ay0 = (pv[0] - pv[1]) / 2.0;
    const double ax1 = (pu[2] - pu[3]) / 2.0, ay1 = (pv[2] - pv[3]) / 2.0;
    const double ex = fmax(fabs(ax0), fabs(ax1)), ey = fmax(fabs(ay0), fabs(ay1));
    double fx0 = floor(cu - ex), fx1 = floor(cu + ex), fy0 = floor(cv - ey), fy1 = floor(cv + ey);
    if (fx0 < 0.0) fx0 = 0.0;
    if (fy0 < 0.0) fy0 = 0.0;
    if (fx1 > (double)(v.W - 1)) fx1 = (double)(v.W - 1);
    if (fy1 > (double)(v.H - 1)) fy1 = (double)(v.H - 1);
    if (fx0 > fx1 || fy0 > fy1) return s;  // empty box: scored, no pixel
    s.x0 = (int)fx0;
    s.x1 = (int)fx1;
    s.y0 = (int)fy0;
    s.y1 = (int)fy1;
    return s;
}

// The 3-sigma test of pixel (x, y): the ray through its centre meets the
// surfel plane in front of the camera at tangent coordinates (u, v) with
// u^2 + v^2 <= 9.  *hit: accepted and the mask reaches tau_M.
__device__ __forceinline__ bool pixel_covered(const DView& v, const SurfelView& s, int x, int y, double tau_M,
                                              double eps, bool* hit) {
    const double xi = ((double)x + 0.5 - v.cx) / v.fx;
    const double zeta = ((double)y + 0.5 - v.cy) / v.fy;
    const double m00 = s.A[0] - xi * s.A[2], m01 = s.B[0] - xi * s.B[2];
    const double m10 = s.A[1] - zeta * s.A[2], m11 = s.B[1] - zeta * s.B[2];
    const double r0 = xi * s.a[2] - s.a[0], r1 = zeta * s.a[2] - s.a[1];
    const double det = m00 * m11 - m01 * m10;
    *hit = false;
    if (det == 0.0) return false;
    const double u = (r0 * m11 - m01 * r1) / det;
    const double w = (m00 * r1 - r0 * m10) / det;
    const double z = (s.a[2] + u * s.A[2]) + w * s.B[2];
    if (!(u * u + w * w <= 9.0) || !(z > eps)) return false;
    *hit = (double)ldg(v.mask + (size_t)y * (size_t)v.W + (size_t)x) >= tau_M;
    return true;
}

struct CoverageArgs {
    const float* xyz;
    const float* scales;
    const float* quats;
    int64_t n;
    const uint8_t* labels_in;
    DGrid g;
    double inv_h;
    const uint32_t* act;
    const int64_t* n_act;
    const uint64_t* vmask;
    const DView* views;
    int32_t n_views;
    double tau_M, tau_kappa, eps;
    double* kappa;
    uint8_t* labels_out;
    unsigned long long* kept;
};

// Position of the voxel with Morton code m in the Morton-ordered active list,
// or -1.
__device__ __forceinline__ int64_t find_active(const uint32_t* __restrict__ act, int64_t na, const DGrid& g,
                                               uint32_t m) {
    const uint32_t msk = (uint32_t)g.dim - 1u;
    int64_t lo = 0, hi = na;  // first entry whose code is >= m
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        const uint32_t l = act[mid];
        const uint32_t c = spread3(l & msk) | (spread3((l >> g.log2dim) & msk) << 1) |
                           (spread3(l >> (2 * g.log2dim)) << 2);
        if (c < m)
            lo = mid + 1;
        else
            hi = mid;
    }
    if (lo >= na) return -1;
    const uint32_t l = act[lo];
    const uint32_t c =
        spread3(l & msk) | (spread3((l >> g.log2dim) & msk) << 1) | (spread3(l >> (2 * g.log2dim)) << 2);
    return c == m ? lo : -1;
}

// One lane per surfel; the views are walked in a loop that is uniform across
// the wavefront (the union of the lanes' view bitmasks), so a view record is a
// scalar load and large footprints can be swept by the whole wavefront.
__global__ __launch_bounds__(256) void k_surfel_coverage(CoverageArgs a) {
    const int lane = threadIdx.x & 63;
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const bool live = i < a.n;
    uint64_t vm = 0;
    double mu[3] = {0.0, 0.0, 0.0}, t0[3] = {0.0, 0.0, 0.0}, t1[3] = {0.0, 0.0, 0.0};
    const bool labelled = live && a.labels_in[i] != 0;
    if (labelled) {
        const uint32_t m = morton_of(a.xyz[3 * i], a.xyz[3 * i + 1], a.xyz[3 * i + 2], a.g, a.inv_h);
        if (m != 0xFFFFFFFFu) {
            const int64_t k = find_active(a.act, *a.n_act, a.g, m);
            if (k >= 0) vm = a.vmask[k];
        }
        double Rm[9];
        if (vm && quat_axes(a.quats + 4 * i, Rm)) {
            const double s0 = (double)a.scales[2 * i], s1 = (double)a.scales[2 * i + 1];
            for (int k = 0; k < 3; ++k) {
                mu[k] = (double)a.xyz[3 * i + k];
                t0[k] = s0 * Rm[3 * k + 0];
                t1[k] = s1 * Rm[3 * k + 1];
            }
        } else {
            vm = 0;
        }
    }
    if (a.n_views < 64) vm &= (1ull << a.n_views) - 1ull;
    uint64_t all = vm;
    for (int off = 32; off > 0; off >>= 1) all |= (uint64_t)__shfl_xor((unsigned long long)all, off);
    all = ((uint64_t)__builtin_amdgcn_readfirstlane((int)(all >> 32)) << 32) |
          (uint32_t)__builtin_amdgcn_readfirstlane((int)(all & 0xFFFFFFFFu));
    double kap = 0.0;
    while (all) {  // uniform
        const int s = __ffsll((unsigned long long)all) - 1;
        all &= all - 1;
        const DView& v = a.views[s];
        const bool mine = (vm >> s) & 1u;
        SurfelView sv{};
        if (mine) sv = surfel_in_view(v, mu, t0, t1, a.eps);
        const int64_t bw = sv.x1 - sv.x0 + 1, bh = sv.y1 - sv.y0 + 1;
        const int64_t area = (bw > 0 && bh > 0) ? bw * bh : 0;
        const bool big = mine && sv.scored && area > kSerialPixels;
        if (mine && sv.scored && !big) {
            int64_t total = 0, hits = 0;
            for (int y = sv.y0; y <= sv.y1; ++y)
                for (int x = sv.x0; x <= sv.x1; ++x) {
                    bool h;
                    if (pixel_covered(v, sv, x, y, a.tau_M, a.eps, &h)) {
                        total += 1;
                        hits += h ? 1 : 0;
                    }
                }
            const double ks = (double)hits / (double)(total > 1 ? total : 1);
            if (ks > kap) kap = ks;
        }
        uint64_t todo = __ballot(big);
        while (todo) {  // uniform: the wavefront sweeps one large footprint at a time
            const int l = __ffsll((unsigned long long)todo) - 1;
            todo &= todo - 1;
            SurfelView w;
            for (int k = 0; k < 3; ++k) {
                w.a[k] = __shfl(sv.a[k], l);
                w.A[k] = __shfl(sv.A[k], l);
                w.B[k] = __shfl(sv.B[k], l);
            }
            w.x0 = __shfl(sv.x0, l);
            w.x1 = __shfl(sv.x1, l);
            w.y0 = __shfl(sv.y0, l);
            w.y1 = __shfl(sv.y1, l);
            w.scored = true;
            const int64_t ww = (int64_t)(w.x1 - w.x0 + 1), wa = ww * (int64_t)(w.y1 - w.y0 + 1);
            long long total = 0, hits = 0;
            for (int64_t k = lane; k < wa; k += 64) {
                bool h;
                if (pixel_covered(v, w, w.x0 + (int)(k % ww), w.y0 + (int)(k / ww), a.tau_M, a.eps, &h)) {
                    total += 1;
                    hits += h ? 1 : 0;
                }
            }
            for (int off = 32; off > 0; off >>= 1) {
                total += __shfl_xor(total, off);
                hits += __shfl_xor(hits, off);
            }
            if (lane == l) {
                const double ks = (double)hits / (double)(total > 1 ? total : 1);
                if (ks > kap) kap = ks;
            }
        }
    }
    const bool keep = labelled && kap >= a.tau_kappa;
    if (live) {
        a.kappa[i] = kap;
        a.labels_out[i] = keep ? 1 : 0;
    }
    const uint64_t nk = (uint64_t)__popcll(__ballot(keep));
    if (lane == 0 && nk && a.kept) atomicAdd(a.kept, (unsigned long long)nk);
}

}  // namespace

hipError_t launch_surfel_coverage(const float* xyz, const float* scales, const float* quats, int64_t n,
                                  const uint8_t* labels_in, const DGrid& g, const uint32_t* act,
                                  const int64_t* n_act, const uint64_t* vmask, const DView* views, int32_t n_views,
                                  double tau_M, double tau_kappa, double eps, double* kappa, uint8_t* labels_out,
                                  int64_t* kept, hipStream_t st) {
    if (kept) {
        hipError_t e = launch_fill_u32((uint32_t*)kept, 0u, 2, st);
        if (e != hipSuccess) return e;
    }
    if (n <= 0) return hipSuccess;
    CoverageArgs a{xyz,  scales, quats, n,      labels_in, g,          1.0 / g.h,  act,
                   n_act, vmask, views, n_views, tau_M,    tau_kappa, eps,        kappa, labels_out,
                   (unsigned long long*)kept};
    hipLaunchKernelGGL(k_surfel_coverage, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, a);
    return hipGetLastError();
}

}  // namespace divas
