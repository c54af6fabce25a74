// Per-sample device math of the thick path and of its differentiable variant,
// shared by the fusion and the reverse-mode kernels.  Every binary64 expression
// is written in the operation order of the arithmetic convention (the library
// is compiled without FMA contraction), so the pixel chosen and every gate
// decision are reproducible.
#pragma once

#include "kernels.h"

namespace divas {

// Load through a global-address-space pointer.  The maps are reached through
// pointers held in the view records, which the compiler would otherwise
// dereference with flat instructions; those also count against the scalar
// load counter, so waiting for a view record's fields would wait for the map
// gathers as well.
template <class T>
__device__ __forceinline__ T ldg(const T* p) {
    return *(const __attribute__((address_space(1))) T*)p;
}

// Four consecutive floats (16-byte aligned) through the global address space.
__device__ __forceinline__ float4 ldg4(const float* p) {
    typedef float v4 __attribute__((ext_vector_type(4)));
    const v4 q = *(const __attribute__((address_space(1))) v4*)p;
    return make_float4(q.x, q.y, q.z, q.w);
}

__device__ __forceinline__ double center_depth(const DView& v, int x, int y) {
    size_t i = (size_t)y * (size_t)v.W + (size_t)x;
    return ((double)ldg(v.dmin + i) + (double)ldg(v.dmax + i)) / 2.0;
}

// The depth values one sample may need at pixel (x, y): the depth triple and,
// for the depth-gradient factor, d_min and d_max of the four clamp-to-edge
// neighbours.  All eleven loads are issued together.
struct PixelDepths {
    float dmin, dmed, dmax;
    float nmin[4], nmax[4];  // neighbours x+1, x-1, y+1, y-1
};

__device__ __forceinline__ PixelDepths load_depths(const DView& v, int x, int y) {
    const int xm = x > 0 ? x - 1 : 0, xp = x < v.W - 1 ? x + 1 : v.W - 1;
    const int ym = y > 0 ? y - 1 : 0, yp = y < v.H - 1 ? y + 1 : v.H - 1;
    const size_t W = (size_t)v.W;
    const size_t p = (size_t)y * W + (size_t)x;
    const size_t q[4] = {(size_t)y * W + (size_t)xp, (size_t)y * W + (size_t)xm, (size_t)yp * W + (size_t)x,
                         (size_t)ym * W + (size_t)x};
    PixelDepths d;
    d.dmin = ldg(v.dmin + p);
    d.dmed = ldg(v.dmed + p);
    d.dmax = ldg(v.dmax + p);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        d.nmin[k] = ldg(v.dmin + q[k]);
        d.nmax[k] = ldg(v.dmax + q[k]);
    }
    return d;
}

// Squared centre-depth gradient G = g_x^2 + g_y^2 of App. D from preloaded
// neighbour depths (clamp-to-edge central differences of (d_min + d_max) / 2).
__device__ __forceinline__ double grad_sq_of(const PixelDepths& d) {
    const double cxp = ((double)d.nmin[0] + (double)d.nmax[0]) / 2.0;
    const double cxm = ((double)d.nmin[1] + (double)d.nmax[1]) / 2.0;
    const double cyp = ((double)d.nmin[2] + (double)d.nmax[2]) / 2.0;
    const double cym = ((double)d.nmin[3] + (double)d.nmax[3]) / 2.0;
    const double gx = cxp - cxm;
    const double gy = cyp - cym;
    return gx * gx + gy * gy;
}

// Depth-gradient factor of App. D from preloaded neighbour depths (same
// arithmetic as pi_dg).
__device__ __forceinline__ double pi_dg_of(const PixelDepths& d, double k) { return exp(-k * grad_sq_of(d)); }

// Depth-gradient factor of App. D at pixel (x, y), clamp-to-edge differences.
__device__ __forceinline__ double pi_dg(const DView& v, int x, int y, double k) {
    int xm = x > 0 ? x - 1 : 0, xp = x < v.W - 1 ? x + 1 : v.W - 1;
    int ym = y > 0 ? y - 1 : 0, yp = y < v.H - 1 ? y + 1 : v.H - 1;
    double gx = center_depth(v, xp, y) - center_depth(v, xm, y);
    double gy = center_depth(v, x, yp) - center_depth(v, x, ym);
    double G = gx * gx + gy * gy;
    return exp(-k * G);
}

__device__ __forceinline__ bool project_point(const DView& v, const double* p, double eps, double* u, double* vv) {
    double d0 = p[0] - v.o[0], d1 = p[1] - v.o[1], d2 = p[2] - v.o[2];
    double qx = (v.R[0] * d0 + v.R[3] * d1) + v.R[6] * d2;
    double qy = (v.R[1] * d0 + v.R[4] * d1) + v.R[7] * d2;
    double qz = (v.R[2] * d0 + v.R[5] * d1) + v.R[8] * d2;
    if (!(qz > eps)) return false;
    *u = (v.fx * qx) / qz + v.cx;
    *vv = (v.fy * qy) / qz + v.cy;
    return true;
}

// Footprint box of voxel iv in view v (footprint statistics of Sec. 3.5): the
// pixel box of its 8 projected corners, floor(min)..floor(max) inclusive,
// clipped to the image.  false when a corner is behind the camera or the box
// is empty.
__device__ __forceinline__ bool footprint_box(const DView& v, const DGrid& g, const uint32_t* iv, double eps, int* x0,
                                              int* x1, int* y0, int* y1) {
    double umin = INFINITY, umax = -INFINITY, vmin = INFINITY, vmax = -INFINITY;
    bool front = true;
    for (int j = 0; j < 8; ++j) {
        double p[3], u = 0.0, vv = 0.0;
        for (int a = 0; a < 3; ++a) p[a] = g.origin[a] + (double)(iv[a] + ((j >> a) & 1)) * g.h;
        front &= project_point(v, p, eps, &u, &vv);
        umin = fmin(umin, u);
        umax = fmax(umax, u);
        vmin = fmin(vmin, vv);
        vmax = fmax(vmax, vv);
    }
    double fx0 = floor(umin), fx1 = floor(umax), fy0 = floor(vmin), fy1 = floor(vmax);
    if (fx0 < 0.0) fx0 = 0.0;
    if (fy0 < 0.0) fy0 = 0.0;
    if (fx1 > (double)(v.W - 1)) fx1 = (double)(v.W - 1);
    if (fy1 > (double)(v.H - 1)) fy1 = (double)(v.H - 1);
    const bool ok = front && fx0 <= fx1 && fy0 <= fy1;
    *x0 = ok ? (int)fx0 : 0;
    *x1 = ok ? (int)fx1 : -1;
    *y0 = ok ? (int)fy0 : 0;
    *y1 = ok ? (int)fy1 : -1;
    return ok;
}

// The layered predicate n > mean + sigma (population sigma) over a box of A
// pixels whose counts sum to S1 and whose squares sum to S2, exactly in
// integers: nA - S1 > 0 and (nA - S1)^2 > A S2 - S1^2 (128-bit); and
// E = max(n - mean, 0) = (nA - S1) / A in binary64.
__device__ __forceinline__ void layered_of(uint32_t n, int64_t A, uint64_t S1, uint64_t S2, bool* layered, double* E) {
    const int64_t ex = (int64_t)n * A - (int64_t)S1;
    const __int128 lhs = (__int128)ex * (__int128)ex;
    const __int128 rhs = (__int128)A * (__int128)S2 - (__int128)S1 * (__int128)S1;
    *layered = (ex > 0) && (lhs > rhs);
    *E = ex > 0 ? (double)ex / (double)A : 0.0;
}

// Sums of n_samp and n_samp^2 over the box [x0, x1] x [y0, y1] of every lane
// with `need` (a wave-uniform call).  The statistics are read straight from
// the count plane: a voxel covers a few pixels, so this costs far less than
// integral images of every pixel of every view.  A box of at most
// kSerialBox pixels is summed by its own lane; a larger one (a voxel close to
// the camera) by the whole wavefront, one box at a time, with integer sums
// reduced across the lanes.  Integer sums: the result does not depend on the
// order.
constexpr int64_t kSerialBox = 64;
__device__ __forceinline__ void box_sums_wave(const uint16_t* __restrict__ ns, int W, bool need, int x0, int x1,
                                              int y0, int y1, int lane, uint64_t* S1, uint64_t* S2) {
    const int64_t bw = (int64_t)(x1 - x0 + 1), A = need ? bw * (int64_t)(y1 - y0 + 1) : 0;
    const bool big = A > kSerialBox;
    uint64_t s1 = 0, s2 = 0;
    if (need && !big)
        for (int y = y0; y <= y1; ++y)
            for (int x = x0; x <= x1; ++x) {
                const uint64_t n = ldg(ns + (size_t)y * (size_t)W + (size_t)x);
                s1 += n;
                s2 += n * n;
            }
    uint64_t todo = __ballot(big);
    while (todo) {  // uniform
        const int l = __ffsll((unsigned long long)todo) - 1;
        todo &= todo - 1;
        const int bx0 = __shfl(x0, l), bx1 = __shfl(x1, l), by0 = __shfl(y0, l), by1 = __shfl(y1, l);
        const int64_t w = (int64_t)(bx1 - bx0 + 1), a = w * (int64_t)(by1 - by0 + 1);
        unsigned long long t1 = 0, t2 = 0;
        for (int64_t k = lane; k < a; k += 64) {
            const unsigned long long n =
                ldg(ns + (size_t)(by0 + (int)(k / w)) * (size_t)W + (size_t)(bx0 + (int)(k % w)));
            t1 += n;
            t2 += n * n;
        }
        for (int off = 32; off > 0; off >>= 1) {
            t1 += __shfl_xor(t1, off);
            t2 += __shfl_xor(t2, off);
        }
        if (lane == l) {
            s1 = t1;
            s2 = t2;
        }
    }
    *S1 = s1;
    *S2 = s2;
}

// Footprint statistics of a thick-path sample (Sec. 3.5 "footprint
// statistics"): for the lanes with `need` (a wave-uniform call), the layered
// predicate and E of pixel (px, py) against the n_samp statistics of the
// voxel's footprint box.  A lane without need, or whose box is missing (a
// corner behind the camera), gets layered = false and E = 0.
__device__ __forceinline__ void footprint_stats_wave(const DView& v, const DGrid& g, const uint32_t* iv, double eps,
                                                     bool need, int px, int py, int lane, bool* layered, double* E) {
    int x0 = 0, x1 = -1, y0 = 0, y1 = -1;
    const bool box = need && footprint_box(v, g, iv, eps, &x0, &x1, &y0, &y1);
    uint64_t S1 = 0, S2 = 0;
    box_sums_wave(v.nsamp, v.W, box, x0, x1, y0, y1, lane, &S1, &S2);
    *layered = false;
    *E = 0.0;
    if (box) {
        const uint32_t n = ldg(v.nsamp + (size_t)py * (size_t)v.W + (size_t)px);
        layered_of(n, (int64_t)(x1 - x0 + 1) * (int64_t)(y1 - y0 + 1), S1, S2, layered, E);
    }
}

// First part of a thick-path sample: projection, frame test and the pixel's
// bit of the gate bitmask (mask >= mask_gate).  The byte load is issued here,
// so that a caller can start the next view's sample while the current one
// finishes.  Branch-free: every lane computes the projection and loads a byte
// (that of pixel (0, 0) when the centre is behind the camera or outside the
// frame), so the loads of several heads can be in flight together.
struct SampleHead {
    double qz;
    int px, py;
    uint32_t bits;  // the bitmask byte holding the pixel
    bool in;        // in front of the camera and inside the frame
};

// The projection part of a head (no load): camera Z, pixel, frame test.
__device__ __forceinline__ SampleHead sample_proj(const DView& v, const double* c, double eps) {
    SampleHead h;
    const double d0 = c[0] - v.o[0], d1 = c[1] - v.o[1], d2 = c[2] - v.o[2];
    const double qx = (v.R[0] * d0 + v.R[3] * d1) + v.R[6] * d2;
    const double qy = (v.R[1] * d0 + v.R[4] * d1) + v.R[7] * d2;
    const double qz = (v.R[2] * d0 + v.R[5] * d1) + v.R[8] * d2;
    const double u = (v.fx * qx) / qz + v.cx;  // used only when qz > eps
    const double vv = (v.fy * qy) / qz + v.cy;
    // evaluated without short-circuit branches
    h.in = (qz > eps) & (u >= 0.0) & (u < (double)v.W) & (vv >= 0.0) & (vv < (double)v.H);
    h.px = (int)floor(h.in ? u : 0.0);
    h.py = (int)floor(h.in ? vv : 0.0);
    h.bits = 0u;
    h.qz = qz;
    return h;
}

// The byte of view v's gate bitmask that holds the head's pixel.
__device__ __forceinline__ uint32_t gate_byte(const DView& v, const SampleHead& h) {
    return ldg(v.mbits + (size_t)h.py * (size_t)v.mpitch + (size_t)(h.px >> 3));
}

__device__ __forceinline__ SampleHead sample_head(const DView& v, const double* c, double eps) {
    SampleHead h = sample_proj(v, c, eps);
    h.bits = gate_byte(v, h);
    return h;
}

// Whether a sample's pixel passes the thick-path entry gate (its bit of the
// gate bitmask, mask >= mask_gate), for a head in frame.
__device__ __forceinline__ bool head_passes(const SampleHead& hd) { return hd.in && ((hd.bits >> (hd.px & 7)) & 1u); }

// What a thick-path sample reads at its pixel once the gate bit is set: the
// mask value, the depth triple, and the squared depth gradient G of App. D
// from the four neighbours' d_min / d_max.  All twelve loads are issued
// together; only G is kept of the neighbours.
struct PixelSample {
    float m, dmin, dmed, dmax;
    double G;
};

__device__ __forceinline__ PixelSample sample_load(const DView& v, const SampleHead& hd) {
    const float m = ldg(v.mask + (size_t)hd.py * (size_t)v.W + (size_t)hd.px);
    const PixelDepths pd = load_depths(v, hd.px, hd.py);
    return PixelSample{m, pd.dmin, pd.dmed, pd.dmax, grad_sq_of(pd)};
}

// Whether a gathered sample can vote at all, from its depths alone: a surface
// at the pixel (D_med >= eps), a trusted pixel (D_min <= D_med), and the
// asymmetric depth gate of Eq. asym-gate passing at the widest tolerance it
// can have, gamma h (the tightened gamma h / (1 + beta E) never exceeds it
// when gamma, beta >= 0), with the front reference where the pixel is
// see-through or `maybe_layered` (footprint statistics not yet known).  Exact:
// a sample that fails here fails the full test too.  With negative gamma or
// beta every gathered sample stays a candidate.
__device__ __forceinline__ bool depth_candidate(const DView& v, const DGrid& g, const DParams& P, double qz,
                                                const PixelSample& s, bool maybe_layered) {
    const double dmin = (double)s.dmin, dmed = (double)s.dmed;
    const bool surface = !(dmed < P.eps), trusted = dmin <= dmed;
    if (!(P.gamma >= 0.0 && P.beta >= 0.0)) return surface & trusted;
    const double t = P.gamma * g.h;
    const bool seethru = dmed > P.gamma_st * v.d_cam;
    const bool front_ok = qz - dmin <= t, back_ok = fabs(qz - dmed) <= t;
    const bool possible = seethru ? front_ok : (back_ok | (maybe_layered & front_ok));
    return surface & trusted & possible;
}

// The rest of a thick-path sample past the gate and the loads: planar-to-ray
// conversion through the sampled pixel's centre, reference switch, the
// asymmetric depth gate with tightening, the spatial gate with the
// depth-gradient factor, and the Gaussian weight.  layered and E are the
// sample's footprint statistics (false and 0 without n_samp).  Returns true
// with the weight w and the mask value m when the view votes.
//
// Work is skipped only where it cannot change the result: the tolerance
// gamma h / (1 + beta E) is gamma h exactly when E = 0 (x / 1 = x), the
// depth-gradient factor is evaluated only when delta <= h (for k >= 0 it is
// at most 1, so h pi_dg <= h), and the weight only for a vote.
__device__ __forceinline__ bool sample_decide(const DView& v, const DGrid& g, const DParams& P, const double* c,
                                              const SampleHead& hd, const PixelSample& s, bool layered, double E,
                                              double* w_out, double* m_out) {
    const double eps = P.eps;
    const int px = hd.px, py = hd.py;
    const double dmin = (double)s.dmin, dmed = (double)s.dmed, dmax = (double)s.dmax;
    const double xd = hd.qz;
    bool ok = !(dmed < eps);  // a surface at this pixel
    ok &= dmin <= dmed;       // trusted
    const double d0 = c[0] - v.o[0], d1 = c[1] - v.o[1], d2 = c[2] - v.o[2];
    // ray through the sampled pixel's centre, planar-to-ray conversion
    const double r0 = ((double)px + 0.5 - v.cx) / v.fx;
    const double r1 = ((double)py + 0.5 - v.cy) / v.fy;
    const double w0 = (v.R[0] * r0 + v.R[1] * r1) + v.R[2];
    const double w1 = (v.R[3] * r0 + v.R[4] * r1) + v.R[5];
    const double w2 = (v.R[6] * r0 + v.R[7] * r1) + v.R[8];
    const double nrm = sqrt((w0 * w0 + w1 * w1) + w2 * w2);
    const double h0 = w0 / nrm, h1 = w1 / nrm, h2 = w2 / nrm;
    const double cosv = (v.R[2] * h0 + v.R[5] * h1) + v.R[8] * h2;
    const double dmin_r = dmin / cosv, dmed_r = dmed / cosv;
    const bool seethru = dmed > P.gamma_st * v.d_cam;
    const bool front = layered | seethru;
    const double dref_r = front ? dmin_r : dmed_r;
    const double ts = (d0 * h0 + d1 * h1) + d2 * h2;
    double th = ts < dmin_r ? dmin_r : ts;
    th = th > dref_r ? dref_r : th;
    const double e0 = c[0] - (v.o[0] + th * h0);
    const double e1 = c[1] - (v.o[1] + th * h1);
    const double e2 = c[2] - (v.o[2] + th * h2);
    const double delta = sqrt((e0 * e0 + e1 * e1) + e2 * e2);
    const double gh = P.gamma * g.h;
    const double t_depth = E == 0.0 ? gh : gh / (1.0 + P.beta * E);
    const bool valid = front ? (xd - dmin <= t_depth) : (fabs(xd - dmed) <= t_depth);
    ok &= valid;
    // spatial gate delta <= h pi_dg
    ok &= !(P.k_grad >= 0.0) || delta <= g.h;
    if (ok) ok = delta <= g.h * exp(-P.k_grad * s.G);
    if (ok) {
        const double dmax_r = dmax / cosv;
        const double d_ctr = (dmin_r + dmax_r) / 2.0;
        double d_hw = (dmax_r - dmin_r) / 2.0;
        d_hw = d_hw < eps ? eps : d_hw;
        const double rr = (th - d_ctr) / d_hw;
        *w_out = exp(-P.alpha1 * (rr * rr));
        *m_out = (double)s.m;
    }
    return ok;
}

// A whole thick-path sample of the lanes (wave-uniform call): the gate bit of
// the head, the loads, the depth-only candidate test, the footprint statistics
// of the candidates when the view carries n_samp (NSAMP), and the rest.
// *gathered: the sample passed the gate and read the maps.
template <bool NSAMP>
__device__ __forceinline__ bool thick_sample_wave(const DView& v, const DGrid& g, const DParams& P, const uint32_t* iv,
                                                  const double* c, const SampleHead& hd, bool live, int lane,
                                                  double* w_out, double* m_out, bool* gathered) {
    const bool pass = live && head_passes(hd);
    PixelSample s{};
    if (pass) s = sample_load(v, hd);
    *gathered = pass;
    const bool ns = NSAMP && v.nsamp != nullptr;  // uniform
    const bool cand = pass && depth_candidate(v, g, P, hd.qz, s, ns);
    bool layered = false;
    double E = 0.0;
    if (ns) footprint_stats_wave(v, g, iv, P.eps, cand, hd.px, hd.py, lane, &layered, &E);
    bool vote = false;
    if (cand) vote = sample_decide(v, g, P, c, hd, s, layered, E, w_out, m_out);
    return vote;
}

// Thin-structure score of one voxel in one view (Alg. gs-thin; Eqs. thin-nmin,
// gs-coverage, thin-d2min, thin-tthin-gs), evaluated by a whole wavefront:
// every lane passes the same voxel and gets the same result.  The footprint is
// the 8-corner box (floor(min)..floor(max) inclusive, clipped); the lanes share
// its pixels, counting the depth-consistent ones and, among them, those with
// M~ > 0.5, whose unprojected surface points give the smallest squared
// distance to the centre and whose largest M~ is the score.  The counts (sums),
// the peak (max) and the nearest point (min) are reduced across the wavefront,
// so the result does not depend on how the pixels are shared.
__device__ __forceinline__ double thin_score_wave(const DView& v, const DGrid& g, const DParams& P, const uint32_t* iv,
                                                  const double* c, double xd, int lane) {
    const double eps = P.eps;
    double umin = INFINITY, umax = -INFINITY, vmin = INFINITY, vmax = -INFINITY;
    bool front_all = true;
    for (int j = 0; j < 8; ++j) {
        double p[3], u, vv;
        for (int a = 0; a < 3; ++a) p[a] = g.origin[a] + (double)(iv[a] + ((j >> a) & 1)) * g.h;
        if (!project_point(v, p, eps, &u, &vv)) {
            front_all = false;
            break;
        }
        umin = fmin(umin, u);
        umax = fmax(umax, u);
        vmin = fmin(vmin, vv);
        vmax = fmax(vmax, vv);
    }
    if (!front_all) return 0.0;
    double fx0 = floor(umin), fx1 = floor(umax), fy0 = floor(vmin), fy1 = floor(vmax);
    if (fx0 < 0.0) fx0 = 0.0;
    if (fy0 < 0.0) fy0 = 0.0;
    if (fx1 > (double)(v.W - 1)) fx1 = (double)(v.W - 1);
    if (fy1 > (double)(v.H - 1)) fy1 = (double)(v.H - 1);
    if (fx0 > fx1 || fy0 > fy1) return 0.0;
    const int x0 = (int)fx0, x1 = (int)fx1, y0 = (int)fy0, y1 = (int)fy1;
    const int bw = x1 - x0 + 1;
    const int64_t Ai = (int64_t)bw * (int64_t)(y1 - y0 + 1);
    const double A = (double)bw * (double)(y1 - y0 + 1);
    double n_min = ceil(P.rho_occ * A);
    if (n_min < P.n_abs) n_min = P.n_abs;
    // at most A pixels can be depth-consistent: a footprint smaller than the
    // support floor scores 0 without a sweep (uniform across the wavefront)
    if (A < n_min) return 0.0;
    const bool stats = v.nsamp != nullptr;
    uint64_t S1 = 0, S2 = 0;
    if (stats) {  // n_samp sums over the footprint, reduced across the wavefront
        unsigned long long t1 = 0, t2 = 0;
        for (int64_t k = lane; k < Ai; k += 64) {
            const unsigned long long n =
                ldg(v.nsamp + (size_t)(y0 + (int)(k / bw)) * (size_t)v.W + (size_t)(x0 + (int)(k % bw)));
            t1 += n;
            t2 += n * n;
        }
        for (int off = 32; off > 0; off >>= 1) {
            t1 += __shfl_xor(t1, off);
            t2 += __shfl_xor(t2, off);
        }
        S1 = t1;
        S2 = t2;
    }
    unsigned n_depth = 0, n_md = 0;
    double m_max = 0.0, d2 = INFINITY;
    for (int64_t k = lane; k < Ai; k += 64) {
        const int x = x0 + (int)(k % bw), y = y0 + (int)(k / bw);
        const size_t pix = (size_t)y * (size_t)v.W + (size_t)x;
        const double m = (double)ldg(v.mask + pix);
        const double dmin = (double)ldg(v.dmin + pix), dmed = (double)ldg(v.dmed + pix);
        if (dmed < eps) continue;  // no surface
        bool layered = false;
        double E = 0.0;
        if (stats) layered_of(ldg(v.nsamp + pix), Ai, S1, S2, &layered, &E);
        const double eta = 1.0 / (1.0 + P.beta * E);
        const double tau = (P.gamma * g.h) * eta;
        const bool seethru = dmed > P.gamma_st * v.d_cam;
        const bool front = (layered || seethru) && dmin <= dmed;  // front hit only when trusted
        const bool valid = front ? (xd - dmin <= tau) : (fabs(xd - dmed) <= tau);
        if (!valid) continue;
        n_depth += 1;
        if (!(m > 0.5)) continue;
        n_md += 1;
        if (m > m_max) m_max = m;
        const double d = layered ? dmin : dmed;
        const double cxp = ((double)x + 0.5 - v.cx) / v.fx * d;
        const double cyp = ((double)y + 0.5 - v.cy) / v.fy * d;
        const double e0 = (((v.R[0] * cxp + v.R[1] * cyp) + v.R[2] * d) + v.o[0]) - c[0];
        const double e1 = (((v.R[3] * cxp + v.R[4] * cyp) + v.R[5] * d) + v.o[1]) - c[1];
        const double e2 = (((v.R[6] * cxp + v.R[7] * cyp) + v.R[8] * d) + v.o[2]) - c[2];
        const double q = (e0 * e0 + e1 * e1) + e2 * e2;
        if (q < d2) d2 = q;
    }
    for (int off = 32; off > 0; off >>= 1) {
        n_depth += (unsigned)__shfl_xor((int)n_depth, off);
        n_md += (unsigned)__shfl_xor((int)n_md, off);
        const double a = __shfl_xor(m_max, off), b = __shfl_xor(d2, off);
        m_max = a > m_max ? a : m_max;
        d2 = b < d2 ? b : d2;
    }
    if ((double)n_depth < n_min) return 0.0;  // degeneracy floor
    const double p_cov = (double)n_md / (double)n_depth;
    const double g15 = 1.5 * g.h;
    return (p_cov >= P.rho_cover && d2 <= g15 * g15) ? m_max : 0.0;
}

// Entry of the thin fallback for a sample the thick path rejected (Alg.
// gs-fusion): the centre in frame, the behind-surface gate (Eq. behind-gate)
// and the density floor; *xd is the voxel's planar depth.
__device__ __forceinline__ bool thin_eligible(const DView& v, const DGrid& g, const DParams& P, const double* c,
                                              uint32_t rho, double* xd) {
    const double eps = P.eps;
    const double d0 = c[0] - v.o[0], d1 = c[1] - v.o[1], d2 = c[2] - v.o[2];
    const double qx = (v.R[0] * d0 + v.R[3] * d1) + v.R[6] * d2;
    const double qy = (v.R[1] * d0 + v.R[4] * d1) + v.R[7] * d2;
    const double qz = (v.R[2] * d0 + v.R[5] * d1) + v.R[8] * d2;
    if (!(qz > eps)) return false;
    const double u = (v.fx * qx) / qz + v.cx;
    const double vv = (v.fy * qy) / qz + v.cy;
    if (!(u >= 0.0 && u < (double)v.W && vv >= 0.0 && vv < (double)v.H)) return false;
    const size_t pix = (size_t)floor(vv) * (size_t)v.W + (size_t)floor(u);
    const double dmin = (double)ldg(v.dmin + pix), dmed = (double)ldg(v.dmed + pix);
    const bool trusted = dmin <= dmed;
    const bool seethru = dmed > P.gamma_st * v.d_cam;
    const double d_surf = (trusted && seethru) ? dmin : dmed;
    if (qz > d_surf + 2.0 * g.h) return false;  // behind the visible surface
    if (!((double)rho >= P.rho_thin)) return false;
    *xd = qz;
    return true;
}

// One (voxel, view) sample of the NeRF thick path (Alg. nerf-fusion, thick
// branch; Eqs. distance_cond, dist_tol, depth_tol, nerf-accept, nerf-vote).
// The ray parameter t_proj of the voxel centre is clamped into [D_min, D_max]
// as written.  By default the depth tuple is camera Z and so is the voxel's
// depth x_d; with nerf_ray_depths the tuple holds distances along the pixel
// ray and x_d = t_proj.  Returns true with the weight w and the mask value m
// when the view votes.
__device__ __forceinline__ bool nerf_sample(const DView& v, const DGrid& g, const DParams& P, const double* c,
                                            double* w_out, double* m_out, bool* gathered) {
    const double eps = P.eps;
    const double d0 = c[0] - v.o[0], d1 = c[1] - v.o[1], d2 = c[2] - v.o[2];
    const double qx = (v.R[0] * d0 + v.R[3] * d1) + v.R[6] * d2;
    const double qy = (v.R[1] * d0 + v.R[4] * d1) + v.R[7] * d2;
    const double qz = (v.R[2] * d0 + v.R[5] * d1) + v.R[8] * d2;
    if (!(qz > eps)) return false;
    const double u = (v.fx * qx) / qz + v.cx;
    const double vv = (v.fy * qy) / qz + v.cy;
    if (!(u >= 0.0 && u < (double)v.W && vv >= 0.0 && vv < (double)v.H)) return false;
    const int px = (int)floor(u), py = (int)floor(vv);
    const size_t pix = (size_t)py * (size_t)v.W + (size_t)px;
    const double m = (double)ldg(v.mask + pix);
    if (!(m >= P.mask_gate)) return false;  // thick-path entry gate
    *gathered = true;
    const PixelDepths pd = load_depths(v, px, py);
    const double ns = v.nsamp ? (double)ldg(v.nsamp + pix) : 0.0;
    const double dmin = (double)pd.dmin, dexp = (double)pd.dmed, dmax = (double)pd.dmax;
    bool ok = !(dexp < eps);  // a surface at this pixel
    // closest point of the ray segment [d_min, d_max] to the voxel centre
    const double r0 = ((double)px + 0.5 - v.cx) / v.fx;
    const double r1 = ((double)py + 0.5 - v.cy) / v.fy;
    const double w0 = (v.R[0] * r0 + v.R[1] * r1) + v.R[2];
    const double w1 = (v.R[3] * r0 + v.R[4] * r1) + v.R[5];
    const double w2 = (v.R[6] * r0 + v.R[7] * r1) + v.R[8];
    const double nrm = sqrt((w0 * w0 + w1 * w1) + w2 * w2);
    const double h0 = w0 / nrm, h1 = w1 / nrm, h2 = w2 / nrm;
    const double tp = (d0 * h0 + d1 * h1) + d2 * h2;
    double tc = tp < dmin ? dmin : tp;
    tc = tc > dmax ? dmax : tc;
    const double e0 = c[0] - (v.o[0] + tc * h0);
    const double e1 = c[1] - (v.o[1] + tc * h1);
    const double e2 = c[2] - (v.o[2] + tc * h2);
    const double delta = sqrt((e0 * e0 + e1 * e1) + e2 * e2);
    // spatial tolerance with the band slack; depth tolerance with the capped bonus
    const double tau_sp = g.h * pi_dg_of(pd, P.k_grad) + P.lambda_range * (dmax - dmin);
    double b = P.beta * ns;
    b = b > P.b_max ? P.b_max : b;
    const double tau_d = (P.gamma + b) * g.h;
    const double xd = P.nerf_ray_depths ? tp : qz;  // the voxel's depth in this view
    ok &= (delta <= tau_sp) & (fabs(xd - dexp) <= tau_d);
    // Gaussian fall-off from the band midpoint
    const double mu = (dmin + dmax) / 2.0;
    double hd = (dmax - dmin) / 2.0;
    hd = hd < eps ? eps : hd;
    const double r = fabs(tc - mu) / hd;
    *w_out = exp(-P.alpha1 * (r * r));
    *m_out = m;
    return ok;
}

// Entry of the NeRF thin path for a sample the thick path did not accept
// (Alg. nerf-fusion): the centre in frame, its mask above 0.1 and the voxel's
// density at least rho_thin; *xd is the voxel's depth (camera Z, or t_proj on
// the centre pixel's ray with nerf_ray_depths).
__device__ __forceinline__ bool nerf_thin_eligible(const DView& v, const DGrid& g, const DParams& P, const double* c,
                                                   uint32_t rho, double* xd) {
    const double d0 = c[0] - v.o[0], d1 = c[1] - v.o[1], d2 = c[2] - v.o[2];
    const double qx = (v.R[0] * d0 + v.R[3] * d1) + v.R[6] * d2;
    const double qy = (v.R[1] * d0 + v.R[4] * d1) + v.R[7] * d2;
    const double qz = (v.R[2] * d0 + v.R[5] * d1) + v.R[8] * d2;
    if (!(qz > P.eps)) return false;
    const double u = (v.fx * qx) / qz + v.cx;
    const double vv = (v.fy * qy) / qz + v.cy;
    if (!(u >= 0.0 && u < (double)v.W && vv >= 0.0 && vv < (double)v.H)) return false;
    const int px = (int)floor(u), py = (int)floor(vv);
    const double m = (double)ldg(v.mask + (size_t)py * (size_t)v.W + (size_t)px);
    if (!(m > 0.1)) return false;
    if (!((double)rho >= P.rho_thin)) return false;
    if (P.nerf_ray_depths) {
        const double r0 = ((double)px + 0.5 - v.cx) / v.fx;
        const double r1 = ((double)py + 0.5 - v.cy) / v.fy;
        const double w0 = (v.R[0] * r0 + v.R[1] * r1) + v.R[2];
        const double w1 = (v.R[3] * r0 + v.R[4] * r1) + v.R[5];
        const double w2 = (v.R[6] * r0 + v.R[7] * r1) + v.R[8];
        const double nrm = sqrt((w0 * w0 + w1 * w1) + w2 * w2);
        const double h0 = w0 / nrm, h1 = w1 / nrm, h2 = w2 / nrm;
        *xd = (d0 * h0 + d1 * h1) + d2 * h2;
    } else {
        *xd = qz;
    }
    return true;
}

// Thin-structure score of one voxel in one view under the NeRF path (Alg.
// nerf-thin; Eqs. nerf-thindepth, nerf-support, nerf-counters,
// nerf-coverage, nerf-thin), evaluated by a whole wavefront (every lane passes
// the same voxel and gets the same result): over the 8-corner footprint
// (floor(min)..floor(max), clipped; N_pixels its pixel count) the lanes count
// the supportive pixels (M~ > 0.5 and |x_d - D_exp| <= (2 gamma + b) h with
// the pixel's own capped bonus b) and take the largest M~ of any pixel; the
// sum and the maximum are reduced across the wavefront.  The score is that
// peak when the supportive fraction reaches rho_cover, else 0.
__device__ __forceinline__ double nerf_thin_score_wave(const DView& v, const DGrid& g, const DParams& P,
                                                       const uint32_t* iv, double xd, int lane) {
    const double eps = P.eps;
    double umin = INFINITY, umax = -INFINITY, vmin = INFINITY, vmax = -INFINITY;
    for (int j = 0; j < 8; ++j) {
        double p[3], u, vv;
        for (int a = 0; a < 3; ++a) p[a] = g.origin[a] + (double)(iv[a] + ((j >> a) & 1)) * g.h;
        if (!project_point(v, p, eps, &u, &vv)) return 0.0;
        umin = fmin(umin, u);
        umax = fmax(umax, u);
        vmin = fmin(vmin, vv);
        vmax = fmax(vmax, vv);
    }
    double fx0 = floor(umin), fx1 = floor(umax), fy0 = floor(vmin), fy1 = floor(vmax);
    if (fx0 < 0.0) fx0 = 0.0;
    if (fy0 < 0.0) fy0 = 0.0;
    if (fx1 > (double)(v.W - 1)) fx1 = (double)(v.W - 1);
    if (fy1 > (double)(v.H - 1)) fy1 = (double)(v.H - 1);
    if (fx0 > fx1 || fy0 > fy1) return 0.0;
    const int x0 = (int)fx0, x1 = (int)fx1, y0 = (int)fy0, y1 = (int)fy1;
    const int bw = x1 - x0 + 1;
    const int64_t Ai = (int64_t)bw * (int64_t)(y1 - y0 + 1);
    const double n_pixels = (double)bw * (double)(y1 - y0 + 1);
    unsigned n_valid = 0;
    double m_max = 0.0;
    for (int64_t k = lane; k < Ai; k += 64) {
        const int x = x0 + (int)(k % bw), y = y0 + (int)(k / bw);
        const size_t pix = (size_t)y * (size_t)v.W + (size_t)x;
        const double m = (double)ldg(v.mask + pix);
        const double dexp = (double)ldg(v.dmed + pix);
        const double ns = v.nsamp ? (double)ldg(v.nsamp + pix) : 0.0;
        double b = P.beta * ns;
        b = b > P.b_max ? P.b_max : b;
        const double tau = (2.0 * P.gamma + b) * g.h;
        n_valid += (m > 0.5 && fabs(xd - dexp) <= tau) ? 1u : 0u;
        m_max = m > m_max ? m : m_max;
    }
    for (int off = 32; off > 0; off >>= 1) {
        n_valid += (unsigned)__shfl_xor((int)n_valid, off);
        const double a = __shfl_xor(m_max, off);
        m_max = a > m_max ? a : m_max;
    }
    const double p_cov = (double)n_valid / n_pixels;
    return p_cov >= P.rho_cover ? m_max : 0.0;
}

__device__ __forceinline__ double sigm(double x) { return 1.0 / (1.0 + exp(-x)); }

// Differentiable variant: every in-frame view with a trusted surface votes
// sigmoid(logit) * s * w with the soft depth test s; the spatial gate is hard.
__device__ __forceinline__ bool diff_sample(const DView& v, const DGrid& g, const DParams& P, const double* c,
                                            double* sw_out, double* m_out, bool* gathered) {
    const double eps = P.eps;
    double d0 = c[0] - v.o[0], d1 = c[1] - v.o[1], d2 = c[2] - v.o[2];
    double qx = (v.R[0] * d0 + v.R[3] * d1) + v.R[6] * d2;
    double qy = (v.R[1] * d0 + v.R[4] * d1) + v.R[7] * d2;
    double qz = (v.R[2] * d0 + v.R[5] * d1) + v.R[8] * d2;
    if (!(qz > eps)) return false;
    double u = (v.fx * qx) / qz + v.cx;
    double vv = (v.fy * qy) / qz + v.cy;
    if (!(u >= 0.0 && u < (double)v.W && vv >= 0.0 && vv < (double)v.H)) return false;
    int px = (int)floor(u), py = (int)floor(vv);
    size_t pix = (size_t)py * (size_t)v.W + (size_t)px;
    const float lgf = ldg(v.mask + pix);
    *gathered = true;
    const PixelDepths pd = load_depths(v, px, py);
    double dmed = (double)pd.dmed;
    if (dmed < eps) return false;
    double dmin = (double)pd.dmin, dmax = (double)pd.dmax;
    if (!(dmin <= dmed)) return false;
    double lg = (double)lgf;
    double xd = qz;
    double r0 = ((double)px + 0.5 - v.cx) / v.fx;
    double r1 = ((double)py + 0.5 - v.cy) / v.fy;
    double w0 = (v.R[0] * r0 + v.R[1] * r1) + v.R[2];
    double w1 = (v.R[3] * r0 + v.R[4] * r1) + v.R[5];
    double w2 = (v.R[6] * r0 + v.R[7] * r1) + v.R[8];
    double nrm = sqrt((w0 * w0 + w1 * w1) + w2 * w2);
    double h0 = w0 / nrm, h1 = w1 / nrm, h2 = w2 / nrm;
    double cosv = (v.R[2] * h0 + v.R[5] * h1) + v.R[8] * h2;
    double dmin_r = dmin / cosv, dmed_r = dmed / cosv, dmax_r = dmax / cosv;
    bool front = dmed > P.gamma_st * v.d_cam;
    double dref_r = front ? dmin_r : dmed_r;
    double ts = (d0 * h0 + d1 * h1) + d2 * h2;
    double th = ts < dmin_r ? dmin_r : ts;
    if (th > dref_r) th = dref_r;
    double e0 = c[0] - (v.o[0] + th * h0);
    double e1 = c[1] - (v.o[1] + th * h1);
    double e2 = c[2] - (v.o[2] + th * h2);
    double delta = sqrt((e0 * e0 + e1 * e1) + e2 * e2);
    double tau_sp = g.h * pi_dg_of(pd, P.k_grad);
    if (!(delta <= tau_sp)) return false;
    double e = front ? (xd - dmin) : fabs(xd - dmed);
    double s = sigm((P.gamma * g.h - e) / P.soft_width);
    double d_ctr = (dmin_r + dmax_r) / 2.0;
    double d_hw = (dmax_r - dmin_r) / 2.0;
    if (d_hw < eps) d_hw = eps;
    double rr = (th - d_ctr) / d_hw;
    double w = exp(-P.alpha1 * (rr * rr));
    *sw_out = s * w;
    *m_out = sigm(lg);
    return true;
}


// Differentiable vote with its partial derivatives: the same decisions as
// diff_sample, plus d(m)/d(logit) and d(s w)/d(planar depths) at the pixel.
struct DiffVote {
    int64_t pix;
    double m, sw, dm_dl, dsw_dmin, dsw_dmed, dsw_dmax;
};

__device__ __forceinline__ bool diff_vote_grad(const DView& v, const DGrid& g, const DParams& P, const double* c,
                                               DiffVote* out) {
    const double eps = P.eps;
    double d0 = c[0] - v.o[0], d1 = c[1] - v.o[1], d2 = c[2] - v.o[2];
    double qx = (v.R[0] * d0 + v.R[3] * d1) + v.R[6] * d2;
    double qy = (v.R[1] * d0 + v.R[4] * d1) + v.R[7] * d2;
    double qz = (v.R[2] * d0 + v.R[5] * d1) + v.R[8] * d2;
    if (!(qz > eps)) return false;
    double u = (v.fx * qx) / qz + v.cx;
    double vv = (v.fy * qy) / qz + v.cy;
    if (!(u >= 0.0 && u < (double)v.W && vv >= 0.0 && vv < (double)v.H)) return false;
    int px = (int)floor(u), py = (int)floor(vv);
    size_t pix = (size_t)py * (size_t)v.W + (size_t)px;
    const float lgf = ldg(v.mask + pix);
    const PixelDepths pd = load_depths(v, px, py);
    double dmed = (double)pd.dmed;
    if (dmed < eps) return false;
    double dmin = (double)pd.dmin, dmax = (double)pd.dmax;
    if (!(dmin <= dmed)) return false;
    double lg = (double)lgf;
    double xd = qz;
    double r0 = ((double)px + 0.5 - v.cx) / v.fx;
    double r1 = ((double)py + 0.5 - v.cy) / v.fy;
    double w0 = (v.R[0] * r0 + v.R[1] * r1) + v.R[2];
    double w1 = (v.R[3] * r0 + v.R[4] * r1) + v.R[5];
    double w2 = (v.R[6] * r0 + v.R[7] * r1) + v.R[8];
    double nrm = sqrt((w0 * w0 + w1 * w1) + w2 * w2);
    double h0 = w0 / nrm, h1 = w1 / nrm, h2 = w2 / nrm;
    double cosv = (v.R[2] * h0 + v.R[5] * h1) + v.R[8] * h2;
    double dmin_r = dmin / cosv, dmed_r = dmed / cosv, dmax_r = dmax / cosv;
    bool front = dmed > P.gamma_st * v.d_cam;
    double dref_r = front ? dmin_r : dmed_r;
    double ts = (d0 * h0 + d1 * h1) + d2 * h2;
    bool lo_clamp = ts < dmin_r;
    double th = lo_clamp ? dmin_r : ts;
    bool hi_clamp = th > dref_r;
    if (hi_clamp) th = dref_r;
    double e0 = c[0] - (v.o[0] + th * h0);
    double e1 = c[1] - (v.o[1] + th * h1);
    double e2 = c[2] - (v.o[2] + th * h2);
    double delta = sqrt((e0 * e0 + e1 * e1) + e2 * e2);
    double tau_sp = g.h * pi_dg(v, px, py, P.k_grad);
    if (!(delta <= tau_sp)) return false;
    // soft depth test s = sigmoid((gamma h - e) / w_s)
    double e, de_dmin = 0.0, de_dmed = 0.0;
    if (front) {
        e = xd - dmin;
        de_dmin = -1.0;
    } else {
        e = fabs(xd - dmed);
        de_dmed = (xd - dmed) > 0.0 ? -1.0 : ((xd - dmed) < 0.0 ? 1.0 : 0.0);
    }
    double s = sigm((P.gamma * g.h - e) / P.soft_width);
    double ds_de = -s * (1.0 - s) / P.soft_width;
    // depth weight w = exp(-alpha1 r^2), r = (t - d_ctr) / d_hw
    double d_ctr = (dmin_r + dmax_r) / 2.0;
    double hw_raw = (dmax_r - dmin_r) / 2.0;
    bool hw_floor = hw_raw < eps;
    double d_hw = hw_floor ? eps : hw_raw;
    double rr = (th - d_ctr) / d_hw;
    double w = exp(-P.alpha1 * (rr * rr));
    double dw_dr = -2.0 * P.alpha1 * rr * w;
    double dth_dminr = (lo_clamp && !hi_clamp) ? 1.0 : 0.0;
    double dth_drefr = hi_clamp ? 1.0 : 0.0;
    double dr_dth = 1.0 / d_hw;
    double dr_dctr = -1.0 / d_hw;
    double dr_dhw = hw_floor ? 0.0 : -rr / d_hw;
    double dr_dminr = dr_dth * dth_dminr + dr_dctr * 0.5 + dr_dhw * (-0.5);
    double dr_dmaxr = dr_dctr * 0.5 + dr_dhw * 0.5;
    double dr_dmedr = 0.0;
    if (front)
        dr_dminr += dr_dth * dth_drefr;
    else
        dr_dmedr += dr_dth * dth_drefr;
    double dw_dmin = dw_dr * dr_dminr / cosv;
    double dw_dmed = dw_dr * dr_dmedr / cosv;
    double dw_dmax = dw_dr * dr_dmaxr / cosv;
    double m = sigm(lg);
    out->pix = (int64_t)pix;
    out->m = m;
    out->sw = s * w;
    out->dm_dl = m * (1.0 - m);
    out->dsw_dmin = ds_de * de_dmin * w + s * dw_dmin;
    out->dsw_dmed = ds_de * de_dmed * w + s * dw_dmed;
    out->dsw_dmax = s * dw_dmax;
    return true;
}

}  // namespace divas
