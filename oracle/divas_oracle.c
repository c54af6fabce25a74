/*
 * CPU ORACLE for depth-weighted voxel aggregation (DivAS, arXiv 2601.04860).
 *
 * THIS IS TEST INFRASTRUCTURE.  It is a plain, slow, obviously-correct FP64
 * implementation used only by the test suite, the smoke check and the
 * benchmark's CPU-baseline leg.  The HIP library never links, calls or
 * includes anything from this file, and this file shares no code with it.
 *
 * What it computes (each function cites the passage it follows):
 *   O0  occupancy -> Morton-ordered active list      (Sec. 3.5 "Occupancy by
 *       Morton-scattered opacity"; App. F "Occupancy grid construction")
 *   O1  per-pixel depth-gradient factor pi_dg         (App. D, Eq. for g_depth)
 *   O2  thick-path depth-weighted vote per voxel      (Alg. gs-fusion without
 *       the thin-structure call; Eqs. planar-to-ray, seethrough, asym-gate,
 *       tightening, gs-spatial, gs-depthweight, vmask)
 *   O3  compact fusion + consensus threshold          (Eq. compact-fusion)
 *   O4  label lookup                                  (Eq. pass1, Alg. vox2surfel Pass 1)
 *   OT  2DGS thin-structure fallback                  (Alg. gs-thin; Eqs. behind-gate,
 *       thin-nmin, gs-coverage, thin-d2min, thin-tthin-gs)
 *   ON  NeRF thick path and its thin path             (Alg. nerf-fusion, Alg. nerf-thin;
 *       Eqs. distance_cond, dist_tol, depth_tol, nerf-accept, nerf-vote,
 *       nerf-thindepth, nerf-support, nerf-counters, nerf-coverage, nerf-thin)
 *   OP  voxel-to-surfel Pass 3 footprint coverage     (Alg. vox2surfel Pass 3;
 *       Eqs. keys-no-depth, cov-atomics, kappa, final-F)
 *   OA  differentiable variant (soft depth test, logits) and its exact
 *       reverse-mode gradient, written vote by vote.
 *
 * Arithmetic convention (the decision-relevant quantities are evaluated in
 * the operation order written below, in IEEE binary64, without contraction
 * into fused multiply-adds; the build uses -ffp-contract=off):
 *   voxel centre   c_k = origin_k + ((double)i_k + 0.5) * h
 *   voxel corner   x_k = origin_k + (double)j_k * h,  j_k in {i_k, i_k + 1}
 *   camera coords  d = c - o;  q_a = (R[0][a]*d_0 + R[1][a]*d_1) + R[2][a]*d_2
 *   pixel coords   u = (fx*q_x)/q_z + cx,   v = (fy*q_y)/q_z + cy
 *   pixel ray      r = ((px+0.5-cx)/fx, (py+0.5-cy)/fy, 1);
 *                  w_a = (R[a][0]*r_0 + R[a][1]*r_1) + R[a][2]
 *                  n = sqrt((w_0*w_0 + w_1*w_1) + w_2*w_2);  dhat = w / n
 *   obliquity      cos = (R[0][2]*dhat_0 + R[1][2]*dhat_1) + R[2][2]*dhat_2
 * R is the rotation block of the row-major 3x4 camera-to-world matrix
 * [R | o]; its columns are the camera right, down and forward axes.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct {
    double fx, fy, cx, cy;
    double c2w[12];      /* row-major [R | o] */
    int32_t width, height;
    double d_cam;
} ocam;

typedef struct {
    double gamma, beta, gamma_st, alpha1, k_grad, eps, tau_cons, mask_gate, soft_width;
} oparams;

typedef struct {
    const float* mask;   /* mask (or logit for the differentiable variant), H x W row-major */
    const float* dmin;
    const float* dmed;
    const float* dmax;
    const uint16_t* nsamp;  /* may be NULL */
} omaps;

/* ------------------------------------------------------------------ Morton */
/* Morton (Z-order) code: bit b of x goes to bit 3b, of y to 3b+1, of z to 3b+2. */
static uint64_t morton3(uint32_t x, uint32_t y, uint32_t z) {
    uint64_t m = 0;
    for (int b = 0; b < 21; ++b) {
        m |= (uint64_t)((x >> b) & 1u) << (3 * b);
        m |= (uint64_t)((y >> b) & 1u) << (3 * b + 1);
        m |= (uint64_t)((z >> b) & 1u) << (3 * b + 2);
    }
    return m;
}

uint64_t oracle_morton3(uint32_t x, uint32_t y, uint32_t z) { return morton3(x, y, z); }

/* ------------------------------------------------------------ voxel index */
/* Voxel of a point: floor((mu - origin) / h) per axis, in binary64.  Returns 0
 * for NaN coordinates or any axis outside [0, dim) (Eq. pass1 with the AABB /
 * NaN filter of Alg. vox2surfel; the grid is given by its min corner). */
static int point_voxel(const float* p, const double* origin, double h, int32_t dim,
                       int64_t* out_lin) {
    int64_t idx[3];
    for (int k = 0; k < 3; ++k) {
        double x = (double)p[k];
        if (x != x) return 0;
        double f = floor((x - origin[k]) / h);
        if (!(f >= 0.0) || !(f < (double)dim)) return 0;
        idx[k] = (int64_t)f;
    }
    *out_lin = idx[0] + (int64_t)dim * (idx[1] + (int64_t)dim * idx[2]);
    return 1;
}

int64_t oracle_point_voxel(const float* p, const double* origin, double h, int32_t dim) {
    int64_t lin;
    return point_voxel(p, origin, h, dim, &lin) ? lin : -1;
}

/* -------------------------------------------------------------- O0 occupancy */
typedef struct { int64_t lin; int64_t pt; } pv_pair;

static int cmp_pv(const void* a, const void* b) {
    const pv_pair* x = (const pv_pair*)a;
    const pv_pair* y = (const pv_pair*)b;
    if (x->lin != y->lin) return x->lin < y->lin ? -1 : 1;
    return x->pt < y->pt ? -1 : (x->pt > y->pt ? 1 : 0);
}

typedef struct { uint64_t key; uint32_t lin; double rho; } mk_entry;

static int cmp_mk(const void* a, const void* b) {
    const mk_entry* x = (const mk_entry*)a;
    const mk_entry* y = (const mk_entry*)b;
    return x->key < y->key ? -1 : (x->key > y->key ? 1 : 0);
}

/* Density rho[v] = sum of the opacities of the points whose voxel is v (opacity
 * 1 when NULL), summed in increasing point order; active iff rho >= tau_occ
 * (the active list of the occupancy construction).  Writes the active voxels'
 * linear indices x + g*y + g*g*z sorted by Morton code and returns their
 * number.  out_rho (optional) receives rho per returned entry. */
int64_t oracle_occupancy(const float* xyz, const float* opacity, int64_t n,
                         const double* origin, double h, int32_t dim, double tau_occ,
                         uint32_t* out_lin, double* out_rho) {
    pv_pair* pv = (pv_pair*)malloc(sizeof(pv_pair) * (size_t)(n > 0 ? n : 1));
    int64_t m = 0;
    for (int64_t i = 0; i < n; ++i) {
        int64_t lin;
        if (point_voxel(xyz + 3 * i, origin, h, dim, &lin)) {
            pv[m].lin = lin;
            pv[m].pt = i;
            ++m;
        }
    }
    qsort(pv, (size_t)m, sizeof(pv_pair), cmp_pv);
    mk_entry* act = (mk_entry*)malloc(sizeof(mk_entry) * (size_t)(m > 0 ? m : 1));
    int64_t na = 0;
    for (int64_t s = 0; s < m;) {
        int64_t e = s;
        double r = 0.0;
        while (e < m && pv[e].lin == pv[s].lin) {
            r += opacity ? (double)opacity[pv[e].pt] : 1.0;
            ++e;
        }
        if (r >= tau_occ) {
            int64_t lin = pv[s].lin;
            uint32_t x = (uint32_t)(lin % dim), y = (uint32_t)((lin / dim) % dim),
                     z = (uint32_t)(lin / ((int64_t)dim * dim));
            act[na].key = morton3(x, y, z);
            act[na].lin = (uint32_t)lin;
            act[na].rho = r;
            ++na;
        }
        s = e;
    }
    /* the Morton code is a bijection of the voxel index, so the order is total */
    qsort(act, (size_t)na, sizeof(mk_entry), cmp_mk);
    for (int64_t i = 0; i < na; ++i) {
        out_lin[i] = act[i].lin;
        if (out_rho) out_rho[i] = act[i].rho;
    }
    free(pv);
    free(act);
    return na;
}

/* ----------------------------------------------------------- camera helpers */
#define R_(c, a, b) ((c)->c2w[(a) * 4 + (b)])

/* Camera coordinates of world point p (see the arithmetic convention). */
static void to_camera(const ocam* c, const double* p, double* q, double* dd) {
    double d0 = p[0] - c->c2w[3], d1 = p[1] - c->c2w[7], d2 = p[2] - c->c2w[11];
    for (int a = 0; a < 3; ++a) q[a] = (R_(c, 0, a) * d0 + R_(c, 1, a) * d1) + R_(c, 2, a) * d2;
    if (dd) { dd[0] = d0; dd[1] = d1; dd[2] = d2; }
}

/* Unit world direction of the ray through the centre of pixel (px, py) and
 * its obliquity cos = <forward, dhat> (Eq. planar-to-ray). */
static void pixel_ray(const ocam* c, int px, int py, double* dhat, double* cosv) {
    double r0 = ((double)px + 0.5 - c->cx) / c->fx;
    double r1 = ((double)py + 0.5 - c->cy) / c->fy;
    double w[3];
    for (int a = 0; a < 3; ++a) w[a] = (R_(c, a, 0) * r0 + R_(c, a, 1) * r1) + R_(c, a, 2);
    double n = sqrt((w[0] * w[0] + w[1] * w[1]) + w[2] * w[2]);
    for (int a = 0; a < 3; ++a) dhat[a] = w[a] / n;
    *cosv = (R_(c, 0, 2) * dhat[0] + R_(c, 1, 2) * dhat[1]) + R_(c, 2, 2) * dhat[2];
}

/* Pinhole projection of world point p.  Returns 1 and the continuous pixel
 * coordinates when the point is in front (q_z > eps); 0 otherwise. */
int oracle_project(const ocam* c, const double* p, double eps, double* u, double* v, double* qz) {
    double q[3];
    to_camera(c, p, q, NULL);
    *qz = q[2];
    if (!(q[2] > eps)) return 0;
    *u = (c->fx * q[0]) / q[2] + c->cx;
    *v = (c->fy * q[1]) / q[2] + c->cy;
    return 1;
}

void oracle_pixel_ray(const ocam* c, int px, int py, double* dhat, double* cosv) {
    pixel_ray(c, px, py, dhat, cosv);
}

/* ------------------------------------------------------------------ O1 pi_dg */
/* Depth-gradient factor of App. D: d = (D_min + D_max)/2, central differences
 * with clamp-to-edge neighbours, G = g_x^2 + g_y^2, pi = exp(-k G). */
static double center_depth(const omaps* m, int W, int x, int y) {
    size_t i = (size_t)y * (size_t)W + (size_t)x;
    return ((double)m->dmin[i] + (double)m->dmax[i]) / 2.0;
}

static double pi_dg_at(const omaps* m, int W, int H, int x, int y, double k) {
    int xm = x > 0 ? x - 1 : 0, xp = x < W - 1 ? x + 1 : W - 1;
    int ym = y > 0 ? y - 1 : 0, yp = y < H - 1 ? y + 1 : H - 1;
    double gx = center_depth(m, W, xp, y) - center_depth(m, W, xm, y);
    double gy = center_depth(m, W, x, yp) - center_depth(m, W, x, ym);
    double G = gx * gx + gy * gy;
    return exp(-k * G);
}

void oracle_pi_dg_map(const float* dmin, const float* dmax, int W, int H, double k, double* out) {
    omaps m = {NULL, dmin, NULL, dmax, NULL};
    for (int y = 0; y < H; ++y)
        for (int x = 0; x < W; ++x) out[(size_t)y * W + x] = pi_dg_at(&m, W, H, x, y, k);
}

/* -------------------------------------------------- footprint statistics */
/* Projected footprint of voxel (i,j,k): the pixel bounding box of its 8
 * corners, floor(min)..floor(max) inclusive, clipped to the image.  Returns 0
 * when a corner is not in front of the camera (no footprint). */
static int footprint(const ocam* c, const double* origin, double h, const int64_t* iv, double eps,
                     int* x0, int* x1, int* y0, int* y1) {
    double umin = INFINITY, umax = -INFINITY, vmin = INFINITY, vmax = -INFINITY;
    for (int j = 0; j < 8; ++j) {
        double p[3], u, v, qz;
        for (int a = 0; a < 3; ++a) p[a] = origin[a] + (double)(iv[a] + ((j >> a) & 1)) * h;
        if (!oracle_project(c, p, eps, &u, &v, &qz)) return 0;
        if (u < umin) umin = u;
        if (u > umax) umax = u;
        if (v < vmin) vmin = v;
        if (v > vmax) vmax = v;
    }
    double fx0 = floor(umin), fx1 = floor(umax), fy0 = floor(vmin), fy1 = floor(vmax);
    if (fx0 < 0.0) fx0 = 0.0;
    if (fy0 < 0.0) fy0 = 0.0;
    if (fx1 > (double)(c->width - 1)) fx1 = (double)(c->width - 1);
    if (fy1 > (double)(c->height - 1)) fy1 = (double)(c->height - 1);
    if (fx0 > fx1 || fy0 > fy1) return 0;
    *x0 = (int)fx0; *x1 = (int)fx1; *y0 = (int)fy0; *y1 = (int)fy1;
    return 1;
}

/* Layered predicate n > mean + sigma (population sigma) over the footprint,
 * evaluated exactly in integers: with A pixels, S1 = sum n, S2 = sum n^2,
 * n > S1/A + sqrt(S2/A - (S1/A)^2)  <=>  nA - S1 > 0 and (nA - S1)^2 > A S2 - S1^2.
 * E = max(n - mean, 0) (Eq. tightening) is returned in binary64. */
static void footprint_stats(const uint16_t* ns, int W, int x0, int x1, int y0, int y1, uint16_t n,
                            int* layered, double* E) {
    uint64_t S1 = 0, S2 = 0;
    for (int y = y0; y <= y1; ++y)
        for (int x = x0; x <= x1; ++x) {
            uint64_t t = ns[(size_t)y * W + x];
            S1 += t;
            S2 += t * t;
        }
    int64_t A = (int64_t)(x1 - x0 + 1) * (int64_t)(y1 - y0 + 1);
    int64_t ex = (int64_t)n * A - (int64_t)S1;
    __int128 lhs = (__int128)ex * (__int128)ex;
    __int128 rhs = (__int128)A * (__int128)S2 - (__int128)S1 * (__int128)S1;
    *layered = (ex > 0) && (lhs > rhs);
    *E = ex > 0 ? (double)ex / (double)A : 0.0;
}

void oracle_footprint_stats(const uint16_t* ns, int W, int x0, int x1, int y0, int y1, uint16_t n,
                            int* layered, double* E) {
    footprint_stats(ns, W, x0, x1, y0, y1, n, layered, E);
}

/* ------------------------------------------------------- O2/O3 the fusion */
typedef struct {
    double* P;        /* [n_act] fused probability (binary64) */
    double* W;        /* [n_act] */
    double* Z;        /* [n_act] */
    uint64_t* vraw;   /* [n_act] bitmask of accepted views (before the consensus mask) */
    uint64_t* vout;   /* [n_act] bitmask kept only for segmented voxels */
    uint8_t* seg;     /* [n_act] P >= tau_cons */
    double* margin;   /* [n_act] smallest relative slack of any spatial-gate test, or NULL */
    int64_t counts[3];/* n_seg, n_threshold_flagged (|P - tau| <= 1e-5), n_votes */
} oresult;

/* One (voxel, view) sample of the thick path (Alg. gs-fusion, thick branch).
 * Returns 1 and the weight w (and m) when the view votes for the voxel. */
static int thick_sample(const ocam* c, const omaps* mp, const oparams* pr, const double* origin,
                        double h, const int64_t* iv, const double* ctr, double* w_out,
                        double* m_out, double* margin) {
    const int W = c->width, H = c->height;
    double q[3], dd[3];
    to_camera(c, ctr, q, dd);
    if (!(q[2] > pr->eps)) return 0;                      /* behind the camera */
    double u = (c->fx * q[0]) / q[2] + c->cx;
    double v = (c->fy * q[1]) / q[2] + c->cy;
    if (!(u >= 0.0 && u < (double)W && v >= 0.0 && v < (double)H)) return 0;  /* out of frame */
    int px = (int)floor(u), py = (int)floor(v);
    size_t pix = (size_t)py * (size_t)W + (size_t)px;
    double m = (double)mp->mask[pix];
    double dmin = (double)mp->dmin[pix], dmed = (double)mp->dmed[pix], dmax = (double)mp->dmax[pix];
    if (dmed < pr->eps) return 0;                          /* no surface at this pixel */
    double xd = q[2];                                      /* planar voxel depth */
    if (!(m >= pr->mask_gate)) return 0;                   /* thick-path entry gate */
    /* planar-to-ray conversion through the sampled pixel's centre */
    double dh[3], cosv;
    pixel_ray(c, px, py, dh, &cosv);
    double dmin_r = dmin / cosv, dmed_r = dmed / cosv, dmax_r = dmax / cosv;
    /* footprint statistics (integral-image query in the paper) */
    int layered = 0;
    double E = 0.0;
    if (mp->nsamp) {
        int x0, x1, y0, y1;
        if (footprint(c, origin, h, iv, pr->eps, &x0, &x1, &y0, &y1))
            footprint_stats(mp->nsamp, W, x0, x1, y0, y1, mp->nsamp[pix], &layered, &E);
    }
    int seethru = dmed > pr->gamma_st * c->d_cam;
    int trusted = dmin <= dmed;
    if (!trusted) return 0;                                /* defer to the thin path */
    int front = layered || seethru;
    double dref_r = front ? dmin_r : dmed_r;
    double ts = (dd[0] * dh[0] + dd[1] * dh[1]) + dd[2] * dh[2];
    double th = ts < dmin_r ? dmin_r : ts;
    if (th > dref_r) th = dref_r;
    double e0 = ctr[0] - (c->c2w[3] + th * dh[0]);
    double e1 = ctr[1] - (c->c2w[7] + th * dh[1]);
    double e2 = ctr[2] - (c->c2w[11] + th * dh[2]);
    double delta = sqrt((e0 * e0 + e1 * e1) + e2 * e2);
    double tau_sp = h * pi_dg_at(mp, W, H, px, py, pr->k_grad);
    double t_depth = (pr->gamma * h) / (1.0 + pr->beta * E);
    int valid = front ? (xd - dmin <= t_depth) : (fabs(xd - dmed) <= t_depth);
    if (margin && tau_sp > 0.0) {
        double s = fabs(delta - tau_sp) / tau_sp;
        if (s < *margin) *margin = s;
    }
    if (!(delta <= tau_sp && valid)) return 0;
    double d_ctr = (dmin_r + dmax_r) / 2.0;
    double d_hw = (dmax_r - dmin_r) / 2.0;
    if (d_hw < pr->eps) d_hw = pr->eps;
    double rr = (th - d_ctr) / d_hw;
    *w_out = exp(-pr->alpha1 * (rr * rr));
    *m_out = m;
    return 1;
}

/* --------------------------------------------- thin-structure path (NEXT-1) */
typedef struct {
    double rho_thin, tau_thin, rho_cover, rho_occ, n_abs;
} othin;

/* Thin-structure score t of a voxel in one view (Alg. gs-thin; Eqs.
 * thin-d2min, thin-nmin, gs-coverage, thin-tthin-gs): a sweep of the pixels of
 * the voxel's projected footprint (the 8-corner box, floor(min)..floor(max)
 * inclusive, clipped), counting the depth-consistent pixels and, among them,
 * those with M~ > 0.5, whose unprojected surface points give the smallest
 * squared distance to the centre and whose largest M~ is the score. */
static double thin_score(const ocam* c, const omaps* mp, const oparams* pr, const othin* th,
                         const double* origin, double h, const int64_t* iv, const double* ctr, double xd) {
    const int W = c->width;
    int x0, x1, y0, y1;
    if (!footprint(c, origin, h, iv, pr->eps, &x0, &x1, &y0, &y1)) return 0.0;
    const double A = (double)(x1 - x0 + 1) * (double)(y1 - y0 + 1);   /* pixel count of the footprint */
    double n_min = ceil(th->rho_occ * A);
    if (n_min < th->n_abs) n_min = th->n_abs;
    int64_t n_depth = 0, n_md = 0;
    double m_max = 0.0, d2 = INFINITY;
    for (int y = y0; y <= y1; ++y)
        for (int x = x0; x <= x1; ++x) {
            size_t pix = (size_t)y * (size_t)W + (size_t)x;
            double m = (double)mp->mask[pix];
            double dmin = (double)mp->dmin[pix], dmed = (double)mp->dmed[pix];
            if (dmed < pr->eps) continue;                     /* no surface */
            int layered = 0;
            double E = 0.0;
            if (mp->nsamp) footprint_stats(mp->nsamp, W, x0, x1, y0, y1, mp->nsamp[pix], &layered, &E);
            double eta = 1.0 / (1.0 + pr->beta * E);
            double tau = (pr->gamma * h) * eta;
            int seethru = dmed > pr->gamma_st * c->d_cam;
            int trusted = dmin <= dmed;
            int front = (layered || seethru) && trusted;       /* Eq. asym-gate: front hit only when trusted */
            int valid = front ? (xd - dmin <= tau) : (fabs(xd - dmed) <= tau);
            if (!valid) continue;
            n_depth += 1;
            if (!(m > 0.5)) continue;
            n_md += 1;
            if (m > m_max) m_max = m;
            /* unproject the pixel centre at its layered-aware planar depth */
            double d = layered ? dmin : dmed;
            double cxp = ((double)x + 0.5 - c->cx) / c->fx * d;
            double cyp = ((double)y + 0.5 - c->cy) / c->fy * d;
            double e[3];
            for (int a = 0; a < 3; ++a)
                e[a] = (((R_(c, a, 0) * cxp + R_(c, a, 1) * cyp) + R_(c, a, 2) * d) + c->c2w[a * 4 + 3]) - ctr[a];
            double q = (e[0] * e[0] + e[1] * e[1]) + e[2] * e[2];
            if (q < d2) d2 = q;
        }
    if ((double)n_depth < n_min) return 0.0;                  /* degeneracy floor */
    double p_cov = (double)n_md / (double)n_depth;
    double g = 1.5 * h;
    if (p_cov >= th->rho_cover && d2 <= g * g) return m_max;
    return 0.0;
}

/* ------------------------------------------------ NeRF thick path (NEXT-2) */
typedef struct {
    double lambda_range, b_max;
    /* Depth semantics of the tuple.  0 (the paper's statement that both
     * renderers report camera Z): D_min, D_exp, D_max are planar, x_d is the
     * voxel's camera Z, and the ray parameter t_proj is clamped into
     * [D_min, D_max] as written, without conversion.  1: the tuple holds
     * distances along the pixel ray and x_d is t_proj. */
    int ray_depths;
    /* thin-structure path of Alg. nerf-thin (0 = off) and its constants */
    int thin;
    double rho_thin, tau_thin, rho_cover;
} onerf;

/* Unit direction of the centre ray of the pixel holding the projection of
 * ctr, its ray parameter t_proj = <ctr - o, dhat> and the camera Z. */
static void nerf_ray_terms(const ocam* c, const double* ctr, int px, int py, double* dh, double* tp, double* qz) {
    double q[3], dd[3], cosv;
    to_camera(c, ctr, q, dd);
    pixel_ray(c, px, py, dh, &cosv);
    *tp = (dd[0] * dh[0] + dd[1] * dh[1]) + dd[2] * dh[2];
    *qz = q[2];
}

/* One (voxel, view) sample of the NeRF thick path (Alg. nerf-fusion, thick
 * branch; Eqs. distance_cond, dist_tol, depth_tol, nerf-accept, nerf-vote).
 * The scene contraction is the identity and the density floor is the
 * occupancy threshold of the active list.  The mask plane holds M~, the depth
 * planes D_min, D_exp, D_max; n_samp (optional) relaxes the depth tolerance.
 * *centre_m receives the mask value at the projected pixel (for the thin
 * fallback's eligibility) and *in_frame whether there is one. */
static int nerf_sample(const ocam* c, const omaps* mp, const oparams* pr, const onerf* nr, double h,
                       const double* ctr, double* w_out, double* m_out, double* margin, int* in_frame,
                       double* centre_m, int* cpx, int* cpy) {
    const int W = c->width, H = c->height;
    double q[3], dd[3];
    *in_frame = 0;
    to_camera(c, ctr, q, dd);
    if (!(q[2] > pr->eps)) return 0;                      /* behind the camera */
    double u = (c->fx * q[0]) / q[2] + c->cx;
    double v = (c->fy * q[1]) / q[2] + c->cy;
    if (!(u >= 0.0 && u < (double)W && v >= 0.0 && v < (double)H)) return 0;  /* out of frame */
    int px = (int)floor(u), py = (int)floor(v);
    size_t pix = (size_t)py * (size_t)W + (size_t)px;
    double m = (double)mp->mask[pix];
    *in_frame = 1;
    *centre_m = m;
    *cpx = px;
    *cpy = py;
    if (!(m >= pr->mask_gate)) return 0;                   /* thick-path entry gate */
    double dmin = (double)mp->dmin[pix], dexp = (double)mp->dmed[pix], dmax = (double)mp->dmax[pix];
    if (dexp < pr->eps) return 0;                          /* no surface at this pixel */
    double ns = mp->nsamp ? (double)mp->nsamp[pix] : 0.0;
    /* closest point of the ray segment [d_min, d_max] to the voxel centre */
    double dh[3], tp, qz;
    nerf_ray_terms(c, ctr, px, py, dh, &tp, &qz);
    double tc = tp < dmin ? dmin : tp;
    if (tc > dmax) tc = dmax;
    double e0 = ctr[0] - (c->c2w[3] + tc * dh[0]);
    double e1 = ctr[1] - (c->c2w[7] + tc * dh[1]);
    double e2 = ctr[2] - (c->c2w[11] + tc * dh[2]);
    double delta = sqrt((e0 * e0 + e1 * e1) + e2 * e2);
    /* spatial tolerance with the band slack, depth tolerance with the bonus */
    double tau_sp = h * pi_dg_at(mp, W, H, px, py, pr->k_grad) + nr->lambda_range * (dmax - dmin);
    double b = pr->beta * ns;
    if (b > nr->b_max) b = nr->b_max;
    double tau_d = (pr->gamma + b) * h;
    double xd = nr->ray_depths ? tp : qz;                  /* the voxel's depth in this view */
    if (margin && tau_sp > 0.0) {
        double s = fabs(delta - tau_sp) / tau_sp;
        if (s < *margin) *margin = s;
    }
    if (!(delta <= tau_sp && fabs(xd - dexp) <= tau_d)) return 0;
    /* Gaussian fall-off from the band midpoint */
    double mu = (dmin + dmax) / 2.0;
    double hd = (dmax - dmin) / 2.0;
    if (hd < pr->eps) hd = pr->eps;
    double r = fabs(tc - mu) / hd;
    *w_out = exp(-pr->alpha1 * (r * r));
    *m_out = m;
    return 1;
}

/* Thin-structure score of a voxel in one view under the NeRF path (Alg.
 * nerf-thin; Eqs. nerf-thindepth, nerf-support, nerf-counters, nerf-coverage,
 * nerf-thin): over the footprint (the pixel box of the 8 projected corners,
 * floor(min)..floor(max) inclusive, clipped; N_pixels its pixel count) count
 * the supportive pixels (M~ > 0.5 and |x_d - D_exp| <= (2 gamma + b) h with
 * the pixel's own capped bonus b) and take the largest M~ of any footprint
 * pixel; the score is that peak when the supportive fraction reaches
 * rho_cover, else 0. */
static double nerf_thin_score(const ocam* c, const omaps* mp, const oparams* pr, const onerf* nr,
                              const double* origin, double h, const int64_t* iv, double xd) {
    const int W = c->width;
    int x0, x1, y0, y1;
    if (!footprint(c, origin, h, iv, pr->eps, &x0, &x1, &y0, &y1)) return 0.0;
    const double n_pixels = (double)(x1 - x0 + 1) * (double)(y1 - y0 + 1);
    int64_t n_valid = 0;
    double m_max = 0.0;
    for (int y = y0; y <= y1; ++y)
        for (int x = x0; x <= x1; ++x) {
            size_t pix = (size_t)y * (size_t)W + (size_t)x;
            double m = (double)mp->mask[pix];
            double dexp = (double)mp->dmed[pix];
            double ns = mp->nsamp ? (double)mp->nsamp[pix] : 0.0;
            double b = pr->beta * ns;
            if (b > nr->b_max) b = nr->b_max;
            double tau = (2.0 * pr->gamma + b) * h;
            if (m > 0.5 && fabs(xd - dexp) <= tau) n_valid += 1;
            if (m > m_max) m_max = m;
        }
    double p_cov = (double)n_valid / n_pixels;
    return p_cov >= nr->rho_cover ? m_max : 0.0;
}

static void voxel_coords(uint32_t lin, int32_t dim, int64_t* iv) {
    iv[0] = (int64_t)(lin % (uint32_t)dim);
    iv[1] = (int64_t)((lin / (uint32_t)dim) % (uint32_t)dim);
    iv[2] = (int64_t)(lin / ((uint32_t)dim * (uint32_t)dim));
}

static void voxel_center(const double* origin, double h, const int64_t* iv, double* ctr) {
    for (int a = 0; a < 3; ++a) ctr[a] = origin[a] + ((double)iv[a] + 0.5) * h;
}

/* Thick-path fusion of all views over the active list, then the compact-fusion
 * rule and the consensus threshold.  Views are visited in increasing index and
 * their votes accumulated in binary64 in that order.  nr == NULL: the 2DGS
 * thick path; otherwise the NeRF thick path with those constants. */
static void fuse_all(const uint32_t* act, int64_t n_act, const double* origin, double h, int32_t dim,
                     int32_t n_views, const ocam* cams, const omaps* maps, const oparams* pr, const onerf* nr,
                     const othin* th, const double* rho, int n_threads, oresult* out) {
    int64_t nseg = 0, nflag = 0, nvotes = 0;
#ifdef _OPENMP
    if (n_threads > 0) omp_set_num_threads(n_threads);
#pragma omp parallel for schedule(static) reduction(+ : nseg, nflag, nvotes)
#endif
    for (int64_t a = 0; a < n_act; ++a) {
        int64_t iv[3];
        double ctr[3];
        voxel_coords(act[a], dim, iv);
        voxel_center(origin, h, iv, ctr);
        double Wx = 0.0, Zx = 0.0, mg = INFINITY;
        uint64_t vm = 0;
        for (int s = 0; s < n_views; ++s) {
            double w, m, cm = 0.0;
            int in_frame = 0, cpx = 0, cpy = 0;
            const int vote = nr ? nerf_sample(&cams[s], &maps[s], pr, nr, h, ctr, &w, &m, &mg, &in_frame, &cm,
                                              &cpx, &cpy)
                                : thick_sample(&cams[s], &maps[s], pr, origin, h, iv, ctr, &w, &m, &mg);
            if (vote) {
                Wx += m * w;
                Zx += w;
                vm |= (uint64_t)1 << s;
            } else if (nr && nr->thin) {
                /* thin fallback of Alg. nerf-fusion: the centre in frame, a
                 * non-trivial mask there (> 0.1) and the thin density floor */
                if (!in_frame || !(cm > 0.1) || !(rho[a] >= nr->rho_thin)) continue;
                double dh[3], tp, qz;
                nerf_ray_terms(&cams[s], ctr, cpx, cpy, dh, &tp, &qz);
                double t = nerf_thin_score(&cams[s], &maps[s], pr, nr, origin, h, iv, nr->ray_depths ? tp : qz);
                if (t >= nr->tau_thin) {
                    Wx += t;
                    Zx += 1.0;
                    vm |= (uint64_t)1 << s;
                }
            } else if (th) {
                /* thin fallback of Alg. gs-fusion: the centre in frame, the
                 * behind-surface gate (Eq. behind-gate) and the density floor */
                const ocam* c = &cams[s];
                double q[3];
                to_camera(c, ctr, q, NULL);
                if (!(q[2] > pr->eps)) continue;
                double u = (c->fx * q[0]) / q[2] + c->cx;
                double v = (c->fy * q[1]) / q[2] + c->cy;
                if (!(u >= 0.0 && u < (double)c->width && v >= 0.0 && v < (double)c->height)) continue;
                size_t pix = (size_t)floor(v) * (size_t)c->width + (size_t)floor(u);
                double dmin = (double)maps[s].dmin[pix], dmed = (double)maps[s].dmed[pix];
                int trusted = dmin <= dmed;
                int seethru = dmed > pr->gamma_st * c->d_cam;
                double d_surf = (trusted && seethru) ? dmin : dmed;
                if (q[2] > d_surf + 2.0 * h) continue;             /* behind the visible surface */
                if (!(rho[a] >= th->rho_thin)) continue;
                double t = thin_score(c, &maps[s], pr, th, origin, h, iv, ctr, q[2]);
                if (t >= th->tau_thin) {
                    Wx += t;
                    Zx += 1.0;
                    vm |= (uint64_t)1 << s;
                }
            }
        }
        double P = Zx > pr->eps ? Wx / Zx : 0.0;
        int seg = P >= pr->tau_cons;
        out->P[a] = P;
        if (out->W) out->W[a] = Wx;
        if (out->Z) out->Z[a] = Zx;
        out->vraw[a] = vm;
        out->vout[a] = seg ? vm : 0;
        out->seg[a] = (uint8_t)seg;
        if (out->margin) out->margin[a] = mg;
        nseg += seg;
        nflag += fabs(P - pr->tau_cons) <= 1e-5;
        nvotes += __builtin_popcountll(vm);
    }
    out->counts[0] = nseg;
    out->counts[1] = nflag;
    out->counts[2] = nvotes;
}

void oracle_fuse(const uint32_t* act, int64_t n_act, const double* origin, double h, int32_t dim,
                 int32_t n_views, const ocam* cams, const omaps* maps, const oparams* pr,
                 int n_threads, oresult* out) {
    fuse_all(act, n_act, origin, h, dim, n_views, cams, maps, pr, NULL, NULL, NULL, n_threads, out);
}

/* The 2DGS fusion with the thin-structure fallback: rho[a] is the density of
 * active voxel a (summed opacity of its points). */
void oracle_fuse_thin(const uint32_t* act, int64_t n_act, const double* origin, double h, int32_t dim,
                      int32_t n_views, const ocam* cams, const omaps* maps, const oparams* pr, const double* rho,
                      double rho_thin, double tau_thin, double rho_cover, double rho_occ, double n_abs,
                      int n_threads, oresult* out) {
    const othin th = {rho_thin, tau_thin, rho_cover, rho_occ, n_abs};
    fuse_all(act, n_act, origin, h, dim, n_views, cams, maps, pr, NULL, &th, rho, n_threads, out);
}

/* The NeRF fusion (thick path, plus the thin path when nr->thin): rho[a] is
 * the density of active voxel a, read only by the thin path (may be NULL
 * otherwise). */
void oracle_fuse_nerf(const uint32_t* act, int64_t n_act, const double* origin, double h, int32_t dim,
                      int32_t n_views, const ocam* cams, const omaps* maps, const oparams* pr,
                      const onerf* nr, const double* rho, int n_threads, oresult* out) {
    fuse_all(act, n_act, origin, h, dim, n_views, cams, maps, pr, nr, NULL, rho, n_threads, out);
}

/* ------------------------------------------------------------ O4 labels */
static int cmp_u32(const void* a, const void* b) {
    uint32_t x = *(const uint32_t*)a, y = *(const uint32_t*)b;
    return x < y ? -1 : (x > y ? 1 : 0);
}

/* label = 1 iff the point's voxel is a segmented voxel (Eq. pass1). */
void oracle_label(const float* xyz, int64_t n, const double* origin, double h, int32_t dim,
                  const uint32_t* seg_lin, int64_t n_seg, uint8_t* labels) {
    uint32_t* s = (uint32_t*)malloc(sizeof(uint32_t) * (size_t)(n_seg > 0 ? n_seg : 1));
    memcpy(s, seg_lin, sizeof(uint32_t) * (size_t)n_seg);
    qsort(s, (size_t)n_seg, sizeof(uint32_t), cmp_u32);
    for (int64_t i = 0; i < n; ++i) {
        int64_t lin;
        labels[i] = 0;
        if (!point_voxel(xyz + 3 * i, origin, h, dim, &lin)) continue;
        uint32_t key = (uint32_t)lin;
        labels[i] = bsearch(&key, s, (size_t)n_seg, sizeof(uint32_t), cmp_u32) != NULL;
    }
    free(s);
}

/* ------------------------------------- voxel-to-surfel Pass 3 (NEXT-3) */
/* Rotation of the unit quaternion q = (w, x, y, z) (normalised here in
 * binary64); column k of Rm is the surfel's k-th local axis in world space
 * (columns 0 and 1 span the tangent plane). */
static int quat_rotation(const float* q4, double* Rm) {
    double w = q4[0], x = q4[1], y = q4[2], z = q4[3];
    double n = sqrt(((w * w + x * x) + y * y) + z * z);
    if (!(n > 0.0) || !isfinite(n)) return 0;
    w /= n; x /= n; y /= n; z /= n;
    Rm[0] = 1.0 - 2.0 * (y * y + z * z); Rm[1] = 2.0 * (x * y - w * z);       Rm[2] = 2.0 * (x * z + w * y);
    Rm[3] = 2.0 * (x * y + w * z);       Rm[4] = 1.0 - 2.0 * (x * x + z * z); Rm[5] = 2.0 * (y * z - w * x);
    Rm[6] = 2.0 * (x * z - w * y);       Rm[7] = 2.0 * (y * z + w * x);       Rm[8] = 1.0 - 2.0 * (x * x + y * y);
    return 1;
}

/* Camera-frame image of a world direction (rotation only). */
static void dir_to_camera(const ocam* c, const double* t, double* q) {
    for (int a = 0; a < 3; ++a) q[a] = (R_(c, 0, a) * t[0] + R_(c, 1, a) * t[1]) + R_(c, 2, a) * t[2];
}

/* Coverage counts of one surfel in one view (Alg. vox2surfel Pass 3, steps
 * (ii) and (iv); Eq. cov-atomics).  The two tangent semi-axes t_k = s_k R e_k
 * and the centre are taken to the camera frame (a, A, B); the centre and the
 * four tips a +- A, a +- B must lie in front of the camera, else the view
 * does not score the surfel (returns 0).  The projected tangent vectors are
 * alpha_k = (pi(tip_k+) - pi(tip_k-)) / 2, the 1-sigma box is
 * [c_x - e_x, c_x + e_x] x [c_y - e_y, c_y + e_y] with e the larger |alpha| per
 * image axis, and its pixels floor(lo)..floor(hi) (clipped) are visited.  A
 * visited pixel is accepted when the ray through its centre meets the surfel
 * plane, in front of the camera, at tangent coordinates (u, v) (units of the
 * two scales) with u^2 + v^2 <= 9 (the 3-sigma test); the 2 x 2 system of the
 * two image-plane conditions is solved by Cramer's rule.  Accepted pixels
 * count towards *total, those with M~ >= tau_M also towards *mask_hit. */
static int surfel_view_counts(const ocam* c, const float* mask, double tau_M, double eps, const double* mu,
                              const double* t0, const double* t1, int64_t* total, int64_t* mask_hit) {
    double a[3], A[3], B[3];
    to_camera(c, mu, a, NULL);
    dir_to_camera(c, t0, A);
    dir_to_camera(c, t1, B);
    if (!(a[2] > eps)) return 0;
    double tip[4][3];
    for (int k = 0; k < 3; ++k) {
        tip[0][k] = a[k] + A[k];
        tip[1][k] = a[k] - A[k];
        tip[2][k] = a[k] + B[k];
        tip[3][k] = a[k] - B[k];
    }
    double pu[4], pv[4];
    for (int j = 0; j < 4; ++j) {
        if (!(tip[j][2] > eps)) return 0;
        pu[j] = (c->fx * tip[j][0]) / tip[j][2] + c->cx;
        pv[j] = (c->fy * tip[j][1]) / tip[j][2] + c->cy;
    }
    double cu = (c->fx * a[0]) / a[2] + c->cx;
    double cv = (c->fy * a[1]) / a[2] + c->cy;
    double ax0 = (pu[0] - pu[1]) / 2.0, ay0 = (pv[0] - pv[1]) / 2.0;
    double ax1 = (pu[2] - pu[3]) / 2.0, ay1 = (pv[2] - pv[3]) / 2.0;
    double ex = fmax(fabs(ax0), fabs(ax1)), ey = fmax(fabs(ay0), fabs(ay1));
    double fx0 = floor(cu - ex), fx1 = floor(cu + ex), fy0 = floor(cv - ey), fy1 = floor(cv + ey);
    if (fx0 < 0.0) fx0 = 0.0;
    if (fy0 < 0.0) fy0 = 0.0;
    if (fx1 > (double)(c->width - 1)) fx1 = (double)(c->width - 1);
    if (fy1 > (double)(c->height - 1)) fy1 = (double)(c->height - 1);
    *total = 0;
    *mask_hit = 0;
    if (fx0 > fx1 || fy0 > fy1) return 1;
    for (int y = (int)fy0; y <= (int)fy1; ++y)
        for (int x = (int)fx0; x <= (int)fx1; ++x) {
            double xi = ((double)x + 0.5 - c->cx) / c->fx;
            double zeta = ((double)y + 0.5 - c->cy) / c->fy;
            double m00 = A[0] - xi * A[2], m01 = B[0] - xi * B[2];
            double m10 = A[1] - zeta * A[2], m11 = B[1] - zeta * B[2];
            double r0 = xi * a[2] - a[0], r1 = zeta * a[2] - a[1];
            double det = m00 * m11 - m01 * m10;
            if (det == 0.0) continue;
            double u = (r0 * m11 - m01 * r1) / det;
            double v = (m00 * r1 - r0 * m10) / det;
            double z = (a[2] + u * A[2]) + v * B[2];
            if (!(u * u + v * v <= 9.0) || !(z > eps)) continue;
            *total += 1;
            if ((double)mask[(size_t)y * (size_t)c->width + (size_t)x] >= tau_M) *mask_hit += 1;
        }
    return 1;
}

typedef struct { uint32_t lin; int64_t idx; } lin_idx;

static int cmp_lin(const void* a, const void* b) {
    uint32_t x = ((const lin_idx*)a)->lin, y = ((const lin_idx*)b)->lin;
    return x < y ? -1 : (x > y ? 1 : 0);
}

/* Pass 3 of Alg. vox2surfel (Eqs. keys-no-depth, cov-atomics, kappa,
 * final-F): for every surfel i with labels_in[i] = 1 (the Pass 2 labels) and
 * every view s whose bit is set in the view-coverage bitmask of the surfel's
 * voxel (the voxel of its centre, as in Pass 1; vmask[a] is the fusion's
 * Eq. vmask output of active voxel a), kappa_s = mask_hit / max(total, 1) in
 * binary64 and kappa_i = max over those views (0 when none); labels_out[i] =
 * labels_in[i] and kappa_i >= tau_kappa.  Surfel i has centre xyz[3i..],
 * tangent scales scales[2i..] and rotation quats[4i..] (w, x, y, z).
 * Returns the number of surfels kept. */
int64_t oracle_surfel_coverage(const float* xyz, const float* scales, const float* quats, int64_t n,
                               const uint8_t* labels_in, const double* origin, double h, int32_t dim,
                               const uint32_t* act, int64_t n_act, const uint64_t* vmask, int32_t n_views,
                               const ocam* cams, const omaps* maps, double tau_M, double tau_kappa, double eps,
                               double* kappa, uint8_t* labels_out) {
    lin_idx* sorted = (lin_idx*)malloc(sizeof(lin_idx) * (size_t)(n_act > 0 ? n_act : 1));
    for (int64_t i = 0; i < n_act; ++i) {
        sorted[i].lin = act[i];
        sorted[i].idx = i;
    }
    qsort(sorted, (size_t)n_act, sizeof(lin_idx), cmp_lin);
    int64_t kept = 0;
    for (int64_t i = 0; i < n; ++i) {
        double k_i = 0.0;
        labels_out[i] = 0;
        kappa[i] = 0.0;
        if (!labels_in[i]) continue;
        int64_t lin;
        uint64_t vm = 0;
        if (point_voxel(xyz + 3 * i, origin, h, dim, &lin)) {
            lin_idx key = {(uint32_t)lin, 0};
            const lin_idx* hit = (const lin_idx*)bsearch(&key, sorted, (size_t)n_act, sizeof(lin_idx), cmp_lin);
            if (hit) vm = vmask[hit->idx];
        }
        double Rm[9];
        if (vm && quat_rotation(quats + 4 * i, Rm)) {
            double mu[3], t0[3], t1[3];
            for (int k = 0; k < 3; ++k) {
                mu[k] = (double)xyz[3 * i + k];
                t0[k] = (double)scales[2 * i] * Rm[3 * k + 0];
                t1[k] = (double)scales[2 * i + 1] * Rm[3 * k + 1];
            }
            for (int s = 0; s < n_views; ++s) {
                if (!((vm >> s) & 1u)) continue;                 /* step (i): view gating */
                int64_t total, hitc;
                if (!surfel_view_counts(&cams[s], maps[s].mask, tau_M, eps, mu, t0, t1, &total, &hitc)) continue;
                double ks = (double)hitc / (double)(total > 1 ? total : 1);
                if (ks > k_i) k_i = ks;
            }
        }
        kappa[i] = k_i;
        labels_out[i] = k_i >= tau_kappa;
        kept += labels_out[i];
    }
    free(sorted);
    return kept;
}

/* Coverage counts of one surfel in one view (for the pins). */
int oracle_surfel_view_counts(const ocam* c, const float* mask, double tau_M, double eps, const float* xyz,
                              const float* scale2, const float* quat, int64_t* total, int64_t* mask_hit) {
    double Rm[9], mu[3], t0[3], t1[3];
    if (!quat_rotation(quat, Rm)) return 0;
    for (int k = 0; k < 3; ++k) {
        mu[k] = (double)xyz[k];
        t0[k] = (double)scale2[0] * Rm[3 * k + 0];
        t1[k] = (double)scale2[1] * Rm[3 * k + 1];
    }
    return surfel_view_counts(c, mask, tau_M, eps, mu, t0, t1, total, mask_hit);
}

/* --------------------------------------------- OA differentiable variant */
/* Differentiable form of the thick path used to refine 2D masks from a 3D
 * consistency loss.  Not a construct of the paper, which is optimisation-free;
 * it replaces the hard parts that carry the 2D evidence by smooth ones:
 *   m = sigmoid(logit) at the projected pixel; every in-frame view with a
 *   surface votes (mask gate 0); the depth gate becomes
 *   s = sigmoid((gamma h - e) / w_s) with e = |x_d - D_med| (or x_d - D_min
 *   for see-through pixels); the spatial gate stays hard;
 *   W += m s w, Z += s w, P = W / Z (Z > eps, else 0).
 * No n_samp statistics are used (E = 0, layered = false). */
static double sigm(double x) { return 1.0 / (1.0 + exp(-x)); }

typedef struct {
    size_t pix;
    int lo, hi, front, hw_floor;  /* branches taken: clamps, front reference, half-width floor */
    double m, s, w;           /* mask, soft depth test, depth weight */
    double dm_dl;             /* dm / dlogit */
    double dsw_dmin, dsw_dmed, dsw_dmax;  /* d(s*w) / d(planar depths) */
} dvote;

static int diff_sample(const ocam* c, const omaps* mp, const oparams* pr, double h,
                       const double* ctr, dvote* out) {
    const int W = c->width, H = c->height;
    double q[3], dd[3];
    to_camera(c, ctr, q, dd);
    if (!(q[2] > pr->eps)) return 0;
    double u = (c->fx * q[0]) / q[2] + c->cx;
    double v = (c->fy * q[1]) / q[2] + c->cy;
    if (!(u >= 0.0 && u < (double)W && v >= 0.0 && v < (double)H)) return 0;
    int px = (int)floor(u), py = (int)floor(v);
    size_t pix = (size_t)py * (size_t)W + (size_t)px;
    double lg = (double)mp->mask[pix];
    double dmin = (double)mp->dmin[pix], dmed = (double)mp->dmed[pix], dmax = (double)mp->dmax[pix];
    if (dmed < pr->eps) return 0;
    double xd = q[2];
    double dh[3], cosv;
    pixel_ray(c, px, py, dh, &cosv);
    double dmin_r = dmin / cosv, dmed_r = dmed / cosv, dmax_r = dmax / cosv;
    int seethru = dmed > pr->gamma_st * c->d_cam;
    if (!(dmin <= dmed)) return 0;
    int front = seethru;
    double dref_r = front ? dmin_r : dmed_r;
    double ts = (dd[0] * dh[0] + dd[1] * dh[1]) + dd[2] * dh[2];
    int lo_clamp = ts < dmin_r;
    double th = lo_clamp ? dmin_r : ts;
    int hi_clamp = th > dref_r;
    if (hi_clamp) th = dref_r;
    double e0 = ctr[0] - (c->c2w[3] + th * dh[0]);
    double e1 = ctr[1] - (c->c2w[7] + th * dh[1]);
    double e2 = ctr[2] - (c->c2w[11] + th * dh[2]);
    double delta = sqrt((e0 * e0 + e1 * e1) + e2 * e2);
    double tau_sp = h * pi_dg_at(mp, W, H, px, py, pr->k_grad);
    if (!(delta <= tau_sp)) return 0;
    /* soft depth test */
    double e, de_dmin = 0.0, de_dmed = 0.0;
    if (front) { e = xd - dmin; de_dmin = -1.0; }
    else { e = fabs(xd - dmed); de_dmed = (xd - dmed) > 0.0 ? -1.0 : ((xd - dmed) < 0.0 ? 1.0 : 0.0); }
    double s = sigm((pr->gamma * h - e) / pr->soft_width);
    double ds_de = -s * (1.0 - s) / pr->soft_width;
    /* depth weight */
    double d_ctr = (dmin_r + dmax_r) / 2.0;
    double hw_raw = (dmax_r - dmin_r) / 2.0;
    int hw_floor = hw_raw < pr->eps;
    double d_hw = hw_floor ? pr->eps : hw_raw;
    double rr = (th - d_ctr) / d_hw;
    double w = exp(-pr->alpha1 * (rr * rr));
    double dw_dr = -2.0 * pr->alpha1 * rr * w;
    /* r = (th - d_ctr) / d_hw ; partials w.r.t. the ray-space depths */
    double dth_dminr = lo_clamp && !hi_clamp ? 1.0 : 0.0;
    double dth_drefr = hi_clamp ? 1.0 : 0.0;
    double dr_dth = 1.0 / d_hw;
    double dr_dctr = -1.0 / d_hw;
    double dr_dhw = hw_floor ? 0.0 : -rr / d_hw;
    double dr_dminr = dr_dth * dth_dminr + dr_dctr * 0.5 + dr_dhw * (-0.5);
    double dr_dmaxr = dr_dctr * 0.5 + dr_dhw * 0.5;
    double dr_dmedr = 0.0;
    if (front) dr_dminr += dr_dth * dth_drefr; else dr_dmedr += dr_dth * dth_drefr;
    /* chain to planar depths: d_r = d / cos */
    double dw_dmin = dw_dr * dr_dminr / cosv;
    double dw_dmed = dw_dr * dr_dmedr / cosv;
    double dw_dmax = dw_dr * dr_dmaxr / cosv;
    out->pix = pix;
    out->lo = lo_clamp;
    out->hi = hi_clamp;
    out->front = front;
    out->hw_floor = hw_floor;
    out->m = sigm(lg);
    out->dm_dl = out->m * (1.0 - out->m);
    out->s = s;
    out->w = w;
    out->dsw_dmin = ds_de * de_dmin * w + s * dw_dmin;
    out->dsw_dmed = ds_de * de_dmed * w + s * dw_dmed;
    out->dsw_dmax = s * dw_dmax;
    return 1;
}

/* Forward of the differentiable variant: P, W, Z per active voxel. */
void oracle_fuse_diff(const uint32_t* act, int64_t n_act, const double* origin, double h,
                      int32_t dim, int32_t n_views, const ocam* cams, const omaps* maps,
                      const oparams* pr, double* P, double* Wo, double* Zo) {
    for (int64_t a = 0; a < n_act; ++a) {
        int64_t iv[3];
        double ctr[3];
        voxel_coords(act[a], dim, iv);
        voxel_center(origin, h, iv, ctr);
        double Wx = 0.0, Zx = 0.0;
        for (int s = 0; s < n_views; ++s) {
            dvote dv;
            if (diff_sample(&cams[s], &maps[s], pr, h, ctr, &dv)) {
                Wx += dv.m * (dv.s * dv.w);
                Zx += dv.s * dv.w;
            }
        }
        P[a] = Zx > pr->eps ? Wx / Zx : 0.0;
        if (Wo) Wo[a] = Wx;
        if (Zo) Zo[a] = Zx;
    }
}

/* Reverse mode: given dL/dP per voxel, accumulate dL/dlogit and dL/d(depths)
 * per pixel of every view.  With P = W/Z and one vote contributing m*s*w to W
 * and s*w to Z:  dP/dm = s w / Z,  dP/d(s w) = (m - P) / Z.  Gradient arrays
 * are H*W per view, zero-initialised here, accumulated in voxel order. */
void oracle_fuse_diff_grad(const uint32_t* act, int64_t n_act, const double* origin, double h,
                           int32_t dim, int32_t n_views, const ocam* cams, const omaps* maps,
                           const oparams* pr, const double* gP, double** g_logit,
                           double** g_dmin, double** g_dmed, double** g_dmax) {
    for (int s = 0; s < n_views; ++s) {
        size_t npx = (size_t)cams[s].width * (size_t)cams[s].height;
        if (g_logit && g_logit[s]) memset(g_logit[s], 0, npx * sizeof(double));
        if (g_dmin && g_dmin[s]) memset(g_dmin[s], 0, npx * sizeof(double));
        if (g_dmed && g_dmed[s]) memset(g_dmed[s], 0, npx * sizeof(double));
        if (g_dmax && g_dmax[s]) memset(g_dmax[s], 0, npx * sizeof(double));
    }
    for (int64_t a = 0; a < n_act; ++a) {
        int64_t iv[3];
        double ctr[3];
        voxel_coords(act[a], dim, iv);
        voxel_center(origin, h, iv, ctr);
        double Wx = 0.0, Zx = 0.0;
        for (int s = 0; s < n_views; ++s) {
            dvote dv;
            if (diff_sample(&cams[s], &maps[s], pr, h, ctr, &dv)) {
                Wx += dv.m * (dv.s * dv.w);
                Zx += dv.s * dv.w;
            }
        }
        if (!(Zx > pr->eps) || gP[a] == 0.0) continue;
        double P = Wx / Zx;
        for (int s = 0; s < n_views; ++s) {
            dvote dv;
            if (!diff_sample(&cams[s], &maps[s], pr, h, ctr, &dv)) continue;
            double g = gP[a] / Zx;
            double gsw = g * (dv.m - P);
            if (g_logit && g_logit[s]) g_logit[s][dv.pix] += g * (dv.s * dv.w) * dv.dm_dl;
            if (g_dmin && g_dmin[s]) g_dmin[s][dv.pix] += gsw * dv.dsw_dmin;
            if (g_dmed && g_dmed[s]) g_dmed[s][dv.pix] += gsw * dv.dsw_dmed;
            if (g_dmax && g_dmax[s]) g_dmax[s][dv.pix] += gsw * dv.dsw_dmax;
        }
    }
}

/* Which branches of the differentiable vote the voxels with coef != 0 take
 * (a test diagnostic): out[0] votes, out[1] lower clamps, out[2] upper
 * clamps, out[3] front references, out[4] half-width floors, out[5] pixels
 * receiving >= 3 votes, out[6] the most votes one pixel receives. */
void oracle_fuse_diff_branches(const uint32_t* act, int64_t n_act, const double* origin, double h, int32_t dim,
                               int32_t n_views, const ocam* cams, const omaps* maps, const oparams* pr,
                               const double* coef, int64_t* out) {
    for (int k = 0; k < 7; ++k) out[k] = 0;
    for (int s = 0; s < n_views; ++s) {
        size_t npx = (size_t)cams[s].width * (size_t)cams[s].height;
        int32_t* cnt = (int32_t*)calloc(npx, sizeof(int32_t));
        for (int64_t a = 0; a < n_act; ++a) {
            if (coef[a] == 0.0) continue;
            int64_t iv[3];
            double ctr[3];
            voxel_coords(act[a], dim, iv);
            voxel_center(origin, h, iv, ctr);
            dvote dv;
            if (!diff_sample(&cams[s], &maps[s], pr, h, ctr, &dv)) continue;
            out[0] += 1;
            out[1] += dv.lo;
            out[2] += dv.hi;
            out[3] += dv.front;
            out[4] += dv.hw_floor;
            cnt[dv.pix] += 1;
        }
        for (size_t i = 0; i < npx; ++i) {
            out[5] += cnt[i] >= 3;
            if (cnt[i] > out[6]) out[6] = cnt[i];
        }
        free(cnt);
    }
}

int oracle_num_threads(void) {
#ifdef _OPENMP
    int n = 0;
#pragma omp parallel
    {
#pragma omp single
        n = omp_get_num_threads();
    }
    return n;
#else
    return 1;
#endif
}
