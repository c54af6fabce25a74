"""Mutation check of the oracle's pins (CPU only).

Each mutant plants one plausible mistake in the C oracle (a dropped term, a
flipped comparison, a wrong index, a wrong reference depth, a transposed
operand).  It is compiled into a temporary directory and the oracle pins are
run against it through DIVAS_ORACLE_LIB; every mutant must fail at least one
pin.  The committed source is never modified.
"""
import concurrent.futures as cf
import os
import subprocess
import sys
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "divas_oracle.c")
PINS = sorted(os.path.join("tests", f) for f in os.listdir(os.path.join(ROOT, "tests"))
              if f.startswith("test_oracle_") and f.endswith(".py") and f != os.path.basename(__file__))

# (name, text to replace, replacement, which occurrence (1-based))
MUTANTS = [
    # thick path (Alg. gs-fusion, Eqs. planar-to-ray, asym-gate, tightening, gs-spatial, gs-depthweight)
    ("front gate with an absolute value", "(xd - dmin <= t_depth)", "(fabs(xd - dmin) <= t_depth)", 1),
    ("median gate one-sided", "(fabs(xd - dmed) <= t_depth)", "(xd - dmed <= t_depth)", 1),
    ("tightening multiplies", "(pr->gamma * h) / (1.0 + pr->beta * E)", "(pr->gamma * h) * (1.0 + pr->beta * E)", 1),
    ("planar-to-ray multiplies", "double dmin_r = dmin / cosv, dmed_r = dmed / cosv, dmax_r = dmax / cosv;",
     "double dmin_r = dmin * cosv, dmed_r = dmed * cosv, dmax_r = dmax * cosv;", 1),
    ("no planar-to-ray", "double dmin_r = dmin / cosv, dmed_r = dmed / cosv, dmax_r = dmax / cosv;",
     "double dmin_r = dmin, dmed_r = dmed, dmax_r = dmax;", 1),
    ("see-through reversed", "int seethru = dmed > pr->gamma_st * c->d_cam;", "int seethru = dmed < pr->gamma_st * c->d_cam;", 1),
    ("front reference swapped", "double dref_r = front ? dmin_r : dmed_r;", "double dref_r = front ? dmed_r : dmin_r;", 1),
    ("no lower clamp", "double th = ts < dmin_r ? dmin_r : ts;", "double th = ts;", 1),
    ("no depth-gradient factor", "double tau_sp = h * pi_dg_at(mp, W, H, px, py, pr->k_grad);", "double tau_sp = h;", 1),
    ("weight centre at the median", "double d_ctr = (dmin_r + dmax_r) / 2.0;", "double d_ctr = (dmin_r + dmed_r) / 2.0;", 1),
    ("weight half-width doubled", "double d_hw = (dmax_r - dmin_r) / 2.0;", "double d_hw = (dmax_r - dmin_r);", 1),
    ("untrusted pixels vote", "if (!trusted) return 0;", ";", 1),
    ("strict mask gate", "if (!(m >= pr->mask_gate)) return 0;", "if (!(m > pr->mask_gate)) return 0;", 1),
    ("pixel rounded", "int px = (int)floor(u), py = (int)floor(v);", "int px = (int)round(u), py = (int)floor(v);", 1),
    ("ray through the pixel corner", "double r0 = ((double)px + 0.5 - c->cx) / c->fx;",
     "double r0 = ((double)px - c->cx) / c->fx;", 1),
    ("vote weight dropped", "Wx += m * w;\n                Zx += w;", "Wx += m;\n                Zx += 1.0;", 1),
    ("strict consensus", "int seg = P >= pr->tau_cons;", "int seg = P > pr->tau_cons;", 1),
    ("bitmask not masked", "out->vout[a] = seg ? vm : 0;", "out->vout[a] = vm;", 1),
    ("voxel centre at the corner", "ctr[a] = origin[a] + ((double)iv[a] + 0.5) * h;", "ctr[a] = origin[a] + ((double)iv[a]) * h;", 1),
    ("projection uses y for u", "double u = (c->fx * q[0]) / q[2] + c->cx;", "double u = (c->fx * q[1]) / q[2] + c->cx;", 1),
    ("camera rotation transposed", "q[a] = (R_(c, 0, a) * d0 + R_(c, 1, a) * d1) + R_(c, 2, a) * d2;",
     "q[a] = (R_(c, a, 0) * d0 + R_(c, a, 1) * d1) + R_(c, a, 2) * d2;", 1),
    ("pi_dg drops the y gradient", "double G = gx * gx + gy * gy;", "double G = gx * gx;", 1),
    ("pi_dg centre depth from D_min", "return ((double)m->dmin[i] + (double)m->dmax[i]) / 2.0;", "return (double)m->dmin[i];", 1),
    # footprint statistics (Eqs. seethrough, tightening)
    ("excess not divided by A", "*E = ex > 0 ? (double)ex / (double)A : 0.0;", "*E = ex > 0 ? (double)ex : 0.0;", 1),
    ("layered without the sign test", "*layered = (ex > 0) && (lhs > rhs);", "*layered = (lhs > rhs);", 1),
    ("stats area without +1", "int64_t A = (int64_t)(x1 - x0 + 1) * (int64_t)(y1 - y0 + 1);",
     "int64_t A = (int64_t)(x1 - x0) * (int64_t)(y1 - y0 + 1);", 1),
    ("footprint ignores a corner behind", "if (!oracle_project(c, p, eps, &u, &v, &qz)) return 0;",
     "if (!oracle_project(c, p, eps, &u, &v, &qz)) continue;", 1),
    # occupancy, index, Morton, labels
    ("occupancy strict", "if (r >= tau_occ) {", "if (r > tau_occ) {", 1),
    ("index upper face inclusive", "if (!(f >= 0.0) || !(f < (double)dim)) return 0;", "if (!(f >= 0.0) || !(f <= (double)dim)) return 0;", 1),
    ("Morton y bit", "m |= (uint64_t)((y >> b) & 1u) << (3 * b + 1);", "m |= (uint64_t)((y >> b) & 1u) << (3 * b);", 1),
    ("label inverted", "labels[i] = bsearch(&key, s, (size_t)n_seg, sizeof(uint32_t), cmp_u32) != NULL;",
     "labels[i] = bsearch(&key, s, (size_t)n_seg, sizeof(uint32_t), cmp_u32) == NULL;", 1),
    # 2DGS thin path (Alg. gs-thin, Eqs. behind-gate, thin-nmin, gs-coverage, thin-d2min)
    ("n_min floor", "double n_min = ceil(th->rho_occ * A);", "double n_min = floor(th->rho_occ * A);", 1),
    ("A_B without +1", "const double A = (double)(x1 - x0 + 1) * (double)(y1 - y0 + 1);",
     "const double A = (double)(x1 - x0) * (double)(y1 - y0);", 1),
    ("thin without per-pixel statistics",
     "if (mp->nsamp) footprint_stats(mp->nsamp, W, x0, x1, y0, y1, mp->nsamp[pix], &layered, &E);", ";", 1),
    ("thin statistics of the corner pixel", "footprint_stats(mp->nsamp, W, x0, x1, y0, y1, mp->nsamp[pix], &layered, &E);",
     "footprint_stats(mp->nsamp, W, x0, x1, y0, y1, mp->nsamp[(size_t)y0 * W + x0], &layered, &E);", 2),
    ("thin unprojects at D_med", "double d = layered ? dmin : dmed;", "double d = dmed;", 1),
    ("thin without see-through", "int front = (layered || seethru) && trusted;", "int front = layered && trusted;", 1),
    ("thin without trust", "int front = (layered || seethru) && trusted;", "int front = (layered || seethru);", 1),
    ("thin coverage over the area", "double p_cov = (double)n_md / (double)n_depth;", "double p_cov = (double)n_md / A;", 1),
    ("thin distance gate 2h", "double g = 1.5 * h;", "double g = 2.0 * h;", 1),
    ("behind gate 3h", "if (q[2] > d_surf + 2.0 * h) continue;", "if (q[2] > d_surf + 3.0 * h) continue;", 1),
    ("behind gate on D_med", "double d_surf = (trusted && seethru) ? dmin : dmed;", "double d_surf = dmed;", 1),
    ("thin mask test dropped", "if (!(m > 0.5)) continue;", "if (!(m >= 0.0)) continue;", 1),
    ("thin vote weighted", "Wx += t;\n                    Zx += 1.0;\n                    vm |= (uint64_t)1 << s;\n                }\n            }\n        }",
     "Wx += t;\n                    Zx += t;\n                    vm |= (uint64_t)1 << s;\n                }\n            }\n        }", 1),
    # NeRF thick path (Alg. nerf-fusion, Eqs. dist_tol, depth_tol, nerf-vote)
    ("NeRF bonus halved", "double b = pr->beta * ns;", "double b = 0.5 * pr->beta * ns;", 1),
    ("NeRF bonus uncapped", "if (b > nr->b_max) b = nr->b_max;\n    double tau_d", "double tau_d", 1),
    ("NeRF without band slack", " + nr->lambda_range * (dmax - dmin);", ";", 1),
    ("NeRF depth modes swapped", "double xd = nr->ray_depths ? tp : qz;", "double xd = nr->ray_depths ? qz : tp;", 1),
    ("NeRF clamp to D_exp", "if (tc > dmax) tc = dmax;", "if (tc > dexp) tc = dexp;", 1),
    ("NeRF weight from the unclamped t", "double r = fabs(tc - mu) / hd;", "double r = fabs(tp - mu) / hd;", 1),
    # NeRF thin path (Alg. nerf-thin, Eqs. nerf-thindepth, nerf-support, nerf-counters, nerf-coverage)
    ("NeRF thin multiplier not doubled", "double tau = (2.0 * pr->gamma + b) * h;", "double tau = (pr->gamma + b) * h;", 1),
    ("NeRF thin without bonus", "double tau = (2.0 * pr->gamma + b) * h;", "double tau = (2.0 * pr->gamma) * h;", 1),
    ("NeRF thin peak over supportive pixels",
     "if (m > 0.5 && fabs(xd - dexp) <= tau) n_valid += 1;\n            if (m > m_max) m_max = m;",
     "if (m > 0.5 && fabs(xd - dexp) <= tau) {\n                n_valid += 1;\n                if (m > m_max) m_max = m;\n            }", 1),
    ("NeRF thin N_pixels without +1", "const double n_pixels = (double)(x1 - x0 + 1) * (double)(y1 - y0 + 1);",
     "const double n_pixels = (double)(x1 - x0) * (double)(y1 - y0);", 1),
    ("NeRF thin eligibility at 0.5", "!(cm > 0.1)", "!(cm > 0.5)", 1),
    ("NeRF thin without density floor", " || !(rho[a] >= nr->rho_thin)", "", 1),
    # Pass 3 (Alg. vox2surfel; Eqs. cov-atomics, kappa, final-F)
    ("3-sigma box", "double ex = fmax(fabs(ax0), fabs(ax1)), ey = fmax(fabs(ay0), fabs(ay1));",
     "double ex = 3.0 * fmax(fabs(ax0), fabs(ax1)), ey = 3.0 * fmax(fabs(ay0), fabs(ay1));", 1),
    ("1-sigma acceptance", "if (!(u * u + v * v <= 9.0) || !(z > eps)) continue;", "if (!(u * u + v * v <= 1.0) || !(z > eps)) continue;", 1),
    ("Cramer sign", "double u = (r0 * m11 - m01 * r1) / det;", "double u = (r0 * m11 + m01 * r1) / det;", 1),
    ("Cramer rows swapped", "double v = (m00 * r1 - r0 * m10) / det;", "double v = (m10 * r1 - r0 * m00) / det;", 1),
    ("kappa mean over views", "if (ks > k_i) k_i = ks;", "k_i += ks / (double)n_views;", 1),
    ("no view gating", "if (!((vm >> s) & 1u)) continue;", ";", 1),
    ("strict mask threshold", ">= tau_M) *mask_hit += 1;", "> tau_M) *mask_hit += 1;", 1),
    ("strict coverage threshold", "labels_out[i] = k_i >= tau_kappa;", "labels_out[i] = k_i > tau_kappa;", 1),
    ("quaternion sign", "Rm[1] = 2.0 * (x * y - w * z);", "Rm[1] = 2.0 * (x * y + w * z);", 1),
    ("tip projection halved wrong", "double ax0 = (pu[0] - pu[1]) / 2.0, ay0 = (pv[0] - pv[1]) / 2.0;",
     "double ax0 = (pu[0] - pu[1]), ay0 = (pv[0] - pv[1]);", 1),
    # differentiable variant and its reverse mode
    ("soft test derivative sign", "double ds_de = -s * (1.0 - s) / pr->soft_width;", "double ds_de = s * (1.0 - s) / pr->soft_width;", 1),
    ("logit gradient without sigmoid'", "g_logit[s][dv.pix] += g * (dv.s * dv.w) * dv.dm_dl;", "g_logit[s][dv.pix] += g * (dv.s * dv.w);", 1),
    ("depth gradient without -P", "double gsw = g * (dv.m - P);", "double gsw = g * dv.m;", 1),
    ("median gradient without the soft test", "out->dsw_dmed = ds_de * de_dmed * w + s * dw_dmed;", "out->dsw_dmed = s * dw_dmed;", 1),
    ("max gradient of the half-width", "double dr_dmaxr = dr_dctr * 0.5 + dr_dhw * 0.5;", "double dr_dmaxr = dr_dctr * 0.5;", 1),
]


def _mutate(text, old, new, occ):
    pos = -1
    for _ in range(occ):
        pos = text.find(old, pos + 1)
        assert pos >= 0, f"mutation site not found: {old!r} (occurrence {occ})"
    return text[:pos] + new + text[pos + len(old):]


def _run(idx, tmp):
    name, old, new, occ = MUTANTS[idx]
    src = open(SRC).read()
    mut = _mutate(src, old, new, occ)
    c = os.path.join(tmp, f"m{idx}.c")
    so = os.path.join(tmp, f"m{idx}.so")
    open(c, "w").write(mut)
    subprocess.check_call(["gcc", "-O1", "-std=gnu11", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC",
                           "-shared", "-w", "-o", so, c, "-lm"])
    env = dict(os.environ, DIVAS_ORACLE_LIB=so, OMP_NUM_THREADS="1")
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider", "-m", "not gpu"] + PINS,
                       cwd=ROOT, env=env, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, timeout=600)
    return name, r.returncode


def test_mutation_sites_exist():
    src = open(SRC).read()
    for name, old, new, occ in MUTANTS:
        _mutate(src, old, new, occ)


def test_every_planted_mistake_fails_a_pin():
    workers = max(1, min(8, (os.cpu_count() or 2)))
    with tempfile.TemporaryDirectory() as tmp, cf.ThreadPoolExecutor(workers) as ex:
        results = list(ex.map(lambda i: _run(i, tmp), range(len(MUTANTS))))
    survived = [name for name, rc in results if rc == 0]
    assert not survived, f"mutants that pass every pin: {survived}"
