#!/usr/bin/env python3
"""Benchmark of the depth-weighted voxel aggregation hot path on one MI355X.

A step is one pass of the whole path over one batch of synthetic input: the
occupancy construction (active list from the points), the per-view pre-pass,
culling and thick-path fusion of all views with the compact-fusion rule and
the consensus threshold, and the voxel-lookup labels of all points.  Inputs are
resident in HBM before timing starts.  The metric is voxel-view fusion
samples/s: (active voxels x views) / seconds per step.

Prints ONE JSON line (rank 0) with the metric, a roofline object for the
dominant kernel (HIP-event timing of that kernel on the launch stream), and the
CPU oracle timed on a bounded sample of the same workload.

  python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload c3|c2|c1]
  python bench.py --copy-calibration     (a 64 MiB device copy, for the PMC
                                          FETCH_SIZE / WRITE_SIZE scale factor)
  python bench.py --summarize KIND ...   (rocprofv3 CSV output -> the summaries
                                          kept with the sources; no GPU)
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X published HBM3E bandwidth

WORKLOADS = {
    "c3": "unbounded-360: 60 primitives + background shell in [-4,4]^3, 3M Gaussian centres, 512^3 grid "
          "(~1.8% active), 16 views 1264x832 on a ring",
    "c2": "forward-facing: 20 spheres/boxes, 300k Gaussian centres, 256^3 grid, 10 views 504x378",
    "c1": "tiny analytic: unit sphere on a ground square, 20k points, 64^3 grid, 4 views 128x96",
}
# HBM traffic per kernel from rocprofv3 FETCH_SIZE / WRITE_SIZE runs of this
# workload (used only while the kernel sources are unchanged)
TRAFFIC_FILES = {"c3": "traffic_unbounded_512.json"}
HEAVY_TRAFFIC_FILE = "traffic_heavy_unbounded_512.json"


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def copy_calibration():
    import torch
    n = 64 << 20
    a = torch.empty(n // 4, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    a.fill_(1.0)
    torch.cuda.synchronize()
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_calibration_bytes": n, "launches": 3}))


def kernel_source_hash():
    """Hash of the HIP sources: PMC traffic measured on other sources is stale."""
    import glob
    import hashlib
    h = hashlib.sha1()
    for f in sorted(glob.glob(os.path.join(ROOT, "paper_2601_04860_amd", "csrc", "*"))):
        if f.endswith((".hip", ".h", ".cpp")):
            h.update(os.path.basename(f).encode())
            with open(f, "rb") as fh:
                h.update(fh.read())
    return h.hexdigest()[:16]


def algorithmic_bytes(scene, n_act, work, foot, own_labels=False):
    """Compulsory HBM bytes per launch of each single-kernel phase: every byte
    the method makes that kernel read or write, counted once (no credit for
    caches, no charge for re-reads).  `work` is the device's count of the hot
    path's units in the last fusion."""
    S = len(scene.views)
    px = sum(v.mask.size for v in scene.views)
    words = sum(((v.mask.shape[1] + 7) // 8 + 63) // 64 * ((v.mask.shape[0] + 7) // 8) for v in scene.views)
    chunks = (n_act + 63) // 64
    return {
        # mask planes read once; the hot-tile words and the gate bitmask (one bit per pixel) written
        "views": px * 4 + words * 8 + px // 8,
        # chunk box (16 B) and view word (8 B) per chunk, one hot-tile word (8 B) per (chunk, view)
        "cull": chunks * (16 + 8 + 8 * S),
        # fuse_kernel_bytes: per chunk, per voxel, and the distinct bytes read where it gathers
        "fuse": fuse_kernel_bytes(n_act, work, foot),
        # points in (their coordinates, or with own_labels the voxel codes the
        # occupancy build kept), one label byte out, the segmentation bitfield
        # read once
        "label": len(scene.label_points) * (5 if own_labels else 13) + scene.dim ** 3 // 8,
    }


def fusion_alg_bytes(scene, n_act):
    """Bytes of one full fusion as the method is specified (all four maps of
    every view read once, 16 B per pixel; index in, P and view bitmask out;
    the segmentation bitfield written): the per-sample figure of the roofline
    in samples/s."""
    px = sum(v.mask.size for v in scene.views)
    return px * 16 + n_act * 16 + scene.dim ** 3 // 8


def gather_footprint(scene, act, mask_gate, use_nsamp):
    """Distinct bytes the fusion kernel must read at the pixels where it
    gathers, computed on the host from the same projection (binary64): for
    every view, the pixels hit by an active voxel centre in frame whose mask
    passes the gate.  Each such pixel is read once for its mask value and depth
    triple (16 B); its four clamp-to-edge neighbours once for d_min and d_max
    (8 B, unless already counted); with n_samp the counts of every pixel of
    the union of the footprint boxes (2 B), which the kernel sums.  Also the
    distinct gate-bitmask bytes of in-frame samples."""
    import numpy as np
    dim, h = scene.dim, scene.voxel
    a = np.asarray(act, np.int64)
    iv = np.stack([a % dim, (a // dim) % dim, a // (dim * dim)], 1).astype(np.float64)
    cen = np.asarray(scene.origin, np.float64)[None, :] + (iv + 0.5) * h
    tot = {"pixels": 0, "pixel_bytes": 0, "neighbour_bytes": 0, "nsamp_bytes": 0, "gate_bytes": 0,
           "gathered_samples": 0}
    for v in scene.views:
        cam = v.cam
        R, o = cam["c2w"][:, :3], cam["c2w"][:, 3]
        W, H = cam["width"], cam["height"]
        q = (cen - o[None, :]) @ R
        qz = q[:, 2]
        with np.errstate(divide="ignore", invalid="ignore"):
            u = cam["fx"] * q[:, 0] / qz + cam["cx"]
            vv = cam["fy"] * q[:, 1] / qz + cam["cy"]
        ok = (qz > 1e-6) & (u >= 0) & (u < W) & (vv >= 0) & (vv < H)
        px, py = np.floor(u[ok]).astype(np.int64), np.floor(vv[ok]).astype(np.int64)
        pix = py * W + px
        tot["gate_bytes"] += int(np.unique(py * ((W + 7) // 8) + (px >> 3)).size)
        sel = v.mask.reshape(-1)[pix].astype(np.float64) >= mask_gate
        tot["gathered_samples"] += int(sel.sum())
        g = np.unique(pix[sel])
        tot["pixels"] += int(g.size)
        tot["pixel_bytes"] += int(g.size) * 16
        gx, gy = g % W, g // W
        nb = np.concatenate([gy * W + np.minimum(gx + 1, W - 1), gy * W + np.maximum(gx - 1, 0),
                             np.minimum(gy + 1, H - 1) * W + gx, np.maximum(gy - 1, 0) * W + gx])
        nb = np.setdiff1d(np.unique(nb), g, assume_unique=True)
        tot["neighbour_bytes"] += int(nb.size) * 8
        if use_nsamp:
            ivs = iv[ok][sel]
            us, vs_ = [], []
            bad = np.zeros(len(ivs), bool)
            for j in range(8):
                cj = np.asarray(scene.origin)[None, :] + (ivs + np.array([j & 1, (j >> 1) & 1, (j >> 2) & 1])) * h
                qj = (cj - o[None, :]) @ R
                bad |= ~(qj[:, 2] > 1e-6)
                with np.errstate(divide="ignore", invalid="ignore"):
                    us.append(cam["fx"] * qj[:, 0] / qj[:, 2] + cam["cx"])
                    vs_.append(cam["fy"] * qj[:, 1] / qj[:, 2] + cam["cy"])
            us, vs_ = np.stack(us), np.stack(vs_)
            x0 = np.clip(np.floor(us.min(0)), 0, W - 1).astype(np.int64)
            x1 = np.clip(np.floor(us.max(0)), 0, W - 1).astype(np.int64)
            y0 = np.clip(np.floor(vs_.min(0)), 0, H - 1).astype(np.int64)
            y1 = np.clip(np.floor(vs_.max(0)), 0, H - 1).astype(np.int64)
            keep = ~bad
            # union of the boxes: a 2D difference image, integrated
            diff = np.zeros((H + 1, W + 1), np.int64)
            W1 = W + 1
            for yy, xx, sg in ((y0, x0, 1), (y0, x1 + 1, -1), (y1 + 1, x0, -1), (y1 + 1, x1 + 1, 1)):
                np.add.at(diff.reshape(-1), yy[keep] * W1 + xx[keep], sg)
            cover = np.cumsum(np.cumsum(diff, 0), 1)[:H, :W] > 0
            tot["nsamp_bytes"] += int(cover.sum()) * 2
    tot["total"] = tot["pixel_bytes"] + tot["neighbour_bytes"] + tot["nsamp_bytes"] + tot["gate_bytes"]
    return tot


def fuse_kernel_bytes(n_act, work, foot):
    """Algorithmic bytes of one launch of the fusion kernel: the view word of
    every chunk (8 B), the old segmentation flag in and P and the view bitmask
    out for every voxel (13 B), the index of every voxel of a chunk with views
    to evaluate (4 B), and the distinct bytes it must read where it gathers
    (gather_footprint)."""
    chunks = (n_act + 63) // 64
    hot_vox = min(n_act, work["hot_chunks"] * 64)
    return chunks * 8 + n_act * 13 + hot_vox * 4 + foot["total"]


def short_kernel_name(name, keep_template=False):
    """'void divas::(anonymous namespace)::k_fuse_all<0>(divas::FuseArgs)' ->
    'k_fuse_all' (return type, namespaces, call arguments and, unless asked
    to keep them, template arguments dropped)."""
    n = name.strip()
    if n.startswith("void "):
        n = n[5:]

    def strip_group(t, open_ch, close_ch):  # a trailing balanced (...) or <...>
        if not t.endswith(close_ch):
            return t
        depth = 0
        for k in range(len(t) - 1, -1, -1):
            depth += (t[k] == close_ch) - (t[k] == open_ch)
            if depth == 0:
                return t[:k].rstrip()
        return t

    n = strip_group(n, "(", ")")
    base = strip_group(n, "<", ">")
    tmpl = n[len(base):].strip() if keep_template else ""
    n = base
    return n.replace("(anonymous namespace)", "anon").split("::")[-1] + tmpl


def _pmc_rows(path):
    """Per short kernel name: the list of per-dispatch values of each counter
    in a rocprofv3 counter_collection.csv."""
    import csv
    per = {}
    with open(path, newline="") as f:
        for r in csv.DictReader(f):
            k = short_kernel_name(r["Kernel_Name"])
            per.setdefault(k, {}).setdefault(r["Counter_Name"], {})
            d = per[k][r["Counter_Name"]]
            disp = r["Dispatch_Id"]
            d[disp] = d.get(disp, 0.0) + float(r["Counter_Value"])  # summed over dimensions
    return {k: {c: list(v.values()) for c, v in cs.items()} for k, cs in per.items()}


def _median(v):
    import statistics
    return statistics.median(v) if v else 0.0


def summarize(argv):
    """Summaries of rocprofv3 CSV output, kept under profiles/:

    trace STATS_CSV              markdown table of a --kernel-trace --stats run
    counters CSV [CSV ...]       markdown table of PMC runs (median per dispatch)
    traffic OUT KEY FETCH_CSV WRITE_CSV CAL_FETCH_CSV CAL_WRITE_CSV
                                 HBM bytes per launch (median over dispatches),
                                 each counter scaled by what it reads for the
                                 64 MiB copy of --copy-calibration; merged into
                                 OUT under KEY ('-' for the whole step) with the
                                 hash of the HIP sources
    traffic-md OUT               markdown table of such a file
    """
    import csv
    kind = argv[0] if argv else ""
    if kind == "trace":
        rows = []
        with open(argv[1], newline="") as f:
            for r in csv.DictReader(f):
                rows.append((short_kernel_name(r["Name"], keep_template=True), int(r["Calls"]), float(r["AverageNs"]) / 1e3,
                             float(r["MinNs"]) / 1e3, float(r["MaxNs"]) / 1e3, float(r["Percentage"])))
        print("| kernel | calls | avg us | min us | max us | share |\n|---|---:|---:|---:|---:|---:|")
        for n, c, a, lo, hi, pc in sorted(rows, key=lambda r: -r[5]):
            print(f"| {n} | {c} | {a:.2f} | {lo:.2f} | {hi:.2f} | {pc:.1f}% |")
    elif kind == "counters":
        per = {}
        for path in argv[1:]:
            for k, cs in _pmc_rows(path).items():
                for c, v in cs.items():
                    per.setdefault(k, {})[c] = _median(v)
        names = sorted({c for cs in per.values() for c in cs})
        print("| kernel | " + " | ".join(names) + " |\n|---|" + "---:|" * len(names))
        for k in sorted(per, key=lambda k: -per[k].get("SQ_WAVE_CYCLES", per[k].get(names[0], 0))):
            print(f"| {k} | " + " | ".join(f"{per[k].get(c, float('nan')):.3g}" for c in names) + " |")
    elif kind == "traffic":
        out, key, fetch, write, cfetch, cwrite = argv[1:7]
        cal = 64 << 20

        def factor(path, counter):
            v = _pmc_rows(path).get("copyBuffer", {}) or _pmc_rows(path).get("__amd_rocclr_copyBuffer", {})
            vals = [x for x in v.get(counter, []) if x > 0]
            return cal / (_median(vals) * 1024.0)

        ff, fw = factor(cfetch, "FETCH_SIZE"), factor(cwrite, "WRITE_SIZE")
        rd = {k: _median(cs.get("FETCH_SIZE", [])) * 1024.0 * ff for k, cs in _pmc_rows(fetch).items()}
        wr = {k: _median(cs.get("WRITE_SIZE", [])) * 1024.0 * fw for k, cs in _pmc_rows(write).items()}
        kernels = {k: {"read_bytes": int(rd.get(k, 0)), "write_bytes": int(wr.get(k, 0)),
                       "bytes": int(rd.get(k, 0) + wr.get(k, 0))} for k in sorted(set(rd) | set(wr))}
        doc = {}
        if os.path.exists(out):
            with open(out) as f:
                doc = json.load(f)
        doc["source_hash"] = kernel_source_hash()
        doc["factors"] = {"FETCH_SIZE": round(ff, 4), "WRITE_SIZE": round(fw, 4)}
        if key == "-":
            doc["kernels"] = kernels
        else:
            doc.setdefault("legs", {})[key] = {"kernels": kernels}
        with open(out, "w") as f:
            json.dump(doc, f, indent=1, sort_keys=True)
            f.write("\n")
    elif kind == "traffic-md":
        with open(argv[1]) as f:
            doc = json.load(f)
        groups = [("", doc["kernels"])] if "kernels" in doc else []
        groups += [(k, v["kernels"]) for k, v in sorted(doc.get("legs", {}).items())]
        print(f"factors: FETCH_SIZE {doc['factors']['FETCH_SIZE']}, WRITE_SIZE {doc['factors']['WRITE_SIZE']}; "
              f"source hash {doc['source_hash']}\n")
        for g, ks in groups:
            if g:
                print(f"\n{g}:\n")
            print("| kernel | read MB | write MB | total MB |\n|---|---:|---:|---:|")
            for k, v in sorted(ks.items(), key=lambda kv: -kv[1]["bytes"]):
                if v["bytes"] >= 1e5:
                    print(f"| {k} | {v['read_bytes'] / 1e6:.2f} | {v['write_bytes'] / 1e6:.2f} | "
                          f"{v['bytes'] / 1e6:.2f} |")
    else:
        print(summarize.__doc__, file=sys.stderr)
        sys.exit(2)


HEAVY_LEGS = (("R2", dict(mask_gate=0.0), False), ("R1 n_samp", {}, True), ("R2 n_samp", dict(mask_gate=0.0), True))


def _load_traffic(name):
    """The per-kernel traffic file under profiles/, or None when it is missing
    or was measured on other HIP sources."""
    path = os.path.join(ROOT, "profiles", name)
    try:
        with open(path) as f:
            tr = json.load(f)
    except (OSError, ValueError):
        return None
    return tr if tr.get("source_hash") == kernel_source_hash() else None


def heavy_legs(ctx, scene, xyz, log_fn, steps=20, only=None):
    """The unbounded workload's fusion where the thick path runs on most
    samples: reading R2 (mask gate 0: every in-frame sample with a surface is
    gathered and tested), and the footprint statistics (n_samp sums over each
    gathered voxel's footprint), under R1 and R2.  Per leg: time per full fusion (pre-pass, cull,
    fusion, threshold), the fusion kernel's average launch time from HIP events
    on its stream, its algorithmic bytes and their rate against the 8 TB/s
    peak."""
    import torch

    import paper_2601_04860_amd as dv
    from tests import _helpers as H
    out = {}
    tr = _load_traffic(HEAVY_TRAFFIC_FILE)
    for name, kw, nsamp in HEAVY_LEGS:
        if only is not None and name != only:
            continue
        lp = dv.default_params(scene.voxel, **kw)
        s = dv.Session(ctx, dict(origin=scene.origin, voxel=scene.voxel, dim=scene.dim), xyz, params=lp,
                       max_views=len(scene.views), max_view_pixels=max(v.mask.size for v in scene.views))
        vs = H.upload_views(scene.views, use_nsamp=nsamp)
        res = s.alloc_result()
        n_act = s.info()["n_active"]
        for _ in range(3):
            s.fuse_views(vs, res)
        torch.cuda.synchronize()
        s.set_timing(phases=("fuse",))
        s.timings(reset=True)
        t0 = time.perf_counter()
        for _ in range(steps):
            s.fuse_views(vs, res)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / steps
        f_ms, f_n = s.timings(reset=True)["fuse"]
        s.set_timing(True)
        for _ in range(steps):
            s.fuse_views(vs, res)
        torch.cuda.synchronize()
        ph = {k: round(v[0] / v[1], 5) for k, v in s.timings(reset=True).items() if v[1]}
        s.set_timing(False)
        ph["fuse"] = round(f_ms / f_n, 5)
        work = s.fusion_work()
        act = s.active_indices()
        s.close()
        foot = gather_footprint(scene, act, lp.mask_gate, nsamp)
        kb = fuse_kernel_bytes(n_act, work, foot)
        f_avg = f_ms / f_n
        gbs = kb / (f_avg * 1e-3) / 1e9
        samples = n_act * len(scene.views)
        traffic = None
        if tr is not None:
            traffic = tr.get("legs", {}).get(name, {}).get("kernels", {}).get("k_fuse_all", {}).get("bytes")
        px = sum(v.mask.size for v in scene.views)
        words = sum(((v.mask.shape[1] + 7) // 8 + 63) // 64 * ((v.mask.shape[0] + 7) // 8) for v in scene.views)
        # the pre-pass: mask planes in, hot-tile words and gate bits out
        pre_b = px * 4 + words * 8 + px // 8
        out[name] = {"mask_gate": lp.mask_gate, "n_samp": nsamp, "ms_per_fusion": round(ms, 5),
                     "samples_per_s": samples / (ms * 1e-3), "phases_avg_ms": ph, "fusion_work": work,
                     "prepass": {"alg_bytes": int(pre_b),
                                 "achieved_GBps": round(pre_b / (ph["views"] * 1e-3) / 1e9, 1) if ph.get("views")
                                 else None},
                     "fuse_kernel": {"avg_launch_ms": round(f_avg, 5), "alg_bytes": int(kb),
                                     "achieved_GBps": round(gbs, 1), "frac": round(gbs / HBM_PEAK_GBS, 4),
                                     "traffic": traffic, "gather_footprint": foot}}
        log_fn(f"[bench] C3 {name}: {ms:.4f} ms per fusion, fusion kernel {f_avg * 1e3:.1f} us, "
               f"{kb / 1e6:.1f} MB alg -> {gbs:.0f} GB/s ({gbs / HBM_PEAK_GBS:.3f}), "
               f"{work['gathered']} gathered samples")
    return out


def cpu_baseline(scene, params, budget_s=12.0):
    """The oracle as it stands, timed on this host, median of 3 runs each:
    - all threads: whole steps (occupancy, fusion of all views with OpenMP
      over voxels, labels);
    - one thread: the fusion of all views over a fixed sample of the active
      voxels (every 8th, so a run stays near a second), scaled per sample.
    The budget bounds the number of whole steps per timed run."""
    import statistics

    import numpy as np
    import oracle
    oracle.build(force=False)
    threads = oracle.num_threads()
    act = oracle.occupancy(scene.points, scene.grid)
    S = len(scene.views)

    last = {}

    def whole_step():
        a = oracle.occupancy(scene.points, scene.grid)
        res = oracle.fuse(a, scene.grid, scene.views, params, n_threads=threads, with_margin=False)
        last["labels"] = oracle.label(scene.label_points, scene.grid, a[res["seg"].astype(bool)])
        last["act"], last["vout"] = a, res["vout"]

    t0 = time.perf_counter()
    whole_step()
    t_one = time.perf_counter() - t0
    per_run = max(1, min(10, int(budget_s / 3 / max(t_one, 1e-3))))
    runs = []
    for _ in range(3):
        t0 = time.perf_counter()
        for _ in range(per_run):
            whole_step()
        runs.append((time.perf_counter() - t0) / per_run)
    t_med = statistics.median(runs)
    sub = np.ascontiguousarray(act[::8])
    runs1 = []
    for _ in range(3):
        t0 = time.perf_counter()
        oracle.fuse(sub, scene.grid, scene.views, params, n_threads=1, with_margin=False)
        runs1.append(time.perf_counter() - t0)
    t1_med = statistics.median(runs1)
    out = {"value": len(act) * S / t_med, "unit": "voxel-view samples/s", "cores": threads, "kind": "oracle",
           "sample": f"whole steps of the same workload ({S} views, all {len(act)} active voxels), median of 3 "
                     f"runs of {per_run} steps; fusion on {threads} OpenMP threads, occupancy and labels "
                     f"single-threaded",
           "seconds_per_step": round(t_med, 4),
           "single_thread": {"value": len(sub) * S / t1_med, "unit": "voxel-view samples/s", "cores": 1,
                             "sample": f"fusion of all {S} views over every 8th active voxel ({len(sub)}), "
                                       f"median of 3 runs", "seconds": round(t1_med, 4)}}
    # the grid construction of the same points, once (numpy, one thread)
    import oracle.grid_stats as G
    t0 = time.perf_counter()
    G.grid_from_points(scene.points, synthetic_scales(scene), g_max=1024)
    out["grid_construction_ms"] = round((time.perf_counter() - t0) * 1e3, 1)
    # the band-pass refinement of every view's mask, once (numpy, one thread)
    import oracle.mask_refine as R
    t0 = time.perf_counter()
    for v in scene.views:
        R.refine_bandpass(v.mask, v.dmed, view_prompts(v.mask))
    out["mask_refinement_ms_per_view"] = round((time.perf_counter() - t0) * 1e3 / len(scene.views), 2)
    # the needle cull of one scale pair per point, once
    import oracle.surfel_map as SM
    t0 = time.perf_counter()
    SM.needle_cull(np.ones(len(scene.points), np.uint8), synthetic_surfel_scales(scene))
    out["needle_cull_ms"] = round((time.perf_counter() - t0) * 1e3, 1)
    # Pass 3 after the step's Pass 1 labels and the needle cull, once (C, one thread)
    scales, quats = synthetic_surfel_scales(scene), synthetic_surfel_quats(scene)
    lab2 = SM.needle_cull(last["labels"], scales)[0]
    t0 = time.perf_counter()
    oracle.surfel_coverage(np.asarray(scene.label_points, np.float32), scales, quats, lab2, scene.grid, last["act"],
                           last["vout"], scene.views)
    out["surfel_coverage_ms"] = round((time.perf_counter() - t0) * 1e3, 1)
    return out


def synthetic_surfel_quats(scene):
    """Seeded random rotations (w, x, y, z; normalised by the callee) of the
    synthetic surfels."""
    import numpy as np
    rng = np.random.default_rng(8765)
    return rng.standard_normal((len(scene.label_points), 4)).astype(np.float32)


def surfel_bench(ctx, scene, xyz, log_fn, reps=10):
    """Pass 3 of the voxel-to-surfel mapping on the unbounded workload: the
    3M points as surfels (synthetic scales and rotations) after the fusion of
    the 16 views, Pass 1 (voxel lookup labels) and Pass 2 (the needle cull);
    the footprint coverage kappa over every view the surfel's voxel voted in,
    and the final labels.  Host clock around each call, which waits for its
    own device work."""
    import torch

    import paper_2601_04860_amd as dv
    from tests import _helpers as H
    lp = dv.default_params(scene.voxel)
    s = dv.Session(ctx, dict(origin=scene.origin, voxel=scene.voxel, dim=scene.dim), xyz, params=lp,
                   max_views=len(scene.views), max_view_pixels=max(v.mask.size for v in scene.views))
    res = s.fuse_views(H.upload_views(scene.views))
    pts = xyz if scene.label_points is scene.points else H.to_dev(scene.label_points)
    lab = s.label_points(pts)
    scales = H.to_dev(synthetic_surfel_scales(scene))
    quats = H.to_dev(synthetic_surfel_quats(scene))
    dv.needle_cull(ctx, scales, lab)
    n_in = int(lab.sum().item())
    out_lab = torch.empty_like(lab)
    s.surfel_coverage(pts, scales, quats, lab, res["vmask"], labels_out=out_lab)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        _, _, kept = s.surfel_coverage(pts, scales, quats, lab, res["vmask"], labels_out=out_lab)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / reps
    n = int(pts.shape[0])
    s.close()
    out = {"surfels": n, "labelled_after_pass2": n_in, "kept": int(kept.item()), "views": len(scene.views),
           "ms": round(ms, 4), "surfels_per_s": n / (ms * 1e-3),
           "timing": "host clock around each call, which waits for its own device work"}
    log_fn(f"[bench] Pass 3 coverage {ms:.3f} ms for {n} surfels ({n_in} labelled, {out['kept']} kept)")
    return out


def synthetic_surfel_scales(scene):
    """Two seeded log-normal tangent scales per point, 1 % stretched into
    needles (a stand-in for trained 2DGS surfels)."""
    import numpy as np
    rng = np.random.default_rng(4321)
    n = len(scene.points)
    s = scene.voxel / 3 * np.exp(0.5 * rng.standard_normal((n, 2)))
    k = rng.random(n) < 0.01
    s[k, 0] *= np.exp(rng.random(int(k.sum())) * 8)
    return s.astype(np.float32)


def synthetic_scales(scene):
    """One seeded log-normal scale per point around a third of the voxel edge
    (a stand-in for the larger tangent scale of a trained surfel)."""
    import numpy as np
    rng = np.random.default_rng(1234)
    return (scene.voxel / 3 * np.exp(0.5 * rng.standard_normal(len(scene.points)))).astype(np.float32)


def serving_bench(ctx, log_fn, rate=200.0, n_requests=4000, reps=5, offline_only=False):
    """Batched (one persistent launch sequence for many sessions) against plain
    per-session and per-(session, view) launches on the serving workload, then
    the click stream through the continuous-batching server: Poisson arrivals at
    `rate`, p50 / p99 latency from arrival to completion, and the saturated
    request rate against plain per-request launches."""
    import numpy as np
    import torch

    import paper_2601_04860_amd as dv
    import scenes
    from paper_2601_04860_amd.serving import DeviceWorkload, run_click_stream, run_plain
    from tests import _helpers as H

    t0 = time.perf_counter()
    wl = scenes.config_scene("c5")
    dw = DeviceWorkload(wl, H.to_dev)
    log_fn(f"[serve] workload ready in {time.perf_counter() - t0:.1f}s")
    # ---- offline: 32 sessions x all resident views
    n_sess = 32
    sess, work = [], []
    samples = 0
    for i in range(n_sess):
        k, t = dw.pairs[i % len(dw.pairs)]
        sc = dw.scenes[k]
        p = dv.default_params(sc.voxel, retain_state=1)
        nres = len(dw.resident[(k, t)].cams)
        s = dv.Session(ctx, dw.grids[k], dw.xyz[k], params=p, max_views=nres, max_view_pixels=dw.max_pix[k])
        res = s.alloc_result()
        n_act = s.info()["n_active"]
        samples += n_act * nres
        sess.append((s, (k, t), nres, res))
        work.append((s, dv.BATCH_FUSE, dw.resident[(k, t)], None, 0, res))
    torch.cuda.synchronize()

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(reps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t) / reps

    def plain_sessions():
        for s, kt, nres, res in sess:
            s.fuse_views(dw.resident[kt], res)

    def plain_views():
        for s, kt, nres, res in sess:
            vs = dw.resident[kt]
            s.fuse_views(vs.subset(0, 1), res)
            for v in range(1, nres):
                s.update_view(v, vs, v, res)

    batch = dv.Batch(ctx, max_items=n_sess, max_new_views=64 * n_sess, use_graph=True)
    cfg = batch.tune(work)
    t_batch = timed(lambda: batch.run(work))
    t_sess = timed(plain_sessions)
    t_views = timed(plain_views)
    batch.close()
    for s, *_ in sess:
        s.close()
    offline = {"sessions": n_sess, "samples": int(samples),
               "batched_ms": round(t_batch * 1e3, 4), "plain_per_session_ms": round(t_sess * 1e3, 4),
               "plain_per_view_ms": round(t_views * 1e3, 4),
               "batched_samples_per_s": samples / t_batch, "plain_per_session_samples_per_s": samples / t_sess,
               "plain_per_view_samples_per_s": samples / t_views,
               "speedup_vs_per_view": round(t_views / t_batch, 3), "speedup_vs_per_session": round(t_sess / t_batch, 3),
               "tuned": cfg}
    log_fn(f"[serve] offline batched {t_batch * 1e3:.3f} ms vs per-session {t_sess * 1e3:.3f} ms "
           f"vs per-view {t_views * 1e3:.3f} ms")
    offline["click_updates"] = click_update_bench(ctx, dw, log_fn)
    if offline_only:
        return {"offline": offline}
    # ---- online: Poisson click stream through the server
    st = run_click_stream(ctx, dw, n_requests=n_requests, rate=rate, log=log_fn)
    sat = run_click_stream(ctx, dw, n_requests=n_requests // 2, saturate=True, log=log_fn)
    plain = run_plain(ctx, dw, n_requests=512)
    sat_full = run_click_stream(ctx, dw, n_requests=n_requests // 2, saturate=True, log=log_fn, resident=False)
    plain_full = run_plain(ctx, dw, n_requests=512, resident=False)
    online = {"rate_per_s": rate, "requests": n_requests, "p50_ms": st["p50_ms"], "p99_ms": st["p99_ms"],
              "mean_ms": st["mean_ms"], "max_ms": st["max_ms"], "mean_batch": st["mean_batch"],
              "admission_waits": st["admission_waits"], "failures": st["failures"],
              "sessions_opened": st["sessions_opened"],
              "saturated_requests_per_s": sat["throughput"], "saturated_p50_ms": sat["p50_ms"],
              "saturated_p99_ms": sat["p99_ms"], "saturated_mean_batch": sat["mean_batch"],
              "plain_requests_per_s": plain["throughput"],
              "outputs": "one result buffer per session, clicks folded into it (resident outputs)",
              "full_writes": {"saturated_requests_per_s": sat_full["throughput"],
                              "saturated_p50_ms": sat_full["p50_ms"], "plain_requests_per_s": plain_full["throughput"]}}
    log_fn(f"[serve] {rate:.0f}/s: p50 {st['p50_ms']:.3f} ms p99 {st['p99_ms']:.3f} ms; saturated "
           f"{sat['throughput']:.1f} req/s vs plain {plain['throughput']:.1f} req/s")
    return {"workload": "4 scenes (128^3 4x504x378, 256^3 8x504x378, 512^3 12x1264x832, 512^3 16x1264x832), "
                        "15 (scene, target) pairs, 6 centroid click views per scene",
            "offline": offline, "online": online}


def click_update_bench(ctx, dw, log_fn, n_sess=32, rounds=6):
    """Click updates of the serving workload: 32 sessions that fused their
    resident views each append one click view per round (a fold), all in one
    batched launch sequence or session by session, into the buffers of their
    previous call; with resident outputs (only the chunks the click reaches
    are written) and without (every entry written)."""
    import torch

    import paper_2601_04860_amd as dv
    out = {"sessions": n_sess, "rounds": rounds}
    for resident in (True, False):
        times = {}
        for mode in ("batched", "per_session"):
            sess = []
            for i in range(n_sess):
                k, t = dw.pairs[i % len(dw.pairs)]
                sc = dw.scenes[k]
                p = dv.default_params(sc.voxel, retain_state=1, resident_outputs=1 if resident else 0)
                nres = len(dw.resident[(k, t)].cams)
                s = dv.Session(ctx, dw.grids[k], dw.xyz[k], params=p, max_views=nres + rounds + 1,
                               max_view_pixels=dw.max_pix[k])
                res = s.alloc_result()
                s.fuse_views(dw.resident[(k, t)], res)
                sess.append((s, (k, t), nres, res))
            b = dv.Batch(ctx, max_items=n_sess, max_new_views=n_sess, use_graph=True) if mode == "batched" else None

            def one_round(r):
                if b is not None:
                    b.run([(s, dv.BATCH_UPDATE, dw.clicks[kt], r % len(dw.clicks[kt].cams), nres + r, res)
                           for s, kt, nres, res in sess])
                else:
                    for s, kt, nres, res in sess:
                        s.update_view(nres + r, dw.clicks[kt], r % len(dw.clicks[kt].cams), res)

            one_round(0)  # warm-up (also builds the graph)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for r in range(1, rounds + 1):
                one_round(r)
            torch.cuda.synchronize()
            times[mode] = (time.perf_counter() - t0) * 1e3 / rounds
            if b is not None:
                b.close()
            for s, *_ in sess:
                s.close()
        key = "resident_outputs" if resident else "full_writes"
        out[key] = {"batched_ms_per_round": round(times["batched"], 4),
                    "per_session_ms_per_round": round(times["per_session"], 4),
                    "speedup": round(times["per_session"] / times["batched"], 3)}
        log_fn(f"[serve] click updates ({key}): batched {times['batched']:.3f} ms vs per-session "
               f"{times['per_session']:.3f} ms per round of {n_sess}")
    return out


def targets_bench(ctx, log_fn, reps=10):
    """Several target objects of one scene: the largest scene of the serving
    workload (512^3, 16 views 1264x832, 8 targets) fused for every target by
    divas_fuse_targets, forced together (shared projection, depth gathers and
    gates) and with its automatic schedule, against the same sessions fused one
    after another (divas_fuse_views per target).  Outputs are bit-identical
    (tested)."""
    import torch

    import paper_2601_04860_amd as dv
    import scenes
    from tests import _helpers as H
    wl = scenes.config_scene("c5")
    sc = wl["scenes"][3]
    T = len(sc.views[0].masks)
    grid = dict(origin=sc.origin, voxel=sc.voxel, dim=sc.dim)
    xyz = H.to_dev(sc.points)
    mp = max(v.mask.size for v in sc.views)
    out = {"workload": f"{sc.dim}^3 grid, {len(sc.points)} points, {len(sc.views)} views "
                       f"{sc.views[0].mask.shape[1]}x{sc.views[0].mask.shape[0]}, {T} targets"}
    for gate in (0.5, 0.0):
        lp = dv.default_params(sc.voxel, mask_gate=gate)
        base = dv.Session(ctx, grid, xyz, params=lp, max_views=len(sc.views), max_view_pixels=mp)
        sess = [base] + [dv.Session.target(base, params=lp, max_views=len(sc.views), max_view_pixels=mp)
                         for _ in range(T - 1)]
        vs0 = H.upload_views(sc.views)
        sets = [vs0.with_masks([H.to_dev(v.masks[t]) for v in sc.views]) for t in range(T)]
        res = [s.alloc_result() for s in sess]

        def one_by_one():
            for s, v, r in zip(sess, sets, res):
                s.fuse_views(v, r)

        def together():
            dv.fuse_targets(sess, sets, res, schedule="together")

        def auto():
            dv.fuse_targets(sess, sets, res, schedule="auto")

        times = {}
        for name, fn in (("one_after_another", one_by_one), ("together", together), ("auto", auto)):
            fn()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(reps):
                fn()
            torch.cuda.synchronize()
            times[name] = (time.perf_counter() - t0) * 1e3 / reps
        n_act = base.info()["n_active"]
        for s in reversed(sess):
            s.close()
        key = "R1" if gate > 0 else "R2 (mask gate 0)"
        samples = n_act * len(sc.views) * T
        out[key] = {"one_after_another_ms": round(times["one_after_another"], 4),
                    "together_ms": round(times["together"], 4), "auto_ms": round(times["auto"], 4),
                    "speedup_together": round(times["one_after_another"] / times["together"], 3),
                    "speedup_auto": round(times["one_after_another"] / times["auto"], 3),
                    "target_samples_per_s_auto": samples / (times["auto"] * 1e-3), "n_active": n_act}
        log_fn(f"[bench] {T} targets {key}: {times['together']:.3f} ms together, {times['auto']:.3f} ms auto, "
               f"{times['one_after_another']:.3f} ms one after another")
    return out


def forward_facing_bench(ctx, log_fn, steps=50):
    """Full fusion (pre-pass, cull, fusion, threshold) of the forward-facing
    workload (256^3, 10 views 504x378): samples/s of the fusion alone, with the
    active list built once (inputs resident)."""
    import torch

    import paper_2601_04860_amd as dv
    import scenes
    from tests import _helpers as H
    sc = scenes.config_scene("c2")
    lp = dv.default_params(sc.voxel)
    xyz = H.to_dev(sc.points)
    s = dv.Session(ctx, dict(origin=sc.origin, voxel=sc.voxel, dim=sc.dim), xyz, params=lp,
                   max_views=len(sc.views), max_view_pixels=max(v.mask.size for v in sc.views))
    vs = H.upload_views(sc.views)
    res = s.alloc_result()
    n_act = s.info()["n_active"]
    for _ in range(5):
        s.fuse_views(vs, res)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        s.fuse_views(vs, res)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / steps
    s.close()
    samples = n_act * len(sc.views)
    log_fn(f"[bench] forward-facing fusion {ms:.4f} ms, {samples / (ms * 1e-3):.4g} samples/s")
    return {"workload": WORKLOADS["c2"], "n_active": n_act, "views": len(sc.views), "ms_per_fusion": round(ms, 5),
            "samples_per_s": samples / (ms * 1e-3)}


def grid_bench(ctx, scene, log_fn, reps=10):
    """Scene-statistic grid construction (Eq. scene-norm, Eq. voxel-size) of
    the workload's points with one synthetic scale per point: GPU time per
    call, inputs resident (the oracle's time is in the CPU baseline)."""
    import torch

    import paper_2601_04860_amd as dv
    from tests import _helpers as H
    xyz, sc = H.to_dev(scene.points), H.to_dev(synthetic_scales(scene))
    g_max = 1024
    dv.grid_from_points(ctx, xyz, sc, g_max=g_max)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        grid, st = dv.grid_from_points(ctx, xyz, sc, g_max=g_max)
    ms = (time.perf_counter() - t0) * 1e3 / reps
    n = len(scene.points)
    out = {"points": n, "g_max": g_max, "ms": round(ms, 4), "points_per_s": n / (ms * 1e-3),
           "dim": grid["dim"], "voxel": grid["voxel"], "b": st["b"],
           "selections": "3 coordinate medians and the scale median (4 passes of 8-bit digits over 32-bit keys), "
                         "the P99 distance (8 passes over 64-bit keys), two ranks each",
           "timing": "host clock around the call, which waits for its own device work"}
    # Pass 2 of the voxel-to-surfel mapping on the same points as surfels
    sc2 = H.to_dev(synthetic_surfel_scales(scene))
    lab = torch.ones(n, dtype=torch.uint8, device="cuda")
    dv.needle_cull(ctx, sc2, lab)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        lab.fill_(1)
        tau, cut = dv.needle_cull(ctx, sc2, lab)
    out["needle_cull_ms"] = round((time.perf_counter() - t0) * 1e3 / reps, 4)
    out["needle_culled"] = cut
    log_fn(f"[bench] grid construction {ms:.3f} ms, needle cull {out['needle_cull_ms']} ms for {n} points")
    return out


def nerf_bench(ctx, scene, xyz, log_fn, steps=30):
    """Full fusion (pre-pass, cull, fusion, threshold) of the workload under
    the NeRF thick path (Mip-NeRF 360 column of the NeRF table), with the
    depth tuple read as camera Z (the library's default reading); inputs
    resident."""
    import torch

    import paper_2601_04860_amd as dv
    from tests import _helpers as H
    lp = dv.nerf_params(scene.voxel, "360")
    s = dv.Session(ctx, dict(origin=scene.origin, voxel=scene.voxel, dim=scene.dim), xyz, params=lp,
                   max_views=len(scene.views), max_view_pixels=max(v.mask.size for v in scene.views))
    vs = H.upload_views(scene.views)
    res = s.alloc_result()
    n_act = s.info()["n_active"]
    for _ in range(3):
        s.fuse_views(vs, res)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        s.fuse_views(vs, res)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / steps
    work = s.fusion_work()
    s.close()
    samples = n_act * len(scene.views)
    log_fn(f"[bench] NeRF-variant fusion {ms:.4f} ms, {samples / (ms * 1e-3):.4g} samples/s")
    return {"variant": "NeRF thick path, Mip-NeRF 360 constants, camera-Z depths", "ms_per_fusion": round(ms, 5),
            "samples_per_s": samples / (ms * 1e-3), "fusion_work": work}


def thin_bench(ctx, log_fn, steps=30):
    """Fusion with the thin-structure paths (2DGS fallback, NeRF thin path)
    beside the thick path alone, on the tiny sphere scene (20k points, 4 views,
    density floor 5 points) at two voxel footprints: a coarse 32^3 grid seen at
    256x192, f = 300 (40-60 pixels per voxel), and a zoomed 16^3 grid seen at
    512x384, f = 800 (about 1,000 pixels per voxel)."""
    import torch

    import paper_2601_04860_amd as dv
    import scenes
    from tests import _helpers as H
    cases = (("coarse", dict(dim=32, width=256, height=192, focal=300.0),
              "tiny sphere, 32^3 grid, 20k points, 4 views 256x192 (voxel footprints of 40-60 pixels)"),
             ("zoomed", dict(dim=16, width=512, height=384, focal=800.0),
              "tiny sphere, 16^3 grid, 20k points, 4 views 512x384, f = 800 (voxel footprints of about 1,000 "
              "pixels)"))
    out = {}
    for key, kw, desc in cases:
        sc = scenes.make_tiny_sphere(n_points=20000, n_views=4, seed=1, **kw)
        xyz = H.to_dev(sc.points)
        vs = H.upload_views(sc.views)
        leg = {"workload": desc}
        kinds = (("thick_only", dv.default_params(sc.voxel)),
                 ("with_thin", dv.default_params(sc.voxel, thin=1, rho_thin=5.0)),
                 ("nerf_thick_only", dv.nerf_params(sc.voxel, "360")),
                 ("nerf_with_thin", dv.nerf_params(sc.voxel, "360", thin=1, rho_thin=5.0)))
        for name, lp in kinds:
            s = dv.Session(ctx, dict(origin=sc.origin, voxel=sc.voxel, dim=sc.dim), xyz, params=lp,
                           max_views=len(sc.views), max_view_pixels=sc.views[0].mask.size)
            res = s.alloc_result()
            for _ in range(3):
                s.fuse_views(vs, res)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(steps):
                s.fuse_views(vs, res)
            torch.cuda.synchronize()
            ms = (time.perf_counter() - t0) * 1e3 / steps
            n_act = s.info()["n_active"]
            s.close()
            leg[name] = {"ms_per_fusion": round(ms, 5), "n_active": n_act,
                         "samples_per_s": n_act * len(sc.views) / (ms * 1e-3)}
        out[key] = leg
        log_fn(f"[bench] thin paths ({key}): 2DGS {leg['with_thin']['ms_per_fusion']} ms vs thick only "
               f"{leg['thick_only']['ms_per_fusion']} ms; NeRF {leg['nerf_with_thin']['ms_per_fusion']} ms vs "
               f"{leg['nerf_thick_only']['ms_per_fusion']} ms per fusion")
    return out


def view_prompts(mask, k=3):
    """Synthetic positive prompts of a view: its k highest-mask pixels (x, y)."""
    import numpy as np
    order = np.argsort(-mask.reshape(-1), kind="stable")[:k]
    w = mask.shape[1]
    return [(int(i % w), int(i // w)) for i in order]


def refine_bench(ctx, scene, log_fn, reps=5):
    """Depth refinement of every view's mask (band-pass and min-max), inputs
    resident: GPU time per view against its algorithmic bytes (mask and depth
    read once, refined mask written once: 12 B per pixel)."""
    import torch

    import paper_2601_04860_amd as dv
    from tests import _helpers as H
    planes = [(H.to_dev(v.mask), H.to_dev(v.dmed), view_prompts(v.mask)) for v in scene.views]
    outs = [torch.empty_like(m) for m, _, _ in planes]
    res = {}
    for kind in ("bandpass", "minmax"):
        def run():
            for (m, d, pr), o in zip(planes, outs):
                if kind == "bandpass":
                    dv.refine_mask_bandpass(ctx, m, d, pr, out=o)
                else:
                    dv.refine_mask_minmax(ctx, m, d, out=o)
        run()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            run()
        ms = (time.perf_counter() - t0) * 1e3 / (reps * len(planes))
        px = int(scene.views[0].mask.size)
        gbs = px * 12 / (ms * 1e-3) / 1e9
        res[kind] = {"ms_per_view": round(ms, 4), "alg_GBps": round(gbs, 1), "frac": round(gbs / HBM_PEAK_GBS, 4)}
    res["view_pixels"] = int(scene.views[0].mask.size)
    res["views"] = len(scene.views)
    res["timing"] = "host clock around each call, which waits for its own device work (band-pass: four " \
                    "selection passes over the depth keys for d_far)"
    log_fn(f"[bench] mask refinement per view: band-pass {res['bandpass']['ms_per_view']} ms, "
           f"min-max {res['minmax']['ms_per_view']} ms")
    return res


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="c3", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=12.0)
    ap.add_argument("--copy-calibration", action="store_true")
    ap.add_argument("--no-serve", action="store_true", help="skip the batched / serving measurements")
    ap.add_argument("--no-legs", action="store_true",
                    help="skip the NeRF-variant, grid-construction and mask-refinement legs")
    ap.add_argument("--only", choices=("heavy", "targets", "serve-offline", "thin", "surfel"),
                    help="run only one leg (the heavy-path legs of the unbounded workload, or the multi-target "
                         "leg) and print it, for profiling")
    ap.add_argument("--leg", choices=[n for n, _, _ in HEAVY_LEGS],
                    help="with --only heavy: that leg alone (one PMC run per leg)")
    ap.add_argument("--summarize", nargs=argparse.REMAINDER,
                    help="summaries of rocprofv3 CSV output (no GPU): trace | counters | traffic | traffic-md ...")
    args = ap.parse_args()
    if args.summarize is not None:
        summarize(args.summarize)
        return

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        msg = ("bench.py measures one GPU: this build runs the hot path on a single MI355X "
               "(the multi-GPU split is described in DESIGN.md, not run); use --gpus 1")
        if int(os.environ.get("RANK", "0")) == 0:
            print(msg, file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    if args.copy_calibration:
        copy_calibration()
        return

    import paper_2601_04860_amd as dv
    import scenes
    from tests import _helpers as H

    t_gen = time.perf_counter()
    scene = scenes.config_scene(args.workload)
    log(f"[bench] scene {args.workload} ready in {time.perf_counter() - t_gen:.1f}s")
    lp = dv.default_params(scene.voxel)
    ctx = dv.Context(0)
    xyz = H.to_dev(scene.points)
    if args.only == "heavy":
        print(json.dumps({"heavy_legs": heavy_legs(ctx, scene, xyz, log, steps=args.steps, only=args.leg)}),
              flush=True)
        return
    if args.only == "targets":
        print(json.dumps({"multi_target": targets_bench(ctx, log)}), flush=True)
        return
    if args.only == "surfel":
        print(json.dumps({"surfel_coverage": surfel_bench(ctx, scene, xyz, log)}), flush=True)
        return
    if args.only == "thin":
        print(json.dumps({"thin_fallback": thin_bench(ctx, log)}), flush=True)
        return
    if args.only == "serve-offline":
        print(json.dumps({"serving": serving_bench(ctx, log, offline_only=True)}), flush=True)
        return
    # the labels of the session's own points come from the voxel codes its
    # occupancy build of the same step kept
    own_labels = scene.label_points is scene.points
    lab_xyz = xyz if own_labels else H.to_dev(scene.label_points)
    sess = dv.Session(ctx, dict(origin=scene.origin, voxel=scene.voxel, dim=scene.dim), xyz, params=lp,
                      max_views=len(scene.views), max_view_pixels=max(v.mask.size for v in scene.views))
    vs = H.upload_views(scene.views)
    n_act = sess.info()["n_active"]
    res = sess.alloc_result()
    labels = torch.empty(len(scene.label_points), dtype=torch.uint8, device="cuda")
    stream = torch.cuda.current_stream()

    def step():
        sess.rebuild(xyz)
        sess.fuse_views(vs, res)
        if own_labels:
            sess.label_session_points(labels)
        else:
            sess.label_points(lab_xyz, labels)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    log(f"[bench] warmup done: n_active={n_act}")
    # timed region: the fusion kernel (the dominant one) carries HIP events
    # taken from its own dispatch on the session's stream
    sess.set_timing(phases=("fuse",))
    sess.timings(reset=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ph_fuse = sess.timings(reset=True)["fuse"]
    # per-phase breakdown: a second pass of the same steps with every phase timed
    sess.set_timing(True)
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    ph = sess.timings(reset=True)
    sess.set_timing(False)
    ph["fuse"] = ph_fuse
    ms_step = (t1 - t0) * 1e3 / args.steps
    S = len(scene.views)
    samples = n_act * S
    value = samples / (ms_step * 1e-3)
    log(f"[bench] {args.steps} steps: {ms_step:.4f} ms/step, {value:.4g} samples/s")
    if own_labels and not torch.equal(labels, sess.label_points(lab_xyz, torch.empty_like(labels))):
        raise SystemExit("the labels from the occupancy's voxel codes differ from the coordinate lookup")

    work = sess.fusion_work()
    act_host = sess.active_indices()
    foot = gather_footprint(scene, act_host, lp.mask_gate, False)
    alg = algorithmic_bytes(scene, n_act, work, foot, own_labels)
    phases = {}
    for name, (ms, n) in ph.items():
        if n == 0:
            continue
        avg_ms = ms / n
        entry = {"avg_ms": round(avg_ms, 5), "launches": n}
        if name in alg:
            entry["alg_bytes"] = int(alg[name])
            entry["alg_GBps"] = round(alg[name] / (avg_ms * 1e-3) / 1e9, 1)
        phases[name] = entry
    # dominant kernel: the single-kernel phase with the most time (the
    # occupancy phase is several kernels; the pre-pass is one without n_samp)
    kernels = {"views": "k_tile_flags", "cull": "k_cull", "fuse": "k_fuse_all",
               "label": "k_label_codes4" if own_labels else "k_label4"}
    single = {k: v for k, v in phases.items() if k in kernels}
    dom = max(single, key=lambda k: single[k]["avg_ms"] * single[k]["launches"])
    kern = kernels[dom]
    achieved = single[dom]["alg_GBps"]
    tr = _load_traffic(TRAFFIC_FILES.get(args.workload, "none"))
    traffic = tr["kernels"][kern]["bytes"] if tr is not None and kern in tr.get("kernels", {}) else None
    roofline = {"bound": "hbm", "kernel": kern, "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                "alg_bytes_per_launch": single[dom]["alg_bytes"], "avg_launch_ms": single[dom]["avg_ms"]}
    roofline["gather_footprint"] = foot
    # The fusion as one unit (pre-pass, cull, fusion) in samples/s beside the
    # rate a kernel reading every view's four planes in full (16 B per pixel)
    # would reach at 8 TB/s.  This is a dense-equivalent rate, NOT an HBM
    # fraction: the cull skips most of those bytes, which no kernel reads.
    fus_ms = sum(phases[k]["avg_ms"] for k in ("views", "cull", "fuse") if k in phases)
    fb = fusion_alg_bytes(scene, n_act)
    dense = {"ms": round(fus_ms, 5), "samples_per_s": samples / (fus_ms * 1e-3),
             "dense_bytes_per_sample": round(fb / samples, 3),
             "dense_samples_per_s_at_8TBps": HBM_PEAK_GBS * 1e9 / (fb / samples),
             "ratio_not_an_hbm_fraction": round((samples / (fus_ms * 1e-3)) / (HBM_PEAK_GBS * 1e9 / (fb / samples)),
                                                4)}

    cpu = None
    if not args.no_cpu_baseline:
        log("[bench] cpu oracle baseline ...")
        cpu = cpu_baseline(scene, H.oracle_params(lp), budget_s=args.cpu_budget)
        log(f"[bench] cpu baseline {cpu['value']:.4g} samples/s on {cpu['cores']} threads")

    ff = None
    if args.workload == "c3" and not args.no_serve:
        try:
            ff = forward_facing_bench(ctx, log)
        except Exception as e:  # reported, never fatal for the headline line
            ff = {"error": f"{type(e).__name__}: {e}"}
            log(f"[bench] forward-facing failed: {ff['error']}")

    heavy = None
    if args.workload == "c3" and not args.no_legs:
        try:
            heavy = heavy_legs(ctx, scene, xyz, log)
        except Exception as e:  # reported, never fatal for the headline line
            heavy = {"error": f"{type(e).__name__}: {e}"}
            log(f"[bench] heavy legs failed: {heavy['error']}")

    targets_leg = None
    if args.workload == "c3" and not args.no_legs:
        try:
            targets_leg = targets_bench(ctx, log)
        except Exception as e:  # reported, never fatal for the headline line
            targets_leg = {"error": f"{type(e).__name__}: {e}"}
            log(f"[bench] multi-target leg failed: {targets_leg['error']}")

    nerf_leg = None
    if not args.no_legs:
        try:
            nerf_leg = nerf_bench(ctx, scene, xyz, log)
        except Exception as e:  # reported, never fatal for the headline line
            nerf_leg = {"error": f"{type(e).__name__}: {e}"}
            log(f"[bench] NeRF variant failed: {nerf_leg['error']}")

    thin_leg = None
    if not args.no_legs:
        try:
            thin_leg = thin_bench(ctx, log)
        except Exception as e:  # reported, never fatal for the headline line
            thin_leg = {"error": f"{type(e).__name__}: {e}"}
            log(f"[bench] thin fallback failed: {thin_leg['error']}")

    surfel_leg = None
    if args.workload == "c3" and not args.no_legs:
        try:
            surfel_leg = surfel_bench(ctx, scene, xyz, log)
        except Exception as e:  # reported, never fatal for the headline line
            surfel_leg = {"error": f"{type(e).__name__}: {e}"}
            log(f"[bench] Pass 3 failed: {surfel_leg['error']}")

    grid_leg = None
    if not args.no_legs:
        try:
            grid_leg = grid_bench(ctx, scene, log)
        except Exception as e:  # reported, never fatal for the headline line
            grid_leg = {"error": f"{type(e).__name__}: {e}"}
            log(f"[bench] grid construction failed: {grid_leg['error']}")

    refine_leg = None
    if not args.no_legs:
        try:
            refine_leg = refine_bench(ctx, scene, log)
        except Exception as e:  # reported, never fatal for the headline line
            refine_leg = {"error": f"{type(e).__name__}: {e}"}
            log(f"[bench] mask refinement failed: {refine_leg['error']}")

    serve = None
    if not args.no_serve:
        try:
            serve = serving_bench(ctx, log)
        except Exception as e:  # reported, never fatal for the headline line
            serve = {"error": f"{type(e).__name__}: {e}"}
            log(f"[serve] failed: {serve['error']}")

    out = {
        "metric": "voxel-view fusion samples/s (% HBM roofline)",
        "value": value,
        "unit": "voxel-view samples/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": WORKLOADS[args.workload], "grid": scene.dim, "views": S,
                   "view_pixels": int(scene.views[0].mask.size), "points": len(scene.points),
                   "n_active": n_act, "samples_per_step": samples,
                   "step": "occupancy + per-view pre-pass + cull + fusion + threshold + labels",
                   "mask_gate": lp.mask_gate},
        "roofline": roofline,
        "dense_equivalent": dense,
        "heavy_legs": heavy,
        "multi_target": targets_leg,
        "fusion_work": work,
        "phases": phases,
        "phases_timing": "fuse: HIP events on the fusion kernel's dispatch inside the timed region; other phases: "
                         "a second pass of the same steps with every phase timed",
        "cpu_baseline": cpu,
        "serving": serve,
        "forward_facing": ff,
        "nerf_variant": nerf_leg,
        "thin_fallback": thin_leg,
        "surfel_coverage": surfel_leg,
        "grid_construction": grid_leg,
        "mask_refinement": refine_leg,
        "paper_context": "per-update fusion kernel under 70 ms on an A100 in the paper (thick and thin paths, "
                         "and for 2DGS the voxel-to-surfel mapping); not the same work or hardware",
    }
    sess.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
