"""Click-stream driver for the continuous-batching server.

The native server (libdivas) does the scheduling; this module only feeds it a
stream of click-driven view updates with Poisson arrivals over many sessions
that open (HBM admission), fuse their resident views, take a bounded number of
clicks and close, and it reports latency percentiles and throughput.  It also
runs the same requests through plain per-request launches for comparison.
"""
from __future__ import annotations

import time

import numpy as np

from . import BATCH_FUSE, BATCH_UPDATE, Server, ViewSet, default_params, make_grid, session_info


class DeviceWorkload:
    """Serving workload resident in device memory: per scene its points and
    depth maps, per (scene, target) the resident and click views."""

    def __init__(self, wl, to_dev):
        self.scenes = wl["scenes"]
        self.pools = wl["pools"]
        self.pairs = wl["pairs"]
        self.xyz = [to_dev(s.points) for s in self.scenes]
        self.grids = [dict(origin=s.origin, voxel=s.voxel, dim=s.dim) for s in self.scenes]
        self.max_pix = [max(v.mask.size for v in s.views + wl["pools"][k]) for k, s in enumerate(self.scenes)]
        depth = []
        for k, s in enumerate(self.scenes):
            res = [(to_dev(v.dmin), to_dev(v.dmed), to_dev(v.dmax)) for v in s.views]
            clk = [(to_dev(v.dmin), to_dev(v.dmed), to_dev(v.dmax)) for v in wl["pools"][k]]
            depth.append((res, clk))
        self.resident = {}
        self.clicks = {}
        for (k, t) in self.pairs:
            s = self.scenes[k]
            vs = ViewSet()
            for v, (dn, dm, dx) in zip(s.views, depth[k][0]):
                vs.add(v.cam, v.d_cam, to_dev(v.masks[t]), dn, dm, dx)
            self.resident[(k, t)] = vs
            cs = ViewSet()
            for v, (dn, dm, dx) in zip(wl["pools"][k], depth[k][1]):
                cs.add(v.cam, v.d_cam, to_dev(v.masks[t]), dn, dm, dx)
            self.clicks[(k, t)] = cs


def _alloc(n, torch):
    return dict(P=torch.empty(max(n, 1), dtype=torch.float32, device="cuda"),
                vmask=torch.empty(max(n, 1), dtype=torch.int64, device="cuda"),
                counts=torch.zeros(3, dtype=torch.int64, device="cuda"), seg_bits=None)


def run_click_stream(ctx, dw, n_requests=4000, rate=200.0, n_sessions=32, clicks_per_session=16, seed=5,
                     saturate=False, n_streams=2, max_batch=64, use_graph=True, churn=False, log=None,
                     resident=True):
    """Serve n_requests click updates arriving Poisson(rate) (all at t=0 when
    saturate) over n_sessions live sessions cycling over the workload's
    (scene, target) pairs; each click appends one view.  After
    clicks_per_session clicks a session starts over: it re-fuses its resident
    views (a FUSE request), or, with churn, closes and a new session of the same
    pair opens (admission by HBM footprint, occupancy rebuilt).  Latency is
    reported over the click requests (arrival to observed completion).  Each
    session keeps one result buffer; with `resident` its clicks fold into it
    (params.resident_outputs)."""
    import torch
    rng = np.random.default_rng(seed)
    srv = Server(ctx, n_streams=n_streams, max_batch=max_batch, max_new_views=max(64, max_batch),
                 use_graph=use_graph)
    gaps = rng.exponential(1.0 / rate, size=n_requests)
    arrivals = np.cumsum(gaps) if not saturate else np.zeros(n_requests)
    live = []  # per slot: dict(sid, pair, clicks, res)
    opened = resets = 0

    def open_slot(i):
        nonlocal opened
        k, t = dw.pairs[i % len(dw.pairs)]
        sc = dw.scenes[k]
        p = default_params(sc.voxel, retain_state=1, resident_outputs=1 if resident else 0)
        nres = len(dw.resident[(k, t)].cams)
        sid = srv.open_session(dw.grids[k], dw.xyz[k], p, max_views=nres + clicks_per_session,
                               max_view_pixels=dw.max_pix[k])
        res = _alloc(len(sc.points), torch)
        srv.submit(sid, BATCH_FUSE, dw.resident[(k, t)], None, 0, res, arrival=srv.now())
        opened += 1
        return dict(sid=sid, pair=(k, t), clicks=0, res=res)

    for i in range(n_sessions):
        live.append(open_slot(i))
    srv.drain(timeout=120.0)
    torch.cuda.synchronize()
    t_start = srv.now() + 0.05
    tickets = []
    for j in range(n_requests):
        target = t_start + arrivals[j]
        while True:
            dt = target - srv.now()
            if dt <= 0:
                break
            time.sleep(min(dt, 0.002) if dt > 0.0005 else 0)
        i = int(rng.integers(n_sessions))
        slot = live[i]
        if slot["clicks"] >= clicks_per_session:
            if churn:
                srv.close_session(slot["sid"])
                live[i] = slot = open_slot(i)
            else:
                srv.submit(slot["sid"], BATCH_FUSE, dw.resident[slot["pair"]], None, 0, slot["res"], arrival=target)
                slot["clicks"] = 0
                resets += 1
        pool = dw.clicks[slot["pair"]]
        idx = int(rng.integers(len(pool.cams)))
        tk = srv.submit(slot["sid"], BATCH_UPDATE, pool, idx, -1, slot["res"], arrival=target)
        slot["clicks"] += 1
        tickets.append(tk)
        if log and j and j % 1000 == 0:
            log(f"[serve] submitted {j} requests, {srv.stats()['completed_updates']} done")
    srv.drain(timeout=300.0)
    t_end = srv.now()
    st = srv.stats()
    lat = np.array([srv.wait(tk, 0.0)[1] for tk in tickets])
    for slot in live:
        srv.close_session(slot["sid"])
    srv.drain(timeout=60.0)
    srv.close()
    span = t_end - t_start
    return dict(requests=n_requests, rate=rate if not saturate else None, seconds=span,
                throughput=n_requests / span if span > 0 else None, p50_ms=float(np.percentile(lat, 50)),
                p99_ms=float(np.percentile(lat, 99)), mean_ms=float(lat.mean()), max_ms=float(lat.max()),
                batches=st["batches"], mean_batch=st["batched_requests"] / max(st["batches"], 1),
                admission_waits=st["admission_waits"], max_queue=st["max_queue"], failures=st["failures"],
                sessions_opened=opened, resets=resets)


def run_plain(ctx, dw, n_requests=512, n_sessions=8, clicks_per_session=16, seed=5, log=None, resident=True):
    """The same kind of click updates through plain per-request launches
    (divas_update_view on one stream, no batching, one result buffer per
    session, folded into with `resident`); returns requests/s."""
    import torch

    from . import Session
    rng = np.random.default_rng(seed)
    sess = []
    for i in range(n_sessions):
        k, t = dw.pairs[i % len(dw.pairs)]
        sc = dw.scenes[k]
        p = default_params(sc.voxel, retain_state=1, resident_outputs=1 if resident else 0)
        nres = len(dw.resident[(k, t)].cams)
        s = Session(ctx, dw.grids[k], dw.xyz[k], params=p, max_views=nres + clicks_per_session,
                    max_view_pixels=dw.max_pix[k])
        res = s.alloc_result()
        s.fuse_views(dw.resident[(k, t)], res)
        sess.append(dict(s=s, pair=(k, t), nres=nres, clicks=0, res=res))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    done = 0
    while done < n_requests:
        i = int(rng.integers(n_sessions))
        e = sess[i]
        if e["clicks"] >= clicks_per_session:
            e["s"].fuse_views(dw.resident[e["pair"]], e["res"])  # session restarts
            e["clicks"] = 0
        pool = dw.clicks[e["pair"]]
        idx = int(rng.integers(len(pool.cams)))
        e["s"].update_view(e["nres"] + e["clicks"], pool, idx, e["res"])
        e["clicks"] += 1
        done += 1
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    for e in sess:
        e["s"].close()
    return dict(requests=n_requests, seconds=dt, throughput=n_requests / dt)
