"""Reference gradient for the differentiable fusion -- TEST INFRASTRUCTURE ONLY.

An independent, vectorised float64 PyTorch-CPU implementation of the
differentiable thick-path forward (soft depth test on mask logits, hard
spatial gate, depth weight of Eq. gs-depthweight, compact-fusion ratio); its
gradient comes from autograd.  It shares no code with ``divas_oracle.c`` or
with the HIP library and is used to cross-check both.
"""
from __future__ import annotations

import numpy as np
import torch


def fused_P(active, grid, views, params, logits, dmins, dmeds, dmaxs):
    """P per active voxel as a differentiable function of per-view tensors
    (lists of [H, W] float64 tensors)."""
    g = int(grid["dim"])
    h = float(grid["voxel"])
    origin = torch.tensor(np.asarray(grid["origin"], np.float64))
    act = torch.as_tensor(np.asarray(active, np.int64))
    ijk = torch.stack([act % g, (act // g) % g, act // (g * g)], 1).double()
    ctr = origin + (ijk + 0.5) * h
    eps = params["eps"]
    Wacc = torch.zeros(len(act), dtype=torch.float64)
    Zacc = torch.zeros(len(act), dtype=torch.float64)
    for s, v in enumerate(views):
        cam = v.cam
        Wd, Hd = cam["width"], cam["height"]
        R = torch.tensor(cam["c2w"][:, :3])
        o = torch.tensor(cam["c2w"][:, 3])
        dd = ctr - o
        q = dd @ R          # q_a = sum_b R[b, a] d_b
        qz = q[:, 2]
        front_ok = qz > eps
        qzs = torch.where(front_ok, qz, torch.ones_like(qz))
        u = (cam["fx"] * q[:, 0]) / qzs + cam["cx"]
        vv = (cam["fy"] * q[:, 1]) / qzs + cam["cy"]
        inb = front_ok & (u >= 0) & (u < Wd) & (vv >= 0) & (vv < Hd)
        px = torch.where(inb, torch.floor(u), torch.zeros_like(u)).long()
        py = torch.where(inb, torch.floor(vv), torch.zeros_like(vv)).long()
        pix = py * Wd + px
        lg = logits[s].reshape(-1)[pix]
        dmin = dmins[s].reshape(-1)[pix]
        dmed = dmeds[s].reshape(-1)[pix]
        dmax = dmaxs[s].reshape(-1)[pix]
        ok = inb & (dmed.detach() >= eps) & (dmin.detach() <= dmed.detach())
        r = torch.stack([(px.double() + 0.5 - cam["cx"]) / cam["fx"],
                         (py.double() + 0.5 - cam["cy"]) / cam["fy"],
                         torch.ones(len(act), dtype=torch.float64)], 1)
        wdir = r @ R.T
        dh = wdir / torch.linalg.norm(wdir, dim=1, keepdim=True)
        cosv = dh @ R[:, 2]
        dmin_r, dmed_r, dmax_r = dmin / cosv, dmed / cosv, dmax / cosv
        front = dmed.detach() > params["gamma_st"] * v.d_cam
        dref_r = torch.where(front, dmin_r, dmed_r)
        ts = (dd * dh).sum(1)
        th = torch.minimum(torch.maximum(ts, dmin_r), dref_r)
        p = o + th[:, None] * dh
        delta = torch.linalg.norm(ctr - p, dim=1)
        # pi_dg from the (detached) centre depth map; it only gates
        dc = 0.5 * (dmins[s].detach() + dmaxs[s].detach())
        xm = (px - 1).clamp(min=0)
        xp = (px + 1).clamp(max=Wd - 1)
        ym = (py - 1).clamp(min=0)
        yp = (py + 1).clamp(max=Hd - 1)
        gx = dc[py, xp] - dc[py, xm]
        gy = dc[yp, px] - dc[ym, px]
        pidg = torch.exp(-params["k_grad"] * (gx * gx + gy * gy))
        ok = ok & (delta.detach() <= h * pidg)
        e = torch.where(front, q[:, 2] - dmin, torch.abs(q[:, 2] - dmed))
        s_soft = torch.sigmoid((params["gamma"] * h - e) / params["soft_width"])
        d_ctr = 0.5 * (dmin_r + dmax_r)
        d_hw = torch.clamp(0.5 * (dmax_r - dmin_r), min=eps)
        rr = (th - d_ctr) / d_hw
        w = torch.exp(-params["alpha1"] * rr * rr)
        m = torch.sigmoid(lg)
        sw = torch.where(ok, s_soft * w, torch.zeros_like(w))
        Wacc = Wacc + m * sw
        Zacc = Zacc + sw
    Zs = torch.where(Zacc > eps, Zacc, torch.ones_like(Zacc))
    return torch.where(Zacc > eps, Wacc / Zs, torch.zeros_like(Zacc))


def grads(active, grid, views, params, grad_P):
    """d(sum grad_P * P) / d(logit, dmin, dmed, dmax) per view, float64."""
    L = [torch.tensor(v.logit.astype(np.float64), requires_grad=True) for v in views]
    Dn = [torch.tensor(v.dmin.astype(np.float64), requires_grad=True) for v in views]
    Dm = [torch.tensor(v.dmed.astype(np.float64), requires_grad=True) for v in views]
    Dx = [torch.tensor(v.dmax.astype(np.float64), requires_grad=True) for v in views]
    P = fused_P(active, grid, views, params, L, Dn, Dm, Dx)
    (P * torch.as_tensor(np.asarray(grad_P, np.float64))).sum().backward()
    out = {"logit": [t.grad.numpy() for t in L], "dmin": [t.grad.numpy() for t in Dn],
           "dmed": [t.grad.numpy() for t in Dm], "dmax": [t.grad.numpy() for t in Dx]}
    return P.detach().numpy(), out
