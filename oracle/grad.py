"""FP64 reference gradients of transfer + relight -- TEST INFRASTRUCTURE ONLY.

The direct transfer (Eq. 1-2, 4, 7, 9, 29 with alpha at the peak density
along the ray) is re-expressed here in torch float64 so that reverse-mode
autograd gives d(loss)/d(opacity, mean, log-scale, quaternion, normal, light
SH).  The discrete decisions of the method (hemisphere test, hit test,
opaque cut-off, alpha clamp) are taken from detached values and held as
constant masks, so the result is the almost-everywhere gradient of the
piecewise-smooth forward.  Brute force over all pairs; meant for scenes of a
few hundred splats.
"""
from __future__ import annotations

import math

import numpy as np
import torch

from . import DEFAULT_CUT, tables


def _rotation(q):
    qn = q / q.norm(dim=-1, keepdim=True)
    w, x, y, z = qn.unbind(-1)
    return torch.stack([
        torch.stack([1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)], -1),
        torch.stack([2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)], -1),
        torch.stack([2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)], -1),
    ], -2)


def transfer_torch(means, quats, log_scales, opacity, normals, dirs, Y, cut=None, sources=None):
    """Direct transfer t[count, K] as a differentiable torch float64 graph.

    All tensor arguments are float64; ``dirs`` [S,3] and ``Y`` [S,K] are
    constants.
    """
    c = dict(DEFAULT_CUT)
    if cut:
        c.update(cut)
    n = means.shape[0]
    S = dirs.shape[0]
    if sources is None:
        sources = torch.arange(n)
    R = _rotation(quats)                                           # [N,3,3]
    inv_var = torch.exp(-2.0 * log_scales)                         # [N,3]
    sinv = R @ torch.diag_embed(inv_var) @ R.transpose(-1, -2)     # Sigma^-1, Eq. 2
    sw = torch.einsum("jab,sb->sja", sinv, dirs)                   # [S,N,3]
    a = (sw * dirs[:, None, :]).sum(-1)                            # w^T Sinv w  [S,N]
    mu_i = means[sources]                                          # [I,3]
    rel = means[None, :, :] - mu_i[:, None, :]                     # mu_j - mu_i [I,N,3]
    b = torch.einsum("ija,sja->isj", rel, sw)                      # [I,S,N]
    t = b / a[None]                                                # peak position t*
    e = mu_i[:, None, None, :] + t[..., None] * dirs[None, :, None, :] - means[None, None, :, :]
    d2 = torch.einsum("isja,jab,isjb->isj", e, sinv, e)            # d^2 at the peak
    cosw = normals[sources] @ dirs.T                               # [I,S]
    with torch.no_grad():
        not_self = torch.ones(len(sources), 1, n, dtype=torch.bool)
        not_self[torch.arange(len(sources)), 0, sources] = False
        traced = cosw > 0.0
        hit = (t > c["t_min"]) & (d2 <= c["sigma_cut"] ** 2) & not_self & traced[..., None]
        raw = opacity[None, None, :] * torch.exp(-0.5 * d2)
        clamped = raw > c["alpha_max"]
        hit &= torch.where(clamped, torch.full_like(raw, c["alpha_max"]), raw) >= c["alpha_min"]
    alpha = opacity[None, None, :] * torch.exp(-0.5 * d2)
    alpha = torch.where(clamped, torch.full_like(alpha, c["alpha_max"]), alpha)
    alpha = torch.where(hit, alpha, torch.zeros_like(alpha))
    V = torch.prod(1.0 - alpha, dim=-1)                            # [I,S]
    with torch.no_grad():
        keep = (V >= c["T_eps"]) & traced
    V = torch.where(keep, V, torch.zeros_like(V))
    cpos = torch.where(traced, cosw, torch.zeros_like(cosw))
    return (4.0 * math.pi / S) * (V * cpos) @ Y                    # [I,K]


def loss_and_grads(scene, num_dirs, bands, light, target, seed=0, cut=None, chunk=16):
    """L = 1/2 sum (C - C_hat)^2 with C = relight(t_dir, light); returns the
    loss, the transfer and the gradient with respect to every input."""
    dirs_np, Y_np = tables(num_dirs, seed, bands)
    dirs = torch.from_numpy(dirs_np)
    Y = torch.from_numpy(Y_np)
    params = {k: torch.tensor(np.asarray(scene[k], dtype=np.float64), requires_grad=True)
              for k in ("means", "quats", "log_scales", "opacity", "normals")}
    L = torch.tensor(np.asarray(light, dtype=np.float64), requires_grad=True)      # [B,3,K]
    tgt = torch.from_numpy(np.asarray(target, dtype=np.float64))                    # [N,B,3]
    n = params["means"].shape[0]
    total = 0.0
    ts = []
    for start in range(0, n, chunk):
        src = torch.arange(start, min(n, start + chunk))
        t = transfer_torch(params["means"], params["quats"], params["log_scales"], params["opacity"],
                           params["normals"], dirs, Y, cut, src)
        C = torch.einsum("nk,bck->nbc", t, L)
        loss = 0.5 * ((C - tgt[src]) ** 2).sum()
        loss.backward()
        total += float(loss.detach())
        ts.append(t.detach().numpy())
    grads = {k: v.grad.numpy().copy() for k, v in params.items()}
    grads["light"] = L.grad.numpy().copy()
    return dict(loss=total, t=np.concatenate(ts, 0), grads=grads)


def _alpha_of_j(theta, mu_j, origins, dirs):
    """alpha of one Gaussian (theta = opacity, log-scales [3], quaternion [4])
    at its peak density along each ray origins[r] + t dirs[r] (Eq. 1, 27)."""
    o, ls, q = theta[0], theta[1:4], theta[4:8]
    R = _rotation(q[None])[0]
    sinv = R @ torch.diag(torch.exp(-2.0 * ls)) @ R.T
    rel = mu_j[None, :] - origins                                  # [R,3]
    sw = dirs @ sinv                                               # [R,3]
    a = (sw * dirs).sum(-1)
    b = (rel * sw).sum(-1)
    t = b / a
    d2 = ((rel @ sinv) * rel).sum(-1) - b * b / a
    return o * torch.exp(-0.5 * d2), t, d2


def gaussian_param_grads(scene, j, num_dirs, bands, d_transfer, seed=0, cut=None, margins=None, chunk=16384,
                         threads=None):
    """FP64 d(loss)/d(opacity, log-scales, quaternion, normal) of Gaussian j
    alone, for any loss whose derivative with respect to the direct transfer
    is ``d_transfer`` [n, K]; meant for scenes far too large for the
    autograd reference above.

    Opacity, scales and rotation of j enter the other splats' transfers only
    through alpha_j on the rays that hit j.  For such a ray of source i along
    w_s with visibility V, dV / d alpha_j = -V / (1 - alpha_j) and
    d t_i[k] / dV = (4 pi / S) c Y_k(w_s), so only the visibility of those
    rays is needed.  The normal enters j's own transfer only:
    d t_j[k] / d n_j = (4 pi / S) sum_{s: c_s > 0} V_s Y_k(w_s) w_s.
    Rays whose decisions lie within the FP32 margins of a threshold (hit test,
    hemisphere test) are counted as the oracle decides and their gradient is
    also summed, in magnitude, into ``allow``.
    Returns dict(grads={opacity, log_scales, quats, normals}, allow={...},
    rays=number of rays through j).
    """
    from . import DEFAULT_MARGINS, rays_vis
    c_ = dict(DEFAULT_CUT)
    if cut:
        c_.update(cut)
    mar = DEFAULT_MARGINS if margins is None else margins
    dirs, Y = tables(num_dirs, seed, bands)
    S = dirs.shape[0]
    wq = 4.0 * math.pi / S
    means = np.asarray(scene["means"], dtype=np.float64)
    normals = np.asarray(scene["normals"], dtype=np.float64)
    dT = np.asarray(d_transfer, dtype=np.float64)
    n = means.shape[0]
    theta0 = np.concatenate([[float(scene["opacity"][j])], np.asarray(scene["log_scales"][j], np.float64),
                             np.asarray(scene["quats"][j], np.float64)])
    theta = torch.tensor(theta0, dtype=torch.float64)
    mu_j = torch.from_numpy(means[j].copy())
    smin = float(np.exp(theta0[1:4]).min())
    D = torch.from_numpy(dirs)
    # every ray of every other source against Gaussian j
    src_l, dir_l, amb_l, hit_l = [], [], [], []
    with torch.no_grad():
        R = _rotation(theta[4:8][None])[0]
        sinv = R @ torch.diag(torch.exp(-2.0 * theta[1:4])) @ R.T
        sw = D @ sinv
        a = (sw * D).sum(-1)                                       # [S]
        for start in range(0, n, chunk):
            idx = torch.arange(start, min(n, start + chunk))
            rel = mu_j[None, :] - torch.from_numpy(means[start:start + len(idx)])
            b = rel @ sw.T                                         # [m,S]
            t = b / a[None]
            d2 = ((rel @ sinv) * rel).sum(-1)[:, None] - b * b / a[None]
            cw = torch.from_numpy(normals[start:start + len(idx)]) @ D.T
            raw = float(theta[0]) * torch.exp(-0.5 * d2)
            hit = (t > c_["t_min"]) & (d2 <= c_["sigma_cut"] ** 2) & (cw > 0)
            hit &= torch.clamp(raw, max=c_["alpha_max"]) >= c_["alpha_min"]
            dist = rel.norm(dim=-1)[:, None]
            md2 = mar[1] * (1.0 + dist / smin)
            mt = mar[2] * (1.0 + dist)
            near = (t > c_["t_min"] - mt) & (d2 <= c_["sigma_cut"] ** 2 + md2)
            amb = near & (((d2 - c_["sigma_cut"] ** 2).abs() <= md2) | ((t - c_["t_min"]).abs() <= mt))
            amb |= near & (cw.abs() <= mar[0])
            keep = (hit | amb) & (cw > -mar[0])
            keep[idx == j] = False
            ii, ss = torch.nonzero(keep, as_tuple=True)
            src_l.append(idx[ii])
            dir_l.append(ss)
            amb_l.append(amb[ii, ss])
            hit_l.append(hit[ii, ss])
    src = torch.cat(src_l).numpy()
    sdir = torch.cat(dir_l).numpy()
    amb = torch.cat(amb_l).numpy()
    hit = torch.cat(hit_l).numpy()
    V = rays_vis(scene, src, dirs[sdir], cut=cut, threads=threads)
    cw = np.einsum("ra,ra->r", normals[src], dirs[sdir])
    dLdV = wq * np.abs(cw) * np.einsum("rk,rk->r", dT[src], Y[sdir])
    th = theta.clone().requires_grad_(True)
    alpha, _, _ = _alpha_of_j(th, mu_j, torch.from_numpy(means[src]), D[sdir])
    with torch.no_grad():
        clamped = alpha > c_["alpha_max"]
    coef = torch.from_numpy(dLdV * V)
    f = coef * torch.log1p(-torch.clamp(alpha, max=c_["alpha_max"]))
    f = torch.where(clamped, torch.zeros_like(f), f)
    # the oracle's decisions for every ray; ambiguous ones also bound the deviation
    g = torch.autograd.grad((f * torch.from_numpy(hit.astype(np.float64))).sum(), th, retain_graph=True,
                            allow_unused=True)[0]
    g = np.zeros(8) if g is None else g.numpy()
    allow = np.zeros(8)
    for r in np.nonzero(amb)[0]:
        allow += np.abs(torch.autograd.grad(f[r], th, retain_graph=True)[0].numpy())
    # the normal, through j's own rays
    cj = dirs @ normals[j]
    own = np.nonzero(cj > -mar[0])[0]
    Vj = rays_vis(scene, np.full(len(own), j), dirs[own], cut=cut, threads=threads)
    per = wq * Vj * (Y[own] @ dT[j])
    dn = ((cj[own] > 0) * per)[:, None] * dirs[own]
    amb_c = np.abs(cj[own]) <= mar[0]
    dn_allow = np.abs(per[amb_c, None] * dirs[own][amb_c]).sum(0)
    grads = dict(opacity=g[0], log_scales=g[1:4], quats=g[4:8], normals=dn.sum(0))
    allows = dict(opacity=allow[0], log_scales=allow[1:4], quats=allow[4:8], normals=dn_allow)
    return dict(grads=grads, allow=allows, rays=int(len(src)))

