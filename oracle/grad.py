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


def transfer_torch(means, quats, log_scales, opacity, normals, dirs, Y, cut=None, sources=None, flip=None,
                   want_amb=None):
    """Direct transfer t[count, K] as a differentiable torch float64 graph.

    All tensor arguments are float64; ``dirs`` [S,3] and ``Y`` [S,K] are
    constants.  ``flip`` (optional) reverses chosen decisions: dict with any of
    "hit" [count,S,N], "traced" [count,S], "keep" [count,S] boolean masks.
    ``want_amb`` (the rounding margins, optional): also return the masks of
    decisions within their margins, dict(hit=..., traced=..., keep=...).
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
    flip = flip or {}
    with torch.no_grad():
        not_self = torch.ones(len(sources), 1, n, dtype=torch.bool)
        not_self[torch.arange(len(sources)), 0, sources] = False
        traced = cosw > c["c_min"]
        if "traced" in flip:
            traced ^= flip["traced"]
        hit = (t > c["t_min"]) & (d2 <= c["sigma_cut"] ** 2) & not_self
        raw = opacity[None, None, :] * torch.exp(-0.5 * d2)
        clamped = raw > c["alpha_max"]
        hit &= torch.where(clamped, torch.full_like(raw, c["alpha_max"]), raw) >= c["alpha_min"]
        if "hit" in flip:
            hit ^= flip["hit"] & not_self
        hit &= traced[..., None]
    alpha = opacity[None, None, :] * torch.exp(-0.5 * d2)
    alpha = torch.where(clamped, torch.full_like(alpha, c["alpha_max"]), alpha)
    alpha = torch.where(hit, alpha, torch.zeros_like(alpha))
    V = torch.prod(1.0 - alpha, dim=-1)                            # [I,S]
    with torch.no_grad():
        keep = V >= c["T_eps"]
        if "keep" in flip:
            keep ^= flip["keep"]
        keep &= traced
    V = torch.where(keep, V, torch.zeros_like(V))
    cpos = torch.where(traced, cosw, torch.zeros_like(cosw))
    out = (4.0 * math.pi / S) * (V * cpos) @ Y                     # [I,K]
    if want_amb is None:
        return out
    mar = want_amb
    with torch.no_grad():
        s_ = torch.exp(log_scales)
        kappa = (s_.max(-1).values / s_.min(-1).values)[None, None, :]
        md2 = mar[1] * (1.0 + kappa)
        mt = mar[2] * (1.0 + d2.clamp(min=0.0).sqrt()) / a.sqrt()[None] + mar[4] * t.abs()
        cut2 = c["sigma_cut"] ** 2
        near = (t > c["t_min"] - mt) & (d2 <= cut2 + md2)
        amb_hit = near & (((d2 - cut2).abs() <= md2) | ((t - c["t_min"]).abs() <= mt)) & not_self
        amb_traced = (cosw - c["c_min"]).abs() <= mar[0]
        Vraw = torch.prod(1.0 - alpha, dim=-1)
        amb_keep = ((Vraw / c["T_eps"] - 1.0).abs() <= mar[3]) & traced
    return out, dict(hit=amb_hit & (traced | amb_traced)[..., None], traced=amb_traced, keep=amb_keep)


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


def gradient_allowance(scene, num_dirs, bands, light, target, seed=0, cut=None, margins=None):
    """Per-component bound on how far the gradient of
    L = 1/2 sum (relight(t, light) - target)^2 may move when decisions within
    the FP32 rounding margins of their thresholds (hit test, hemisphere test,
    T_eps cut-off) go the other way: for every such decision, the change in
    the gradient of its source's term L_i (a decision of source i's rays moves
    t_i only, so only L_i) when it alone is reversed, summed in magnitude.
    Returns dict(grads=allowance per input as in loss_and_grads, items=number
    of near-threshold decisions)."""
    from . import DEFAULT_MARGINS
    mar = DEFAULT_MARGINS if margins is None else margins
    dirs_np, Y_np = tables(num_dirs, seed, bands)
    dirs = torch.from_numpy(dirs_np)
    Y = torch.from_numpy(Y_np)
    keys = ("means", "quats", "log_scales", "opacity", "normals")
    base = {k: torch.tensor(np.asarray(scene[k], dtype=np.float64)) for k in keys}
    Lt = torch.tensor(np.asarray(light, dtype=np.float64))
    tgt = torch.from_numpy(np.asarray(target, dtype=np.float64))
    n = base["means"].shape[0]
    allow = {k: np.zeros(tuple(v.shape)) for k, v in base.items()}
    allow["light"] = np.zeros(tuple(Lt.shape))
    items = 0

    def grad_i(i, flip):
        p = {k: v.clone().requires_grad_(True) for k, v in base.items()}
        L = Lt.clone().requires_grad_(True)
        t = transfer_torch(p["means"], p["quats"], p["log_scales"], p["opacity"], p["normals"], dirs, Y, cut,
                           torch.tensor([i]), flip=flip)
        C = torch.einsum("nk,bck->nbc", t, L)
        (0.5 * ((C - tgt[i:i + 1]) ** 2).sum()).backward()
        out = {k: v.grad.numpy().copy() for k, v in p.items()}
        out["light"] = L.grad.numpy().copy()
        return out

    for i in range(n):
        with torch.no_grad():
            _, amb = transfer_torch(base["means"], base["quats"], base["log_scales"], base["opacity"],
                                    base["normals"], dirs, Y, cut, torch.tensor([i]), want_amb=mar)
        found = [("hit", idx) for idx in torch.nonzero(amb["hit"])]
        found += [("traced", idx) for idx in torch.nonzero(amb["traced"])]
        found += [("keep", idx) for idx in torch.nonzero(amb["keep"])]
        if not found:
            continue
        g0 = grad_i(i, None)
        for kind, idx in found:
            m = torch.zeros_like(amb[kind])
            m[tuple(idx.tolist())] = True
            g1 = grad_i(i, {kind: m})
            for k in allow:
                allow[k] += np.abs(g1[k] - g0[k])
            items += 1
    return dict(grads=allow, items=items)


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


def _own_ray_hits(scene, j, dirs, rays, c_, mar, chunk=16):
    """Hits of the rays of source j along dirs[rays] (every other Gaussian
    tested, FP64): per hit its ray position, Gaussian index, and whether its
    predicate lies within the rounding margins (kept for the deviation bound
    with the alpha it would have)."""
    means = torch.from_numpy(np.asarray(scene["means"], dtype=np.float64))
    quats = torch.from_numpy(np.asarray(scene["quats"], dtype=np.float64))
    ls = torch.from_numpy(np.asarray(scene["log_scales"], dtype=np.float64))
    R = _rotation(quats)
    sinv = R @ torch.diag_embed(torch.exp(-2.0 * ls)) @ R.transpose(-1, -2)
    smax, smin = torch.exp(ls).max(-1).values, torch.exp(ls).min(-1).values
    rel = means - means[j][None, :]                                # mu_k - origin
    D = torch.from_numpy(dirs[rays])
    out_r, out_k, out_amb, out_hit = [], [], [], []
    with torch.no_grad():
        for r0 in range(0, len(rays), chunk):
            w = D[r0:r0 + chunk]                                   # [m,3]
            sw = torch.einsum("kab,mb->mka", sinv, w)              # [m,N,3]
            a = (sw * w[:, None, :]).sum(-1)
            b = (sw * rel[None]).sum(-1)
            t = b / a
            d2 = torch.einsum("ka,kab,kb->k", rel, sinv, rel)[None] - b * b / a
            md2 = mar[1] * (1.0 + smax / smin)[None]
            mt = mar[2] * (1.0 + d2.clamp(min=0.0).sqrt()) / a.sqrt() + mar[4] * t.abs()
            hit = (t > c_["t_min"]) & (d2 <= c_["sigma_cut"] ** 2)
            near = (t > c_["t_min"] - mt) & (d2 <= c_["sigma_cut"] ** 2 + md2)
            amb = near & (((d2 - c_["sigma_cut"] ** 2).abs() <= md2) | ((t - c_["t_min"]).abs() <= mt))
            keep = hit | amb
            keep[:, j] = False
            rr, kk = torch.nonzero(keep, as_tuple=True)
            out_r.append(rr + r0)
            out_k.append(kk)
            out_amb.append(amb[rr, kk])
            out_hit.append(hit[rr, kk])
    return (torch.cat(out_r).numpy(), torch.cat(out_k).numpy(), torch.cat(out_amb).numpy(),
            torch.cat(out_hit).numpy())


def _alpha_from_origin(origin, scene, ks, dirs_r):
    """alpha of Gaussians ks at their peak density along origin + t dirs_r
    (Eq. 1, 27), differentiable in the origin."""
    mu = torch.from_numpy(np.asarray(scene["means"], dtype=np.float64)[ks])
    q = torch.from_numpy(np.asarray(scene["quats"], dtype=np.float64)[ks])
    ls = torch.from_numpy(np.asarray(scene["log_scales"], dtype=np.float64)[ks])
    o = torch.from_numpy(np.asarray(scene["opacity"], dtype=np.float64)[ks])
    R = _rotation(q)
    sinv = R @ torch.diag_embed(torch.exp(-2.0 * ls)) @ R.transpose(-1, -2)
    rel = mu - origin[None, :]
    sw = torch.einsum("kab,kb->ka", sinv, dirs_r)
    a = (sw * dirs_r).sum(-1)
    b = (rel * sw).sum(-1)
    d2 = torch.einsum("ka,kab,kb->k", rel, sinv, rel) - b * b / a
    return o * torch.exp(-0.5 * d2)


def gaussian_param_grads(scene, j, num_dirs, bands, d_transfer, seed=0, cut=None, margins=None, chunk=16384,
                         threads=None):
    """FP64 d(loss)/d(opacity, log-scales, quaternion, mean, normal) of
    Gaussian j alone, for any loss whose derivative with respect to the direct
    transfer is ``d_transfer`` [n, K]; meant for scenes far too large for the
    autograd reference above.

    Opacity, scales, rotation and mean of j enter the other splats' transfers
    through alpha_j on the rays that hit j.  For such a ray of source i along
    w_s with visibility V, dV / d alpha_j = -V / (1 - alpha_j) and
    d t_i[k] / dV = (4 pi / S) c Y_k(w_s), so only the visibility of those
    rays is needed.  The mean is also the origin of j's own rays, whose
    visibility V = prod_h (1 - alpha_h) over their hits h moves with it:
    dV / d mu_j = V sum_h d log(1 - alpha_h) / d mu_j.  The normal enters j's
    own transfer only: d t_j[k] / d n_j = (4 pi / S) sum_{s: c_s > 0} V_s
    Y_k(w_s) w_s.  Rays whose decisions lie within the FP32 margins of a
    threshold (hit test, hemisphere test) are counted as the oracle decides
    and their gradient is also summed, in magnitude, into ``allow``.
    Returns dict(grads={opacity, log_scales, quats, means, normals},
    allow={...}, rays=number of rays through j).
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
    smax = float(np.exp(theta0[1:4]).max())
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
            hit = (t > c_["t_min"]) & (d2 <= c_["sigma_cut"] ** 2) & (cw > c_["c_min"])
            hit &= torch.clamp(raw, max=c_["alpha_max"]) >= c_["alpha_min"]
            md2 = mar[1] * (1.0 + smax / smin)
            mt = mar[2] * (1.0 + d2.clamp(min=0.0).sqrt()) / a.sqrt()[None, :] + mar[4] * t.abs()
            near = (t > c_["t_min"] - mt) & (d2 <= c_["sigma_cut"] ** 2 + md2)
            amb = near & (((d2 - c_["sigma_cut"] ** 2).abs() <= md2) | ((t - c_["t_min"]).abs() <= mt))
            amb |= near & ((cw - c_["c_min"]).abs() <= mar[0])
            keep = (hit | amb) & (cw > c_["c_min"] - mar[0])
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
    mu = mu_j.clone().requires_grad_(True)
    alpha, _, _ = _alpha_of_j(th, mu, torch.from_numpy(means[src]), D[sdir])
    with torch.no_grad():
        clamped = alpha > c_["alpha_max"]
    coef = torch.from_numpy(dLdV * V)
    f = coef * torch.log1p(-torch.clamp(alpha, max=c_["alpha_max"]))
    f = torch.where(clamped, torch.zeros_like(f), f)
    # the oracle's decisions for every ray; ambiguous ones also bound the deviation
    g = torch.autograd.grad((f * torch.from_numpy(hit.astype(np.float64))).sum(), [th, mu], retain_graph=True,
                            allow_unused=True)
    g_th = np.zeros(8) if g[0] is None else g[0].numpy()
    g_mu = np.zeros(3) if g[1] is None else g[1].numpy().copy()
    allow = np.zeros(8)
    allow_mu = np.zeros(3)
    for r in np.nonzero(amb)[0]:
        gr = torch.autograd.grad(f[r], [th, mu], retain_graph=True)
        allow += np.abs(gr[0].numpy())
        allow_mu += np.abs(gr[1].numpy())
    # j's own rays: the normal through c, the mean as the rays' origin
    cj = dirs @ normals[j]
    own = np.nonzero(cj > c_["c_min"] - mar[0])[0]
    Vj = rays_vis(scene, np.full(len(own), j), dirs[own], cut=cut, threads=threads)
    per = wq * Vj * (Y[own] @ dT[j])
    dn = ((cj[own] > c_["c_min"]) * per)[:, None] * dirs[own]
    amb_c = np.abs(cj[own] - c_["c_min"]) <= mar[0]
    dn_allow = np.abs(per[amb_c, None] * dirs[own][amb_c]).sum(0)
    rr, kk, amb_h, hit_h = _own_ray_hits(scene, j, dirs, own, c_, mar)
    origin = mu_j.clone().requires_grad_(True)
    a_h = _alpha_from_origin(origin, scene, kk, D[own[rr]])
    with torch.no_grad():
        clamped_h = a_h > c_["alpha_max"]
    coef_h = torch.from_numpy(wq * np.abs(cj[own[rr]]) * Vj[rr] * (Y[own[rr]] @ dT[j]))
    f_h = coef_h * torch.log1p(-torch.clamp(a_h, max=c_["alpha_max"]))
    f_h = torch.where(clamped_h, torch.zeros_like(f_h), f_h)
    counted = torch.from_numpy((hit_h & (cj[own[rr]] > c_["c_min"])).astype(np.float64))
    if len(rr):
        g_mu += torch.autograd.grad((f_h * counted).sum(), origin, retain_graph=True)[0].numpy()
        for h in np.nonzero(amb_h | amb_c[rr])[0]:
            allow_mu += np.abs(torch.autograd.grad(f_h[h], origin, retain_graph=True)[0].numpy())
    grads = dict(opacity=g_th[0], log_scales=g_th[1:4], quats=g_th[4:8], means=g_mu, normals=dn.sum(0))
    allows = dict(opacity=allow[0], log_scales=allow[1:4], quats=allow[4:8], means=allow_mu, normals=dn_allow)
    return dict(grads=grads, allow=allows, rays=int(len(src)), own_hits=int(len(rr)))
