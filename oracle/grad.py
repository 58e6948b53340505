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
