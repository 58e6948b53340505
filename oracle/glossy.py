"""FP64 reference of the glossy transfer matrix -- TEST INFRASTRUCTURE ONLY.

The paper's transfer for glossy splats (Sec. 4.5, "transfer matrix for
unknown direction", Eq. 36-41) with the BRDF of Sec. 4.2:

    f(wi, wo) = (1 - m) rho / pi + D F G / (4 (wi . n)(wo . n))
    T(wi, wo) = f(wi, wo) (wi . n) V(wi)
    t'_ab     = (4 pi / S)^2 sum_s sum_p Y_a(w_s) T(w_s, w_p) Y_b(w_p)

over the S stratified directions for both wi (index s) and wo (index p),
with T = 0 unless wi . n > 0 and wo . n > 0.  The outgoing radiance under a
light l (SH coefficients l_a) seen from direction wo is
sum_b (sum_a l_a t'_ab) Y_b(wo).  The supplementary material the paper
refers to for D, F and G is not available; the terms are the common
real-time Disney-style choices:

    D  GGX / Trowbridge-Reitz with alpha = r^2:
       D = alpha^2 / (pi ((n.h)^2 (alpha^2 - 1) + 1)^2)
    F  Schlick with F0 = 0.04 (1 - m) + m rho (per channel):
       F = F0 + (1 - F0)(1 - wo.h)^5
    G  Smith with the Schlick-GGX term, k = (r + 1)^2 / 8:
       G = G1(wi.n) G1(wo.n),  G1(x) = x / (x (1 - k) + k)

and h = (wi + wo) / |wi + wo|.  Everything is evaluated straight from these
formulas in FP64, one (splat, wi, wo) triple at a time (vectorised over the
pairs), with the visibility V of each wi ray from the oracle's brute-force
tracer (or given).
"""
from __future__ import annotations

import math

import numpy as np

EPS_C = 1e-6       # |n . w| within this of 0: an FP32 evaluation may put w on either side


def ggx_d(noh, alpha):
    a2 = alpha * alpha
    x = noh * noh * (a2 - 1.0) + 1.0
    return a2 / (math.pi * x * x)


def schlick_g1(x, k):
    return x / (x * (1.0 - k) + k)


def brdf(n, wi, wo, rho, rough, metal):
    """f(wi, wo) per channel for unit n, wi, wo [..., 3] with wi.n > 0 and
    wo.n > 0; rho [3]."""
    n, wi, wo = (np.asarray(a, dtype=np.float64) for a in (n, wi, wo))
    rho = np.asarray(rho, dtype=np.float64)
    ci = np.sum(wi * n, -1)
    co = np.sum(wo * n, -1)
    h = wi + wo
    h = h / np.linalg.norm(h, axis=-1, keepdims=True)
    noh = np.sum(n * h, -1)
    voh = np.sum(wo * h, -1)
    alpha = rough * rough
    k = (rough + 1.0) ** 2 / 8.0
    D = ggx_d(noh, alpha)
    G = schlick_g1(ci, k) * schlick_g1(co, k)
    F0 = 0.04 * (1.0 - metal) + metal * rho
    F = F0 + (1.0 - F0) * (1.0 - voh)[..., None] ** 5
    spec = (D * G / (4.0 * ci * co))[..., None] * F
    return (1.0 - metal) * rho / math.pi + spec


def _brdf_bound(n, wi, wo, rho, rough, metal):
    """|f| with the Smith terms divided out by hand, D F / (4 (ci (1-k) + k)
    (co (1-k) + k)) + the diffuse part, which equals |f| above the horizon and
    stays finite at it (ci, co clipped at 0)."""
    rho = np.asarray(rho, dtype=np.float64)
    ci = np.maximum(np.sum(wi * n, -1), 0.0)
    co = np.maximum(np.sum(wo * n, -1), 0.0)
    h = wi + wo
    h = h / np.linalg.norm(h, axis=-1, keepdims=True)
    noh = np.sum(n * h, -1)
    voh = np.sum(wo * h, -1)
    k = (rough + 1.0) ** 2 / 8.0
    D = ggx_d(noh, rough * rough)
    F0 = 0.04 * (1.0 - metal) + metal * rho
    F = F0 + (1.0 - F0) * (1.0 - voh)[..., None] ** 5
    return (1.0 - metal) * rho / math.pi + (D / (4.0 * (ci * (1 - k) + k) * (co * (1 - k) + k)))[..., None] * F


def transfer_matrix(normal, rho, rough, metal, dirs, Y, vis, devc=None):
    """t'[3, K, K] of one splat (Eq. 40) from its per-direction visibility
    vis[S] (read where n . w_s > 0).

    With `devc` [S] (a bound on |c_s| |V_fp32 - V| for each input ray, 0 for
    clear rays), also returns a bound on how far an FP32 evaluation may
    legitimately land: from those rays, from the directions within EPS_C of
    the horizon, where it may count a term or not (input side: the term
    carries the factor c, so at most EPS_C of it; output side: f stays finite
    there, the whole term), and from FP32 rounding; and the matrix of |terms|."""
    S, K = Y.shape
    wq = 4.0 * math.pi / S
    c = dirs @ normal
    s_in = np.nonzero(c > 0.0)[0]
    out = np.zeros((3, K, K))
    if s_in.size:
        wi = np.repeat(dirs[s_in][:, None, :], s_in.size, 1)
        wo = np.repeat(dirs[s_in][None, :, :], s_in.size, 0)
        f = brdf(normal, wi, wo, rho, rough, metal)                 # [s, p, 3]
        T = f * (c[s_in] * vis[s_in])[:, None, None]
        Ys = Y[s_in]
        out = wq * wq * np.einsum("sa,spc,pb->cab", Ys, T, Ys)
    if devc is None:
        return out
    near = np.nonzero(c > -EPS_C)[0]                                 # every direction that may count
    wi = np.repeat(dirs[near][:, None, :], near.size, 1)
    wo = np.repeat(dirs[near][None, :, :], near.size, 0)
    B = _brdf_bound(normal, wi, wo, rho, rough, metal)               # [s, p, 3]
    cn = c[near]
    v_in = np.where(cn > 0.0, np.abs(vis[near]), 0.0)
    amb = np.abs(cn) <= EPS_C
    w_term = (devc[near][:, None] * (cn > 0.0)[None, :]               # V of a clear input ray moves
              + (np.maximum(cn, 0.0) * v_in)[:, None] * amb[None, :]  # an output direction at the horizon
              + (np.abs(cn) * amb)[:, None])                         # an input direction at the horizon
    Ya = np.abs(Y[near])
    allow = wq * wq * np.einsum("sa,spc,sp,pb->cab", Ya, B, w_term, Ya)
    scale = np.zeros((3, K, K))
    if s_in.size:
        scale = wq * wq * np.einsum("sa,spc,pb->cab", np.abs(Ys), np.abs(T), np.abs(Ys))
    # FP32 evaluation: the half-vector terms are sums of products of unit
    # vectors (absolute error a few eps) that the GGX lobe of width alpha
    # amplifies by up to 1/alpha; the sums over s and p add about one eps
    # per term summed
    eps32 = 2.0 ** -24
    fp32 = scale * (32 * eps32 * (1.0 + 1.0 / (rough * rough)) + (s_in.size + 16) * eps32)
    return out, allow + fp32, scale


def glossy_transfer(scene, num_dirs, bands, roughness, metallic, seed=0, sources=None, vis=None,
                    want_allow=False):
    """t'[count, 3, K, K] of the listed sources (Eq. 36-41).  `vis` [count, S]
    overrides the traced visibility (entries for n . w <= 0 are not read).
    With `want_allow`, returns dict(t, allow, scale): allow bounds the change
    an FP32 evaluation can legitimately make (a tracer's different V on rays
    within rounding of a cut, horizon decisions, rounding), scale is the
    matrix of |terms|."""
    import oracle
    dirs, Y = oracle.tables(num_dirs, seed, bands)
    n = scene["means"].shape[0]
    src = np.arange(n) if sources is None else np.asarray(sources)
    devc = None
    if vis is None:
        # per-direction V and its deviation bound: the direct transfer with an
        # identity basis gives (4 pi / S) V c per direction and (4 pi / S) |dev|
        r = oracle.direct_transfer(scene, num_dirs, num_dirs, seed, sources=src, want_vis=True,
                                   want_allow=want_allow, dirs=dirs, Y=np.eye(num_dirs))
        vis = r["vis"]
        if want_allow:
            devc = r["allow"] / (4.0 * math.pi / num_dirs)          # per ray c |dV| (+ |c| at the horizon)
    elif want_allow:
        devc = np.zeros((src.size, num_dirs))                        # the given V is exact for both sides
    vis = np.asarray(vis, dtype=np.float64)
    K = Y.shape[1]
    t = np.zeros((src.size, 3, K, K))
    allow = np.zeros_like(t) if want_allow else None
    scale = np.zeros_like(t) if want_allow else None
    nrm = np.asarray(scene["normals"], dtype=np.float64)
    alb = np.asarray(scene["albedo"], dtype=np.float64)
    for q, i in enumerate(src):
        nv = nrm[i] / np.linalg.norm(nrm[i])
        if want_allow:
            t[q], allow[q], scale[q] = transfer_matrix(nv, alb[i], float(roughness[i]), float(metallic[i]), dirs, Y,
                                                       vis[q], devc=devc[q])
        else:
            t[q] = transfer_matrix(nv, alb[i], float(roughness[i]), float(metallic[i]), dirs, Y, vis[q])
    if want_allow:
        return dict(t=t, allow=allow, scale=scale)
    return t


def view_transfer(t, view_sh):
    """Per splat the transfer vector seen from one direction: z[c, a] =
    sum_b t'[c, a, b] Y_b(wo), with view_sh[count, K] = Y(wo) of each splat."""
    return np.einsum("ncab,nb->nca", t, view_sh)
