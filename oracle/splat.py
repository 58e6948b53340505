"""FP64 reference of Gaussian splatting -- TEST INFRASTRUCTURE ONLY.

The rasterizer the paper renders with (Sec. 3.1): Sigma = R S S^T R^T,
Sigma' = J W Sigma W^T J^T (EWA splatting; the 2D covariance gets the usual
0.3 pixel^2 low-pass), colours blended front to back (Eq. 4).  Per pixel,
every Gaussian with alpha >= 1/255 counts, in increasing camera depth (then
index); alpha = min(0.99, o exp(-d^T Sigma'^-1 d / 2)); the walk stops before
the Gaussian that would take T below 1e-4.  Pixel (px, py) sits at
(px + 0.5, py + 0.5); a Gaussian projects to (fx x/z + cx, fy y/z + cy); the
Jacobian takes x/z and y/z held within 1.3 times the frustum.  No tiles, no
sort keys: brute force over pixels x Gaussians.
"""
from __future__ import annotations

import numpy as np

ALPHA_MIN = 1.0 / 255.0
ALPHA_MAX = 0.99
T_STOP = 1e-4
DILATE = 0.3
EPS32 = 2.0 ** -24          # float32 unit roundoff, for the allowance of a float32 renderer


def _rot(q):
    q = q / np.linalg.norm(q, axis=-1, keepdims=True)
    w, x, y, z = q[:, 0], q[:, 1], q[:, 2], q[:, 3]
    return np.stack([
        np.stack([1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)], -1),
        np.stack([2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)], -1),
        np.stack([2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)], -1)], -2)


def project(scene, view, fx, fy, cx, cy, width, height, near_z, want_err=False):
    """Per Gaussian: screen centre [n,2], conic (inverse 2D covariance)
    [n,2,2], camera depth [n], visible mask [n]; with `want_err`, also a dict
    of first-order float32 error bounds (see `_float32_errors`)."""
    mu = np.asarray(scene["means"], dtype=np.float64)
    op = np.asarray(scene["opacity"], dtype=np.float64)
    V = np.asarray(view, dtype=np.float64).reshape(3, 4)
    xc = mu @ V[:, :3].T + V[:, 3]
    x, y, z = xc[:, 0], xc[:, 1], xc[:, 2]
    with np.errstate(divide="ignore", invalid="ignore"):
        R = _rot(np.asarray(scene["quats"], dtype=np.float64))
        s2 = np.exp(2.0 * np.asarray(scene["log_scales"], dtype=np.float64))
        sig = np.einsum("nab,nb,ncb->nac", R, s2, R)
        sig_c = np.einsum("ab,nbc,dc->nad", V[:, :3], sig, V[:, :3])
        lim = (-1.3 * cx / fx, 1.3 * (width - cx) / fx, -1.3 * cy / fy, 1.3 * (height - cy) / fy)
        tx = np.clip(x / z, lim[0], lim[1]) * z
        ty = np.clip(y / z, lim[2], lim[3]) * z
        J = np.zeros((mu.shape[0], 2, 3))
        J[:, 0, 0] = fx / z
        J[:, 0, 2] = -fx * tx / (z * z)
        J[:, 1, 1] = fy / z
        J[:, 1, 2] = -fy * ty / (z * z)
        cov = np.einsum("nab,nbc,ndc->nad", J, sig_c, J) + DILATE * np.eye(2)
        det = cov[:, 0, 0] * cov[:, 1, 1] - cov[:, 0, 1] * cov[:, 1, 0]
        conic = np.stack([np.stack([cov[:, 1, 1], -cov[:, 0, 1]], -1),
                          np.stack([-cov[:, 1, 0], cov[:, 0, 0]], -1)], -2) / det[:, None, None]
        uv = np.stack([fx * x / z + cx, fy * y / z + cy], -1)
    visible = (z >= near_z) & (det > 0) & (op > ALPHA_MIN)
    if want_err:
        return uv, conic, z, visible, _float32_errors(mu, V, xc, uv, cov, fx, fy, cx, cy)
    return uv, conic, z, visible


def _float32_errors(mu, V, xc, uv, cov, fx, fy, cx, cy):
    """What a float32 evaluation of the same formulas can be off by, to first
    order: camera-space coordinates (a 4-term dot product each), the screen
    centre (one division and a scale-and-shift), and the 2D covariance, whose
    entries carry a few roundings relative to its largest eigenvalue, so that
    its inverse is off by a multiple of eps times its condition number."""
    with np.errstate(divide="ignore", invalid="ignore"):
        mag = np.abs(mu) @ np.abs(V[:, :3]).T + np.abs(V[:, 3])
        dxyz = 4 * EPS32 * mag
        az = np.abs(xc[:, 2])
        du = fx * (dxyz[:, 0] + np.abs(xc[:, 0] / xc[:, 2]) * dxyz[:, 2]) / az + 4 * EPS32 * (np.abs(uv[:, 0]) + abs(cx))
        dv = fy * (dxyz[:, 1] + np.abs(xc[:, 1] / xc[:, 2]) * dxyz[:, 2]) / az + 4 * EPS32 * (np.abs(uv[:, 1]) + abs(cy))
        mid = 0.5 * (cov[:, 0, 0] + cov[:, 1, 1])
        rad = np.sqrt(np.maximum(mid ** 2 - (cov[:, 0, 0] * cov[:, 1, 1] - cov[:, 0, 1] ** 2), 0.0))
        lmin, lmax = mid - rad, mid + rad
    return dict(duv=np.hypot(du, dv), dz=dxyz[:, 2] + EPS32 * az, lmin=lmin, kappa=lmax / lmin)


def _reaches(uv, conic, op, idx, P, chunk=1 << 22):
    """Mask over `idx`: the Gaussians whose alpha reaches 1/510 at one of the
    pixel centres P.  The rest stay below half the 1/255 cut everywhere and
    change neither a result nor an allowance there."""
    keep = np.zeros(idx.size, dtype=bool)
    step = max(1, chunk // max(1, P.shape[0]))
    for a in range(0, idx.size, step):
        g = idx[a:a + step]
        d = uv[g][:, None, :] - P[None, :, :]
        power = -0.5 * np.einsum("gpa,gab,gpb->gp", d, conic[g], d)
        keep[a:a + step] = (op[g][:, None] * np.exp(power) >= 0.5 * ALPHA_MIN).any(1)
    return keep


def render(scene, colours, view, fx, fy, cx, cy, width, height, near_z, background=(0.0, 0.0, 0.0),
           pixels=None, want_allow=False):
    """Image [H, W, 3] and final transmittance [H, W] (or, with `pixels` =
    (px, py) index arrays, the values at those pixels only).

    With `want_allow`, also per-pixel bounds (colour, transmittance) on how far
    a float32 renderer of the same definition may legitimately land from this
    result: every alpha carries a relative error e from the float32 centre and
    conic (`_float32_errors`) plus the exponential; a change of alpha_h moves C
    by at most 2 max|c| T_h |d alpha_h| and T by at most T_h |d alpha_h|.  Where
    a decision sits within its error of its threshold, the other outcome is
    allowed for: alpha near 1/255 (the Gaussian may count or not: C moves by
    at most 2 max|c| alpha_h T_h, T by alpha_h T_h); the new T near 1e-4 (the
    walk may stop here or go on: C and T move by at most max|c| T_h and T_h);
    two taken Gaussians closer in depth than their float32 depth errors (they
    may swap: C moves by at most 2 max|c| alpha_g alpha_h T_g, T not at all)."""
    pr = project(scene, view, fx, fy, cx, cy, width, height, near_z, want_err=want_allow)
    uv, conic, z, visible = pr[:4]
    op = np.asarray(scene["opacity"], dtype=np.float64)
    col = np.asarray(colours, dtype=np.float64)
    bg = np.asarray(background, dtype=np.float64)
    if pixels is None:
        py, px = np.mgrid[0:height, 0:width]
        px, py = px.ravel(), py.ravel()
    else:
        px, py = (np.asarray(a) for a in pixels)
    P = np.stack([px + 0.5, py + 0.5], -1)
    idx = np.nonzero(visible)[0]
    if pixels is not None:
        idx = idx[_reaches(uv, conic, op, idx, P)]
    order = idx[np.lexsort((idx, z[idx]))]           # by depth, then index
    npix = P.shape[0]
    T = np.ones(npix)
    C = np.zeros((npix, 3))
    live = np.ones(npix, dtype=bool)
    if want_allow:
        err = pr[4]
        cont = np.zeros(npix)            # sum of T_h alpha_h e_h over taken Gaussians
        disc = np.zeros(npix)            # near-threshold decisions, in units of 2 max|c|
        trel = np.zeros(npix)            # relative error bound of T
        taken = np.zeros(npix)
        z_prev = np.full(npix, np.nan)
        dz_prev = np.zeros(npix)
        T_prev = np.ones(npix)
        a_prev = np.zeros(npix)
    for g in order:
        d = uv[g][None, :] - P
        power = -0.5 * np.einsum("pa,ab,pb->p", d, conic[g], d)
        alpha = np.minimum(ALPHA_MAX, op[g] * np.exp(power))
        take = live & (alpha >= ALPHA_MIN) & (power <= 0.0)
        Tn = T * (1.0 - alpha)
        if want_allow:
            q = np.maximum(-2.0 * power, 0.0)
            # the exponential itself: an FP32 exp may go through 2^(x log2 e),
            # whose rounded product adds about |x| log2(e) eps (|x| = q / 2)
            e = 0.5 * (24 * EPS32 * err["kappa"][g] * q + 2 * np.sqrt(q / err["lmin"][g]) * err["duv"][g]) \
                + (4 + q) * EPS32
            if not 24 * EPS32 * err["kappa"][g] < 0.5:
                e = np.full(npix, np.inf)
            near_alpha = live & (np.abs(alpha - ALPHA_MIN) <= 4 * e * alpha)
            disc += np.where(near_alpha, T * alpha * (1 + 4 * e), 0.0)
            trel_n = trel + alpha * e / (1.0 - alpha) + 2 * EPS32
            disc += np.where(take & (np.abs(Tn - T_STOP) <= 4 * trel_n * Tn), T, 0.0)
            tie = take & (np.abs(z[g] - z_prev) <= 2 * (err["dz"][g] + dz_prev))
            disc += np.where(tie, T_prev * a_prev * alpha, 0.0)
        stop = take & (Tn < T_STOP)
        live &= ~stop
        take &= ~stop
        C[take] += col[g][None, :] * (alpha[take] * T[take])[:, None]
        if want_allow:
            cont += np.where(take, T * alpha * e, 0.0)
            trel = np.where(take, trel_n, trel)
            taken += take
            T_prev = np.where(take, T, T_prev)
            a_prev = np.where(take, alpha, a_prev)
            z_prev = np.where(take, z[g], z_prev)
            dz_prev = np.where(take, err["dz"][g], dz_prev)
        T = np.where(take, Tn, T)
    img = C + T[:, None] * bg[None, :]
    out = [img, T]
    if want_allow:
        maxc = np.abs(col).max() if col.size else 0.0
        allow_T = np.minimum(cont + disc + T * trel + 4 * EPS32, 1.0)
        # alpha errors reach C through cont (their effect on T included); the
        # rest is the rounding of each product T (1 - alpha) and each sum
        allow_C = maxc * (2 * (cont + disc) + 2 * EPS32 * (2 * taken + 1)) + np.abs(bg).max() * allow_T
        out += [allow_C, allow_T]
    if pixels is None:
        out = [out[0].reshape(height, width, 3)] + [a.reshape(height, width) for a in out[1:]]
    return tuple(out)
