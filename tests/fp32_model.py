"""A float32 model of the GPU ray-Gaussian test, for sizing the oracle's
rounding margins (test infrastructure; the HIP library is not imported).

The margins of the oracle bound how far an FP32 evaluation of the hit
predicates (hemisphere c = n . w > 0; peak depth t* > t_min; Mahalanobis
distance d^2 <= sigma_cut^2 at the peak; transmittance against T_eps) may
lie from the exact values.  This module restates, operation by operation in
NumPy float32, how the GPU path forms those values:

* the Gaussian record: the quaternion normalised by a reciprocal square
  root, R(q) (Eq. 2), 1/s = exp(-log s), whitening rows W = diag(1/s) R^T;
* a first estimate of t* from o' = W (origin - mu), d' = W w;
* the exact stage: x = origin - mu + t w from the exact two-float difference
  origin - mu (TwoSum), p = W x, one Newton step on t, d^2 = |p|^2;
* alpha = o exp(-d^2 / 2) (an exp2 of a rounded product), T = prod(1 - alpha).

Every float32 operation rounds to nearest; fused multiply-adds round once
(the product of two float32 values is exact in float64).  The hardware's
approximate operations (reciprocal square root, reciprocal, exp, exp2) are
modelled as the correctly rounded value moved by up to one unit in the last
place, at random, so that the model errs on the side of larger errors.
"""
from __future__ import annotations

import numpy as np

F32 = np.float32


def rn(x):
    """Round float64 values to float32."""
    return np.asarray(x, dtype=np.float64).astype(F32)


def fma(a, b, c):
    """a * b + c rounded once to float32 (a b is exact in float64)."""
    return rn(np.asarray(a, np.float64) * np.asarray(b, np.float64) + np.asarray(c, np.float64))


def approx(exact, rng):
    """A hardware approximation: the float32 rounding of `exact` moved by up
    to one ulp at random."""
    r = rn(exact)
    k = rng.integers(-1, 2, size=np.shape(r))
    up = np.nextafter(r, F32(np.inf))
    dn = np.nextafter(r, F32(-np.inf))
    return np.where(k > 0, up, np.where(k < 0, dn, r)).astype(F32)


def _mul(a, b):
    return rn(np.asarray(a, np.float64) * np.asarray(b, np.float64))


def _dot(a, b):
    """3-vectors along the last axis: fma(a2, b2, fma(a1, b1, a0 b0))."""
    return fma(a[..., 2], b[..., 2], fma(a[..., 1], b[..., 1], _mul(a[..., 0], b[..., 0])))


def records(quats, log_scales, rng):
    """Whitening rows W [n, 3, 3] (row a = column a of R divided by s_a) as
    the GPU builds them from float32 quaternions and log-scales."""
    q = rn(quats)
    qw, qx, qy, qz = q[:, 0], q[:, 1], q[:, 2], q[:, 3]
    qn2 = fma(qz, qz, fma(qy, qy, fma(qx, qx, _mul(qw, qw))))
    inv = approx(1.0 / np.sqrt(qn2.astype(np.float64)), rng)
    qw, qx, qy, qz = _mul(qw, inv), _mul(qx, inv), _mul(qy, inv), _mul(qz, inv)
    one, two = F32(1.0), F32(2.0)
    R = np.empty((len(q), 3, 3), dtype=F32)
    R[:, 0, 0] = rn(one - _mul(two, fma(qz, qz, _mul(qy, qy))))
    R[:, 0, 1] = _mul(two, fma(-qw, qz, _mul(qx, qy)))
    R[:, 0, 2] = _mul(two, fma(qw, qy, _mul(qx, qz)))
    R[:, 1, 0] = _mul(two, fma(qw, qz, _mul(qx, qy)))
    R[:, 1, 1] = rn(one - _mul(two, fma(qz, qz, _mul(qx, qx))))
    R[:, 1, 2] = _mul(two, fma(-qw, qx, _mul(qy, qz)))
    R[:, 2, 0] = _mul(two, fma(-qw, qy, _mul(qx, qz)))
    R[:, 2, 1] = _mul(two, fma(qw, qx, _mul(qy, qz)))
    R[:, 2, 2] = rn(one - _mul(two, fma(qy, qy, _mul(qx, qx))))
    inv_s = approx(np.exp(-rn(log_scales).astype(np.float64)), rng)
    W = np.empty_like(R)
    for a in range(3):
        W[:, a, :] = _mul(R[:, :, a], inv_s[:, a:a + 1])
    return W


def ray_test(W, mu, origin, w, rng):
    """Peak depth t* and d^2 of rays origin[r] + t w[r] against Gaussians
    (W[r], mu[r]) as the GPU's exact stage computes them, and the first
    stage's conservative `maybe` flag (given 1 / s_min per Gaussian through
    W).  All arguments [r, ...]; returns float64 copies."""
    o = rn(origin)
    m = rn(mu)
    wd = rn(w)
    dx = rn(o.astype(np.float64) - m)            # origin - mu, rounded
    bb = rn(dx.astype(np.float64) - o)
    ex = rn(rn(o.astype(np.float64) - rn(dx.astype(np.float64) - bb)) - rn(m.astype(np.float64) + bb))
    op = np.stack([_dot(W[:, a, :], dx) for a in range(3)], -1)      # o' = W (origin - mu)
    e = np.stack([_dot(W[:, a, :], wd) for a in range(3)], -1)       # d' = W w
    ia = approx(1.0 / _dot(e, e).astype(np.float64), rng)
    t = -_mul(_dot(op, e), ia)
    p_pre = np.stack([fma(t, e[:, a], op[:, a]) for a in range(3)], -1)
    d2_pre = _dot(p_pre, p_pre)
    smin_inv = np.max(np.linalg.norm(W.astype(np.float64), axis=2), axis=1)
    err = rn(2e-6 * (np.abs(dx).astype(np.float64).sum(1) * smin_inv + 1.0))
    x = np.stack([rn(fma(t, wd[:, a], dx[:, a]).astype(np.float64) + ex[:, a]) for a in range(3)], -1)
    p = np.stack([_dot(W[:, a, :], x) for a in range(3)], -1)
    dt = _mul(_dot(p, e), ia)
    t = rn(t.astype(np.float64) - dt)
    p = np.stack([fma(-dt, e[:, a], p[:, a]) for a in range(3)], -1)
    d2 = _dot(p, p)
    return t.astype(np.float64), d2.astype(np.float64), d2_pre.astype(np.float64), err.astype(np.float64)


def hemisphere(normals, w):
    """c = n . w in float32."""
    return _dot(rn(normals), rn(w)).astype(np.float64)


def alpha(opacity, d2, alpha_max, rng):
    """alpha = min(o exp(-d^2 / 2), alpha_max) with exp as exp2 of the
    rounded product by log2(e), both in float32."""
    arg = _mul(rn(-0.5 * np.asarray(d2, np.float64)), F32(1.4426950408889634))
    E = approx(np.exp2(arg.astype(np.float64)), rng)
    return np.minimum(_mul(rn(opacity), E), F32(alpha_max))


def transmittance(alphas):
    """prod(1 - alpha) in float32, in the given order."""
    T = F32(1.0)
    for a in alphas:
        T = _mul(T, rn(F32(1.0) - a))
    return float(T)
