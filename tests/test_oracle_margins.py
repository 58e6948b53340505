"""Sizing of the oracle's rounding margins against a float32 model of the GPU
evaluation (tests/fp32_model.py), on the geometry of the surface workload
(100,000 splats, S = 256) and the million-splat workload (S = 512).

The parity rule lets a near-threshold predicate go either way when the value
it tests lies within its margin of the threshold (the reading of the
paper's ray tracing, Sec. 4.4, under FP32 rounding).  Each margin must be at
least 10x the largest deviation of the float32 model from the exact FP64
value over every sampled (ray, Gaussian) pair within reach of the 3-sigma
extent, and the first, conservative stage of the GPU test must never drop a
pair that the exact stage would hit."""
import numpy as np
import pytest

import fp32_model as fm
import scenegen

SAFETY = 10.0


def _rotation(q):
    q = q / np.linalg.norm(q, axis=1, keepdims=True)
    w, x, y, z = q.T
    return np.stack([np.stack([1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)], -1),
                     np.stack([2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)], -1),
                     np.stack([2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)], -1)], -2)


def _pairs(scene, dirs, n_src, seed, max_rays=None):
    """Every (ray, Gaussian) pair with exact d^2 <= 12 and the peak ahead of
    -3.3 s_max, for the traced rays of sampled sources; exact t*, d^2 in FP64
    (Eq. 1-2: Sigma^-1 = R diag(s^-2) R^T)."""
    rng = np.random.default_rng(seed)
    sc = {k: np.asarray(v, np.float32).astype(np.float64) for k, v in scene.items()}
    n = sc["means"].shape[0]
    s = np.exp(sc["log_scales"])
    smax = s.max(1)
    R = _rotation(sc["quats"])
    sinv = np.einsum("nab,nb,ncb->nac", R, 1.0 / s ** 2, R)
    out = []
    for i in rng.choice(n, n_src, replace=False):
        c = sc["normals"][i] @ dirs.T
        rays = np.nonzero(c > 0)[0]
        if max_rays and len(rays) > max_rays:
            rays = rng.choice(rays, max_rays, replace=False)
        o = sc["means"][i]
        rel = sc["means"] - o
        for sd in rays:
            w = dirs[sd]
            proj = rel @ w
            perp2 = (rel * rel).sum(1) - proj ** 2
            cand = np.nonzero((perp2 <= (3.3 * smax) ** 2) & (proj > -3.3 * smax))[0]
            cand = cand[cand != i]
            sw = sinv[cand] @ w
            t = (rel[cand] * sw).sum(1) / (sw * w).sum(1)
            e = o + t[:, None] * w - sc["means"][cand]
            d2 = np.einsum("na,nab,nb->n", e, sinv[cand], e)
            keep = d2 <= 12.0
            out.append((np.full(keep.sum(), i), np.full(keep.sum(), sd), cand[keep], t[keep], d2[keep]))
    I, Sd, J, T, D2 = (np.concatenate(x) for x in zip(*out))
    return sc, I, Sd, J, T, D2


@pytest.mark.slow
@pytest.mark.parametrize("name,n_src,max_rays", [("surface100k", 12, None), ("million", 4, 150)])
def test_margins_cover_fp32_model(oracle_mod, name, n_src, max_rays):
    w = scenegen.workload(name)
    dirs = oracle_mod.directions(w["num_dirs"])
    sc, I, Sd, J, T, D2 = _pairs(w["scene"], dirs, n_src, 11, max_rays)
    assert len(J) > 20000 and (D2 <= 9.0).sum() > 5000 and (np.abs(D2 - 9.0) < 0.5).sum() > 100
    rng = np.random.default_rng(12)
    mar_c, mar_d2, mar_t, mar_T, mar_tr = oracle_mod.DEFAULT_MARGINS
    s = np.exp(sc["log_scales"][J])
    kappa = s.max(1) / s.min(1)
    W = fm.records(sc["quats"][J], sc["log_scales"][J], rng)
    t32, d2_32, d2_pre, err = fm.ray_test(W, sc["means"][J], sc["means"][I], dirs[Sd], rng)
    # d^2 against sigma_cut^2: margin mar_d2 (1 + kappa)
    r_d2 = np.abs(d2_32 - D2) / (1.0 + kappa)
    # t* against t_min: margin mar_t (1 + d) / |W w| + mar_tr |t*|, |W w|^2 = w^T Sigma^-1 w
    Ww = np.linalg.norm(np.einsum("nab,nb->na", _rotation(sc["quats"][J]).transpose(0, 2, 1), dirs[Sd]) / s, axis=1)
    r_t = np.abs(t32 - T) / (mar_t * (1.0 + np.sqrt(D2)) / Ww + mar_tr * np.abs(T))
    # the first stage keeps every pair the exact stage hits
    lim = 3.0 + err
    dropped = (d2_32 <= 9.0) & ~(d2_pre <= lim * lim)
    # hemisphere c = n . w against 0
    c32 = fm.hemisphere(sc["normals"][I], dirs[Sd])
    r_c = np.abs(c32 - (sc["normals"][I] * dirs[Sd]).sum(1))
    # transmittance of each sampled ray (product over its exact hits) against T_eps
    a32 = fm.alpha(sc["opacity"][J], d2_32, 0.99, rng)
    a64 = np.minimum(sc["opacity"][J] * np.exp(-0.5 * D2), 0.99)
    key = I.astype(np.int64) * 100_000 + Sd
    order = np.argsort(key, kind="stable")
    _, starts = np.unique(key[order], return_index=True)
    r_T = []
    for a, b in zip(starts, list(starts[1:]) + [len(order)]):
        h = order[a:b]
        h = h[(D2[h] <= 9.0) & (T[h] > 0.0)]
        T64 = float(np.prod(1.0 - a64[h]))
        if len(h) and T64 >= 0.5e-4:
            r_T.append(abs(fm.transmittance(a32[h]) / T64 - 1.0))
    r_T = np.array(r_T)
    print(f"{name}: {len(J)} pairs, {len(r_T)} rays; largest error / margin scale: d2 {r_d2.max():.2e} "
          f"(margin {mar_d2:.0e}), t {r_t.max():.2e} (of its margin), c {r_c.max():.2e} ({mar_c:.0e}), "
          f"T {r_T.max():.2e} ({mar_T:.0e})")
    assert not dropped.any()
    assert SAFETY * r_d2.max() <= mar_d2
    assert SAFETY * r_t.max() <= 1.0
    assert SAFETY * r_c.max() <= mar_c
    assert SAFETY * r_T.max() <= mar_T
