"""Pins of the glossy transfer-matrix oracle (Sec. 4.2 BRDF, Sec. 4.5 Eq. 36-41):
the BRDF at closed-form angles, reciprocity, the GGX normalisation, the
double sum's index placement on separable BRDFs, and the directional albedo
against an independent adaptive integral."""
import math

import numpy as np
import pytest
from scipy import integrate

import oracle
import scenegen
from oracle import glossy


def _unit(v):
    v = np.asarray(v, dtype=np.float64)
    return v / np.linalg.norm(v, axis=-1, keepdims=True)


def test_brdf_at_normal_incidence():
    """wi = wo = n: h = n, D = 1 / (pi alpha^2), G = 1, F = F0."""
    n = np.array([0.0, 0.0, 1.0])
    rho = np.array([0.2, 0.5, 0.8])
    for r, m in ((0.5, 0.3), (0.9, 0.0), (0.25, 1.0)):
        f = glossy.brdf(n, n, n, rho, r, m)
        F0 = 0.04 * (1 - m) + m * rho
        expect = (1 - m) * rho / math.pi + F0 / (4 * math.pi * r ** 4)
        assert np.allclose(f, expect, rtol=1e-12)


def test_brdf_hand_computed_off_axis():
    """wi at 60 degrees and wo at 30 degrees from n on the same side of one
    plane: h lies at 45 degrees, 15 degrees from wo."""
    n = np.array([0.0, 0.0, 1.0])
    wi = np.array([math.sin(math.radians(60)), 0.0, math.cos(math.radians(60))])
    wo = np.array([math.sin(math.radians(30)), 0.0, math.cos(math.radians(30))])
    r, m, rho = 0.6, 0.0, np.array([0.5, 0.5, 0.5])
    noh, voh = math.cos(math.radians(45)), math.cos(math.radians(15))
    a2 = r ** 4
    D = a2 / (math.pi * (noh ** 2 * (a2 - 1) + 1) ** 2)
    k = (r + 1) ** 2 / 8
    ci, co = 0.5, math.cos(math.radians(30))
    G = (ci / (ci * (1 - k) + k)) * (co / (co * (1 - k) + k))
    F = 0.04 + 0.96 * (1 - voh) ** 5
    expect = 0.5 / math.pi + D * F * G / (4 * ci * co)
    assert np.allclose(glossy.brdf(n, wi, wo, rho, r, m), expect, rtol=1e-12)


def test_brdf_reciprocity():
    rng = np.random.default_rng(0)
    n = _unit(rng.standard_normal(3))
    for _ in range(50):
        a, b = _unit(rng.standard_normal((2, 3)))
        a, b = (v if v @ n > 0 else -v for v in (a, b))
        rho = rng.uniform(0, 1, 3)
        r, m = rng.uniform(0.1, 1.0), rng.uniform(0, 1)
        assert np.allclose(glossy.brdf(n, a, b, rho, r, m), glossy.brdf(n, b, a, rho, r, m), rtol=1e-12)


@pytest.mark.parametrize("r", [0.2, 0.5, 0.9])
def test_ggx_normalisation(r):
    """The projected microfacet distribution integrates to one."""
    val, _ = integrate.quad(lambda th: glossy.ggx_d(math.cos(th), r * r) * math.cos(th) * math.sin(th),
                            0, math.pi / 2, limit=200, points=[0.0, r * r])
    assert math.isclose(2 * math.pi * val, 1.0, rel_tol=1e-8)


def test_schlick_limits():
    n = np.array([0.0, 0.0, 1.0])
    rho = np.array([0.3, 0.6, 0.9])
    # wi and wo almost opposite, both just above the horizon: h = n, wo . h -> 0, F -> 1 for any F0
    wi = _unit([1.0, 0.0, 1e-8])
    wo = _unit([-1.0, 0.0, 1e-8])
    f = glossy.brdf(n, wi, wo, rho, 0.5, 1.0)
    h = _unit(wi + wo)
    k = (1.5) ** 2 / 8
    g1 = wi @ n / ((wi @ n) * (1 - k) + k)
    D = glossy.ggx_d(h @ n, 0.25)
    assert np.allclose(f, D * g1 * g1 / (4 * (wi @ n) ** 2) * 1.0, rtol=1e-6)


def _one_splat(n_vec, S=128, bands=4):
    dirs, Y = oracle.tables(S, 0, bands)
    return _unit(n_vec), dirs, Y


def test_separable_brdf_gives_rank_one(monkeypatch):
    """With f(wi, wo) = g(wi) k(wo) the double sum factors:
    t'_ab = (wq sum_s Y_a g c V)(wq sum_p k Y_b), input index first."""
    n, dirs, Y = _one_splat([0.3, -0.2, 0.9])
    S = dirs.shape[0]
    wq = 4 * math.pi / S
    g = lambda w: 1.0 + 0.7 * w[..., 0] + 0.2 * w[..., 2] ** 2
    k = lambda w: 0.5 - 0.4 * w[..., 1] + 0.3 * w[..., 0] * w[..., 2]
    ch = np.array([1.0, 2.0, -0.5])
    monkeypatch.setattr(glossy, "brdf", lambda n_, wi, wo, rho, r, m: (g(wi) * k(wo))[..., None] * ch)
    vis = np.random.default_rng(3).uniform(0, 1, S)
    t = glossy.transfer_matrix(n, np.ones(3), 0.5, 0.0, dirs, Y, vis)
    c = dirs @ n
    up = c > 0
    left = wq * np.einsum("sa,s->a", Y[up], g(dirs[up]) * c[up] * vis[up])
    right = wq * np.einsum("pb,p->b", Y[up], k(dirs[up]))
    for j in range(3):
        assert np.allclose(t[j], ch[j] * np.outer(left, right), rtol=1e-12, atol=1e-14)
    assert not np.allclose(t[0], t[0].T, atol=1e-3)          # the two factors differ, so would a transpose


def test_lambertian_part_is_direct_transfer_times_hemisphere(monkeypatch):
    """A constant BRDF rho/pi: t'_ab = (rho / pi) t_dir[a] h[b], t_dir the
    direct transfer of the same splat (the pinned direct oracle) and h the
    hemisphere integral of Y_b, which for n = z approaches sqrt(pi),
    sqrt(3 pi)/2, 0, -sqrt(7 pi)/8 on the zonal terms."""
    monkeypatch.setattr(glossy, "brdf", lambda n_, wi, wo, rho, r, m: np.broadcast_to(
        np.asarray(rho) / math.pi, wi.shape[:-1] + (3,)))
    sc = scenegen.random_cloud(25, 7)
    sc["normals"][:] = [0.0, 0.0, 1.0]
    S, bands = 256, 4
    rho = sc["albedo"]
    t = glossy.glossy_transfer(sc, S, bands, np.full(25, 0.5), np.zeros(25), sources=[0, 3])
    td = oracle.direct_transfer(sc, S, bands, sources=[0, 3])["t"]
    dirs, Y = oracle.tables(S, 0, bands)
    h = 4 * math.pi / S * Y[dirs[:, 2] > 0].sum(0)
    for q, i in enumerate([0, 3]):
        for ch in range(3):
            assert np.allclose(t[q, ch], rho[i, ch] / math.pi * np.outer(td[q], h), rtol=1e-10, atol=1e-13)
    # the output side, read off the oracle's first row: the hemisphere integrals
    # (to the stratified quadrature's accuracy at the horizon, ~1/sqrt(S))
    h_ora = t[0, 0, 0] / (rho[0, 0] / math.pi * td[0, 0])
    zonal = {0: math.sqrt(math.pi), 2: math.sqrt(3 * math.pi) / 2, 6: 0.0, 12: -math.sqrt(7 * math.pi) / 8}
    for k_, v in zonal.items():
        assert abs(h_ora[k_] - v) < 0.05
    assert np.abs(h_ora[[1, 3, 4, 5, 7, 8, 9, 10, 11, 13, 14, 15]]).max() < 0.05


def _albedo_integral(n, wo, rho, r, m):
    """E(wo) = int f(wi, wo) (wi . n) dwi over the hemisphere, adaptive
    quadrature in the frame of n (independent of the oracle's directions)."""
    t1 = _unit(np.cross(n, [0.3, 0.5, 0.7]))
    t2 = np.cross(n, t1)

    def integrand(phi, th, ch):
        wi = math.sin(th) * (math.cos(phi) * t1 + math.sin(phi) * t2) + math.cos(th) * n
        return glossy.brdf(n, wi, wo, rho, r, m)[ch] * math.cos(th) * math.sin(th)
    return [integrate.dblquad(integrand, 0, math.pi / 2, 0, 2 * math.pi, args=(ch,), epsabs=1e-7)[0]
            for ch in range(3)]


def test_directional_albedo_by_relighting_a_white_sky():
    """A constant unit light and no occlusion: sum_a l_a t'_ab with l = e_0 / Y_00
    is the quadrature projection of E(wo) onto Y_b.  Reconstructing with the
    same outgoing directions, sum_b u_b Y_b(w_p) summed against Y again must
    match E computed by an independent adaptive integral, per direction, to
    the stratified quadrature's accuracy; and E <= 1 (energy)."""
    S, bands = 1024, 4
    dirs, Y = oracle.tables(S, 0, bands)
    n = _unit([0.2, 0.1, 1.0])
    rho, r, m = np.array([0.9, 0.6, 0.3]), 0.9, 0.4
    c = dirs @ n
    t = glossy.transfer_matrix(n, rho, r, m, dirs, Y, np.ones(S))
    l0 = 1.0 / (0.5 / math.sqrt(math.pi))
    u = l0 * t[:, 0, :]                                       # [3, K]
    wq = 4 * math.pi / S
    # u_b = wq sum_p E_hat(w_p) Y_b(w_p) with E_hat the inner quadrature; check it
    # against the same outer sum over the adaptive E at a subset of directions
    rng = np.random.default_rng(4)
    pick = rng.choice(np.nonzero(c > 0.05)[0], 6, replace=False)
    E = np.array([_albedo_integral(n, dirs[p], rho, r, m) for p in pick])      # [6, 3]
    up = np.nonzero(c > 0)[0]
    inner = np.stack([wq * np.einsum("sc,s->c", glossy.brdf(n, dirs[up], np.repeat(dirs[p][None], up.size, 0),
                                                            rho, r, m), c[up]) for p in pick])
    assert np.allclose(inner, E, rtol=2e-2)
    assert (E <= 1.0 + 1e-6).all()
    # and u is exactly that inner quadrature projected on the outgoing directions
    all_inner = np.stack([wq * np.einsum("sc,s->c", glossy.brdf(n, dirs[up], np.repeat(dirs[p][None], up.size, 0),
                                                                rho, r, m), c[up]) for p in up])
    u_ref = wq * np.einsum("pc,pb->cb", all_inner, Y[up])
    assert np.allclose(u, u_ref, rtol=1e-10, atol=1e-13)


def test_visibility_enters_linearly():
    sc = scenegen.random_cloud(20, 9)
    S, bands = 64, 3
    rng = np.random.default_rng(10)
    rough, metal = rng.uniform(0.2, 0.9, 20), rng.uniform(0, 1, 20)
    traced = glossy.glossy_transfer(sc, S, bands, rough, metal, sources=[1, 2])
    vis = oracle.direct_transfer(sc, S, bands, sources=[1, 2], want_vis=True)["vis"]
    given = glossy.glossy_transfer(sc, S, bands, rough, metal, sources=[1, 2], vis=vis)
    assert np.array_equal(traced, given)
    half = glossy.glossy_transfer(sc, S, bands, rough, metal, sources=[1, 2], vis=0.5 * vis)
    assert np.allclose(half, 0.5 * traced, rtol=1e-12, atol=1e-15)
    assert (glossy.glossy_transfer(sc, S, bands, rough, metal, sources=[1], vis=np.zeros((1, S))) == 0).all()


def test_view_transfer_contracts_the_output_index():
    """z[c][a] = sum_b t'[c][a][b] Y_b(wo): a unit matrix entry (a = 2, b = 5)
    gives Y_5(wo) in slot a = 2 and zeros elsewhere; a light l then sees
    l_2 Y_5(wo), the outgoing radiance of Eq. 41 for that entry."""
    wo = _unit([[0.3, -0.5, 0.8]])
    y = oracle.sh_basis(4, wo)                      # [1, 16]
    t = np.zeros((1, 3, 16, 16))
    t[0, 1, 2, 5] = 1.0
    z = glossy.view_transfer(t, y)
    expect = np.zeros((1, 3, 16))
    expect[0, 1, 2] = y[0, 5]
    assert np.array_equal(z, expect)
    # Y_5 is the (l = 2, m = -1) function: -sqrt(15 / (4 pi)) y z for a unit vector
    assert math.isclose(y[0, 5], -math.sqrt(15 / (4 * math.pi)) * wo[0, 1] * wo[0, 2], rel_tol=1e-12)
