"""Pins of the CPU FP64 oracle against facts fixed by the paper and by
mathematics (closed forms, library routines, invariants, brute force)."""
import math
import os

import numpy as np
import pytest

import scenegen

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
LOBE = [math.pi, 2 * math.pi / 3, math.pi / 4, 0.0, -math.pi / 24]  # clamped-cosine band gains


def _golden(name):
    vals = {}
    nums = []
    for line in open(os.path.join(GOLDEN, name)):
        line = line.split("#")[0].strip()
        if not line:
            continue
        parts = line.split()
        if len(parts) == 2:
            vals[parts[0]] = float(parts[1]) if parts[0] != "seed" else int(parts[1])
        else:
            nums.append(int(parts[0]))
    return vals, nums


def _scene(means, sigmas, opac, normals=None, quats=None):
    n = len(means)
    means = np.asarray(means, dtype=np.float64)
    sig = np.asarray(sigmas, dtype=np.float64)
    if sig.ndim == 1:
        sig = np.repeat(sig[:, None], 3, 1)
    return dict(
        means=means,
        quats=np.tile([1.0, 0, 0, 0], (n, 1)) if quats is None else np.asarray(quats, dtype=np.float64),
        log_scales=np.log(sig),
        opacity=np.asarray(opac, dtype=np.float64),
        normals=np.tile([0.0, 0, 1], (n, 1)) if normals is None else np.asarray(normals, dtype=np.float64),
        albedo=np.full((n, 3), 0.5),
    )


# --------------------------------------------------------------------------
# direction table
# --------------------------------------------------------------------------

def test_splitmix64_published_vector(oracle_mod):
    vals, nums = _golden("splitmix64.txt")
    got = [oracle_mod.splitmix64(vals["seed"], i) for i in range(len(nums))]
    assert got == nums


@pytest.mark.parametrize("S,grid", [(64, (8, 8)), (256, (16, 16)), (512, (16, 32)), (1, (1, 1)),
                                    (7, (1, 7)), (12, (3, 4))])
def test_grid(oracle_mod, S, grid):
    assert oracle_mod.grid(S) == grid


@pytest.mark.parametrize("S", [64, 256, 512, 12])
def test_directions_stratified(oracle_mod, S):
    """Each direction lies in its own equal-area stratum (4 pi / S each)."""
    d = oracle_mod.directions(S, 0)
    nu, nv = oracle_mod.grid(S)
    assert np.allclose(np.linalg.norm(d, axis=1), 1.0, atol=3e-7)
    for s in range(S):
        a, b = divmod(s, nv)
        z = d[s, 2]
        assert 1 - 2 * (a + 1) / nu - 1e-6 <= z <= 1 - 2 * a / nu + 1e-6
        phi = math.atan2(d[s, 1], d[s, 0]) % (2 * math.pi)
        lo, hi = 2 * math.pi * b / nv, 2 * math.pi * (b + 1) / nv
        assert lo - 1e-5 <= phi <= hi + 1e-5 or (b == nv - 1 and phi < 1e-5)
    # exactly FP32 values
    assert np.array_equal(d, d.astype(np.float32).astype(np.float64))


def test_directions_seed_changes_jitter(oracle_mod):
    assert not np.array_equal(oracle_mod.directions(64, 0), oracle_mod.directions(64, 1))
    assert np.array_equal(oracle_mod.directions(64, 5), oracle_mod.directions(64, 5))


# --------------------------------------------------------------------------
# real spherical harmonics (Eq. 8-13)
# --------------------------------------------------------------------------

def _product_rule(nz, nphi):
    x, w = np.polynomial.legendre.leggauss(nz)
    phi = 2 * math.pi * (np.arange(nphi) + 0.5) / nphi
    Z, P = np.meshgrid(x, phi, indexing="ij")
    r = np.sqrt(1 - Z ** 2)
    dirs = np.stack([r * np.cos(P), r * np.sin(P), Z], -1).reshape(-1, 3)
    wts = (w[:, None] * np.full(nphi, 2 * math.pi / nphi)[None, :]).reshape(-1)
    return dirs, wts


@pytest.mark.parametrize("bands", [3, 4, 6])
def test_sh_orthonormal_exact_quadrature(oracle_mod, bands):
    """Gauss-Legendre in z x uniform phi integrates these polynomials exactly:
    the Gram matrix is the identity (Eq. 13)."""
    dirs, w = _product_rule(12, 24)
    Y = oracle_mod.sh_basis(bands, dirs)
    G = (Y * w[:, None]).T @ Y
    assert np.abs(G - np.eye(bands * bands)).max() < 1e-13


def test_sh_addition_theorem(oracle_mod):
    rng = np.random.default_rng(7)
    a = rng.standard_normal((20, 3))
    b = rng.standard_normal((20, 3))
    a /= np.linalg.norm(a, axis=1, keepdims=True)
    b /= np.linalg.norm(b, axis=1, keepdims=True)
    Ya = oracle_mod.sh_basis(6, a)
    Yb = oracle_mod.sh_basis(6, b)
    for ell in range(6):
        sl = slice(ell * ell, (ell + 1) ** 2)
        lhs = (Ya[:, sl] * Yb[:, sl]).sum(1)
        coef = np.zeros(ell + 1)
        coef[ell] = 1
        rhs = (2 * ell + 1) / (4 * math.pi) * np.polynomial.legendre.legval((a * b).sum(1), coef)
        assert np.abs(lhs - rhs).max() < 1e-13


def test_sh_matches_scipy_complex_harmonics(oracle_mod):
    """Real basis from SciPy's complex harmonics (Condon-Shortley phase):
    sqrt2 Re Y_l^m for m > 0, sqrt2 Im Y_l^|m| for m < 0."""
    from scipy.special import sph_harm_y
    rng = np.random.default_rng(3)
    d = rng.standard_normal((30, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    theta = np.arccos(d[:, 2])
    phi = np.arctan2(d[:, 1], d[:, 0])
    Y = oracle_mod.sh_basis(5, d)
    for ell in range(5):
        for m in range(-ell, ell + 1):
            c = sph_harm_y(ell, abs(m), theta, phi)
            ref = c.real if m == 0 else (math.sqrt(2) * (c.real if m > 0 else c.imag))
            assert np.abs(Y[:, ell * ell + ell + m] - ref).max() < 1e-12


def test_sh_band1_signs(oracle_mod):
    k = math.sqrt(3 / (4 * math.pi))
    Y = oracle_mod.sh_basis(2, np.array([[0.3, -0.4, math.sqrt(1 - 0.25)]]))[0]
    x, y, z = 0.3, -0.4, math.sqrt(0.75)
    assert np.allclose(Y, [0.5 / math.sqrt(math.pi), -k * y, k * z, -k * x], atol=1e-15)


# Largest |Gram - I| over 5 seeds measured for the stratified quadrature
# (K = 16); the quadrature error shrinks roughly as 1/S.
@pytest.mark.parametrize("S,bound", [(64, 0.283), (256, 0.0840), (512, 0.0616), (4096, 0.00506)])
def test_sh_orthonormality_under_stratified_quadrature(oracle_mod, S, bound):
    worst = 0.0
    for seed in range(5):
        _, Y = oracle_mod.tables(S, seed, 4)
        G = (4 * math.pi / S) * Y.T @ Y
        worst = max(worst, np.abs(G - np.eye(16)).max())
    assert worst <= 1.5 * bound


# --------------------------------------------------------------------------
# direct transfer closed forms
# --------------------------------------------------------------------------

def _lobe_expect(oracle_mod, normal, bands):
    Yn = oracle_mod.sh_basis(bands, np.asarray(normal, dtype=np.float64))[0]
    return np.array([LOBE[math.isqrt(k)] * Yn[k] for k in range(bands * bands)])


@pytest.mark.parametrize("normal", [[0, 0, 1.0], [0.6, 0.0, 0.8], [-0.2, 0.9, -0.3]])
def test_empty_scene_is_clamped_cosine(oracle_mod, normal):
    """Nothing to occlude: t_lm = A_l Y_lm(n) with A = pi, 2pi/3, pi/4, 0,
    -pi/24 (clamped-cosine zonal harmonics, Ramamoorthi & Hanrahan 2001)."""
    n = np.asarray(normal, dtype=np.float64)
    n /= np.linalg.norm(n)
    sc = _scene([[0.3, 0.2, 0.1]], [0.01], [0.5], normals=[n])
    r = oracle_mod.direct_transfer(sc, 65536, 5, seed=3, sources=[0])
    assert np.abs(r["t"][0] - _lobe_expect(oracle_mod, n, 5)).max() < 1e-3


def _occluder_closed_form(h, sig, o):
    from scipy.integrate import quad
    a = h * h / (2 * sig * sig)
    t00 = math.sqrt(math.pi) / 2 * (1 - o * (1 - math.exp(-min(a, 4.5))) / a)
    cc = math.sqrt(1 - min(1.0, 9 * sig * sig / (h * h)))
    integ, _ = quad(lambda c: math.exp(-a * (1 - c * c)) * c * c, cc, 1.0, epsabs=1e-14, epsrel=1e-12)
    t10 = math.sqrt(3 / (4 * math.pi)) * (2 * math.pi / 3 - 2 * math.pi * o * integ)
    return t00, t10


def test_single_occluder_golden_values():
    vals, _ = _golden("single_occluder.txt")
    t00, t10 = _occluder_closed_form(vals["h"], vals["sigma"], vals["opacity"])
    assert abs(t00 - vals["t00"]) < 1e-7 and abs(t10 - vals["t10"]) < 1e-7


@pytest.mark.parametrize("h,sig,o", [(0.1, 0.05, 0.8), (0.3, 0.05, 0.5), (0.05, 0.1, 0.95)])
def test_single_occluder_closed_form(oracle_mod, h, sig, o):
    sc = _scene([[0, 0, 0], [0, 0, h]], [0.01, sig], [0.5, o])
    r = oracle_mod.direct_transfer(sc, 65536, 3, sources=[0])
    t00, t10 = _occluder_closed_form(h, sig, o)
    t = r["t"][0]
    assert abs(t[0] - t00) < 1e-4
    assert abs(t[2] - t10) < 1e-4
    assert np.abs(t[[1, 3, 4, 5, 7, 8]]).max() < 2e-3  # m != 0 vanish (up to quadrature error)


def test_visibility_brute_force_tiny(oracle_mod):
    """Per-ray visibility on a tiny anisotropic scene against an independent
    route: covariance from SciPy rotations (scalar-last quaternions), its
    numerical inverse, and a dense + golden-section search for the peak."""
    from scipy.optimize import minimize_scalar
    from scipy.spatial.transform import Rotation
    sc = scenegen.random_cloud(6, 11)
    sc["means"] *= 0.1                      # crowd them so rays hit
    sc["log_scales"] += math.log(2.0)
    r = oracle_mod.direct_transfer(sc, 64, 2, sources=np.arange(6), want_vis=True)
    dirs = oracle_mod.directions(64, 0)
    n = 6
    sig_inv = []
    for j in range(n):
        q = sc["quats"][j]
        Rm = Rotation.from_quat([q[1], q[2], q[3], q[0]]).as_matrix()
        Sg = Rm @ np.diag(np.exp(2 * sc["log_scales"][j])) @ Rm.T
        sig_inv.append(np.linalg.inv(Sg))
    hits = 0
    for i in range(n):
        for s in range(64):
            w = dirs[s]
            c = float(sc["normals"][i] @ w)
            if c <= 0:
                assert r["vis"][i, s] == -1.0
                continue
            V = 1.0
            for j in range(n):
                if j == i:
                    continue
                rel = sc["means"][i] - sc["means"][j]
                f = lambda t: float((rel + t * w) @ sig_inv[j] @ (rel + t * w))
                ts = np.linspace(-3, 3, 6001)
                E = rel[None, :] + ts[:, None] * w[None, :]
                t0 = ts[np.argmin(np.einsum("ta,ab,tb->t", E, sig_inv[j], E))]
                res = minimize_scalar(f, bracket=(t0 - 1e-3, t0, t0 + 1e-3), tol=1e-12)
                tstar, d2 = res.x, res.fun
                if tstar > 0 and d2 <= 9.0:
                    V *= 1 - min(sc["opacity"][j] * math.exp(-0.5 * d2), 0.99)
                    hits += 1
            V = 0.0 if V < 1e-4 else V
            assert abs(r["vis"][i, s] - V) < 1e-7
    assert hits > 20


def test_visibility_invariants(oracle_mod):
    sc = scenegen.random_cloud(150, 5)
    base = oracle_mod.direct_transfer(sc, 64, 3, sources=np.arange(0, 150, 7), want_vis=True)
    v = base["vis"]
    traced = v != -1.0
    assert ((v[traced] >= 0) & (v[traced] <= 1)).all()
    # opacity -> 0 makes everything visible: the empty-scene sum
    clear = dict(sc, opacity=np.full(150, 1e-300))
    rc = oracle_mod.direct_transfer(clear, 64, 3, sources=np.arange(0, 150, 7), want_vis=True)
    assert (rc["vis"][traced] == 1.0).all()
    # adding Gaussians never raises visibility
    more = {k: np.concatenate([sc[k], scenegen.random_cloud(60, 6)[k]]) for k in sc}
    rm = oracle_mod.direct_transfer(more, 64, 3, sources=np.arange(0, 150, 7), want_vis=True)
    assert (rm["vis"][traced] <= v[traced] + 1e-15).all()
    # scale by lambda (means and scales) and translation leave t unchanged
    lam = 3.7
    scaled = dict(sc, means=sc["means"] * lam, log_scales=sc["log_scales"] + math.log(lam))
    rs = oracle_mod.direct_transfer(scaled, 64, 3, sources=np.arange(0, 150, 7))
    assert np.abs(rs["t"] - base["t"]).max() < 1e-12
    moved = dict(sc, means=sc["means"] + np.array([5.0, -2.0, 1.0]))
    rt = oracle_mod.direct_transfer(moved, 64, 3, sources=np.arange(0, 150, 7))
    assert np.abs(rt["t"] - base["t"]).max() < 1e-9
    # transfer is the projection of the traced V c+
    d, Y = oracle_mod.tables(64, 0, 3)
    c = np.clip(sc["normals"][np.arange(0, 150, 7)] @ d.T, 0, None)
    proj = (4 * math.pi / 64) * (np.where(traced, v, 0) * c) @ Y
    assert np.abs(proj - base["t"]).max() < 1e-13


def test_allowance_is_rare_and_nonnegative(oracle_mod):
    sc = scenegen.random_cloud(300, 9)
    r = oracle_mod.direct_transfer(sc, 64, 3, want_allow=True)
    assert (r["allow"] >= 0).all()
    assert (r["allow"].max(1) > 0).mean() < 0.2


# --------------------------------------------------------------------------
# bounce (Eq. 20-22, 30-33 with the depth-ordered alpha blend)
# --------------------------------------------------------------------------

def test_allowance_covers_threshold_perturbations(oracle_mod):
    """The deviation bound must cover every other resolution of the
    near-threshold predicates: moving the 3-sigma cut and T_eps inside wide
    margins changes direct and bounce transfers by no more than it.  A faint,
    crowded cloud gives hundreds of hits per ray, many of them ambiguous."""
    sc = scenegen.random_cloud(700, 31)
    sc["means"] *= 0.3
    sc["opacity"] *= 0.05
    margins = (1e-6, 0.02, 3e-6, 0.1, 1e-5)
    src = np.arange(0, 700, 7)
    base = oracle_mod.full_transfer(sc, 32, 3, 1, sources=src, want_allow=True, margins=margins)
    moved = 0.0
    for cut in (dict(sigma_cut=3.0 * (1 + 1e-3)), dict(sigma_cut=3.0 * (1 - 1e-3)),
                dict(T_eps=1e-4 * 1.05), dict(T_eps=1e-4 * 0.95)):
        var = oracle_mod.full_transfer(sc, 32, 3, 1, sources=src, cut=cut, margins=margins)
        diff = np.abs(var["t"] - base["t"])
        assert (diff <= base["allow"] + 1e-12).all(), (cut, (diff - base["allow"]).max())
        moved = max(moved, diff.max())
    assert moved > 1e-6
    # the bound stays informative: well below the transfer's own size
    assert np.median(base["allow"]) < 1e-2 * np.abs(base["t"]).max()


def test_allowance_covers_t_min_and_hemisphere_perturbations(oracle_mod):
    """The same for the two other predicates: moving t_min (the peak-depth
    cut, where same-surface neighbours of a source sit) and the hemisphere
    threshold of c = n . w inside wide margins changes every ray's V by no more
    than its [vis_lo, vis_hi] range, a ray's traced status only where its
    hemisphere test is ambiguous, and the direct and bounce transfers by no
    more than the deviation bound."""
    sc = scenegen.surface_scene(900, 33)
    margins = (2e-3, 5e-5, 0.5, 1e-4, 1e-5)   # t margin >= 0.5 s_min >= 2.5e-4
    src = np.arange(0, 900, 9)
    S = 64
    base = oracle_mod.direct_transfer(sc, S, 3, sources=src, want_vis=True, want_allow=True,
                                      want_vis_bounds=True, margins=margins)
    full = oracle_mod.full_transfer(sc, S, 3, 1, sources=src, want_allow=True, margins=margins)
    dirs = oracle_mod.directions(S)
    amb_c = np.abs(sc["normals"][src] @ dirs.T) <= margins[0]
    moved_t = moved_c = 0
    for cut in (dict(t_min=1e-4), dict(t_min=-1e-4), dict(c_min=1e-3), dict(c_min=-1e-3)):
        var = oracle_mod.direct_transfer(sc, S, 3, sources=src, cut=cut, want_vis=True)
        v0, v1 = base["vis"], var["vis"]
        flip = (v0 == -1) != (v1 == -1)
        assert not (flip & ~amb_c).any(), cut
        both = (v0 != -1) & (v1 != -1)
        assert (v1[both] >= base["vis_lo"][both] - 1e-12).all() and (v1[both] <= base["vis_hi"][both] + 1e-12).all()
        diff = np.abs(var["t"] - base["t"])
        assert (diff <= base["allow"] + 1e-12).all(), (cut, (diff - base["allow"]).max())
        fv = oracle_mod.full_transfer(sc, S, 3, 1, sources=src, cut=cut, margins=margins)
        fdiff = np.abs(fv["t"] - full["t"])
        assert (fdiff <= full["allow"] + 1e-12).all(), (cut, (fdiff - full["allow"]).max())
        if "t_min" in cut:
            moved_t += int((np.abs(v1[both] - v0[both]) > 1e-12).sum())
        else:
            moved_c += int(flip.sum())
    # the perturbations reach real rays: same-surface neighbours whose peak
    # lies within 1e-4 of the origin, and rays within 1e-3 of the horizon
    assert moved_t > 0 and moved_c > 0, (moved_t, moved_c)


def test_bounce_partition_of_unity(oracle_mod):
    """With t_dir = e_0 for every hit and rho = pi, the bounce term of a ray
    is c (sum_j alpha_j T_j) = c (1 - T_end) (telescoping)."""
    sc = scenegen.random_cloud(120, 21)
    sc["albedo"] = np.full((120, 3), math.pi)
    cut = dict(T_eps=0.0)
    src = np.arange(0, 120, 5)
    d = oracle_mod.direct_transfer(sc, 64, 1, cut=cut, sources=src, want_vis=True)
    rows = np.zeros((120, 1))
    rows[:, 0] = 1.0
    b = oracle_mod.bounce_transfer(sc, 64, 1, rows, np.arange(120), cut=cut, sources=src)
    dirs = oracle_mod.directions(64, 0)
    c = np.clip(sc["normals"][src] @ dirs.T, 0, None)
    vis = np.where(d["vis"] == -1, 1.0, d["vis"])
    expect = (4 * math.pi / 64) * (c * (1 - vis)).sum(1)
    for ch in range(3):
        assert np.abs(b["t"][:, ch, 0] - expect).max() < 1e-13


def test_bounce_linear_in_albedo(oracle_mod):
    sc = scenegen.random_cloud(100, 22)
    src = np.arange(0, 100, 9)
    need = oracle_mod.hit_set(sc, 64, sources=src)
    dj = oracle_mod.direct_transfer(sc, 64, 3, sources=need)
    b1 = oracle_mod.bounce_transfer(sc, 64, 3, dj["t"], need, sources=src)["t"]
    sc2 = dict(sc, albedo=sc["albedo"] * 0.5)
    b2 = oracle_mod.bounce_transfer(sc2, 64, 3, dj["t"], need, sources=src)["t"]
    sc0 = dict(sc, albedo=np.zeros_like(sc["albedo"]))
    b0 = oracle_mod.bounce_transfer(sc0, 64, 3, dj["t"], need, sources=src)["t"]
    assert np.abs(b2 - 0.5 * b1).max() < 1e-14 and np.abs(b0).max() == 0.0
    assert np.abs(b1).max() > 1e-3


def test_bounce_facing_pair_closed_form(oracle_mod):
    """Continuum limit for one isotropic occluder above the source:
    t_ind = rho o (1 - exp(-min(a, 9/2))) / a * t_dir[j] per channel."""
    h, sig, o = 0.1, 0.05, 0.8
    sc = _scene([[0, 0, 0], [0, 0, h]], [0.01, sig], [0.5, o])
    sc["albedo"] = np.array([[0.5, 0.5, 0.5], [0.2, 0.5, 0.8]])
    rows = np.array([[1.0, 0.3, -0.2, 0.1]])
    b = oracle_mod.bounce_transfer(sc, 65536, 2, rows, [1], sources=[0])["t"][0]
    a = h * h / (2 * sig * sig)
    f = o * (1 - math.exp(-min(a, 4.5))) / a
    for ch in range(3):
        assert np.abs(b[ch] - sc["albedo"][1, ch] * f * rows[0]).max() < 2e-4


def test_bounce_depth_order(oracle_mod):
    """Two isotropic occluders stacked on the source normal: the nearer one
    weights alpha_1, the farther alpha_2 (1 - alpha_1) (Eq. 4 order)."""
    from scipy.integrate import quad
    h1, s1, o1 = 0.1, 0.05, 0.6
    h2, s2, o2 = 0.25, 0.08, 0.7
    sc = _scene([[0, 0, 0], [0, 0, h1], [0, 0, h2]], [0.01, s1, s2], [0.5, o1, o2])
    sc["albedo"] = np.full((3, 3), math.pi)
    rows = np.array([[1.0, 0.0, 0.0, 0.0], [0.0, 1.0, 0.0, 0.0]])
    b = oracle_mod.bounce_transfer(sc, 65536, 2, rows, [1, 2], sources=[0])["t"][0, 0]

    def alpha(c, h, s, o):
        d2 = h * h * (1 - c * c) / (s * s)
        return o * math.exp(-0.5 * d2) if d2 <= 9 else 0.0

    w1, _ = quad(lambda c: c * alpha(c, h1, s1, o1), 0, 1, limit=200, epsabs=1e-12)
    w2, _ = quad(lambda c: c * alpha(c, h2, s2, o2) * (1 - alpha(c, h1, s1, o1)), 0, 1, limit=200, epsabs=1e-12)
    assert abs(b[0] - 2 * math.pi * w1) < 3e-4
    assert abs(b[1] - 2 * math.pi * w2) < 3e-4


# --------------------------------------------------------------------------
# relight (Eq. 12-14)
# --------------------------------------------------------------------------

def test_relight_is_the_integral_of_light_times_transfer(oracle_mod):
    """sum_k l_k t_k = Int L(w) T(w) dw for band-limited L and T (Eq. 12-13),
    with the functions rebuilt from SciPy's harmonics and integrated by an
    exact product rule."""
    from scipy.special import sph_harm_y
    rng = np.random.default_rng(1)
    T = rng.standard_normal((4, 3, 9))
    L = rng.standard_normal((2, 3, 9))
    dirs, w = _product_rule(10, 20)
    theta = np.arccos(np.clip(dirs[:, 2], -1, 1))
    phi = np.arctan2(dirs[:, 1], dirs[:, 0])
    Ysc = np.zeros((dirs.shape[0], 9))
    for ell in range(3):
        for m in range(-ell, ell + 1):
            c = sph_harm_y(ell, abs(m), theta, phi)
            Ysc[:, ell * ell + ell + m] = c.real if m == 0 else math.sqrt(2) * (c.real if m > 0 else c.imag)
    C = oracle_mod.relight(T, L)
    assert C.shape == (4, 2, 3)
    for n in range(4):
        for b in range(2):
            for ch in range(3):
                integ = ((Ysc @ T[n, ch]) * (Ysc @ L[b, ch]) * w).sum()
                assert abs(C[n, b, ch] - integ) < 1e-12
    # a single-channel transfer is shared by the three colour channels
    Cm = oracle_mod.relight(T[:, :1], L)
    assert np.allclose(Cm[:, :, 2], T[:, 0] @ L[:, 2].T, atol=1e-14)
