"""Pins of the splatting oracle against closed forms: footprint of a Gaussian
on the optical axis, front-to-back order, the transmittance stop, the 0.3
pixel^2 low-pass, and near-plane culling."""
import math

import numpy as np

from oracle import splat

VIEW = [1, 0, 0, 0, 0, 1, 0, 0, 0, 0, 1, 0]       # camera at the origin looking along +z
F, W, H = 100.0, 64, 48
CX, CY = 32.0, 24.0


def _scene(means, scales, opacity):
    n = len(means)
    return dict(means=np.asarray(means, dtype=np.float64),
                quats=np.tile([1.0, 0.0, 0.0, 0.0], (n, 1)),
                log_scales=np.log(np.asarray(scales, dtype=np.float64)),
                opacity=np.asarray(opacity, dtype=np.float64))


def _render(sc, col, pixels=None, bg=(0.0, 0.0, 0.0)):
    return splat.render(sc, col, VIEW, F, F, CX, CY, W, H, 0.1, bg, pixels=pixels)


def test_single_gaussian_on_axis():
    """An isotropic Gaussian at depth z on the axis: Sigma' = ((F s / z)^2 + 0.3) I
    around the principal point, so alpha = o exp(-r^2 / (2 v))."""
    z, s, o = 2.0, 0.05, 0.8
    sc = _scene([[0.0, 0.0, z]], [[s, s, s]], [o])
    v = (F * s / z) ** 2 + 0.3
    px = np.array([31, 32, 35, 28, 40])
    py = np.array([23, 24, 24, 20, 30])
    img, T = _render(sc, [[1.0, 0.5, 0.25]], (px, py))
    r2 = (px + 0.5 - CX) ** 2 + (py + 0.5 - CY) ** 2
    a = np.minimum(0.99, o * np.exp(-r2 / (2 * v)))
    a = np.where(a >= 1 / 255, a, 0.0)
    assert np.allclose(img[:, 0], a, rtol=1e-12, atol=1e-15)
    assert np.allclose(img[:, 2], 0.25 * a, rtol=1e-12, atol=1e-15)
    assert np.allclose(T, 1 - a, rtol=1e-12)


def test_front_to_back_order():
    """Two Gaussians on the axis: C = c_near a_near + c_far a_far (1 - a_near),
    whichever comes first in the list."""
    sc = _scene([[0.0, 0.0, 3.0], [0.0, 0.0, 2.0]], [[0.1] * 3, [0.1] * 3], [0.6, 0.7])
    pix = (np.array([31, 32]), np.array([23, 24]))
    img, _ = _render(sc, [[1.0, 0.0, 0.0], [0.0, 1.0, 0.0]], pix)
    uv = np.array([pix[0] + 0.5 - CX, pix[1] + 0.5 - CY])
    r2 = (uv ** 2).sum(0)
    a_far = 0.6 * np.exp(-r2 / (2 * ((F * 0.1 / 3) ** 2 + 0.3)))
    a_near = 0.7 * np.exp(-r2 / (2 * ((F * 0.1 / 2) ** 2 + 0.3)))
    assert np.allclose(img[:, 1], a_near, rtol=1e-12)
    assert np.allclose(img[:, 0], a_far * (1 - a_near), rtol=1e-12)


def test_transmittance_stop():
    """Four coincident layers of alpha 0.95 at the pixel under their centre:
    T = 1, 0.05, 0.0025, 1.25e-4; the fourth would take it below 1e-4."""
    sc = _scene([[0.0, 0.0, 2.0 + 0.1 * k] for k in range(4)], [[0.5] * 3] * 4, [0.95] * 4)
    # the pixel centre sits exactly on the projected centres
    img, T = splat.render(sc, np.ones((4, 3)), VIEW, F, F, 32.5, 24.5, W, H, 0.1, pixels=(np.array([32]), np.array([24])))
    assert math.isclose(img[0, 0], 0.95 * (1 + 0.05 + 0.0025), rel_tol=1e-12)
    assert math.isclose(T[0], 0.05 ** 3, rel_tol=1e-12)


def test_low_pass_of_a_tiny_gaussian():
    """A point-like Gaussian still covers the 0.3 pixel^2 low-pass."""
    sc = _scene([[0.0, 0.0, 2.0]], [[1e-6] * 3], [0.9])
    img, _ = splat.render(sc, np.ones((1, 3)), VIEW, F, F, 32.5, 24.5, W, H, 0.1,
                          pixels=(np.array([32, 33]), np.array([24, 24])))
    assert math.isclose(img[0, 0], 0.9, rel_tol=1e-9)
    assert math.isclose(img[1, 0], 0.9 * math.exp(-1.0 / (2 * 0.3)), rel_tol=1e-6)


def test_near_plane_and_background():
    sc = _scene([[0.0, 0.0, 0.05], [0.0, 0.0, -2.0]], [[0.1] * 3] * 2, [0.9, 0.9])
    img, T = _render(sc, np.ones((2, 3)), bg=(0.2, 0.3, 0.4))
    assert np.allclose(T, 1.0)
    assert np.allclose(img, np.array([0.2, 0.3, 0.4])[None, None, :])


def _random_quats(n, rng):
    q = rng.standard_normal((n, 4))
    return q / np.linalg.norm(q, axis=1, keepdims=True)


def test_projected_covariance_matches_sampled_points():
    """EWA's 2D covariance is the first-order covariance of the projected
    points: sample a small rotated anisotropic Gaussian off the axis, project
    every sample through the pinhole, and compare."""
    rng = np.random.default_rng(5)
    from scipy.spatial.transform import Rotation
    q = _random_quats(1, rng)
    mu = np.array([[0.4, -0.25, 3.0]])
    sc = dict(means=mu, quats=q, log_scales=np.log([[0.004, 0.0015, 0.0008]]), opacity=np.array([0.5]))
    view = np.array([[0.8, 0.0, -0.6, 0.1], [0.0, 1.0, 0.0, -0.2], [0.6, 0.0, 0.8, 0.5]])
    fx, fy, cx, cy = 300.0, 280.0, 160.0, 120.0
    uv, conic, z, vis = splat.project(sc, view.ravel(), fx, fy, cx, cy, 320, 240, 0.1)
    assert vis[0]
    R = Rotation.from_quat(np.concatenate([q[:, 1:], q[:, :1]], 1)).as_matrix()[0]
    pts = mu[0] + (rng.standard_normal((400000, 3)) * np.array([0.004, 0.0015, 0.0008])) @ R.T
    xc = pts @ view[:, :3].T + view[:, 3]
    p2 = np.stack([fx * xc[:, 0] / xc[:, 2] + cx, fy * xc[:, 1] / xc[:, 2] + cy], 1)
    emp = np.cov(p2.T)
    cov = np.linalg.inv(conic[0]) - 0.3 * np.eye(2)
    assert np.allclose(cov, emp, rtol=0.02, atol=0.02 * np.abs(emp).max())
    assert np.allclose(uv[0], p2.mean(0), atol=0.01)


def test_rigid_motion_invariance():
    """Moving the world and the camera by the same rigid motion leaves the
    image unchanged."""
    rng = np.random.default_rng(6)
    from scipy.spatial.transform import Rotation
    n = 30
    sc = dict(means=rng.uniform(-0.5, 0.5, (n, 3)) + [0, 0, 2.5], quats=_random_quats(n, rng),
              log_scales=np.log(rng.uniform(0.03, 0.12, (n, 3))), opacity=rng.uniform(0.2, 0.95, n))
    col = rng.uniform(0, 1, (n, 3))
    img0, T0 = splat.render(sc, col, VIEW, F, F, CX, CY, W, H, 0.1)
    G = Rotation.from_rotvec([0.3, -0.5, 0.2]).as_matrix()
    tr = np.array([1.0, -2.0, 0.5])
    qg = Rotation.from_matrix(G) * Rotation.from_quat(np.concatenate([sc["quats"][:, 1:], sc["quats"][:, :1]], 1))
    xyzw = qg.as_quat()
    sc2 = dict(sc, means=sc["means"] @ G.T + tr, quats=np.concatenate([xyzw[:, 3:], xyzw[:, :3]], 1))
    V2 = np.concatenate([G.T, (-G.T @ tr)[:, None]], 1)      # x_cam = G^T (x' - tr)
    img1, T1 = splat.render(sc2, col, V2.ravel(), F, F, CX, CY, W, H, 0.1)
    assert (T0 < 0.999).mean() > 0.2
    assert np.allclose(img0, img1, atol=1e-9)
    assert np.allclose(T0, T1, atol=1e-9)


def _look_at(eye, target, up=(0.0, 0.0, 1.0)):
    eye, target, up = (np.asarray(v, dtype=np.float64) for v in (eye, target, up))
    f = (target - eye) / np.linalg.norm(target - eye)
    r = np.cross(f, up)
    r /= np.linalg.norm(r)
    R = np.stack([r, np.cross(f, r), f])
    return np.concatenate([R, (-R @ eye)[:, None]], 1).ravel()


def _small_scene(seed=3):
    import scenegen
    return scenegen._concat([scenegen.surface_scene(600, seed), scenegen.shells(3, 150, seed + 1)])


def test_sampled_pixels_equal_full_image():
    """Rendering a few pixels (which first drops the Gaussians that cannot
    reach them) gives the same values as the full image there."""
    sc = _small_scene()
    col = np.random.default_rng(1).uniform(0, 1, (sc["means"].shape[0], 3))
    view = _look_at((0.0, -4.0, 2.5), (0.0, 0.0, 0.7))
    full = splat.render(sc, col, view, 60.0, 60.0, 40.0, 30.0, 80, 60, 0.05, (0.1, 0.2, 0.3), want_allow=True)
    rng = np.random.default_rng(2)
    px, py = rng.integers(0, 80, 50), rng.integers(0, 60, 50)
    part = splat.render(sc, col, view, 60.0, 60.0, 40.0, 30.0, 80, 60, 0.05, (0.1, 0.2, 0.3), pixels=(px, py),
                        want_allow=True)
    assert np.array_equal(part[0], full[0][py, px])
    assert np.array_equal(part[1], full[1][py, px])
    assert np.allclose(part[2], full[2][py, px], rtol=1e-12)
    assert (full[1] < 0.5).mean() > 0.1                 # the scene covers part of the frame


def test_allowance_covers_float32_sized_perturbations():
    """Nudging every input by about one float32 rounding moves each pixel by
    less than its allowance, and the allowance stays small on most pixels."""
    sc = _small_scene(4)
    n = sc["means"].shape[0]
    rng = np.random.default_rng(5)
    col = rng.uniform(0, 1, (n, 3))
    view = _look_at((0.3, -3.5, 2.0), (0.0, 0.0, 0.8))
    args = (view, 60.0, 60.0, 40.0, 30.0, 80, 60, 0.05, (0.0, 0.0, 0.0))
    img, T, aC, aT = splat.render(sc, col, *args, want_allow=True)
    worst = 0.0
    for trial in range(3):
        u = lambda shape: rng.uniform(-1, 1, shape) * 2 * splat.EPS32
        sp = dict(sc, means=sc["means"] * (1 + u((n, 3))), quats=sc["quats"] * (1 + u((n, 4))),
                  log_scales=sc["log_scales"] + u((n, 3)) * np.abs(sc["log_scales"]))
        img2, T2 = splat.render(sp, col, *args)
        assert (np.abs(img2 - img) <= aC[..., None] + 1e-12).all()
        assert (np.abs(T2 - T) <= aT + 1e-12).all()
        worst = max(worst, np.abs(img2 - img).max())
    assert np.median(aC) < 1e-4
    assert worst > 0.0
