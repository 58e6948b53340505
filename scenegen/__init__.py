"""Seeded synthetic inputs for the PRTGS transfer path.

This module is the only code shared by the CPU oracle and the HIP path.  It
draws scenes, lights, loss targets and parameter picks, and nothing else: it
computes no visibility, no spherical harmonics and no transfer.  Every draw
uses NumPy's PCG64 ``default_rng(seed)`` in a fixed order, so a scene is fully
determined by its generator name, size and seed.

A scene is a dict of float64 arrays (callers cast to float32 for the GPU):

* ``means``      [N,3]  Gaussian centres (the mean x of Eq. 1)
* ``quats``      [N,4]  rotation quaternions (w, x, y, z), unit length
* ``log_scales`` [N,3]  log of the per-axis scales (S of Eq. 2)
* ``opacity``    [N]    learned opacity sigma_i of the hit Gaussian
* ``normals``    [N,3]  per-splat unit normal n_i (Sec. 4.3)
* ``albedo``     [N,3]  diffuse albedo rho in [0, 1] (Sec. 4.2)

The paper evaluates on TensoIR Synthetic, DTU and Mip-NeRF 360, none of which
is available here; the surface scene (a sphere resting on a plane), the
ellipsoid shells and the random cloud stand in for them at the teaser's
million-splat scale.
"""
from __future__ import annotations

import math

import numpy as np

# Seeds of the standard workloads.
SEED_DIRS = 0
SEED_SCENE = 1000
SEED_LIGHT = 2000
SEED_TARGET = 3000
SEED_FD_PICK = 4000


# ----------------------------------------------------------------------------
# quaternion helpers used only to *place* splats (frames of the generators)
# ----------------------------------------------------------------------------

def _qmul(a, b):
    """Hamilton product of quaternion arrays [...,4] in (w,x,y,z) order."""
    aw, ax, ay, az = np.moveaxis(a, -1, 0)
    bw, bx, by, bz = np.moveaxis(b, -1, 0)
    return np.stack([
        aw * bw - ax * bx - ay * by - az * bz,
        aw * bx + ax * bw + ay * bz - az * by,
        aw * by - ax * bz + ay * bw + az * bx,
        aw * bz + ax * by - ay * bx + az * bw,
    ], axis=-1)


def _qrotate(q, v):
    """Rotate vectors v [...,3] by unit quaternions q [...,4] as q v q*."""
    vq = np.concatenate([np.zeros(v.shape[:-1] + (1,)), v], axis=-1)
    qc = q * np.array([1.0, -1.0, -1.0, -1.0])
    return _qmul(_qmul(q, vq), qc)[..., 1:]


def _frame_quat(normals, angle):
    """Quaternion whose rotated z axis is ``normals`` and whose rotated x axis
    makes ``angle`` with the shortest-arc image of the world x axis."""
    n = normals
    w = 1.0 + n[:, 2]
    arc = np.stack([w, -n[:, 1], n[:, 0], np.zeros_like(w)], axis=-1)
    flip = w < 1e-9  # n == -z: any half turn about a horizontal axis
    arc[flip] = np.array([0.0, 1.0, 0.0, 0.0])
    arc /= np.linalg.norm(arc, axis=-1, keepdims=True)
    spin = np.stack([np.cos(angle / 2), np.zeros_like(angle), np.zeros_like(angle),
                     np.sin(angle / 2)], axis=-1)
    q = _qmul(arc, spin)
    q[q[:, 0] < 0] *= -1.0
    return q / np.linalg.norm(q, axis=-1, keepdims=True)


def _unit_vectors(rng, n):
    v = rng.standard_normal((n, 3))
    return v / np.linalg.norm(v, axis=-1, keepdims=True)


# ----------------------------------------------------------------------------
# scenes
# ----------------------------------------------------------------------------

def random_cloud(n: int, seed: int) -> dict:
    """Gaussians scattered in the unit cube with random shapes.

    Means uniform in [0,1]^3, log-scales uniform in [ln 0.01, ln 0.05] per
    axis, uniformly random rotations, opacity uniform in [0.1, 0.99]; the
    normal is the splat's shortest principal axis.
    """
    rng = np.random.default_rng(seed)
    means = rng.uniform(0.0, 1.0, (n, 3))
    log_scales = rng.uniform(math.log(0.01), math.log(0.05), (n, 3))
    q = rng.standard_normal((n, 4))
    q /= np.linalg.norm(q, axis=-1, keepdims=True)
    opacity = rng.uniform(0.1, 0.99, n)
    albedo = rng.uniform(0.2, 0.8, (n, 3))
    axis = np.argmin(log_scales, axis=1)  # ties resolve to the lowest axis
    e = np.zeros((n, 3))
    e[np.arange(n), axis] = 1.0
    normals = _qrotate(q, e)
    normals /= np.linalg.norm(normals, axis=-1, keepdims=True)
    return dict(means=means, quats=q, log_scales=log_scales, opacity=opacity,
                normals=normals, albedo=albedo)


def _surface_splats(rng, points, normals, opacity_range=(0.5, 0.99)):
    """Flat splats tangent to a surface at ``points`` with outward ``normals``."""
    n = points.shape[0]
    points = points + rng.normal(0.0, 0.002, (n, 3))
    s1 = rng.uniform(0.005, 0.02, n)
    s2 = rng.uniform(0.005, 0.02, n)
    s3 = 0.1 * np.minimum(s1, s2)
    angle = rng.uniform(0.0, 2.0 * math.pi, n)
    q = _frame_quat(normals, angle)
    opacity = rng.uniform(opacity_range[0], opacity_range[1], n)
    albedo = rng.uniform(0.2, 0.8, (n, 3))
    return dict(means=points, quats=q, log_scales=np.log(np.stack([s1, s2, s3], -1)),
                opacity=opacity, normals=normals.copy(), albedo=albedo)


def _concat(parts):
    return {k: np.concatenate([p[k] for p in parts], axis=0) for k in parts[0]}


def surface_scene(n: int, seed: int) -> dict:
    """A unit sphere (centre (0,0,1)) resting on the 4x4 plane z = 0.

    Splats are split between the surfaces by area, jittered by N(0, 0.002^2),
    have tangent scales uniform in [0.005, 0.02] and a normal-axis scale of a
    tenth of the smaller tangent scale, opacity uniform in [0.5, 0.99] and
    albedo uniform in [0.2, 0.8].
    """
    rng = np.random.default_rng(seed)
    n_sphere = int(round(n * 4.0 * math.pi / (4.0 * math.pi + 16.0)))
    n_plane = n - n_sphere
    u = _unit_vectors(rng, n_sphere)
    sphere_pts = u + np.array([0.0, 0.0, 1.0])
    xy = rng.uniform(-2.0, 2.0, (n_plane, 2))
    plane_pts = np.concatenate([xy, np.zeros((n_plane, 1))], axis=-1)
    plane_n = np.tile(np.array([0.0, 0.0, 1.0]), (n_plane, 1))
    sphere = _surface_splats(rng, sphere_pts, u)
    plane = _surface_splats(rng, plane_pts, plane_n)
    return _concat([sphere, plane])


def shells(count: int, per_shell: int, seed: int) -> dict:
    """``count`` random ellipsoid shells of ``per_shell`` splats each.

    Centres uniform in [-1.8,1.8]^2 x [0.2,1.8], semi-axes uniform in
    [0.1, 0.5]^3, uniformly random orientation; splat rules as in
    :func:`surface_scene`.
    """
    rng = np.random.default_rng(seed)
    parts = []
    for _ in range(count):
        c = np.concatenate([rng.uniform(-1.8, 1.8, 2), rng.uniform(0.2, 1.8, 1)])
        a = rng.uniform(0.1, 0.5, 3)
        qo = rng.standard_normal(4)
        qo /= np.linalg.norm(qo)
        u = _unit_vectors(rng, per_shell)
        pts = c + _qrotate(np.broadcast_to(qo, (per_shell, 4)), a * u)
        nrm = _qrotate(np.broadcast_to(qo, (per_shell, 4)), u / a)
        nrm /= np.linalg.norm(nrm, axis=-1, keepdims=True)
        parts.append(_surface_splats(rng, pts, nrm))
    return _concat(parts)


def million_scene(seed: int, n_surface: int = 200_000, n_shells: int = 20,
                  per_shell: int = 40_000) -> dict:
    """Surface scene plus ellipsoid shells (1,000,000 splats by default)."""
    return _concat([surface_scene(n_surface, seed), shells(n_shells, per_shell, seed + 1)])


def subset(scene: dict, idx) -> dict:
    return {k: v[idx] for k, v in scene.items()}


def seeded_subset(scene: dict, count: int, seed: int) -> dict:
    """First ``count`` splats of a seeded permutation, as a scene of its own."""
    rng = np.random.default_rng(seed)
    perm = rng.permutation(scene["means"].shape[0])[:count]
    return subset(scene, np.sort(perm))


# ----------------------------------------------------------------------------
# lights, synthetic transfers, targets
# ----------------------------------------------------------------------------

def light_sh(num_envs: int, bands: int, seed: int, band_decay: bool = False) -> np.ndarray:
    """Light SH coefficients [B, 3, K], K = bands^2, drawn N(0,1) (optionally
    divided by l+1 for band l)."""
    rng = np.random.default_rng(seed)
    k = bands * bands
    light = rng.standard_normal((num_envs, 3, k))
    if band_decay:
        ell = np.floor(np.sqrt(np.arange(k))).astype(np.float64)
        light /= (ell + 1.0)
    return light


# Per-band gains of a clamped cosine lobe for bands 0..4; used only to give
# synthetic transfer vectors a realistic spectrum.
_LOBE_GAIN = [math.pi, 2.0 * math.pi / 3.0, math.pi / 4.0, 0.0, -math.pi / 24.0]


def synthetic_transfers(n: int, bands: int, channels: int, seed: int) -> np.ndarray:
    """Random transfer vectors [N, C, K] with the spectrum of lit, partly
    occluded diffuse splats.

    Band l of splat n is a random direction in R^(2l+1) of length
    |g_l| sqrt((2l+1)/(4 pi)) (the length an unoccluded clamped-cosine
    transfer has in that band), scaled by a visibility v ~ U[0.2, 1] and a
    per-channel factor ~ U[0.8, 1.2], plus N(0, 0.02^2) noise.
    """
    rng = np.random.default_rng(seed)
    k = bands * bands
    out = np.empty((n, channels, k))
    v = rng.uniform(0.2, 1.0, n)
    tint = rng.uniform(0.8, 1.2, (n, channels))
    for ell in range(bands):
        width = 2 * ell + 1
        g = _LOBE_GAIN[ell] if ell < len(_LOBE_GAIN) else 0.0
        d = rng.standard_normal((n, width))
        d /= np.linalg.norm(d, axis=-1, keepdims=True)
        mag = abs(g) * math.sqrt(width / (4.0 * math.pi))
        band = d * mag * np.sign(g if g != 0 else 1.0)
        out[:, :, ell * ell: ell * ell + width] = (v[:, None, None] * tint[:, :, None]) * band[:, None, :]
    out += rng.normal(0.0, 0.02, out.shape)
    return out


def materials(n: int, seed: int) -> tuple:
    """Glossy materials: roughness ~ U[0.1, 1], metallic ~ U[0, 1]."""
    rng = np.random.default_rng(seed)
    return rng.uniform(0.1, 1.0, n), rng.uniform(0.0, 1.0, n)


def colour_targets(n: int, num_envs: int, seed: int) -> np.ndarray:
    """Loss targets C_hat [N, B, 3] ~ N(0, 1)."""
    return np.random.default_rng(seed).standard_normal((n, num_envs, 3))


# ----------------------------------------------------------------------------
# the standard workloads
# ----------------------------------------------------------------------------

WORKLOADS = {
    # name: (description, builder)
    "cloud1k": "random cloud, N=1,000; S=64 directions, 3 SH bands (9 coeffs), direct",
    "surface100k": "sphere-on-plane surface scene, N=100,000; S=256, 4 bands (16 coeffs), direct",
    "million": "surface scene 200k + 20 shells x 40k = 1,000,000; S=512, 4 bands, RGB + one bounce",
    "relight3m": "3,000,000 synthetic RGB transfers, 16 coeffs, B=64 light environments",
    "grad200k": "surface scene N=200,000; S=256, 4 bands, direct; adjoint under an L2 loss",
    "glossy100k": "surface scene N=100,000 with roughness U[0.1,1], metallic U[0,1]; S=256, 4 bands, "
                  "glossy transfer matrices 3 x 16 x 16",
}


def workload(name: str) -> dict:
    """Inputs of a standard workload (scene + parameters), float64."""
    if name == "cloud1k":
        return dict(scene=random_cloud(1000, SEED_SCENE + 0), num_dirs=64, bands=3, bounces=0,
                    light=light_sh(1, 3, SEED_LIGHT + 0))
    if name == "surface100k":
        return dict(scene=surface_scene(100_000, SEED_SCENE + 1), num_dirs=256, bands=4, bounces=0,
                    light=light_sh(1, 4, SEED_LIGHT + 1))
    if name == "million":
        return dict(scene=million_scene(SEED_SCENE + 2), num_dirs=512, bands=4, bounces=1,
                    light=light_sh(1, 4, SEED_LIGHT + 2))
    if name == "relight3m":
        return dict(transfer=synthetic_transfers(3_000_000, 4, 3, SEED_SCENE + 3), bands=4,
                    light=light_sh(64, 4, SEED_LIGHT + 3, band_decay=True))
    if name == "grad200k":
        return dict(scene=surface_scene(200_000, SEED_SCENE + 4), num_dirs=256, bands=4, bounces=0,
                    light=light_sh(1, 4, SEED_LIGHT + 4))
    if name == "glossy100k":
        rough, metal = materials(100_000, SEED_SCENE + 5)
        return dict(scene=surface_scene(100_000, SEED_SCENE + 1), num_dirs=256, bands=4, bounces=0,
                    roughness=rough, metallic=metal, light=light_sh(1, 4, SEED_LIGHT + 1))
    raise KeyError(name)
