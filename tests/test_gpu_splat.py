"""GPU parity of the splatting rasterizer (Sec. 3.1, Eq. 4: projected 2D
Gaussians blended front to back) against the FP64 oracle, per pixel within
the oracle's float32 allowance."""
import numpy as np
import pytest

import scenegen
from helpers import as_f32

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def prt():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2408_03538_amd as p
    return p


def _oracle_camera(cam):
    """The float32 camera the GPU sees, as the oracle's arguments."""
    return dict(view=[cam.view[i] for i in range(12)], fx=cam.fx, fy=cam.fy, cx=cam.cx, cy=cam.cy,
                width=cam.width, height=cam.height, near_z=cam.near_z,
                background=tuple(cam.background[i] for i in range(3)))


def _compare(prt, scene, colours, cam, pixels=None, max_instances=None):
    import torch
    from oracle import splat
    sc = prt.Scene.from_arrays(scene)
    col = torch.tensor(colours, dtype=torch.float32, device="cuda")
    img, T, inst = prt.splat_render(sc, col, cam, max_instances=max_instances, want_T=True)
    img, T = img.cpu().numpy().astype(np.float64), T.cpu().numpy().astype(np.float64)
    oc = _oracle_camera(cam)
    ref = splat.render(scene, np.asarray(colours, dtype=np.float32).astype(np.float64), oc["view"], oc["fx"], oc["fy"],
                       oc["cx"], oc["cy"], oc["width"], oc["height"], oc["near_z"], oc["background"], pixels=pixels,
                       want_allow=True)
    if pixels is not None:
        px, py = pixels
        img, T = img[py, px], T[py, px]
    ref_img, ref_T, allow_C, allow_T = ref
    dC = np.abs(img - ref_img).max(-1)
    dT = np.abs(T - ref_T)
    bad = (dC > allow_C + 1e-6) | (dT > allow_T + 1e-6)
    if bad.any():
        k = np.argmax(dC - allow_C)
        raise AssertionError(f"{bad.sum()} of {bad.size} pixels outside the allowance; worst |dC| "
                             f"{dC.ravel()[k]:.3e} vs allowance {allow_C.ravel()[k]:.3e}")
    return dict(dC=dC, dT=dT, allow_C=allow_C, T=ref_T, instances=inst)


def _small_scene(seed):
    """The million-splat recipe at a few thousand splats."""
    return as_f32(scenegen._concat([scenegen.surface_scene(3000, seed), scenegen.shells(4, 500, seed + 1)]))


@pytest.mark.parametrize("width,height", [(160, 96), (150, 90), (37, 20)])
def test_splat_parity_full_frame(prt, width, height):
    """Every pixel of a small frame (ragged tiles included) against the oracle."""
    scene = _small_scene(71)
    n = scene["means"].shape[0]
    colours = np.random.default_rng(72).uniform(0, 1, (n, 3))
    cam = prt.camera(prt.look_at((0.0, -3.6, 2.4), (0.0, 0.0, 0.6)), width, height, 50.0, 0.05, (0.1, 0.2, 0.3))
    r = _compare(prt, scene, colours, cam)
    covered = r["T"] < 0.5
    assert covered.mean() > 0.2                          # much of the frame is covered
    assert np.median(r["allow_C"][covered]) < 2e-3       # and the allowance there is tight
    assert r["instances"] > 0
    print(f"{width}x{height}: covered {covered.mean():.2f}, |dC| max {r['dC'].max():.2e}, "
          f"median on covered {np.median(r['dC'][covered]):.2e}, allowance median {np.median(r['allow_C'][covered]):.2e}")


def test_splat_close_up_and_behind(prt):
    """A camera inside the scene: Gaussians behind it and across the near
    plane, large footprints, the Jacobian clamp at the frame's edges."""
    scene = _small_scene(73)
    n = scene["means"].shape[0]
    colours = np.random.default_rng(74).uniform(0, 1, (n, 3))
    cam = prt.camera(prt.look_at((0.3, -0.8, 0.6), (0.0, 0.5, 0.9)), 128, 80, 70.0, 0.02)
    r = _compare(prt, scene, colours, cam)
    covered = r["T"] < 0.5
    assert covered.mean() > 0.15
    print(f"close-up: covered {covered.mean():.2f}, |dC| max {r['dC'].max():.2e}, "
          f"median on covered {np.median(r['dC'][covered]):.2e}")


def test_splat_relit_colours_strided(prt):
    """Colours taken straight from a [n, B, 3] relight output (row stride 3B)
    give the same image as a contiguous copy."""
    import torch
    scene = _small_scene(75)
    n = scene["means"].shape[0]
    sc = prt.Scene.from_arrays(scene)
    out = torch.rand((n, 5, 3), device="cuda")
    cam = prt.camera(prt.look_at((0.0, -5.5, 3.0), (0.0, 0.0, 0.8)), 96, 64)
    a, _, _ = prt.splat_render(sc, out[:, 2], cam)
    b, _, _ = prt.splat_render(sc, out[:, 2].contiguous(), cam)
    assert torch.equal(a, b)


def test_splat_nothing_visible(prt):
    """Every Gaussian behind the camera: background everywhere, T = 1."""
    import torch
    scene = _small_scene(76)
    sc = prt.Scene.from_arrays(scene)
    cam = prt.camera(prt.look_at((0.0, -5.5, 3.0), (0.0, -9.0, 3.0)), 64, 48, background=(0.25, 0.5, 0.75))
    img, T, inst = prt.splat_render(sc, torch.ones((sc.n, 3), device="cuda"), cam, want_T=True, check=True)
    assert inst == 0
    assert torch.equal(T, torch.ones_like(T))
    assert torch.equal(img, torch.tensor([0.25, 0.5, 0.75], device="cuda").expand_as(img))


def test_splat_workspace_too_small(prt):
    import torch
    scene = _small_scene(77)
    sc = prt.Scene.from_arrays(scene)
    cam = prt.camera(prt.look_at((0.0, -5.5, 3.0), (0.0, 0.0, 0.8)), 96, 64)
    col = torch.ones((sc.n, 3), device="cuda")
    _, _, inst = prt.splat_render(sc, col, cam)
    with pytest.raises(prt.PrtgsError):
        prt.splat_render(sc, col, cam, max_instances=inst - 1)
    img, _, inst2 = prt.splat_render(sc, col, cam, max_instances=inst)
    assert inst2 == inst


def test_splat_nonfinite_gaussian_is_skipped(prt):
    """A NaN mean raises the non-finite flag; the rest renders as if that
    Gaussian were absent."""
    import torch
    scene = _small_scene(78)
    scene["means"][5] = np.nan
    n = scene["means"].shape[0]
    colours = np.random.default_rng(79).uniform(0, 1, (n, 3))
    cam = prt.camera(prt.look_at((0.0, -5.5, 3.0), (0.0, 0.0, 0.8)), 64, 48)
    sc = prt.Scene.from_arrays(scene)
    with pytest.raises(FloatingPointError):
        prt.splat_render(sc, torch.tensor(colours, dtype=torch.float32, device="cuda"), cam, check=True)
    _compare(prt, scene, colours, cam)


def test_splat_1080p_million_sampled(prt):
    """The million-splat scene at 1920 x 1080 with relit colours: sampled
    pixels (spread over the frame and over covered tiles) against the oracle."""
    import torch
    scene = as_f32(scenegen.million_scene(0))
    n = scene["means"].shape[0]
    colours = np.random.default_rng(80).uniform(0, 1, (n, 3)).astype(np.float32)
    cam = prt.camera(prt.look_at((0.0, -5.5, 3.0), (0.0, 0.0, 0.8)), 1920, 1080, 50.0, 0.05)
    rng = np.random.default_rng(81)
    px, py = rng.integers(400, 1560, 96), rng.integers(250, 960, 96)      # where the scene projects
    # plus pixels on tile borders and the frame's last row / column
    px = np.concatenate([px, [0, 15, 16, 1919, 960, 961, 1919]])
    py = np.concatenate([py, [0, 15, 16, 1079, 540, 539, 0]])
    r = _compare(prt, scene, colours, cam, pixels=(px, py))
    covered = r["T"] < 0.5
    assert covered.mean() > 0.1
    assert np.median(r["allow_C"][covered]) < 5e-3
    print(f"1080p: {r['instances']} instances, covered {covered.mean():.2f}, |dC| max {r['dC'].max():.2e}, "
          f"median on covered {np.median(r['dC'][covered]):.2e}")


def test_splat_general_intrinsics(prt):
    """fx != fy and an off-centre principal point (the Jacobian clamp then
    differs per side), with a rotated, translated camera."""
    scene = _small_scene(82)
    n = scene["means"].shape[0]
    colours = np.random.default_rng(83).uniform(0, 1, (n, 3))
    cam = prt.camera(prt.look_at((1.5, -3.0, 2.2), (-0.2, 0.3, 0.5), up=(0.1, 0.0, 1.0)), 112, 72, 55.0, 0.05,
                     (0.05, 0.0, 0.1))
    cam.fx, cam.fy, cam.cx, cam.cy = 95.0, 70.0, 40.0, 45.5
    r = _compare(prt, scene, colours, cam)
    assert (r["T"] < 0.5).mean() > 0.1


def test_splat_workspace_grows_when_defaulted(prt):
    """A few Gaussians that each cover the whole frame need more than 64 pairs
    per Gaussian: the default workspace grows to the reported count."""
    n = 12
    rng = np.random.default_rng(84)
    scene = as_f32(dict(means=np.column_stack([rng.uniform(-0.2, 0.2, (n, 2)), rng.uniform(1.5, 3.0, n)]),
                        quats=np.tile([1.0, 0.0, 0.0, 0.0], (n, 1)), log_scales=np.log(np.full((n, 3), 1.5)),
                        opacity=rng.uniform(0.05, 0.3, n), normals=np.tile([0.0, 0.0, -1.0], (n, 1)),
                        albedo=np.full((n, 3), 0.5)))
    colours = rng.uniform(0, 1, (n, 3))
    cam = prt.camera([1, 0, 0, 0, 0, 1, 0, 0, 0, 0, 1, 0], 256, 192, 60.0, 0.05)
    r = _compare(prt, scene, colours, cam)
    assert r["instances"] > 64 * n
