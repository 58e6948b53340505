"""The C ABI library: it loads, exports every declared symbol, and rejects bad
arguments on the host before touching the GPU."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "prtgs.h")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(prtgs_[a-z0-9_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    from paper_2408_03538_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        pytest.fail("libprtgs.so is not built (python -m paper_2408_03538_amd.build)")
    return _lib.load()


def test_every_declared_symbol_is_exported(lib):
    names = _declared()
    assert len(names) >= 15
    for name in names:
        assert hasattr(lib, name), name


def test_binding_covers_the_header():
    from paper_2408_03538_amd import _lib
    assert set(_declared()) == set(_lib.SIGNATURES)


def test_abi_version(lib):
    assert lib.prtgs_abi_version() == 5


def test_size_queries(lib):
    from paper_2408_03538_amd import _lib
    assert lib.prtgs_bvh_bytes(0) == 0
    small, big = lib.prtgs_bvh_bytes(1000), lib.prtgs_bvh_bytes(1_000_000)
    assert small >= 1000 * 64 + 999 * 64 and big > 100 * small
    assert lib.prtgs_build_workspace_bytes(1000) > 0
    d = _lib.TransferDesc(64, 3, 0, 0, 3.0, 0.0, 1e-4, 0.0, 0.99, 0, 1.0)
    assert lib.prtgs_transfer_workspace_bytes(ctypes.byref(d), 1000) > 64 * 4 * 12
    bad = _lib.TransferDesc(64, 9, 0, 0, 3.0, 0.0, 1e-4, 0.0, 0.99, 0, 1.0)
    assert lib.prtgs_transfer_workspace_bytes(ctypes.byref(bad), 1000) == 0
    assert lib.prtgs_relight_backward_workspace_bytes(100, 16, 3, 64) > 0


@pytest.mark.parametrize("desc,status", [
    ((64, 3, 0, 0, 3.0, 0.0, 1e-4, 0.0, 0.99, 0, 1.0), 1),     # NULL pointers in the scene
    ((0, 3, 0, 0, 3.0, 0.0, 1e-4, 0.0, 0.99, 0, 1.0), 1),      # no directions
    ((64, 5, 0, 0, 3.0, 0.0, 1e-4, 0.0, 0.99, 0, 1.0), 1),     # too many bands
    ((64, 3, 0, 2, 3.0, 0.0, 1e-4, 0.0, 0.99, 0, 1.0), 1),     # two bounces
    ((64, 3, 0, 0, 4.0, 0.0, 1e-4, 0.0, 0.99, 0, 1.0), 1),     # cut-off beyond the 3-sigma boxes
    ((64, 3, 0, 0, 3.0, 0.0, 1e-4, 0.0, 1.0, 0, 1.0), 1),      # alpha_max = 1
    ((64, 3, 0, 1, 3.0, 0.0, 1e-4, 0.0, 0.99, 2, 1.0), 1),     # unknown bounce mode
    ((64, 3, 0, 9, 3.0, 0.0, 1e-4, 0.0, 0.99, 1, 1.0), 1),     # more than 8 index bounces
    ((64, 3, 0, 2, 3.0, 0.0, 1e-4, 0.0, 0.99, 1, 0.0), 1),     # t_same = 0
    ((64, 3, 0, 0, 3.0, 0.0, 1e-4, 0.0, 0.99, 0, 1.0, 3, 0), 1),   # 3 sources per wave
    ((64, 3, 0, 0, 3.0, 0.0, 1e-4, 0.0, 0.99, 0, 1.0, 128, 0), 1), # 128 sources per wave
    ((64, 3, 0, 0, 3.0, 0.0, 1e-4, 0.0, 0.99, 0, 1.0, 16, 65), 1), # 65 direction parts
    ((64, 3, 0, 0, 3.0, 0.0, 1e-4, 0.0, 0.99, 0, 1.0, 16, -1), 1), # negative direction parts
])
def test_transfer_validation(lib, desc, status):
    from paper_2408_03538_amd import _lib
    g = _lib.Gaussians(10, None, None, None, None, None, None)
    d = _lib.TransferDesc(*desc)
    st = lib.prtgs_precompute_transfer(ctypes.byref(g), None, ctypes.byref(d), 0, 10, None, None, None, 0, None)
    assert st == status
    assert lib.prtgs_last_error()


def test_build_validation(lib):
    from paper_2408_03538_amd import _lib
    assert lib.prtgs_build_bvh(None, None, 0, None, 0, None) == 1
    g = _lib.Gaussians(0, 256, 256, 256, 256, 256, None)
    assert lib.prtgs_build_bvh(ctypes.byref(g), 256, 1 << 20, 256, 1 << 20, None) == 1
    g = _lib.Gaussians(100, 256, 256, 256, 256, 256, None)
    assert lib.prtgs_build_bvh(ctypes.byref(g), 256, 16, 256, 1 << 20, None) == 2   # BVH buffer too small
    assert lib.prtgs_build_bvh(ctypes.byref(g), 257, 1 << 20, 256, 1 << 20, None) == 1  # misaligned
    assert b"aligned" in lib.prtgs_last_error()


def test_relight_validation(lib):
    assert lib.prtgs_relight(10, 5, 1, 256, 0, 4, 256, 256, 0, None) == 1     # K = 5
    assert lib.prtgs_relight(10, 16, 2, 256, 0, 4, 256, 256, 0, None) == 1    # C = 2
    assert lib.prtgs_relight(10, 16, 3, 256, 0, 0, 256, 256, 0, None) == 1    # B = 0
    assert lib.prtgs_relight(10, 16, 3, 256, 0, 4, 256, 256, 1, None) == 1    # bf16 output
    assert lib.prtgs_relight(0, 16, 3, None, 0, 4, None, None, 0, None) == 0  # nothing to do
    assert lib.prtgs_pack(10, None, None, 1, None) == 1
    assert lib.prtgs_pack(10, 256, 256, 0, None) == 1                         # F32 is not a packed type


def test_backward_rejects_bounce(lib):
    from paper_2408_03538_amd import _lib
    g = _lib.Gaussians(10, 256, 256, 256, 256, 256, 256)
    d = _lib.TransferDesc(64, 3, 0, 1, 3.0, 0.0, 1e-4, 0.0, 0.99, 0, 1.0)
    gr = _lib.Grads(None, None, None, None, None)
    st = lib.prtgs_transfer_backward(ctypes.byref(g), 256, ctypes.byref(d), 256, None, ctypes.byref(gr), 256, 1 << 30,
                                     None)
    assert st == 3


def test_bounce_needs_whole_range(lib):
    from paper_2408_03538_amd import _lib
    g = _lib.Gaussians(10, 256, 256, 256, 256, 256, 256)
    d = _lib.TransferDesc(64, 3, 0, 1, 3.0, 0.0, 1e-4, 0.0, 0.99, 0, 1.0)
    st = lib.prtgs_precompute_transfer(ctypes.byref(g), 256, ctypes.byref(d), 2, 5, 256, None, 256, 1 << 30, None)
    assert st == 1


def align(x):
    return (x + 255) // 256 * 256


def test_index_mode_workspace(lib):
    """Both bounce modes hold the hit lists (1000 waves of 256 entries per
    lane); the blend adds its per-lane hit records, the index mode the index
    matrix and two bounce terms."""
    from paper_2408_03538_amd import _lib
    direct = _lib.TransferDesc(64, 3, 0, 0, 3.0, 0.0, 1e-4, 0.0, 0.99, 0, 1.0)
    blend = _lib.TransferDesc(64, 3, 0, 1, 3.0, 0.0, 1e-4, 0.0, 0.99, 0, 1.0)
    index = _lib.TransferDesc(64, 3, 0, 3, 3.0, 0.0, 1e-4, 0.0, 0.99, 1, 1.0)
    d = lib.prtgs_transfer_workspace_bytes(ctypes.byref(direct), 1000)
    b = lib.prtgs_transfer_workspace_bytes(ctypes.byref(blend), 1000)
    i = lib.prtgs_transfer_workspace_bytes(ctypes.byref(index), 1000)
    lists = 1000 * 256 * 64 * (8 + 4)
    # hit lists + records + part sums (1000 sources: one per wave, S = 64 in one part)
    assert b >= d + lists + 1000 * 256 * 64 * 8 + 1 * 1000 * 3 * 9 * 4
    assert i >= d + lists + 1000 * 64 * 4 + 2 * 1000 * 3 * 9 * 4   # hit lists + index matrix + two bounce terms
    assert i < d + lists + 1000 * 256 * 64 * 8                  # no hit records
    # past 4096 sources the two-walk blend's lists and records hold 4096 persistent waves
    # (4 per SIMD), the index mode's lists 5120 (5 per SIMD); the blend also
    # keeps bounce sums for each of its direction parts (8 sources per wave,
    # S = 64: 8 parts)
    n = 20000
    d = lib.prtgs_transfer_workspace_bytes(ctypes.byref(direct), n)
    b = lib.prtgs_transfer_workspace_bytes(ctypes.byref(blend), n)
    i = lib.prtgs_transfer_workspace_bytes(ctypes.byref(index), n)
    common = align(n * 16 * 4) + align(n * 64 * 4) + 256   # leaf-order transfer + albedo (16 floats), cut depths, counter
    assert b - d - common == align(4096 * 256 * 64 * 8) * 2 + align(4096 * 256 * 64 * 4) + align(8 * n * 3 * 9 * 4)
    assert i - d - common - align(n * 64 * 4) - 2 * align(n * 3 * 9 * 4) == \
        align(5120 * 256 * 64 * 8) + align(5120 * 256 * 64 * 4)


def test_blend_parts_workspace(lib):
    """The blend's bounce sums take 12 K bytes per source and direction part,
    for the parts the call keeps: 64 from 16 sources per wave at S = 512 by
    default, fewer when the caller asks for fewer; the index mode keeps none."""
    from paper_2408_03538_amd import _lib
    n, K = 40000, 9
    size = lambda *a: lib.prtgs_transfer_workspace_bytes(ctypes.byref(_lib.TransferDesc(*a)), n)
    blend = (512, 3, 0, 1, 3.0, 0.0, 1e-4, 0.0, 0.99, 0, 1.0)
    assert _lib.BLEND_PARTS_MAX == 64
    assert size(*blend, 0, 0) == size(*blend, 16, 64)                   # the default: G = 16, 64 parts
    for parts in (1, 8, 32):
        assert size(*blend, 16, 64) - size(*blend, 16, parts) == align(64 * n * 3 * K * 4) - align(parts * n * 3 * K * 4)
    # 4 sources per wave hold 32 batches of 16 directions: no more parts than that
    assert size(*blend, 4, 64) == size(*blend, 4, 32)
    index = (512, 3, 0, 1, 3.0, 0.0, 1e-4, 0.0, 0.99, 1, 1.0)
    assert size(*index, 16, 64) == size(*index, 16, 8)


def test_self_transfer_validation(lib):
    assert lib.prtgs_self_transfer(10, 64, 5, 256, 256, 256, 256, 256, 1, 512, None, None) == 1   # K = 5
    assert lib.prtgs_self_transfer(10, 64, 9, 256, 256, 256, 256, 256, 2, 512, None, None) == 1   # c_prev = 2
    assert lib.prtgs_self_transfer(10, 64, 9, 256, 256, 256, 256, 256, 1, 256, None, None) == 1   # aliasing
    assert lib.prtgs_self_transfer(10, 64, 9, None, 256, 256, 256, 256, 1, 512, None, None) == 1  # NULL
    assert lib.prtgs_self_transfer(0, 64, 9, None, None, None, None, None, 1, None, None, None) == 0


def _camera(**kw):
    from paper_2408_03538_amd import _lib
    c = _lib.Camera()
    for i, v in enumerate([1, 0, 0, 0, 0, 1, 0, 0, 0, 0, 1, 0]):
        c.view[i] = v
    c.fx = c.fy = 100.0
    c.cx, c.cy, c.width, c.height, c.near_z = 32.0, 24.0, 64, 48, 0.05
    for k, v in kw.items():
        setattr(c, k, v)
    return c


def _gaussians(n=10):
    from paper_2408_03538_amd import _lib
    g = _lib.Gaussians()
    g.n = n
    for name in ("means", "quats", "log_scales", "opacity", "normals"):
        setattr(g, name, 256)
    return g


@pytest.mark.parametrize("cam", [dict(width=0), dict(height=20000), dict(near_z=0.0), dict(fx=0.0),
                                 dict(cy=float("nan"))])
def test_splat_camera_validation(lib, cam):
    img = ctypes.c_void_p(256)
    assert lib.prtgs_splat_render(ctypes.byref(_gaussians()), 256, 3, ctypes.byref(_camera(**cam)), img, None,
                                  100, 256, 1 << 20, None, None) == 1


def test_splat_render_validation(lib):
    g, c = _gaussians(), _camera()
    nan_view = _camera()
    nan_view.view[5] = float("inf")
    call = lambda g=g, col=256, stride=3, cam=c, image=256, mi=100, ws=256: lib.prtgs_splat_render(
        ctypes.byref(g), col, stride, ctypes.byref(cam), image, None, mi, ws, 1 << 20, None, None)
    assert call(g=_gaussians(0)) == 1                 # no Gaussians
    assert call(cam=nan_view) == 1                    # non-finite view
    assert call(col=None) == 1
    assert call(image=None) == 1
    assert call(ws=None) == 1
    assert call(stride=2) == 1                        # rows shorter than RGB
    assert call(ws=512 + 8) == 1                      # workspace not 256-byte aligned
    assert call(mi=-1) == 1
    assert call(mi=1 << 32) == 1                      # pair index must fit 32 bits
    assert lib.prtgs_splat_workspace_bytes(0, 64, 48, 100) == 0
    assert lib.prtgs_splat_workspace_bytes(10, 0, 48, 100) == 0
    assert lib.prtgs_splat_workspace_bytes(10, 64, 48, 1 << 32) == 0


def test_bench_refuses_more_than_one_gpu():
    """bench.py runs on one GPU: --gpus 2 exits with a message before touching a device."""
    import subprocess
    import sys
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True, text=True,
                       timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_glossy_validation(lib):
    from paper_2408_03538_amd import _lib
    g = _gaussians()
    g.albedo = 256
    d = lambda S=64, bands=4: _lib.TransferDesc(S, bands, 0, 0, 3.0, 0.0, 1e-4, 0.0, 0.99, 0, 1.0)
    assert lib.prtgs_glossy_workspace_bytes(ctypes.byref(d())) > 64 * 4 * 19
    assert lib.prtgs_glossy_workspace_bytes(ctypes.byref(d(S=513))) == 0      # more than 512 directions
    assert lib.prtgs_glossy_workspace_bytes(ctypes.byref(d(bands=2))) == 0    # 3 or 4 bands only
    call = lambda g=g, desc=d(), rough=256, vis=256, out=256, ws=256: lib.prtgs_glossy_transfer(
        ctypes.byref(g), rough, 256, ctypes.byref(desc), vis, out, ws, 1 << 20, None)
    no_albedo = _gaussians()
    assert call(g=no_albedo) == 1
    assert call(desc=d(S=600)) == 1
    assert call(desc=d(bands=5)) == 1
    assert call(rough=None) == 1
    assert call(vis=None) == 1
    assert call(out=None) == 1
    assert call(ws=256 + 4) == 1                    # workspace not 256-byte aligned
    assert lib.prtgs_glossy_transfer(ctypes.byref(g), 256, 256, ctypes.byref(d()), 256, 256, 256, 16, None) == 2


def test_glossy_view_validation(lib):
    eye = (ctypes.c_float * 3)(0.0, 0.0, 5.0)
    bad = (ctypes.c_float * 3)(0.0, float("nan"), 5.0)
    assert lib.prtgs_glossy_view(10, 5, 256, 256, eye, 256, None) == 1          # K must be 9 or 16
    assert lib.prtgs_glossy_view(10, 16, 256, 256, bad, 256, None) == 1         # eye not finite
    assert lib.prtgs_glossy_view(10, 16, None, 256, eye, 256, None) == 1
    assert lib.prtgs_glossy_view(-1, 16, 256, 256, eye, 256, None) == 1
    assert lib.prtgs_glossy_view(0, 16, None, None, eye, None, None) == 0       # nothing to do


def test_noalloc_host_validation(lib):
    """The no-allocation transfer refuses, on the host and before any device
    work, a call whose rays exceed its static scratch, and a bounce."""
    from paper_2408_03538_amd import _lib
    g = _lib.Gaussians(100000, 256, 256, 256, 256, 256, 256)
    d = _lib.TransferDesc(512, 4, 0, 0, 3.0, 0.0, 1e-4, 0.0, 0.99, 0, 1.0)
    st = lib.prtgs_precompute_transfer_noalloc(ctypes.byref(g), 256, ctypes.byref(d), 0, 100000, 256, None, None, None)
    assert st == _lib.ERR_WORKSPACE_TOO_SMALL
    assert b"scratch" in lib.prtgs_last_error()
    b = _lib.TransferDesc(64, 3, 0, 1, 3.0, 0.0, 1e-4, 0.0, 0.99, 0, 1.0)
    assert lib.prtgs_precompute_transfer_noalloc(ctypes.byref(g), 256, ctypes.byref(b), 0, 10, 256, None, None,
                                                 None) == 3
    assert lib.prtgs_precompute_transfer_noalloc(ctypes.byref(g), 257, ctypes.byref(d), 0, 10, 256, None, None,
                                                 None) == 1     # misaligned BVH


def test_one_walk_workspace(lib):
    """bounce_records (blend, one bounce) adds the record arena (8 bytes a
    word), a 256-byte counter and, per work item (direction part x source
    group), an 8-byte chain head and a 4-byte deferral mark, and its hit lists
    hold the one walk's 7168 persistent waves (7 per SIMD) instead of the
    two-walk kernel's 4096; it is ignored in index mode and without a bounce,
    and a negative size is refused."""
    from paper_2408_03538_amd import _lib
    n, R = 20000, 1_000_000
    args = (64, 3, 0, 1, 3.0, 0.0, 1e-4, 0.0, 0.99, 0, 1.0, 16, 4)
    size = lambda *a: lib.prtgs_transfer_workspace_bytes(ctypes.byref(_lib.TransferDesc(*a)), n)
    two, one = size(*args, 0), size(*args, R)
    items = (n + 15) // 16 * 4
    lists = sum(align(7168 * 256 * 64 * b) - align(4096 * 256 * 64 * b) for b in (8, 4, 8))   # keys, alphas, records
    assert one - two == 256 + align(8 * items) + align(4 * items) + align(8 * R) + lists
    index = (64, 3, 0, 3, 3.0, 0.0, 1e-4, 0.0, 0.99, 1, 1.0, 16, 4)
    assert size(*index, R) == size(*index, 0)
    direct = (64, 3, 0, 0, 3.0, 0.0, 1e-4, 0.0, 0.99, 0, 1.0, 16, 4)
    assert size(*direct, R) == size(*direct, 0)
    assert size(*args, -1) == 0
    # the binding passes the field through
    import paper_2408_03538_amd as prt
    assert prt.TransferParams(num_dirs=64, sh_bands=3, bounces=1, bounce_records=R).c_struct().bounce_records == R
