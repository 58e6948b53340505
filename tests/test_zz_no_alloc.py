"""The no-allocation direct transfer, called through the C ABI, against the
workspace entry point on the same inputs: two calls in a row (the second on
a smaller scene, so the static scratch holds the first call's contents), a
source range, and the visibilities.  Both run the same kernels in the same
work split, so the results must be identical bit for bit."""
import ctypes

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


def _both(prt, scene, S, bands, first=0, count=None):
    import torch
    from paper_2408_03538_amd import _lib
    lib = _lib.load()
    sc = prt.Scene.from_arrays(scene)
    n = sc.n
    count = n - first if count is None else count
    bvh = prt.build_bvh(sc, check=True)
    params = prt.TransferParams(num_dirs=S, sh_bands=bands)
    g = sc.c_struct()
    d = params.c_struct()
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    K = bands * bands
    # the workspace entry point
    ws_bytes = lib.prtgs_transfer_workspace_bytes(ctypes.byref(d), n)
    ws = torch.empty(ws_bytes, dtype=torch.uint8, device="cuda")
    t_ref = torch.full((n, 1, K), 7.0, dtype=torch.float32, device="cuda")
    v_ref = torch.full((n, S), 7.0, dtype=torch.float32, device="cuda")
    _lib.check(lib.prtgs_precompute_transfer(ctypes.byref(g), bvh.buffer.data_ptr(), ctypes.byref(d), first, count,
                                             t_ref.data_ptr(), v_ref.data_ptr(), ws.data_ptr(), ws_bytes, stream))
    # the no-allocation entry point (caller's flag word)
    t_na = torch.full((n, 1, K), 7.0, dtype=torch.float32, device="cuda")
    v_na = torch.full((n, S), 7.0, dtype=torch.float32, device="cuda")
    flags = torch.full((1,), 12345, dtype=torch.int32, device="cuda")
    _lib.check(lib.prtgs_precompute_transfer_noalloc(ctypes.byref(g), bvh.buffer.data_ptr(), ctypes.byref(d), first,
                                                     count, t_na.data_ptr(), v_na.data_ptr(), flags.data_ptr(),
                                                     stream))
    torch.cuda.synchronize()
    assert int(ws[:4].view(torch.int32).item()) == 0
    assert int(flags.item()) == 0
    return t_ref, v_ref, t_na, v_na


def test_noalloc_matches_workspace_entry_point(prt):
    import torch
    print("no-alloc: cloud 3000, S = 128, 16 coefficients", flush=True)
    big = as_f32(scenegen.random_cloud(3000, 71))
    t_ref, v_ref, t_na, v_na = _both(prt, big, 128, 4)
    assert torch.equal(t_ref, t_na) and torch.equal(v_ref, v_na)
    assert (t_na != 7.0).all()
    print("no-alloc: cloud 700, S = 64, 9 coefficients (second call, smaller)", flush=True)
    small = as_f32(scenegen.random_cloud(700, 72))
    t_ref, v_ref, t_na, v_na = _both(prt, small, 64, 3)
    assert torch.equal(t_ref, t_na) and torch.equal(v_ref, v_na)
    assert (t_na != 7.0).all()


def test_noalloc_source_range_and_surface(prt):
    """A leaf range of a surface scene (4 sources per wave, rays weighted in
    scratch sized by the range, not the scene)."""
    import torch
    print("no-alloc: surface 6000, leaf range [1000, 3500), S = 256", flush=True)
    scene = as_f32(scenegen.surface_scene(6000, 73))
    t_ref, v_ref, t_na, v_na = _both(prt, scene, 256, 4, first=1000, count=2500)
    assert torch.equal(t_ref, t_na) and torch.equal(v_ref, v_na)
    # rows outside the range are left alone by both
    assert int((t_na != 7.0).all(dim=2).sum().item()) == 2500


def test_noalloc_rejects_oversized_call(prt):
    """More rays than the static scratch holds: an error, nothing enqueued."""
    import torch
    from paper_2408_03538_amd import _lib
    lib = _lib.load()
    scene = as_f32(scenegen.random_cloud(40000, 74))
    sc = prt.Scene.from_arrays(scene)
    bvh = prt.build_bvh(sc)
    params = prt.TransferParams(num_dirs=512, sh_bands=4, sources_per_wave=8)
    d = params.c_struct()
    out = torch.full((sc.n, 1, 16), 7.0, dtype=torch.float32, device="cuda")
    st = lib.prtgs_precompute_transfer_noalloc(ctypes.byref(sc.c_struct()), bvh.buffer.data_ptr(), ctypes.byref(d), 0,
                                               sc.n, out.data_ptr(), None, None,
                                               ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert st == _lib.ERR_WORKSPACE_TOO_SMALL
    torch.cuda.synchronize()
    assert (out == 7.0).all()
    # the same scene in ranges that fit (ranges of whole 8-source groups, the
    # work split fixed): identical to one call with a workspace
    ref = prt.precompute_transfer(sc, bvh, params)
    per = 16000
    for first in range(0, sc.n, per):
        cnt = min(per, sc.n - first)
        _lib.check(lib.prtgs_precompute_transfer_noalloc(
            ctypes.byref(sc.c_struct()), bvh.buffer.data_ptr(), ctypes.byref(d), first, cnt, out.data_ptr(), None,
            None, ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)))
    torch.cuda.synchronize()
    assert torch.equal(out, ref)


def test_noalloc_python_binding(prt):
    """The binding of the same name (argument marshalling only): with out, vis
    and flags preallocated, then with out allocated for a leaf range, each
    equal to the workspace entry point; bounces != 0 is refused."""
    import torch
    print("no-alloc binding: surface 3000, S = 128", flush=True)
    scene = as_f32(scenegen.surface_scene(3000, 75))
    sc = prt.Scene.from_arrays(scene)
    bvh = prt.build_bvh(sc, check=True)
    params = prt.TransferParams(num_dirs=128, sh_bands=4)
    ref, vref = prt.precompute_transfer(sc, bvh, params, want_vis=True, check=True)
    out = torch.full((sc.n, 1, 16), 7.0, dtype=torch.float32, device="cuda")
    vis = torch.full((sc.n, 128), 7.0, dtype=torch.float32, device="cuda")
    flags = torch.full((1,), 12345, dtype=torch.int32, device="cuda")
    got = prt.precompute_transfer_noalloc(sc, bvh, params, out=out, vis=vis, flags=flags, check=True)
    assert got is out
    assert torch.equal(out, ref) and torch.equal(vis, vref)
    assert int(flags.item()) == 0
    ref2 = prt.precompute_transfer(sc, bvh, params, first=500, count=1000)
    got2 = prt.precompute_transfer_noalloc(sc, bvh, params, first=500, count=1000, check=True)
    assert torch.equal(got2, ref2)
    with pytest.raises(prt.PrtgsError):
        prt.precompute_transfer_noalloc(sc, bvh, prt.TransferParams(num_dirs=128, sh_bands=4, bounces=1))
