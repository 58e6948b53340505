"""Python binding of the PRTGS HIP library: argument marshalling only.

Every function here takes and returns torch tensors on the GPU, allocates the
caller-side buffers the C ABI asks for (BVH storage, workspaces, outputs) and
passes raw device pointers plus the current HIP stream to the library.  No
step of the computation runs in Python or in torch.
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass, field

import torch

from . import _lib

F32 = torch.float32


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _alloc(nbytes: int, device) -> torch.Tensor:
    buf = torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=device)
    if buf.data_ptr() % 256:
        raise RuntimeError("device allocation is not 256-byte aligned")
    return buf


def _dev_f32(x, device, shape=None):
    t = torch.as_tensor(x, dtype=F32, device=device).contiguous()
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"expected shape {shape}, got {tuple(t.shape)}")
    return t


@dataclass
class Scene:
    """Gaussian splats on the GPU (float32, contiguous)."""
    means: torch.Tensor
    quats: torch.Tensor
    log_scales: torch.Tensor
    opacity: torch.Tensor
    normals: torch.Tensor
    albedo: torch.Tensor | None = None

    @property
    def n(self) -> int:
        return int(self.means.shape[0])

    @property
    def device(self):
        return self.means.device

    @staticmethod
    def from_arrays(arrays: dict, device="cuda") -> "Scene":
        n = len(arrays["means"])
        return Scene(
            means=_dev_f32(arrays["means"], device, (n, 3)),
            quats=_dev_f32(arrays["quats"], device, (n, 4)),
            log_scales=_dev_f32(arrays["log_scales"], device, (n, 3)),
            opacity=_dev_f32(arrays["opacity"], device, (n,)),
            normals=_dev_f32(arrays["normals"], device, (n, 3)),
            albedo=_dev_f32(arrays["albedo"], device, (n, 3)) if arrays.get("albedo") is not None else None,
        )

    def c_struct(self) -> _lib.Gaussians:
        for name in ("means", "quats", "log_scales", "opacity", "normals"):
            t = getattr(self, name)
            if t.dtype != F32 or not t.is_contiguous() or not t.is_cuda:
                raise ValueError(f"{name} must be a contiguous float32 GPU tensor")
        return _lib.Gaussians(self.n, self.means.data_ptr(), self.quats.data_ptr(), self.log_scales.data_ptr(),
                              self.opacity.data_ptr(), self.normals.data_ptr(),
                              self.albedo.data_ptr() if self.albedo is not None else None)


@dataclass
class TransferParams:
    """Transfer parameters (directions, SH bands, bounce, cutoffs)."""
    num_dirs: int = 64
    sh_bands: int = 3
    seed: int = 0
    bounces: int = 0
    sigma_cut: float = 3.0
    t_min: float = 0.0
    T_eps: float = 1e-4
    alpha_min: float = 0.0
    alpha_max: float = 0.99
    bounce_mode: str = "blend"     # "blend" (depth-ordered alpha blend, 1 bounce) or "index" (argmax, n bounces)
    t_same: float = 1.0            # index mode: same-surface filter (1 = off)
    sources_per_wave: int = 0      # work split (0 = the library's choice); changes only the last bits
    direction_parts: int = 0
    bounce_records: int = 0        # blend: record arena (8-byte words) for one walk per ray; 0 = two walks

    @property
    def K(self) -> int:
        return self.sh_bands * self.sh_bands

    @property
    def channels(self) -> int:
        return 3 if self.bounces else 1

    def c_struct(self) -> _lib.TransferDesc:
        mode = {"blend": _lib.BOUNCE_BLEND, "index": _lib.BOUNCE_INDEX}[self.bounce_mode]
        return _lib.TransferDesc(self.num_dirs, self.sh_bands, self.seed, self.bounces, self.sigma_cut, self.t_min,
                                 self.T_eps, self.alpha_min, self.alpha_max, mode, self.t_same,
                                 self.sources_per_wave, self.direction_parts, self.bounce_records)

    def cut(self) -> dict:
        return dict(sigma_cut=self.sigma_cut, t_min=self.t_min, T_eps=self.T_eps, alpha_min=self.alpha_min,
                    alpha_max=self.alpha_max)


@dataclass
class Bvh:
    buffer: torch.Tensor
    n: int
    flags: torch.Tensor = field(repr=False, default=None)   # build workspace (flag word at byte 0)

    def leaf_order(self) -> torch.Tensor:
        out = torch.empty(self.n, dtype=torch.int32, device=self.buffer.device)
        _lib.check(_lib.load().prtgs_bvh_leaf_order(_ptr(self.buffer), self.n, _ptr(out), _stream()))
        return out


def read_flags(ws: torch.Tensor) -> int:
    """Device flag word of a workspace (synchronises with the stream)."""
    return int(ws[:4].view(torch.int32).item())


def check_flags(ws: torch.Tensor, what: str = "kernel"):
    f = read_flags(ws)
    if f & _lib.FLAG_NONFINITE:
        raise FloatingPointError(f"{what}: a non-finite input reached the device")
    if f & _lib.FLAG_STACK_OVERFLOW:
        raise RuntimeError(f"{what}: BVH deeper than the traversal stack")
    if f & _lib.FLAG_BAD_TREE:
        raise RuntimeError(f"{what}: malformed BVH (buffer built for another scene?)")
    if f & _lib.FLAG_BAD_INDEX:
        raise IndexError(f"{what}: an index-matrix entry lies outside [-1, n)")
    if f & _lib.FLAG_ROUND_CAP:
        raise RuntimeError(f"{what}: a bounce ray needed more traversal rounds than the library allows")


# ----------------------------------------------------------------------------
# entry points (same names as the C ABI, without the prefix)
# ----------------------------------------------------------------------------

def abi_version() -> int:
    return int(_lib.load().prtgs_abi_version())


def direction_table(num_dirs: int, seed: int, sh_bands: int, device="cuda"):
    """FP64 and FP32 direction / SH-basis tables computed on the device."""
    K = sh_bands * sh_bands
    d64 = torch.empty((num_dirs, 3), dtype=torch.float64, device=device)
    y64 = torch.empty((num_dirs, K), dtype=torch.float64, device=device)
    d32 = torch.empty((num_dirs, 3), dtype=F32, device=device)
    y32 = torch.empty((num_dirs, K), dtype=F32, device=device)
    _lib.check(_lib.load().prtgs_direction_table(num_dirs, seed, sh_bands, _ptr(d64), _ptr(y64), _ptr(d32), _ptr(y32),
                                                 _stream()))
    return d64, y64, d32, y32


def build_bvh(scene: Scene, check: bool = False, workspace: "Workspace | None" = None, out: Bvh | None = None) -> Bvh:
    """LBVH over the scene (reusing ``out``'s buffer and ``workspace`` if given)."""
    lib = _lib.load()
    g = scene.c_struct()
    nbytes = lib.prtgs_bvh_bytes(scene.n)
    wbytes = lib.prtgs_build_workspace_bytes(scene.n)
    if out is not None and out.n == scene.n and out.buffer.numel() >= nbytes:
        buf = out.buffer
    else:
        buf = _alloc(nbytes, scene.device)
    ws = workspace.get(wbytes, scene.device) if workspace is not None else _alloc(wbytes, scene.device)
    _lib.check(lib.prtgs_build_bvh(ctypes.byref(g), _ptr(buf), buf.numel(), _ptr(ws), ws.numel(), _stream()))
    bvh = Bvh(buf, scene.n, ws)
    if check:
        check_flags(ws, "build_bvh")
    return bvh


class Workspace:
    """A reusable device workspace that grows on demand."""

    def __init__(self):
        self.buf = None

    def get(self, nbytes: int, device) -> torch.Tensor:
        if self.buf is None or self.buf.numel() < nbytes or self.buf.device != torch.device(device):
            self.buf = _alloc(nbytes, device)
        return self.buf


def precompute_transfer(scene: Scene, bvh: Bvh, params: TransferParams, first: int = 0, count: int | None = None,
                        out: torch.Tensor | None = None, want_vis: bool = False, workspace: Workspace | None = None,
                        check: bool = False):
    """Transfer vectors [n, C, K] (C = 3 with a bounce) of the sources in leaf
    positions [first, first + count); optionally the per-ray visibility."""
    lib = _lib.load()
    n = scene.n
    count = n - first if count is None else count
    g = scene.c_struct()
    d = params.c_struct()
    wbytes = lib.prtgs_transfer_workspace_bytes(ctypes.byref(d), n)
    if wbytes == 0:
        raise _lib.PrtgsError(1, "invalid transfer parameters")
    ws = (workspace or Workspace()).get(wbytes, scene.device)
    if out is None:
        out = torch.zeros((n, params.channels, params.K), dtype=F32, device=scene.device)
    vis = torch.full((n, params.num_dirs), float("nan"), dtype=F32, device=scene.device) if want_vis else None
    _lib.check(lib.prtgs_precompute_transfer(ctypes.byref(g), _ptr(bvh.buffer), ctypes.byref(d), first, count,
                                             _ptr(out), _ptr(vis), _ptr(ws), ws.numel(), _stream()))
    if check:
        check_flags(ws, "precompute_transfer")
    return (out, vis) if want_vis else out


def precompute_transfer_noalloc(scene: Scene, bvh: Bvh, params: TransferParams, first: int = 0,
                                count: int | None = None, out: torch.Tensor | None = None,
                                vis: torch.Tensor | None = None, flags: torch.Tensor | None = None,
                                check: bool = False):
    """The direct transfer (params.bounces == 0) through the library's
    no-allocation entry point: no workspace; its scratch is a static device
    array inside the library, shared by every call on the GPU (serialise
    overlapping calls).  Pass ``out`` [n, 1, K], ``vis`` [n, S] (optional) and
    ``flags`` (int32 [1], optional) preallocated for a call that allocates
    nothing; ``out`` and, with ``check``, ``flags`` are allocated here if
    missing.  Returns ``out``."""
    lib = _lib.load()
    n = scene.n
    count = n - first if count is None else count
    g = scene.c_struct()
    d = params.c_struct()
    if out is None:
        out = torch.zeros((n, 1, params.K), dtype=F32, device=scene.device)
    if out.dtype != F32 or tuple(out.shape) != (n, 1, params.K) or not out.is_contiguous():
        raise ValueError("out must be contiguous float32 [n, 1, K]")
    if vis is not None and (vis.dtype != F32 or tuple(vis.shape) != (n, params.num_dirs) or not vis.is_contiguous()):
        raise ValueError("vis must be contiguous float32 [n, num_dirs]")
    if flags is None and check:
        flags = torch.zeros(1, dtype=torch.int32, device=scene.device)
    if flags is not None and (flags.dtype != torch.int32 or flags.numel() < 1):
        raise ValueError("flags must be an int32 tensor of at least one element")
    _lib.check(lib.prtgs_precompute_transfer_noalloc(ctypes.byref(g), _ptr(bvh.buffer), ctypes.byref(d), first,
                                                     count, _ptr(out), _ptr(vis), _ptr(flags), _stream()))
    if check:
        check_flags(flags, "precompute_transfer_noalloc")
    return out


def index_matrix(scene: Scene, bvh: Bvh, params: TransferParams, workspace: Workspace | None = None,
                 check: bool = False) -> torch.Tensor:
    """The paper's index matrix [n, S] int32 (original indices, -1 = none)."""
    lib = _lib.load()
    n = scene.n
    g = scene.c_struct()
    d = params.c_struct()
    d.bounce_mode = _lib.BOUNCE_INDEX
    d.bounces = max(1, d.bounces)
    wbytes = lib.prtgs_transfer_workspace_bytes(ctypes.byref(d), n)
    if wbytes == 0:
        raise _lib.PrtgsError(1, "invalid transfer parameters")
    ws = (workspace or Workspace()).get(wbytes, scene.device)
    idx = torch.empty((n, params.num_dirs), dtype=torch.int32, device=scene.device)
    _lib.check(lib.prtgs_index_matrix(ctypes.byref(g), _ptr(bvh.buffer), ctypes.byref(d), _ptr(idx), _ptr(ws),
                                      ws.numel(), _stream()))
    if check:
        check_flags(ws, "index_matrix")
    return idx


def self_transfer(scene: Scene, params: TransferParams, index: torch.Tensor, t_prev: torch.Tensor,
                  out: torch.Tensor | None = None, check: bool = False) -> torch.Tensor:
    """One step of the recursive self-transfer: [n, 3, K] from t_prev [n, 1 or 3, K]
    and the index matrix [n, S] (Eq. 32-34)."""
    lib = _lib.load()
    n, S, K = scene.n, params.num_dirs, params.K
    if index.shape != (n, S) or index.dtype != torch.int32:
        raise ValueError("index must be int32 [n, num_dirs]")
    if t_prev.dim() != 3 or t_prev.shape[0] != n or t_prev.shape[1] not in (1, 3) or t_prev.shape[2] != K:
        raise ValueError("t_prev must be [n, 1 or 3, K]")
    if scene.albedo is None:
        raise ValueError("the self-transfer needs the albedo")
    dirs = direction_table(S, params.seed, params.sh_bands)[2].contiguous()
    tp = t_prev.to(F32).contiguous()
    index = index.contiguous()
    if out is None:
        out = torch.empty((n, 3, K), dtype=F32, device=scene.device)
    flags = torch.zeros(1, dtype=torch.int32, device=scene.device)
    _lib.check(lib.prtgs_self_transfer(n, S, K, _ptr(dirs), _ptr(scene.normals), _ptr(scene.albedo), _ptr(index),
                                       _ptr(tp), tp.shape[1], _ptr(out), _ptr(flags), _stream()))
    if check and int(flags.item()) & _lib.FLAG_BAD_INDEX:
        raise IndexError("self_transfer: an index-matrix entry lies outside [-1, n)")
    return out


def glossy_transfer(scene: Scene, params: TransferParams, vis: torch.Tensor, roughness: torch.Tensor,
                    metallic: torch.Tensor, out: torch.Tensor | None = None, workspace: Workspace | None = None,
                    check: bool = False) -> torch.Tensor:
    """Glossy transfer matrices [n, 3, K, K] (see prtgs_glossy_transfer) from
    the per-ray visibility of precompute_transfer(..., want_vis=True)."""
    lib = _lib.load()
    n, S, K = scene.n, params.num_dirs, params.K
    if scene.albedo is None:
        raise ValueError("glossy transfer needs the scene's albedo")
    if vis.shape != (n, S) or vis.dtype != F32 or not vis.is_contiguous():
        raise ValueError("vis must be contiguous float32 [n, S]")
    for name, t in (("roughness", roughness), ("metallic", metallic)):
        if t.shape != (n,) or t.dtype != F32 or not t.is_contiguous():
            raise ValueError(f"{name} must be contiguous float32 [n]")
    g = scene.c_struct()
    d = params.c_struct()
    wbytes = lib.prtgs_glossy_workspace_bytes(ctypes.byref(d))
    if wbytes == 0:
        raise _lib.PrtgsError(1, "invalid glossy parameters (num_dirs <= 512, sh_bands 3 or 4)")
    ws = (workspace or Workspace()).get(wbytes, scene.device)
    if out is None:
        out = torch.empty((n, 3, K, K), dtype=F32, device=scene.device)
    _lib.check(lib.prtgs_glossy_transfer(ctypes.byref(g), _ptr(roughness), _ptr(metallic), ctypes.byref(d), _ptr(vis),
                                         _ptr(out), _ptr(ws), ws.numel(), _stream()))
    if check:
        check_flags(ws, "glossy_transfer")
    return out


def glossy_view(matrices: torch.Tensor, means: torch.Tensor, eye, out: torch.Tensor | None = None) -> torch.Tensor:
    """The view step: transfer vectors [n, 3, K] of the matrices seen from
    `eye` (per splat, the direction from its centre to the eye)."""
    lib = _lib.load()
    n, K = matrices.shape[0], matrices.shape[-1]
    if matrices.shape != (n, 3, K, K) or matrices.dtype != F32 or not matrices.is_contiguous():
        raise ValueError("matrices must be contiguous float32 [n, 3, K, K]")
    if means.shape != (n, 3) or means.dtype != F32 or not means.is_contiguous():
        raise ValueError("means must be contiguous float32 [n, 3]")
    if out is None:
        out = torch.empty((n, 3, K), dtype=F32, device=matrices.device)
    e = (ctypes.c_float * 3)(*[float(v) for v in eye])
    _lib.check(lib.prtgs_glossy_view(n, K, _ptr(matrices), _ptr(means), e, _ptr(out), _stream()))
    return out


def look_at(eye, target, up=(0.0, 0.0, 1.0)) -> list:
    """World-to-camera [R | t] rows (12 floats) of a camera at `eye` looking
    at `target` (camera +z forward, +y down in the image)."""
    import numpy as np
    eye, target, up = (np.asarray(v, dtype=np.float64) for v in (eye, target, up))
    f = target - eye
    f /= np.linalg.norm(f)
    r = np.cross(f, up)
    r /= np.linalg.norm(r)
    d = np.cross(f, r)
    R = np.stack([r, d, f])
    t = -R @ eye
    return [float(x) for x in np.concatenate([R, t[:, None]], axis=1).ravel()]


def camera(view, width: int, height: int, fov_y_deg: float = 50.0, near_z: float = 0.05,
           background=(0.0, 0.0, 0.0)) -> "_lib.Camera":
    """A pinhole camera with the principal point at the image centre."""
    import math
    fy = 0.5 * height / math.tan(math.radians(fov_y_deg) / 2)
    c = _lib.Camera()
    for i, x in enumerate(view):
        c.view[i] = x
    c.fx, c.fy, c.cx, c.cy = fy, fy, 0.5 * width, 0.5 * height
    c.width, c.height, c.near_z = width, height, near_z
    for i in range(3):
        c.background[i] = background[i]
    return c


def splat_render(scene: Scene, colours: torch.Tensor, cam, max_instances: int | None = None,
                 workspace: Workspace | None = None, want_T: bool = False, check: bool = False):
    """Render per-splat colours ([n, 3], or a [n, B, 3] relight output with
    `colours[:, b]`) with Gaussian splatting.  Returns (image [H, W, 3],
    final transmittance [H, W] or None, number of (Gaussian, tile) pairs).
    With max_instances left at None the workspace starts at 64 pairs per
    Gaussian and grows to the reported count if a frame needs more."""
    lib = _lib.load()
    n = scene.n
    if colours.dim() != 2 or colours.shape[0] != n or colours.shape[1] != 3 or colours.dtype != F32:
        raise ValueError("colours must be float32 [n, 3] (rows may be strided)")
    if colours.stride(1) != 1:
        raise ValueError("colour rows must be contiguous")
    grow = max_instances is None
    if grow:
        max_instances = min(64 * n, 2**32 - 1)
    g = scene.c_struct()
    image = torch.empty((cam.height, cam.width, 3), dtype=F32, device=scene.device)
    T = torch.empty((cam.height, cam.width), dtype=F32, device=scene.device) if want_T else None
    workspace = workspace or Workspace()
    while True:
        wbytes = lib.prtgs_splat_workspace_bytes(n, cam.width, cam.height, max_instances)
        if wbytes == 0:
            raise _lib.PrtgsError(1, "invalid splat parameters")
        ws = workspace.get(wbytes, scene.device)
        inst = ctypes.c_int64(0)
        st = lib.prtgs_splat_render(ctypes.byref(g), _ptr(colours), colours.stride(0), ctypes.byref(cam), _ptr(image),
                                    _ptr(T), max_instances, _ptr(ws), ws.numel(), ctypes.byref(inst), _stream())
        if grow and st == _lib.ERR_WORKSPACE_TOO_SMALL and max_instances < inst.value <= 2**32 - 1:
            max_instances = int(inst.value)
            continue
        _lib.check(st)
        break
    if check:
        check_flags(ws, "splat_render")
    return image, T, int(inst.value)


def traversal_stats(scene: Scene, bvh: Bvh, params: TransferParams, first: int = 0, count: int | None = None,
                    workspace: Workspace | None = None) -> dict:
    """Single-ray work counts of the direct pass, or with ``params.bounces``
    (blend) of the bounce walk, or of the one walk with ``bounce_records``
    (see prtgs_traversal_stats)."""
    lib = _lib.load()
    n = scene.n
    count = n - first if count is None else count
    g = scene.c_struct()
    d = params.c_struct()
    d_ws = params.c_struct()   # the counted walk keeps no records: no arena
    d_ws.bounce_records = min(d_ws.bounce_records, 1)
    wbytes = lib.prtgs_transfer_workspace_bytes(ctypes.byref(d_ws), n)
    ws = (workspace or Workspace()).get(wbytes, scene.device)
    stats = torch.zeros(8, dtype=torch.int64, device=scene.device)
    _lib.check(lib.prtgs_traversal_stats(ctypes.byref(g), _ptr(bvh.buffer), ctypes.byref(d), first, count, _ptr(stats),
                                         _ptr(ws), ws.numel(), _stream()))
    v = stats.cpu().tolist()
    check_flags(ws, "traversal_stats")
    out = dict(traced_rays=v[0], box_tests=v[1], prim_tests=v[2], wave_node_visits=v[3], wave_prim_visits=v[4])
    if params.bounces:
        out.update(blended_hits=v[5], listed_hits=v[6], rounds=v[7])
    return out


def record_arena_words(scene: Scene, bvh: Bvh, params: TransferParams, spare: float = 0.05,
                       stats: dict | None = None) -> int:
    """Record arena (8-byte words) for the blended bounce in one walk per ray:
    one record per blended hit and a 17-word block header per (work item,
    direction batch, traversal round), counted by a counted walk (or taken
    from `stats`, the traversal_stats of that walk), plus `spare`.  Work
    whose records would not fit is redone by two walks, so a smaller arena is
    slower, never wrong."""
    probe = TransferParams(**{**params.__dict__, "bounces": 1, "bounce_mode": "blend", "bounce_records": 1})
    st = stats if stats is not None else traversal_stats(scene, bvh, probe)
    blocks = scene.n * params.num_dirs // 64 * st["rounds"] / max(1, st["traced_rays"])
    return int((1.0 + spare) * (st["blended_hits"] + 17 * blocks)) + (1 << 20)


def pack(x: torch.Tensor, dtype: str) -> torch.Tensor:
    """float32 -> bf16 / f16 storage with round-to-nearest-even."""
    tdt = {"bf16": torch.bfloat16, "f16": torch.float16}[dtype]
    x = x.contiguous()
    if x.dtype != F32:
        raise ValueError("pack expects float32")
    out = torch.empty(x.shape, dtype=tdt, device=x.device)
    _lib.check(_lib.load().prtgs_pack(x.numel(), _ptr(x), _ptr(out), _lib.DTYPES[dtype], _stream()))
    return out


_TORCH_TO_DT = {torch.float32: "f32", torch.bfloat16: "bf16", torch.float16: "f16"}


def relight(transfer: torch.Tensor, light: torch.Tensor, out_dtype: str = "f32", out: torch.Tensor | None = None):
    """colour [n, B, 3] = transfer [n, C, K] . light [B, 3, K] (Eq. 14)."""
    if transfer.dim() != 3 or light.dim() != 3 or light.shape[1] != 3:
        raise ValueError("transfer must be [n, C, K] and light [B, 3, K]")
    n, C, K = transfer.shape
    B = light.shape[0]
    if light.shape[2] != K:
        raise ValueError("transfer and light disagree on K")
    transfer = transfer.contiguous()
    light = light.to(F32).contiguous()
    odt = {"f32": torch.float32, "f16": torch.float16}[out_dtype]
    if out is None:
        out = torch.empty((n, B, 3), dtype=odt, device=transfer.device)
    _lib.check(_lib.load().prtgs_relight(n, K, C, _ptr(transfer), _lib.DTYPES[_TORCH_TO_DT[transfer.dtype]], B,
                                         _ptr(light), _ptr(out), _lib.DTYPES[out_dtype], _stream()))
    return out


def relight_backward(transfer: torch.Tensor, light: torch.Tensor, d_colour: torch.Tensor, want_dT=True, want_dL=True):
    lib = _lib.load()
    n, C, K = transfer.shape
    B = light.shape[0]
    transfer = transfer.to(F32).contiguous()
    light = light.to(F32).contiguous()
    d_colour = d_colour.to(F32).contiguous()
    dT = torch.empty_like(transfer) if want_dT else None
    dL = torch.empty_like(light) if want_dL else None
    wbytes = lib.prtgs_relight_backward_workspace_bytes(n, K, C, B)
    ws = _alloc(wbytes, transfer.device)
    _lib.check(lib.prtgs_relight_backward(n, K, C, _ptr(transfer), B, _ptr(light), _ptr(d_colour), _ptr(dT), _ptr(dL),
                                          _ptr(ws), wbytes, _stream()))
    return dT, dL


def transfer_backward(scene: Scene, bvh: Bvh, params: TransferParams, d_transfer: torch.Tensor,
                      grads: dict | None = None, workspace: Workspace | None = None, check: bool = False,
                      vis: torch.Tensor | None = None) -> dict:
    """dLoss/d(means, quats, log_scales, opacity, normals) from dLoss/dtransfer
    (direct transfer, [n, 1, K]); accumulated into ``grads`` if given.
    ``vis``: the forward's per-ray visibilities [n, S] (all sources), which
    spare the backward one traversal per ray."""
    lib = _lib.load()
    n = scene.n
    dev = scene.device
    if grads is None:
        grads = dict(means=torch.zeros((n, 3), dtype=F32, device=dev), quats=torch.zeros((n, 4), dtype=F32, device=dev),
                     log_scales=torch.zeros((n, 3), dtype=F32, device=dev),
                     opacity=torch.zeros((n,), dtype=F32, device=dev),
                     normals=torch.zeros((n, 3), dtype=F32, device=dev))
    g = scene.c_struct()
    d = params.c_struct()
    gr = _lib.Grads(*(grads[k].data_ptr() if grads.get(k) is not None else None
                      for k in ("means", "quats", "log_scales", "opacity", "normals")))
    wbytes = lib.prtgs_transfer_backward_workspace_bytes(ctypes.byref(d), n)
    if wbytes == 0:
        raise _lib.PrtgsError(1, "invalid transfer parameters")
    ws = (workspace or Workspace()).get(wbytes, dev)
    dt = d_transfer.to(F32).contiguous()
    if vis is not None and (vis.shape != (n, params.num_dirs) or vis.dtype != F32 or not vis.is_contiguous()):
        raise ValueError("vis must be a contiguous float32 [n, num_dirs] tensor")
    _lib.check(lib.prtgs_transfer_backward(ctypes.byref(g), _ptr(bvh.buffer), ctypes.byref(d), _ptr(dt), _ptr(vis),
                                           ctypes.byref(gr), _ptr(ws), ws.numel(), _stream()))
    if check:
        check_flags(ws, "transfer_backward")
    return grads
