"""ctypes declarations of the C ABI in include/prtgs.h."""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libprtgs.so")

PRTGS_OK = 0
ABI_VERSION = 5   # PRTGS_ABI_VERSION of include/prtgs.h that these declarations follow
STATUS_NAMES = {0: "ok", 1: "invalid argument", 2: "workspace too small", 3: "unsupported", 4: "HIP error"}
ERR_WORKSPACE_TOO_SMALL = 2
DTYPES = {"f32": 0, "bf16": 1, "f16": 2}
FLAG_NONFINITE = 0x1
FLAG_STACK_OVERFLOW = 0x2
FLAG_BAD_TREE = 0x4
FLAG_BAD_INDEX = 0x8
FLAG_ROUND_CAP = 0x10
FLAG_RECORDS_DEFERRED = 0x20   # informational: part of a one-walk blend was redone with two walks
BOUNCE_HIT_LIST = 256     # PRTGS_BOUNCE_HIT_LIST
BLEND_PARTS_MAX = 64      # PRTGS_BLEND_PARTS_MAX
NOALLOC_SCRATCH_BYTES = 64 << 20   # PRTGS_NOALLOC_SCRATCH_MIB
BOUNCE_BLEND = 0
BOUNCE_INDEX = 1

c_size_t = ctypes.c_size_t
c_void_p = ctypes.c_void_p
c_int32 = ctypes.c_int32
c_int64 = ctypes.c_int64
c_uint64 = ctypes.c_uint64
c_float = ctypes.c_float


class Gaussians(ctypes.Structure):
    _fields_ = [("n", c_int32), ("means", c_void_p), ("quats", c_void_p), ("log_scales", c_void_p),
                ("opacity", c_void_p), ("normals", c_void_p), ("albedo", c_void_p)]


class TransferDesc(ctypes.Structure):
    _fields_ = [("num_dirs", c_int32), ("sh_bands", c_int32), ("seed", c_uint64), ("bounces", c_int32),
                ("sigma_cut", c_float), ("t_min", c_float), ("T_eps", c_float), ("alpha_min", c_float),
                ("alpha_max", c_float), ("bounce_mode", c_int32), ("t_same", c_float),
                ("sources_per_wave", c_int32), ("direction_parts", c_int32), ("bounce_records", ctypes.c_int64)]


class Camera(ctypes.Structure):
    _fields_ = [("view", c_float * 12), ("fx", c_float), ("fy", c_float), ("cx", c_float), ("cy", c_float),
                ("width", c_int32), ("height", c_int32), ("near_z", c_float), ("background", c_float * 3)]


class Grads(ctypes.Structure):
    _fields_ = [("d_means", c_void_p), ("d_quats", c_void_p), ("d_log_scales", c_void_p),
                ("d_opacity", c_void_p), ("d_normals", c_void_p)]


# name: (restype, argtypes)
SIGNATURES = {
    "prtgs_abi_version": (c_int32, []),
    "prtgs_last_error": (ctypes.c_char_p, []),
    "prtgs_status_string": (ctypes.c_char_p, [c_int32]),
    "prtgs_direction_table": (c_int32, [c_int32, c_uint64, c_int32, c_void_p, c_void_p, c_void_p, c_void_p,
                                        c_void_p]),
    "prtgs_bvh_bytes": (c_size_t, [c_int32]),
    "prtgs_build_workspace_bytes": (c_size_t, [c_int32]),
    "prtgs_build_bvh": (c_int32, [ctypes.POINTER(Gaussians), c_void_p, c_size_t, c_void_p, c_size_t, c_void_p]),
    "prtgs_bvh_leaf_order": (c_int32, [c_void_p, c_int32, c_void_p, c_void_p]),
    "prtgs_transfer_workspace_bytes": (c_size_t, [ctypes.POINTER(TransferDesc), c_int32]),
    "prtgs_precompute_transfer": (c_int32, [ctypes.POINTER(Gaussians), c_void_p, ctypes.POINTER(TransferDesc),
                                            c_int32, c_int32, c_void_p, c_void_p, c_void_p, c_size_t, c_void_p]),
    "prtgs_precompute_transfer_noalloc": (c_int32, [ctypes.POINTER(Gaussians), c_void_p, ctypes.POINTER(TransferDesc),
                                                    c_int32, c_int32, c_void_p, c_void_p, c_void_p, c_void_p]),
    "prtgs_index_matrix": (c_int32, [ctypes.POINTER(Gaussians), c_void_p, ctypes.POINTER(TransferDesc), c_void_p,
                                     c_void_p, c_size_t, c_void_p]),
    "prtgs_self_transfer": (c_int32, [c_int32, c_int32, c_int32, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p,
                                      c_int32, c_void_p, c_void_p, c_void_p]),
    "prtgs_glossy_workspace_bytes": (c_size_t, [ctypes.POINTER(TransferDesc)]),
    "prtgs_glossy_transfer": (c_int32, [ctypes.POINTER(Gaussians), c_void_p, c_void_p, ctypes.POINTER(TransferDesc),
                                        c_void_p, c_void_p, c_void_p, c_size_t, c_void_p]),
    "prtgs_glossy_view": (c_int32, [c_int32, c_int32, c_void_p, c_void_p, ctypes.POINTER(c_float), c_void_p,
                                    c_void_p]),
    "prtgs_splat_workspace_bytes": (c_size_t, [c_int32, c_int32, c_int32, ctypes.c_int64]),
    "prtgs_splat_render": (c_int32, [ctypes.POINTER(Gaussians), c_void_p, ctypes.c_int64, ctypes.POINTER(Camera),
                                     c_void_p, c_void_p, ctypes.c_int64, c_void_p, c_size_t,
                                     ctypes.POINTER(ctypes.c_int64), c_void_p]),
    "prtgs_traversal_stats": (c_int32, [ctypes.POINTER(Gaussians), c_void_p, ctypes.POINTER(TransferDesc), c_int32,
                                        c_int32, c_void_p, c_void_p, c_size_t, c_void_p]),
    "prtgs_pack": (c_int32, [c_int64, c_void_p, c_void_p, c_int32, c_void_p]),
    "prtgs_relight": (c_int32, [c_int32, c_int32, c_int32, c_void_p, c_int32, c_int32, c_void_p, c_void_p,
                                c_int32, c_void_p]),
    "prtgs_relight_backward_workspace_bytes": (c_size_t, [c_int32, c_int32, c_int32, c_int32]),
    "prtgs_relight_backward": (c_int32, [c_int32, c_int32, c_int32, c_void_p, c_int32, c_void_p, c_void_p,
                                         c_void_p, c_void_p, c_void_p, c_size_t, c_void_p]),
    "prtgs_transfer_backward_workspace_bytes": (c_size_t, [ctypes.POINTER(TransferDesc), c_int32]),
    "prtgs_transfer_backward": (c_int32, [ctypes.POINTER(Gaussians), c_void_p, ctypes.POINTER(TransferDesc),
                                          c_void_p, c_void_p, ctypes.POINTER(Grads), c_void_p, c_size_t, c_void_p]),
}

_handle = None


def load():
    """Loads the built library; raises if it has not been built."""
    global _handle
    if _handle is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2408_03538_amd.build`")
        lib = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        if lib.prtgs_abi_version() != ABI_VERSION:
            raise RuntimeError(f"{LIB_PATH} has ABI {lib.prtgs_abi_version()}, these bindings expect {ABI_VERSION}: "
                               "rebuild it with `python -m paper_2408_03538_amd.build`")
        _handle = lib
    return _handle


class PrtgsError(RuntimeError):
    def __init__(self, status, message):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


def check(status: int):
    if status != PRTGS_OK:
        msg = load().prtgs_last_error()
        raise PrtgsError(status, msg.decode() if msg else "")
