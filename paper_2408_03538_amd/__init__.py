"""PRTGS radiance-transfer precompute for 3D Gaussian splats on MI355X.

Hand-written HIP kernels for gfx950 behind a C ABI (``include/prtgs.h``,
``libprtgs.so``); this package is the thin Python binding.  Build the
library with ``python -m paper_2408_03538_amd.build``.
"""
from .api import (Bvh, Scene, TransferParams, Workspace, abi_version, build_bvh, camera, check_flags,
                  direction_table, glossy_transfer, glossy_view, index_matrix, look_at, pack, precompute_transfer,
                  precompute_transfer_noalloc, read_flags, record_arena_words, relight,
                  relight_backward, self_transfer, splat_render, transfer_backward, traversal_stats)
from ._lib import PrtgsError
from .autograd import PRTGSTransfer, transfer_and_relight

__all__ = ["Bvh", "Scene", "TransferParams", "Workspace", "abi_version", "build_bvh", "check_flags",
           "direction_table", "index_matrix", "pack", "precompute_transfer",
           "precompute_transfer_noalloc", "read_flags", "record_arena_words",
           "relight",
           "relight_backward", "self_transfer", "splat_render", "transfer_backward", "traversal_stats",
           "camera", "look_at", "glossy_transfer", "glossy_view", "PRTGSTransfer", "transfer_and_relight",
           "PrtgsError"]
