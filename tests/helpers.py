"""Shared test helpers: FP32 rounding of generated scenes and parity checks."""
import numpy as np


def as_f32(arrays: dict) -> dict:
    """The scene the GPU sees (float32), promoted back to float64 so that the
    oracle gets exactly the same inputs."""
    return {k: np.asarray(v, dtype=np.float32).astype(np.float64) for k, v in arrays.items()}


def assert_transfer_parity(gpu, ref, allow, tol=1e-4, what="transfer"):
    """|gpu - ref| <= tol + allow elementwise (allow: the oracle's bound for
    rays whose cut-off predicates lie within FP32 rounding of a threshold)."""
    gpu = np.asarray(gpu, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    err = np.abs(gpu - ref)
    bound = tol + np.asarray(allow, dtype=np.float64)
    bad = err > bound
    if bad.any():
        idx = np.argwhere(bad)[:5]
        raise AssertionError(f"{what}: {bad.sum()} of {bad.size} coefficients off; worst excess "
                             f"{(err - bound).max():.3e}; first {idx.tolist()}; "
                             f"gpu {gpu[tuple(idx[0])]:.7f} ref {ref[tuple(idx[0])]:.7f} allow {allow[tuple(idx[0])]:.3e}")
    return float(err.max())
