"""Shared test helpers: FP32 rounding of generated scenes, parity checks and
progress lines."""
import numpy as np

# pytest's capture fixture of the running test (set by tests/conftest.py), so
# that progress lines pass the output capture
_capture = None


def say(msg):
    """Print a progress line at once, also while pytest captures the test's
    output: a long full-size test would otherwise print nothing until it
    ends, and a harness that watches the output for silence would take it
    for hung."""
    if _capture is not None:
        with _capture.disabled():
            print(msg, flush=True)
    else:
        print(msg, flush=True)


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


# Relative FP32 error allowed on a ray's transmittance: 10x the largest error
# of the float32 model of the GPU's product of (1 - alpha) over its hits
# (tests/test_oracle_margins.py measured 3.6e-6).
VIS_REL_TOL = 4e-5


def assert_ray_vis(gpu, ref, cos, mar_c, what="visibility"):
    """Per-ray parity of the visibility.  gpu: [count, S] V from the GPU (-1 =
    not traced); ref: the oracle's direct_transfer with want_vis and
    want_vis_bounds; cos: [count, S] n . w in FP64; mar_c: the hemisphere
    margin.  A ray whose hemisphere test is unambiguous is traced by both or
    by neither; one within the margin may go either way.  Every ray the GPU
    traces has V within [vis_lo, vis_hi] (the range over the other
    resolutions of its near-threshold predicates; one value for most rays) up
    to FP32 rounding of the product.  Returns (rays traced by the GPU, rays
    with a range wider than the rounding tolerance)."""
    gpu = np.asarray(gpu, dtype=np.float64)
    lo, hi, vis = ref["vis_lo"], ref["vis_hi"], ref["vis"]
    amb_c = np.abs(cos) <= mar_c
    traced = gpu != -1.0
    assert not (traced & (vis == -1.0) & ~amb_c).any(), f"{what}: the GPU traced a ray below the horizon"
    assert not (~traced & (vis != -1.0) & ~amb_c).any(), f"{what}: the GPU skipped a ray above the horizon"
    assert (lo[traced] >= 0.0).all()
    tol = VIS_REL_TOL * hi + 1e-9
    out = traced & ~((gpu >= lo - tol) & (gpu <= hi + tol))
    if out.any():
        idx = np.argwhere(out)[:5]
        r, c = idx[0]
        raise AssertionError(f"{what}: {out.sum()} rays outside their range; first {idx.tolist()}: gpu {gpu[r, c]:.7f} "
                             f"range [{lo[r, c]:.7f}, {hi[r, c]:.7f}] oracle {vis[r, c]:.7f}")
    wide = traced & (hi - lo > tol)
    return int(traced.sum()), int(wide.sum())
