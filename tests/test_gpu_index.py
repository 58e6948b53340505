"""GPU parity of the paper's own bounce (index matrix + recursive
self-transfer, Sec. 4.4 Eq. 26 and Sec. 4.5 Eq. 32-35) against the oracle."""
import math

import numpy as np
import pytest

import scenegen
from helpers import as_f32, assert_transfer_parity

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def prt():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2408_03538_amd as p
    return p


def _scene(seed=21):
    """The million-splat recipe at a few thousand splats."""
    return as_f32(scenegen._concat([scenegen.surface_scene(2500, seed), scenegen.shells(4, 800, seed + 1)]))


@pytest.mark.parametrize("S,t_same", [(64, 1.0), (64, 0.8), (32, 0.95)])
def test_index_matrix_parity(prt, oracle_mod, S, t_same):
    """Every unambiguous ray picks the same Gaussian; ambiguous ones (ties,
    near-threshold decisions) are rare and pick a Gaussian or -1."""
    scene = _scene()
    n = scene["means"].shape[0]
    sc = prt.Scene.from_arrays(scene)
    bvh = prt.build_bvh(sc, check=True)
    params = prt.TransferParams(num_dirs=S, sh_bands=3, bounce_mode="index", bounces=1, t_same=t_same)
    idx = prt.index_matrix(sc, bvh, params, check=True).cpu().numpy()
    ref, amb = oracle_mod.index_matrix(scene, S, t_same=t_same)
    assert (ref >= 0).mean() > 0.02                # the bounce has something to gather
    assert np.array_equal(idx[~amb], ref[~amb])
    assert amb.mean() < 0.01
    assert ((idx >= -1) & (idx < n)).all()


@pytest.mark.parametrize("c_prev", [1, 3])
def test_self_transfer_parity(prt, oracle_mod, c_prev):
    """One gather step on the oracle's index matrix and a random previous
    term: FP32 sums against FP64."""
    import torch
    scene = _scene(31)
    n, S, K = scene["means"].shape[0], 64, 16
    ref_idx, _ = oracle_mod.index_matrix(scene, S)
    t_prev = np.random.default_rng(7).standard_normal((n, c_prev, K)).astype(np.float32).astype(np.float64)
    sc = prt.Scene.from_arrays(scene)
    params = prt.TransferParams(num_dirs=S, sh_bands=4)
    got = prt.self_transfer(sc, params, torch.tensor(ref_idx, device="cuda"),
                            torch.tensor(t_prev, dtype=torch.float32, device="cuda"), check=True).cpu().numpy()
    ref = oracle_mod.self_transfer(scene, S, ref_idx, t_prev)
    scale = np.abs(ref).max()
    assert np.abs(got - ref).max() <= 2e-6 * scale


def _index_allowance(oracle_mod, scene, S, idx, amb, terms, allow0):
    """Bound on legitimate deviation of sum_m T^m: the direct term's own
    bound, carried through each gather (albedo <= 1), plus, per ambiguous ray,
    the largest term it could gather instead (twice)."""
    dirs = oracle_mod.directions(S, 0)
    c = np.clip(scene["normals"] @ dirs.T, 0, None)
    wq = 4 * math.pi / S
    A_prev = np.repeat(allow0, 3, axis=1)            # [n, 3, K]
    total = A_prev.copy()
    for m in range(1, len(terms)):
        big = np.abs(terms[m - 1]).max()
        amb_part = wq * (c * amb).sum(1) * 2.0 / math.pi * big
        g = np.where(idx[..., None, None] >= 0, A_prev[np.maximum(idx, 0)], 0.0)   # [n, S, 3, K]
        prop = wq / math.pi * np.einsum("ns,nsck->nck", c, g)
        A_prev = amb_part[:, None, None] + prop
        total += A_prev
    return total


def test_index_transfer_end_to_end(prt, oracle_mod):
    """precompute_transfer in index mode with 3 bounces: every source against
    the oracle's sum of T^0 .. T^3."""
    scene = _scene(41)
    S, bands, M = 64, 4, 3
    sc = prt.Scene.from_arrays(scene)
    bvh = prt.build_bvh(sc, check=True)
    params = prt.TransferParams(num_dirs=S, sh_bands=bands, bounce_mode="index", bounces=M)
    t = prt.precompute_transfer(sc, bvh, params, check=True).cpu().numpy()
    ref = oracle_mod.index_transfer(scene, S, bands, M)
    allow0 = oracle_mod.direct_transfer(scene, S, bands, want_allow=True)["allow"][:, None, :]
    allow = _index_allowance(oracle_mod, scene, S, ref["index"], ref["amb"], ref["terms"], allow0)
    err = assert_transfer_parity(t, ref["t"], allow, tol=2e-4, what="index transfer")
    # the bounces are not negligible here
    assert np.abs(ref["t"] - np.repeat(ref["terms"][0], 3, axis=1)).max() > 1e-2
    print(f"index transfer max |dt| = {err:.2e}")


def test_index_pipeline_equals_composition(prt):
    """The precompute's index mode equals index_matrix + self_transfer steps
    composed by hand (same kernels, same order of sums)."""
    import torch
    scene = _scene(51)
    S, bands, M = 64, 3, 2
    sc = prt.Scene.from_arrays(scene)
    bvh = prt.build_bvh(sc)
    p_idx = prt.TransferParams(num_dirs=S, sh_bands=bands, bounce_mode="index", bounces=M, t_same=0.9)
    t = prt.precompute_transfer(sc, bvh, p_idx)
    d = prt.precompute_transfer(sc, bvh, prt.TransferParams(num_dirs=S, sh_bands=bands))
    idx = prt.index_matrix(sc, bvh, p_idx)
    total = d.repeat(1, 3, 1)
    prev = total.clone()
    for _ in range(M):
        prev = prt.self_transfer(sc, p_idx, idx, prev)
        total = total + prev
    assert torch.allclose(t, total, rtol=1e-6, atol=1e-7)


def test_index_zero_albedo_is_direct(prt):
    import torch
    scene = _scene(61)
    scene["albedo"][:] = 0.0
    sc = prt.Scene.from_arrays(scene)
    bvh = prt.build_bvh(sc)
    t = prt.precompute_transfer(sc, bvh, prt.TransferParams(num_dirs=64, sh_bands=4, bounce_mode="index", bounces=4))
    d = prt.precompute_transfer(sc, bvh, prt.TransferParams(num_dirs=64, sh_bands=4))
    for ch in range(3):
        assert torch.equal(t[:, ch], d[:, 0])
