"""Pins of the oracle's index matrix and recursive self-transfer (the paper's
own bounce: Sec. 4.4 Eq. 26 with the same-surface filter, Sec. 4.5 Eq. 32-35)
against an independent NumPy walk, closed forms and special cases."""
import math

import numpy as np
import pytest
from scipy.spatial.transform import Rotation

import scenegen


def _numpy_index(sc, S, t_same, T_eps=1e-4, alpha_max=0.99):
    """Per ray, straight from the definition: hits sorted by (t*, j), T in
    front of each, W = alpha T max(-w.n_j, 0) over hits with T <= t_same,
    argmax (first on ties), walk ending after the hit that takes T below T_eps."""
    import oracle
    dirs = oracle.directions(S, 0)
    mu = np.asarray(sc["means"], dtype=np.float64)
    n = mu.shape[0]
    q = np.asarray(sc["quats"], dtype=np.float64)
    R = Rotation.from_quat(np.concatenate([q[:, 1:], q[:, :1]], axis=1)).as_matrix()
    s2 = np.exp(-2.0 * np.asarray(sc["log_scales"], dtype=np.float64))
    sinv = np.einsum("nab,nb,ncb->nac", R, s2, R)
    nrm = np.asarray(sc["normals"], dtype=np.float64)
    op = np.asarray(sc["opacity"], dtype=np.float64)
    idx = np.full((n, S), -1)
    for i in range(n):
        for s in range(S):
            w = dirs[s]
            if not nrm[i] @ w > 0:
                continue
            hits = []
            for j in range(n):
                if j == i:
                    continue
                rel = mu[j] - mu[i]
                a = w @ sinv[j] @ w
                t = (rel @ sinv[j] @ w) / a
                e = mu[i] + t * w - mu[j]
                d2 = e @ sinv[j] @ e
                if t > 0.0 and d2 <= 9.0:
                    hits.append((t, j, min(op[j] * math.exp(-0.5 * d2), alpha_max)))
            hits.sort()
            T, best, bestW = 1.0, -1, 0.0
            for t, j, al in hits:
                if T <= t_same:
                    W = al * T * max(-(w @ nrm[j]), 0.0)
                    if W > bestW:
                        best, bestW = j, W
                T *= 1.0 - al
                if T < T_eps:
                    break
            idx[i, s] = best
    return idx


@pytest.mark.parametrize("t_same", [1.0, 0.9, 0.5])
def test_index_matches_numpy_walk(oracle_mod, t_same):
    sc = scenegen.random_cloud(40, 51)
    sc["means"] *= 0.3
    idx, amb = oracle_mod.index_matrix(sc, 32, t_same=t_same)
    ref = _numpy_index(sc, 32, t_same)
    assert (idx >= 0).sum() > 40
    assert np.array_equal(idx[~amb], ref[~amb])
    assert amb.mean() < 0.05


def _plates(normal_z=-1.0, o_near=0.3, o_far=0.9):
    """A source at the origin facing +z under two wide flat Gaussians at
    z = 0.5 and z = 0.8 whose normals are (0, 0, normal_z)."""
    sc = dict(means=np.array([[0.0, 0.0, 0.0], [0.0, 0.0, 0.5], [0.0, 0.0, 0.8]]),
              quats=np.tile([1.0, 0.0, 0.0, 0.0], (3, 1)),
              log_scales=np.log(np.array([[0.01, 0.01, 0.001], [10.0, 10.0, 0.001], [10.0, 10.0, 0.001]])),
              opacity=np.array([0.5, o_near, o_far]),
              normals=np.array([[0.0, 0.0, 1.0], [0.0, 0.0, normal_z], [0.0, 0.0, normal_z]]),
              albedo=np.full((3, 3), 0.5))
    return sc


def test_index_facing_and_depth_weights(oracle_mod):
    """Both plates face the source: W_near = 0.3 f, W_far = 0.9 (1 - 0.3) f, so
    the far plate wins every upward ray; t_same = 0.8 filters the near plate
    only (T = 1 in front of it), t_same = 0.6 both; plates facing away give
    no weight at all."""
    S = 64
    dirs = oracle_mod.directions(S, 0)
    up = dirs[:, 2] > 0.3                    # these rays cross both plates within 0.3 sigma of their centres
    for t_same, expect in ((1.0, 2), (0.8, 2), (0.6, -1)):
        idx, _ = oracle_mod.index_matrix(_plates(), S, t_same=t_same, sources=[0])
        assert (idx[0, up] == expect).all(), (t_same, idx[0, up])
        assert (idx[0, ~(dirs[:, 2] > 0)] == -1).all()
    idx, _ = oracle_mod.index_matrix(_plates(o_near=0.8, o_far=0.5), S, sources=[0])
    assert (idx[0, up] == 1).all()            # 0.8 > 0.5 x 0.2
    idx, _ = oracle_mod.index_matrix(_plates(normal_z=1.0), S, sources=[0])
    assert (idx == -1).all()


def test_self_transfer_closed_form(oracle_mod):
    """Every ray of every splat but 0 picks splat 0, splat 0's rays pick
    splat 1: T^1_i = a_i (rho_0 / pi) t_0 and T^1_0 = a_0 (rho_1 / pi) t_1 with
    a_i = (4 pi / S) sum_s max(0, n_i . w_s); a second step chains them."""
    S, K, n = 48, 9, 6
    sc = scenegen.random_cloud(n, 52)
    dirs = oracle_mod.directions(S, 0)
    a = (4 * math.pi / S) * np.clip(sc["normals"] @ dirs.T, 0, None).sum(1)
    idx = np.zeros((n, S), dtype=np.int32)
    idx[0] = 1
    idx[2, ::3] = -1                          # some rays of splat 2 hit nothing
    a2 = (4 * math.pi / S) * np.clip(sc["normals"][2] @ dirs.T, 0, None)
    a2 = a2.sum() - a2[::3].sum()
    t0 = np.random.default_rng(53).standard_normal((n, 1, K))
    t1 = oracle_mod.self_transfer(sc, S, idx, t0)
    rho = sc["albedo"]
    for ch in range(3):
        assert np.allclose(t1[0, ch], a[0] * rho[1, ch] / math.pi * t0[1, 0], rtol=1e-12, atol=1e-14)
        assert np.allclose(t1[2, ch], a2 * rho[0, ch] / math.pi * t0[0, 0], rtol=1e-12, atol=1e-14)
        for i in (1, 3, 4, 5):
            assert np.allclose(t1[i, ch], a[i] * rho[0, ch] / math.pi * t0[0, 0], rtol=1e-12, atol=1e-14)
    t2 = oracle_mod.self_transfer(sc, S, idx, t1)
    for ch in range(3):
        assert np.allclose(t2[3, ch], a[3] * rho[0, ch] / math.pi * a[0] * rho[1, ch] / math.pi * t0[1, 0],
                           rtol=1e-12, atol=1e-14)


def test_index_transfer_with_everything_filtered_is_direct(oracle_mod):
    sc = scenegen.random_cloud(40, 54)
    sc["means"] *= 0.5
    r = oracle_mod.index_transfer(sc, 32, 3, 2, t_same=1e-12)
    assert (r["index"] == -1).all()
    for ch in range(3):
        assert np.array_equal(r["t"][:, ch], r["terms"][0][:, 0])
