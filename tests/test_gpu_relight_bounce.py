"""GPU parity of the one-bounce transfer, the relight GEMM (FP32 / BF16 / F16)
and its adjoint against the CPU FP64 oracle."""
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


def _small_million_like(seed=21):
    """The million-splat recipe at a few thousand splats: surface scene plus
    ellipsoid shells."""
    return scenegen._concat([scenegen.surface_scene(2500, seed), scenegen.shells(4, 800, seed + 1)])


@pytest.mark.parametrize("S,bands", [(64, 4), (32, 3)])
def test_bounce_parity_sampled(prt, oracle_mod, S, bands):
    scene = as_f32(_small_million_like())
    n = scene["means"].shape[0]
    params = prt.TransferParams(num_dirs=S, sh_bands=bands, bounces=1)
    sc = prt.Scene.from_arrays(scene)
    bvh = prt.build_bvh(sc, check=True)
    t = prt.precompute_transfer(sc, bvh, params, check=True).cpu().numpy()
    src = np.random.default_rng(3).choice(n, 200, replace=False)
    ref = oracle_mod.full_transfer(scene, S, bands, 1, sources=src, want_allow=True)
    err = assert_transfer_parity(t[src], ref["t"], ref["allow"], what="bounce transfer")
    # the bounce term is not negligible in this scene
    assert np.abs(ref["t_ind"]).max() > 1e-2
    print(f"bounce max |dt| = {err:.2e}, max |t_ind| = {np.abs(ref['t_ind']).max():.3f}")


@pytest.mark.parametrize("n_surface", [901, 1902])
def test_bounce_source_count_not_whole_blocks(prt, oracle_mod, n_surface):
    """Source counts (1201, 2202) whose persistent bounce launch does not
    fill its last block of 4 waves: the spare waves hold no hit lists and must
    take no work.  Blend and index matrix against the oracle, flags clear."""
    scene = as_f32(scenegen._concat([scenegen.surface_scene(n_surface, 31), scenegen.shells(1, 300, 32)]))
    n = scene["means"].shape[0]
    assert n % 4 != 0
    S, bands = 32, 3
    sc = prt.Scene.from_arrays(scene)
    bvh = prt.build_bvh(sc, check=True)
    t = prt.precompute_transfer(sc, bvh, prt.TransferParams(num_dirs=S, sh_bands=bands, bounces=1),
                                check=True).cpu().numpy()
    src = np.random.default_rng(5).choice(n, 80, replace=False)
    ref = oracle_mod.full_transfer(scene, S, bands, 1, sources=src, want_allow=True)
    assert_transfer_parity(t[src], ref["t"], ref["allow"], what="bounce transfer")
    params = prt.TransferParams(num_dirs=S, sh_bands=bands, bounce_mode="index", bounces=1)
    idx = prt.index_matrix(sc, bvh, params, check=True).cpu().numpy()
    ref_idx, amb = oracle_mod.index_matrix(scene, S, t_same=params.t_same, sources=src)
    assert np.array_equal(idx[src][~amb], ref_idx[~amb])
    assert ((idx >= -1) & (idx < n)).all()


def test_bounce_many_faint_hits(prt, oracle_mod):
    """A crowded, faint cloud: rays meet hundreds of Gaussians before the
    transmittance falls below T_eps (or never do), so a ray can list more hits
    than its hit list holds in one round (PRTGS_BOUNCE_HIT_LIST) and needs
    further rounds."""
    from paper_2408_03538_amd import _lib
    scene = scenegen.random_cloud(1500, 23)
    scene["means"] *= 0.3
    scene["opacity"] *= 0.04
    scene = as_f32(scene)
    n = scene["means"].shape[0]
    S, bands = 32, 3
    src = np.random.default_rng(4).choice(n, 60, replace=False)
    # hits along the sampled sources' rays (3-sigma ellipsoids crossed ahead of
    # the origin): some ray has more than a list holds
    R = np.stack([_rot(q) for q in scene["quats"].astype(np.float64)])
    inv_s2 = np.exp(-2.0 * scene["log_scales"].astype(np.float64))
    Ainv = np.einsum("nij,nj,nkj->nik", R, inv_s2, R)
    dirs = oracle_mod.directions(S)
    most = 0
    for i in src:
        o = scene["means"][i].astype(np.float64)
        dx = scene["means"] - o
        for w in dirs[scene["normals"][i] @ dirs.T > 0]:
            a = np.einsum("i,nij,j->n", w, Ainv, w)
            b = np.einsum("i,nij,nj->n", w, Ainv, dx)
            c = np.einsum("ni,nij,nj->n", dx, Ainv, dx)
            most = max(most, int(((c - b * b / a < 9.0) & (b / a > 0)).sum()))
    assert most > _lib.BOUNCE_HIT_LIST, most
    params = prt.TransferParams(num_dirs=S, sh_bands=bands, bounces=1)
    sc = prt.Scene.from_arrays(scene)
    bvh = prt.build_bvh(sc, check=True)
    t = prt.precompute_transfer(sc, bvh, params, check=True).cpu().numpy()
    st = prt.traversal_stats(sc, bvh, params)
    assert st["rounds"] > st["traced_rays"]          # some rays overflowed their list
    ref = oracle_mod.full_transfer(scene, S, bands, 1, sources=src, want_allow=True)
    err = assert_transfer_parity(t[src], ref["t"], ref["allow"], what="bounce transfer")
    assert np.abs(ref["t_ind"]).max() > 1e-2
    print(f"faint cloud: bounce max |dt| = {err:.2e}, max |t_ind| = {np.abs(ref['t_ind']).max():.3f}")


def _million_recipe(n_surface, per_shell, seed):
    """The million-splat recipe (surface scene + 20 ellipsoid shells) at a
    size the brute-force oracle finishes."""
    return scenegen._concat([scenegen.surface_scene(n_surface, seed), scenegen.shells(20, per_shell, seed + 1)])


@pytest.mark.parametrize("S", [512, 256])
def test_bounce_parity_million_launch_shape(prt, oracle_mod, S):
    """The launch shape of the million-splat workload: 16 sources per wave
    and 64 direction parts, each with sums of its own for the blend (one part
    holds 2 direction batches at S = 512, 1 at S = 256), on an 8,000-splat
    scene of the same recipe.  24 sampled sources against the oracle's full
    transfer (direct + bounce); the index matrix of the paper's bounce in the
    same launch shape against the oracle's.  A part dropped or added twice
    moves the bounce term by a sixty-fourth of its size, still beyond the
    allowance."""
    scene = as_f32(_million_recipe(1600, 320, 41))
    n = scene["means"].shape[0]
    sc = prt.Scene.from_arrays(scene)
    bvh = prt.build_bvh(sc, check=True)
    params = prt.TransferParams(num_dirs=S, sh_bands=4, bounces=1, sources_per_wave=16, direction_parts=64)
    t = prt.precompute_transfer(sc, bvh, params, check=True).cpu().numpy()
    src = np.random.default_rng(43).choice(n, 24, replace=False)
    print(f"million-shape bounce S = {S}: oracle on 24 sources", flush=True)
    ref = oracle_mod.full_transfer(scene, S, 4, 1, sources=src, want_allow=True)
    err = assert_transfer_parity(t[src], ref["t"], ref["allow"], what="bounce transfer")
    ind = np.abs(ref["t_ind"][:, :, 0])
    assert np.median(ind / (1e-4 + ref["allow"][:, :, 0])) > 64.0   # a sixty-fourth of the term is visible
    # the same sums in one part: the regrouping moves only the last bits
    one = prt.precompute_transfer(sc, bvh, prt.TransferParams(num_dirs=S, sh_bands=4, bounces=1, sources_per_wave=16,
                                                              direction_parts=1), check=True).cpu().numpy()
    assert np.abs(one - t).max() <= 1e-5 * (1.0 + np.abs(t).max())
    pidx = prt.TransferParams(num_dirs=S, sh_bands=4, bounce_mode="index", bounces=1, sources_per_wave=16,
                              direction_parts=64)
    idx = prt.index_matrix(sc, bvh, pidx, check=True).cpu().numpy()
    ref_idx, amb = oracle_mod.index_matrix(scene, S, sources=src)
    assert (ref_idx >= 0).sum() > 200
    assert np.array_equal(idx[src][~amb], ref_idx[~amb])
    print(f"million-shape bounce S = {S}: max |dt| {err:.2e}, max |t_ind| {ind.max():.3f}, "
          f"{int(amb.sum())} ambiguous index rays of {amb.size}")


def test_bounce_coincident_hits_progress(prt, oracle_mod):
    """300 coincident faint splats in front of a few sources: every ray
    through them lists 300 hits at the same peak depth, more than its hit
    list holds, and the list's mean depth equals every listed depth.  The
    compaction must still keep the nearest hit, so each round blends one
    and the walk ends (no round cap, no flag), matching the oracle."""
    rng = np.random.default_rng(51)
    m = 300
    cluster = dict(means=np.tile([0.0, 0.0, 1.0], (m, 1)), quats=np.tile([1.0, 0.0, 0.0, 0.0], (m, 1)),
                   log_scales=np.full((m, 3), np.log(0.12)), opacity=np.full(m, 0.004),
                   normals=np.tile([0.0, 0.0, -1.0], (m, 1)), albedo=np.full((m, 3), 0.6))
    k = 4
    srcs = dict(means=np.column_stack([rng.uniform(-0.05, 0.05, (k, 2)), np.zeros(k)]),
                quats=np.tile([1.0, 0.0, 0.0, 0.0], (k, 1)), log_scales=np.full((k, 3), np.log(0.01)),
                opacity=np.full(k, 0.5), normals=np.tile([0.0, 0.0, 1.0], (k, 1)), albedo=np.full((k, 3), 0.5))
    scene = as_f32(scenegen._concat([srcs, cluster]))
    S = 256
    params = prt.TransferParams(num_dirs=S, sh_bands=3, bounces=1)
    sc = prt.Scene.from_arrays(scene)
    bvh = prt.build_bvh(sc, check=True)
    t = prt.precompute_transfer(sc, bvh, params, check=True).cpu().numpy()
    st = prt.traversal_stats(sc, bvh, params)
    assert st["rounds"] > st["traced_rays"] + 10       # the lists overflowed and were compacted
    ref = oracle_mod.full_transfer(scene, S, 3, 1, sources=np.arange(k), want_allow=True)
    assert np.abs(ref["t_ind"]).max() > 1e-2
    assert_transfer_parity(t[:k], ref["t"], ref["allow"], what="coincident bounce")


def _rot(q):
    w, x, y, z = q / np.linalg.norm(q)
    return np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
                     [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
                     [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)]])


def test_bounce_zero_albedo_is_direct(prt):
    import torch
    scene = as_f32(_small_million_like(5))
    scene["albedo"][:] = 0.0
    sc = prt.Scene.from_arrays(scene)
    bvh = prt.build_bvh(sc)
    tb = prt.precompute_transfer(sc, bvh, prt.TransferParams(num_dirs=64, sh_bands=4, bounces=1))
    td = prt.precompute_transfer(sc, bvh, prt.TransferParams(num_dirs=64, sh_bands=4, bounces=0))
    for ch in range(3):
        assert torch.equal(tb[:, ch], td[:, 0])


# ---------------------------------------------------------------------------
# relight
# ---------------------------------------------------------------------------

def _relight_inputs(n, C, K, B, seed):
    bands = int(round(K ** 0.5))
    T = scenegen.synthetic_transfers(n, bands, C, seed).astype(np.float32).astype(np.float64)
    L = scenegen.light_sh(B, bands, seed + 1, band_decay=True).astype(np.float32).astype(np.float64)
    return T, L


def _scale(T, L):
    """sum_k |T_k L_k| per output (the error scale of a dot product)."""
    return np.einsum("nck,bck->nbc", np.abs(T), np.abs(L)) if T.shape[1] == 3 else \
        np.einsum("nk,bck->nbc", np.abs(T[:, 0]), np.abs(L))


@pytest.mark.parametrize("n,C,K,B", [(5000, 1, 16, 1), (5000, 3, 16, 64), (777, 3, 9, 7), (1000, 1, 4, 100),
                                     (333, 3, 16, 256), (17, 1, 1, 3), (1001, 3, 16, 18), (513, 1, 4, 33)])
def test_relight_f32(prt, oracle_mod, n, C, K, B):
    """FP32 transfer and colours against the FP64 product: the one-thread-per-
    colour kernel (fewer than 16 lights, K = 1 or 9) and the FP32 MFMA one,
    with whole 32-light chunks (16-byte row stores) and partial ones or light
    counts not divisible by 4 (18, 33, the last 4 of 100: element stores)."""
    import torch
    T, L = _relight_inputs(n, C, K, B, 40 + K)
    out = prt.relight(torch.tensor(T, dtype=torch.float32, device="cuda"),
                      torch.tensor(L, dtype=torch.float32, device="cuda"))
    ref = oracle_mod.relight(T, L)
    err = np.abs(out.cpu().numpy() - ref)
    assert (err <= 2e-6 * _scale(T, L) + 1e-12).all(), err.max()


def test_pack_rounds_to_nearest_even(prt):
    import torch
    x = torch.randn(100003, dtype=torch.float32) * 3
    x[:4] = torch.tensor([1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, -0.0, 65504.0])
    for name, dt in (("bf16", torch.bfloat16), ("f16", torch.float16)):
        got = prt.pack(x.cuda(), name).cpu()
        assert torch.equal(got.view(torch.int16), x.to(dt).view(torch.int16))


@pytest.mark.parametrize("tdt", ["bf16", "f16"])
@pytest.mark.parametrize("n,C,K,B", [(5000, 3, 16, 64), (4099, 1, 16, 1), (999, 3, 9, 7), (300, 1, 4, 100),
                                     (123, 3, 16, 256)])
@pytest.mark.parametrize("odt", ["f16", "f32"])
def test_relight_mfma(prt, oracle_mod, tdt, n, C, K, B, odt):
    """16-bit storage on MFMA.  Exact layout check: against the FP64 product of
    the *rounded* transfer (rounded on the CPU), only the light split and the
    output rounding remain; against the unrounded transfer the error is the
    storage error, <= u_T sum|T L| + u_out |C|."""
    import torch
    tdtype = {"bf16": torch.bfloat16, "f16": torch.float16}[tdt]
    T, L = _relight_inputs(n, C, K, B, 60 + K)
    T16 = torch.tensor(T, dtype=torch.float32).to(tdtype)
    out = prt.relight(T16.cuda(), torch.tensor(L, dtype=torch.float32, device="cuda"), out_dtype=odt)
    got = out.float().cpu().numpy().astype(np.float64)
    scale = _scale(T, L)
    u_out = 2.0 ** -11 if odt == "f16" else 2.0 ** -24
    ref_q = oracle_mod.relight(T16.to(torch.float64).numpy(), L)
    err_q = np.abs(got - ref_q)
    u_split = 2.0 ** -16 if tdt == "bf16" else 2.0 ** -22   # light = hi + lo, both 16-bit
    assert (err_q <= u_out * np.abs(ref_q) + (u_split + 2e-6) * scale + 1e-12).all(), err_q.max()
    ref = oracle_mod.relight(T, L)
    u_T = 2.0 ** -8 if tdt == "bf16" else 2.0 ** -11
    err = np.abs(got - ref)
    assert (err <= u_T * scale + u_out * np.abs(ref) + (u_split + 2e-6) * scale + 1e-12).all()
    primary = (err / np.maximum(scale, 1e-30)).max()
    assert primary <= 1e-2
    print(f"{tdt}->{odt} C={C} K={K} B={B}: max |dC|/sum|TL| = {primary:.2e}")


@pytest.mark.parametrize("n,C,K,B", [(3000, 1, 16, 1), (2000, 3, 16, 64), (517, 3, 9, 5)])
def test_relight_backward(prt, oracle_mod, n, C, K, B):
    import torch
    T, L = _relight_inputs(n, C, K, B, 80)
    dC = np.random.default_rng(81).standard_normal((n, B, 3)).astype(np.float32).astype(np.float64)
    dT, dL = prt.relight_backward(torch.tensor(T, dtype=torch.float32, device="cuda"),
                                  torch.tensor(L, dtype=torch.float32, device="cuda"),
                                  torch.tensor(dC, dtype=torch.float32, device="cuda"))
    rT, rL = oracle_mod.relight_grads(T, L, dC)
    sT = np.einsum("nbc,bck->nk", np.abs(dC), np.abs(L))[:, None, :] if C == 1 else \
        np.einsum("nbc,bck->nck", np.abs(dC), np.abs(L))
    assert (np.abs(dT.cpu().numpy() - rT) <= 1e-5 * sT + 1e-12).all()
    sL = np.einsum("nbc,nk->bck", np.abs(dC), np.abs(T[:, 0])) if C == 1 else \
        np.einsum("nbc,nck->bck", np.abs(dC), np.abs(T))
    assert (np.abs(dL.cpu().numpy() - rL) <= 1e-6 * sL + 1e-12).all()
