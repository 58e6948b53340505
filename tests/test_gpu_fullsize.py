"""Full-size workloads, in the launch configuration the benchmark times.

The oracle is brute force, so at these sizes it checks sampled outputs one by
one (the transfer of randomly drawn sources); where no sampled output is
within its reach (the bounce needs the direct transfer of every splat a ray
hits, the gradient needs the whole forward), properties that hold at any size
are checked instead.
"""
import math

import numpy as np
import pytest

import scenegen
from helpers import as_f32, assert_ray_vis, assert_transfer_parity, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def prt():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2408_03538_amd as p
    return p


def _workload_scene(name):
    w = scenegen.workload(name)
    return w, as_f32(w["scene"])


def _sampled_parity(prt, oracle_mod, what, scene, S, bands, src, allow_share):
    """Transfer and per-ray visibility of the sampled sources against the
    oracle, in the default launch configuration; the share of coefficients
    whose near-threshold allowance exceeds the 1e-4 tolerance is printed and
    bounded."""
    import torch
    sc = prt.Scene.from_arrays(scene)
    bvh = prt.build_bvh(sc, check=True)
    params = prt.TransferParams(num_dirs=S, sh_bands=bands)
    t, vis = prt.precompute_transfer(sc, bvh, params, want_vis=True, check=True)
    rows = torch.tensor(src, device=t.device)
    assert torch.isfinite(t).all()
    t_s = t[rows, 0, :].cpu().numpy()
    v_s = vis[rows].cpu().numpy()
    del t, vis
    say(f"{what}: oracle on {len(src)} sources")
    ref = oracle_mod.direct_transfer(scene, S, bands, sources=src, want_vis=True, want_allow=True, want_vis_bounds=True)
    err = assert_transfer_parity(t_s, ref["t"], ref["allow"])
    cos = scene["normals"][src] @ oracle_mod.directions(S).T
    rays, wide = assert_ray_vis(v_s, ref, cos, oracle_mod.DEFAULT_MARGINS[0], what)
    share = float((ref["allow"] > 1e-4).mean())
    say(f"{what}: max |dt| = {err:.2e}; {rays} rays within their range ({wide} near a threshold); coefficients "
         f"with allowance > 1e-4: {100 * share:.2f}% (largest {ref['allow'].max():.1e})")
    assert share < allow_share


def test_surface100k_sampled_sources(prt, oracle_mod):
    """100,000-splat surface scene, S = 256, 16 coeffs: 48 sources against
    the oracle, transfer and every ray.  Same-surface neighbours put peak
    depths within the t* margin of the origin on some grazing rays, hence
    the allowance on ~4% of the coefficients (every ray is checked on its
    own as well)."""
    w, scene = _workload_scene("surface100k")
    src = np.random.default_rng(100).choice(scene["means"].shape[0], 48, replace=False)
    _sampled_parity(prt, oracle_mod, "surface100k", scene, w["num_dirs"], w["bands"], src, 0.05)


def test_million_direct_sampled_sources(prt, oracle_mod):
    """1,000,000 splats (surface + 20 shells), S = 512, 16 coeffs: the direct
    transfer and every ray of 6 sources against the oracle."""
    w, scene = _workload_scene("million")
    n = scene["means"].shape[0]
    rng = np.random.default_rng(101)
    # three surface splats, three shell splats
    src = np.concatenate([rng.choice(200_000, 3, replace=False), 200_000 + rng.choice(n - 200_000, 3, replace=False)])
    _sampled_parity(prt, oracle_mod, "million", scene, w["num_dirs"], w["bands"], src, 0.01)


def test_million_bounce_properties(prt):
    """The one-bounce pass on the full million-splat scene.  With albedo
    (a, 2a, 0) the blue channel must be the direct transfer bit for bit, the
    green bounce term twice the red one (scaling by 2 is exact), the bounce
    DC term non-negative and, per ray, the blend weights at most the occluded
    fraction 1 - V, so that
      t_ind[i, c, 0] <= (4 pi / S) sum_s c_s (1 - V_s) max_j rho_jc t_dir[j, 0] / pi."""
    import torch
    w, scene = _workload_scene("million")
    n = scene["means"].shape[0]
    a = scene["albedo"][:, 0].copy()
    scene["albedo"] = np.stack([a, 2.0 * a, np.zeros_like(a)], axis=1)
    sc = prt.Scene.from_arrays(scene)
    bvh = prt.build_bvh(sc, check=True)
    S, bands = w["num_dirs"], w["bands"]
    say("million: direct transfer with visibility")
    td, vis = prt.precompute_transfer(sc, bvh, prt.TransferParams(num_dirs=S, sh_bands=bands), want_vis=True,
                                      check=True)
    say("million: direct + bounce")
    tb = prt.precompute_transfer(sc, bvh, prt.TransferParams(num_dirs=S, sh_bands=bands, bounces=1), check=True)
    assert torch.equal(tb[:, 2], td[:, 0])
    d = td[:, 0].double()
    ind0 = tb[:, 0].double() - d
    ind1 = tb[:, 1].double() - d
    scale = d.abs() + 1.0
    lin = ((ind1 - 2.0 * ind0).abs() / scale).max().item()
    assert lin < 2e-5, lin
    assert ind0[:, 0].min().item() > -2e-5
    assert ind0.abs().max().item() > 1e-2          # the bounce is not negligible
    # the bound on the DC term, for 2,000 sampled sources
    rows = np.random.default_rng(102).choice(n, 2000, replace=False)
    rows_t = torch.tensor(rows, device=td.device)
    V = vis[rows_t].double().cpu().numpy()
    dirs = prt.direction_table(S, 0, bands)[2].double().cpu().numpy()
    c = scene["normals"][rows] @ dirs.T
    occluded = np.where(c > 0, c * (1.0 - np.clip(V, 0.0, 1.0)), 0.0).sum(1)
    rho_t = (torch.tensor(scene["albedo"][:, 0], device=td.device, dtype=torch.float64) * td[:, 0, 0].double())
    bound = (4 * math.pi / S) * occluded * rho_t.max().item() / math.pi
    got = ind0[rows_t, 0].cpu().numpy()
    assert (got <= bound + 2e-5).all(), float((got - bound).max())
    say(f"million bounce: linearity {lin:.1e}, max bounce DC {got.max():.3f} (bound {bound.max():.3f})")


def test_million_index_sampled_rows(prt, oracle_mod):
    """The paper's bounce on the full million-splat scene (S = 512): the index
    matrix rows of 4 sources against the oracle, and the 3-bounce transfer
    finite and above the direct one in every channel's DC term (gathered
    terms of non-negative DC transfers are non-negative)."""
    import torch
    w, scene = _workload_scene("million")
    n = scene["means"].shape[0]
    sc = prt.Scene.from_arrays(scene)
    bvh = prt.build_bvh(sc, check=True)
    S, bands = w["num_dirs"], w["bands"]
    params = prt.TransferParams(num_dirs=S, sh_bands=bands, bounce_mode="index", bounces=3)
    say("million: index matrix")
    idx = prt.index_matrix(sc, bvh, params, check=True)
    rng = np.random.default_rng(106)
    rows = np.concatenate([rng.choice(200_000, 2, replace=False), 200_000 + rng.choice(n - 200_000, 2, replace=False)])
    say("million: oracle index rows of 4 sources")
    ref, amb = oracle_mod.index_matrix(scene, S, sources=rows)
    got = idx[torch.tensor(rows, device=idx.device)].cpu().numpy()
    assert (ref >= 0).sum() > 20
    assert np.array_equal(got[~amb], ref[~amb])
    # rays meet hundreds of Gaussians here, so some choice often hangs on a
    # hit at the 3-sigma edge (measured: ~6% of these rows)
    assert amb.mean() < 0.1
    say("million: 3-bounce transfer")
    t = prt.precompute_transfer(sc, bvh, params, check=True)
    d = prt.precompute_transfer(sc, bvh, prt.TransferParams(num_dirs=S, sh_bands=bands))
    assert torch.isfinite(t).all()
    gain = (t[:, :, 0] - d[:, :, 0]).double()
    assert gain.min().item() > -2e-5 and gain.max().item() > 1e-2
    say(f"million index: {int((got >= 0).sum())} indexed rays in the sample, max DC gain {gain.max().item():.3f}")


def test_relight3m_full(prt, oracle_mod):
    """3,000,000 RGB transfers x 64 lights in FP32, BF16 and F16 storage:
    sampled colours against the FP64 product, relative to sum |T| |L|."""
    import torch
    w = scenegen.workload("relight3m")
    T64 = np.asarray(w["transfer"], np.float32).astype(np.float64)
    L64 = np.asarray(w["light"], np.float32).astype(np.float64)
    T = torch.tensor(T64, dtype=torch.float32, device="cuda")
    L = torch.tensor(L64, dtype=torch.float32, device="cuda")
    rows = np.random.default_rng(103).choice(T.shape[0], 20000, replace=False)
    ref = oracle_mod.relight(T64[rows], L64)
    scale = np.einsum("nck,bck->nbc", np.abs(T64[rows]), np.abs(L64))
    rows_t = torch.tensor(rows, device="cuda")
    bounds = {("f32", "f32"): 2e-6, ("bf16", "f16"): 1e-2, ("f16", "f16"): 1e-2, ("bf16", "f32"): 1e-2}
    for (tdt, odt), bound in bounds.items():
        say(f"relight3m: {tdt} -> {odt}")
        t = T if tdt == "f32" else prt.pack(T, tdt)
        out = prt.relight(t, L, out_dtype=odt)
        got = out[rows_t].double().cpu().numpy()
        rel = np.abs(got - ref) / scale
        assert rel.max() <= bound, (tdt, odt, rel.max())
        say(f"relight3m {tdt} -> {odt}: max rel err {rel.max():.2e}, mean {rel.mean():.2e}")
        del out


def _grad200k_adjoint(prt, scene, w):
    """The adjoint at the 200k configuration under the linear loss
    sum(W * colour), W ~ N(0, 1) fixed (so d loss / d transfer = W . light)."""
    import torch
    n = scene["means"].shape[0]
    keys = ("means", "quats", "log_scales", "opacity", "normals")
    params = prt.TransferParams(num_dirs=w["num_dirs"], sh_bands=w["bands"])
    L64 = np.asarray(w["light"], np.float32).astype(np.float64)
    W64 = np.random.default_rng(104).standard_normal((n, 1, 3)).astype(np.float32).astype(np.float64)
    light = torch.tensor(L64, dtype=torch.float32, device="cuda")
    Wt = torch.tensor(W64, dtype=torch.float32, device="cuda")
    ten = {k: torch.tensor(scene[k], dtype=torch.float32, device="cuda", requires_grad=True) for k in keys}
    col = prt.transfer_and_relight(*[ten[k] for k in keys], light, params)
    (col * Wt).sum().backward()
    g = {k: ten[k].grad.double().cpu().numpy() for k in keys}
    dT = np.einsum("nbc,bck->nk", W64, L64)              # d loss / d transfer
    return g, dT


def test_grad200k_sampled_gaussians(prt):
    """200,000 surface splats, S = 256, 16 coeffs, transfer + relight under a
    linear loss: the adjoint's gradient with respect to the opacity,
    log-scales, quaternion, mean and normal of 8 sampled Gaussians against the
    FP64 oracle (per-ray references: these parameters act only through
    alpha_j on the rays that hit j, the mean also as the origin of j's own
    rays, and the normal through j's own rays), per component within 1e-3
    relative plus the bound of rays within FP32 rounding of a threshold."""
    from oracle.grad import gaussian_param_grads
    w, scene = _workload_scene("grad200k")
    n = scene["means"].shape[0]
    say("grad200k: forward + backward")
    g, dT = _grad200k_adjoint(prt, scene, w)
    picks = np.random.default_rng(105).choice(n, 8, replace=False)
    refs = []
    for j in picks:
        say(f"grad200k: oracle for Gaussian {j}")
        refs.append(gaussian_param_grads(scene, int(j), w["num_dirs"], w["bands"], dT))
    for key in ("opacity", "log_scales", "quats", "means", "normals"):
        scale = max(np.abs(np.asarray(r["grads"][key])).max() for r in refs)
        for j, r in zip(picks, refs):
            ref = np.asarray(r["grads"][key], dtype=np.float64)
            got = np.asarray(g[key][j], dtype=np.float64)
            tol = 1e-3 * np.maximum(np.abs(ref), 1e-2 * scale) + np.asarray(r["allow"][key])
            assert (np.abs(got - ref) <= tol).all(), (key, int(j), got, ref, r["allow"][key])
        say(f"grad200k {key}: ok (largest |g| {scale:.3e})")


def test_grad200k_central_differences(prt, oracle_mod):
    """The 200k configuration's adjoint against central differences of the
    FP64 oracle forward on 64 random parameters (16 Gaussians x 4 of their 14
    parameters, drawn with the finite-difference seed).  The loss is linear in
    the transfer, so only the rays a parameter can move enter the difference:
    the rays of other sources that reach Gaussian j (its peak within
    d^2 <= 10, ahead of the origin by more than -3 s_max) and, for the mean
    and normal, j's own rays; each is traced through all 200,000 Gaussians by
    the oracle.  Steps h = 1e-3 and h / 4 (means: in units of the Gaussian's
    smallest scale), combined by Richardson extrapolation; a parameter whose
    two estimates disagree has a cut-off decision inside the step and is
    skipped.  Within 1e-3 of max(|estimate|, 1e-2 of the largest estimate of
    that input)."""
    import math
    import torch
    from oracle.grad import _rotation
    w, scene = _workload_scene("grad200k")
    n = scene["means"].shape[0]
    S, bands = w["num_dirs"], w["bands"]
    say("grad200k FD: forward + backward")
    g, dT = _grad200k_adjoint(prt, scene, w)
    dirs, Y = oracle_mod.tables(S, 0, bands)
    wq = 4.0 * math.pi / S
    means = scene["means"]
    rng = np.random.default_rng(scenegen.SEED_FD_PICK)
    comps = [("opacity", ())] + [("log_scales", (a,)) for a in range(3)] + [("quats", (a,)) for a in range(4)] + \
            [("means", (a,)) for a in range(3)] + [("normals", (a,)) for a in range(3)]
    results = []
    D = torch.from_numpy(dirs)
    for q, j in enumerate(rng.choice(n, 16, replace=False)):
        j = int(j)
        say(f"grad200k FD: Gaussian {q + 1} of 16 (index {j})")
        # rays of other sources that reach j (FP64, every source)
        with torch.no_grad():
            R = _rotation(torch.from_numpy(scene["quats"][j][None]))[0]
            sinv = R @ torch.diag(torch.exp(-2.0 * torch.from_numpy(scene["log_scales"][j]))) @ R.T
            sw = D @ sinv
            a = (sw * D).sum(-1)
            rel = torch.from_numpy(means[j][None, :] - means)
            b = rel @ sw.T
            t = b / a[None]
            d2 = ((rel @ sinv) * rel).sum(-1)[:, None] - b * b / a[None]
            cw = torch.from_numpy(scene["normals"]) @ D.T
            smax = float(np.exp(scene["log_scales"][j]).max())
            reach = (d2 <= 10.0) & (t > -3.0 * smax) & (cw > 0.0)
            reach[j] = False
            ii, ss = (x.numpy() for x in torch.nonzero(reach, as_tuple=True))
        own = np.nonzero(scene["normals"][j] @ dirs.T > -1e-3)[0]
        src = np.concatenate([ii, np.full(len(own), j)])
        sdir = np.concatenate([ss, own])
        coef_other = wq * (scene["normals"][ii] * dirs[ss]).sum(1) * np.einsum("rk,rk->r", dT[ii], Y[ss])
        yj = Y[own] @ dT[j]

        def loss_rays(sc):
            V = oracle_mod.rays_vis(sc, src, dirs[sdir])
            c_own = dirs[own] @ sc["normals"][j]
            return float((coef_other * V[:len(ii)]).sum() + (wq * np.maximum(c_own, 0.0) * yj * V[len(ii):]).sum())

        picks = [comps[k] for k in rng.choice(len(comps), 4, replace=False)]
        for key, sub in picks:
            idx = (j,) + sub
            h0 = 1e-3 * (float(np.exp(scene["log_scales"][j]).min()) if key == "means" else 1.0)
            est = []
            for h in (h0, h0 / 4):
                vals = []
                for sgn in (1, -1):
                    pert = dict(scene)
                    pert[key] = scene[key].copy()
                    pert[key][idx] += sgn * h
                    vals.append(loss_rays(pert))
                est.append((vals[0] - vals[1]) / (2 * h))
            results.append((key, idx, est, float(g[key][idx])))
        say(f"grad200k FD: Gaussian {j}, {len(ii)} rays through it, {len(own)} of its own")
    checked = 0
    for key, idx, est, got in results:
        scale = max(abs(est[1]), 1e-2 * max(abs(e[1]) for k, _, e, _ in results if k == key), 1e-12)
        if abs(est[0] - est[1]) > 2e-3 * scale:
            continue                               # a cut-off crossed inside the step
        checked += 1
        rich = (16.0 * est[1] - est[0]) / 15.0
        assert abs(got - rich) <= 1e-3 * scale, (key, idx, got, est)
    say(f"grad200k FD: {checked} of {len(results)} parameters checked, by input: "
         f"{ {k: sum(1 for r in results if r[0] == k) for k in dict(comps)} }")
    # thousands of rays reach each Gaussian, so about half the parameters have
    # a cut-off decision inside +-h and are skipped
    assert checked >= 24
