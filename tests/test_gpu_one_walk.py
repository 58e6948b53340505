"""GPU parity of the blended bounce in one walk per ray (bounce_records > 0:
the walk that blends each ray's hits also gives its visibility, and the
blended hits' records wait in an arena until every direct transfer exists)
against the CPU FP64 oracle, against the two-walk blend, and with an arena too
small for the work, where the items whose records do not fit are redone by
the two-walk pass."""
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


def _small_million_like(seed=21):
    """The million-splat recipe at a few thousand splats: surface scene plus
    ellipsoid shells."""
    return scenegen._concat([scenegen.surface_scene(2500, seed), scenegen.shells(4, 800, seed + 1)])


def _run(prt, sc, bvh, params, want_vis=False):
    """Transfer (and visibility) of every source with its own workspace;
    returns them with the workspace's flag word."""
    ws = prt.Workspace()
    res = prt.precompute_transfer(sc, bvh, params, want_vis=want_vis, workspace=ws, check=True)
    flags = prt.read_flags(ws.buf)
    if want_vis:
        return res[0].cpu().numpy(), res[1].cpu().numpy(), flags
    return res.cpu().numpy(), None, flags


def _params(prt, S, bands, records, **kw):
    return prt.TransferParams(num_dirs=S, sh_bands=bands, bounces=1, bounce_records=records, **kw)


def test_one_walk_parity_sampled(prt, oracle_mod):
    """One walk against the oracle's full transfer (direct + bounce) and its
    per-ray visibility ranges on 200 sampled sources, and against the
    two-walk blend on every source: the visibility products are formed in
    depth order instead of traversal order, which moves only rays within
    rounding of T_eps and the last bits of the others."""
    from paper_2408_03538_amd import _lib
    S, bands = 64, 4
    scene = as_f32(_small_million_like())
    n = scene["means"].shape[0]
    sc = prt.Scene.from_arrays(scene)
    bvh = prt.build_bvh(sc, check=True)
    # the library's sizing rule leaves room for every record
    R = prt.record_arena_words(sc, bvh, _params(prt, S, bands, 0))
    t1, vis1, f1 = _run(prt, sc, bvh, _params(prt, S, bands, R), want_vis=True)
    assert not f1 & _lib.FLAG_RECORDS_DEFERRED
    src = np.random.default_rng(3).choice(n, 200, replace=False)
    say("one walk: oracle on 200 sources")
    ref = oracle_mod.full_transfer(scene, S, bands, 1, sources=src, want_allow=True)
    err = assert_transfer_parity(t1[src], ref["t"], ref["allow"], what="one-walk transfer")
    assert np.abs(ref["t_ind"]).max() > 1e-2
    vref = oracle_mod.direct_transfer(scene, S, bands, sources=src, want_vis=True, want_vis_bounds=True)
    cos = scene["normals"][src].astype(np.float64) @ oracle_mod.directions(S).T
    rays, wide = assert_ray_vis(vis1[src], vref, cos, oracle_mod.DEFAULT_MARGINS[0], "one-walk visibility")
    t2, vis2, _ = _run(prt, sc, bvh, _params(prt, S, bands, 0), want_vis=True)
    assert np.abs(t1 - t2).max() <= 1e-4
    traced = vis2 != -1.0
    assert np.array_equal(vis1 != -1.0, traced)
    dv = np.abs(vis1 - vis2)[traced]
    # each product rounded differently (a few ulps per factor); a ray at T_eps may be 0 on one side only
    assert (dv <= 1e-5 + 1e-5 * vis2[traced]).mean() > 0.9999
    assert (dv <= 1.01e-4 + 1e-5 * vis2[traced]).all()
    say(f"one walk: max |dt| = {err:.2e} vs oracle; {rays} rays within their range ({wide} near a threshold); "
         f"max |t1 - t2| = {np.abs(t1 - t2).max():.2e} vs two walks")


def _million_recipe(n_surface, per_shell, seed):
    return scenegen._concat([scenegen.surface_scene(n_surface, seed), scenegen.shells(20, per_shell, seed + 1)])


def test_one_walk_million_launch_shape(prt, oracle_mod):
    """The launch shape of the million-splat workload (16 sources per wave,
    64 direction parts, each with sums of its own, S = 512) on an 8,000-splat
    scene of the same recipe: 24 sampled sources against the oracle, every
    source against the two-walk blend."""
    S = 512
    scene = as_f32(_million_recipe(1600, 320, 41))
    n = scene["means"].shape[0]
    sc = prt.Scene.from_arrays(scene)
    bvh = prt.build_bvh(sc, check=True)
    kw = dict(sources_per_wave=16, direction_parts=64)
    t1, _, _ = _run(prt, sc, bvh, _params(prt, S, 4, n * S * 16, **kw))
    t2, _, _ = _run(prt, sc, bvh, _params(prt, S, 4, 0, **kw))
    assert np.abs(t1 - t2).max() <= 1e-4
    src = np.random.default_rng(43).choice(n, 24, replace=False)
    say("one walk, million shape: oracle on 24 sources")
    ref = oracle_mod.full_transfer(scene, S, 4, 1, sources=src, want_allow=True)
    err = assert_transfer_parity(t1[src], ref["t"], ref["allow"], what="one-walk transfer")
    say(f"one walk, million shape: max |dt| = {err:.2e}")


@pytest.mark.parametrize("fraction,spw", [(0.3, 0), (0.0, 0), (0.3, 16), (0.3, 2)])
def test_one_walk_deferred_work(prt, fraction, spw):
    """An arena that holds a fraction of the records (or a single word): the
    items whose blocks do not fit are redone by the two-walk pass
    (PRTGS_FLAG_RECORDS_DEFERRED), and the transfer and visibility equal the
    one walk's with room for every record.  The redone items blend the same
    hits in the same order and sum each round's records in the same order;
    only a ray that needs several traversal rounds could split its hits
    differently between rounds, and none does here.  Sources per wave: the
    default (4 here: 16 lanes per source), 16 (4 lanes) and 2 (32 lanes), so
    the lane sums of a source take trees of different depths."""
    from paper_2408_03538_amd import _lib
    S, bands = 64, 4
    scene = as_f32(_small_million_like(25))
    n = scene["means"].shape[0]
    sc = prt.Scene.from_arrays(scene)
    bvh = prt.build_bvh(sc, check=True)
    kw = dict(sources_per_wave=spw) if spw else {}
    big = _params(prt, S, bands, n * S * 16, **kw)
    st = prt.traversal_stats(sc, bvh, big)
    assert st["rounds"] == st["traced_rays"]
    t1, vis1, f1 = _run(prt, sc, bvh, big, want_vis=True)
    small = _params(prt, S, bands, max(1, int(fraction * st["blended_hits"])), **kw)
    t2, vis2, f2 = _run(prt, sc, bvh, small, want_vis=True)
    assert not f1 & _lib.FLAG_RECORDS_DEFERRED
    assert f2 & _lib.FLAG_RECORDS_DEFERRED
    assert np.array_equal(vis1, vis2)
    assert np.array_equal(t1, t2)


def test_one_walk_many_faint_hits(prt, oracle_mod):
    """A crowded, faint cloud whose rays list more hits than a round's list
    holds (further traversal rounds, each starting at the deepest cut found so
    far) in one walk, with room for every record and with a quarter of it."""
    from paper_2408_03538_amd import _lib
    scene = scenegen.random_cloud(1500, 23)
    scene["means"] *= 0.3
    scene["opacity"] *= 0.04
    scene = as_f32(scene)
    n = scene["means"].shape[0]
    S, bands = 32, 3
    sc = prt.Scene.from_arrays(scene)
    bvh = prt.build_bvh(sc, check=True)
    big = _params(prt, S, bands, n * S * 64)
    st = prt.traversal_stats(sc, bvh, big)
    assert st["rounds"] > st["traced_rays"]
    t1, _, _ = _run(prt, sc, bvh, big)
    t2, _, f2 = _run(prt, sc, bvh, _params(prt, S, bands, st["blended_hits"] // 4))
    assert f2 & _lib.FLAG_RECORDS_DEFERRED
    src = np.random.default_rng(4).choice(n, 60, replace=False)
    say("one walk, faint cloud: oracle on 60 sources")
    ref = oracle_mod.full_transfer(scene, S, bands, 1, sources=src, want_allow=True)
    for t, what in ((t1, "one walk"), (t2, "one walk, deferred items")):
        err = assert_transfer_parity(t[src], ref["t"], ref["allow"], what=what)
        say(f"faint cloud, {what}: max |dt| = {err:.2e}")
    assert np.abs(t1 - t2).max() <= 1e-5 * (1.0 + np.abs(t1).max())


def test_one_walk_source_count_not_whole_blocks(prt, oracle_mod):
    """1,201 sources: the persistent launch does not fill its last block of 4
    waves, and the record sums run one wave per item."""
    scene = as_f32(scenegen._concat([scenegen.surface_scene(901, 31), scenegen.shells(1, 300, 32)]))
    n = scene["means"].shape[0]
    assert n % 4 != 0
    S, bands = 32, 3
    sc = prt.Scene.from_arrays(scene)
    bvh = prt.build_bvh(sc, check=True)
    t1, _, _ = _run(prt, sc, bvh, _params(prt, S, bands, n * S * 16))
    src = np.random.default_rng(5).choice(n, 80, replace=False)
    ref = oracle_mod.full_transfer(scene, S, bands, 1, sources=src, want_allow=True)
    assert_transfer_parity(t1[src], ref["t"], ref["allow"], what="one-walk transfer")
    t2, _, _ = _run(prt, sc, bvh, _params(prt, S, bands, 0))
    assert np.abs(t1 - t2).max() <= 1e-4


def test_one_walk_work_counts(prt):
    """The counted one walk traces the rays the two walks trace and blends
    the same hits; its traversal work replaces both walks'."""
    S, bands = 64, 4
    scene = as_f32(_small_million_like())
    sc = prt.Scene.from_arrays(scene)
    bvh = prt.build_bvh(sc, check=True)
    n = scene["means"].shape[0]
    one = prt.traversal_stats(sc, bvh, _params(prt, S, bands, n * S * 16))
    two = prt.traversal_stats(sc, bvh, _params(prt, S, bands, 0))
    direct = prt.traversal_stats(sc, bvh, prt.TransferParams(num_dirs=S, sh_bands=bands))
    assert one["traced_rays"] == two["traced_rays"] == direct["traced_rays"]
    assert abs(one["blended_hits"] - two["blended_hits"]) <= 1e-3 * two["blended_hits"]
    assert one["box_tests"] < two["box_tests"] + direct["box_tests"]
    say(f"box tests per ray: one walk {one['box_tests'] / one['traced_rays']:.1f}, two walks "
         f"{two['box_tests'] / two['traced_rays']:.1f} + {direct['box_tests'] / direct['traced_rays']:.1f}")


@pytest.mark.parametrize("S,shape", [(64, None), (512, (16, 64))])
def test_one_walk_index_matrix(prt, oracle_mod, S, shape):
    """The paper's index matrix in one walk (bounce_records > 0: the walk
    that picks each ray's hit also yields its visibility; no direct pass, no
    arena).  Against the oracle on every sampled ray it marks unambiguous,
    against the two-walk matrix on every ray (they differ only where a
    visibility product rounds across T_eps), and the transfer with 3 gather
    bounces against the two-walk one wherever the two matrices agree."""
    scene = as_f32(_small_million_like(27) if shape is None else _million_recipe(1600, 320, 41))
    n = scene["means"].shape[0]
    sc = prt.Scene.from_arrays(scene)
    bvh = prt.build_bvh(sc, check=True)
    kw = {} if shape is None else dict(sources_per_wave=shape[0], direction_parts=shape[1])
    p1 = prt.TransferParams(num_dirs=S, sh_bands=4, bounce_mode="index", bounces=3, bounce_records=1, **kw)
    p2 = prt.TransferParams(num_dirs=S, sh_bands=4, bounce_mode="index", bounces=3, **kw)
    idx1 = prt.index_matrix(sc, bvh, p1, check=True).cpu().numpy()
    idx2 = prt.index_matrix(sc, bvh, p2, check=True).cpu().numpy()
    differ = idx1 != idx2
    assert differ.mean() < 1e-3
    src = np.random.default_rng(44).choice(n, 24, replace=False)
    say(f"one-walk index matrix S = {S}: oracle on 24 sources")
    ref_idx, amb = oracle_mod.index_matrix(scene, S, sources=src)
    assert np.array_equal(idx1[src][~amb], ref_idx[~amb])
    t1, _, _ = _run(prt, sc, bvh, p1)
    t2, _, _ = _run(prt, sc, bvh, p2)
    same = ~differ.any(axis=1)
    assert same.mean() > 0.99
    assert np.abs(t1 - t2)[same].max() <= 1e-4
    say(f"one-walk index matrix S = {S}: {differ.sum()} of {differ.size} entries differ from two walks; "
         f"max |dt| where they agree {np.abs(t1 - t2)[same].max():.2e}")
