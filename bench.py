#!/usr/bin/env python3
"""Benchmark of the PRTGS transfer precompute on one MI355X.

A step is one pass of the hot path over the million-splat workload (a unit
sphere on a 4x4 plane with 200,000 surface splats plus 20 ellipsoid shells of
40,000 splats each: 1,000,000 Gaussians, S = 512 directions, 16 SH
coefficients, RGB transfer with one interreflection bounce): BVH build, the
transfer (one walk per ray gives each ray's visibility and blends its hits;
the blended hits' records wait in a workspace arena until every direct
transfer exists) and relighting under one light.  `value` is nominal rays
(N * S) per second of the whole step, inputs already resident on the GPU.
The same JSON line carries the breakdown, the roofline of the transfer call
(the step's dominant work), the same transfer as two walks (direct pass, then
bounce walk) for comparison, and the secondary measurements: the 100k-splat
surface workload (direct transfer only), the paper's index-matrix bounce, a
relit 1080p frame, glossy matrices, relighting 3M splats x 64 lights with FP32
vs BF16 / F16 storage, forward vs forward + backward on 200k splats, and the
CPU oracle baseline.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-extras] [--no-cpu]
    python bench.py --copy-mib M      # plain device copy (counter calibration)
    python bench.py --million-only    # the headline step alone (for profiling; --two-walks: as two walks)
    python bench.py --index-only      # the million-splat index matrix (--two-walks: direct pass + index walk)
    python bench.py --frame-only      # relit 1080p frames of the million-splat scene
    python bench.py --relight-only    # the 3M x 64 relight alone
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# MI355X published peaks
PEAK_HBM_GBS = 8000.0
PEAK_FP32_TFLOPS = 157.3
PEAK_BF16_TFLOPS = 2500.0

# Algorithmic cost of single-ray traversal work: a child-box test reads one
# FP32 box plus a reference (32 B) and costs ~15 flops; a Gaussian test reads
# the minimal parameterisation mu, q, 1/s, o (44 B) and costs ~70 flops.  A
# blended hit of the bounce reads the hit splat's direct transfer and albedo
# (16 x 4 + 12 = 76 B at 16 coefficients).
BYTES_PER_BOX_TEST = 32
BYTES_PER_PRIM_TEST = 44
FLOPS_PER_BOX_TEST = 15
FLOPS_PER_PRIM_TEST = 70

# Counter measurements (rocprofv3 --pmc, one run per counter set; FETCH_SIZE
# scaled by 2.0 and WRITE_SIZE by 1.0, the factors a 1 GiB copy reads), valid
# only for the kernel sources they were measured on (hash below), else null.
# direct: traversal + projection of the 100k surface workload
# (profiles/direct_kernel_surface100k_hbm_counters.md,
# profiles/direct_kernel_surface100k_sq_counters.md); one walk: every kernel of
# the million-splat one-walk transfer call (fused_kernel<16>, accumulate_kernel<16>,
# project_kernel<16>, add_parts_kernel and the deferred-item pass), summed
# (profiles/one_walk_million_counters.md).
MEASURED = {
    "direct_surface100k": {"sources_sha256_16": "0acb27b42cfd1486", "bytes_per_launch": 7.2786e9,
                           "valu_instructions_per_launch": 1.0735e10},
    "one_walk_million": {"sources_sha256_16": "0acb27b42cfd1486", "bytes_per_launch": 5.2305e12,
                         "valu_instructions_per_launch": 1.3882e12},
}
KERNEL_SOURCES = ["paper_2408_03538_amd/csrc/transfer.hip", "paper_2408_03538_amd/csrc/trace.hpp",
                  "paper_2408_03538_amd/csrc/common.hpp", "paper_2408_03538_amd/csrc/capi.hip"]   # capi: work split
# VALU issue rate: 1024 SIMDs at 2.4 GHz, one wave64 FP32 instruction per 2
# cycles (the rate behind the 157.3 TFLOP/s FP32 peak)
VALU_WAVE_INSTR_PER_S = 1024 * 2.4e9 / 2


def kernel_sources_hash():
    import hashlib
    m = hashlib.sha256()
    for p in KERNEL_SOURCES:
        with open(os.path.join(ROOT, p), "rb") as f:
            m.update(f.read())
    return m.hexdigest()[:16]


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-extras", action="store_true", help="skip the secondary measurements")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-seconds", type=float, default=20.0, help="CPU oracle baseline budget")
    ap.add_argument("--copy-mib", type=int, default=0, help="only run a plain device copy of this size")
    ap.add_argument("--million-only", action="store_true",
                    help="only the headline steps, with no statistics pass (profiling runs)")
    ap.add_argument("--frame-only", action="store_true",
                    help="only time relit 1080p frames of the million-splat scene (synthetic transfers)")
    ap.add_argument("--relight-only", action="store_true",
                    help="only time the 3M x 64 relight in FP32, BF16 and F16 storage")
    ap.add_argument("--surface-only", action="store_true",
                    help="only the 100k surface workload (direct transfer; profiling runs)")
    ap.add_argument("--two-walks", action="store_true",
                    help="with --index-only or --million-only: the direct pass and the walk as two walks")
    ap.add_argument("--index-only", action="store_true",
                    help="only the million-splat index matrix (the paper's bounce; profiling runs)")
    return ap.parse_args()


class Timer:
    """HIP events on the current stream (the library launches there)."""

    def __init__(self, torch):
        self.torch = torch
        self.marks = {}

    def start(self, name):
        ev = self.torch.cuda.Event(enable_timing=True)
        ev.record()
        self.marks.setdefault(name, []).append([ev, None])

    def stop(self, name):
        ev = self.torch.cuda.Event(enable_timing=True)
        ev.record()
        self.marks[name][-1][1] = ev

    def ms(self, name):
        return [a.elapsed_time(b) for a, b in self.marks.get(name, [])]


def workload_setup(prt, torch, scenegen, name):
    import numpy as np
    w = scenegen.workload(name)
    arr = {k: np.asarray(v, dtype=np.float32) for k, v in w["scene"].items()}
    sc = prt.Scene.from_arrays(arr)
    params = prt.TransferParams(num_dirs=w["num_dirs"], sh_bands=w["bands"], bounces=w["bounces"])
    light = torch.tensor(w["light"], dtype=torch.float32, device="cuda")
    return arr, sc, params, light


def copy_only(mib):
    """A plain device-to-device copy of `mib` MiB (read + write), for scaling
    the HBM byte counters."""
    import torch
    x = torch.ones(mib * (1 << 20) // 4, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    for _ in range(3):
        y.copy_(x)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read": x.numel() * 4, "copy_bytes_written": y.numel() * 4}))


def measured(key):
    """A counter measurement, if it was taken on the current kernel sources."""
    m = MEASURED[key]
    return m if m["sources_sha256_16"] == kernel_sources_hash() else None


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); this library has no multi-GPU path.",
              file=sys.stderr)
        sys.exit(2)
    if args.copy_mib:
        copy_only(args.copy_mib)
        return
    import numpy as np
    import torch

    import paper_2408_03538_amd as prt
    import scenegen

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    if args.frame_only:
        frame_only(prt, torch, scenegen, np)
        return
    if args.relight_only:
        print(json.dumps({"relight_3m": bench_relight(prt, torch, scenegen, np, args.steps)}), flush=True)
        return
    if args.surface_only:
        print(json.dumps({"surface100k_direct": bench_surface100k(prt, torch, scenegen, np, args.steps,
                                                                   args.warmup)}), flush=True)
        return
    log("generating the million-splat workload")
    arr, sc, params, light = workload_setup(prt, torch, scenegen, "million")
    n, S = sc.n, params.num_dirs
    one_walk_stats = None
    if args.index_only:
        bvh = prt.build_bvh(sc)
        p_idx = prt.TransferParams(num_dirs=S, sh_bands=params.sh_bands, bounce_mode="index", bounces=1,
                                   bounce_records=0 if args.two_walks else 1)
        ws = prt.Workspace()
        for _ in range(max(1, args.steps)):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record()
            idx = prt.index_matrix(sc, bvh, p_idx, workspace=ws)
            b.record()
            torch.cuda.synchronize()
            log(f"index matrix ({'direct pass + index walk' if args.two_walks else 'one walk'}): "
                f"{a.elapsed_time(b):.1f} ms")
            del idx
        return
    # the blend in one walk per ray: its records' arena sized from a counted walk
    if args.two_walks:
        if not args.million_only:
            raise SystemExit("--two-walks times the million-splat step only with --million-only or --index-only")
        params.bounce_records = 0
    else:
        one_walk_stats, params.bounce_records = record_arena(prt, torch, sc, params)
        log(f"record arena: {params.bounce_records / 1e9:.2f}e9 words ({8 * params.bounce_records / 1e9:.1f} GB)")
    res = time_steps(prt, torch, np, sc, params, light, args.steps, args.warmup)
    ms_step = res["ms_step"]
    log(f"step {ms_step:.1f} ms: build {res['build']:.2f} ms, transfer {res['transfer']:.1f} ms, "
        f"relight {res['relight']:.4f} ms")
    if args.million_only:
        print(json.dumps({"ms_per_step": ms_step, "steps": args.steps}), flush=True)
        return
    result = {
        "metric": "transfer precompute Grays/s + relit splats/s; BF16 vs FP32, fwd+bwd vs fwd",
        "value": round(n * S / (ms_step * 1e-3) / 1e9, 5),
        "unit": "Grays/s (nominal N*S rays per second of the whole step)",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "million: unit sphere on a 4x4 plane (200,000 splats) + 20 ellipsoid shells x 40,000 "
                               "splats, N=1,000,000, S=512, 16 SH coeffs x RGB, direct + 1 bounce (one walk per ray)",
                   "n_splats": n, "num_dirs": S, "sh_coeffs": params.K, "channels": params.channels,
                   "bounces": params.bounces},
    }
    result.update(million_breakdown(prt, torch, np, sc, params, res, args.steps, one_walk_stats))
    result["relit_splats_per_s"] = round(n / (res["relight"] * 1e-3), 1)
    transfer_out, bvh = res["transfer_out"], res["bvh"]
    res.clear()
    torch.cuda.empty_cache()
    if not args.no_extras:
        result["million_extras"] = bench_million_extras(prt, torch, scenegen, np, sc, bvh, params, light,
                                                        transfer_out)
        del transfer_out, bvh
        torch.cuda.empty_cache()
        result["surface100k_direct"] = bench_surface100k(prt, torch, scenegen, np, 20, 3)
        result["relight_3m"] = bench_relight(prt, torch, scenegen, np, 20)
        result["backward_200k"] = bench_backward(prt, torch, scenegen, np, 20)
        result["glossy_100k"] = bench_glossy(prt, torch, scenegen, np, 20)
    if not args.no_cpu:
        result["cpu_baseline"] = cpu_baseline(arr, params, args.cpu_seconds)
    print(json.dumps(result), flush=True)


def roofline_of(kernel, stats, ms, bytes_per_unit, extra_unit_bytes=None, counters=None):
    """Roofline of one traversal kernel: algorithmic bytes of the single-ray
    work it performs per traced ray, times the rays of one launch, over the
    measured launch time, against the HBM peak (the HBM-roofline-implied ray
    throughput); beside it the DRAM traffic the counters measured and the
    share of the VALU issue rate the kernel used."""
    traced = stats["traced_rays"]
    achieved = traced * bytes_per_unit / (ms * 1e-3) / 1e9
    out = {
        "kernel": kernel,
        "bound": "hbm",
        "achieved": round(achieved, 1),
        "peak": PEAK_HBM_GBS,
        "unit": "GB/s",
        "frac": round(achieved / PEAK_HBM_GBS, 4),
        "traffic": counters["bytes_per_launch"] if counters else None,
        "traffic_unit": "bytes per launch (FETCH_SIZE x 2.0 + WRITE_SIZE, copy-calibrated)",
        "what_frac_means": "traced rays/s over the HBM-roofline-implied ray rate 8 TB/s / algorithmic bytes per ray",
        "units_per_launch": traced,
        "unit_of_work": "traced ray",
        "algorithmic_bytes_per_unit": round(bytes_per_unit, 1),
        "ms_per_launch": round(ms, 3),
    }
    if extra_unit_bytes:
        out["algorithmic_bytes_terms"] = extra_unit_bytes
    if counters and counters.get("bytes_per_launch"):
        out["measured_dram_GBps"] = round(counters["bytes_per_launch"] / (ms * 1e-3) / 1e9, 1)
        out["measured_dram_frac"] = round(counters["bytes_per_launch"] / (ms * 1e-3) / 1e9 / PEAK_HBM_GBS, 4)
    if counters and counters.get("valu_instructions_per_launch"):
        out["valu_issue_frac"] = round(counters["valu_instructions_per_launch"] / (VALU_WAVE_INSTR_PER_S * ms * 1e-3), 3)
    return out


def record_arena(prt, torch, sc, params):
    """Work counts of the one walk (a counted run, outside any timed region)
    and the record arena the library's sizing rule gives for them (one record
    per blended hit, a block header per work item, direction batch and round,
    5% to spare)."""
    bvh = prt.build_bvh(sc)
    probe = prt.TransferParams(**{**params.__dict__, "bounce_records": 1})
    st = prt.traversal_stats(sc, bvh, probe)
    words = prt.record_arena_words(sc, bvh, params, stats=st)
    del bvh
    torch.cuda.empty_cache()
    return st, words


def million_breakdown(prt, torch, np, sc, params, res, steps, sb):
    """The headline transfer call (the blend in one walk per ray) beside the
    direct pass alone and the two-walk blend (HIP events on the library's
    stream), the single-ray work of each walk, and the roofline of the
    one-walk call, which is the step's dominant work."""
    def timed(p, channels):
        out = torch.zeros((sc.n, channels, p.K), dtype=torch.float32, device="cuda")
        ws = prt.Workspace()
        prt.precompute_transfer(sc, res["bvh"], p, out=out, workspace=ws)
        times = []
        for _ in range(max(3, min(steps, 5))):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record()
            prt.precompute_transfer(sc, res["bvh"], p, out=out, workspace=ws)
            b.record()
            torch.cuda.synchronize()
            times.append(a.elapsed_time(b))
        prt.check_flags(ws.buf, "transfer")
        del out, ws
        torch.cuda.empty_cache()
        return float(np.median(times))

    direct = prt.TransferParams(num_dirs=params.num_dirs, sh_bands=params.sh_bands, bounces=0)
    two = prt.TransferParams(**{**params.__dict__, "bounce_records": 0})
    t_direct = timed(direct, 1)
    t_two = timed(two, 3)
    t_transfer = float(np.median(res["transfer_all"]))
    sd = prt.traversal_stats(sc, res["bvh"], direct)
    s2 = prt.traversal_stats(sc, res["bvh"], two)
    torch.cuda.empty_cache()
    K = params.K
    td = sd["traced_rays"]
    d_box, d_prim = sd["box_tests"] / td, sd["prim_tests"] / td
    tb = sb["traced_rays"]
    b_box, b_prim = sb["box_tests"] / tb, sb["prim_tests"] / tb
    blended, listed, rounds = sb["blended_hits"] / tb, sb["listed_hits"] / tb, sb["rounds"] / tb
    hit_bytes = 4 * K + 12
    # direct: traversal + the ray's weight written and read back by the projection
    b_direct = BYTES_PER_BOX_TEST * d_box + BYTES_PER_PRIM_TEST * d_prim
    # one walk: its traversal, the hits blended (their direct transfer and
    # albedo read), the ray's weight written for and read by the projection
    b_one = BYTES_PER_BOX_TEST * b_box + BYTES_PER_PRIM_TEST * b_prim + hit_bytes * blended + 8
    log(f"million: one-walk call {t_transfer:.0f} ms ({b_box:.0f} box / {b_prim:.0f} Gaussian tests per ray, "
        f"{blended:.1f} blended / {listed:.1f} listed hits, {rounds:.3f} rounds); two walks {t_two:.0f} ms, "
        f"direct pass alone {t_direct:.0f} ms ({d_box:.0f} / {d_prim:.0f} per ray)")
    roof = roofline_of("fused_kernel<16> + project_kernel + accumulate_kernel: the whole one-walk transfer call "
                       "(visibility, projection, bounce; the walk is ~92% of it, the record sums ~8%), "
                       "timed around the call",
                       sb, t_transfer, b_one,
                       {"box_tests": round(b_box, 2), "prim_tests": round(b_prim, 2),
                        "blended_hits": round(blended, 2), "bytes_per_blended_hit": hit_bytes,
                        "listed_hits": round(listed, 2), "rounds": round(rounds, 4), "ray_weight_bytes": 8},
                       measured("one_walk_million"))
    roof["packet_node_visits_per_64_rays"] = round(sb["wave_node_visits"] / (tb / 64), 1)
    roof["packet_gaussian_visits_per_64_rays"] = round(sb["wave_prim_visits"] / (tb / 64), 1)
    direct_roof = roofline_of("direct_kernel + project_kernel (visibility traversal, then SH projection; "
                              "the direct transfer alone, not part of the step)", sd,
                              t_direct, b_direct, {"box_tests": round(d_box, 2), "prim_tests": round(d_prim, 2)})
    direct_roof["packet_node_visits_per_64_rays"] = round(sd["wave_node_visits"] / (td / 64), 1)
    direct_roof["packet_gaussian_visits_per_64_rays"] = round(sd["wave_prim_visits"] / (td / 64), 1)
    t2 = s2["traced_rays"]
    return {
        "breakdown_ms": {"build_bvh": round(res["build"], 3), "transfer_call": round(t_transfer, 2),
                         "relight": round(res["relight"], 4)},
        "traced_rays": td,
        "record_arena_words": params.bounce_records,
        "grays_per_s_without_build": round(sc.n * params.num_dirs / ((res["ms_step"] - res["build"]) * 1e-3) / 1e9,
                                           5),
        "roofline": roof,
        "two_walks": {"what": "the same transfer with the direct pass and the bounce walk as two walks "
                              "(bounce_records = 0), not part of the step",
                      "transfer_call_ms": round(t_two, 2), "direct_pass_ms": round(t_direct, 2),
                      "bounce_walk_ms": round(t_two - t_direct, 2),
                      "bounce_walk_box_tests_per_ray": round(s2["box_tests"] / t2, 2),
                      "bounce_walk_prim_tests_per_ray": round(s2["prim_tests"] / t2, 2)},
        "direct_traced_grays_per_s": round(td / (t_direct * 1e-3) / 1e9, 4),
        "direct_roofline": direct_roof,
    }


def time_steps(prt, torch, np, sc, params, light, steps, warmup):
    """Whole-step timing (wall clock around synchronised steps) plus HIP
    events around each library call, on the stream the library launches on."""
    ws_build, ws_tr = prt.Workspace(), prt.Workspace()
    transfer = torch.zeros((sc.n, params.channels, params.K), dtype=torch.float32, device="cuda")
    colour = torch.empty((sc.n, light.shape[0], 3), dtype=torch.float32, device="cuda")
    holder = {}
    timer = Timer(torch)

    def step(record):
        if record:
            timer.start("build")
        holder["bvh"] = prt.build_bvh(sc, workspace=ws_build, out=holder.get("bvh"))
        if record:
            timer.stop("build")
            timer.start("transfer")
        prt.precompute_transfer(sc, holder["bvh"], params, out=transfer, workspace=ws_tr)
        if record:
            timer.stop("transfer")
            timer.start("relight")
        prt.relight(transfer, light, out=colour)
        if record:
            timer.stop("relight")

    for _ in range(warmup):
        step(False)
    torch.cuda.synchronize()
    timer.marks.clear()
    t0 = time.perf_counter()
    for _ in range(steps):
        step(True)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    prt.check_flags(ws_tr.buf, "transfer")
    return {"ms_step": wall * 1e3 / steps, "build": float(np.mean(timer.ms("build"))),
            "transfer": float(np.mean(timer.ms("transfer"))), "relight": float(np.mean(timer.ms("relight"))),
            "transfer_all": timer.ms("transfer"), "bvh": holder["bvh"], "transfer_out": transfer}


def bench_surface100k(prt, torch, scenegen, np, steps, warmup):
    """The 100k-splat surface workload (S = 256, 16 coefficients, direct
    transfer only): build + transfer + relight per step, and the roofline of
    its traversal kernel."""
    log("surface100k: direct transfer")
    arr, sc, params, light = workload_setup(prt, torch, scenegen, "surface100k")
    res = time_steps(prt, torch, np, sc, params, light, steps, warmup)
    stats = prt.traversal_stats(sc, res["bvh"], params)
    traced = stats["traced_rays"]
    n_box, n_prim = stats["box_tests"] / traced, stats["prim_tests"] / traced
    b_ray = BYTES_PER_BOX_TEST * n_box + BYTES_PER_PRIM_TEST * n_prim
    f_ray = FLOPS_PER_BOX_TEST * n_box + FLOPS_PER_PRIM_TEST * n_prim
    t_kernel = float(np.median(res["transfer_all"]))
    roof = roofline_of("direct_kernel + project_kernel (visibility traversal, then SH projection; one call)", stats,
                       t_kernel, b_ray, {"box_tests": round(n_box, 2), "prim_tests": round(n_prim, 2)},
                       measured("direct_surface100k"))
    roof["alu_view"] = {"algorithmic_flops_per_ray": round(f_ray, 1),
                        "achieved_TFLOPs": round(traced / (t_kernel * 1e-3) * f_ray / 1e12, 3),
                        "peak_TFLOPs": PEAK_FP32_TFLOPS,
                        "packet_node_visits_per_64_rays": round(stats["wave_node_visits"] / (traced / 64), 1),
                        "packet_gaussian_visits_per_64_rays": round(stats["wave_prim_visits"] / (traced / 64), 1)}
    log(f"surface100k: step {res['ms_step']:.2f} ms, transfer {t_kernel:.2f} ms, frac {roof['frac']}")
    out = {"workload": "surface100k: unit sphere on a 4x4 plane, N=100,000, S=256, 16 SH coeffs, direct",
           "steps": steps, "ms_per_step": round(res["ms_step"], 3),
           "nominal_grays_per_s": round(sc.n * params.num_dirs / (res["ms_step"] * 1e-3) / 1e9, 4),
           "traced_grays_per_s": round(traced / (t_kernel * 1e-3) / 1e9, 4),
           "breakdown_ms": {"build_bvh": round(res["build"], 4), "transfer": round(t_kernel, 4),
                            "relight": round(res["relight"], 5)},
           "roofline": roof}
    del res
    torch.cuda.empty_cache()
    return out


def bench_million_extras(prt, torch, scenegen, np, sc, bvh, params, light, transfer_out):
    """On the million-splat scene: the paper's own bounce (index matrix, then
    3 bounces by gathers), a relit 1080p frame, glossy matrices at S = 512."""
    out_d = {}
    # one walk per ray (the index matrix with the visibility), and the two-walk form beside it
    p_idx = prt.TransferParams(num_dirs=params.num_dirs, sh_bands=params.sh_bands, bounce_mode="index", bounces=3,
                               bounce_records=1)
    p_two = prt.TransferParams(**{**p_idx.__dict__, "bounce_records": 0})
    out3 = torch.zeros((sc.n, 3, params.K), dtype=torch.float32, device="cuda")
    ws3 = prt.Workspace()
    prt.precompute_transfer(sc, bvh, p_idx, out=out3, workspace=ws3)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(6)]
    ev[0].record()
    prt.precompute_transfer(sc, bvh, p_idx, out=out3, workspace=ws3)
    ev[1].record()
    idx = prt.index_matrix(sc, bvh, p_idx, workspace=ws3)
    ev[2].record()
    prev = prt.self_transfer(sc, p_idx, idx, out3)
    ev[3].record()
    prt.index_matrix(sc, bvh, p_two, workspace=ws3)
    ev[4].record()
    prt.precompute_transfer(sc, bvh, p_two, out=out3, workspace=ws3)
    ev[5].record()
    torch.cuda.synchronize()
    t_all, t_idx, t_gather = ev[0].elapsed_time(ev[1]), ev[1].elapsed_time(ev[2]), ev[2].elapsed_time(ev[3])
    out_d["index_bounces"] = {
        "workload": "million, the paper's bounce: index matrix (one walk per ray, with the visibility) + 3 bounces "
                    "by gathers",
        "ms_index_walk_plus_3_bounces": round(t_all, 2), "ms_index_matrix": round(t_idx, 2),
        "ms_per_gather_bounce": round(t_gather, 3),
        "two_walks": {"ms_direct_plus_index_matrix": round(ev[3].elapsed_time(ev[4]), 2),
                      "ms_direct_plus_3_bounces": round(ev[4].elapsed_time(ev[5]), 2)}}
    # algorithmic bytes of one gather bounce: the index rows, normals and
    # outputs, plus one RGB transfer row and albedo per indexed ray
    nidx = int((idx >= 0).sum().item())
    g_bytes = sc.n * (4 * params.num_dirs + 12 + 12 * params.K) + nidx * (12 * params.K + 12)
    out_d["index_bounces"]["indexed_rays"] = nidx
    out_d["index_bounces"]["gather_GBps"] = round(g_bytes / (t_gather * 1e-3) / 1e9, 1)
    log(f"million index mode: one walk + 3 bounces {t_all:.0f} ms (two walks "
        f"{ev[4].elapsed_time(ev[5]):.0f} ms), one gather bounce {t_gather:.2f} ms")
    del out3, ws3, idx, prev
    torch.cuda.empty_cache()
    out_d["frame_1080p"] = bench_frame(prt, torch, np, sc, transfer_out, light)
    torch.cuda.empty_cache()
    out_d["glossy_1m"] = bench_glossy_million(prt, torch, scenegen, np, sc, bvh, params)
    torch.cuda.empty_cache()
    return out_d


def bench_glossy_million(prt, torch, scenegen, np, sc, bvh, params):
    """Glossy matrices of the million-splat scene at S = 512 from its direct
    pass's visibilities (materials U[0.1, 1] x U[0, 1])."""
    rough, metal = scenegen.materials(sc.n, scenegen.SEED_SCENE + 6)
    r = torch.tensor(rough, dtype=torch.float32, device="cuda")
    m = torch.tensor(metal, dtype=torch.float32, device="cuda")
    pd = prt.TransferParams(num_dirs=params.num_dirs, sh_bands=params.sh_bands)
    _, vis = prt.precompute_transfer(sc, bvh, pd, want_vis=True)
    ws = prt.Workspace()
    M = prt.glossy_transfer(sc, pd, vis, r, m, workspace=ws)
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    prt.glossy_transfer(sc, pd, vis, r, m, out=M, workspace=ws)
    b.record()
    torch.cuda.synchronize()
    ms = a.elapsed_time(b)
    log(f"glossy 1M x 512: {ms:.1f} ms")
    del M, vis
    return {"workload": "million-splat scene, S=512, 3 x 16 x 16 matrices, roughness U[0.1,1], metallic U[0,1]",
            "ms_glossy_matrices": round(ms, 2), "matrices_per_s": round(sc.n / (ms * 1e-3), 1)}


def frame_only(prt, torch, scenegen, np):
    """Frames of the million-splat scene with synthetic RGB transfers (the
    precompute's output has the same shape; the frame does not depend on
    its values beyond the colours)."""
    log("million-splat scene, synthetic transfers")
    w = scenegen.workload("million")
    sc = prt.Scene.from_arrays({k: np.asarray(v, dtype=np.float32) for k, v in w["scene"].items()})
    t = torch.tensor(scenegen.synthetic_transfers(sc.n, w["bands"], 3, scenegen.SEED_SCENE + 2),
                     dtype=torch.float32, device="cuda")
    light = torch.tensor(w["light"], dtype=torch.float32, device="cuda")
    print(json.dumps({"frame_1080p": bench_frame(prt, torch, np, sc, t, light)}), flush=True)


def bench_frame(prt, torch, np, sc, transfer, light, frames=20):
    """A relit frame at 1920 x 1080: relight every splat under one light
    environment, then splat the colours (projection, tile binning, sort,
    front-to-back blending).  Wall clock per frame includes the one host
    synchronisation that reads the number of (Gaussian, tile) pairs."""
    cam = prt.camera(prt.look_at((0.0, -5.5, 3.0), (0.0, 0.0, 0.8)), 1920, 1080, 50.0, 0.05)
    light1 = light[:1].contiguous()
    colours = torch.empty((sc.n, 1, 3), dtype=torch.float32, device="cuda")
    ws = prt.Workspace()

    def frame():
        prt.relight(transfer, light1, out=colours)
        return prt.splat_render(sc, colours[:, 0], cam, workspace=ws)

    prt.relight(transfer, light1, out=colours)
    _, T, inst = prt.splat_render(sc, colours[:, 0], cam, workspace=ws, want_T=True)
    covered = float((T < 0.5).float().mean().item())
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(frames):
        img, _, _ = frame()
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / frames
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    prt.relight(transfer, light1, out=colours)
    b.record()
    torch.cuda.synchronize()
    log(f"1080p frame: {ms:.2f} ms ({1e3 / ms:.0f} fps), {inst} (Gaussian, tile) pairs")
    return {"workload": "million-splat scene relit under one light, splatted at 1920x1080",
            "ms_per_frame": round(ms, 3), "fps": round(1e3 / ms, 1), "ms_relight": round(a.elapsed_time(b), 4),
            "gaussian_tile_pairs": inst, "covered_pixel_frac_T_below_half": round(covered, 3)}


def measured_copy_GBps(torch, mib=1024, reps=10):
    """Read + write bandwidth of a plain 1 GiB device copy, for scale."""
    x = torch.ones(mib * (1 << 20) // 4, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    y.copy_(x)
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        y.copy_(x)
    b.record()
    torch.cuda.synchronize()
    ms = a.elapsed_time(b) / reps
    del x, y
    return round(2 * mib * (1 << 20) / (ms * 1e-3) / 1e9, 1)


def bench_relight(prt, torch, scenegen, np, steps):
    """3,000,000 RGB transfers x 64 lights: FP32, BF16 and F16 storage."""
    import oracle
    log("relight: 3M x 64 lights")
    w = scenegen.workload("relight3m")
    T = torch.tensor(w["transfer"], dtype=torch.float32, device="cuda")
    L = torch.tensor(w["light"], dtype=torch.float32, device="cuda")
    n, B = T.shape[0], L.shape[0]
    T16 = {"bf16": prt.pack(T, "bf16"), "f16": prt.pack(T, "f16")}
    out32 = torch.empty((n, B, 3), dtype=torch.float32, device="cuda")
    out16 = torch.empty((n, B, 3), dtype=torch.float16, device="cuda")
    modes = {"f32->f32": (T, out32, "f32"), "bf16->f16": (T16["bf16"], out16, "f16"),
             "f16->f16": (T16["f16"], out16, "f16"), "bf16->f32": (T16["bf16"], out32, "f32")}
    rows = np.random.default_rng(0).choice(n, 20000, replace=False)
    ref = oracle.relight(np.asarray(w["transfer"], np.float32).astype(np.float64)[rows],
                         np.asarray(w["light"], np.float32).astype(np.float64))
    scale = np.einsum("nck,bck->nbc", np.abs(np.asarray(w["transfer"], np.float32)[rows].astype(np.float64)),
                      np.abs(np.asarray(w["light"], np.float32).astype(np.float64)))
    res = {}
    for name, (t, out, odt) in modes.items():
        prt.relight(t, L, out_dtype=odt, out=out)
        torch.cuda.synchronize()
        # launches back to back between two events: the per-launch host
        # overhead (comparable to a 0.4 ms kernel) stays off the clock
        reps = 10
        evs = []
        for _ in range(max(5, steps)):
            a = torch.cuda.Event(enable_timing=True)
            b = torch.cuda.Event(enable_timing=True)
            a.record()
            for _ in range(reps):
                prt.relight(t, L, out_dtype=odt, out=out)
            b.record()
            evs.append((a, b))
        torch.cuda.synchronize()
        ms = float(np.median([a.elapsed_time(b) for a, b in evs])) / reps
        in_bytes = t.numel() * t.element_size()
        out_bytes = out.numel() * out.element_size()
        got = out[torch.tensor(rows, device="cuda")].float().cpu().numpy().astype(np.float64)
        err = np.abs(got - ref)
        res[name] = {"ms": round(ms, 4), "pairs_per_s": round(n * B / (ms * 1e-3), 1),
                     "hbm_GBps": round((in_bytes + out_bytes) / (ms * 1e-3) / 1e9, 1),
                     "hbm_frac": round((in_bytes + out_bytes) / (ms * 1e-3) / 1e9 / PEAK_HBM_GBS, 4),
                     "max_rel_err": float((err / scale).max()), "mean_rel_err": float((err / scale).mean())}
        # the dot products themselves (2 K flops per splat, light and channel)
        # against the dense peak of the unit that runs them
        flops = n * B * 3 * 2 * T.shape[2]
        peak = PEAK_FP32_TFLOPS if odt == "f32" and t.dtype == torch.float32 else PEAK_BF16_TFLOPS
        res[name]["algorithmic_TFLOPs"] = round(flops / (ms * 1e-3) / 1e12, 2)
        res[name]["compute_frac"] = round(flops / (ms * 1e-3) / 1e12 / peak, 4)
        log(f"relight {name}: {ms:.3f} ms, {res[name]['hbm_GBps']} GB/s, max err {res[name]['max_rel_err']:.2e}")
    res["speedup_bf16_f16out_vs_f32"] = round(res["f32->f32"]["ms"] / res["bf16->f16"]["ms"], 3)
    res["speedup_bf16_f32out_vs_f32"] = round(res["f32->f32"]["ms"] / res["bf16->f32"]["ms"], 3)
    res["workload"] = "3,000,000 splats x 16 coeffs x RGB, 64 light environments"
    res["copy_GBps"] = measured_copy_GBps(torch)
    del T, T16, out32, out16
    torch.cuda.empty_cache()
    return res


def bench_glossy(prt, torch, scenegen, np, steps):
    """Glossy transfer matrices of the 100k surface scene (S = 256, 3 x 16 x 16
    per splat) from the direct pass's visibilities, and the per-frame view +
    relight of those matrices."""
    log("glossy matrices: 100k x 256")
    w = scenegen.workload("glossy100k")
    arr = {k: np.asarray(v, dtype=np.float32) for k, v in w["scene"].items()}
    sc = prt.Scene.from_arrays(arr)
    params = prt.TransferParams(num_dirs=w["num_dirs"], sh_bands=w["bands"])
    rough = torch.tensor(w["roughness"], dtype=torch.float32, device="cuda")
    metal = torch.tensor(w["metallic"], dtype=torch.float32, device="cuda")
    light = torch.tensor(w["light"], dtype=torch.float32, device="cuda")
    bvh = prt.build_bvh(sc)
    _, vis = prt.precompute_transfer(sc, bvh, params, want_vis=True)
    ws = prt.Workspace()
    M = prt.glossy_transfer(sc, params, vis, rough, metal, workspace=ws)
    torch.cuda.synchronize()
    reps = max(3, steps // 4)
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        prt.glossy_transfer(sc, params, vis, rough, metal, out=M, workspace=ws)
    b.record()
    torch.cuda.synchronize()
    ms = a.elapsed_time(b) / reps
    # the upper hemisphere of each normal, as the kernel lists it
    dirs = prt.direction_table(params.num_dirs, 0, params.sh_bands)[2]
    H = ((sc.normals @ dirs.T) > 0).sum(1).double()
    Hp = torch.ceil(H / 16) * 16
    # MFMA work: (Hp / 4) x (Hp / 16) 16x16x4 steps for U (two matrices), 4 per
    # output block for the contraction over p; 2048 flops per 16x16x4
    mfma_flops = float((2 * (Hp / 4) * (Hp / 16) * 2048 + 2 * 4 * (Hp / 16) * 2048).sum().item())
    pairs = float((H * H).sum().item())
    eye = (0.0, -5.5, 3.0)
    z = prt.glossy_view(M, sc.means, eye)
    col = prt.relight(z, light)
    torch.cuda.synchronize()
    c, d = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    c.record()
    for _ in range(10):
        prt.glossy_view(M, sc.means, eye, out=z)
        prt.relight(z, light, out=col)
    d.record()
    torch.cuda.synchronize()
    ms_frame = c.elapsed_time(d) / 10
    log(f"glossy: {ms:.2f} ms per 100k matrices, view + relight {ms_frame:.3f} ms")
    out = {"workload": "glossy100k: surface scene N=100,000, S=256, 3 x 16 x 16 matrices, roughness U[0.1,1], "
                       "metallic U[0,1]",
           "ms_glossy_matrices": round(ms, 3), "matrices_per_s": round(sc.n / (ms * 1e-3), 1),
           "brdf_pairs_per_s": round(pairs / (ms * 1e-3), 1),
           "mfma_TFLOPs": round(mfma_flops / (ms * 1e-3) / 1e12, 2), "mfma_peak_fp32_TFLOPs": PEAK_FP32_TFLOPS,
           "ms_view_plus_relight": round(ms_frame, 4),
           "view_bytes_GBps": round(M.numel() * 4 / (ms_frame * 1e-3) / 1e9, 1)}
    del M, vis, bvh
    torch.cuda.empty_cache()
    return out


def bench_backward(prt, torch, scenegen, np, steps):
    """200k surface splats, S=256, 16 coeffs: forward vs forward + backward."""
    log("backward: 200k splats, S=256")
    w = scenegen.workload("grad200k")
    arr = {k: np.asarray(v, dtype=np.float32) for k, v in w["scene"].items()}
    keys = ("means", "quats", "log_scales", "opacity", "normals")
    ten = {k: torch.tensor(arr[k], device="cuda", requires_grad=True) for k in keys}
    L = torch.tensor(w["light"], dtype=torch.float32, device="cuda", requires_grad=True)
    tgt = torch.tensor(scenegen.colour_targets(arr["means"].shape[0], 1, scenegen.SEED_TARGET + 4),
                       dtype=torch.float32, device="cuda")
    params = prt.TransferParams(num_dirs=w["num_dirs"], sh_bands=w["bands"])

    def fwd():
        col = prt.transfer_and_relight(*[ten[k] for k in keys], L, params)
        return 0.5 * ((col - tgt) ** 2).sum()

    def fwd_bwd():
        loss = fwd()
        loss.backward()
        for v in list(ten.values()) + [L]:
            v.grad = None

    res = {}
    for name, fn in (("fwd", fwd), ("fwd_bwd", fwd_bwd)):
        fn()
        torch.cuda.synchronize()
        times = []
        for _ in range(max(3, steps)):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            fn()
            torch.cuda.synchronize()
            times.append(time.perf_counter() - t0)
        res[name + "_ms"] = round(float(np.median(times)) * 1e3, 3)
    res["ratio_fwd_bwd_over_fwd"] = round(res["fwd_bwd_ms"] / res["fwd_ms"], 3)
    res["workload"] = "surface scene 200k, S=256, 16 coeffs, direct transfer + relight, L2 loss"
    log(f"backward: fwd {res['fwd_ms']} ms, fwd+bwd {res['fwd_bwd_ms']} ms")
    return res


def cpu_baseline(arr, params, seconds):
    """The oracle as it stands (brute force over all Gaussians per ray, FP64,
    all host cores) on randomly sampled sources of the same workload, batch
    by batch until the time budget is spent: each source's direct pass (every
    traced ray tested against all N Gaussians) and, with a bounce, its bounce
    walk (the same rays again, every hit listed, sorted and blended).  The
    walk weighs the hit splats' direct transfers, which in the whole job come
    from the direct pass already timed here; for timing alone it is given a
    table of ones (the brute-force cost does not depend on the values)."""
    import numpy as np

    import oracle
    oracle.build()
    scene = {k: v.astype(np.float64) for k, v in arr.items()}
    n = scene["means"].shape[0]
    S, bands = params.num_dirs, params.sh_bands
    threads = oracle.default_threads()
    dirs = oracle.directions(S)
    ones = np.ones((n, bands * bands)) if params.bounces else None
    every = np.arange(n)
    rng = np.random.default_rng(7)
    log(f"cpu baseline: oracle, {threads} threads, ~{seconds:.0f} s")
    done = traced = 0
    t_direct = t_bounce = 0.0
    batch = max(threads, 16)
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < seconds:
        src = rng.choice(n, batch, replace=False)
        a = time.perf_counter()
        oracle.direct_transfer(scene, S, bands, sources=src, margins=None, threads=threads)
        b = time.perf_counter()
        if params.bounces:
            oracle.bounce_transfer(scene, S, bands, ones, every, sources=src, threads=threads)
        c = time.perf_counter()
        t_direct += b - a
        t_bounce += c - b
        done += batch
        traced += int((scene["normals"][src] @ dirs.T > 0.0).sum())
    elapsed = t_direct + t_bounce
    value = done * S / elapsed / 1e9
    try:
        model = [ln.split(":", 1)[1].strip() for ln in open("/proc/cpuinfo") if ln.startswith("model name")][0]
    except (OSError, IndexError):
        model = "unknown"
    passes = 2 if params.bounces else 1
    what = "direct pass + bounce walk" if params.bounces else "direct pass"
    try:
        other = cpu_oracle_rates(threads)
    except Exception as e:   # context figures only: the line is still printed, with the error
        log(f"cpu oracle rates of the other workloads failed: {e!r}")
        other = {"error": repr(e)}
    return {"value": value, "unit": "Grays/s (nominal N*S rays per second)", "cores": threads, "kind": "oracle",
            "sample": f"{done} random sources of the {n}-splat workload ({done * S} nominal rays, {traced} traced, "
                      f"{what}: {t_direct:.1f} s + {t_bounce:.1f} s), each traced ray tested against all {n} "
                      f"Gaussians per pass, FP64",
            "ray_gaussian_tests_per_s": round(passes * traced * (n - 1) / elapsed, 1),
            "direct_pass_traced_rays_per_s": round(traced / t_direct, 1),
            "cpu_model": model,
            "other_workloads": other}


def cpu_oracle_rates(threads, sampled_sources=32):
    """The oracle's rates on the other workloads, a few seconds each (context
    for their GPU figures, not targets): the 1000-splat cloud in full and a
    seeded sample of sources of the 100k surface and of the 200k gradient
    workload (direct pass: every traced ray against all N Gaussians, FP64),
    and the FP64 autograd gradient of the 500-splat subset of the 200k scene
    (transfer + relight + L2 loss, every input)."""
    import numpy as np

    import oracle
    import scenegen
    from oracle.grad import loss_and_grads

    out = {}
    for name, full in (("cloud1k", True), ("surface100k", False), ("grad200k", False)):
        w = scenegen.workload(name)
        scene = w["scene"]
        n, S = scene["means"].shape[0], w["num_dirs"]
        src = np.arange(n) if full else np.random.default_rng(11).choice(n, sampled_sources, replace=False)
        dirs = oracle.directions(S)
        traced = int((scene["normals"][src] @ dirs.T > 0.0).sum())
        t0 = time.perf_counter()
        oracle.direct_transfer(scene, S, w["bands"], sources=src, margins=None, threads=threads)
        sec = time.perf_counter() - t0
        out[name] = {"sample": f"{'all' if full else 'random'} {len(src)} sources of {n}, S={S}, direct pass, "
                               f"{traced} traced rays, {sec:.2f} s",
                     "grays_per_s_nominal": len(src) * S / sec / 1e9,
                     "traced_rays_per_s": round(traced / sec, 1),
                     "ray_gaussian_tests_per_s": round(traced * (n - 1) / sec, 1)}
        log(f"cpu oracle {name}: {traced / sec:.0f} traced rays/s")
    w = scenegen.workload("grad200k")
    sub = scenegen.seeded_subset(w["scene"], 500, scenegen.SEED_FD_PICK)
    tgt = scenegen.colour_targets(500, 1, scenegen.SEED_TARGET + 4)
    t0 = time.perf_counter()
    loss_and_grads(sub, w["num_dirs"], w["bands"], w["light"], tgt)
    sec = time.perf_counter() - t0
    out["grad200k_subset500"] = {"sample": f"the 500-splat subset of the 200k scene, S={w['num_dirs']}, FP64 "
                                           f"autograd of transfer + relight + L2 loss, {sec:.2f} s",
                                 "seconds_per_gradient": round(sec, 3)}
    log(f"cpu oracle gradient, 500-splat subset: {sec:.1f} s")
    return out


if __name__ == "__main__":
    main()
