#!/usr/bin/env python3
"""Benchmark of the PRTGS transfer precompute on one MI355X.

A step is one pass of the hot path over the 100k-splat surface workload (a
unit sphere on a 4x4 plane, 100,000 Gaussians, S = 256 directions, 16 SH
coefficients, direct visibility transfer): BVH build, transfer precompute
and relighting under one light.  `value` is nominal rays (N * S) per second
of the whole step, inputs already resident on the GPU.  The same JSON line
carries the secondary measurements: the million-splat workload with one
interreflection bounce, relighting 3M splats x 64 lights with FP32 vs BF16 /
F16 storage, forward vs forward + backward on 200k splats, and the CPU oracle
baseline.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-extras] [--no-cpu]
    python bench.py --copy-mib M      # plain device copy (counter calibration)
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
# the minimal parameterisation mu, q, 1/s, o (44 B) and costs ~70 flops.
BYTES_PER_BOX_TEST = 32
BYTES_PER_PRIM_TEST = 44
FLOPS_PER_BOX_TEST = 15
FLOPS_PER_PRIM_TEST = 70


# HBM traffic of one transfer call on this workload (traversal + projection
# kernels), from two rocprofv3 counter runs (FETCH_SIZE and WRITE_SIZE, scaled
# by a 1 GiB copy): see profiles/direct_kernel_surface100k_hbm_counters.md.
# Valid only for the kernel sources it was measured on (hash below); null
# otherwise.
MEASURED_TRAFFIC = {"sources_sha256_16": "11f86c8f31e409da", "bytes_per_launch": 7.273e9}
# VALU wave instructions of the traversal kernel per launch on this workload
# (SQ_INSTS_VALU, profiles/direct_kernel_surface100k_sq_counters.md), valid
# for the same sources; with the live launch time it gives the share of the
# VALU issue rate the kernel uses (1024 SIMDs at 2.4 GHz, one wave64 FP32
# instruction per 2 cycles: the rate behind the 157.3 TFLOP/s FP32 peak).
MEASURED_VALU = {"sources_sha256_16": "11f86c8f31e409da", "instructions_per_launch": 1.173e10}
KERNEL_SOURCES = ["paper_2408_03538_amd/csrc/transfer.hip", "paper_2408_03538_amd/csrc/trace.hpp",
                  "paper_2408_03538_amd/csrc/common.hpp", "paper_2408_03538_amd/csrc/capi.hip"]   # capi: work split


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
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-extras", action="store_true", help="skip the relight and backward measurements")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-seconds", type=float, default=15.0, help="CPU oracle baseline budget")
    ap.add_argument("--copy-mib", type=int, default=0, help="only run a plain device copy of this size")
    ap.add_argument("--frame-only", action="store_true",
                    help="only time relit 1080p frames of the million-splat scene (synthetic transfers)")
    ap.add_argument("--relight-only", action="store_true",
                    help="only time the 3M x 64 relight in FP32, BF16 and F16 storage")
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
    log("generating the 100k surface workload")
    arr, sc, params, light = workload_setup(prt, torch, scenegen, "surface100k")
    n, S = sc.n, params.num_dirs
    res = time_steps(prt, torch, np, sc, params, light, args.steps, args.warmup)
    ms_step = res["ms_step"]
    log(f"step {ms_step:.2f} ms: build {res['build']:.3f} ms, transfer {res['transfer']:.2f} ms, "
        f"relight {res['relight']:.4f} ms")

    stats = prt.traversal_stats(sc, res["bvh"], params)
    traced = stats["traced_rays"]
    n_box = stats["box_tests"] / traced
    n_prim = stats["prim_tests"] / traced
    b_ray = BYTES_PER_BOX_TEST * n_box + BYTES_PER_PRIM_TEST * n_prim
    f_ray = FLOPS_PER_BOX_TEST * n_box + FLOPS_PER_PRIM_TEST * n_prim
    t_kernel = res["transfer"]
    rays_per_s = traced / (t_kernel * 1e-3)
    achieved = rays_per_s * b_ray / 1e9
    log(f"per traced ray: {n_box:.1f} box tests, {n_prim:.1f} Gaussian tests = {b_ray:.0f} algorithmic bytes; "
        f"{achieved:.0f} GB/s algorithmic")
    roofline = {
        "kernel": "direct_kernel + project_kernel (visibility traversal, then SH projection; one call)",
        "bound": "hbm",
        "achieved": round(achieved, 1),
        "peak": PEAK_HBM_GBS,
        "unit": "GB/s",
        "frac": round(achieved / PEAK_HBM_GBS, 4),
        "traffic": (MEASURED_TRAFFIC["bytes_per_launch"]
                    if kernel_sources_hash() == MEASURED_TRAFFIC["sources_sha256_16"] else None),
        "traffic_unit": "bytes per launch (FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
        "units_per_launch": traced,
        "unit_of_work": "traced ray",
        "algorithmic_bytes_per_unit": round(b_ray, 1),
        "per_ray": {"box_tests": round(n_box, 2), "prim_tests": round(n_prim, 2)},
        "ms_per_launch": round(t_kernel, 4),
        "valu_issue": ({"instructions_per_launch": MEASURED_VALU["instructions_per_launch"],
                        "busy_frac": round(MEASURED_VALU["instructions_per_launch"]
                                           / (1024 * 2.4e9 / 2 * t_kernel * 1e-3), 3)}
                       if kernel_sources_hash() == MEASURED_VALU["sources_sha256_16"] else None),
        "alu_view": {"algorithmic_flops_per_ray": round(f_ray, 1),
                     "achieved_TFLOPs": round(rays_per_s * f_ray / 1e12, 3), "peak_TFLOPs": PEAK_FP32_TFLOPS,
                     "packet_node_visits_per_64_rays": round(stats["wave_node_visits"] / (traced / 64), 1),
                     "packet_gaussian_visits_per_64_rays": round(stats["wave_prim_visits"] / (traced / 64), 1)},
    }
    value = n * S / (ms_step * 1e-3) / 1e9
    result = {
        "metric": "transfer precompute Grays/s + relit splats/s; BF16 vs FP32, fwd+bwd vs fwd",
        "value": round(value, 4),
        "unit": "Grays/s (nominal N*S rays per second of the whole step)",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "surface100k: unit sphere on a 4x4 plane, N=100,000, S=256, 16 SH coeffs, direct",
                   "n_splats": n, "num_dirs": S, "sh_coeffs": params.K, "channels": params.channels,
                   "bounces": params.bounces},
        "breakdown_ms": {"build_bvh": round(res["build"], 4), "transfer": round(res["transfer"], 4),
                         "relight": round(res["relight"], 5)},
        "traced_grays_per_s": round(rays_per_s / 1e9, 4),
        "relit_splats_per_s": round(n / (res["relight"] * 1e-3), 1),
        "traced_rays": traced,
        "roofline": roofline,
    }
    res.clear()
    torch.cuda.empty_cache()
    if not args.no_extras:
        result["million_bounce"] = bench_million(prt, torch, scenegen, np)
        result["relight_3m"] = bench_relight(prt, torch, scenegen, np, args.steps)
        result["backward_200k"] = bench_backward(prt, torch, scenegen, np, args.steps)
        result["glossy_100k"] = bench_glossy(prt, torch, scenegen, np, args.steps)
    if not args.no_cpu:
        result["cpu_baseline"] = cpu_baseline(arr, params, args.cpu_seconds)
    print(json.dumps(result), flush=True)


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
    prt.check_flags(ws_tr.buf, "transfer")
    timer.marks.clear()
    t0 = time.perf_counter()
    for _ in range(steps):
        step(True)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return {"ms_step": wall * 1e3 / steps, "build": float(np.mean(timer.ms("build"))),
            "transfer": float(np.mean(timer.ms("transfer"))), "relight": float(np.mean(timer.ms("relight"))),
            "bvh": holder["bvh"], "transfer_out": transfer}


def bench_million(prt, torch, scenegen, np):
    """1,000,000 splats, S=512, 16 coeffs, RGB with one bounce: one timed
    step (build + direct + bounce + relight) after one warm-up step."""
    log("million-splat workload with one bounce")
    arr, sc, params, light = workload_setup(prt, torch, scenegen, "million")
    res = time_steps(prt, torch, np, sc, params, light, 1, 1)
    direct = prt.TransferParams(num_dirs=params.num_dirs, sh_bands=params.sh_bands, bounces=0)
    out = torch.zeros((sc.n, 1, params.K), dtype=torch.float32, device="cuda")
    ws = prt.Workspace()
    prt.precompute_transfer(sc, res["bvh"], direct, out=out, workspace=ws)
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    prt.precompute_transfer(sc, res["bvh"], direct, out=out, workspace=ws)
    b.record()
    torch.cuda.synchronize()
    t_direct = a.elapsed_time(b)
    stats = prt.traversal_stats(sc, res["bvh"], direct)
    traced = stats["traced_rays"]
    n_box, n_prim = stats["box_tests"] / traced, stats["prim_tests"] / traced
    b_ray = BYTES_PER_BOX_TEST * n_box + BYTES_PER_PRIM_TEST * n_prim
    out_d = {"workload": "million: surface scene 200k + 20 shells x 40k, S=512, 16 coeffs, RGB + 1 bounce",
             "ms_per_step": round(res["ms_step"], 2),
             "nominal_grays_per_s": round(sc.n * params.num_dirs / (res["ms_step"] * 1e-3) / 1e9, 4),
             "breakdown_ms": {"build_bvh": round(res["build"], 3), "direct_pass": round(t_direct, 2),
                              "bounce_pass": round(res["transfer"] - t_direct, 2), "relight": round(res["relight"], 4)},
             "direct_traced_grays_per_s": round(traced / (t_direct * 1e-3) / 1e9, 4),
             "per_ray": {"box_tests": round(n_box, 2), "prim_tests": round(n_prim, 2),
                         "algorithmic_bytes": round(b_ray, 1)},
             "direct_hbm_implied_frac": round(traced / (t_direct * 1e-3) * b_ray / 1e9 / PEAK_HBM_GBS, 4)}
    log(f"million: step {res['ms_step']:.0f} ms, direct {t_direct:.0f} ms")
    # the paper's own bounce: index matrix once, then n bounces by gathers
    p_idx = prt.TransferParams(num_dirs=params.num_dirs, sh_bands=params.sh_bands, bounce_mode="index", bounces=3)
    out3 = torch.zeros((sc.n, 3, params.K), dtype=torch.float32, device="cuda")
    ws3 = prt.Workspace()
    prt.precompute_transfer(sc, res["bvh"], p_idx, out=out3, workspace=ws3)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
    ev[0].record()
    prt.precompute_transfer(sc, res["bvh"], p_idx, out=out3, workspace=ws3)
    ev[1].record()
    idx = prt.index_matrix(sc, res["bvh"], p_idx, workspace=ws3)
    ev[2].record()
    prev = prt.self_transfer(sc, p_idx, idx, out3)
    ev[3].record()
    torch.cuda.synchronize()
    t_all, t_idx, t_gather = ev[0].elapsed_time(ev[1]), ev[1].elapsed_time(ev[2]), ev[2].elapsed_time(ev[3])
    out_d["index_bounces"] = {
        "workload": "million, the paper's bounce: index matrix + 3 bounces by gathers",
        "ms_direct_plus_3_bounces": round(t_all, 2), "ms_direct_plus_index_matrix": round(t_idx, 2),
        "ms_per_gather_bounce": round(t_gather, 3)}
    # algorithmic bytes of one gather bounce: the index rows, normals and
    # outputs, plus one RGB transfer row and albedo per indexed ray
    nidx = int((idx >= 0).sum().item())
    g_bytes = sc.n * (4 * params.num_dirs + 12 + 12 * params.K) + nidx * (12 * params.K + 12)
    out_d["index_bounces"]["indexed_rays"] = nidx
    out_d["index_bounces"]["gather_GBps"] = round(g_bytes / (t_gather * 1e-3) / 1e9, 1)
    log(f"million index mode: direct + index + 3 bounces {t_all:.0f} ms, one gather bounce {t_gather:.2f} ms")
    del out3, ws3, idx, prev
    out_d["frame_1080p"] = bench_frame(prt, torch, np, sc, res["transfer_out"], light)
    del out
    torch.cuda.empty_cache()
    out_d["glossy_1m"] = bench_glossy_million(prt, torch, scenegen, np, sc, res["bvh"], params)
    del res
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
    """The oracle (brute force over all Gaussians per ray, FP64, all host
    cores) on randomly sampled sources of the same workload, in batches until
    the time budget is spent."""
    import numpy as np

    import oracle
    oracle.build()
    scene = {k: v.astype(np.float64) for k, v in arr.items()}
    n = scene["means"].shape[0]
    threads = oracle.default_threads()
    rng = np.random.default_rng(7)
    log(f"cpu baseline: oracle, {threads} threads, ~{seconds:.0f} s")
    done = 0
    t0 = time.perf_counter()
    batch = max(threads, 16)
    while time.perf_counter() - t0 < seconds:
        src = rng.choice(n, batch, replace=False)
        oracle.direct_transfer(scene, params.num_dirs, params.sh_bands, sources=src, margins=None, threads=threads)
        done += batch
    elapsed = time.perf_counter() - t0
    value = done * params.num_dirs / elapsed / 1e9
    try:
        model = [ln.split(":", 1)[1].strip() for ln in open("/proc/cpuinfo") if ln.startswith("model name")][0]
    except (OSError, IndexError):
        model = "unknown"
    return {"value": value, "unit": "Grays/s (nominal N*S rays per second)", "cores": threads, "kind": "oracle",
            "sample": f"{done} random sources of the 100k surface workload ({done * params.num_dirs} nominal rays, "
                      f"{elapsed:.1f} s), each traced ray tested against all {n} Gaussians, FP64",
            "cpu_model": model}


if __name__ == "__main__":
    main()
