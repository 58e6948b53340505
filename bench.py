#!/usr/bin/env python3
"""Benchmark of the PRTGS transfer precompute on one MI355X.

A step is one pass of the whole hot path over the million-splat workload
(surface scene 200k + 20 ellipsoid shells x 40k = 1,000,000 Gaussians,
S = 512 directions, 16 SH coefficients, RGB transfer with one interreflection
bounce): BVH build, direct transfer, bounce, and relighting under one light.
`value` is nominal rays (N * S) per second of the whole step, inputs already
resident on the GPU.  Secondary measurements (relight throughput in FP32 /
BF16 / F16 on 3M splats x 64 lights, forward vs forward + backward on 200k
splats) and the CPU oracle baseline are added as extra fields of the same
JSON line.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-extras] [--no-cpu]
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


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-extras", action="store_true", help="skip the relight and backward measurements")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-sources", type=int, default=12, help="sampled sources of the CPU oracle baseline")
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


def million_step_setup(prt, torch, scenegen):
    import numpy as np
    w = scenegen.workload("million")
    arr = {k: np.asarray(v, dtype=np.float32) for k, v in w["scene"].items()}
    sc = prt.Scene.from_arrays(arr)
    params = prt.TransferParams(num_dirs=w["num_dirs"], sh_bands=w["bands"], bounces=w["bounces"])
    light = torch.tensor(w["light"], dtype=torch.float32, device="cuda")
    return arr, sc, params, light


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); this build has no multi-GPU path.",
              file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    import paper_2408_03538_amd as prt
    import scenegen

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    log("generating the million-splat workload")
    arr, sc, params, light = million_step_setup(prt, torch, scenegen)
    n, S = sc.n, params.num_dirs

    # buffers allocated once, outside the timed region
    ws_build = prt.Workspace()
    ws_tr = prt.Workspace()
    transfer = torch.zeros((n, params.channels, params.K), dtype=torch.float32, device="cuda")
    colour = torch.empty((n, 1, 3), dtype=torch.float32, device="cuda")
    bvh_holder = {}
    timer = Timer(torch)

    def step(record=True):
        if record:
            timer.start("build")
        bvh = prt.build_bvh(sc, workspace=ws_build, out=bvh_holder.get("bvh"))
        bvh_holder["bvh"] = bvh
        if record:
            timer.stop("build")
            timer.start("transfer")
        prt.precompute_transfer(sc, bvh, params, out=transfer, workspace=ws_tr)
        if record:
            timer.stop("transfer")
            timer.start("relight")
        prt.relight(transfer, light, out=colour)
        if record:
            timer.stop("relight")

    log("warmup")
    for _ in range(args.warmup):
        step(record=False)
    torch.cuda.synchronize()
    prt.check_flags(ws_tr.buf, "transfer")
    log(f"timing {args.steps} steps")
    timer.marks.clear()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_step = wall * 1e3 / args.steps
    t_build = float(np.mean(timer.ms("build")))
    t_transfer = float(np.mean(timer.ms("transfer")))
    t_relight = float(np.mean(timer.ms("relight")))
    log(f"step {ms_step:.1f} ms: build {t_build:.2f} ms, transfer {t_transfer:.1f} ms, relight {t_relight:.3f} ms")

    # split of the transfer into its two traversal passes, and the per-ray work
    direct_params = prt.TransferParams(num_dirs=S, sh_bands=params.sh_bands, bounces=0)
    direct_out = torch.zeros((n, 1, params.K), dtype=torch.float32, device="cuda")
    ws_d = prt.Workspace()
    for _ in range(1):
        prt.precompute_transfer(sc, bvh_holder["bvh"], direct_params, out=direct_out, workspace=ws_d)
    tdir = []
    for _ in range(max(2, args.steps)):
        timer.start("direct")
        prt.precompute_transfer(sc, bvh_holder["bvh"], direct_params, out=direct_out, workspace=ws_d)
        timer.stop("direct")
    torch.cuda.synchronize()
    t_direct = float(np.mean(timer.ms("direct")))
    t_bounce = t_transfer - t_direct
    stats = prt.traversal_stats(sc, bvh_holder["bvh"], direct_params)
    traced = stats["traced_rays"]
    n_box = stats["box_tests"] / traced
    n_prim = stats["prim_tests"] / traced
    log(f"direct {t_direct:.1f} ms, bounce {t_bounce:.1f} ms; per traced ray: {n_box:.1f} box tests, "
        f"{n_prim:.1f} Gaussian tests; packet visits {stats['wave_node_visits']} nodes")
    b_ray = BYTES_PER_BOX_TEST * n_box + BYTES_PER_PRIM_TEST * n_prim
    f_ray = FLOPS_PER_BOX_TEST * n_box + FLOPS_PER_PRIM_TEST * n_prim
    direct_rays_per_s = traced / (t_direct * 1e-3)
    achieved_flops = direct_rays_per_s * f_ray / 1e12
    roofline = {
        "kernel": "direct_kernel (visibility traversal + SH projection)",
        "bound": "alu",
        "achieved": round(achieved_flops, 3),
        "peak": PEAK_FP32_TFLOPS,
        "unit": "TFLOP/s",
        "frac": round(achieved_flops / PEAK_FP32_TFLOPS, 4),
        "traffic": None,
        "per_ray": {"box_tests": round(n_box, 2), "prim_tests": round(n_prim, 2),
                    "algorithmic_bytes": round(b_ray, 1), "algorithmic_flops": round(f_ray, 1)},
        "hbm_implied": {"rays_per_s_at_8TBps": round(PEAK_HBM_GBS * 1e9 / b_ray, 1),
                        "measured_rays_per_s": round(direct_rays_per_s, 1),
                        "frac": round(direct_rays_per_s / (PEAK_HBM_GBS * 1e9 / b_ray), 4)},
        "ms_per_launch": round(t_direct, 3),
    }

    value = n * S / (ms_step * 1e-3) / 1e9
    result = {
        "metric": "transfer precompute Grays/s + relit splats/s; BF16 vs FP32, fwd+bwd vs fwd",
        "value": round(value, 4),
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
        "config": {"workload": "million: surface scene 200k + 20 shells x 40k, S=512, 16 SH coeffs, RGB + 1 bounce",
                   "n_splats": n, "num_dirs": S, "sh_coeffs": params.K, "channels": params.channels,
                   "bounces": params.bounces},
        "breakdown_ms": {"build_bvh": round(t_build, 3), "transfer": round(t_transfer, 3),
                         "direct_pass": round(t_direct, 3), "bounce_pass": round(t_bounce, 3),
                         "relight": round(t_relight, 4)},
        "traced_grays_per_s_direct": round(direct_rays_per_s / 1e9, 4),
        "traced_rays": traced,
        "roofline": roofline,
    }

    del transfer, direct_out, colour
    bvh_holder.clear()
    ws_build.buf = ws_tr.buf = ws_d.buf = None
    torch.cuda.empty_cache()
    if not args.no_extras:
        result["relight"] = bench_relight(prt, torch, scenegen, np, args.steps)
        result["backward"] = bench_backward(prt, torch, scenegen, np, args.steps)
    if not args.no_cpu:
        result["cpu_baseline"] = cpu_baseline(arr, params, args.cpu_sources)
    print(json.dumps(result), flush=True)


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
        evs = []
        for _ in range(max(5, steps)):
            a = torch.cuda.Event(enable_timing=True)
            b = torch.cuda.Event(enable_timing=True)
            a.record()
            prt.relight(t, L, out_dtype=odt, out=out)
            b.record()
            evs.append((a, b))
        torch.cuda.synchronize()
        ms = float(np.median([a.elapsed_time(b) for a, b in evs]))
        in_bytes = t.numel() * t.element_size()
        out_bytes = out.numel() * out.element_size()
        got = out[torch.tensor(rows, device="cuda")].float().cpu().numpy().astype(np.float64)
        err = np.abs(got - ref)
        res[name] = {"ms": round(ms, 4), "pairs_per_s": round(n * B / (ms * 1e-3), 1),
                     "hbm_GBps": round((in_bytes + out_bytes) / (ms * 1e-3) / 1e9, 1),
                     "hbm_frac": round((in_bytes + out_bytes) / (ms * 1e-3) / 1e9 / PEAK_HBM_GBS, 4),
                     "max_rel_err": float((err / scale).max()), "mean_rel_err": float((err / scale).mean())}
        log(f"relight {name}: {ms:.3f} ms, {res[name]['hbm_GBps']} GB/s, max err {res[name]['max_rel_err']:.2e}")
    res["speedup_bf16_f16out_vs_f32"] = round(res["f32->f32"]["ms"] / res["bf16->f16"]["ms"], 3)
    res["speedup_bf16_f32out_vs_f32"] = round(res["f32->f32"]["ms"] / res["bf16->f32"]["ms"], 3)
    res["workload"] = "3,000,000 splats x 16 coeffs x RGB, 64 light environments"
    del T, T16, out32, out16
    torch.cuda.empty_cache()
    return res


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


def cpu_baseline(arr, params, count):
    """The oracle (brute force, FP64, all host cores) on sampled sources of
    the same workload: direct pass plus the bounce pass (the bounce's
    per-ray cost does not depend on the values of the hit splats' direct
    transfers, which are set to zero here)."""
    import numpy as np

    import oracle
    oracle.build()
    scene = {k: v.astype(np.float64) for k, v in arr.items()}
    n = scene["means"].shape[0]
    src = np.random.default_rng(7).choice(n, count, replace=False)
    threads = oracle.default_threads()
    log(f"cpu baseline: oracle on {count} sources, {threads} threads")
    t0 = time.perf_counter()
    oracle.direct_transfer(scene, params.num_dirs, params.sh_bands, sources=src, margins=None, threads=threads)
    t1 = time.perf_counter()
    zeros = np.zeros((n, params.K))
    oracle.bounce_transfer(scene, params.num_dirs, params.sh_bands, zeros, np.arange(n), sources=src, threads=threads)
    t2 = time.perf_counter()
    rays = count * params.num_dirs
    value = rays / (t2 - t0) / 1e9
    try:
        model = [l.split(":", 1)[1].strip() for l in open("/proc/cpuinfo") if l.startswith("model name")][0]
    except (OSError, IndexError):
        model = "unknown"
    return {"value": value, "unit": "Grays/s (nominal N*S rays per second)", "cores": threads, "kind": "oracle",
            "sample": f"{count} random sources of the million-splat workload, direct + bounce passes "
                      f"({t1 - t0:.1f} s + {t2 - t1:.1f} s), brute force over all 1M Gaussians per ray, FP64",
            "cpu_model": model}


if __name__ == "__main__":
    main()
