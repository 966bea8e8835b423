#!/usr/bin/env python3
"""Throughput of the funnel transform forward + adjoint on one MI355X.

Workload: a batch of 32 synthetic 1024x1024 float32 line images (5 mixed
ridge/step lines each, Gaussian noise), both parameter spaces (Np = 2048).
One step = funnel_forward of the batch + funnel_adjoint of the loss gradient
(sign of P at every line's focus cell).  Prints one JSON line.

  python bench.py [--steps K] [--warmup W] [--gpus 1] [--no-cpu-baseline]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0     # MI355X HBM3E, AMD published


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def focus_cells(lines, N, M, Np):
    """(space, row, col) where each line focuses (Eq. 19): regular space for
    lines row = k col + b, inverse space for transposed lines."""
    out = []
    for ln in lines:
        if not ln.transposed:
            bc = ln.b + ln.k * M / 2 - N / 2
            out.append((0, int(round(bc)) + Np // 2, (int(round(-ln.k * M / 2)) + M // 2) % M))
        else:
            bc = ln.b + ln.k * N / 2 - M / 2
            out.append((1, int(round(bc)) + Np // 2, (int(round(-ln.k * N / 2)) + N // 2) % N))
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--batch", type=int, default=32)
    ap.add_argument("--size", type=int, default=1024)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=12.0,
                    help="the CPU oracle sample takes whole images until this much time has passed")
    ap.add_argument("--no-autotune", action="store_true", help="keep the plan's default tile variants")
    ap.add_argument("--autotune", action="store_true",
                    help="tune the tile variants on this GPU even where a committed counter table names the "
                         "variants it measured (the default starts from those, so that its traffic applies)")
    ap.add_argument("--variants", type=str, default="",
                    help="comma-separated tile variant per launch (role order of funnel_plan_variants); "
                         "skips the autotuner, so counter runs time the variants a timed run picked")
    ap.add_argument("--workload", choices=["grad", "chirpz", "ragged", "precision", "verify", "volume"],
                    default="grad",
                    help="grad: the 32 x 1024^2 batch (default); ragged: 256 images of mixed sizes; "
                         "precision: 8 x 2048^2 in FP32 and with the split-precision matrix-core passes; "
                         "volume: plane detection in 4 volumes of 256^3 (App. A)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only; --gpus {args.gpus} is not supported "
              "(images are independent: a multi-GPU run would shard the batch)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1904_09409_amd import funnel as F
    from paper_1904_09409_amd import synth

    F.load_library()  # fails loudly if the HIP library is missing
    if args.workload == "ragged":
        return ragged_bench(args, torch, F, synth)
    if args.workload == "precision":
        return precision_bench(args, torch, F, synth)
    if args.workload == "verify":
        return verify_bench(args, torch, F, synth)
    if args.workload == "volume":
        return volume_bench(args, torch, F, synth)
    B, N, M = args.batch, args.size, args.size
    log(f"generating {B} synthetic {N}x{M} images")
    t0 = time.time()
    imgs = synth.batch("grad", count=B, size=N, seed=0)
    host = synth.stack(imgs)
    log(f"  {time.time() - t0:.1f} s")

    nvmt = "chirpz" if args.workload == "chirpz" else "linear"
    plan = F.FunnelPlan(B, N, M, 0, F.FT_SPACE_BOTH, nvmt=nvmt)
    Np = plan.Np
    tuned = None
    if args.variants:
        for role, v in enumerate(int(t) for t in args.variants.split(",")):
            F.funnel_plan_set_variant(plan.handle, role, v)
        variants_from = "given"
    elif args.autotune:
        tuned = F.funnel_autotune(plan.handle)   # set-up, outside the timed region
        variants_from = "autotuner"
    elif args.no_autotune:
        variants_from = "plan defaults"
    else:
        variants_from = benchmark_variants(F, plan, nvmt)
        tuned = variants_from == "autotuner" or None
    x = torch.from_numpy(host).cuda()
    planes = plan.forward(x)
    torch.cuda.synchronize()
    # loss = sum over lines of |P| at the focus cell -> dL/dP = sign(P) there
    dP = torch.zeros_like(planes)
    views = plan.views(planes)
    dviews = plan.views(dP)
    for b, im in enumerate(imgs):
        for sp, r, c in focus_cells(im.lines, N, M, Np):
            src = views.regular if sp == 0 else views.inverse
            dst = dviews.regular if sp == 0 else dviews.inverse
            dst[b, r, c] = torch.sign(src[b, r, c])
    dI = torch.empty_like(x)
    torch.cuda.synchronize()

    def step():
        plan.forward(x, planes)
        plan.adjoint(dP, dI)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    start, end = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    start.record()
    for _ in range(args.steps):
        step()
    end.record()
    torch.cuda.synchronize()
    ms_per_step = start.elapsed_time(end) / args.steps
    mpix = B * N * M / (ms_per_step * 1e-3) / 1e6

    # per-kernel event times over a second timed region of the same launches
    F.funnel_profile_enable(plan.handle, args.steps * 16)
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    kernels = F.funnel_profile_read(plan.handle)
    F.funnel_profile_disable(plan.handle)
    for k in kernels:
        k["avg_ms"] = k["total_ms"] / k["launches"]
        k["gbps"] = k["bytes_per_launch"] / k["avg_ms"] / 1e6
    kernels.sort(key=lambda k: -k["total_ms"])
    dom = kernels[0]
    step_bytes = sum(k["bytes_per_launch"] * k["launches"] for k in kernels) / args.steps
    step_kernel_ms = sum(k["total_ms"] for k in kernels) / args.steps

    copy_gbps, copy_ms = copy_bandwidth(torch)
    variants = F.funnel_plan_variants(plan.handle)
    traffic = measured_traffic(dom["name"], variants[ROLES_2D.index(dom["name"])], nvmt)

    cpu = cpu_fft = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(imgs, dP, plan, N, M, args.cpu_seconds, nvmt)
        if nvmt == "linear":
            cpu_fft = cpu_fft_reference(imgs, dP, N, M, Np, 5.0)

    out = {
        "metric": ("Mpixel/s funnel fwd+adjoint, 1024^2 fp32 batch; % of HBM roofline" if nvmt == "linear" else
                   "Mpixel/s funnel fwd+adjoint with the chirp-z NVMT, 1024^2 fp32 batch; % of HBM roofline"),
        "value": round(mpix, 1),
        "unit": "Mpixel/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": f"{B} x {N}x{M} fp32 synthetic line images (5 ridge/step lines, noise), "
                        f"regular+inverse space, Np={Np}, forward + adjoint"
                        + (", chirp-z NVMT" if nvmt == "chirpz" else ""),
            "batch": B, "rows": N, "cols": M, "padded_len": Np, "spaces": "both", "nvmt": nvmt,
        },
        "roofline": {
            "bound": "hbm",
            "kernel": dom["name"],
            "achieved": round(dom["gbps"], 1),
            "peak": HBM_PEAK_GBPS,
            "unit": "GB/s",
            "frac": round(dom["gbps"] / HBM_PEAK_GBPS, 4),
            "traffic": (traffic or {}).get("bytes"),
            "traffic_detail": traffic,
            "step_algorithmic_gbps": round(step_bytes / (ms_per_step * 1e6), 1),
            "step_frac": round(step_bytes / (ms_per_step * 1e6) / HBM_PEAK_GBPS, 4),
            "step_bytes": step_bytes,
            "kernel_ms_sum": round(step_kernel_ms, 4),
            "copy_gbps": round(copy_gbps, 1),
            "copy_ms": round(copy_ms, 4),
            "frac_of_copy": round(dom["gbps"] / copy_gbps, 4),
        },
        "kernels": [{"name": k["name"], "avg_ms": round(k["avg_ms"], 4),
                     "bytes": k["bytes_per_launch"], "gbps": round(k["gbps"], 1)} for k in kernels],
        "cpu_baseline": cpu,
        "cpu_fft_reference": cpu_fft,
        "tile_variants": variants,
        "autotuned": tuned is not None,
        "variants_from": variants_from,
    }
    print(json.dumps(out), flush=True)


def benchmark_variants(F, plan, nvmt: str = "linear") -> str:
    """Give a 2D plan the tile variants the default benchmark run times: the
    set the committed counter table measured while the kernel sources still
    match it (so its traffic figures apply), else the autotuner's choice on
    this GPU.  The parity tests call this too, so that they check the very
    kernels the benchmark line is measured on.  Returns where the variants
    came from."""
    measured = measured_variants(nvmt, ROLES_2D)
    if measured:
        for role, v in enumerate(measured):
            F.funnel_plan_set_variant(plan.handle, role, v)
        return "counter table"
    F.funnel_autotune(plan.handle)   # set-up, outside any timed region
    return "autotuner"


def ragged_bench(args, torch, F, synth, count=256):
    """Forward + adjoint of 256 images drawn from 240x320 / 480x640 /
    720x1280 / 1080x1920 (H x W), both spaces.  The ragged plan runs either
    schedule: its size classes' launches on concurrent streams, or one
    persistent launch per pass kind over a work queue of every class's tiles;
    each is timed eagerly and as one replayed HIP graph, beside one uniform
    plan per size class run back to back.  value = the graph replay of the
    schedule the autotuner picked."""
    log(f"generating {count} ragged synthetic images")
    ims = synth.batch("ragged", count=count, seed=0)
    shapes = [im.image.shape for im in ims]
    px = sum(int(np.prod(s)) for s in shapes)
    plan = F.RaggedPlan(shapes)
    tuned = [] if args.no_autotune else F.funnel_autotune(plan.handle)
    picked = plan.schedule
    x = plan.pack([im.image for im in ims])
    planes = plan.forward(x)
    dP = torch.randn_like(planes)
    dI = plan.adjoint(dP)
    torch.cuda.synchronize()

    def timeit(fn):
        for _ in range(args.warmup):
            fn()
        torch.cuda.synchronize()
        s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        s.record()
        for _ in range(args.steps):
            fn()
        e.record()
        torch.cuda.synchronize()
        return s.elapsed_time(e) / args.steps

    sched = {}
    kernels = {}
    names = {F.FT_SCHEDULE_CLASS_STREAMS: "class_streams", F.FT_SCHEDULE_QUEUE: "queue"}
    for sc in (F.FT_SCHEDULE_CLASS_STREAMS, F.FT_SCHEDULE_QUEUE):
        plan.set_schedule(sc)
        sched[names[sc] + "_eager"] = round(timeit(lambda: (plan.forward(x, planes), plan.adjoint(dP, dI))), 4)
        graph = F.FunnelGraph(plan, F.FT_GRAPH_FORWARD | F.FT_GRAPH_ADJOINT, x, planes, dP, dI)
        sched[names[sc] + "_graph"] = round(timeit(graph.launch), 4)
        del graph
        F.funnel_profile_enable(plan.handle, args.steps * 64)
        for _ in range(args.steps):
            plan.forward(x, planes)
            plan.adjoint(dP, dI)
        torch.cuda.synchronize()
        ks = F.funnel_profile_read(plan.handle, cap=64)
        F.funnel_profile_disable(plan.handle)
        kernels[names[sc]] = sorted(({"name": k["name"], "avg_ms": round(k["total_ms"] / k["launches"], 4),
                                      "gbps": round(k["bytes_per_launch"] / (k["total_ms"] / k["launches"]) / 1e6, 1)}
                                     for k in ks), key=lambda k: -k["avg_ms"])[:12]
    plan.set_schedule(picked)
    # per-size baseline: one uniform plan per size class, launched one after another
    by = {}
    for i, s in enumerate(shapes):
        by.setdefault(tuple(s), []).append(i)
    uni = []
    for s, idx in by.items():
        p = F.FunnelPlan(len(idx), *s)
        if not args.no_autotune:
            F.funnel_autotune(p.handle)
        xi = torch.from_numpy(np.stack([ims[i].image for i in idx])).cuda()
        pi = p.forward(xi)
        uni.append((p, xi, pi, torch.randn_like(pi), torch.empty_like(xi)))
    torch.cuda.synchronize()

    def seq():
        for p, xi, pi, dpi, dii in uni:
            p.forward(xi, pi)
            p.adjoint(dpi, dii)

    sched["sequential_per_size_plans"] = round(timeit(seq), 4)
    graph_ms = sched[names[picked] + "_graph"]
    # algorithmic bytes of the step by the 3-pass model (both spaces, forward + adjoint)
    step_bytes = 0.0
    for (N, M), idx in by.items():
        h = (N + M) // 2 - 1
        for W in (M, N):
            step_bytes += 2 * len(idx) * (4.0 * N * M + 32.0 * h * W + 4.0 * (N + M) * W)
    gbps = step_bytes / (graph_ms * 1e6)
    out = {
        "metric": "Mpixel/s funnel fwd+adjoint, ragged 256-image mix (240x320..1080x1920), fp32",
        "value": round(px / (graph_ms * 1e-3) / 1e6, 1), "unit": "Mpixel/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": graph_ms,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"{count} ragged images, {px / 1e6:.1f} Mpixel, both spaces, forward + adjoint",
                   "size_classes": {f"{s[0]}x{s[1]}": len(v) for s, v in by.items()},
                   "schedule": names[picked]},
        "roofline": {"bound": "hbm", "kernel": "whole step (3-pass byte model)", "achieved": round(gbps, 1),
                     "peak": HBM_PEAK_GBPS, "unit": "GB/s", "frac": round(gbps / HBM_PEAK_GBPS, 4),
                     "step_bytes": step_bytes},
        "schedules_ms": sched,
        "kernels": kernels,
        "autotune_schedule": [t for t in tuned if t["name"] == "schedule"],
    }
    print(json.dumps(out), flush=True)


def precision_bench(args, torch, F, synth, B=8, size=2048):
    """Forward + adjoint of 8 x 2048^2 images (10 lines, sigma 0.1), both
    spaces, with FP32 butterflies and with the BF16 / FP16 hi+lo matrix-core
    DFT passes; each plan autotuned.  value = the FP32 path; the line also
    carries every precision's step time and per-launch HBM rates."""
    log(f"generating {B} synthetic {size}x{size} images")
    imgs = synth.batch("precision", count=B, size=size, seed=0)
    x = torch.from_numpy(synth.stack(imgs)).cuda()
    res = {}
    for name, prec in (("fp32", F.FT_PREC_FP32), ("bf16x3", F.FT_PREC_BF16X3), ("fp16x3", F.FT_PREC_FP16X3)):
        plan = F.FunnelPlan(B, size, size, 0, F.FT_SPACE_BOTH, prec)
        if not args.no_autotune:
            F.funnel_autotune(plan.handle)
        planes = plan.forward(x)
        dP = torch.randn_like(planes)
        dI = torch.empty_like(x)
        torch.cuda.synchronize()

        def step():
            plan.forward(x, planes)
            plan.adjoint(dP, dI)

        for _ in range(args.warmup):
            step()
        torch.cuda.synchronize()
        s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        s.record()
        for _ in range(args.steps):
            step()
        e.record()
        torch.cuda.synchronize()
        ms = s.elapsed_time(e) / args.steps
        F.funnel_profile_enable(plan.handle, args.steps * 16)
        for _ in range(args.steps):
            step()
        torch.cuda.synchronize()
        kernels = F.funnel_profile_read(plan.handle)
        F.funnel_profile_disable(plan.handle)
        step_bytes = sum(k["bytes_per_launch"] * k["launches"] for k in kernels) / args.steps
        for k in kernels:
            k["avg_ms"] = k["total_ms"] / k["launches"]
            k["gbps"] = k["bytes_per_launch"] / k["avg_ms"] / 1e6
        kernels.sort(key=lambda k: -k["total_ms"])
        res[name] = {"ms_per_step": round(ms, 4), "mpix_s": round(B * size * size / (ms * 1e-3) / 1e6, 1),
                     "step_algorithmic_gbps": round(step_bytes / (ms * 1e6), 1),
                     "kernels": [{"name": k["name"], "avg_ms": round(k["avg_ms"], 4), "gbps": round(k["gbps"], 1)}
                                 for k in kernels],
                     "tile_variants": F.funnel_plan_variants(plan.handle)}
        log(f"  {name}: {ms:.4f} ms/step")
        del plan, planes, dP, dI
    dom = res["fp32"]["kernels"][0]
    out = {
        "metric": "Mpixel/s funnel fwd+adjoint, 8 x 2048^2 batch: FP32 and split-precision matrix-core DFT passes",
        "value": res["fp32"]["mpix_s"], "unit": "Mpixel/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": res["fp32"]["ms_per_step"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"{B} x {size}x{size} fp32 synthetic line images (10 lines, sigma 0.1), "
                               f"both spaces, Np={2 * size}, forward + adjoint"},
        "roofline": {"bound": "hbm", "kernel": dom["name"], "achieved": dom["gbps"], "peak": HBM_PEAK_GBPS,
                     "unit": "GB/s", "frac": round(dom["gbps"] / HBM_PEAK_GBPS, 4)},
        "precisions": res,
    }
    print(json.dumps(out), flush=True)


def verify_bench(args, torch, F, synth, K=16, D=3):
    """Peak extraction (K per plane), Sec. 4.5 line verification (a 7-pixel
    band) and sub-cell refinement (4 Newton steps, including its recomputation
    of the forward spectra) of the 32 x 1024^2 benchmark batch, timed
    separately with HIP events on the launch stream after one forward pass."""
    B, N = args.batch, args.size
    imgs = synth.batch("grad", count=B, size=N, seed=0)
    x = torch.from_numpy(synth.stack(imgs)).cuda()
    plan = F.FunnelPlan(B, N, N)
    planes = plan.forward(x)
    rec, cnt = plan.peaks(planes, K=K)
    out = plan.verify(x, rec, cnt, D, 0.08, 64)
    torch.cuda.synchronize()

    def timed(fn):
        for _ in range(args.warmup):
            fn()
        s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        s.record()
        for _ in range(args.steps):
            fn()
        e.record()
        torch.cuda.synchronize()
        return s.elapsed_time(e) / args.steps

    ms_peaks = timed(lambda: plan.peaks(planes, K=K))
    ms_verify = timed(lambda: plan.verify(x, rec, cnt, D, 0.08, 64, ))
    ms_refine = timed(lambda: plan.refine(x, rec, cnt, 4))
    chk = F.checks_to_numpy(out)
    n_lines = int(cnt.sum().item())
    # algorithmic bytes of one verification launch: every band position reads
    # 2D+2 pixels; each peak record is read and each check record written once
    vbytes = float(chk["length"].sum()) * (2 * D + 2) * 4 + B * plan.nspaces * K * (28 + 40)
    gbps = vbytes / (ms_verify * 1e6)
    res = {
        "metric": "lines verified per second (Sec. 4.5, 7-pixel band) on the 32 x 1024^2 batch",
        "value": round(n_lines / (ms_verify * 1e-3), 1), "unit": "lines/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_verify, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"{B} x {N}x{N}, both spaces, K={K} peaks per plane, band half-width {D}",
                   "lines": n_lines, "verified": int(chk["verified"].sum()), "peaks_ms": round(ms_peaks, 4),
                   "refine_ms": round(ms_refine, 4), "refine_iters": 4},
        "roofline": {"bound": "hbm", "kernel": "k_verify", "achieved": round(gbps, 1), "peak": HBM_PEAK_GBPS,
                     "unit": "GB/s", "frac": round(gbps / HBM_PEAK_GBPS, 5), "traffic": None,
                     "bytes_per_launch": vbytes},
        "cpu_baseline": None,
    }
    print(json.dumps(res), flush=True)


def volume_bench(args, torch, F, synth, B=4, N=256, K=16):
    """Plane detection in volumes (App. A): one step is the forward
    transform of 4 synthetic 256^3 volumes (2-6 sheets each, noise 0.1) in
    all three parameter spaces (depth z, x and y: planes of every
    orientation; padded depth 768) and the 3D peak detection of their
    parameter volumes (K = 16 per volume and space)."""
    log(f"generating {B} synthetic {N}^3 volumes")
    t0 = time.time()
    vols = synth.volume_batch(B, N, seed=0)
    x = torch.from_numpy(np.stack([v.volume for v in vols])).cuda()
    log(f"  {time.time() - t0:.1f} s")
    plan = F.VolumePlan(B, N, N, N, spaces=F.FT_VOL_SPACE_ALL)
    tuned = None
    measured = None if (args.variants or args.autotune or args.no_autotune) else measured_variants("volume", ROLES_VOL)
    if args.variants or measured:
        vs = [int(t) for t in args.variants.split(",")] if args.variants else measured
        for role, v in enumerate(vs):
            if v >= 0:
                F.funnel_volume_set_variant(plan.handle, role, v)
    elif not args.no_autotune:
        tuned = plan.autotune()   # set-up, outside the timed region
    P = plan.new_params()
    pk_ws = torch.empty(F.funnel_volume_peaks_workspace_size(plan.handle, K), dtype=torch.uint8, device="cuda")
    rec = torch.empty((B, plan.nspaces, K, F.PLANE_PEAK_WORDS), dtype=torch.int32, device="cuda")
    cnt = torch.empty((B, plan.nspaces), dtype=torch.int32, device="cuda")

    def step():
        plan.forward(x, P)
        F.funnel_volume_peaks(plan.handle, P, K, 0.0, 1, 0, rec, cnt, pk_ws)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    s.record()
    for _ in range(args.steps):
        step()
    e.record()
    torch.cuda.synchronize()
    ms_per_step = s.elapsed_time(e) / args.steps
    mvox = B * N ** 3 / (ms_per_step * 1e-3) / 1e6

    # per-kernel event times of the forward launches over a second timed region,
    # and the peak detection's own time around its call
    F.funnel_volume_profile_enable(plan.handle, args.steps * 16)
    pe = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    for i in range(args.steps):
        plan.forward(x, P)
        pe[i][0].record()
        F.funnel_volume_peaks(plan.handle, P, K, 0.0, 1, 0, rec, cnt, pk_ws)
        pe[i][1].record()
    torch.cuda.synchronize()
    kernels = F.funnel_volume_profile_read(plan.handle)
    F.funnel_volume_profile_disable(plan.handle)
    peaks_ms = sum(a.elapsed_time(b) for a, b in pe) / args.steps
    for k in kernels:
        k["avg_ms"] = k["total_ms"] / k["launches"]
        k["gbps"] = k["bytes_per_launch"] / k["avg_ms"] / 1e6
    kernels.sort(key=lambda k: -k["total_ms"])
    dom = kernels[0]
    fwd_bytes = sum(k["bytes_per_launch"] * k["launches"] for k in kernels) / args.steps
    fwd_ms = sum(k["total_ms"] for k in kernels) / args.steps
    variants = F.funnel_volume_variants(plan.handle)
    traffic = measured_traffic(dom["name"], variants[ROLES_VOL.index(dom["name"])] if dom["name"] in ROLES_VOL else -1,
                               "volume")
    copy_gbps, copy_ms = copy_bandwidth(torch)
    found = F.plane_peaks_to_numpy(rec, cnt)

    cpu = None
    if not args.no_cpu_baseline:
        from oracle import funnel_oracle as O
        try:
            from threadpoolctl import threadpool_info
            cores = max([d.get("num_threads", 1) for d in threadpool_info()] or [1])
        except Exception:
            cores = os.cpu_count() or 1
        t0 = time.time()
        Po = O.forward_volume_space(vols[0].volume.astype(np.float64), "z")
        O.peaks_list_volume(np.abs(Po), K, 0.0, 1, O.volume_boundary_mask(N, N, N, plan.Nzp), True)
        dt = time.time() - t0
        # the three spaces of a cube are the same work: one space's sample counts a third of a volume
        cpu = {"value": round(N ** 3 / 3 / dt / 1e6, 4), "unit": "Mvoxel/s", "cores": int(cores), "kind": "oracle",
               "sample": f"the z space of 1 of the {B} {N}^3 volumes, forward transform + 3D peaks, {dt:.1f} s; "
                         "the x and y spaces of a cube are the same work, so it counts as a third of the volume"}

    out = {
        "metric": "Mvoxel/s plane detection in volumes, all orientations (App. A forward transform in the "
                  "z, x and y spaces + 3D peaks), 4 x 256^3 fp32",
        "value": round(mvox, 1), "unit": "Mvoxel/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4), "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"{B} x {N}^3 fp32 synthetic volumes (2-6 planar sheets, noise 0.1), padded depth "
                               f"{plan.Nzp}, forward transform in the z, x and y spaces + 3D peaks (K={K} per space, "
                               "radius 1)",
                   "batch": B, "depth": N, "rows": N, "cols": N, "padded_len": plan.Nzp, "spaces": "z,x,y"},
        "roofline": {
            "bound": "hbm", "kernel": dom["name"], "achieved": round(dom["gbps"], 1), "peak": HBM_PEAK_GBPS,
            "unit": "GB/s", "frac": round(dom["gbps"] / HBM_PEAK_GBPS, 4),
            "traffic": (traffic or {}).get("bytes"), "traffic_detail": traffic,
            "forward_algorithmic_gbps": round(fwd_bytes / (fwd_ms * 1e6), 1),
            "forward_frac": round(fwd_bytes / (fwd_ms * 1e6) / HBM_PEAK_GBPS, 4),
            "forward_bytes": fwd_bytes, "forward_kernel_ms": round(fwd_ms, 4), "peaks_ms": round(peaks_ms, 4),
            "copy_gbps": round(copy_gbps, 1), "copy_ms": round(copy_ms, 4),
            "frac_of_copy": round(dom["gbps"] / copy_gbps, 4),
        },
        "kernels": [{"name": k["name"], "avg_ms": round(k["avg_ms"], 4), "bytes": k["bytes_per_launch"],
                     "gbps": round(k["gbps"], 1)} for k in kernels],
        "planes_found": [[int(len(f)) for f in per] for per in found],
        "sheets": [len(v.sheets) for v in vols],
        "cpu_baseline": cpu, "tile_variants": variants, "autotuned": tuned is not None,
        "variants_from": "counter table" if measured else ("autotuner" if tuned is not None else "given"),
    }
    print(json.dumps(out), flush=True)


def kernel_sources(nvmt: str = "linear"):
    """The sources that define the kernels of the forward + adjoint passes
    (their hash ties a committed counter table to the code it measured);
    "volume": the four passes of the volume transform."""
    csrc = os.path.join(ROOT, "paper_1904_09409_amd", "csrc")
    names = ["fft_core.hpp", "fft_mfma.hpp", "funnel_lengths.hpp", "funnel_passes.hpp"]
    if nvmt == "chirpz":
        names.append("funnel_chirp.hip")
    if nvmt == "volume":
        names.append("funnel_volume.hip")
    return [os.path.join(csrc, n) for n in names]


TRAFFIC_TABLES = {"linear": "funnel_fwd_adj_32x1024_traffic.json", "chirpz": "funnel_chirpz_32x1024_traffic.json",
                  "volume": "funnel_volume_4x256_traffic.json"}
# launch names in the role order of funnel_plan_variants / funnel_volume_variants
ROLES_2D = ["fwd.regular.A", "fwd.regular.B", "fwd.regular.C", "fwd.inverse.A", "fwd.inverse.B", "fwd.inverse.C",
            "adj.regular.Ct", "adj.regular.Bt", "adj.regular.At", "adj.inverse.Ct", "adj.inverse.Bt",
            "adj.inverse.At"]
ROLES_VOL = [f"volume.{s}{r}" for s in ("", "x.", "y.") for r in ("A", "Bx", "By", "C")]


def _traffic_table(nvmt: str):
    """The committed counter table of a workload, if the kernel sources still
    hash to the value recorded in it."""
    import hashlib
    path = os.path.join(ROOT, "profiles", TRAFFIC_TABLES[nvmt])
    if not os.path.exists(path):
        return None
    t = json.load(open(path))
    h = hashlib.sha256()
    for f in kernel_sources(nvmt):
        h.update(open(f, "rb").read())
    return t if h.hexdigest() == t.get("source_hash") else None


def measured_variants(nvmt: str, roles):
    """The tile variant of every launch in the committed counter table (the
    set its profiled runs pinned), or None when the table is stale or
    incomplete: then the autotuner picks."""
    t = _traffic_table(nvmt)
    if t is None or any(r not in t.get("launches", {}) for r in roles):
        return None
    return [int(t["launches"][r]["variant"]) for r in roles]


def measured_traffic(launch: str, variant: int, nvmt: str = "linear"):
    """HBM bytes of one launch from the committed rocprofv3 FETCH_SIZE /
    WRITE_SIZE table, if the kernel sources are unchanged since it was taken."""
    t = _traffic_table(nvmt)
    if t is None or launch not in t.get("launches", {}):
        return None
    e = t["launches"][launch]
    if e.get("variant") != variant:
        # a second tile variant the autotuner picks on some boxes, measured separately
        e = t.get("alternates", {}).get(launch, {}).get(str(variant))
        if e is None:
            return None
    return {"bytes": e["read_bytes"] + e["write_bytes"], "read_bytes": e["read_bytes"],
            "write_bytes": e["write_bytes"], "kernel": e["kernel"]}


def copy_bandwidth(torch, nbytes=1 << 30, reps=10):
    """Device-to-device copy of 1 GiB (read + write counted): the practical
    HBM ceiling on this GPU, and a reference kernel of known traffic."""
    a = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda").fill_(1.0)
    b = torch.empty_like(a)
    for _ in range(2):
        b.copy_(a)
    torch.cuda.synchronize()
    s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    s.record()
    for _ in range(reps):
        b.copy_(a)
    e.record()
    torch.cuda.synchronize()
    ms = s.elapsed_time(e) / reps
    del a, b
    return 2 * nbytes / ms / 1e6, ms


def cpu_baseline(imgs, dP, plan, N, M, seconds, nvmt="linear"):
    """The FP64 oracle, as it stands, on a bounded sample: forward (both
    spaces) and adjoint of whole images of the same workload, one after the
    other, until `seconds` have passed.  The chirp-z oracle (a dense
    scaled-frequency DFT per frequency row) takes about a minute per image, so
    its sample is the regular space of one image, forward + adjoint; the
    inverse space of a square image is the same work, so the rate counts
    half a pixel per pixel of that sample."""
    from oracle import funnel_oracle as O
    try:
        from threadpoolctl import threadpool_info
        cores = max([d.get("num_threads", 1) for d in threadpool_info()] or [1])
    except Exception:
        cores = os.cpu_count() or 1
    Np = plan.Np
    dPh = dP.cpu().numpy()
    if nvmt == "chirpz":
        # the y-DFT stages of one image's regular space in full, the row stage
        # (chirp-z NVMT + x' DFT and its transpose) on its first k frequency
        # rows, scaled by h / k (every row costs the same)
        img = np.asarray(imgs[0].image, dtype=np.float64)
        h, k = Np // 2 - 1, 160
        d = dPh[0, : Np * M].reshape(Np, M).astype(np.float64)
        t0 = time.time()
        S = O.spectrum_y(O.expand(img, Np))
        dG = (2.0 / Np) * (O._ydft_matrix(Np) @ d)
        t1 = time.time()
        G = O.nvmt_dft_chirpz(S[:k], Np)
        O._nvmt_dft_chirpz_transpose(dG[:k], Np)
        t2 = time.time()
        O.idft_y(np.concatenate([G, S[k:]]), Np)               # C on a full-size spectrum
        np.real(np.conj(O._ydft_matrix(Np)).T @ dG)            # the adjoint's A^T on a full-size one
        t3 = time.time()
        est = (t1 - t0) + (t2 - t1) * h / k + (t3 - t2)
        return {"value": round(0.5 * N * M / est / 1e6, 4), "unit": "Mpixel/s", "cores": int(cores),
                "kind": "oracle",
                "sample": f"regular space of 1 of the {plan.batch} {N}x{M} images, forward + adjoint: y DFTs "
                          f"in full, the chirp-z row stage on {k} of its {h} frequency rows scaled by {h}/{k} "
                          f"({t3 - t0:.1f} s timed, {est:.1f} s estimated), counted as half of the image's work"}
    t0 = time.time()
    n = 0
    for b, im in enumerate(imgs):
        O.forward(im.image, Np)
        reg = dPh[b, : Np * M].reshape(Np, M).astype(np.float64)
        inv = dPh[b, Np * M:].reshape(Np, N).astype(np.float64)
        O.adjoint(reg, inv, N, M, Np)
        n += 1
        if time.time() - t0 >= seconds:
            break
    dt = time.time() - t0
    return {"value": round(n * N * M / dt / 1e6, 4), "unit": "Mpixel/s", "cores": int(cores), "kind": "oracle",
            "sample": f"{n} of the {plan.batch} {N}x{M} images, forward both spaces + adjoint, {dt:.1f} s"}


# ------------------------------------------------------------------ FFT-based CPU reference
#
# The same transform as the oracle (linear NVMT), with the three DFTs of each
# space done by FFTs instead of explicit matrices, FP64: a fair CPU throughput
# figure beside the GPU's (the oracle's dense DFTs cost O(L) per element).
# Context only: it is not the oracle, and nothing but this benchmark's report
# uses it; tests/test_cpu_fft_reference.py pins it to the oracle.

def _fft_space_forward(img, Np, fft):
    """Parameter plane P[Np, W] of the regular space of img [H, W]: the y DFT
    of the expanded frame, the NVMT by linear interpolation, the x' DFT and
    the Hermitian inverse y DFT, with centred coordinates folded into signs
    (exp(-j 2 pi n y / L) over y = r - L/2 is (-1)^n times the FFT)."""
    H, W = img.shape
    h, top = Np // 2 - 1, (Np - H) // 2
    pad = np.zeros((Np, W))
    pad[top:top + H] = img
    n2 = np.arange(1, h + 1)
    sg = np.where(n2 % 2 == 1, -1.0, 1.0)[:, None]
    S = fft.fft(pad, axis=0)[1:h + 1] * sg
    # NVMT: g[n2, x'] = (1 - t) f[i0] + t f[i0 + 1], i0 = floor((x' Np + W n2) / (2 n2))
    xp = np.arange(W, dtype=np.int64) - W // 2
    num = xp[None, :] * Np + W * n2[:, None]
    den = 2 * n2[:, None]
    i0 = num // den
    t = (num - i0 * den) / den
    rows = np.arange(h)[:, None]
    f0 = np.where((i0 >= 0) & (i0 < W), S[rows, np.clip(i0, 0, W - 1)], 0.0)
    f1 = np.where((i0 + 1 >= 0) & (i0 + 1 < W), S[rows, np.clip(i0 + 1, 0, W - 1)], 0.0)
    g = (1.0 - t) * f0 + t * f1
    # x' DFT over centred x' and m1: G[p] = (-1)^(p + W/2) FFT(g (-1)^q)[p]
    alt = np.where(np.arange(W) % 2 == 1, -1.0, 1.0)
    G = fft.fft(g * alt[None, :], axis=1) * (alt * (-1.0) ** (W // 2))[None, :]
    # P[r, m1] = (2 / Np) Re sum_n2 G[n2] (-1)^n2 exp(+j 2 pi n2 r / Np)
    X = np.zeros((Np, W), dtype=np.complex128)
    X[1:h + 1] = G * sg
    return 2.0 * fft.ifft(X, axis=0).real


def _fft_space_adjoint(dP, H, W, Np, fft):
    """Transpose of _fft_space_forward: dI [H, W] from dP [Np, W]."""
    h, top = Np // 2 - 1, (Np - H) // 2
    n2 = np.arange(1, h + 1)
    sg = np.where(n2 % 2 == 1, -1.0, 1.0)[:, None]
    dG = (2.0 / Np) * fft.fft(dP, axis=0)[1:h + 1] * sg
    # conjugate-transposed x' DFT: dg[q] = (-1)^(q + W/2) W IFFT(dG (-1)^p)[q]
    alt = np.where(np.arange(W) % 2 == 1, -1.0, 1.0)
    dg = W * fft.ifft(dG * alt[None, :], axis=1) * (alt * (-1.0) ** (W // 2))[None, :]
    # transposed interpolation: dS[i0] += (1 - t) dg, dS[i0 + 1] += t dg
    xp = np.arange(W, dtype=np.int64) - W // 2
    num = xp[None, :] * Np + W * n2[:, None]
    den = 2 * n2[:, None]
    i0 = num // den
    t = (num - i0 * den) / den
    rows = np.broadcast_to(np.arange(h)[:, None], i0.shape)
    dS = np.zeros((h, W), dtype=np.complex128)
    for idx, wgt in ((i0, 1.0 - t), (i0 + 1, t)):
        ok = (idx >= 0) & (idx < W)
        np.add.at(dS, (rows[ok], idx[ok]), wgt[ok] * dg[ok])
    X = np.zeros((Np, W), dtype=np.complex128)
    X[1:h + 1] = dS * sg
    return (Np * fft.ifft(X, axis=0).real)[top:top + H]


def fft_reference_forward(img, Np, fft=np.fft):
    """(regular plane [Np, M], inverse plane [Np, N]) of one image."""
    img = np.asarray(img, dtype=np.float64)
    return _fft_space_forward(img, Np, fft), _fft_space_forward(img.T, Np, fft)


def fft_reference_adjoint(dP_reg, dP_inv, N, M, Np, fft=np.fft):
    """Image gradient [N, M] of both spaces."""
    return _fft_space_adjoint(dP_reg, N, M, Np, fft) + _fft_space_adjoint(dP_inv, M, N, Np, fft).T


def cpu_fft_reference(imgs, dP, N, M, Np, seconds):
    """Throughput of the FFT-based reference (scipy.fft on every core the
    process may use, else numpy's single-threaded FFT) on whole images of the
    workload, forward both spaces + adjoint, until `seconds` have passed."""
    try:
        import functools

        import scipy.fft as sfft
        cores = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)

        class _F:   # scipy.fft with all workers, the numpy.fft call signature
            fft = staticmethod(functools.partial(sfft.fft, workers=cores))
            ifft = staticmethod(functools.partial(sfft.ifft, workers=cores))
        fft, kind = _F, "scipy.fft FP64"
    except Exception:
        fft, kind, cores = np.fft, "numpy.fft FP64", 1
    dPh = dP.cpu().numpy()
    t0, n = time.time(), 0
    for b, im in enumerate(imgs):
        fft_reference_forward(im.image, Np, fft)
        fft_reference_adjoint(dPh[b, : Np * M].reshape(Np, M).astype(np.float64),
                              dPh[b, Np * M:].reshape(Np, N).astype(np.float64), N, M, Np, fft)
        n += 1
        if time.time() - t0 >= seconds:
            break
    dt = time.time() - t0
    return {"value": round(n * N * M / dt / 1e6, 4), "unit": "Mpixel/s", "cores": int(cores),
            "kind": f"FFT-based CPU reference ({kind}), context", 
            "sample": f"{n} of the {len(imgs)} {N}x{M} images, forward both spaces + adjoint, {dt:.1f} s"}


if __name__ == "__main__":
    main()
