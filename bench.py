#!/usr/bin/env python3
"""Benchmark of the matrix-free LM ptychography hot path on one MI355X.

Workload: the joint object+probe problem with a 512x512 object, a 128x128
probe and a 40x40 raster (1600 positions, step 8, +-1 jitter), Poisson data at
1e4 photons per pattern, Gaussian magnitude metric, LM with D = Dg(G) and the
Jacobi preconditioner, at most 10 PCG products per solve.

One step = one outer LM iteration (linearisation with gradient and diagonal,
then attempts of {PCG solve of up to 10 GGN-vector products, trial loss, gain
ratio, damping update}) -- every row of the hot path.  ``value`` = scan
positions pushed through GGN-vector products per second of whole-step wall
time (inputs resident in HBM).  The dominant kernel (the per-position GGN-vector
kernel) is also timed alone with HIP events on its stream for the roofline.

Further keys of the same JSON line: the large scan (2048x2048 object, 256x256
probe, 10 000 positions: the product and LM iterations), LM wall time to the
oracle's final loss for plain, Jacobi, exact-Jacobi and learned PCG, the
method's variants (projected, alternating, intensity-based GGN, stochastic
diagonal, surrogate Poisson metric), the 64-problem uneven batch and the FP64
oracle's product on the host (cpu_baseline).

    python bench.py [--steps K] [--warmup W] [--gpus 1]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, HERE)

HBM_PEAK_GBS = 8000.0        # MI355X HBM3E, GB/s
FP32_PEAK_TFLOPS = 157.3     # MI355X FP32 vector (published; counts packed FP32 instructions)
# FP32 vector peak without packed instructions (the build disables them): 256 CUs x 64 FMA lanes
# x 2 flops x 2.4 GHz
FP32_NONPACKED_TFLOPS = 78.6
METRIC = "GGN·v scan-positions/s + LM wall-time to loss ≤1.01× oracle, learned vs plain"

# HBM-side bytes of one launch of the GGN-vector tile kernel on this workload, from the
# rocprofv3 FETCH_SIZE / WRITE_SIZE runs summarised in
# profiles/ggnv_tile128_joint_obj512_probe128_k1600.md (KiB per dispatch, scaled by what the
# same counters read for a plain 256 MiB copy).  Valid only for the kernel and plan sources they
# were taken on (the plan sets the segments and strips): a different hash of those sources
# reports traffic as null.
TRAFFIC = {"fetch_kib": 225272.9, "write_kib": 261049.2, "fetch_factor": 1.99981, "write_factor": 1.0,
           "grid_scale": 1.0,
           "sources": ["kernels_tile128.hip", "dft.hpp", "internal.hpp", "tile_pixel.hpp", "plan.cpp"],
           "sha256": "571ff43108861f6dc1a648cfc9e57bf998932b4242dd9329f6223ec1b00dd290"}


def measured_traffic():
    import hashlib
    h = hashlib.sha256()
    for f in TRAFFIC["sources"]:
        with open(os.path.join(HERE, "paper_2103_01767_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    if h.hexdigest() != TRAFFIC["sha256"]:
        return None
    return round((TRAFFIC["fetch_kib"] * TRAFFIC["fetch_factor"] + TRAFFIC["write_kib"] * TRAFFIC["write_factor"])
                 * 1024.0)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--calls", type=int, default=50, help="isolated GGN-vector product calls")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-calls", type=int, default=8)
    ap.add_argument("--no-lm", action="store_true", help="skip the LM time-to-target comparison")
    ap.add_argument("--lm-iters", type=int, default=60)
    ap.add_argument("--no-next", action="store_true",
                    help="skip the projected / alternating / intensity-GGN / stochastic-diagonal / surrogate runs")
    ap.add_argument("--poisson-iters", type=int, default=100)
    ap.add_argument("--no-batch", action="store_true", help="skip the uneven-batch measurement")
    ap.add_argument("--no-c4", action="store_true", help="skip the large-scan GGN-vector timing")
    ap.add_argument("--no-autotune", action="store_true", help="keep the default segment count")
    ap.add_argument("--no-mfma", action="store_true", help="skip the DFT-as-MFMA comparison (16x16 and 32x32 probes)")
    ap.add_argument("--only-mfma-trial", action="store_true",
                    help="only the DFT-as-MFMA comparison (one JSON line; for profiling)")
    ap.add_argument("--only-large-scan", action="store_true",
                    help="only time the large-scan GGN-vector product (one JSON line; for profiling)")
    ap.add_argument("--batch-iters", type=int, default=20)
    ap.add_argument("--batch-seg-len", type=int, default=2,
                    help="ptlm_desc.seg_len of the batch's problems (0: each cut as if alone on the GPU)")
    ap.add_argument("--large-lm-iters", type=int, default=3,
                    help="timed LM outer iterations on the large scan (0: skip)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a plain 256 MiB device copy (reference for the HBM byte counters)")
    return ap.parse_args()


def calibrate_copy():
    """A plain device-to-device copy of 256 MiB, five times: what the HBM byte counters read
    for a kernel of known traffic (268435456 B read + 268435456 B written per copy)."""
    import torch
    src = torch.ones(64 << 20, dtype=torch.float32, device="cuda:0")
    dst = torch.empty_like(src)
    for _ in range(5):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes": src.numel() * 4, "copies": 5}), flush=True)


def main():
    args = parse()
    if args.calibrate_copy:
        calibrate_copy()
        return
    if args.gpus != 1:
        print("bench.py runs on exactly one GPU: the library has no multi-GPU path "
              "(the scan positions would be sharded over GPUs, one process each). Use --gpus 1.",
              file=sys.stderr)
        sys.exit(2)

    # the CPU oracle first, while this process has no GPU state (its worker processes fork)
    profiling_only = args.only_large_scan or args.only_mfma_trial
    cpu = None if (args.no_cpu or profiling_only) else cpu_baseline(args.cpu_calls)

    import torch
    import synth
    import paper_2103_01767_amd as pt

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.only_large_scan:
        print(json.dumps(large_scan(dev, args.calls, args.large_lm_iters)), flush=True)
        return
    if args.only_mfma_trial:
        print(json.dumps(mfma_trial(dev, args.calls)), flush=True)
        return
    pr = synth.make_c1()
    K = pr.K
    (ny, nx), (my, mx) = pr.O_true.shape, pr.P_true.shape
    M, N = my * mx, ny * nx
    c64 = lambda a: torch.from_numpy(np.ascontiguousarray(a.astype(np.complex64))).to(dev)
    prob = pt.Problem((ny, nx), (my, mx), pr.pos, metric="gauss", mode="joint", background=pr.background,
                      device=dev)

    # synthetic Poisson counts of the workload (generated once by tests/golden/make_golden.py)
    counts = np.load(os.path.join(HERE, "tests", "golden", "c1_counts.npz"))["y"]
    y = torch.from_numpy(counts.astype(np.float32)).to(dev)

    O = c64(pr.O_init)
    P = c64(pr.P_init)
    params = pt.default_params(scaling=1, precond=1, cg_max=10)
    state = prob.new_state()
    prob.lm_init(params, state)
    stream = torch.cuda.current_stream()

    # ---------------- whole hot path: LM outer iterations
    for _ in range(args.warmup):
        prob.lm_step(O, P, y, params, state)
    torch.cuda.synchronize()
    s0 = pt.state_from_tensor(state)
    t0 = time.perf_counter()
    # the K outer iterations in one library call (ptlm_lm_solve runs ptlm_lm_step K times)
    if args.steps > 0:
        prob.lm_solve(O, P, y, params, args.steps, state)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    s1 = pt.state_from_tensor(state)
    step_s = (t1 - t0) / max(args.steps, 1)
    products = s1.products - s0.products
    attempts = s1.attempts - s0.attempts
    value = K * products / (t1 - t0) if t1 > t0 else float("nan")

    # ---------------- dominant kernel alone: per-position GGN-vector kernel (HIP events)
    prob.linearize(O, P, y)
    tune_scale, tune_ms, tune_xf = prob.autotune(reps=5) if not args.no_autotune else (1.0, None, "fft")
    iso = ggnv_isolated(prob, dev, args.calls, stream)
    kern_ms, call_ms, red_ms = iso["kernel_ms"], iso["call_ms"], iso["reduce_ms"]
    kern_bytes, achieved_gbs, fft_tflops = iso["bytes_per_launch"], iso["achieved_gbs"], iso["fft_tflops"]
    vO, vP = iso["vO"], iso["vP"]
    large = None if args.no_c4 else large_scan(dev, max(3, args.calls // 10), args.large_lm_iters)
    mfma = None if args.no_mfma else mfma_trial(dev, args.calls)

    lm = None if args.no_lm else lm_comparison(prob, pr, dev, args.lm_iters)
    nxt = None if args.no_next else lm_variants(pr, dev, args.lm_iters, args.poisson_iters)
    batch = None if args.no_batch else batch_measure(dev, args.batch_iters, args.batch_seg_len)

    if cpu is not None:
        cpu["lm_small_object_only"].update(gpu_lm_seconds(dev, "small", 20))
        cpu["lm_512_128"].update(gpu_lm_seconds(dev, "512_128", cpu["lm_512_128"]["iters"]))

    line = {
        "metric": METRIC,
        "value": round(value, 1),
        "unit": "scan-positions/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(step_s * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c64/f32 (f64 scalars)",
        "data": "synthetic",
        "config": {"workload": "joint LM, object 512x512, probe 128x128, 40x40 raster step 8 +-1, "
                               "Poisson 1e4 photons/pattern, D=Dg(G), Jacobi PCG, cg_max 10",
                   "positions": K, "probe": [my, mx], "object": [ny, nx]},
        "ggnv_products_per_step": round(products / max(args.steps, 1), 2),
        "lm_attempts_per_step": round(attempts / max(args.steps, 1), 2),
        "ggnv_call_ms": round(call_ms, 4),
        "ggnv_positions_per_s_isolated": round(K / (call_ms * 1e-3), 1),
        "ggnv_kernel_ms": round(kern_ms, 4),
        "ggnv_reduce_ms": round(red_ms, 4),
        "autotune": {"grid_scale": tune_scale, "transform": tune_xf,
                     "ms_at_scales_0.5_1_2": tune_ms[:3] if tune_ms else None},
        "fft_tflops": round(fft_tflops, 2),
        "fft_frac_fp32_peak": round(fft_tflops / FP32_PEAK_TFLOPS, 4),
        "fft_frac_fp32_nonpacked_peak": round(fft_tflops / FP32_NONPACKED_TFLOPS, 4),
        "roofline": {"bound": "hbm", "achieved": round(achieved_gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved_gbs / HBM_PEAK_GBS, 4),
                     "traffic": measured_traffic() if tune_scale == TRAFFIC["grid_scale"] else None,
                     "kernel": "t128::kernel<GGNV> (128x128 tile kernel)", "bytes_per_launch": kern_bytes,
                     "alu": {"achieved": round(fft_tflops, 2), "peak": FP32_NONPACKED_TFLOPS, "unit": "TFLOP/s",
                             "frac": round(fft_tflops / FP32_NONPACKED_TFLOPS, 4),
                             "what": "FFT flops (5 M log2 M per transform, 2 per position) / kernel time, "
                                     "against the FP32 vector peak without packed instructions"}},
        "ggnv_large_scan": large,
        "dft_mfma_trial": mfma,
        "lm_time_to_target": lm,
        "lm_variants": nxt,
        "batch_uneven": batch,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


def ggnv_isolated(prob, dev, calls, stream):
    """HIP-event timing of the GGN-vector product at the current linearisation: the
    per-position kernel alone (stage 1) and with the finishing reductions (stage 2), on the
    stream the library launches on (torch's current stream), random seeded directions."""
    import torch
    (ny, nx), (my, mx) = prob.obj_shape, prob.probe_shape
    K, M, N = prob.K, my * mx, ny * nx
    g2 = torch.Generator(device=dev)
    g2.manual_seed(7)
    vO = torch.randn((ny, nx), dtype=torch.complex64, device=dev, generator=g2)
    vP = torch.randn((my, mx), dtype=torch.complex64, device=dev, generator=g2)
    outO = torch.empty_like(vO)
    outP = torch.empty_like(vP)
    for _ in range(3):
        prob.ggn_vp(vO, vP, out=(outO, outP))
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True),
           torch.cuda.Event(enable_timing=True)) for _ in range(calls)]
    for a, b, c in ev:
        a.record(stream)
        prob.ggn_vp_stage(1, vO, vP)
        b.record(stream)
        prob.ggn_vp_stage(2, vO, vP, out=(outO, outP))
        c.record(stream)
    torch.cuda.synchronize()
    kern_ms = float(np.mean([a.elapsed_time(b) for a, b, _ in ev]))
    call_ms = float(np.median([a.elapsed_time(c) for a, _, c in ev]))
    red_ms = float(np.mean([b.elapsed_time(c) for _, b, c in ev]))
    # algorithmic bytes of one launch of the per-position kernel: the stored phasor field
    # (K*M complex64) plus the object-sized and probe-sized inputs it gathers (O, vO, P, vP)
    kern_bytes = K * M * 8 + 2 * N * 8 + 2 * M * 8
    fft_flops = 2 * 5 * M * math.log2(M) * K  # two 2D FFTs per position (5 M log2 M convention)
    return {"kernel_ms": kern_ms, "call_ms": call_ms, "reduce_ms": red_ms, "bytes_per_launch": kern_bytes,
            "achieved_gbs": kern_bytes / (kern_ms * 1e-3) / 1e9, "fft_tflops": fft_flops / (kern_ms * 1e-3) / 1e12,
            "positions_per_s": K / (call_ms * 1e-3), "vO": vO, "vP": vP}


def mfma_trial(dev, calls):
    """The GGN-vector product with the DFT as matrix products on the matrix cores against the
    FFT tile kernel's, in its standard and its wide tile grouping (ptlm_set_transform "mfma" /
    "fft" / "fft_wide"), on two small-probe scans, joint, object 512x512, raster step 4: probe 16x16
    with a 120x120 raster (14 400 positions) and probe 32x32 with a 116x116 raster (13 456
    positions), each linearised at a seeded random point with seeded stand-in counts (the
    product's cost does not depend on the data).  Whole calls (per-position kernel plus the same
    reductions), HIP events on the library's stream, median of `calls`."""
    import torch
    import synth
    import paper_2103_01767_amd as pt
    c64 = lambda a: torch.from_numpy(np.ascontiguousarray(a.astype(np.complex64))).to(dev)
    stream = torch.cuda.current_stream()
    out_all = {}
    for L, n in ((16, 120), (32, 116)):
        rng = np.random.default_rng(16016 + L)
        step, side = 4, 512
        base = 8 + step * np.arange(n)
        ry, rx = np.meshgrid(base, base, indexing="ij")
        pos = np.stack([ry.ravel(), rx.ravel()], 1).astype(np.int32)
        O = c64(synth.random_complex(rng, (side, side)))
        P = c64(synth.make_probe_fresnel(rng, L, 0.35 * L, 2.0))
        prob = pt.Problem((side, side), (L, L), pos, metric="gauss", mode="joint", background=1e-8, device=dev)
        y = torch.from_numpy(synth.surrogate_counts(rng, len(pos), (L, L), 1e3)).to(dev)
        prob.linearize(O, P, y)
        vO, vP = c64(synth.random_complex(rng, (side, side))), c64(synth.random_complex(rng, (L, L)))
        out = (torch.empty_like(vO), torch.empty_like(vP))
        res = {"workload": "joint, object 512x512, probe %dx%d, %dx%d raster step 4 (%d positions)"
               % (L, L, n, n, n * n)}
        for name in ("fft", "mfma", "fft_wide"):
            prob.set_transform(name)
            fn = prob.ggn_vp
            for _ in range(3):
                fn(vO, vP, out=out)
            torch.cuda.synchronize()
            ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(calls)]
            for a, b in ev:
                a.record(stream)
                fn(vO, vP, out=out)
                b.record(stream)
            torch.cuda.synchronize()
            res[name + "_call_ms"] = round(float(np.median([a.elapsed_time(b) for a, b in ev])), 4)
        prob.set_transform("fft")
        f_out = prob.ggn_vp(vO, vP)
        prob.set_transform("mfma")
        m_out = prob.ggn_vp(vO, vP)
        res["rel_diff"] = float(max(torch.linalg.norm(f_out[i] - m_out[i]) / torch.linalg.norm(f_out[i])
                                    for i in (0, 1)))
        res["mfma_over_fft"] = round(res["mfma_call_ms"] / res["fft_call_ms"], 3)
        res["fft_wide_over_fft"] = round(res["fft_wide_call_ms"] / res["fft_call_ms"], 3)
        out_all["%dx%d" % (L, L)] = res
        del prob
    return out_all


def large_scan(dev, calls, lm_iters=0):
    """GGN-vector product on the large scan: 2048x2048 object, 256x256 probe, 100x100 raster
    (10 000 positions), linearised at the initial guess with seeded stand-in counts of the
    workload's size and photon budget (the product's cost does not depend on the data)."""
    import torch
    import synth
    import paper_2103_01767_amd as pt
    pr = synth.make_c4()
    c64 = lambda a: torch.from_numpy(np.ascontiguousarray(a.astype(np.complex64))).to(dev)
    prob = pt.Problem(pr.O_true.shape, pr.P_true.shape, pr.pos, metric="gauss", mode="joint",
                      background=pr.background, device=dev)
    y = torch.from_numpy(synth.surrogate_counts(np.random.default_rng(1004004), pr.K, pr.P_true.shape,
                                                pr.photons)).to(dev)
    prob.linearize(c64(pr.O_init), c64(pr.P_init), y)
    iso = ggnv_isolated(prob, dev, calls, torch.cuda.current_stream())
    out = {"workload": "joint, object 2048x2048, probe 256x256, 100x100 raster step 16 +-2 (10000 positions)",
           "kernel": "tile256_kernel<GGNV>", "kernel_ms": round(iso["kernel_ms"], 4),
           "call_ms": round(iso["call_ms"], 4), "positions_per_s": round(iso["positions_per_s"], 1),
           "bytes_per_launch": iso["bytes_per_launch"], "achieved_gbs": round(iso["achieved_gbs"], 1),
           "hbm_frac": round(iso["achieved_gbs"] / HBM_PEAK_GBS, 4), "fft_tflops": round(iso["fft_tflops"], 2)}
    del y
    if lm_iters > 0:
        out["lm"] = large_scan_lm(prob, pr, dev, lm_iters)
    del prob
    torch.cuda.empty_cache()
    return out


def large_scan_lm(prob, pr, dev, iters):
    """Outer LM iterations on the large scan (D = Dg(G), at most 10 PCG products per solve),
    with the App. B Jacobi and with the learned preconditioner (network re-run at every
    linearisation, at every third, or run once at the first).  Data: Poisson draws (seeded) of the
    forward model at the true object and probe, about 1e3 photons per pattern.  One untimed
    iteration first, then `iters` timed ones; the reported rate is scan positions through
    GGN-vector products per second."""
    import torch
    import paper_2103_01767_amd as pt
    from paper_2103_01767_amd import learned
    c64 = lambda a: torch.from_numpy(np.ascontiguousarray(a.astype(np.complex64))).to(dev)
    z = prob.forward(c64(pr.O_true), c64(pr.P_true))
    gen = torch.Generator(device=dev)
    gen.manual_seed(1004005)
    y = torch.poisson((z.double() ** 2).float(), generator=gen).contiguous()
    del z
    net = learned.lm_net(learned.load(dev), pr.O_true.shape, dev)
    out = {"data": "Poisson draws of the forward model at the true object and probe", "timed_iters": iters}
    for name, prec, every in (("jacobi", 1, 1), ("learned", 2, 1), ("learned_every_3", 2, 3),
                              ("learned_once", 2, 0)):
        pt.lm_set_cnn(prob, net if prec == 2 else None)
        if prec == 2:
            pt.lm_set_cnn_refresh(prob, every)
        params = pt.default_params(scaling=1, precond=prec, cg_max=10)
        O, P = c64(pr.O_init), c64(pr.P_init)
        st = prob.new_state()
        prob.lm_init(params, st)
        f0 = float(prob.loss(O, P, y).cpu()[0])
        prob.lm_step(O, P, y, params, st)
        torch.cuda.synchronize()
        s0 = pt.state_from_tensor(st)
        t0 = time.perf_counter()
        for _ in range(iters):
            prob.lm_step(O, P, y, params, st)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        s1 = pt.state_from_tensor(st)
        prods = s1.products - s0.products
        out[name] = {"ms_per_iteration": round(el / max(iters, 1) * 1e3, 2),
                     "products_per_iteration": round(prods / max(iters, 1), 2),
                     "ggnv_positions_per_s": round(pr.K * prods / el, 1) if el > 0 else None,
                     "f_start": f0, "f_end": float(prob.loss(O, P, y).cpu()[0])}
    pt.lm_set_cnn(prob, None)
    del y
    return out


def lm_comparison(prob, pr, dev, iters):
    """LM wall time to f <= 1.01 f_oracle, for plain (unpreconditioned), Jacobi and learned PCG
    (network re-run at every linearisation, at every third, or once from the starting probe).

    Data: the stored Poisson counts of the workload; f_oracle: the FP64 oracle's loss after its
    stored number of outer iterations (D = Dg(G), Jacobi PCG) on the same data.  Each variant
    runs from the workload's initial guess for at most ``iters`` outer iterations.
    """
    import torch
    import paper_2103_01767_amd as pt
    from paper_2103_01767_amd import learned
    gold = os.path.join(HERE, "tests", "golden")
    ref = json.load(open(os.path.join(gold, "c1_oracle_lm.json")))
    y = torch.from_numpy(np.load(os.path.join(gold, "c1_counts.npz"))["y"].astype(np.float32)).to(dev)
    target = 1.01 * ref["f_final"]
    c64 = lambda a: torch.from_numpy(np.ascontiguousarray(a.astype(np.complex64))).to(dev)
    net = learned.lm_net(learned.load(dev), pr.O_true.shape, dev)
    out = {"target_loss": target, "oracle_final_loss": ref["f_final"], "oracle_iters": ref["T"],
           "max_iters": iters}
    for name, prec, every in (("plain", 0, 1), ("jacobi", 1, 1), ("jacobi_exact", 3, 1), ("learned", 2, 1),
                              ("learned_every_3", 2, 3), ("learned_once", 2, 0)):
        pt.lm_set_cnn(prob, net if prec == 2 else None)
        if prec == 2:
            pt.lm_set_cnn_refresh(prob, every)
        params = pt.default_params(scaling=1, precond=prec, cg_max=10)
        st = prob.new_state()
        O, P = c64(pr.O_init), c64(pr.P_init)
        prob.lm_init(params, st)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        hit = None
        for t in range(iters):
            prob.lm_step(O, P, y, params, st)
            f = float(prob.loss(O, P, y).cpu()[0])     # also synchronises
            if f <= target:
                hit = t + 1
                break
        el = time.perf_counter() - t0
        s = pt.state_from_tensor(st)
        out[name] = {"reached": hit is not None, "iters": hit if hit is not None else iters,
                     "seconds": round(el, 4), "final_loss": f, "ggnv_products": s.products,
                     "attempts": s.attempts}
    pt.lm_set_cnn(prob, None)
    return out


def _run_lm(prob, params, O, P, y, iters, target=None, f_floor=0.0, stop=True):
    """Outer LM iterations from (O, P) until the loss is <= target (or `iters` of them; all of them
    when not `stop`); the loss is read after every iteration (which also synchronises), alike for
    every variant timed."""
    import torch
    import paper_2103_01767_amd as pt
    st = prob.new_state()
    prob.lm_init(params, st)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    hit, f = None, float("nan")
    for t in range(iters):
        prob.lm_step(O, P, y, params, st)
        f = float(prob.loss(O, P, y).cpu()[0])
        if target is not None and hit is None and f - f_floor <= target - f_floor:
            s = pt.state_from_tensor(st)
            hit = {"iters": t + 1, "seconds": round(time.perf_counter() - t0, 4), "ggnv_products": s.products}
            if stop:
                break
    el = time.perf_counter() - t0
    s = pt.state_from_tensor(st)
    out = {"iters": s.t, "seconds": round(el, 4), "final_loss": f, "ggnv_products": s.products,
           "attempts": s.attempts}
    if target is not None:
        out["reached"] = hit is not None
        out["to_target"] = hit
    return out


def lm_variants(pr, dev, iters, poisson_iters):
    """The method's variants on the same joint 512/128 problem, data and initial guess (Jacobi PCG
    with the App. B diagonal unless stated, D = Dg(G), at most 10 products per solve).

    Gaussian metric, time to f <= 1.01 f_oracle (the target of the LM comparison):
      projected LM (alg:projected_LM, |O| <= 1), alternating LM (alg:alt_LM_ptycho: an object
      step then a probe step per outer iteration), the intensity-based GGN (App. C) and the
      stochastic diagonal estimate (8 sign-field draws per linearisation) as the preconditioner.
    Poisson metric (beta = 0.9): `poisson_iters` outer iterations of plain Poisson LM and of the
      App. E surrogate (sigma from 1 down over the same iterations, then 0): products and final
      loss of both, and the surrogate's time and products to the plain run's final loss (1.01x
      above the metric's minimum).
    """
    import torch
    import paper_2103_01767_amd as pt
    gold = os.path.join(HERE, "tests", "golden")
    ref = json.load(open(os.path.join(gold, "c1_oracle_lm.json")))
    yh = np.load(os.path.join(gold, "c1_counts.npz"))["y"]
    y = torch.from_numpy(yh.astype(np.float32)).to(dev)
    c64 = lambda a: torch.from_numpy(np.ascontiguousarray(a.astype(np.complex64))).to(dev)
    shapes = (pr.O_true.shape, pr.P_true.shape)
    target = 1.01 * ref["f_final"]
    out = {"target_loss": target, "max_iters": iters}
    base = dict(scaling=1, precond=1, cg_max=10)
    for name, ggn, kw in (("projected", "magnitude", dict(project=1)),
                          ("alternating", "magnitude", dict(alternate=1)),
                          ("intensity_ggn", "intensity", {}),
                          ("stochastic_jacobi", "magnitude", dict(precond=4, stoch_samples=8, stoch_seed=7))):
        prob = pt.Problem(*shapes, pr.pos, metric="gauss", mode="joint", background=pr.background, device=dev,
                          ggn=ggn)
        params = pt.default_params(**{**base, **kw})
        out[name] = _run_lm(prob, params, c64(pr.O_init), c64(pr.P_init), y, iters, target)
        del prob
    # Poisson metric: plain vs the App. E surrogate
    yy = yh.astype(np.float64)
    f_min = float(np.sum(yy - yy * np.log(np.where(yy > 0, yy, 1.0))))
    prob = pt.Problem(*shapes, pr.pos, metric="poisson", mode="joint", background=pr.background, device=dev)
    plain = _run_lm(prob, pt.default_params(**base, beta=0.9), c64(pr.O_init), c64(pr.P_init), y, poisson_iters)
    p_target = f_min + 1.01 * (plain["final_loss"] - f_min)
    sur = _run_lm(prob, pt.default_params(**base, beta=0.9, surrogate_T=poisson_iters, surrogate_s0=1.0),
                  c64(pr.O_init), c64(pr.P_init), y, poisson_iters, p_target, f_floor=f_min, stop=False)
    out["poisson"] = {"iters": poisson_iters, "f_min": f_min, "target_loss": p_target, "plain": plain,
                      "surrogate": sur}
    del prob
    return out


def batch_measure(dev, iters, seg_len=0):
    """64 independent joint problems of uneven sizes (object side 128..384 enlarged to fit the
    raster, probe side 32/48/64/96, n x n raster with n in 10..30, step = probe / 4, Poisson
    data at 1e3..1e5 photons per pattern) solved together: one launch per LM-attempt step for
    all problems, attempts replayed from a captured HIP graph.

    Reports, for `iters` outer iterations of Jacobi PLM (D = Dg(G)): wall time and GGN-vector
    scan-positions/s of the batch, with graph replay and with eager launches, and the same
    problems solved one after another; then time to the plain (unpreconditioned) run's final
    batch loss for plain, Jacobi and learned preconditioning (the networks re-run from the
    current probes every 5 outer iterations, ptlm_batch_cnn_refresh, and run once at bind).  Data: Poisson draws of the
    GPU forward model at the true object and probe (seeded)."""
    import torch
    import synth
    import paper_2103_01767_amd as pt
    from paper_2103_01767_amd import learned
    probs = [synth.make_c2_problem(p) for p in range(64)]
    c64 = lambda a: torch.from_numpy(np.ascontiguousarray(a.astype(np.complex64))).to(dev)
    specs = [dict(obj_shape=p.O_true.shape, probe_shape=p.P_true.shape, positions=p.pos, mode="joint",
                  background=p.background, seg_len=seg_len) for p in probs]
    batch = pt.Batch(specs, device=dev)
    gen = torch.Generator(device=dev)
    gen.manual_seed(1002)
    ys = []
    for i, p in enumerate(probs):
        z = batch.problem(i).forward(c64(p.O_true), c64(p.P_true))
        ys.append(torch.poisson((z.double() ** 2).float(), generator=gen).contiguous())
    torch.cuda.synchronize()
    K = np.array([p.K for p in probs])
    KM = int(np.sum(K * np.array([p.P_true.shape[0] * p.P_true.shape[1] for p in probs])))

    def run(prec, use_graph, T, target=None, nets=None, refresh_every=0):
        params = pt.default_params(scaling=1, precond=prec, cg_max=10)
        for i in range(len(probs)):
            pt.lm_set_cnn(batch.problem(i), nets[i] if (prec == 2 and nets) else None)
        Os = [c64(p.O_init) for p in probs]
        Ps = [c64(p.P_init) for p in probs]
        batch.bind(Os, Ps, ys, params, T, use_graph=use_graph)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        hit, attempts, done, last, refreshes = None, 0, False, 0, 0
        while not done and attempts < 30 * T:
            st, n = batch.solve(1 if target is not None else 30 * T, check_every=1 if target is not None else 4)
            attempts += n
            sts = batch.all_states()
            done = all(s.t >= T for s in sts)
            if target is not None and hit is None and sum(s.f for s in sts) <= target:
                hit = time.perf_counter() - t0
                break
            # the networks' inputs follow the probes: re-run them every `refresh_every` outer
            # iterations of the slowest problem
            tmin = min(s.t for s in sts)
            if refresh_every > 0 and tmin >= last + refresh_every:
                batch.cnn_refresh()
                last, refreshes = tmin, refreshes + 1
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        sts = batch.all_states()
        f = sum(float(batch.problem(i).loss(Os[i], Ps[i], ys[i]).cpu()[0]) for i in range(len(probs)))
        prods = sum(s.products for s in sts)
        pos_prods = sum(s.products * int(k) for s, k in zip(sts, K))
        out_r = dict(seconds=round(el, 4), attempts=attempts, final_loss=f, ggnv_products=prods,
                     ggnv_positions_per_s=round(pos_prods / el, 1), reached_s=None if hit is None else round(hit, 4))
        if prec == 2:
            out_r["network_refreshes"] = refreshes
        return out_r

    out = {"problems": len(probs), "positions": int(K.sum()), "pixel_positions": KM, "outer_iters": iters,
           "seg_len": seg_len}
    run(1, True, 2)  # warm-up: compile-time attributes, graph capture path
    out["jacobi_graph"] = run(1, True, iters)
    out["jacobi_eager"] = run(1, False, iters)
    # the same problems one after another through their own handles
    params = pt.default_params(scaling=1, precond=1, cg_max=10)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i, p in enumerate(probs):
        prob = batch.problem(i)
        O, P = c64(p.O_init), c64(p.P_init)
        st = prob.new_state()
        prob.lm_init(params, st)
        prob.lm_solve(O, P, ys[i], params, iters, st)
    torch.cuda.synchronize()
    out["jacobi_one_by_one_seconds"] = round(time.perf_counter() - t0, 4)
    # learned vs plain vs Jacobi: time to the plain run's final batch loss
    plain = run(0, True, iters)
    target = 1.01 * plain["final_loss"]
    out["target_loss"] = target
    out["plain"] = plain
    out["jacobi_to_target"] = run(1, True, iters, target=target)
    net_params = learned.load(dev)
    nets = [learned.lm_net(net_params, p.O_true.shape, dev) for p in probs]
    out["learned_to_target"] = run(2, True, iters, target=target, nets=nets, refresh_every=5)
    out["learned_once_to_target"] = run(2, True, iters, target=target, nets=nets)
    for i in range(len(probs)):
        pt.lm_set_cnn(batch.problem(i), None)
    return out


def host_info():
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {"cpu_model": model, "cpu_count": os.cpu_count()}


def _oracle_worker(conn, O, P, pos, y, b):
    """One process of the parallel oracle product: the linearisation of its positions, then
    GGN-vector products on request (the unchanged oracle; positions contribute additively)."""
    from oracle import ptycho
    lin = ptycho.linearize(O, P, pos, y, b, "gauss", True)
    conn.send("ready")
    while True:
        msg = conn.recv()
        if msg is None:
            break
        conn.send(ptycho.ggn_vp(lin, *msg))
    conn.close()


def cpu_baseline(calls, max_workers=16):
    """The FP64 oracle timed on the host, before the GPU is touched (worker processes are
    forked from a process without GPU state).  GGN-vector products of the 512/128 workload at
    its initial guess with seeded directions: on one core, and over W = min(cores, 16)
    processes each holding a contiguous block of the scan positions (partial products summed);
    the small object-only workload's oracle LM (20 outer iterations) timed here, and the
    stored 512/128 oracle LM's wall time with the host it ran on."""
    import multiprocessing as mp
    import synth
    from oracle import ptycho, solver
    pr = synth.make_c1()
    gold = os.path.join(HERE, "tests", "golden")
    Oh = pr.O_init.astype(np.complex64).astype(np.complex128)
    Ph = pr.P_init.astype(np.complex64).astype(np.complex128)
    yh = np.load(os.path.join(gold, "c1_counts.npz"))["y"].astype(np.float64)
    rng = np.random.default_rng(7)
    vO = synth.random_complex(rng, Oh.shape)
    vP = synth.random_complex(rng, Ph.shape)
    out = {"kind": "oracle", "unit": "scan-positions/s", "host": host_info()}

    # one core
    lin = ptycho.linearize(Oh, Ph, pr.pos, yh, pr.background, "gauss", True)
    times = []
    for _ in range(max(calls, 1)):
        t = time.perf_counter()
        ref = ptycho.ggn_vp(lin, vO, vP)
        times.append(time.perf_counter() - t)
    del lin
    per1 = float(np.median(times))
    out["w1"] = {"value": round(pr.K / per1, 2), "cores": 1, "seconds_per_product": round(per1, 3),
                 "products": len(times)}

    # all cores (at most 16 worker processes)
    W = max(1, min(os.cpu_count() or 1, max_workers))
    ctx = mp.get_context("fork")
    cuts = np.linspace(0, pr.K, W + 1).astype(int)
    pipes, procs = [], []
    for w in range(W):
        a, b = cuts[w], cuts[w + 1]
        parent, child = ctx.Pipe()
        proc = ctx.Process(target=_oracle_worker, args=(child, Oh, Ph, pr.pos[a:b], yh[a:b], pr.background))
        proc.start()
        pipes.append(parent)
        procs.append(proc)
    for c in pipes:
        c.recv()
    times = []
    err = None
    for _ in range(max(calls, 1)):
        t = time.perf_counter()
        for c in pipes:
            c.send((vO, vP))
        parts = [c.recv() for c in pipes]
        gO = sum(p_[0] for p_ in parts)
        gP = sum(p_[1] for p_ in parts)
        times.append(time.perf_counter() - t)
        err = max(float(np.linalg.norm(gO - ref[0]) / np.linalg.norm(ref[0])),
                  float(np.linalg.norm(gP - ref[1]) / np.linalg.norm(ref[1])))
    for c in pipes:
        c.send(None)
    for proc in procs:
        proc.join()
    perW = float(np.median(times))
    out["wall"] = {"value": round(pr.K / perW, 2), "cores": W, "seconds_per_product": round(perW, 3),
                   "products": len(times), "rel_diff_vs_one_core": err}
    out["value"] = out["wall"]["value"]
    out["cores"] = W
    out["sample"] = ("%d GGN-vector products of the 512/128 workload (1600 positions, 128x128, complex128 "
                     "NumPy FFT) on 1 core and %d over %d processes (contiguous position blocks), at the "
                     "initial guess with seeded directions; median %.2f s / %.3f s per product"
                     % (out["w1"]["products"], len(times), W, per1, perW))

    # oracle LM wall time: the small object-only workload here, the 512/128 one stored
    pr0 = synth.make_c0()
    P0 = pr0.P_true.astype(np.complex64).astype(np.complex128)
    y0 = ptycho.intensity(pr0.O_true.astype(np.complex64).astype(np.complex128), P0, pr0.pos,
                          pr0.background).astype(np.float32).astype(np.float64)
    t = time.perf_counter()
    r0 = solver.lm_solve(pr0.O_init.astype(np.complex64).astype(np.complex128), P0, pr0.pos, y0, pr0.background,
                         "gauss", False, solver.LMParams(), 20)
    out["lm_small_object_only"] = {"oracle_seconds": round(time.perf_counter() - t, 3), "iters": 20,
                                   "f_final": r0.f, "cores": 1}
    ref1 = json.load(open(os.path.join(gold, "c1_oracle_lm.json")))
    out["lm_512_128"] = {"oracle_seconds": ref1["seconds"], "iters": ref1["T"], "f_final": ref1["f_final"],
                         "host": ref1.get("host"), "source": "tests/golden/c1_oracle_lm.json"}
    return out


def gpu_lm_seconds(dev, which, iters):
    """GPU wall time of the LM the oracle's timed LM runs: the small object-only workload (plain
    LM, noise-free data) or the 512/128 one (D = Dg(G), Jacobi PCG, the stored counts), from the
    same initial guess, `iters` outer iterations in one ptlm_lm_solve call."""
    import torch
    import synth
    import paper_2103_01767_amd as pt
    c64 = lambda a: torch.from_numpy(np.ascontiguousarray(a.astype(np.complex64))).to(dev)
    if which == "small":
        pr = synth.make_c0()
        P = pr.P_true
        prob = pt.Problem(pr.O_true.shape, P.shape, pr.pos, mode="object", background=pr.background, device=dev)
        y = prob.forward(c64(pr.O_true), c64(P))
        y = (y.double() ** 2).float().contiguous()
        params = pt.default_params()
        O = c64(pr.O_init)
        Pd = c64(P)
    else:
        pr = synth.make_c1()
        prob = pt.Problem(pr.O_true.shape, pr.P_true.shape, pr.pos, mode="joint", background=pr.background,
                          device=dev)
        y = torch.from_numpy(np.load(os.path.join(HERE, "tests", "golden", "c1_counts.npz"))["y"]
                             .astype(np.float32)).to(dev)
        params = pt.default_params(scaling=1, precond=1, cg_max=10)
        O, Pd = c64(pr.O_init), c64(pr.P_init)
    st = prob.new_state()
    prob.lm_init(params, st)
    torch.cuda.synchronize()
    t = time.perf_counter()
    prob.lm_solve(O, Pd, y, params, iters, st)
    torch.cuda.synchronize()
    el = time.perf_counter() - t
    return {"gpu_seconds": round(el, 4), "iters": iters, "f_final": float(prob.loss(O, Pd, y).cpu()[0])}


if __name__ == "__main__":
    main()
