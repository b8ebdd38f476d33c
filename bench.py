#!/usr/bin/env python3
"""Throughput of the randomized truncated SVD on one MI355X.

Workload: the 16384 x 16384 symmetric FP64 channel matrix with
sigma_i = exp(-i/40) plus 1e-8 symmetric Gaussian noise, target rank 256,
oversampling 16 (l = 272), q = 2 power iterations, fixed rank rule, every
product in FP64. One step = one complete decomposition on the device: the
projection P, the sketch, 2q power products with a QR after each, the
projection, the QR of its transpose, the small SVD, the rank rule, the lift of
both factors, the sign rule and the residual pass (2q + 3 = 7 streams of A).

metric value: matrix GB/s = (A streams per step) x 8 m n bytes / (time per step),
with A resident in HBM before the timed region. The roofline object covers the
dominant kernel (the streaming FP64 GEMM, MFMA-bound: intensity l/4 flop per
byte is far above the FP64 ridge of ~9.8 flop/byte); its average duration comes
from HIP events recorded around each streaming pass on the run's stream. The
step time is timed over K steps without those per-phase events; the same K
steps are then run again with them (phase times, the streaming product's
launch durations, and that run's own step time, reported beside the first).

Every plan's product tilings come from the autotuner (rsvd_tune /
rsvd_batch_tune), run before its timed region; the tuned table is reported.

Also reported (same JSON line): the mixed-precision schedules on the same
matrix ("mixed": FP32 and BF16 early products, speed-up over FP64, the
singular-value error against the FP64 run, and the rate of the BF16 plane
products against HBM and BF16 matrix-core peaks) and a 96-channel threshold batch
("batch": the batch planner's concurrent lanes with graph replay against the
same channels run one after another) and the 131072 x 8192 tall matrix
("tall": FP64, FP32 and BF16 schedules with each result's error against the
FP64 run).

Usage: python bench.py [--steps K] [--warmup W] [--gpus 1] [--n 16384] [--no-batch] [--no-tall]
"""

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "rSVD matrix GB/s + % HBM/MFMA roofline, mixed vs FP64 at 1e-6 rel σ error"
PEAK_FP64_TFLOPS = 78.6   # MI355X dense FP64 (vector = matrix)
PEAK_HBM_GBS = 8000.0     # MI355X HBM3E
PEAK_BF16_TFLOPS = 2500.0  # MI355X dense BF16 matrix

# HBM bytes per launch of the streaming product, from rocprofv3 --pmc FETCH_SIZE
# and WRITE_SIZE runs of this benchmark (profiles/rsvd_fp64_16384sq_symmetric_traffic.md).
# FETCH_SIZE is scaled by 2.0 and WRITE_SIZE by 1.0: what the counters read
# for a plain 1 GiB copy kernel. Valid only for the GEMM source they were
# taken with; any other source reports traffic as null.
TRAFFIC_SOURCE_SHA256 = "22708e6b1645ad24"
TRAFFIC_FETCH_BYTES = 1135019 * 1024 * 2.0
TRAFFIC_WRITE_BYTES = 69632 * 1024 * 1.0


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def cpu_baseline(A_np, w, k, p, q, gpu_s=None):
    """Time the CPU FP64 oracle (untuned) on the same matrix: one decomposition."""
    from threadpoolctl import threadpool_info
    from oracle.method import rsvd as oracle_rsvd
    import numpy as np

    threads = max([x.get("num_threads", 1) for x in threadpool_info()] or [1])
    t0 = time.perf_counter()
    ref = oracle_rsvd(A_np, k, p, q, seed=w.seed, symmetric=w.symmetric)
    dt = time.perf_counter() - t0
    passes = 2 * q + 3
    gbs = passes * 8.0 * w.m * w.n / dt / 1e9
    out = {
        "value": round(gbs, 3), "unit": "GB/s", "cores": int(threads), "kind": "oracle",
        "sample": f"one full decomposition of the {w.m}x{w.n} workload ({dt:.1f} s, numpy/OpenBLAS FP64)",
        "seconds": round(dt, 3),
    }
    return out, ref


def batch_leg(dev, reps=2):
    """96 symmetric channels (n_c ~ logU[500, 12000], sigma_i = exp(-i/d_c),
    d_c ~ U[10, 80]) decomposed together by the batch planner, rank by the
    relative threshold 1e-6; (k, p, q) per channel from the threshold rank of
    its spectrum (q = 2). Matrix GB/s over all channels' 2q + 2 streams."""
    import numpy as np
    import torch
    import paper_2307_15572_amd as rs
    import synth

    t0 = time.perf_counter()
    mats, probs = synth.c4(device=dev)
    torch.cuda.synchronize()
    log(f"batch workload: {len(mats)} channels in {time.perf_counter() - t0:.1f} s")
    stream = torch.cuda.current_stream(dev)
    bytes_streamed = sum(8.0 * p["m"] * p["n"] * (2 * p["q"] + 2) for p in probs)
    legs = {}
    for name, prec, lanes, graph in (("mixed_fp32_8lanes_graph", "mixed_fp32", 8, True),
                                      ("fp64_8lanes_graph", "fp64", 8, True),
                                      ("mixed_fp32_sequential", "mixed_fp32", 1, False)):
        pp = []
        for pr in probs:
            d = dict(pr)
            d.pop("d")
            d.update(precision=prec, want_residual=False)
            pp.append(d)
        bp = rs.BatchPlan(pp, lanes=lanes, use_graph=graph)
        bufs = bp.allocate(dev)
        tt = time.perf_counter()
        # the table is process-wide: the sequential leg uses the shapes the
        # lane legs tuned
        ntuned = bp.tune(mats, bufs, reps=1) if lanes > 1 else 0
        tune_s = time.perf_counter() - tt
        bp.run_into(mats, bufs)
        bp.results(bufs)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            bp.run_into(mats, bufs)
        e1.record(stream)
        res = bp.results(bufs)
        ms = e0.elapsed_time(e1) / reps
        bad, worst = 0, 0.0
        for c, (pr, r) in enumerate(zip(probs, res)):
            sig = synth.spectrum_exp(pr["m"], pr["d"])
            count = int(np.count_nonzero(sig >= synth.C4_TAU))
            want = count if bp.l[c] == pr["m"] else min(count, bp.l[c] - pr["p"])
            bad += int(r.rank != want)
            s = bufs["S"][c][: r.rank].cpu().numpy()
            worst = max(worst, float(np.max(np.abs(s - sig[: r.rank]) / sig[: r.rank])))
        legs[name] = {"ms": round(ms, 2), "value": round(bytes_streamed / (ms * 1e-3) / 1e9, 3),
                      "unit": "GB/s", "graph_replayed": bp.graph_used(),
                      "ranks_off_threshold_count": bad,
                      "autotune": {"shapes_added": int(ntuned), "seconds": round(tune_s, 2)},
                      "max_rel_sigma_err_vs_constructed": worst}
        log(f"batch {name}: {ms:.1f} ms, {legs[name]['value']} GB/s")
        del bufs, bp
        torch.cuda.empty_cache()
    seq = legs["mixed_fp32_sequential"]["ms"]
    legs["mixed_fp32_8lanes_graph"]["speedup_vs_sequential"] = round(
        seq / legs["mixed_fp32_8lanes_graph"]["ms"], 3)
    del mats
    torch.cuda.empty_cache()
    return {"workload": "c4_96_channels_threshold_1e-6", "channels": len(probs),
            "sum_n2": int(sum(p["m"] * p["n"] for p in probs)),
            "streams_per_channel": "2q + 2 (q = 2)", "legs": legs}


def tall_leg(dev, reps=2):
    """131072 x 8192 general matrix, sigma_i = 10^(-i/64) + a 1e-9 noise floor,
    k = 512, p = 16 (l = 528), q = 3: the FP64 path and the FP32 / BF16
    precision schedules (the last power product, the projection, QR, small
    SVD and residual in FP64), each result's error against the FP64 run, and
    the FP64 values against the constructed spectrum where they converged."""
    import numpy as np
    import torch
    import paper_2307_15572_amd as rs
    import synth

    t0 = time.perf_counter()
    A, sigma, w = synth.c3_device(device=dev)
    torch.cuda.synchronize()
    log(f"tall workload {w.name} in {time.perf_counter() - t0:.1f} s")
    stream = torch.cuda.current_stream(dev)
    passes = 2 * w.q + 3
    a_bytes = 8.0 * w.m * w.n
    res = {}
    ref = None
    # FP64 values converged to 1e-8 by the power iteration, (s_l / s_j)^(2q+1);
    # the mixed gate applies to them (where FP64 itself has not converged the
    # two runs differ by their own approximation error)
    l = w.k + w.p
    conv = (sigma[l] / sigma[: w.k]) ** (2 * w.q + 1) <= 1e-8
    jc = int(np.max(np.nonzero(conv)))
    for prec, thp in (("fp64", 0), ("mixed_fp32", 1), ("mixed_fp32", 2), ("mixed_bf16", 1),
                      ("mixed_bf16", 3), ("mixed_bf16_split", 1), ("mixed_bf16_split", 2)):
        plan = rs.Plan(w.m, w.n, w.k, w.p, w.q, seed=w.seed, want_residual=True, precision=prec,
                       trailing_hp=thp)
        bufs = plan.allocate(dev)
        plan.run_into(A, bufs)
        plan.result(bufs)
        plan.tune(A, bufs, reps=1)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            plan.run_into(A, bufs)
        e1.record(stream)
        r = plan.result(bufs)
        ms = e0.elapsed_time(e1) / reps
        S = bufs["S"][: r.rank].cpu().numpy()
        leg = {"ms": round(ms, 3), "value": round(passes * a_bytes / (ms * 1e-3) / 1e9, 3),
               "unit": "GB/s", "rank": int(r.rank), "residual": r.residual, "flags": int(r.flags)}
        if prec == "fp64":
            ref = (S, r.residual)
            # converged leading values against the constructed spectrum
            kk = 256
            leg["max_rel_sigma_err_vs_constructed_first256"] = float(
                np.max(np.abs(S[:kk] - sigma[:kk]) / sigma[:kk]))
        else:
            kk = min(len(S), len(ref[0]))
            rel = np.abs(S[:kk] - ref[0][:kk]) / ref[0][:kk]
            ok = rel <= 1e-6
            leg["trailing_fp64_products"] = thp
            leg["max_rel_sigma_err_vs_fp64_converged"] = float(rel[: jc + 1].max())
            leg["meets_1e-6_gate_on_converged"] = bool(ok[: jc + 1].all())
            leg["gate_holds_up_to_index"] = int(kk - 1 if ok.all() else np.argmin(ok) - 1)
            leg["max_rel_sigma_err_vs_fp64_all_kept"] = float(rel.max())
            leg["normwise_sigma_err_vs_fp64"] = float(np.max(np.abs(S[:kk] - ref[0][:kk])) / ref[0][0])
            leg["residual_rel_diff_vs_fp64"] = float(abs(r.residual - ref[1]) / ref[1])
            leg["speedup_vs_fp64"] = round(res["fp64"]["ms"] / ms, 4)
        name = prec if prec == "fp64" else f"{prec}_thp{thp}"
        res[name] = leg
        log(f"tall {name}: {ms:.2f} ms")
        del bufs, plan
        torch.cuda.empty_cache()
    del A
    torch.cuda.empty_cache()
    return {"workload": w.name, "m": w.m, "n": w.n, "k": w.k, "p": w.p, "q": w.q,
            "a_streams_per_step": passes, "spectrum": "10^(-i/64) + 1e-9 noise floor",
            "fp64_converged_indices": f"0..{jc} ((s_l/s_j)^(2q+1) <= 1e-8)", "legs": res}


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--n", type=int, default=16384)
    ap.add_argument("--no-cpu-baseline", action="store_true",
                    help="skip the oracle timing (used for profiler runs)")
    ap.add_argument("--no-batch", action="store_true",
                    help="skip the 96-channel batch leg")
    ap.add_argument("--no-tall", action="store_true",
                    help="skip the 131072 x 8192 mixed-precision leg")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(json.dumps({"error": "this build measures one GPU only; run with --gpus 1",
                          "n_gpus": args.gpus}))
        sys.exit(2)

    import numpy as np
    import torch
    import paper_2307_15572_amd as rs
    import synth

    dev = torch.device("cuda:0")
    log("generating workload")
    t0 = time.perf_counter()
    A_np, sigma, w = synth.c2(n=args.n, device=dev)
    A = torch.from_numpy(A_np).to(dev)
    torch.cuda.synchronize()
    log(f"workload {w.name} ready in {time.perf_counter() - t0:.1f} s")
    k, p, q = w.k, w.p, w.q
    plan = rs.Plan(w.m, w.n, k, p, q, symmetric=w.symmetric, seed=w.seed, want_residual=True)
    bufs = plan.allocate(dev)
    l = plan.l

    for _ in range(args.warmup):
        plan.run_into(A, bufs)
    torch.cuda.synchronize()
    # tile shapes of every product from the autotuner (outside the timed region)
    t0 = time.perf_counter()
    tuned = plan.tune(A, bufs, reps=3)
    tune_s = time.perf_counter() - t0
    log(f"warmup done; autotuner added {tuned} shapes in {tune_s:.2f} s")

    stream = torch.cuda.current_stream(dev)

    def timed(pl, bb, traced):
        """K steps between HIP events on the run's stream; with traced, the
        per-phase HIP events of the library (phase times, streaming-product
        launch durations) are recorded as well."""
        if traced:
            rs.trace_enable(True)
            rs.trace_collect()  # clear
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        t_start = time.perf_counter()
        e0.record(stream)
        for _ in range(args.steps):
            pl.run_into(A, bb)
        e1.record(stream)
        torch.cuda.synchronize()
        wall_s = time.perf_counter() - t_start
        ph = None
        if traced:
            rs.trace_enable(False)
            ph = rs.trace_collect()
        return e0.elapsed_time(e1) / args.steps, wall_s, ph

    # the step time without the phase events, then the same K steps with them
    # (phases and the streaming product's live launch durations)
    ms_step, wall, _ = timed(plan, bufs, False)
    ms_traced, _, phases = timed(plan, bufs, True)
    res = plan.result(bufs)
    log(f"timed {args.steps} steps: {ms_step:.3f} ms/step (host wall {wall / args.steps * 1e3:.3f}); "
        f"with phase events {ms_traced:.3f}")

    passes = 2 * q + 3  # sketch + 2q power products + projection + residual
    a_bytes = 8.0 * w.m * w.n
    value = passes * a_bytes / (ms_step * 1e-3) / 1e9

    gemm_ms, gemm_cnt = phases["stream_gemm"]
    gemm_avg_s = gemm_ms / gemm_cnt * 1e-3
    flops_per_launch = 2.0 * w.m * w.n * l
    achieved = flops_per_launch / gemm_avg_s / 1e12
    import hashlib
    src = os.path.join(ROOT, "paper_2307_15572_amd", "csrc", "gemm.hip")
    same = hashlib.sha256(open(src, "rb").read()).hexdigest()[:16] == TRAFFIC_SOURCE_SHA256
    traffic = round(TRAFFIC_FETCH_BYTES + TRAFFIC_WRITE_BYTES) if same else None
    main_shape = next((e for e in rs.tune_table() if e["kind"] == "fp64_stream" and e["M"] == w.m
                       and e["N"] == l and e["K"] == w.n), None)
    roofline = {
        "bound": "mfma", "achieved": round(achieved, 3), "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
        "frac": round(achieved / PEAK_FP64_TFLOPS, 4), "traffic": traffic,
        "traffic_unit": "bytes per launch (HBM, rocprofv3 FETCH_SIZE + WRITE_SIZE)",
        "algorithmic_bytes": 8.0 * w.m * w.n + 8.0 * (w.n + w.m) * l,
        "kernel": "dgemm_nn_dma_kernel<NT=17, FP64> (A x 272-column panel, LDS-DMA pipeline)",
        "tuned_shape": main_shape,
        "flops_per_launch": flops_per_launch, "avg_ms": round(gemm_avg_s * 1e3, 4),
        "launches": int(gemm_cnt),
    }
    step_roof_ms = (2 * q + 2) * flops_per_launch / (PEAK_FP64_TFLOPS * 1e12) * 1e3 \
        + 2.0 * w.m * w.n * plan.kc / (PEAK_FP64_TFLOPS * 1e12) * 1e3

    out = {
        "metric": METRIC, "value": round(value, 3), "unit": "GB/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_step, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": w.name, "m": w.m, "n": w.n, "k": k, "p": p, "q": q, "l": int(l),
                   "symmetric": True, "rank_rule": "fixed", "precision": "fp64",
                   "a_streams_per_step": passes, "spectrum": "exp(-i/40) + 1e-8 sym. noise"},
        "roofline": roofline,
        "step_fraction_of_mfma_floor": round(step_roof_ms / ms_step, 4),
        "phases_ms_per_step": {kk: round(v[0] / args.steps, 4) for kk, v in phases.items()},
        "ms_per_step_with_phase_events": round(ms_traced, 4),
        "autotune": {"shapes_added": int(tuned), "seconds": round(tune_s, 3)},
        "result": {"rank": int(res.rank), "residual": res.residual, "sweeps": int(res.sweeps),
                   "flags": int(res.flags)},
    }

    # mixed precision: FP32 matrix cores for the early products, the last
    # product before the projection and everything after it in FP64
    mixed = {}
    l_c2 = w.k + w.p
    sig_c2 = sigma
    jc2 = int(np.max(np.nonzero((sig_c2[l_c2] / sig_c2[: w.k]) ** (2 * w.q + 1) <= 1e-8)))
    for prec, thp in (("mixed_fp32", 1), ("mixed_bf16", 1), ("mixed_bf16", 2),
                      ("mixed_bf16_split", 1), ("mixed_bf16_split", 2)):
        mplan = rs.Plan(w.m, w.n, k, p, q, symmetric=w.symmetric, seed=w.seed, want_residual=True,
                        precision=prec, trailing_hp=thp)
        mb = mplan.allocate(dev)
        for _ in range(args.warmup):
            mplan.run_into(A, mb)
        mplan.tune(A, mb, reps=3)
        mms, _, _ = timed(mplan, mb, False)
        _, _, mph = timed(mplan, mb, True)
        mres = mplan.result(mb)
        s64 = bufs["S"][: res.rank].cpu().numpy()
        smx = mb["S"][: mres.rank].cpu().numpy()
        kk = min(res.rank, mres.rank)
        rel = float((np.abs(smx[:kk] - s64[:kk]) / s64[:kk]).max())
        relv = np.abs(smx[:kk] - s64[:kk]) / s64[:kk]
        mixed[f"{prec}_thp{thp}"] = {
            "value": round(passes * a_bytes / (mms * 1e-3) / 1e9, 3), "unit": "GB/s",
            "ms_per_step": round(mms, 4), "trailing_fp64_products": thp,
            "speedup_vs_fp64": round(ms_step / mms, 4),
            "max_rel_sigma_err_vs_fp64": rel,
            "meets_1e-6_gate": rel <= 1e-6,
            "max_rel_sigma_err_vs_fp64_converged": float(relv[: jc2 + 1].max()),
            "fp64_converged_indices": f"0..{jc2}",
            "residual": mres.residual,
            "phases_ms_per_step": {kk: round(v[0] / args.steps, 4) for kk, v in mph.items() if v[1]},
        }
        bms, bcnt = mph["bf16_gemm"]
        if bcnt:
            # BF16 plane product (panel planes + product + split-K sum), per launch:
            # algorithmic bytes = A planes (2 bytes per plane and entry) + the
            # FP64 panel in + the FP64 result out; flops = 2 m n l per BF16 product
            planes = 2 if prec == "mixed_bf16_split" else 1
            avg_s = bms / bcnt * 1e-3
            byts = 2.0 * planes * w.m * w.n + 8.0 * (w.n + w.m) * l
            fl = 2.0 * w.m * w.n * l * (3 if planes == 2 else 1)
            mixed[f"{prec}_thp{thp}"]["bf16_product"] = {
                "launches_per_step": bcnt // args.steps, "avg_ms": round(avg_s * 1e3, 4),
                "algorithmic_bytes": byts, "GBs": round(byts / avg_s / 1e9, 1),
                "frac_hbm": round(byts / avg_s / 1e9 / PEAK_HBM_GBS, 4),
                "TFLOPs": round(fl / avg_s / 1e12, 1),
                "frac_mfma_bf16": round(fl / avg_s / 1e12 / PEAK_BF16_TFLOPS, 4)}
        del mb, mplan
        log(f"{prec} thp={thp}: {mms:.3f} ms/step, max rel sigma err vs FP64 {rel:.2e}")
    out["mixed"] = mixed
    out["autotune"]["table"] = rs.tune_table()

    if not args.no_batch:
        torch.cuda.empty_cache()
        out["batch"] = batch_leg(dev)
    if not args.no_tall:
        torch.cuda.empty_cache()
        out["tall"] = tall_leg(dev)

    if not args.no_cpu_baseline:
        log("timing the CPU oracle")
        cb, ref = cpu_baseline(A_np, w, k, p, q)
        s = bufs["S"][: res.rank].cpu().numpy()
        rel = np.abs(s - ref.s[: res.rank]) / ref.s[: res.rank]
        cb["gpu_vs_oracle_max_rel_sigma_err"] = float(rel.max())
        cb["gpu_vs_oracle_residual_diff"] = float(abs(res.residual - ref.residual))
        out["cpu_baseline"] = cb
    else:
        out["cpu_baseline"] = None
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
