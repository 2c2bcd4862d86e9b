#!/usr/bin/env python3
"""Benchmark of SpAMM inside SP2 on one MI355X.

Workload: the 150-molecule synthetic water cluster (N = 3750, padded to
4096, 32 x 32 leaf blocks, decay length 1.5 A, seed 0), FP32 leaf products.
One step is one full sp2_solve at tau = 1e-6 with F resident on the device
and P written to device memory: Gershgorin scaling, tree build, and every
SP2 iteration's occlusion pass, leaf products with the fused SP2 update,
norm pyramid and FP64 decisions, then the dense read-back.

Printed: one JSON line.  `value` is the SpAMM effective rate over the timed
solves, 65,536 flop per executed 32x32x32 leaf product divided by wall time.
Also reported: SP2 solves/s and p50/p99 solve latency, spamm_multiply of
X_0 * X_0 at tau in {1e-8, 1e-6, 1e-4}, the roofline of the leaf-product
kernel from HIP events recorded around each of its launches, the serving
stream (Poisson arrivals of mixed-size requests, solved one at a time with
FP32 leaves and by the lockstep server with FP32 and with split FP16 hi+lo
leaves: solves/s, p50/p99 latency, error against FP64 leaves), and the FP64
oracle timed on the host cores on a bounded sample.

Other configurations use the same line: --molecules 1000 [--decay 2.5] for
the 1000-molecule system, --precision bf16|fp16|bf16x3|fp16x3 with
--compare-fp64 for the reduced-precision forms, --serve-requests 256 for
the full serving stream.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

LEAF_FLOP = 2 * 32 ** 3            # one 32x32x32 leaf product
PEAK_FP32_TFLOPS = 157.3           # MI355X dense FP32 matrix peak
PEAK_FP64_TFLOPS = 78.6
PEAK_16BIT_TFLOPS = 2500.0        # dense BF16 / FP16 matrix peak
PEAK_HBM_GBS = 8000.0
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic.json")
GEMM_SOURCE = os.path.join(ROOT, "paper_1403_7458_amd", "csrc", "leafgemm.hip")


def source_sha(path: str) -> str:
    with open(path, "rb") as fh:
        return hashlib.sha256(fh.read()).hexdigest()[:16]


def measured_traffic(kernel: str, workload: str):
    """Per-dispatch HBM bytes of `kernel` from the committed rocprofv3 counter
    summary, or None when missing or taken from a different kernel source."""
    try:
        with open(TRAFFIC_FILE) as fh:
            data = json.load(fh)
        ent = data[kernel][workload]
    except (OSError, KeyError, ValueError):
        return None
    if ent.get("source_sha") != source_sha(GEMM_SOURCE):
        return None
    return ent.get("bytes_per_dispatch")


def percentile(xs, q):
    return float(np.percentile(np.asarray(xs), q)) if xs else None


def cpu_baseline(x0: np.ndarray, tau: float, budget_s: float = 12.0):
    """The FP64 oracle's recursive task form (Alg. 1, OpenMP, all host cores)
    on X_0 * X_0: effective GFLOP/s over repeats filling about budget_s."""
    from oracle import alg1
    times, n_exec = [], 0
    t_start = time.perf_counter()
    while True:
        t0 = time.perf_counter()
        _, info = alg1.spamm_alg1(x0, x0, tau)
        times.append(time.perf_counter() - t0)
        n_exec = info["n_exec"]
        if time.perf_counter() - t_start > budget_s or len(times) >= 30:
            break
    t = float(np.median(times))
    return {"value": LEAF_FLOP * n_exec / t / 1e9, "unit": "GFLOP/s",
            "cores": int(alg1.max_threads()), "kind": "oracle",
            "sample": f"{len(times)} x SpAMM X_0*X_0 (tau={tau:g}, {n_exec} leaf products, "
                      f"FP64, recursive task form), median {t:.3f} s each"}


def serving(args, sp, torch, dev, stream):
    """Serving stream: requests of mixed size, decay and tau arriving as a
    Poisson process, solved (a) one at a time with FP32 leaves in arrival
    order, (b) by the lockstep server with FP32 leaves and (c) by the server
    in the serving precision.  Latency = completion (P in device memory) -
    scheduled arrival; solves/s = requests / (last completion - first
    arrival).  Accuracy: ||P - P_64|| / ||P_64|| on a sample of requests,
    P_64 from FP64 leaves at the same tau."""
    from watergen import request_stream, water_cluster_torch
    reqs = request_stream(count=args.serve_requests, rate_per_s=args.serve_rate,
                          seed=args.serve_seed)
    fs = [water_cluster_torch(r.molecules, r.decay, r.seed, device=dev) for r in reqs]
    torch.cuda.synchronize()
    sizes = [f.shape[0] for f, _ in fs]
    order = np.argsort(sizes, kind="stable")
    sample = sorted({int(order[0]), int(order[len(order) // 2]), int(order[-1])})
    free, _ = torch.cuda.mem_get_info()
    budget = int(min(0.6 * free, 128 << 30))

    def wait_until(t):
        while True:
            d = t - time.perf_counter()
            if d <= 0:
                return
            time.sleep(min(d, 1e-3))

    def leg(mode, prec):
        k = len(reqs)
        lat = [0.0] * k
        keep = {}
        iters = 0
        srv = sp.Sp2Server(budget, max_active=64) if mode == "server" else None
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        if srv is None:
            for i, r in enumerate(reqs):
                wait_until(t0 + r.arrival_s)
                out = torch.empty_like(fs[i][0])
                _, st = sp.sp2_solve(fs[i][0], fs[i][1], r.tau, out=out, precision=prec,
                                     stream=stream)
                lat[i] = time.perf_counter() - (t0 + r.arrival_s)
                iters += st["iterations"]
                if i in sample:
                    keep[i] = out
            end = time.perf_counter()
            info = None
        else:
            pend, i, done = {}, 0, 0
            while done < k:
                now = time.perf_counter()
                while i < k and t0 + reqs[i].arrival_s <= now:
                    rid = srv.submit(fs[i][0], fs[i][1], reqs[i].tau, precision=prec)
                    pend[rid] = (i, torch.empty_like(fs[i][0]))
                    i += 1
                moved = False
                for rid in list(pend):
                    j, out = pend[rid]
                    res = srv.poll(rid, out=out)
                    if res is not None:
                        lat[j] = time.perf_counter() - (t0 + reqs[j].arrival_s)
                        iters += res[1]["iterations"]
                        if j in sample:
                            keep[j] = out
                        del pend[rid]
                        done += 1
                        moved = True
                if not moved:
                    time.sleep(2e-4)
            end = time.perf_counter()
            info = srv.stats()
            srv.close()
        res = {"precision": prec, "solves_per_s": round(k / (end - t0), 3),
               "p50_ms": round(percentile(lat, 50) * 1e3, 2),
               "p99_ms": round(percentile(lat, 99) * 1e3, 2),
               "makespan_s": round(end - t0, 3), "sp2_iterations": iters}
        if info is not None:
            res["steps"] = info["steps"]
            res["gemm_launches"] = info["gemm_launches"]
            res["peak_used_gib"] = round(info["peak_used_bytes"] / 2 ** 30, 2)
        return res, keep

    # Warm-up of both paths (library set-up, pools) on the smallest request.
    j0 = int(order[0])
    sp.sp2_solve(fs[j0][0], fs[j0][1], reqs[j0].tau, out=torch.empty_like(fs[j0][0]),
                 stream=stream)
    with sp.Sp2Server(budget) as srv:
        srv.wait(srv.submit(fs[j0][0], fs[j0][1], reqs[j0].tau, precision=args.serve_precision),
                 out=torch.empty_like(fs[j0][0]))
    legs = {}
    outs = {}
    for name, mode, prec in (("serial_fp32", "serial", "fp32"), ("server_fp32", "server", "fp32"),
                             ("server_" + args.serve_precision, "server", args.serve_precision)):
        legs[name], outs[name] = leg(mode, prec)
        torch.cuda.synchronize()
    for j in sample:
        ref = torch.empty_like(fs[j][0])
        sp.sp2_solve(fs[j][0], fs[j][1], reqs[j].tau, out=ref, precision="fp64", stream=stream)
        torch.cuda.synchronize()
        nr = float(torch.linalg.norm(ref))
        for name in legs:
            e = float(torch.linalg.norm(outs[name][j] - ref)) / nr
            legs[name]["rel_err_vs_fp64_max"] = max(legs[name].get("rel_err_vs_fp64_max", 0.0), e)
    return {
        "workload": f"{len(reqs)} SP2 requests, Poisson arrivals at {args.serve_rate:g}/s "
                    f"(stream seed {args.serve_seed}), molecules U{{30..400}} (N 750..10000), "
                    "decay U[1.2, 2.5] A, tau in {1e-6, 1e-5}",
        "n_range": [min(sizes), max(sizes)],
        "accuracy_sample_n": [sizes[j] for j in sample],
        "legs": legs,
    }


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--tau", type=float, default=1e-6)
    ap.add_argument("--molecules", type=int, default=150)
    ap.add_argument("--decay", type=float, default=1.5)
    ap.add_argument("--precision", default="fp32",
                    choices=["fp64", "fp32", "bf16", "fp16", "bf16x3", "fp16x3"])
    ap.add_argument("--full-squares", action="store_true",
                    help="SP2 without symmetric squares (every C block computed)")
    ap.add_argument("--full-square-reference", action="store_true",
                    help="also run one untimed solve with full squares and report the "
                         "full-square-equivalent rate")
    ap.add_argument("--compare-fp64", action="store_true",
                    help="also solve with FP64 leaves and report the error against it")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-multiply", action="store_true")
    ap.add_argument("--serve-requests", type=int, default=64,
                    help="requests in the serving stream (0: skip the serving legs)")
    ap.add_argument("--serve-rate", type=float, default=20.0)
    ap.add_argument("--serve-seed", type=int, default=0)
    ap.add_argument("--serve-precision", default="fp16x3")
    ap.add_argument("--copy-mib", type=int, default=0,
                    help="also run one plain device copy of this many MiB (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the SpAMM/SP2 path "
              "is single-device here and has no multi-GPU form to measure.", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_1403_7458_amd as sp
    from watergen import water_cluster

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(2)
    sp.load()
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()
    w = water_cluster(args.molecules, args.decay, 0)
    n, n_occ, tau, prec = w.n, w.n_occ, args.tau, args.precision
    f = torch.from_numpy(w.f).to(dev)
    p = torch.empty_like(f)

    def solve():
        return sp.sp2_solve(f, n_occ, tau, out=p, precision=prec, stream=stream,
                            symmetric=not args.full_squares)

    for _ in range(args.warmup):
        solve()
    torch.cuda.synchronize()
    # Inside the timed steps only the leaf-product launches are bracketed by
    # events (the roofline's launch durations); each bracket costs host time
    # between launches.
    sp.profile_reset()
    sp.profile_phases("gemm")
    sp.profile_enable(True)
    lat, stats = [], None
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        ts = time.perf_counter()
        _, stats = solve()
        lat.append(time.perf_counter() - ts)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    sp.profile_enable(False)
    prof = sp.profile_read()
    # The per-phase breakdown comes from extra, untimed solves with every
    # phase bracketed.
    phase_steps = 2
    sp.profile_reset()
    sp.profile_phases()
    sp.profile_enable(True)
    for _ in range(phase_steps):
        solve()
    sp.profile_enable(False)
    prof_all = sp.profile_read()

    execs = stats["n_exec_total"]
    value = LEAF_FLOP * execs * args.steps / elapsed / 1e9
    # Accuracy of the last result (measurement only): trace and idempotency.
    pt = p.double()
    tr_err = abs(float(torch.trace(pt)) - n_occ)
    idem = float(torch.linalg.norm(pt @ pt - pt))

    # With --full-square-reference, the same solve with full squares
    # (untimed): the leaf products the plain method executes, for the
    # full-square-equivalent rate.
    full_products = None
    if args.full_square_reference and stats.get("symmetric"):
        _, sfull = sp.sp2_solve(f, n_occ, tau, out=torch.empty_like(f), precision=prec,
                                stream=stream, symmetric=False)
        full_products = sfull["n_exec_total"]

    accuracy = None
    if args.compare_fp64:
        p64 = torch.empty_like(f)
        sp.sp2_solve(f, n_occ, tau, out=p64, precision="fp64", stream=stream)
        torch.cuda.synchronize()
        accuracy = {"rel_err_vs_fp64": float(torch.linalg.norm(p - p64) / torch.linalg.norm(p64)),
                    "fp64_trace_error": abs(float(torch.trace(p64)) - n_occ),
                    "fp64_idempotency": float(torch.linalg.norm(p64 @ p64 - p64))}
        del p64

    # Roofline of the leaf-product kernel: algorithmic flop per launch over
    # the mean launch duration from the events bracketing each launch.  The
    # split forms run three MFMA products per leaf product.
    launches = prof["launches"]["gemm"]
    gemm_ms = prof["ms"]["gemm"] / max(launches, 1)
    per_launch = prof["gemm_products"] / max(launches, 1)
    mfma_per_leaf = 3 if prec.endswith("x3") else 1
    peak = {"fp64": PEAK_FP64_TFLOPS, "fp32": PEAK_FP32_TFLOPS}.get(prec, PEAK_16BIT_TFLOPS)
    achieved = mfma_per_leaf * LEAF_FLOP * per_launch / (gemm_ms * 1e-3) / 1e12
    choice = os.environ.get("SPAMM_LEAF_KERNEL", "w2x2s")
    kname = {"fp64": "k_leaf_gemm_f64 (one wave per C block)",
             "fp32": f"k_leaf_gemm_f32 {choice}"}.get(prec, f"k_leaf_gemm_half_w2x2<{prec}>")
    roofline = {"bound": "mfma", "achieved": round(achieved, 3), "peak": peak,
                "unit": "TFLOP/s", "frac": round(achieved / peak, 4),
                "traffic": measured_traffic(f"leaf_gemm_{prec}_{choice}",
                                            f"water{args.molecules}_decay{args.decay:g}_tau{tau:g}"),
                "kernel": kname + " (fused SP2 update)",
                "launches": launches, "mean_launch_ms": round(gemm_ms, 4),
                "products_per_launch": round(per_launch, 1)}
    phase_ms = {k: round(v / phase_steps, 3) for k, v in prof_all["ms"].items()}
    # HBM-bound passes: algorithmic bytes over the phase time per solve.
    # Ingest: one read of F and one write of X_0's tiles; output: one read of
    # P's tiles and one write of the dense FP64 P.
    tile = {"fp64": 8192, "fp32": 4096, "bf16": 4096, "fp16": 4096}.get(prec, 8192)
    tiles0 = stats["n_blocks"][0] * tile
    tiles_p = stats["n_blocks"][-1] * tile
    passes = {}
    for name, phase, nbytes in (("ingest", "tree", 8 * n * n + tiles0),
                                ("output", "dense", 8 * n * n + tiles_p)):
        ms = prof_all["ms"][phase] / phase_steps
        if ms > 0:
            gbs = nbytes / (ms * 1e-3) / 1e9
            passes[name] = {"bytes": nbytes, "ms": round(ms, 4), "gbs": round(gbs, 1),
                            "frac_of_hbm_peak": round(gbs / PEAK_HBM_GBS, 4)}

    multiply = {}
    x0 = None
    if not args.no_multiply:
        mx, lo, hi = sp.sp2_initial_guess(f, prec, stream=stream)
        for t in (1e-8, 1e-6, 1e-4):
            # Statistics from one untimed call; the timed calls skip the
            # passes only the statistics need.
            mc, st = sp.spamm_multiply(mx, mx, t, stream=stream)
            mc.close()
            times = []
            for _ in range(5):
                torch.cuda.synchronize()
                ts = time.perf_counter()
                mc, _ = sp.spamm_multiply(mx, mx, t, stream=stream, stats=False)
                torch.cuda.synchronize()
                times.append(time.perf_counter() - ts)
                mc.close()
            tm = float(np.median(times))
            multiply[f"{t:g}"] = {
                "gflops": round(LEAF_FLOP * st["n_exec"] / tm / 1e9, 1), "ms": round(tm * 1e3, 3),
                "n_exec": st["n_exec"], "culled_frac_nonzero": round(1 - st["n_exec"] / st["n_nonzero_pairs"], 4),
                "culled_frac_dense": round(1 - st["n_exec"] / st["n_dense"], 4),
                "err_bound": st["err_bound"]}
        mx.close()

    serve = None
    if args.serve_requests > 0:
        serve = serving(args, sp, torch, dev, stream)

    cpu = None
    if not args.no_cpu_baseline:
        from oracle import sp2_oracle as sp2o
        from oracle import spamm_oracle as so
        lo, hi = sp2o.gershgorin(w.f)
        x0 = sp2o.initial_x(w.f, lo, hi, so.padded_size(n))
        cpu = cpu_baseline(x0, tau)

    copy = None
    if args.copy_mib > 0:
        # A plain copy of known size: its FETCH_SIZE / WRITE_SIZE counters
        # calibrate the per-dispatch HBM byte counts of the other kernels.
        nbytes = args.copy_mib << 20
        src = torch.ones(nbytes // 4, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        ts = time.perf_counter()
        dst.copy_(src)
        torch.cuda.synchronize()
        copy = {"bytes_read": nbytes, "bytes_written": nbytes,
                "gbs": round(2 * nbytes / (time.perf_counter() - ts) / 1e9, 1)}
        del src, dst

    line = {
        "metric": "SpAMM effective GFLOP/s & SP2 solves/sec at tau=1e-6; p50/p99 solve latency",
        "value": round(value, 2), "unit": "GFLOP/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(elapsed / args.steps * 1e3, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": {"fp64": "f64", "fp32": "f32", "bf16": "bf16", "fp16": "f16",
                  "bf16x3": "bf16x3 (hi+lo, f32 accumulation)",
                  "fp16x3": "f16x3 (hi+lo, f32 accumulation)"}[prec],
        "data": "synthetic",
        "config": {"workload": f"sp2_solve water cluster {args.molecules} molecules "
                               f"(N={n}, padded {32 * (1 << int(np.ceil(np.log2(n / 32))))}), "
                               f"decay {args.decay:g} A, seed 0, {prec} leaves, tau={tau:g}",
                   "molecules": args.molecules, "n": n, "n_occ": n_occ, "tau": tau,
                   "decay": args.decay, "leaf": 32, "precision": prec},
        "sp2_solves_per_s": round(args.steps / elapsed, 3),
        "latency_ms": {"p50": round(percentile(lat, 50) * 1e3, 3),
                       "p99": round(percentile(lat, 99) * 1e3, 3)},
        "sp2": {"iterations": stats["iterations"], "stop": stats["stop"],
                "symmetric_squares": bool(stats.get("symmetric")),
                "leaf_products": execs, "leaf_products_full_squares": full_products,
                "full_square_equivalent_gflops": None if full_products is None else round(
                    LEAF_FLOP * full_products * args.steps / elapsed / 1e9, 1),
                "trace_error": tr_err, "idempotency": idem, "accuracy": accuracy},
        "phase_ms_per_step": phase_ms,
        "hbm_passes": passes,
        "multiply": multiply,
        "serving": serve,
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    if copy is not None:
        line["copy_calibration"] = copy
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
