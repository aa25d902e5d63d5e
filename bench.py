#!/usr/bin/env python3
"""Throughput of FRAM on one MI355X (gfx950).

A step is one whole solve (Algorithm 1 with SDSN, discretisation and FP64
objective) of the n = 4000 synthetic pair (Erdos-Renyi p = 0.3, U(0,1)
weights, permuted copy with N(0, 0.05) edge noise and 10% outlier nodes,
seed 2000), with A and B resident in HBM before timing starts
(fram_solve_dev).  The headline value is solves/s of the mixed-precision path
(BF16 MFMA GEMMs, FP32 SDSN, FP64 gamma/delta/objective); the same pair is
also timed with FP16 and with FP32 GEMMs.  The library records HIP events
around its launches on the solve's stream during the timed solves (recorded,
not waited for), which gives the per-kernel device times and the roofline of
the dominant kernel.

Further legs, each against the FP64 oracle timed on the host:
* n = 50 (100 seeds, FP32 GEMMs, 100 fixed iterations) and n = 1000
  (10 seeds, FP32, 100 fixed iterations): solves/s and agreement with the
  oracle's permutations;
* batched: 512 independent pairs, n ~ U{20..300}, in one fram_solve_many
  call (pairs/s, inputs uploaded inside the timed call);
* served: Poisson arrivals at 200 requests/s for 20 s after a 5 s warm-up,
  n log-uniform in [30, 2000], through the continuous-batching server
  (p50 / p99 latency from arrival to result, completed requests/s).

Prints one JSON line.  Only one GPU is supported (--gpus 1).
"""
from __future__ import annotations

import argparse
import json
import os
import pathlib
import sys
import time

ROOT = pathlib.Path(__file__).resolve().parent
sys.path.insert(0, str(ROOT))


def _hw_queues_from_argv(argv, default=16):
    """--hw-queues N (1..32), read before anything starts HIP."""
    q = default
    for i, a in enumerate(argv):
        if a == "--hw-queues" and i + 1 < len(argv):
            q = int(argv[i + 1])
        elif a.startswith("--hw-queues="):
            q = int(a.split("=", 1)[1])
    if not 1 <= q <= 32:
        raise SystemExit("--hw-queues must be between 1 and 32")
    return q


# The batched and served legs run many solves at once, one stream each; HIP
# maps a process's streams onto GPU_MAX_HW_QUEUES hardware queues, read when
# HIP starts (before the first device call below).  The benchmark sets the
# count itself (an inherited value would otherwise decide the concurrent legs).
HW_QUEUES = _hw_queues_from_argv(sys.argv[1:])
os.environ["GPU_MAX_HW_QUEUES"] = str(HW_QUEUES)


N_WORKLOAD = 4000
THETA, ITERS, TOL, GAMMA_TOL = 2.0, 100, 1e-6, 1e-6
# Second stop rule: delta has stalled at the floor set by the arithmetic's
# precision (STALL_ITERS iterations in a row without a new smallest delta,
# counted once delta <= 1e-3).  BF16/FP16 gradients make delta level off near
# 1e-4 and FP32 near 1e-6, above the tolerance the FP64 oracle reaches.
STALL_ITERS = 3
HBM_PEAK_GBS = 8000.0
COPY_BYTES = 256 << 20
MFMA_PEAK_TFLOPS = {"bf16": 2500.0, "fp16": 2500.0, "fp32": 157.3}


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def cpu_baseline(pair, T, P, source):
    """Time the FP64 oracle on a bounded sample of the same workload and scale
    it to one solve: one gradient (two n x n GEMMs), 8 SDSN passes and one
    exact LAP, scaled by T outer iterations and P SDSN passes (the oracle's
    own counts for this pair when its stored run is available)."""
    import numpy as np
    from oracle import fram64 as O
    try:
        from threadpoolctl import threadpool_info
        threads = max([i.get("num_threads", 1) for i in threadpool_info()] or [os.cpu_count()])
    except Exception:  # noqa: BLE001
        threads = os.cpu_count()
    As, Bs, _ = O.prescale(pair.A, pair.B)
    n = pair.n
    rng = np.random.default_rng(0)
    N = rng.random((n, n)) ** 8
    N /= N.sum(1, keepdims=True)
    t0 = time.perf_counter()
    X = As @ N @ Bs
    t_grad = time.perf_counter() - t0
    Y = (2.0 / 2) * X / X.max()
    k = 8
    t0 = time.perf_counter()
    for _ in range(k):
        Y = O.p2(O.p1(Y))
    t_pass = (time.perf_counter() - t0) / k
    t0 = time.perf_counter()
    O.discretize(N)
    t_lap = time.perf_counter() - t0
    t_solve = T * t_grad + P * t_pass + t_lap
    return {
        "value": 1.0 / t_solve, "unit": "solves/s", "cores": int(threads), "kind": "oracle",
        "sample": (f"FP64 oracle at n={n}: 1 gradient ({t_grad:.2f}s), {k} SDSN passes "
                   f"({t_pass:.3f}s each), 1 exact LAP ({t_lap:.2f}s); scaled to one solve "
                   f"of T={T} outer iterations and P={P} SDSN passes ({source}) -> "
                   f"{t_solve:.1f}s/solve"),
    }


def measured_traffic(kind, n, passes_per_launch):
    """HBM bytes per launch of the dominant kernel from the committed rocprofv3
    counter summary (FETCH_SIZE + WRITE_SIZE, scaled by the same counters on a
    plain copy of known size), or None when the summary is missing or was
    taken from a different version of the kernel's sources."""
    f = ROOT / "profiles" / "hbm_traffic.json"
    if not f.exists():
        return None
    try:
        rec = json.loads(f.read_text()).get(kind)
        if rec is None or rec.get("n") != n:
            return None
        if rec.get("source_sha256") != kernel_source_hash():
            return None
        return rec["bytes_per_launch"]
    except (ValueError, KeyError):
        return None


def kernel_source_hash():
    import hashlib
    h = hashlib.sha256()
    for name in ("sdsn_onchip.hip", "sdsn.hip", "sdsn_common.h"):
        h.update((ROOT / "paper_2508_00887_amd" / "csrc" / name).read_bytes())
    return h.hexdigest()


def threads_used():
    try:
        from threadpoolctl import threadpool_info
        return max([i.get("num_threads", 1) for i in threadpool_info()] or [os.cpu_count()])
    except Exception:  # noqa: BLE001
        return os.cpu_count()


def small_leg(ctx, config, seeds, cpu_seeds, cpu_iters):
    """n = 50 (config 0) or n = 1000 (config 1) workload: FP32 GEMMs, 100
    fixed outer iterations (tol = 0), every seed solved on the GPU from host
    arrays (fram_solve_ex, uploads included); the FP64 oracle is timed on the
    first `cpu_seeds` seeds with `cpu_iters` outer iterations and scaled to
    100."""
    import numpy as np
    import synth
    from oracle import fram64 as O
    pairs = list(synth.config_pairs(config, list(range(seeds))))
    ctx.solve(pairs[0].A, pairs[0].B, theta=THETA, iters=100, tol=0.0, prec="fp32")
    t0 = time.perf_counter()
    out = [ctx.solve(p.A, p.B, theta=THETA, iters=100, tol=0.0, prec="fp32") for p in pairs]
    sec = (time.perf_counter() - t0) / len(pairs)
    t0 = time.perf_counter()
    same = 0
    for p, (perm, _, _) in zip(pairs[:cpu_seeds], out):
        s_or, _, _, _ = O.solve(p.A, p.B, theta=THETA, iters=cpu_iters)
        if cpu_iters == 100:
            same += int(np.array_equal(perm, s_or))
    cpu = (time.perf_counter() - t0) / cpu_seeds * (100.0 / cpu_iters)
    n = pairs[0].n
    flops = 4.0 * n ** 3 * 100
    return {
        "n": n, "seeds": len(pairs), "solves_per_s": 1.0 / sec, "ms_per_solve": 1e3 * sec,
        "gemm_tflop_per_s_effective": flops / sec / 1e12,
        "mean_accuracy": float(np.mean([np.mean(o[0] == p.perm) for o, p in zip(out, pairs)])),
        "oracle_permutation_equal": (f"{same}/{cpu_seeds}" if cpu_iters == 100 else None),
        "gemm_precision": "fp32",
        "cpu_baseline": {"value": 1.0 / cpu, "unit": "solves/s", "cores": int(threads_used()),
                         "kind": "oracle",
                         "sample": (f"FP64 oracle, {cpu_seeds} seed(s), {cpu_iters} outer "
                                    f"iterations each, scaled to 100")},
    }


def batched_leg(Context, reps=2, cpu_pairs=16):
    """C3: one fram_solve_many call over 512 pairs; best of `reps` calls."""
    import numpy as np
    import synth
    pairs = synth.batched_pairs(512)
    ctx = Context(0)
    best, out = None, None
    for r in range(reps):
        t0 = time.perf_counter()
        perms, objs, stats = ctx.solve_many([q.A for q in pairs], [q.B for q in pairs],
                                            theta=THETA, iters=ITERS, tol=TOL, prec="bf16",
                                            stall_iters=STALL_ITERS)
        dt = time.perf_counter() - t0
        log(f"batched call {r + 1}/{reps}: {dt:.3f}s")
        if best is None or dt < best:
            best, out = dt, (perms, stats)
    ctx.close()
    perms, stats = out
    flops = sum(4.0 * q.n ** 3 * s["outer_iters"] for q, s in zip(pairs, stats))
    res = {
        "pairs": len(pairs), "seconds": best, "pairs_per_s": len(pairs) / best,
        "gemm_tflop_per_s_effective": flops / best / 1e12,
        "mean_accuracy": float(np.mean([np.mean(p == q.perm) for p, q in zip(perms, pairs)])),
        "mean_outer_iters": float(np.mean([s["outer_iters"] for s in stats])),
        "assignments_with_paths": int(sum(1 for s in stats if s["lap_paths"] > 0)),
        "lockstep_pairs": int(sum(1 for q in pairs if 2 <= q.n <= 256)),
        "onchip_projections": int(sum(s["sdsn_onchip"] for s in stats)),
        "onchip_fallbacks": int(sum(s["sdsn_fallbacks"] for s in stats)),
        "gemm_precision": "bf16",
    }
    if cpu_pairs:
        from oracle import fram64 as O
        t0 = time.perf_counter()
        for q in pairs[:cpu_pairs]:
            O.solve(q.A, q.B, theta=THETA, iters=ITERS, tol=TOL, stall_iters=STALL_ITERS)
        dt = time.perf_counter() - t0
        res["cpu_baseline"] = {"value": cpu_pairs / dt, "unit": "pairs/s", "cores": int(threads_used()),
                               "kind": "oracle",
                               "sample": f"FP64 oracle on the first {cpu_pairs} of the 512 pairs "
                                         f"(same stop rule), {dt:.1f}s"}
    return res


def served_leg(rate=200.0, duration_s=30.0, warmup_s=5.0, pool=160):
    """C4 through paper_2508_00887_amd.serve.  Graph generation for every
    request would outrun host memory (about 50 GB), so the first `pool` sizes
    of the trace are generated once and request i solves pool[i % pool]; the
    arrival times and the size distribution are those of the trace."""
    import numpy as np
    import synth
    from paper_2508_00887_amd.serve import Request, Server, summarize
    trace = synth.serve_requests(rate, duration_s, warmup_s)
    graphs = [synth.make_pair(n, 0.3, 0.05, seed) for _, n, seed in trace[:pool]]
    log(f"served: {len(trace)} requests, {len(graphs)} distinct graphs generated")
    reqs = [Request(rid=i, A=graphs[i % pool].A, B=graphs[i % pool].B, arrival=t)
            for i, (t, _, _) in enumerate(trace)]
    srv = Server(hbm_budget_bytes=64 << 30, prec="bf16", theta=THETA, iters=ITERS, tol=TOL,
                 stall_iters=STALL_ITERS)
    done = srv.replay(reqs, timeout_s=warmup_s + duration_s + 120.0)
    summ = summarize(done, warmup_s, duration_s)
    acc = [float(np.mean(r.perm == graphs[r.rid % pool].perm)) for r in done if r.perm is not None]
    summ.update(offered_rate=rate, duration_s=duration_s, warmup_s=warmup_s,
                completed=len(done), submitted=len(reqs), distinct_graphs=len(graphs),
                mean_accuracy=float(np.mean(acc)) if acc else None, gemm_precision="bf16")
    return summ


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--prec", default="bf16", choices=["bf16", "fp16"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp32", action="store_true")
    ap.add_argument("--no-small", action="store_true", help="skip the n = 50 and n = 1000 legs")
    ap.add_argument("--no-fp16", action="store_true", help="skip the second low-precision leg")
    ap.add_argument("--sdsn-mode", default="auto", choices=["auto", "stream", "onchip"])
    ap.add_argument("--no-batched", action="store_true", help="skip the 512-pair leg")
    ap.add_argument("--no-serve", action="store_true", help="skip the served leg")
    ap.add_argument("--serve-seconds", type=float, default=30.0,
                    help="timed seconds of the served leg after its 5 s warm-up (the served workload: 30)")
    ap.add_argument("--hw-queues", type=int, default=16,
                    help="hardware queues per process (GPU_MAX_HW_QUEUES), 1..32")
    ap.add_argument("--serve-rate", type=float, default=200.0,
                    help="offered requests/s of the served leg (the served workload: 200)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 256 MiB device copy (reference for HBM counters)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the FRAM hot path here is a single-GPU build "
              "(run with --gpus 1).", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    if args.copy_calibration:
        # A plain copy of known size: reads and writes COPY_BYTES per launch.
        src = torch.ones(COPY_BYTES // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_per_launch": COPY_BYTES, "launches": 3}), flush=True)
        return

    import synth
    from paper_2508_00887_amd import Context

    log("generating the n=4000 pair (seed 2000)")
    pair = next(synth.config_pairs(2, [0]))
    n = pair.n
    dA = torch.from_numpy(pair.A).cuda()
    dB = torch.from_numpy(pair.B).cuda()
    stream = torch.cuda.current_stream().cuda_stream
    ctx = Context(0)

    def solve(prec, profile=0):
        return ctx.solve_dev(dA.data_ptr(), dB.data_ptr(), n, theta=THETA, iters=ITERS, tol=TOL,
                             prec=prec, gamma_tol=GAMMA_TOL, stream=stream, profile=profile,
                             stall_iters=STALL_ITERS, sdsn_mode=args.sdsn_mode)

    keys = ("ms_gemm", "gemm_launches", "ms_sdsn", "sdsn_launches", "sdsn_passes", "ms_update",
            "ms_stats", "outer_iters")

    def timed(prec, steps, warmup):
        """Wall time per solve over `steps` solves; the library records HIP
        events around its launches on the solve's stream during the same
        solves (profile = 2: recorded, not waited for)."""
        for w in range(warmup):
            solve(prec)
            log(f"warmup {prec} {w + 1}/{warmup} done")
        torch.cuda.synchronize()
        tot = dict.fromkeys(keys, 0.0)
        t0 = time.perf_counter()
        out = None
        for s in range(steps):
            out = solve(prec, profile=2)
            for k in keys:
                tot[k] += out[2][k]
            log(f"step {prec} {s + 1}/{steps} done")
        torch.cuda.synchronize()
        sec = (time.perf_counter() - t0) / steps
        flops = 4.0 * n ** 3 * tot["outer_iters"]
        prof = dict(
            gemm_tflops=flops / (tot["ms_gemm"] * 1e-3) / 1e12,
            gemm_us_per_launch=1e3 * tot["ms_gemm"] / max(1, tot["gemm_launches"]),
            sdsn_launches=int(tot["sdsn_launches"]), sdsn_passes=int(tot["sdsn_passes"]),
            sdsn_us_per_launch=1e3 * tot["ms_sdsn"] / max(1, tot["sdsn_launches"]),
            sdsn_us_per_pass=1e3 * tot["ms_sdsn"] / max(1, tot["sdsn_passes"]),
            ms_per_solve={k: tot[k] / steps for k in ("ms_gemm", "ms_sdsn", "ms_update",
                                                      "ms_stats")},
        )
        return sec, out, prof

    sec_mixed, (perm, obj, st), pm = timed(args.prec, args.steps, args.warmup)
    acc = float(np.mean((perm == pair.perm)[pair.inlier]))
    res = {}
    prof = {args.prec: pm}
    other = "fp16" if args.prec == "bf16" else "bf16"
    if not args.no_fp16:
        sec16, (perm16, obj16, st16), prof[other] = timed(other, max(1, args.steps // 2), 1)
        res[other] = dict(solves_per_s=1.0 / sec16, ms_per_solve=1e3 * sec16,
                          outer_iters=st16["outer_iters"], sdsn_passes=st16["sdsn_passes"],
                          objective=obj16,
                          accuracy=float(np.mean((perm16 == pair.perm)[pair.inlier])))
    if not args.no_fp32:
        sec32, (perm32, obj32, st32), prof["fp32"] = timed("fp32", max(1, args.steps // 2), 1)
        res["fp32"] = dict(solves_per_s=1.0 / sec32, ms_per_solve=1e3 * sec32,
                           outer_iters=st32["outer_iters"], sdsn_passes=st32["sdsn_passes"],
                           objective=obj32,
                           accuracy=float(np.mean((perm32 == pair.perm)[pair.inlier])))
    # Algorithmic bytes of one SDSN pass: read X and write Y once (8 n^2).  The
    # on-chip kernel runs a whole projection per launch and keeps X on chip,
    # so its streaming-equivalent rate can exceed the HBM roofline.
    pass_bytes = 8.0 * n * n
    bytes_per_launch = pass_bytes * pm["sdsn_passes"] / max(1, pm["sdsn_launches"])
    achieved = bytes_per_launch / (pm["sdsn_us_per_launch"] * 1e-6) / 1e9
    onchip = pm["sdsn_launches"] != pm["sdsn_passes"]
    traffic = measured_traffic("sdsn_onchip" if onchip else "sdsn_stream", n,
                               pm["sdsn_passes"] / max(1, pm["sdsn_launches"]))
    golden = ROOT / "tests" / "golden" / "fram_c2_seed2000.json"
    rel_err, g = None, None
    if golden.exists():
        g = json.loads(golden.read_text())
        rel_err = abs(obj - g["objective"]) / abs(g["objective"])
    line = {
        "metric": "solves/s + GEMM TFLOP/s mixed vs FP32 at n=4000, equal accuracy; serve p99 ms",
        "value": 1.0 / sec_mixed,
        "unit": "solves/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": 1e3 * sec_mixed,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": args.prec, "data": "synthetic",
        "config": {"workload": "single pair n=4000, ER p=0.3, U(0,1) weights, noise 0.05, "
                               "10% outliers, seed 2000",
                   "n": n, "theta": THETA, "iters_cap": ITERS, "tol": TOL,
                   "stall_iters": STALL_ITERS, "gamma_tol": GAMMA_TOL,
                   "gemm_precision": args.prec, "sdsn_mode": args.sdsn_mode,
                   "hw_queues": HW_QUEUES},
        "outer_iters": st["outer_iters"], "sdsn_passes": st["sdsn_passes"],
        "accuracy": acc, "objective": obj, "rel_obj_err_vs_oracle": rel_err,
        "lap_paths": st["lap_paths"],
        "gemm_tflops": {k: v["gemm_tflops"] for k, v in prof.items()},
        "profile": prof,
        "roofline": {"bound": "hbm",
                     "kernel": "sdsn_onchip_kernel<256> (one launch per projection)" if onchip
                     else "sdsn tile_kernel (one launch per pass)",
                     "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "bytes_per_launch": bytes_per_launch,
                     "avg_launch_us": pm["sdsn_us_per_launch"],
                     "passes_per_launch": pm["sdsn_passes"] / max(1, pm["sdsn_launches"])},
        "oracle_accuracy": g["accuracy"] if g else None,
        "oracle_outer_iters": g["outer_iters"] if g else None,
        "stop_rule": {"tol": TOL, "stall_iters": STALL_ITERS, "iters_cap": ITERS},
    }
    if other in res:
        line[other] = res[other]
        if g:
            line[other]["rel_obj_err_vs_oracle"] = (abs(res[other]["objective"] - g["objective"])
                                                    / abs(g["objective"]))
    if "fp32" in res:
        line["fp32"] = res["fp32"]
        line["speedup_vs_fp32"] = line["value"] / res["fp32"]["solves_per_s"]
        if g:
            line["fp32"]["rel_obj_err_vs_oracle"] = (abs(res["fp32"]["objective"] - g["objective"])
                                                     / abs(g["objective"]))
    if not args.no_small:
        log("n = 50 leg (100 seeds)")
        line["small_n50"] = small_leg(ctx, 0, 100, 20, 100)
        log("n = 1000 leg (10 seeds)")
        line["small_n1000"] = small_leg(ctx, 1, 10, 1, 10)
    if not args.no_batched:
        log("batched leg: 512 pairs")
        line["batched"] = batched_leg(Context)
    if not args.no_serve:
        log("served leg")
        line["served"] = served_leg(rate=args.serve_rate, duration_s=args.serve_seconds)
    if not args.no_cpu_baseline:
        if g is not None:
            T, P, src = g["outer_iters"], int(sum(g["sdsn_passes"])), "the oracle's stored run"
        else:
            T, P, src = st["outer_iters"], st["sdsn_passes"], "the GPU solve's counts"
        log("timing the CPU oracle sample")
        line["cpu_baseline"] = cpu_baseline(pair, T, P, src)
    ctx.close()
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
