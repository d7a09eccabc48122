#!/usr/bin/env python3
"""Benchmark of the ImLoc pose-estimation hot path (lift + LO-RANSAC PnP,
arXiv 2601.04185 Sec. 3.3) on one MI355X.

A step is one call of the fused batched form for 256 queries: every query's
Philox sampling, float64 P3P, float32 scoring, top-8 selection, float64
Gauss-Newton local optimisation, Cauchy refinement and inlier mask run in
shared launches, replayed as one captured HIP graph.  The queries have
correspondence counts uniform in [5,000, 80,000] and inlier ratios uniform in
[10%, 60%], 4,096 samples each, a 4 px threshold; their correspondences are
resident in HBM before the timed region.

Prints one JSON line: whole-job scored residuals/s (value) with queries/s and
batch latency, the roofline of the scoring kernel (its launch timed with HIP
events on the library's stream), pose recall against the synthetic truth and
pose error against the float64 oracle, the oracle timed on the host cores (all
of them and one), and sub-legs: the single large query, the plain
one-query-per-call form, the serving loop, lifting + RANSAC, the paper's own
settings, mapping-time depth and the multi-camera rig.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import statistics
import subprocess
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "scored residuals/s and queries/s at 1 GPU; p50/p99 query latency at fixed accuracy"
PEAK_F32_TFLOPS = 157.3    # published FP32 vector peak of the MI355X (256 CUs at 2.4 GHz)
PEAK_HBM_GBS = 8000.0      # published HBM3E bandwidth
FLOP_PER_RESIDUAL = 27     # 9 FMA projection + 2 FMA residual + MUL+FMA square + 2 MUL threshold
FLOP_PER_INLIER = 5        # reciprocal, multiply, FMA, add of the truncated cost
ROT_TOL_DEG, T_TOL_REL = 1e-3, 1e-4
RECALL_THRESHOLDS = ((0.25, 2.0), (0.5, 5.0), (1.0, 10.0))   # (m, deg)


def _file_hash(path):
    with open(path, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def _traffic(kernel_src, workload, shape):
    """HBM bytes per launch from the committed counter summary of this
    workload and launch shape, if it was taken on the current source of the
    kernel; else None."""
    ct, pts, wg = shape
    p = os.path.join(ROOT, "profiles", f"score_{workload}_traffic_{ct}x{pts}x{wg}.txt")
    if not os.path.exists(p):
        return None
    d = {}
    for line in open(p):
        if ":" in line and not line.startswith(("#", " ")):
            k, v = line.split(":", 1)
            d[k.strip()] = v.strip()
    if (d.get("workload") != workload or d.get("kernel_src_sha256_16") != _file_hash(kernel_src)
            or d.get("candidates_per_item") != str(ct) or d.get("points_per_item") != str(pts)
            or d.get("workgroups") != str(wg)):
        return None
    try:
        return float(d["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def set_shape(ctx, spec):
    """--score-shape CT,WG[,PTS]: candidates per item, workgroups, correspondences per item."""
    v = [int(x) for x in spec.split(",")]
    ctx.set_score_tuning(v[0], v[1])
    if len(v) > 2:
        ctx.set_score_points(v[2])


def copy_shape(src, dst):
    dst.set_score_tuning(*src.score_tuning())
    dst.set_score_points(src.score_points())


def _score_kernel_name(ct):
    """The scoring kernel's name for a candidate tile (0: the tile is picked per round)."""
    return f"score_kernel<{ct}>" if ct > 0 else "score_kernel<CT picked per round>"


def _rot_deg(Ra, Rb):
    import numpy as np
    M = Ra @ Rb.T
    s = 0.5 * np.array([M[2, 1] - M[1, 2], M[0, 2] - M[2, 0], M[1, 0] - M[0, 1]])
    return float(np.degrees(np.arctan2(np.linalg.norm(s), 0.5 * (np.trace(M) - 1.0))))


def vs_oracle(pairs):
    """pairs: [(R, t, oracle dict)].  Largest rotation error (deg), largest
    translation error relative to max(|t_oracle|, 1 m), and whether every pose
    is within 1e-3 deg and 1e-4 relative translation of the oracle."""
    import numpy as np
    if not pairs:
        return None
    rot = [_rot_deg(R, ref["R"]) for R, t, ref in pairs]
    rel = [float(np.linalg.norm(t - ref["t"]) / max(1.0, np.linalg.norm(ref["t"]))) for R, t, ref in pairs]
    same_status = all((ref["status"] == 0) for _, _, ref in pairs)
    return dict(checked=len(pairs), max_rot_err_vs_oracle_deg=max(rot), max_t_rel_err_vs_oracle=max(rel),
                within_tolerance=bool(same_status and max(rot) <= ROT_TOL_DEG and max(rel) <= T_TOL_REL))


def recall(pairs):
    """pairs: [(R, t, R_true, t_true)] -> recall at the paper's thresholds and
    the median errors (cm, deg)."""
    import numpy as np
    if not pairs:
        return None
    rot = np.array([_rot_deg(R, Rt) for R, t, Rt, tt in pairs])
    tr = np.array([float(np.linalg.norm(t - tt)) for R, t, Rt, tt in pairs])
    out = {f"recall_{m}m_{d}deg": float(np.mean((tr <= m) & (rot <= d))) for m, d in RECALL_THRESHOLDS}
    out.update(median_t_err_cm=float(np.median(tr) * 100.0), median_rot_err_deg=float(np.median(rot)),
               queries=len(pairs))
    return out


def cpu_model():
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for line in out.splitlines():
            if line.startswith("Model name:"):
                return line.split(":", 1)[1].strip()
    except (OSError, subprocess.SubprocessError):
        pass
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def host_threads():
    env = os.environ.get("OMP_NUM_THREADS", "")
    if env.isdigit() and int(env) > 0:
        return int(env)
    try:
        return len(os.sched_getaffinity(0))
    except AttributeError:
        return os.cpu_count() or 1


def oracle_params(prm):
    """Host dict of imloc_ransac_params fields the oracle takes."""
    keys = ("threshold_px", "fixed_samples", "batch", "min_iters", "max_iters", "confidence", "lo_top_k",
            "lo_iters", "max_score_points", "final_iters", "cauchy_scale_px", "exhaustive", "seed", "query_id")
    return {k: getattr(prm, k) for k in keys}


def timed_oracle(run, reps=5, warmup=1):
    """Median wall time of `reps` runs after `warmup` runs; the last result."""
    times, res = [], None
    for i in range(warmup + reps):
        t0 = time.perf_counter()
        res = run()
        if i >= warmup:
            times.append(time.perf_counter() - t0)
    return statistics.median(times), res


# ---------------------------------------------------------------- headline --
def headline(pk, args):
    """The 256-query batch in the fused form (the step), its scoring roofline,
    accuracy, the plain form and the CPU baseline."""
    import numpy as np
    import torch
    from paper_2601_04185_amd import synth
    qs = synth.config3_batch(256)
    ds = [pk.to_device(q) for q in qs]
    Ks = [q.K for q in qs]
    prms = [pk.make_params(threshold_px=4.0, fixed_samples=4096, batch=4096, lo_top_k=8, query_id=i)
            for i in range(len(qs))]
    # the batch's device arrays and their host descriptors are set up once,
    # like the device buffers of a serving process; every call still builds,
    # uploads and runs the whole batch
    batch = pk.BatchQueries(ds, Ks, prms)
    run = lambda c: pk.imloc_lo_ransac_pnp_batch(c, batch, arrays=True)
    ctx = pk.Context(0, graphs=True)  # fixed samples: one captured hipGraph per batch shape, replayed
    tuned = None
    if args.score_shape:
        set_shape(ctx, args.score_shape)
    elif not args.no_tune:
        from paper_2601_04185_amd.autotune import tune_scoring
        tuned = tune_scoring(ctx, lambda c: run(c)[2], reps=args.tune_reps)
    for _ in range(args.warmup):
        run(ctx)
    torch.cuda.synchronize()
    lat = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        s = time.perf_counter()
        status, poses, stats = run(ctx)
        lat.append(time.perf_counter() - s)
    torch.cuda.synchronize()
    total = time.perf_counter() - t0
    assert all(x == 0 for x in status), status
    res = int(stats["residuals"].sum())
    inl = int(stats["inlier_residuals"].sum())
    cand = int(stats["candidates"].sum())
    poses = [(p[:9].reshape(3, 3), p[9:]) for p in poses]

    # the scoring kernel's launch, HIP events on the library's stream (one round: one launch per call)
    tctx = pk.Context(0, timing=True)
    copy_shape(ctx, tctx)
    launch, stage = [], None
    for _ in range(max(5, min(args.steps, 20))):
        _, _, st_t = run(tctx)
        launch.append(float(st_t[0]["ms_score"]) / max(1, int(st_t[0]["score_launches"])))
        stage = {k: float(st_t[0][k]) for k in st_t.dtype.names}
    launch_ms = statistics.median(launch)
    flops = FLOP_PER_RESIDUAL * res + FLOP_PER_INLIER * inl
    achieved = flops / (launch_ms * 1e-3) / 1e12
    ct, wg = ctx.score_tuning()
    pts = ctx.score_points()
    kernel_src = os.path.join(ROOT, "paper_2601_04185_amd", "csrc", "score.hip")
    roofline = dict(bound="alu", achieved=round(achieved, 3), peak=PEAK_F32_TFLOPS, unit="TFLOP/s",
                    frac=round(achieved / PEAK_F32_TFLOPS, 4), traffic=_traffic(kernel_src, "batch256", (ct, pts, wg)),
                    kernel=_score_kernel_name(ct), launch_ms=round(launch_ms, 4), flop_per_launch=int(flops),
                    residuals_per_launch=res, residuals_per_s_kernel=round(res / (launch_ms * 1e-3), 1),
                    launch_shape=dict(candidates_per_item=ct, points_per_item=pts, workgroups=wg))

    out = dict(metric=METRIC, value=round(res * args.steps / total, 1), unit="residuals/s", n_gpus=1,
               steps=args.steps, warmup=args.warmup, ms_per_step=round(total / args.steps * 1e3, 4),
               higher_is_better=True, scaling="weak", vs_baseline=None, dtype="f32", dtype_solve="f64",
               data="synthetic",
               config=dict(workload="256-query batch, fused persistent form replayed as one hipGraph: "
                                    "correspondences uniform in [5,000, 80,000] per query "
                                    f"(total {sum(q.n for q in qs):,}), inlier ratios uniform in [10%, 60%], "
                                    "sigma 1 px, 4,096 P3P samples each, tau 4 px, LO on the top 8, float32 "
                                    "scoring, float64 P3P/LO/refine",
                           queries=len(qs), correspondences=sum(q.n for q in qs), samples_per_query=4096,
                           candidates=cand, residuals_per_step=res, parallelism="1 GPU",
                           graph_captures_replays=list(ctx.graph_counters())),
               queries_per_s=round(len(qs) * args.steps / total, 2),
               p50_ms=round(float(np.percentile(lat, 50)) * 1e3, 4),
               p99_ms=round(float(np.percentile(lat, 99)) * 1e3, 4),
               latency_note="p50/p99 of one whole 256-query batch call (every query of the batch completes together)",
               stage_ms={k: round(stage[k], 4) for k in ("ms_sample", "ms_score", "ms_select", "ms_lo", "ms_refine",
                                                         "ms_total")},
               roofline=roofline)
    if tuned is not None:
        out["autotune"] = dict(best=tuned["best"], table=tuned["table"], reps=args.tune_reps)

    acc = dict(vs_truth=recall([(R, t, q.R, q.t) for (R, t), q in zip(poses, qs)]))
    # the plain form: one query per call, same seeds and parameters
    if not args.no_plain:
        pctx = pk.Context(0, graphs=True)
        copy_shape(ctx, pctx)
        for i in range(4):
            pk.imloc_lo_ransac_pnp(pctx, ds[i], Ks[i], prms[i])
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        plain = [pk.imloc_lo_ransac_pnp(pctx, ds[i], Ks[i], prms[i]) for i in range(len(qs))]
        t_plain = time.perf_counter() - t0
        same = all(np.array_equal(plain[i][1], poses[i][0]) and np.array_equal(plain[i][2], poses[i][1])
                   for i in range(len(qs)))
        out["plain_form"] = dict(ms_per_256=round(t_plain * 1e3, 3), queries_per_s=round(len(qs) / t_plain, 2),
                                 fused_speedup=round(t_plain / (total / args.steps), 3),
                                 poses_identical_to_fused=bool(same))
    if not args.no_cpu_baseline:
        import oracle
        n_all = host_threads()
        sub = list(range(args.cpu_queries))
        opr = [oracle_params(prms[i]) for i in sub]
        oracle.set_threads(n_all)
        used_all = oracle.max_threads()
        t_all, refs = timed_oracle(lambda: [oracle.lo_ransac_pnp(qs[i].corr(), Ks[i], **opr[k])
                                            for k, i in enumerate(sub)])
        res_all = sum(r["residuals"] for r in refs)
        oracle.set_threads(1)
        t_one, ref1 = timed_oracle(lambda: oracle.lo_ransac_pnp(qs[0].corr(), Ks[0], **opr[0]))
        oracle.set_threads(n_all)
        out["cpu_baseline"] = dict(
            value=round(res_all / t_all, 1), unit="residuals/s", cores=used_all, kind="oracle",
            sample=f"queries 0-{len(sub) - 1} of the 256-query batch ({sum(qs[i].n for i in sub):,} "
                   f"correspondences, {res_all:,} residuals), float64 C oracle with OpenMP over candidates; "
                   f"median of 5 runs after 1 warm-up; residuals/s is the rate over the sample (the batch "
                   f"would take {res / (res_all / t_all):.1f} s at it)",
            queries_per_s=round(len(sub) / t_all, 3), cpu_model=cpu_model(),
            one_core=dict(value=round(ref1["residuals"] / t_one, 1), unit="residuals/s", cores=1,
                          sample=f"query 0 of the batch ({qs[0].n:,} correspondences, {ref1['residuals']:,} "
                                 "residuals), median of 5 runs after 1 warm-up",
                          queries_per_s=round(1.0 / t_one, 3)))
        acc["vs_oracle"] = vs_oracle([(poses[i][0], poses[i][1], refs[k]) for k, i in enumerate(sub)])
    out["accuracy"] = acc
    return out


# -------------------------------------------------------------- sub-legs --
def single_large_leg(pk, args):
    """The single large query: 10 views x 5,000 = 50,000 correspondences, 25%
    inliers, 10,000 samples, 6 px, LO top-8 (latency, its own autotuned
    scoring shape, its scoring launch, pose error against the oracle)."""
    import numpy as np
    import torch
    import oracle
    from paper_2601_04185_amd import synth
    q = synth.config2_single_large()
    d = pk.to_device(q)
    kw = dict(threshold_px=6.0, fixed_samples=10000, batch=10000, lo_top_k=8)
    prm = pk.make_params(**kw)
    ctx = pk.Context(0, graphs=True)
    tuned = None
    if not args.no_tune:
        from paper_2601_04185_amd.autotune import tune_scoring
        tuned = tune_scoring(ctx, lambda c: pk.imloc_lo_ransac_pnp(c, d, q.K, prm)[3])
    for _ in range(5):
        pk.imloc_lo_ransac_pnp(ctx, d, q.K, prm)
    torch.cuda.synchronize()
    lat = []
    for _ in range(50):
        s = time.perf_counter()
        rc, R, t, st = pk.imloc_lo_ransac_pnp(ctx, d, q.K, prm)
        lat.append(time.perf_counter() - s)
    tctx = pk.Context(0, timing=True)
    copy_shape(ctx, tctx)
    per, inl, stage = [], [], None
    for _ in range(20):
        _, _, _, s2 = pk.imloc_lo_ransac_pnp(tctx, d, q.K, prm)
        per.append(s2["ms_score"])
        inl.append(s2["inlier_residuals"])
        stage = s2
    launch_ms = statistics.median(per)
    flops = FLOP_PER_RESIDUAL * st["residuals"] + FLOP_PER_INLIER * statistics.median(inl)
    ref = oracle.lo_ransac_pnp(q.corr(), q.K, **oracle_params(prm))
    out = dict(workload="single large query: 10 views x 5,000 = 50,000 correspondences, 25% inliers, sigma 1.5 px, "
                        "10,000 P3P samples, tau 6 px, LO on the top 8, float32 scoring, float64 P3P/LO/refine",
               status=int(rc), p50_ms=round(float(np.percentile(lat, 50)) * 1e3, 4),
               p99_ms=round(float(np.percentile(lat, 99)) * 1e3, 4), queries_per_s=round(len(lat) / sum(lat), 2),
               candidates=st["candidates"], residuals=st["residuals"],
               residuals_per_s=round(st["residuals"] / float(np.median(lat)), 1),
               stage_ms={k: round(stage[k], 4) for k in ("ms_sample", "ms_score", "ms_select", "ms_lo", "ms_refine",
                                                         "ms_total")},
               score_launch=dict(kernel=_score_kernel_name(ctx.score_tuning()[0]), launch_ms=round(launch_ms, 4),
                                 achieved_tflops=round(flops / (launch_ms * 1e-3) / 1e12, 3),
                                 frac_of_peak=round(flops / (launch_ms * 1e-3) / 1e12 / PEAK_F32_TFLOPS, 4),
                                 launch_shape=dict(candidates_per_item=ctx.score_tuning()[0],
                                                   points_per_item=ctx.score_points(),
                                                   workgroups=ctx.score_tuning()[1])),
               accuracy=dict(vs_oracle=vs_oracle([(R, t, ref)]), vs_truth=recall([(R, t, q.R, q.t)])),
               graph_captures_replays=list(ctx.graph_counters()))
    if tuned is not None:
        out["autotune_best"] = tuned["best"]
    return out


def single_small_leg(pk):
    """The float64 parity configuration: 2,000 correspondences, 40% inliers,
    1,024 samples, 4 px, LO top-1, every step in float64."""
    import numpy as np
    import oracle
    from paper_2601_04185_amd import synth
    q = synth.config1_single_small()
    d = pk.to_device(q)
    prm = pk.make_params(threshold_px=4.0, fixed_samples=1024, batch=1024, lo_top_k=1, precision=1)
    ctx = pk.Context(0, graphs=True)
    for _ in range(3):
        pk.imloc_lo_ransac_pnp(ctx, d, q.K, prm)
    lat = []
    for _ in range(20):
        s = time.perf_counter()
        rc, R, t, st = pk.imloc_lo_ransac_pnp(ctx, d, q.K, prm)
        lat.append(time.perf_counter() - s)
    ref = oracle.lo_ransac_pnp(q.corr(), q.K, **oracle_params(prm))
    return dict(workload="2,000 correspondences, 40% inliers, sigma 1 px, 1,024 P3P samples, tau 4 px, LO top-1, "
                         "every step float64",
                status=int(rc), p50_ms=round(float(np.percentile(lat, 50)) * 1e3, 4),
                residuals=st["residuals"], best_h_j_equal_oracle=bool(st["best_h"] == ref["best_h"] and
                                                                       st["best_j"] == ref["best_j"]),
                accuracy=dict(vs_oracle=vs_oracle([(R, t, ref)]), vs_truth=recall([(R, t, q.R, q.t)])))


def serving_leg(pk, args):
    """Continuous batching at the serving workload's scale: 2,000 queries
    with log-normal sizes in [2,000, 200,000] and inlier ratios in [5%, 60%],
    adaptive stopping at 99.9%.  First the saturation rate (all queued at
    once), then Poisson arrivals at 0.25, 0.5, 0.75 and 0.9 of it; latency =
    completion - arrival over the queries after the first 200."""
    import numpy as np
    import oracle
    from paper_2601_04185_amd import synth
    n_q, warm, max_slots = args.serving_queries, args.serving_queries // 10, 64
    arr_unit, ns, eps = synth.serving_arrivals(n_q, rate_qps=1.0)
    qs = [synth.make_query(1005 * 1000 + i, int(ns[i]), float(eps[i]), 1.0) for i in range(n_q)]
    ds = [pk.to_device(q) for q in qs]
    P = [pk.make_params(threshold_px=4.0, confidence=0.999, batch=1024, min_iters=1024, max_iters=100000,
                        lo_top_k=8, query_id=i) for i in range(n_q)]
    srv = pk.Server(0, max_slots=max_slots, max_top_k=8, max_n=200000)

    def run(arrivals):
        t0 = time.perf_counter()
        done_t, tick, i, steps, occ, results = {}, {}, 0, 0, [], {}
        while len(done_t) < n_q:
            now = time.perf_counter() - t0
            while i < n_q and arrivals[i] <= now:
                tick[srv.submit(ds[i], qs[i].K, P[i])] = i
                i += 1
            done, resident, queued = srv.step()
            steps += 1
            occ.append(resident)
            now = time.perf_counter() - t0
            for tk in done:
                done_t[tick[tk]] = now
                results[tick[tk]] = srv.poll(tk)
            if resident == 0 and queued == 0 and i < n_q:
                time.sleep(max(0.0, arrivals[i] - (time.perf_counter() - t0)))
        lat = np.array([done_t[k] - arrivals[k] for k in range(n_q)])
        span = max(done_t[k] for k in range(warm, n_q)) - arrivals[warm]
        return lat[warm:], (n_q - warm) / span, steps, float(np.mean(occ)), results

    _, _, _, _, _ = run(np.zeros(n_q))  # warm-up pass
    t0 = time.perf_counter()
    _, _, sat_steps, sat_occ, _ = run(np.zeros(n_q))
    sat_qps = n_q / (time.perf_counter() - t0)
    loads, served = [], None
    for load in (0.25, 0.5, 0.75, 0.9):
        rate = load * sat_qps
        lat, qps, steps, occ, results = run(arr_unit / rate)
        loads.append(dict(load=load, offered_queries_per_s=round(rate, 1), queries_per_s=round(qps, 1),
                          p50_ms=round(float(np.percentile(lat, 50)) * 1e3, 3),
                          p99_ms=round(float(np.percentile(lat, 99)) * 1e3, 3), latency_samples=int(lat.size),
                          rounds=steps, mean_resident=round(occ, 1)))
        served = results
    # every checked served result equals the query run alone
    ctx = pk.Context(0)
    check = list(range(0, n_q, max(1, n_q // 12)))
    ident = True
    for i in check:
        rc, R, t, st = pk.imloc_lo_ransac_pnp(ctx, ds[i], qs[i].K, P[i])
        ident &= bool(served[i][0] == rc and np.array_equal(served[i][1], R) and np.array_equal(served[i][2], t))
    # float64 oracle on a bounded sample: the first 8 queries with at least 25% inliers and at most 40,000 points
    sample = [i for i in range(n_q) if eps[i] >= 0.25 and ns[i] <= 40000][:8]
    pairs = [(served[i][1], served[i][2], oracle.lo_ransac_pnp(qs[i].corr(), qs[i].K, **oracle_params(P[i])))
             for i in sample]
    srv.close()
    return dict(workload=f"{n_q} queries, correspondences log-normal in [2,000, 200,000] (mean {int(np.mean(ns)):,}), "
                         "inlier ratios uniform in [5%, 60%], sigma 1 px, adaptive stopping at 99.9% (batches of "
                         f"1,024, cap 100,000), tau 4 px, LO top-8, {max_slots} slots; latency over queries "
                         f"{warm}..{n_q - 1}",
                saturation_queries_per_s=round(sat_qps, 1), saturation_rounds=sat_steps,
                saturation_mean_resident=round(sat_occ, 1), loads=loads,
                served_equals_alone=bool(ident), checked_alone=len(check),
                accuracy=dict(vs_oracle=vs_oracle(pairs),
                              oracle_sample="the first 8 queries with inlier ratio >= 25% and <= 40,000 points",
                              vs_truth=recall([(served[i][1], served[i][2], qs[i].R, qs[i].t) for i in range(n_q)])))


def e2e_leg(pk, steps=10):
    """Lifting plus RANSAC: 20 database RGB-D views (640x480 float32 depth) of
    a box-and-plane scene, 8,000 query-to-database matches per view, lifted on
    the GPU, then LO-RANSAC PnP with adaptive stopping at 99.9%."""
    import numpy as np
    import torch
    import oracle
    from paper_2601_04185_amd import synth
    wl = synth.config4_lift_scene()
    m = {k: torch.from_numpy(v).cuda() for k, v in wl.matches.items()}
    depth = torch.from_numpy(wl.depth).cuda()
    prm = pk.make_params(threshold_px=4.0, batch=1024, min_iters=1024, max_iters=100000, confidence=0.999,
                         lo_top_k=8)
    ctx = pk.Context(0)
    n_match = int(m["q_u"].numel())
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)

    def once():
        t0 = time.perf_counter()
        ev0.record()  # the context enqueues on torch's current stream
        g = pk.imloc_lift(ctx, m, depth, wl.cams, wl.poses)
        ev1.record()
        t1 = time.perf_counter()
        corr = {k: g[k] for k in ("u", "v", "X", "Y", "Z", "w")}
        rc, R, t, st = pk.imloc_lo_ransac_pnp(ctx, corr, wl.K_query, prm)
        return t1 - t0, time.perf_counter() - t0, ev0.elapsed_time(ev1), g, rc, R, t, st

    once()
    torch.cuda.synchronize()
    lift_s, tot_s, lift_dev = [], [], []
    for _ in range(steps):
        a, b, dev_ms, g, rc, R, t, st = once()
        lift_s.append(a)
        tot_s.append(b)
        lift_dev.append(dev_ms)
    n_lifted = int(g["n"])
    tl, tt, td = statistics.median(lift_s), statistics.median(tot_s), statistics.median(lift_dev)
    # algorithmic bytes: 24 B of match read, four 4-byte depth taps, 28 B written per kept correspondence
    lift_bytes = n_match * (24 + 16) + n_lifted * 28
    # the oracle lifts the same matches and runs RANSAC on the GPU's lifted correspondences
    ref_lift = oracle.lift(wl.matches, wl.depth, wl.cams, wl.poses)
    src_equal = bool(ref_lift["src"].size == n_lifted and
                     np.array_equal(ref_lift["src"], g["src"][:n_lifted].cpu().numpy()))
    corr_np = {k: g[k][:n_lifted].cpu().numpy() for k in ("u", "v", "X", "Y", "Z", "w")}
    ref = oracle.lo_ransac_pnp(corr_np, wl.K_query, **oracle_params(prm))
    return dict(workload=f"{wl.depth.shape[0]} database views 640x480, {n_match:,} matches (30% correct), lifted to "
                         f"{n_lifted:,} correspondences, adaptive stopping at 99.9%, tau 4 px, LO top-8",
                status=int(rc), ms_per_query=round(tt * 1e3, 3), queries_per_s=round(1.0 / tt, 2),
                lift_device_ms=round(td, 4), lift_matches_per_s_device=round(n_match / (td * 1e-3), 1),
                lift_gb_per_s_device=round(lift_bytes / (td * 1e-3) / 1e9, 2),
                lift_device_note="events on the stream around the whole call: the view-table upload, three "
                                 "kernels and the 4-byte count the binding reads back (the kernels alone: "
                                 "profiles/lift_kernel_trace.md)",
                lift_ms_incl_host=round(tl * 1e3, 4), lift_bytes_algorithmic=int(lift_bytes),
                lift_src_equal_oracle=src_equal, samples=st["samples"], residuals=st["residuals"],
                best_count=st["best_count"],
                accuracy=dict(vs_oracle=vs_oracle([(R, t, ref)]), vs_truth=recall([(R, t, wl.R, wl.t)])))


def paper_mode_leg(pk, steps=10):
    """The paper's own LO-RANSAC settings on the single large query with
    confidence weights: stride subsample to 10,000 scoring points, batches of
    1,000, local optimisation of a new best (top 1), stop at 100,000 samples or
    confidence 1 - 1e-4, Cauchy refinement over all 50,000 points."""
    import numpy as np
    import torch
    import oracle
    from paper_2601_04185_amd import synth
    q = synth.make_query(1002, 50000, 0.25, 1.5, weights="conf", n_views=10)
    d = pk.to_device(q)
    prm = pk.paper_params(6.0)
    ctx = pk.Context(0)
    for _ in range(2):
        pk.imloc_lo_ransac_pnp(ctx, d, q.K, prm)
    torch.cuda.synchronize()
    lat = []
    for _ in range(steps):
        t0 = time.perf_counter()
        rc, R, t, st = pk.imloc_lo_ransac_pnp(ctx, d, q.K, prm)
        lat.append(time.perf_counter() - t0)
    ref = oracle.lo_ransac_pnp(q.corr(), q.K, **oracle_params(prm))
    return dict(workload="50,000 correspondences (10 views x 5,000), 25% inliers, sigma 1.5 px, confidence weights; "
                         "scoring subsample 10,000, batches of 1,000, LO top-1, confidence 0.9999, cap 100,000, "
                         "tau 6 px",
                status=int(rc), p50_ms=round(float(np.percentile(lat, 50)) * 1e3, 3),
                p99_ms=round(float(np.percentile(lat, 99)) * 1e3, 3),
                queries_per_s=round(steps / sum(lat), 2), samples=st["samples"], batches=st["batches"],
                samples_equal_oracle=bool(st["samples"] == ref["samples"]), residuals=st["residuals"],
                accuracy=dict(vs_oracle=vs_oracle([(R, t, ref)]), vs_truth=recall([(R, t, q.R, q.t)])),
                paper_context="the paper's RANSAC loop takes about 200 ms per query on an RTX 4090 "
                              "(CPU sampling and P3P, GPU scoring); context, not a target")


def mapping_depth_leg(pk, steps=10):
    """Mapping-time depth of one 560 x 560 mapping image from dense matches in
    10 covisible views (70% correct, 0.5 px noise): 1-DoF triangulation."""
    import numpy as np
    import torch
    import oracle
    from paper_2601_04185_amd import synth
    w = synth.dense_match_scene(n_views=10, width=560, height=560, seed=1006)
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    mu, mv, cf = dev(w.mu), dev(w.mv), dev(w.conf)
    ctx = pk.Context(0)
    run = lambda: pk.imloc_triangulate_depth(ctx, w.K0, w.T0, w.Ks, w.Ts, mu, mv, cf, want_codes=True)
    run()
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record()
    for _ in range(steps):
        g = run()
    ev1.record()
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1) / steps
    d = g["depth"].cpu().numpy().astype(np.float64)
    inl = g["inliers"].cpu().numpy()
    fin = np.isfinite(w.depth_true)
    ok = d > 0
    rel = np.abs(d[ok & fin] / w.depth_true[ok & fin] - 1)
    r = oracle.triangulate(w.K0, w.T0, w.Ks, w.Ts, w.mu, w.mv, w.conf)
    un = ~r["ambiguous"]
    both = un & (r["depth"] > 0) & (r["depth"] < 1e4)
    H, W = d.shape
    return dict(workload="560 x 560 mapping image, 10 covisible views, dense matches 70% correct (0.5 px noise), "
                         "2-degree inliers, more than 3 inliers kept, float64",
                ms_per_image=round(ms, 4), pixels_per_s=round(H * W / (ms * 1e-3), 1),
                match_bytes_per_image=int(w.mu.nbytes * 3), kept_fraction_of_surface=round(float(ok[fin].mean()), 4),
                median_rel_depth_err_vs_truth=float(np.median(rel)),
                p90_rel_depth_err_vs_truth=float(np.percentile(rel, 90)),
                vs_oracle=dict(pixels=int(H * W), flagged_ambiguous=int((~un).sum()),
                               inliers_equal_unflagged=bool(np.array_equal(inl[un], r["inliers"][un])),
                               kept_equal_unflagged=bool(np.array_equal(d[un] > 0, r["depth"][un] > 0)),
                               max_rel_depth_err=float(np.max(np.abs(d[both] / r["depth"][both] - 1))),
                               median_rel_depth_err=float(np.median(np.abs(d[both] / r["depth"][both] - 1)))),
                paper_context="the paper's dense triangulation takes about 30 ms per image on an RTX 4090; "
                              "context, not a target")


def rig_leg(pk, steps=10):
    """Multi-camera rig queries (generalised absolute pose): a 4-camera head
    rig, 20,000 correspondences (5,000 per camera), 35% inliers, sigma 1 px,
    2,048 samples, tau 4 px, LO on the top 8, float32 scoring."""
    import numpy as np
    import oracle
    from paper_2601_04185_amd import synth
    q = synth.make_rig_query(1007, 20000, 0.35, 1.0)
    d = pk.to_device(q)
    prm = pk.make_params(threshold_px=4.0, fixed_samples=2048, batch=2048, lo_top_k=8)
    ctx = pk.Context(0, graphs=True)  # fixed samples: replayed as one captured hipGraph
    for _ in range(2):
        pk.imloc_rig_lo_ransac_pnp(ctx, d, q.rig, q.cam_start(), prm)
    lat = []
    for _ in range(steps):
        t0 = time.perf_counter()
        rc, R, t, st = pk.imloc_rig_lo_ransac_pnp(ctx, d, q.rig, q.cam_start(), prm)
        lat.append(time.perf_counter() - t0)
    ref = oracle.rig_lo_ransac(q.corr(), q.rig, threshold_px=4.0, fixed_samples=2048, batch=2048, lo_top_k=8)
    return dict(workload="4-camera head rig, 20,000 correspondences (5,000 per camera), 35% inliers, sigma 1 px, "
                         "2,048 generalised-P3P samples, tau 4 px, LO top-8, float32 scoring, float64 solves",
                status=int(rc), p50_ms=round(float(np.percentile(lat, 50)) * 1e3, 3),
                p99_ms=round(float(np.percentile(lat, 99)) * 1e3, 3), queries_per_s=round(steps / sum(lat), 2),
                candidates=st["candidates"], residuals=st["residuals"],
                residuals_per_s=round(st["residuals"] / float(np.median(lat)), 1),
                accuracy=dict(vs_oracle=vs_oracle([(R, t, ref)]), vs_truth=recall([(R, t, q.R, q.t)])),
                graph_captures_replays=list(ctx.graph_counters()))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=30, help="timed fused 256-query batches")
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--tune-reps", type=int, default=3, help="timed runs per candidate scoring shape")
    ap.add_argument("--no-tune", action="store_true", help="keep the default scoring launch shape")
    ap.add_argument("--score-shape", default=None,
                    help="CT,WG[,PTS]: scoring launch shape (candidates per item, workgroups, correspondences per "
                         "item) instead of autotuning")
    ap.add_argument("--cpu-queries", type=int, default=8, help="queries of the batch the all-core oracle runs")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-plain", action="store_true", help="skip the one-query-per-call form")
    ap.add_argument("--serving-queries", type=int, default=2000)
    ap.add_argument("--headline-only", action="store_true", help="skip every sub-leg")
    ap.add_argument("--legs-only", action="store_true",
                    help="skip the headline batch (for profiling a sub-leg alone; the line then has no headline)")
    ap.add_argument("--legs", default="single_large,single_small,serving,lift_ransac,paper_mode,mapping_depth,rig",
                    help="comma-separated sub-legs to run")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MB",
                    help="first run 3 plain device copies of MB MiB (a known-size reference for HBM counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this path runs on one GPU; --gpus {args.gpus} is not supported (queries are independent, "
              f"so more GPUs would each take their own share of queries)", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2601_04185_amd as pk

    if args.calibrate_copy > 0:
        src = torch.ones(args.calibrate_copy * 2 ** 18, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    out = dict(headline="skipped (--legs-only)") if args.legs_only else headline(pk, args)
    legs = [] if args.headline_only else [x for x in args.legs.split(",") if x]
    table = dict(single_large=lambda: single_large_leg(pk, args), single_small=lambda: single_small_leg(pk),
                 serving=lambda: serving_leg(pk, args), lift_ransac=lambda: e2e_leg(pk),
                 paper_mode=lambda: paper_mode_leg(pk), mapping_depth=lambda: mapping_depth_leg(pk),
                 rig=lambda: rig_leg(pk))
    for name in legs:
        out[name] = table[name]()
        print(f"bench.py: leg {name} done", file=sys.stderr, flush=True)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
