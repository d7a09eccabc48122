#!/usr/bin/env python3
"""Benchmark of the ImLoc pose-estimation hot path (lift + LO-RANSAC PnP,
arXiv 2601.04185 Sec. 3.3) on one MI355X.

A step is one whole LO-RANSAC PnP query through the C ABI (sampling, P3P,
scoring, selection, local optimisation, final Cauchy refinement, inlier mask)
with the correspondences already resident in HBM.  The default workload is the
single large query: K = 10 retrieved views x 5,000 dense matches = 50,000
2D-3D correspondences, 10,000 P3P samples, 6 px threshold, local optimisation
of the top 8, float32 scoring with float64 P3P and refinement.

Prints one JSON line: whole-job scored residuals/s (value), queries/s, p50/p99
latency, the pose error against the float64 oracle, the roofline of the
scoring kernel (timed with HIP events on its own stream) and the oracle timed
on the host cores.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "scored residuals/s and queries/s at 1 GPU; p50/p99 query latency at fixed accuracy"
# Non-packed float32 FMA peak: 256 CUs x 4 SIMDs x 16 lanes x 2 flop x 2.4 GHz.
# (The library is compiled with packed float32 instructions disabled; the 157.3 TFLOP/s
# packed figure is reported beside it.)
PEAK_F32_NONPACKED_TFLOPS = 256 * 4 * 16 * 2 * 2.4e9 / 1e12
PEAK_F32_PACKED_TFLOPS = 157.3
FLOP_PER_RESIDUAL = 27     # 9 FMA projection + 2 FMA residual + MUL+FMA square + 2 MUL threshold
FLOP_PER_INLIER = 5        # reciprocal, multiply, FMA, add of the truncated cost

WORKLOADS = {
    "single_large": dict(
        desc="single large query: 10 views x 5,000 = 50,000 correspondences, 25% inliers, sigma 1.5 px, "
             "10,000 P3P samples, tau 6 px, LO on the top 8, float32 scoring, float64 P3P/LO/refine",
        make="config2_single_large",
        params=dict(threshold_px=6.0, fixed_samples=10000, batch=10000, lo_top_k=8, lo_iters=10, final_iters=10,
                    precision=0)),
    "single_small_fp64": dict(
        desc="single query: 2,000 correspondences, 40% inliers, sigma 1 px, 1,024 P3P samples, tau 4 px, "
             "LO on the top 1, every step float64",
        make="config1_single_small",
        params=dict(threshold_px=4.0, fixed_samples=1024, batch=1024, lo_top_k=1, lo_iters=10, final_iters=10,
                    precision=1)),
}


def _file_hash(path):
    with open(path, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def _traffic(kernel_src, workload, shape):
    """HBM bytes per launch from the committed counter summary of this launch
    shape (key: value lines), if it was taken on the current source of the
    kernel, this workload and this shape; else None."""
    ct, wg = shape
    p = os.path.join(ROOT, "profiles", f"score_single_large_traffic_{ct}x{wg}.txt")
    if not os.path.exists(p):
        return None
    d = {}
    for line in open(p):
        if ":" in line and not line.startswith(("#", " ")):
            k, v = line.split(":", 1)
            d[k.strip()] = v.strip()
    if (d.get("workload") != workload or d.get("kernel_src_sha256_16") != _file_hash(kernel_src)
            or d.get("candidates_per_item") != str(ct) or d.get("workgroups") != str(wg)):
        return None
    try:
        return float(d["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def _rot_deg(Ra, Rb):
    import numpy as np
    M = Ra @ Rb.T
    s = 0.5 * np.array([M[2, 1] - M[1, 2], M[0, 2] - M[2, 0], M[1, 0] - M[0, 1]])
    return float(np.degrees(np.arctan2(np.linalg.norm(s), 0.5 * (np.trace(M) - 1.0))))


def batch_leg(pk, ctx_plain, steps, n_queries=256):
    """The 256-query batch: the fused batched form (one call, shared launches)
    against the plain form (one call per query), same seeds and parameters."""
    import numpy as np
    import torch
    from paper_2601_04185_amd import synth
    qs = synth.config3_batch(n_queries)
    ds = [pk.to_device(q) for q in qs]
    Ks = [q.K for q in qs]
    prms = [pk.make_params(threshold_px=4.0, fixed_samples=4096, batch=4096, lo_top_k=8, query_id=i)
            for i in range(len(qs))]
    ctx = pk.Context(0, graphs=True)  # the fixed-sample batch replays as one captured hipGraph
    # the batch's own scoring launch shape (its rounds are far larger than one query's)
    from paper_2601_04185_amd.autotune import tune_scoring
    tuned = tune_scoring(ctx, lambda c: pk.imloc_lo_ransac_pnp_batch(c, ds, Ks, prms)[2], reps=1)
    pk.imloc_lo_ransac_pnp_batch(ctx, ds, Ks, prms)  # warm-up (workspace, capture)
    torch.cuda.synchronize()
    t_f = []
    for _ in range(steps):
        t0 = time.perf_counter()
        status, poses, stats = pk.imloc_lo_ransac_pnp_batch(ctx, ds, Ks, prms)
        t_f.append(time.perf_counter() - t0)
    eager = pk.Context(0)
    eager.set_score_tuning(*ctx.score_tuning())
    pk.imloc_lo_ransac_pnp_batch(eager, ds, Ks, prms)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    pk.imloc_lo_ransac_pnp_batch(eager, ds, Ks, prms)
    t_eager = time.perf_counter() - t0
    res = sum(s["residuals"] for s in stats)
    inl = sum(s["inlier_residuals"] for s in stats)
    tctx = pk.Context(0, timing=True)
    tctx.set_score_tuning(*ctx.score_tuning())
    _, _, st_t = pk.imloc_lo_ransac_pnp_batch(tctx, ds, Ks, prms)
    score_ms = st_t[0]["ms_score"]
    # plain form: one query per call
    for i in range(min(4, len(qs))):
        pk.imloc_lo_ransac_pnp(ctx_plain, ds[i], Ks[i], prms[i])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plain = [pk.imloc_lo_ransac_pnp(ctx_plain, ds[i], Ks[i], prms[i]) for i in range(len(qs))]
    t_plain = time.perf_counter() - t0
    same = all(np.array_equal(plain[i][1], poses[i][0]) and np.array_equal(plain[i][2], poses[i][1])
               for i in range(len(qs)))
    tf = statistics.median(t_f)
    flops = FLOP_PER_RESIDUAL * res + FLOP_PER_INLIER * inl
    return dict(workload=f"{len(qs)} queries, correspondences uniform in [5,000, 80,000] "
                         f"(total {sum(q.n for q in qs):,}), inlier ratios uniform in [10%, 60%], sigma 1 px, "
                         f"4,096 samples each, tau 4 px, LO top-8",
                fused_ms=round(tf * 1e3, 3), fused_queries_per_s=round(len(qs) / tf, 2),
                fused_residuals_per_s=round(res / tf, 1), fused_eager_ms=round(t_eager * 1e3, 3),
                graph_captures_replays=list(ctx.graph_counters()),
                score_launch_shape=dict(zip(("candidates_per_item", "workgroups"), ctx.score_tuning())),
                plain_ms=round(t_plain * 1e3, 3), plain_queries_per_s=round(len(qs) / t_plain, 2),
                speedup_fused_vs_plain=round(t_plain / tf, 3), residuals=res,
                score_ms=round(score_ms, 3), score_tflops=round(flops / (score_ms * 1e-3) / 1e12, 3),
                score_frac_of_peak=round(flops / (score_ms * 1e-3) / 1e12 / PEAK_F32_NONPACKED_TFLOPS, 4),
                poses_identical_fused_vs_plain=bool(same),
                failed=int(sum(1 for x in status if x != 0)))


def serving_leg(pk, n_queries=240, load=0.75, max_slots=64):
    """Continuous batching: queries with log-normal sizes in [2,000, 200,000]
    and inlier ratios in [5%, 60%], adaptive stopping at 99.9%.  First the
    saturation throughput (all queries queued at once), then Poisson arrivals
    at `load` times that rate; latency = completion - arrival."""
    import numpy as np
    from paper_2601_04185_amd import synth
    arr_unit, ns, eps = synth.serving_arrivals(n_queries, rate_qps=1.0)
    qs = [synth.make_query(1005 * 1000 + i, int(ns[i]), float(eps[i]), 1.0) for i in range(n_queries)]
    ds = [pk.to_device(q) for q in qs]
    P = [pk.make_params(threshold_px=4.0, confidence=0.999, batch=1024, min_iters=1024, max_iters=100000,
                        lo_top_k=8, query_id=i) for i in range(n_queries)]
    srv = pk.Server(0, max_slots=max_slots, max_top_k=8, max_n=200000)

    def run(arrivals):
        t0 = time.perf_counter()
        done_t, tick, i, steps, occ = {}, {}, 0, 0, []
        while len(done_t) < n_queries:
            now = time.perf_counter() - t0
            while i < n_queries and arrivals[i] <= now:
                tick[srv.submit(ds[i], qs[i].K, P[i])] = i
                i += 1
            done, resident, queued = srv.step()
            steps += 1
            occ.append(resident)
            now = time.perf_counter() - t0
            for t in done:
                done_t[tick[t]] = now
                srv.poll(t)
            if resident == 0 and queued == 0 and i < n_queries:
                time.sleep(max(0.0, arrivals[i] - (time.perf_counter() - t0)))
        lat = np.array([done_t[k] - arrivals[k] for k in range(n_queries)])
        return (time.perf_counter() - t0), lat, steps, float(np.mean(occ))

    sat_time, _, sat_steps, sat_occ = run(np.zeros(n_queries))
    sat_qps = n_queries / sat_time
    rate = load * sat_qps
    arrivals = arr_unit / rate
    t_open, lat, steps, occ = run(arrivals)
    # every served result equals the query alone
    ctx = pk.Context(0)
    ident = True
    srv2 = pk.Server(0, max_slots=max_slots, max_top_k=8, max_n=200000)
    check = list(range(0, n_queries, max(1, n_queries // 12)))
    tk = {srv2.submit(ds[i], qs[i].K, P[i]): i for i in check}
    got = {}
    while len(got) < len(check):
        done, _, _ = srv2.step()
        for t in done:
            got[tk[t]] = srv2.poll(t)
    for i in check:
        rc, R, t, st = pk.imloc_lo_ransac_pnp(ctx, ds[i], qs[i].K, P[i])
        ident &= bool(got[i][0] == rc and np.array_equal(got[i][1], R) and np.array_equal(got[i][2], t))
    srv.close()
    srv2.close()
    return dict(workload=f"{n_queries} queries, correspondences log-normal in [2,000, 200,000] "
                         f"(mean {int(np.mean(ns)):,}), inlier ratios uniform in [5%, 60%], sigma 1 px, adaptive "
                         f"stopping at 99.9% (batches of 1,024, cap 100,000), tau 4 px, LO top-8, {max_slots} slots",
                saturation_queries_per_s=round(sat_qps, 2), saturation_rounds=sat_steps,
                saturation_mean_resident=round(sat_occ, 1),
                offered_queries_per_s=round(rate, 2), queries_per_s=round(n_queries / t_open, 2),
                p50_ms=round(float(np.percentile(lat, 50)) * 1e3, 3),
                p99_ms=round(float(np.percentile(lat, 99)) * 1e3, 3), rounds=steps, mean_resident=round(occ, 1),
                served_equals_alone=ident, checked=len(check))


def e2e_leg(pk, steps=5):
    """Lifting plus RANSAC: 20 database RGB-D views (640x480 float32 depth) of
    a box-and-plane scene, 8,000 query-to-database matches per view, lifted on
    the GPU, then LO-RANSAC PnP with adaptive stopping at 99.9%."""
    import numpy as np
    import torch
    from paper_2601_04185_amd import synth
    wl = synth.config4_lift_scene()
    m = {k: torch.from_numpy(v).cuda() for k, v in wl.matches.items()}
    depth = torch.from_numpy(wl.depth).cuda()
    prm = pk.make_params(threshold_px=4.0, batch=1024, min_iters=1024, max_iters=100000, confidence=0.999,
                         lo_top_k=8)
    ctx = pk.Context(0)
    n_match = int(m["q_u"].numel())

    def once():
        t0 = time.perf_counter()
        g = pk.imloc_lift(ctx, m, depth, wl.cams, wl.poses)
        t1 = time.perf_counter()
        corr = {k: g[k] for k in ("u", "v", "X", "Y", "Z", "w")}
        rc, R, t, st = pk.imloc_lo_ransac_pnp(ctx, corr, wl.K_query, prm)
        return t1 - t0, time.perf_counter() - t0, g["n"], rc, R, t, st

    once()
    torch.cuda.synchronize()
    lift_s, tot_s = [], []
    for _ in range(steps):
        a, b, n_lifted, rc, R, t, st = once()
        lift_s.append(a)
        tot_s.append(b)
    tl, tt = statistics.median(lift_s), statistics.median(tot_s)
    # algorithmic lift bytes: 24 B of match in, 4 depth taps, 28 B out per lifted correspondence
    lift_bytes = n_match * (24 + 16) + n_lifted * 28
    return dict(workload=f"{wl.depth.shape[0]} database views 640x480, {n_match:,} matches (30% correct), lifted to "
                         f"{n_lifted:,} correspondences, adaptive stopping at 99.9%, tau 4 px, LO top-8",
                status=int(rc), ms_per_query=round(tt * 1e3, 3), queries_per_s=round(1.0 / tt, 2),
                lift_ms=round(tl * 1e3, 4), lift_matches_per_s=round(n_match / tl, 1),
                lift_gb_per_s_incl_host_sync=round(lift_bytes / tl / 1e9, 2),
                samples=st["samples"], residuals=st["residuals"], best_count=st["best_count"],
                rot_err_vs_truth_deg=_rot_deg(R, wl.R), t_err_vs_truth_m=float(np.linalg.norm(t - wl.t)))


def paper_mode_leg(pk, steps=10):
    """The paper's own LO-RANSAC settings on the single large query with
    confidence weights: stride subsample to 10,000 scoring points, batches of
    1,000, local optimisation of a new best (top 1), stop at 100,000 samples or
    confidence 1 - 1e-4, Cauchy refinement over all 50,000 points."""
    import numpy as np
    import torch
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
    return dict(workload="50,000 correspondences (10 views x 5,000), 25% inliers, sigma 1.5 px, confidence weights; "
                         "scoring subsample 10,000, batches of 1,000, LO top-1, confidence 0.9999, cap 100,000, "
                         "tau 6 px",
                status=int(rc), p50_ms=round(float(np.percentile(lat, 50)) * 1e3, 3),
                p99_ms=round(float(np.percentile(lat, 99)) * 1e3, 3),
                queries_per_s=round(steps / sum(lat), 2), samples=st["samples"], batches=st["batches"],
                residuals=st["residuals"], rot_err_vs_truth_deg=_rot_deg(R, q.R),
                t_err_vs_truth_m=float(np.linalg.norm(t - q.t)),
                paper_context="the paper's RANSAC loop takes about 200 ms per query on an RTX 4090 "
                              "(CPU sampling and P3P, GPU scoring); context, not a target")


def mapping_depth_leg(pk, steps=10):
    """Mapping-time depth of one 560 x 560 mapping image from dense matches in
    10 covisible views (70% correct, 0.5 px noise): 1-DoF triangulation."""
    import numpy as np
    import torch
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
    d = g["depth"].cpu().numpy()
    fin = np.isfinite(w.depth_true)
    ok = d > 0
    rel = np.abs(d[ok & fin] / w.depth_true[ok & fin] - 1)
    H, W = d.shape
    return dict(workload="560 x 560 mapping image, 10 covisible views, dense matches 70% correct (0.5 px noise), "
                         "2-degree inliers, more than 3 inliers kept, float64",
                ms_per_image=round(ms, 4), pixels_per_s=round(H * W / (ms * 1e-3), 1),
                match_bytes_per_image=int(w.mu.nbytes * 3), kept_fraction_of_surface=round(float(ok[fin].mean()), 4),
                median_rel_depth_err=float(np.median(rel)), p90_rel_depth_err=float(np.percentile(rel, 90)),
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
                rot_err_vs_oracle_deg=_rot_deg(R, ref["R"]),
                t_rel_err_vs_oracle=float(np.linalg.norm(t - ref["t"]) / max(1.0, np.linalg.norm(ref["t"]))),
                rot_err_vs_truth_deg=_rot_deg(R, q.R), t_err_vs_truth_m=float(np.linalg.norm(t - q.t)),
                graph_captures_replays=list(ctx.graph_counters()))


def cpu_baseline(q, params, reps):
    """The oracle as it stands, on the host cores, on the same query."""
    import oracle
    prm = {k: v for k, v in params.items() if k != "precision"}
    times, ref = [], None
    for _ in range(reps):
        t0 = time.perf_counter()
        ref = oracle.lo_ransac_pnp(q.corr(), q.K, **prm)
        times.append(time.perf_counter() - t0)
    t = statistics.median(times)
    cores = int(os.environ.get("OMP_NUM_THREADS", "0") or 0) or os.cpu_count()
    return ref, dict(value=ref["residuals"] / t, unit="residuals/s", cores=cores, kind="oracle",
                     sample=f"{reps} whole queries of the same workload (float64 C oracle, OpenMP over candidates), "
                            f"median {t * 1e3:.1f} ms/query = {1.0 / t:.3f} queries/s")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="single_large", choices=sorted(WORKLOADS))
    ap.add_argument("--cpu-reps", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batch", action="store_true", help="skip the 256-query fused-vs-plain leg")
    ap.add_argument("--batch-steps", type=int, default=3)
    ap.add_argument("--no-serving", action="store_true", help="skip the continuous-batching leg")
    ap.add_argument("--no-tune", action="store_true", help="keep the default scoring launch shape")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MB",
                    help="first run 3 plain device copies of MB MiB (a known-size reference for HBM counters)")
    ap.add_argument("--score-shape", default=None,
                    help="CT,WG: scoring launch shape (candidates per item, workgroups) instead of autotuning")
    ap.add_argument("--no-e2e", action="store_true", help="skip the lifting + RANSAC leg")
    ap.add_argument("--no-paper-mode", action="store_true", help="skip the paper-settings leg")
    ap.add_argument("--no-mapping", action="store_true", help="skip the mapping-time depth leg")
    ap.add_argument("--no-rig", action="store_true", help="skip the multi-camera rig leg")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this path runs on one GPU; --gpus {args.gpus} is not supported (queries are independent, "
              f"so more GPUs would each take their own share of queries)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    import paper_2601_04185_amd as pk
    from paper_2601_04185_amd import synth

    if args.calibrate_copy > 0:
        src = torch.ones(args.calibrate_copy * 2 ** 18, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    wl = WORKLOADS[args.workload]
    q = getattr(synth, wl["make"])()
    prm = pk.make_params(**wl["params"])
    d = pk.to_device(q)
    # fixed-sample queries are captured once and replayed as a hipGraph
    ctx = pk.Context(0, graphs=prm.fixed_samples > 0)
    tuned = None
    if args.score_shape:
        ct, wg = (int(x) for x in args.score_shape.split(","))
        ctx.set_score_tuning(ct, wg)
    elif not args.no_tune:
        from paper_2601_04185_amd.autotune import tune_scoring
        tuned = tune_scoring(ctx, lambda c: pk.imloc_lo_ransac_pnp(c, d, q.K, prm)[3])

    for _ in range(args.warmup):
        pk.imloc_lo_ransac_pnp(ctx, d, q.K, prm)
    torch.cuda.synchronize()
    lat = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        s = time.perf_counter()
        rc, R, t, st = pk.imloc_lo_ransac_pnp(ctx, d, q.K, prm)
        lat.append(time.perf_counter() - s)
    torch.cuda.synchronize()
    total = time.perf_counter() - t0
    assert rc == 0, f"status {rc}"
    residuals = st["residuals"]

    # per-kernel device time: HIP events recorded on the context stream around each launch
    tctx = pk.Context(0, timing=True)
    tctx.set_score_tuning(*ctx.score_tuning())
    per_launch, inl = [], []
    for _ in range(max(5, min(args.steps, 20))):
        _, _, _, s2 = pk.imloc_lo_ransac_pnp(tctx, d, q.K, prm)
        per_launch.append(s2["ms_score"] / max(1, s2["score_launches"]))
        inl.append(s2["inlier_residuals"] / max(1, s2["score_launches"]))
    stage_ms = {k: s2[k] for k in ("ms_sample", "ms_score", "ms_select", "ms_lo", "ms_refine", "ms_total")}
    launch_ms = statistics.median(per_launch)
    res_per_launch = residuals / max(1, s2["score_launches"])
    flops = FLOP_PER_RESIDUAL * res_per_launch + FLOP_PER_INLIER * statistics.median(inl)
    achieved = flops / (launch_ms * 1e-3) / 1e12
    kernel_src = os.path.join(ROOT, "paper_2601_04185_amd", "csrc", "score.hip")
    roofline = dict(bound="alu", achieved=round(achieved, 3), peak=round(PEAK_F32_NONPACKED_TFLOPS, 2),
                    unit="TFLOP/s", frac=round(achieved / PEAK_F32_NONPACKED_TFLOPS, 4),
                    traffic=_traffic(kernel_src, args.workload, ctx.score_tuning()), kernel="score_f32_kernel",
                    launch_ms=round(launch_ms, 4), flop_per_launch=int(flops),
                    frac_of_packed_peak=round(achieved / PEAK_F32_PACKED_TFLOPS, 4),
                    residuals_per_s_kernel=round(res_per_launch / (launch_ms * 1e-3), 1),
                    launch_shape=dict(zip(("candidates_per_item", "workgroups"), ctx.score_tuning())))

    out = dict(metric=METRIC, value=round(residuals * args.steps / total, 1), unit="residuals/s", n_gpus=1,
               steps=args.steps, warmup=args.warmup, ms_per_step=round(total / args.steps * 1e3, 4),
               higher_is_better=True, scaling="weak", vs_baseline=None,
               dtype="f32" if prm.precision == 0 else "f64", dtype_solve="f64", data="synthetic",
               config=dict(workload=wl["desc"], n_correspondences=q.n, samples=prm.fixed_samples,
                           candidates=st["candidates"], residuals_per_query=residuals, parallelism="1 GPU",
                           graph_replay=list(ctx.graph_counters())),
               queries_per_s=round(args.steps / total, 3),
               p50_ms=round(float(np.percentile(lat, 50)) * 1e3, 4),
               p99_ms=round(float(np.percentile(lat, 99)) * 1e3, 4),
               stage_ms=stage_ms, roofline=roofline)
    if tuned is not None:
        out["autotune"] = dict(best=tuned["best"], table=tuned["table"])
    acc = dict(rot_err_vs_truth_deg=_rot_deg(R, q.R), t_err_vs_truth_m=float(np.linalg.norm(t - q.t)))
    if not args.no_cpu_baseline:
        ref, cb = cpu_baseline(q, wl["params"], args.cpu_reps)
        out["cpu_baseline"] = cb
        acc.update(rot_err_vs_oracle_deg=_rot_deg(R, ref["R"]),
                   t_rel_err_vs_oracle=float(np.linalg.norm(t - ref["t"]) / max(1.0, np.linalg.norm(ref["t"]))),
                   within_tolerance=bool(_rot_deg(R, ref["R"]) <= 1e-3 and
                                         np.linalg.norm(t - ref["t"]) <= 1e-4 * max(1.0, np.linalg.norm(ref["t"]))))
    out["accuracy"] = acc
    if not args.no_batch:
        out["batch256"] = batch_leg(pk, ctx, args.batch_steps)
    if not args.no_serving:
        out["serving"] = serving_leg(pk)
    if not args.no_e2e:
        out["lift_ransac"] = e2e_leg(pk)
    if not args.no_paper_mode:
        out["paper_mode"] = paper_mode_leg(pk)
    if not args.no_mapping:
        out["mapping_depth"] = mapping_depth_leg(pk)
    if not args.no_rig:
        out["rig"] = rig_leg(pk)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
