"""Benchmark of the group-testing range search on one MI355X.

One step = one query call over a batch of queries: query preparation, the
level-wise pool walk, the exact leaf test, the float64 recheck and the result
compaction (the whole query path; the index is built once, offline, as in the
paper).  The timed steps run back to back on one stream through two
workspaces (the next batch is enqueued before the host waits for the previous
one); per-call latency comes from a second run that waits for every call.  Workload: N = 2^20 softmax feature vectors, d = 1000, 1024
queries per batch, rho = 0.9, bfloat16 pool sums.  Beside it: the plain float32
walk, the float8 walk and the exhaustive float32 GEMM on the same batch, and
the CPU float64 oracle on a bounded sample of the same queries.

Prints one JSON line.  Only one GPU is used; --gpus > 1 exits.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "queries/sec at N=1M,d=1000,100% recall vs exhaustive GEMM; p50/p99 latency"
HBM_PEAK_GBS = 8000.0


# Counter-measured HBM traffic per launch (rocprofv3 FETCH_SIZE and WRITE_SIZE,
# scaled by a 1 GiB copy), kept in a profile summary per pool format and batch
# size together with a hash of the kernel sources it was taken on; reported
# only while the sources match.
def counter_summary(pool, nq):
    return os.path.join(ROOT, "profiles", f"counters_walk_{pool}_n1m_d1000_b{nq}_rho0.9.md")


KERNEL_SOURCES = ["k_walk.hip", "gt_numerics.h", "gt_device.h", "gt_internal.h", "gt_api.cpp"]


def kernel_source_hash():
    import hashlib

    h = hashlib.sha256()
    for name in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2311_02573_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def stored_traffic(pool, nq):
    """{kernel: bytes per launch} from the counter summary of this pool format
    and batch size, or {} if it is missing or was taken on other kernel
    sources."""
    try:
        text = open(counter_summary(pool, nq)).read()
    except OSError:
        return {}
    vals, src = {}, None
    for line in text.splitlines():
        line = line.strip()
        if line.startswith("traffic_source_sha256:"):
            src = line.split(":", 1)[1].strip()
        elif line.startswith("traffic_bytes_per_launch "):
            k, v = line[len("traffic_bytes_per_launch "):].rsplit(":", 1)
            vals[k.strip()] = float(v)
    return vals if src == kernel_source_hash() else {}


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def pct(a, p):
    return float(np.percentile(np.asarray(a), p))


def measure_roofline(idx, q, rho, pool, nq, walk_subtract, d, side_steps):
    """Per-kernel-group device time (HIP events on the call's stream, median
    over profiled calls) and algorithmic bytes (each distinct row a kernel
    must read, once: pool rows at d_pad x element size, leaf rows at d x 4,
    plus the subtraction step's 128-byte score records), and the roofline of
    the group with the largest share of the call.  Returns (roofline dict,
    stats of the counting call, first sparse level)."""
    idx.set_option("profile", 1)
    prof = []
    for _ in range(max(3, side_steps)):
        idx.query(q, rho, pool=pool)
        prof.append(idx.stats())
    idx.set_option("profile", 0)
    med = lambda k: float(np.median([p[k] for p in prof]))
    ms_dense, ms_sparse, ms_leaf = med("ms_dense"), med("ms_frontier"), med("ms_leaf")
    n_dense, n_sparse = prof[-1]["dense_launches"], prof[-1]["frontier_launches"]

    idx.set_option("count_unique", 1)
    idx.query(q, rho, pool=pool)
    su = idx.stats()
    idx.set_option("count_unique", 0)
    esz = {"bf16": 2, "fp8": 1, "f32": 4}[pool]
    dp = su["d_pad"]
    h, D = su["head_level"], su["depth"]
    first_sparse = h + n_dense          # dense steps test levels h+1 .. h+n_dense
    uniq = su["unique_rows"]
    dense_bytes = sum(uniq[l] for l in range(h + 1, first_sparse + 1)) * dp * esz
    sparse_bytes = sum(uniq[l] for l in range(first_sparse + 1, D)) * dp * esz
    leaf_bytes = uniq[D] * d * 4
    entries = list(su["entries"])
    # subtraction step (bf16 after a dense step): sparse levels first_sparse ..
    # sub_to read one child row per entry plus the entry's 128-byte score
    # record, and write records for outputs that a subtraction step reads next
    ws = 1 if walk_subtract == -1 else walk_subtract
    sub_to = -1
    if pool == "bf16" and n_dense > 0 and ws > 0 and first_sparse <= D - 2:
        sub_to = D - 2 if ws == 1 else D - 3
    sub_levels = [l for l in range(first_sparse, D - 1) if l <= sub_to]
    rec_bytes = 128 * (sum(entries[l] for l in sub_levels)
                       + sum(entries[l + 1] for l in sub_levels if l + 1 <= sub_to))
    dense_rec_bytes = 128 * entries[first_sparse] if sub_levels else 0
    dense_bytes += dense_rec_bytes
    sparse_bytes += rec_bytes
    raw_sparse = sum(entries[l] * (1 if l in sub_levels else 2)
                     for l in range(first_sparse, D - 1)) * dp * esz
    if n_dense == 0:
        raw_sparse += ((1 << h) * su["last_tiles"] - entries[h]) * 2 * dp * esz
    raw_leaf = entries[D - 1] * 2 * dp * 4
    n_sub = len(sub_levels)
    walk_name = (f"k_walk_level<{pool}>" if n_sub == 0 else
                 "k_walk_sub<bf16>" if n_sub == n_sparse else "k_walk_sub+k_walk_level<bf16>")
    groups = {
        f"k_dense_level<{pool}>": (dense_bytes, ms_dense, n_dense),
        walk_name: (sparse_bytes, ms_sparse, n_sparse),
        "k_leaf": (leaf_bytes, ms_leaf, 1),
    }
    gbps = lambda b, ms: round(b / (ms * 1e-3) / 1e9, 1) if ms > 0 else None
    dom = max(groups, key=lambda k: groups[k][1])
    b, ms, nl = groups[dom]
    achieved = gbps(b, ms)
    roofline = {
        "kernel": dom,
        "bound": "hbm",
        "achieved": achieved,
        "peak": HBM_PEAK_GBS,
        "unit": "GB/s",
        "frac": round(achieved / HBM_PEAK_GBS, 4) if achieved else None,
        "traffic": stored_traffic(pool, nq).get(dom),
        "algorithmic_bytes_per_launch": b / max(1, nl),
        "launches_per_batch": nl,
        "avg_launch_ms": ms / max(1, nl),
        "kernels": {k: {"bytes": v[0], "ms": round(v[1], 4), "launches": v[2], "GBps": gbps(v[0], v[1])}
                    for k, v in groups.items()},
        # per-stage device time of one call (HIP events, median over the profiled calls)
        "stage_ms": {k[3:]: round(med(k), 4) for k in ("ms_prep", "ms_dense", "ms_frontier", "ms_leaf",
                                                      "ms_recheck", "ms_compact", "ms_total")},
        "walk_all_levels": {"bytes": dense_bytes + sparse_bytes, "ms": round(ms_dense + ms_sparse, 4),
                            "GBps": gbps(dense_bytes + sparse_bytes, ms_dense + ms_sparse)},
        "sparse_raw_bytes": raw_sparse,
        "score_record_bytes": {"dense_writes": dense_rec_bytes, "walk_reads_writes": rec_bytes},
        "leaf_raw_bytes": raw_leaf,
        "entries_per_level": {l: entries[l] for l in range(h + 1, D)},
        "tests_per_level": {l: su["pairs"][l] for l in range(h + 1, D)},
        "leaf_pairs": su["leaf_pairs"], "leaf_candidates": su["candidates"],
        "rechecked": su["rechecked"], "results": su["results"],
        "unique_rows_per_level": {l: uniq[l] for l in range(h + 1, D + 1)},
    }
    return roofline, su, first_sparse


def cpu_info():
    """CPU model (from /proc/cpuinfo) and the cores this process may use."""
    model = None
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    nproc = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    return model, nproc


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=1 << 20)
    ap.add_argument("--d", type=int, default=1000)
    ap.add_argument("--nq", type=int, default=1024)
    ap.add_argument("--rho", type=float, default=0.9)
    ap.add_argument("--pool", default="bf16", choices=["bf16", "fp8", "f32"])
    ap.add_argument("--side-steps", type=int, default=5)
    ap.add_argument("--cpu-sample", type=int, default=384,
                    help="queries of the batch the CPU oracle scans (about 10 s on 16 threads)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-side", action="store_true")
    ap.add_argument("--signed-n", type=int, default=1 << 20,
                    help="rows of the signed-descriptor comparator (0: skip it)")
    ap.add_argument("--copy-calib", action="store_true",
                    help="end with a 1 GiB device-to-device copy (reference for memory counters)")
    ap.add_argument("--sweep-dense", action="store_true",
                    help="also time the walk for several dense/sparse split levels")
    ap.add_argument("--dense-last", type=int, default=-2,
                    help="last level walked with dense steps (-2: automatic, -1: none)")
    ap.add_argument("--walk-subtract", type=int, default=-1,
                    help="subtraction step of the bfloat16 walk: 0 off, 1 every sparse level, "
                         "2 all but the last, -1 automatic")
    ap.add_argument("--streams", type=int, default=3,
                    help="headline: 1 = two workspaces on one stream; N > 1 = N workspaces, "
                         "one stream each")
    ap.add_argument("--sweep-subtract", action="store_true",
                    help="also time the walk with each subtraction setting")
    ap.add_argument("--serve-seconds", type=float, default=60.0,
                    help="length of each loaded serving run (0: no serving leg)")
    ap.add_argument("--nq-variant", type=int, default=4096,
                    help="batch size of the bfloat16 / float8 precision variant (0: skip it)")
    ap.add_argument("--leg", default="all", choices=["all", "exh", "serve"],
                    help="exh: only the exhaustive GEMM path on the headline batch, for "
                         "counter profiles of its kernel; serve: only the serving legs")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on exactly one GPU (the library has no multi-GPU path); use --gpus 1",
              file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2311_02573_amd import gt, synth

    if not torch.cuda.is_available():
        print("no GPU visible", file=sys.stderr)
        sys.exit(1)
    dev = torch.device("cuda:0")
    if args.leg == "serve":
        out = {"serving": serving_leg(args.serve_seconds, torch, gt, synth, dev),
               "serving_stress": stress_serving_leg(args.serve_seconds, torch, gt, synth, dev)}
        print(json.dumps(out), flush=True)
        return

    t0 = time.time()
    # one database for the 1024- and the 4096-query batches (neighbours are
    # planted for 4096 queries either way); the headline takes the first nq
    w = synth.workload1(nq=max(args.nq, args.nq_variant), rho=args.rho, n=args.n, d=args.d)
    log(f"generated N={w.n} d={w.d} nq={len(w.queries)} in {time.time() - t0:.1f}s")
    feats = torch.from_numpy(w.feats).to(dev)
    q_all = torch.from_numpy(w.queries).to(dev)
    q = q_all[:args.nq]
    torch.cuda.synchronize()

    t0 = time.time()
    idx = gt.GTIndex(feats, pools=("f32", "bf16", "fp8", "max_bf16"))
    torch.cuda.synchronize()
    build_s = time.time() - t0
    st0 = idx.stats()
    log(f"index built in {build_s * 1e3:.1f} ms, depth {st0['depth']}, head {st0['head_level']}, "
        f"{st0['bytes_device'] / 2**30:.2f} GiB")
    del feats
    torch.cuda.empty_cache()
    if args.dense_last != -2:
        idx.set_option("dense_last", args.dense_last)
    idx.set_option("walk_subtract", args.walk_subtract)

    def run(pool, steps, warmup, qq=None, rho=None):
        qq = q if qq is None else qq
        rho = args.rho if rho is None else rho
        fn = (lambda: idx.exhaustive(qq, rho)) if pool == "exh" else \
            (lambda: idx.query(qq, rho, pool=pool))
        res = None
        for _ in range(warmup):
            res = fn()
        torch.cuda.synchronize()
        lat = []
        t_start = time.perf_counter()
        for _ in range(steps):
            t1 = time.perf_counter()
            res = fn()
            torch.cuda.synchronize()
            lat.append((time.perf_counter() - t1) * 1e3)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t_start
        return res, wall, lat

    def run_pipelined(pool, steps, warmup, streams=1, qq=None, rho=None):
        # W = max(2, streams) workspaces: batch k is enqueued before the host
        # waits for batch k - W + 1, so the host's per-call work overlaps the
        # device's.  On one stream the device runs the batches back to back,
        # in order; with a stream per workspace a batch's first kernels may
        # also run while the previous batches' last ones finish.
        qq = q if qq is None else qq
        rho = args.rho if rho is None else rho
        W = max(2, streams)
        ws = [gt.Workspace(idx, qq.shape[0],
                           stream=torch.cuda.current_stream() if streams == 1 else None)
              for _ in range(W)]

        def go(n):
            r = None
            for k in range(n):
                ws[k % W].submit(qq, rho, pool=pool)
                if k >= W - 1:
                    r = ws[(k - W + 1) % W].finish()
            for k in range(max(0, n - W + 1), n):
                r = ws[k % W].finish()
            return r

        go(max(W, warmup))
        torch.cuda.synchronize()
        t_start = time.perf_counter()
        r = go(steps)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t_start
        for w_ in ws:
            w_.close()
        return r, wall

    if args.leg == "exh":
        # the exhaustive path alone (counter profiles of k_gemm_threshold)
        for _ in range(args.warmup):
            idx.exhaustive(q, args.rho)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for _ in range(args.steps):
            r = idx.exhaustive(q, args.rho)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t1) / args.steps * 1e3
        print(json.dumps({"leg": "exh", "ms_per_call": round(ms, 3), "results": r.total,
                          "queries_per_s": round(args.nq / ms * 1e3, 1)}), flush=True)
        idx.close()
        return

    # ---- headline: the walk on the chosen pool format, batches back to back
    res_p, wall = run_pipelined(args.pool, args.steps, args.warmup, args.streams)
    ms_step = wall / args.steps * 1e3
    qps = args.nq * args.steps / wall
    log(f"{args.pool} walk: {ms_step:.3f} ms/batch, {qps:.0f} queries/s, {res_p.total} results")
    # one call at a time (host waits for each): per-call latency
    res, wall_sync, lat = run(args.pool, args.steps, args.warmup)
    qps_sync = args.nq * args.steps / wall_sync
    log(f"{args.pool} walk, one call at a time: {wall_sync / args.steps * 1e3:.3f} ms/batch, "
        f"{qps_sync:.0f} queries/s")
    same_p = res_p.total == res.total and all(
        np.array_equal(a[0], b[0]) for a, b in zip(res_p.to_lists(), res.to_lists()))
    if not same_p:
        log("WARNING: pipelined and one-at-a-time results differ")

    # ---- kernel timing (HIP events) and algorithmic bytes (distinct rows)
    roofline, su, first_sparse = measure_roofline(idx, q, args.rho, args.pool, args.nq,
                                                  args.walk_subtract, w.d, args.side_steps)
    D = su["depth"]

    # ---- the TNE cost model (paper Sec. 5, Eq. 3) against the walk: lambda
    # fitted to a sample of this workload's similarities, predicted pools per
    # query surviving each level vs the walk's own counts
    from paper_2311_02573_amd import costmodel as cm

    rs = np.random.default_rng(0)
    rows = rs.choice(w.n, size=min(w.n, 65536), replace=False)
    sims = (np.asarray(w.feats[np.sort(rows)], np.float64) @ np.asarray(w.queries[:16], np.float64).T).ravel()
    lam_m = cm.fit_lambda(np.clip(sims, 0.0, 1.0))
    lam_h = cm.fit_lambda_loghist(sims)
    pm = cm.level_survivors(w.n, args.rho, lam_m, D)
    ph = cm.level_survivors(w.n, args.rho, lam_h, D)
    meas = {l: su["pairs"][l + 1] / (2.0 * args.nq) for l in range(first_sparse, D - 1)}
    meas[D - 1] = su["leaf_pairs"] / (2.0 * args.nq)   # two vectors tested per pool
    meas[D] = su["results"] / args.nq
    # the same recursion fed with the index's own pool scores: 64 queries of
    # the batch against 16,384 sampled pools of each level
    t1 = time.time()
    plan = cm.plan(idx, w.queries[:64], args.rho, levels=list(range(first_sparse, D + 1)))
    plan_s = time.time() - t1
    ps = plan["survivors"]
    ratio = {l: (ps[l] / meas[l] if meas[l] > 0 else None) for l in sorted(meas)}
    cost_model = {
        "sample": "16 queries x 65,536 random rows of this workload",
        "lambda_moment_fit": round(lam_m, 2),
        "lambda_loghist_fit": round(lam_h, 2),
        "E_rho_eq3": {"moment": round(cm.expected_tests(w.n, args.rho, lam_m), 1),
                      "loghist": round(cm.expected_tests(w.n, args.rho, lam_h), 1)},
        "survivors_per_query": {l: {"moment": round(pm[l], 1), "loghist": round(ph[l], 1),
                                    "sampled_pools": round(ps[l], 1),
                                    "measured": round(meas[l], 1)} for l in sorted(meas)},
        "sampled_model": {
            "sample": "64 queries of the batch x 16,384 pools of each level (float32 sums)",
            "seconds": round(plan_s, 2),
            "predicted_over_measured": {l: (round(v, 3) if v is not None else None)
                                        for l, v in ratio.items()},
            "within_2x": all(v is not None and 0.5 <= v <= 2.0 for v in ratio.values()),
            "dense_level": plan["dense_level"],
            "dense_level_walked": first_sparse,
            "entries_per_tile": round(plan["entries_per_tile"], 1),
            "results_per_query": round(plan["results_per_query"], 1),
        },
    }
    log(f"cost model: lambda {lam_m:.1f} (moments) / {lam_h:.1f} (log histogram); survivors "
        "per query TNE moments / TNE log-histogram / sampled pools / measured " +
        ", ".join(f"L{l} {v['moment']}/{v['loghist']}/{v['sampled_pools']}/{v['measured']}"
                  for l, v in cost_model["survivors_per_query"].items()) +
        f"; sampled model's dense level {plan['dense_level']} (walked {first_sparse})")

    # ---- the same batch at the other thresholds: walk vs exhaustive GEMM
    rho_sweep = {}
    if not args.no_side:
        for r in (0.8, 0.95):
            rr, wr = run_pipelined(args.pool, args.steps, 2, args.streams, rho=r)
            ex, we, _ = run("exh", 2, 1, rho=r)
            same = rr.total == ex.total and all(
                np.array_equal(a[0], b[0]) for a, b in zip(rr.to_lists(), ex.to_lists()))
            rho_sweep[r] = {"queries_per_s": round(args.nq * args.steps / wr, 1),
                            "ms_per_batch": round(wr / args.steps * 1e3, 4),
                            "results": rr.total, "exhaustive_queries_per_s": round(args.nq * 2 / we, 1),
                            "ids_identical_to_exhaustive": bool(same)}
            log(f"rho={r}: {rho_sweep[r]}")

    # ---- precision variant: batches of nq_variant queries, bfloat16 and
    # float8 pools (same database), each with the roofline of its dominant kernel
    variant = None
    if args.nq_variant > 0 and not args.no_side:
        nqv = args.nq_variant
        qv = q_all[:nqv]
        variant = {"workload": f"softmax(z/0.2) unit features N={w.n} d={w.d} float32, "
                               f"{nqv} queries per batch with planted neighbours, rho={args.rho}",
                   "global_batch": nqv}
        ref_lists = None
        for pool in ("bf16", "fp8"):
            steps_v = max(5, args.steps // 2)
            # the stream count for this batch size, from a short untimed
            # trial: with 4096-query batches two streams measured faster than
            # three (a third batch in flight only competes for L2), with
            # 1024-query batches three
            trial = {}
            for sv in sorted({2, args.streams}):
                _, wt = run_pipelined(pool, 4, 2, sv, qq=qv)
                trial[sv] = wt
            sv = min(trial, key=trial.get)
            rv, wv = run_pipelined(pool, steps_v, 2, sv, qq=qv)
            rl, _, _ = measure_roofline(idx, qv, args.rho, pool, nqv, args.walk_subtract, w.d, 3)
            lists = rv.to_lists()
            same = ref_lists is None or all(np.array_equal(a[0], b[0]) for a, b in zip(lists, ref_lists))
            ref_lists = ref_lists or lists
            variant[pool] = {"queries_per_s": round(nqv * steps_v / wv, 1),
                             "ms_per_batch": round(wv / steps_v * 1e3, 4), "results": rv.total,
                             "pipeline": {"workspaces": max(2, sv), "streams": sv,
                                          "trial_ms_per_batch": {str(k): round(v / 4 * 1e3, 3)
                                                                 for k, v in trial.items()}},
                             "ids_identical_to_bf16": bool(same), "roofline": rl}
            log(f"{nqv}-query batches, {pool} pools: {variant[pool]['ms_per_batch']} ms/batch, "
                f"{variant[pool]['queries_per_s']:.0f} queries/s, roofline {rl['kernel']} "
                f"{rl['frac']}")
        del ref_lists

    sweep = None
    if args.sweep_dense:
        sweep = {}
        for dl in [-1] + list(range(max(1, D - 9), D)):
            idx.set_option("dense_last", dl)
            _, wl, _ = run(args.pool, 5, 1)
            sweep[dl] = round(wl / 5 * 1e3, 3)
        idx.set_option("dense_last", args.dense_last)
        log(f"dense_last sweep (ms/batch): {sweep}")

    sub_sweep = None
    if args.sweep_subtract:
        sub_sweep = {}
        for ws in (0, 1, 2):
            idx.set_option("walk_subtract", ws)
            _, wl, _ = run(args.pool, 5, 1)
            idx.set_option("profile", 1)
            ps = []
            for _ in range(3):
                idx.query(q, args.rho, pool=args.pool)
                ps.append(idx.stats())
            idx.set_option("profile", 0)
            sub_sweep[ws] = {"ms_batch": round(wl / 5 * 1e3, 3),
                             **{k: round(float(np.median([p[k] for p in ps])), 4)
                                for k in ("ms_dense", "ms_frontier", "ms_leaf", "ms_total")},
                             "leaf_pairs": ps[-1]["leaf_pairs"],
                             "tests_per_level": list(ps[-1]["pairs"])}
        idx.set_option("walk_subtract", args.walk_subtract)
        log(f"walk_subtract sweep: {sub_sweep}")

    # ---- comparators and recall against the exhaustive GEMM
    comparators = {}
    exh = None
    if not args.no_side:
        for pool in ("f32", "fp8", "bf16", "max_bf16"):
            if pool == args.pool:
                continue
            r2, wall2, lat2 = run(pool, args.side_steps, 1)
            comparators[f"walk_{pool}_qps"] = round(args.nq * args.side_steps / wall2, 1)
            comparators[f"walk_{pool}_ms"] = round(wall2 / args.side_steps * 1e3, 3)
            if pool == "fp8":
                # the precision variant in the headline's own launch shape
                # (batches back to back over the same workspaces and streams)
                rp, wp = run_pipelined(pool, args.steps, args.warmup, args.streams)
                comparators["walk_fp8_pipelined_qps"] = round(args.nq * args.steps / wp, 1)
                comparators["walk_fp8_pipelined_ms"] = round(wp / args.steps * 1e3, 4)
                comparators["walk_fp8_ids_identical"] = rp.total == res.total and all(
                    np.array_equal(a[0], b[0]) for a, b in zip(rp.to_lists(), res.to_lists()))
                log(f"fp8 walk, batches back to back: {comparators['walk_fp8_pipelined_ms']} ms/batch, "
                    f"{comparators['walk_fp8_pipelined_qps']:.0f} queries/s")
            if pool == "max_bf16":
                # Our-Max pools (paper Sec. 2): same result set, other pruning
                comparators["walk_max_bf16_results_identical"] = r2.total == res.total and all(
                    np.array_equal(a[0], b[0]) for a, b in zip(r2.to_lists(), res.to_lists()))
                idx.set_option("profile", 1)
                idx.query(q, args.rho, pool="max_bf16")
                sm = idx.stats()
                idx.set_option("profile", 0)
                comparators["walk_max_bf16_stage_ms"] = {
                    k[3:]: round(sm[k], 4) for k in ("ms_dense", "ms_frontier", "ms_leaf", "ms_total")}
                comparators["walk_max_bf16_tests_per_level"] = {
                    l: sm["pairs"][l] for l in range(len(sm["pairs"])) if sm["pairs"][l]}
                comparators["walk_max_bf16_leaf_pairs"] = sm["leaf_pairs"]
        exh, wall3, lat3 = run("exh", max(2, args.side_steps // 2), 1)
        n3 = max(2, args.side_steps // 2)
        comparators["exhaustive_f32_qps"] = round(args.nq * n3 / wall3, 1)
        comparators["exhaustive_f32_ms"] = round(wall3 / n3 * 1e3, 3)
        idx.set_option("profile", 1)
        exh = idx.exhaustive(q, args.rho)
        se = idx.stats()
        idx.set_option("profile", 0)
        comparators["exhaustive_gemm_ms"] = se["ms_gemm"]
        # algorithmic flops 2 B N d; the GEMM itself runs over d_pad columns
        flops = 2.0 * args.nq * w.n * w.d
        comparators["exhaustive_gemm_tflops"] = round(flops / (se["ms_gemm"] * 1e-3) / 1e12, 1) \
            if se["ms_gemm"] > 0 else None
        comparators["exhaustive_gemm_tflops_over_d_pad"] = round(
            2.0 * args.nq * w.n * su["d_pad"] / (se["ms_gemm"] * 1e-3) / 1e12, 1) \
            if se["ms_gemm"] > 0 else None
    walk_lists = res.to_lists()
    recall = None
    if exh is not None:
        ex_lists = exh.to_lists()
        same = all(np.array_equal(a[0], b[0]) for a, b in zip(walk_lists, ex_lists))
        tot_ex = sum(len(b[0]) for b in ex_lists)
        hit = sum(len(np.intersect1d(a[0], b[0])) for a, b in zip(walk_lists, ex_lists))
        recall = hit / tot_ex if tot_ex else 1.0
        if not same:
            log("WARNING: walk and exhaustive results differ")

    # ---- CPU oracle on a bounded sample of the same batch
    cpu = None
    if not args.no_cpu and args.cpu_sample > 0:
        ns = min(args.cpu_sample, args.nq)
        cpu = cpu_baseline(w, ns, args.nq, args.rho, walk_lists)

    out = {
        "metric": METRIC,
        "value": round(qps, 1),
        "unit": "queries/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.pool,
        "data": "synthetic",
        "config": {"workload": f"softmax(z/0.2) unit features N={w.n} d={w.d} float32, "
                               f"{args.nq} queries per batch with planted neighbours, "
                               f"rho={args.rho}, {args.pool} pool sums",
                   "global_batch": args.nq, "n": w.n, "d": w.d, "rho": args.rho,
                   "pool": args.pool},
        "latency_ms": {"p50": round(pct(lat, 50), 4), "p99": round(pct(lat, 99), 4)},
        "one_call_at_a_time_qps": round(qps_sync, 1),
        "pipelined_results_identical": bool(same_p),
        "pipeline": {"workspaces": max(2, args.streams), "streams": args.streams},
        "results_per_batch": res.total,
        "recall_vs_exhaustive": recall,
        "index_build_ms": round(build_s * 1e3, 1),
        "roofline": roofline,
        "comparators": comparators,
        "cpu_baseline": cpu,
    }
    out["cost_model"] = cost_model
    if rho_sweep:
        out["rho_sweep"] = rho_sweep
    if variant is not None:
        out["precision_variant"] = variant
    if sweep is not None:
        out["dense_last_sweep_ms"] = sweep
    if sub_sweep is not None:
        out["walk_subtract_sweep"] = sub_sweep
    idx.close()
    del idx, q
    torch.cuda.empty_cache()
    if args.signed_n > 0 and not args.no_side:
        out["signed"] = signed_leg(args, torch, gt, synth, dev)
        torch.cuda.empty_cache()
    if args.serve_seconds > 0:
        out["serving"] = serving_leg(args.serve_seconds, torch, gt, synth, dev)
        out["serving_stress"] = stress_serving_leg(args.serve_seconds, torch, gt, synth, dev)
    print(json.dumps(out), flush=True)
    if args.copy_calib:
        src = torch.ones(1 << 28, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        log("copy reference: 1 GiB read + 1 GiB written")


def cpu_baseline(w, ns, nq, rho, walk_lists):
    """The CPU oracle (canonical float64 scan) timed on the first ns queries of
    a batch against the full database, and its ids compared with the GPU's."""
    import oracle.brute as ob

    threads = ob.default_threads()
    model, nproc = cpu_info()
    t1 = time.perf_counter()
    ora = ob.range_search(w.feats, w.queries[:ns], rho, nthreads=threads)
    cpu_s = time.perf_counter() - t1
    match = all(np.array_equal(walk_lists[b][0], ora[b][0]) for b in range(ns))
    log(f"oracle: {ns} queries in {cpu_s:.1f}s on {threads} threads, match={match}")
    return {"value": round(ns / cpu_s, 3), "unit": "queries/s", "cores": threads,
            "kind": "oracle", "cpu_model": model, "nproc": nproc,
            "sample": f"first {ns} of the {nq} queries against the full database "
                      f"(N={w.n}, d={w.d}); canonical float64 scan, {cpu_s:.1f} s",
            "ids_match_gpu": bool(match)}


def signed_leg(args, torch, gt, synth, dev):
    """Descriptors with negative values (paper Sec. 2: max/min pools): centred
    softmax rows unit(softmax(z/0.2) - 1/d), N = signed_n, d = 512 (the signed
    index's limit), 1024 queries with planted neighbours, rho = args.rho.  The
    max/min walk over bfloat16 and float32 rows and the exhaustive path on the
    same index, timed per call; its leaf and walk against the HBM roofline from
    the distinct rows they read; the CPU oracle on a sample."""
    nq, d = 1024, 512
    w = synth.workload_signed(args.signed_n, d, nq, rho=args.rho, geometric_planted=True)
    F = torch.from_numpy(w.feats).to(dev)
    t0 = time.perf_counter()
    idx = gt.GTIndex(F, pools=("max_f32", "max_bf16", "signed"))
    torch.cuda.synchronize()
    build_ms = (time.perf_counter() - t0) * 1e3
    del F
    q = torch.from_numpy(w.queries).to(dev)
    st0 = idx.stats()
    D, dp, pw = st0["depth"], st0["d_pad"], st0["pool_width"]
    out = {"workload": f"centred softmax unit(softmax(z/0.2) - 1/d) N={w.n} d={d} float32, "
                       f"{nq} queries with planted neighbours, rho={args.rho}, max/min pools",
           "shift_bound": st0["shift_bound"], "pool_width": pw, "index_build_ms": round(build_ms, 1)}
    ref = None
    for pool in ("max_bf16", "max_f32", "exh"):
        call = (lambda: idx.exhaustive(q, args.rho)) if pool == "exh" else \
            (lambda: idx.query(q, args.rho, pool=pool))
        for _ in range(2):
            r = call()
        torch.cuda.synchronize()
        steps = 10
        t1 = time.perf_counter()
        for _ in range(steps):
            r = call()
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t1) / steps * 1e3
        lists = r.to_lists()
        if ref is None:
            ref = lists
        same = all(np.array_equal(a[0], b[0]) for a, b in zip(lists, ref))
        key = "exhaustive_f32" if pool == "exh" else f"walk_{pool}"
        out[key] = {"ms_per_call": round(ms, 3), "queries_per_s": round(nq / ms * 1e3, 1),
                    "results": r.total, "ids_identical_to_max_bf16": bool(same)}
        if pool != "exh":
            idx.set_option("profile", 1)
            idx.query(q, args.rho, pool=pool)
            sp = idx.stats()
            idx.set_option("profile", 0)
            idx.set_option("count_unique", 1)
            idx.query(q, args.rho, pool=pool)
            su = idx.stats()
            idx.set_option("count_unique", 0)
            esz = 2 if pool == "max_bf16" else 4
            walk_b = sum(su["unique_rows"][l] for l in range(1, D)) * pw * esz
            leaf_b = su["unique_rows"][D] * dp * 4
            ms_walk = sp["ms_dense"] + sp["ms_frontier"]
            out[key].update({
                "stage_ms": {k[3:]: round(sp[k], 4)
                             for k in ("ms_prep", "ms_dense", "ms_frontier", "ms_leaf", "ms_total")},
                "tests_per_level": {l: sp["pairs"][l] for l in range(D) if sp["pairs"][l]},
                "leaf_pairs": sp["leaf_pairs"],
                "leaf_GBps": round(leaf_b / (sp["ms_leaf"] * 1e-3) / 1e9, 1) if sp["ms_leaf"] else None,
                "leaf_frac_of_8TBps": round(leaf_b / (sp["ms_leaf"] * 1e-3) / 8e12, 4) if sp["ms_leaf"] else None,
                "walk_GBps": round(walk_b / (ms_walk * 1e-3) / 1e9, 1) if ms_walk else None,
                "algorithmic_bytes": {"walk_rows": walk_b, "leaf_rows": leaf_b}})
        log(f"signed {pool}: {ms:.3f} ms/call, {r.total} results, same={same}")
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(w, 64, nq, args.rho, ref)
    idx.close()
    return out


def _serve_runs(srv_factory, make_q, rho_of, max_batch, seconds, loads, seed_workload,
                insert_rows=None, saturated_requests=400):
    """Saturated rate (a backlog of requests present at t = 0), then a Poisson
    run of `seconds` at each offered load (a fraction of the saturated rate),
    with inserts every 10 ms if insert_rows is given."""
    from paper_2311_02573_amd import serve, synth

    sched = [(0.0, k) for _, k in synth.poisson_arrivals(seed_workload, float(saturated_requests),
                                                         1.0, max_batch, seed_offset=1)]
    srv = srv_factory()
    reqs, wall, _ = serve.run_poisson(srv, sched, make_q, rho_of, 0.0)
    sat = sum(r.nq for r in reqs) / wall
    out = {"saturated_qps": round(sat, 1), "saturated_memory": srv.summary()}
    log(f"serving: saturated {sat:.0f} queries/s ({len(reqs)} requests in {wall:.2f}s), "
        f"{srv.summary()}")
    mean_batch = (max_batch + 1) / 2.0
    for load in loads:
        rate = load * sat / mean_batch
        sched = synth.poisson_arrivals(seed_workload, rate, seconds, max_batch,
                                       seed_offset=int(load * 10))
        srv = srv_factory()
        n_ins = [0]

        def ins(k):
            rows = insert_rows(k)
            n_ins[0] += len(rows)
            return rows

        reqs, wall, _ = serve.run_poisson(
            srv, sched, make_q, rho_of, seconds,
            insert_every_s=0.01 if insert_rows is not None else None,
            insert_rows=ins if insert_rows is not None else None,
            progress=lambda t: log(f"  load {load:.0%}: {t:.0f} s"))
        lat = serve.latency_summary(reqs)
        nq_tot = sum(r.nq for r in reqs)
        out[f"load_{int(load * 100)}"] = dict(
            seconds=round(wall, 1), offered_qps=round(load * sat, 1),
            achieved_qps=round(nq_tot / wall, 1), inserted_rows=n_ins[0],
            inserts_per_s=round(n_ins[0] / wall, 1), memory=srv.summary(), **lat)
        log(f"serving at {load:.0%}: {lat}, {n_ins[0]} rows inserted, {srv.summary()}")
    return out, srv


def serving_leg(seconds, torch, gt, synth, dev):
    """Continuous batching with admission by memory under load.

    Serving workload: N0 = 2^22 float16 rows, d = 512, capacity 2^23,
    requests of U{1..512} queries at rho = 0.9 arriving as a Poisson process,
    10,000 inserted rows per second in groups of 100 every 10 ms; an 8 GiB
    arena for the calls' memory, four streams, calls of up to 1024 queries.
    The saturated rate is measured first (every request waiting at t = 0);
    loaded runs offer 50% and 80% of it.  Latency = completion - arrival, host
    clock."""
    from paper_2311_02573_amd import serve

    t0 = time.time()
    w = synth.workload3()
    feats = w.feats.to(dev)
    qpool = torch.from_numpy(w.queries).to(dev)
    idx = gt.GTIndex(feats, capacity=w.capacity, pools=("f32", "bf16"))
    torch.cuda.synchronize()
    del feats
    log(f"serving index: N0={w.n} d={w.d} f16, capacity {w.capacity}, built in "
        f"{time.time() - t0:.1f}s (incl. generation)")
    # one synchronous 1024-query call, kernel groups timed with HIP events
    idx.query(qpool[:1024], float(w.rho[0]))
    idx.set_option("profile", 1)
    r1 = idx.query(qpool[:1024], float(w.rho[0]))
    st = idx.stats()
    idx.set_option("profile", 0)
    call = {k: round(st[k], 3) for k in ("ms_total", "ms_dense", "ms_frontier", "ms_leaf",
                                         "ms_recheck", "ms_compact")}
    call["results"] = r1.total
    call["leaf_pairs"] = st["leaf_pairs"]
    call["leaf_level_entries"] = st["entries"][st["depth"] - 1]
    call["depth"] = st["depth"]
    log(f"serving index, one 1024-query call: {call}")
    # streaming inserts: groups of 100 rows (the serving rate's unit) and one
    # bulk insert, each call timed to completion on the host clock
    ins_lat = []
    for k in range(50):
        rows = torch.from_numpy(synth.insert_rows(3, 100, w.d, w.temp, offset=100000 + k)).to(
            dev, torch.float16)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        idx.insert(rows)
        torch.cuda.synchronize()
        ins_lat.append((time.perf_counter() - t1) * 1e3)
    bulk = torch.from_numpy(synth.insert_rows(3, 100000, w.d, w.temp, offset=200000)).to(
        dev, torch.float16)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    idx.insert(bulk)
    torch.cuda.synchronize()
    bulk_s = time.perf_counter() - t1
    del bulk
    inserts = {"group_100_rows_ms": {"p50": round(pct(ins_lat, 50), 3), "p99": round(pct(ins_lat, 99), 3)},
               "groups_of_100_rows_per_s": round(100 * 1e3 / float(np.mean(ins_lat)), 1),
               "bulk_100000_rows_per_s": round(1e5 / bulk_s, 1)}
    log(f"serving index, inserts: {inserts}")
    from paper_2311_02573_amd import costmodel as cm

    plan = cm.plan(idx, w.queries[:64], float(w.rho[0]))
    if plan["dense_level"] is not None:
        idx.set_option("dense_start", plan["dense_level"])
    log(f"serving index, sampled cost model: dense level {plan['dense_level']}, "
        f"entries per tile {plan['entries_per_tile']:.0f}, results per query "
        f"{plan['results_per_query']:.0f}")
    backend = serve.GpuBackend(idx)
    nqp = qpool.shape[0]
    make_q = lambda i, k: qpool[(i * 613) % (nqp - 512):(i * 613) % (nqp - 512) + k]
    rho_of = lambda i, k: np.full(k, w.rho[0])
    ins_rows = lambda k: torch.from_numpy(synth.insert_rows(3, 100, w.d, w.temp, offset=k)).to(
        dev, torch.float16)
    budget = 8 << 30
    est = serve.Estimator(entries_per_tile=plan["entries_per_tile"],
                          pairs_per_query=max(1.0, plan["results_per_query"]))

    def factory():
        return serve.Server(backend, budget, streams=4, max_queries=1024, pool="bf16", estimator=est)

    runs, srv = _serve_runs(factory, make_q, rho_of, 512, seconds, (0.5, 0.8), 3, ins_rows)
    out = {"workload": f"N0={w.n} d={w.d} float16, capacity {w.capacity}, bf16 pools, "
                       "requests U{1..512} queries at rho=0.9, Poisson arrivals, "
                       "inserts 10000/s in groups of 100",
           "admission": f"by memory: {budget >> 30} GiB arena, 4 streams, calls of up to 1024 queries",
           "call_1024_queries": call, "inserts": inserts,
           "sampled_cost_model": {"dense_level": plan["dense_level"],
                                  "entries_per_tile": round(plan["entries_per_tile"], 1),
                                  "results_per_query": round(plan["results_per_query"], 1)},
           **runs}
    del srv, backend
    idx.close()
    torch.cuda.empty_cache()
    return out


def stress_serving_leg(seconds, torch, gt, synth, dev):
    """Continuous batching on the stress workload: N = 2^24 rows softmax(z/0.3)
    stored as bfloat16, d = 256; 64 centres with 10^4 near-duplicates each
    (logit noise sigma 0.02) written over uniformly chosen rows; a pool of
    8192 queries of which 10% are a centre plus the same noise (about 10^4
    neighbours each); requests of U{1..2048} queries, each request with its
    own rho uniform in [0.75, 0.95]; admission by memory from a 48 GiB arena,
    four streams, calls of up to 2048 queries.  Saturated rate, then a
    Poisson run at 80% of it; a sample of requests is compared with the
    same queries run alone."""
    from paper_2311_02573_amd import serve

    t0 = time.time()
    w = synth.workload4(n=1 << 24, d=256, nq=8192, clusters=64, per_cluster=10000)
    feats = w.feats.to(dev)
    qpool = torch.from_numpy(w.queries).to(dev)
    idx = gt.GTIndex(feats, pools=("f32", "bf16"))
    torch.cuda.synchronize()
    del feats
    log(f"stress index: N={w.n} d={w.d} bf16, built in {time.time() - t0:.1f}s (incl. generation)")
    g = np.random.default_rng(synth.stream_seed(4, synth.STREAM_ARRIVAL) + 7)
    backend = serve.GpuBackend(idx)
    nqp = qpool.shape[0]
    # queries in pool order, so every request mixes cluster and plain queries
    # as the pool does (cluster queries are its first 10%, spread by a stride)
    perm = torch.from_numpy(g.permutation(nqp)).to(dev)
    qperm = qpool[perm]
    make_q = lambda i, k: qperm[(i * 1031) % (nqp - 2048):(i * 1031) % (nqp - 2048) + k]
    rho_req = g.uniform(0.75, 0.95, size=1 << 16)
    rho_of = lambda i, k: np.full(k, rho_req[i % len(rho_req)])
    from paper_2311_02573_amd import costmodel as cm

    plan = cm.plan(idx, w.queries[::128][:64], 0.85)
    log(f"stress index, sampled cost model at rho 0.85: entries per tile "
        f"{plan['entries_per_tile']:.0f}, results per query {plan['results_per_query']:.0f}")
    budget = 48 << 30
    est = serve.Estimator(entries_per_tile=plan["entries_per_tile"],
                          pairs_per_query=max(1.0, plan["results_per_query"]))

    def factory():
        return serve.Server(backend, budget, streams=4, max_queries=2048, pool="bf16", estimator=est)

    runs, srv = _serve_runs(factory, make_q, rho_of, 2048, seconds, (0.8,), 4,
                            saturated_requests=60)
    # a sample of the last run's requests against the same queries alone
    same = True
    for r in srv.finished[:: max(1, len(srv.finished) // 6)][:6]:
        alone = idx.query(r.queries, r.rho, pool="bf16").to_lists()
        same = same and all(np.array_equal(a[0], b[0]) for a, b in zip(r.results, alone))
    out = {"workload": f"softmax(z/0.3) N={w.n} d={w.d} bfloat16, 64 centres x 10^4 "
                       "near-duplicates (sigma 0.02), 10% cluster queries, requests U{1..2048} "
                       "queries, per-request rho U[0.75, 0.95]",
           "admission": f"by memory: {budget >> 30} GiB arena, 4 streams, calls of up to 2048 queries",
           "mix_equals_alone_sample": bool(same), **runs}
    del srv, backend
    idx.close()
    torch.cuda.empty_cache()
    return out


if __name__ == "__main__":
    main()
