#!/usr/bin/env python3
"""Benchmark: schedulability evaluations per second on one MI355X.

A step is one pass of the whole hot path over one batch resident in HBM:
validation and per-set precompute (prep kernel), evaluation of every
(task set, partitioning) pair with heuristic allocation and per-partition
response-time tests (eval kernel), selection of the best triple, response
times of the chosen triple and of the whole-GPU baseline (final kernel).

Default workload (c3): 1,000,000 seeded synthetic task sets of uneven size,
n uniform in 4..32 tasks, M drawn from {16, 48, 80, 108} compute units,
constrained deadlines, at most K = 4 partitions (3.84e9 evaluations per
step), BF-INA heuristic allocation, run by the batched form (persistent,
autotuned, HIP-graph-captured launch sequences, one per size class).  The
same batch is also timed through the plain one-launch-sequence path, the
first 2,000 sets through the one-launch-per-set path, the 100,000-set n = 10,
M = 80 workload (c2) through its own batched plan, and open-loop serving runs
(uneven queries, Poisson arrivals from 10,000 queries/s up) give p50/p99
admission latency and the saturation rate.

Other workloads: c2 (100,000 sets, n = 10, M = 80), c4 (exhaustive stress,
1,000 sets of 12 tasks on 48 units, every allocation), c5 (serving sweep),
fig4 and fig6 (the paper's Algorithm 1 with free partition sizes on its
Fig. 4 and Figs. 6-8 workloads: 34,000 sets of 50 or of 200 tasks on 68
units; value in task sets/s, with the analysis time per utilisation point).

Prints one JSON line (metric, value in evals/s, ms_per_step, roofline of the
dominant kernel from HIP events on its launch stream, and the CPU oracle timed
on a bounded sample of the same workload on the host's cores).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "schedulability evals/sec (taskset×partitioning); p99 admission latency"
# Minimal VALU issue slots (lane-operations at full rate) per unit of work of
# the engine's algorithm: a response-time term is 3 integer multiplies
# (v_mul_hi_u32 and two v_mad_u64_u32), each issued at quarter rate on CDNA;
# an exact partition test sets up its conflict mask and sums (8); a candidate
# answered from the feasibility frontier is a mask OR, a compare and the
# utilisation update (6).
C_TERM = 9
C_TEST = 8
C_LOOK = 6
# 256 CUs x 128 full-rate 32-bit VALU lane-operations per clock x 2.4 GHz: the
# chip's vector rate (its fp32 vector peak of 157.3 TFLOP/s is 78.6 T fused
# multiply-adds per second, 128 lanes per CU per clock); an add-chain kernel
# measures 65 T lane-operations/s on the device (reported beside it)
PEAK_INT_LANE_OPS = 256 * 128 * 2.4e9


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def kernel_hash() -> str:
    """Hash of the sources the engine library is built from (the library carries the same)."""
    from paper_2105_10312_amd import build
    return build.source_hash()


def traffic_bytes(name):
    """HBM bytes per eval launch from the committed rocprofv3 counter summary,
    or None if it is missing or was taken on a different kernel source."""
    try:
        with open(os.path.join(ROOT, "profiles", name)) as f:
            d = json.load(f)
    except (OSError, ValueError):
        return None
    if d.get("kernel_sha256_16") != kernel_hash():
        return None
    return d.get("hbm_bytes_per_launch")


def cpu_baseline(ts, K, mode, sample_sets, threads, stride=1, admissible=None, policy="FP_DM", flags=0):
    import numpy as np

    import oracle
    from paper_2105_10312_amd import workload
    idx = np.arange(0, ts.n_sets, stride)[:sample_sets]
    sub = workload.subset(ts, idx)
    P = int(sum(oracle.count_partitionings(int(m), K) for m in sub["M"]))
    t0 = time.perf_counter()
    r = oracle.solve(sub, K, mode, nthreads=threads, counters=True, admissible=admissible, policy=policy,
                     flags=flags)
    dt = time.perf_counter() - t0
    c = r["counters"].sum(axis=0)
    return {"evals": P, "seconds": dt, "terms": int(c[0]), "tests": int(c[1]), "combines": int(c[2]),
            "sets": sub.n_sets}


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def lemma1_pruned(ts):
    """Sets that the whole-GPU utilisation bound rejects before any partitioning
    is tried (Lemma 1, floor-Q32 sum of one-unit utilisations above M), computed
    exactly in int64: floor(Cn*2^32/T) = (Cn//T)*2^32 + floor((Cn%T)*2^32/T),
    each term clamped above M*2^32 so the per-set sums cannot overflow."""
    import numpy as np
    if "Cn_table" in ts:  # explicit tables: Cn(1) is each task's first entry
        sizes = np.diff(ts["set_offset"])
        local = np.arange(ts["T"].shape[0]) - np.repeat(ts["set_offset"][:-1], sizes)
        cn = ts["Cn_table"][np.repeat(ts["table_offset"], sizes) + local * np.repeat(ts["M"].astype(np.int64), sizes)]
    else:
        cn = ts["C_seq"] + ts["C_par"]
    T = ts["T"]
    q, r = cn // T, cn % T
    cap = (int(ts["M"].max()) + 1) << 32
    term = np.minimum(q, cap >> 32) * (1 << 32) + (r << 32) // T
    term = np.minimum(term, cap)
    sums = np.add.reduceat(term, ts["set_offset"][:-1])
    return int((sums > ts["M"].astype(np.int64) << 32).sum())


def timed(fn, steps, sync):
    sync()
    t0 = time.perf_counter()
    for _ in range(steps):
        fn()
    sync()
    return (time.perf_counter() - t0) * 1000.0 / steps


def serving_leg(eng, capart, workload, rate, n_queries, seed=5):
    import numpy as np
    ts = workload.config_c5(seed=seed, n_queries=n_queries)
    srv = capart.Server(eng.ctx, K=4, mode="BF_INA", max_tasks=64, max_M=108)
    warm = workload.subset(ts, np.arange(min(200, ts.n_sets)))
    srv.replay(warm, np.zeros(warm.n_sets), collect=False)
    rng = np.random.default_rng(seed)
    arrival = np.cumsum(rng.exponential(1e6 / rate, ts.n_sets))
    _, st = srv.replay(ts, arrival, collect=False)
    srv.close()
    return {"workload": f"{n_queries} queries, n log-uniform 2..64, M in {{16,48,80,108}}, K=4, BF_INA, "
                        f"Poisson arrivals at {rate:g} q/s", "offered_qps": rate, "p50_us": st["p50_us"],
            "p99_us": st["p99_us"], "mean_us": st["mean_us"], "max_us": st["max_us"], "qps": st["queries_per_s"],
            "evals_per_s": st["evals_per_s"], "mean_batch": st["mean_batch"], "rejected": st["rejected"]}


def workload_bounds(ts):
    """Per set, the total one-unit utilisation without any conflict (best) and
    with every task in conflict (worst), as floats (exact ceil-Q32 terms summed
    in integers first)."""
    import numpy as np
    off = ts["set_offset"]
    T = ts["T"].astype(object)
    cn = (ts["C_seq"] + ts["C_par"]).astype(object)
    cc = (ts["k_permille"].astype(object) * cn + 999) // 1000
    q = 1 << 32
    un = -((-cn * q) // T)
    uc = -((-cc * q) // T)
    best = np.array([float(sum(un[off[s]:off[s + 1]])) / q for s in range(ts.n_sets)])
    worst = np.array([float(sum(uc[off[s]:off[s + 1]])) / q for s in range(ts.n_sets)])
    return best, worst


def alg1_cpu_baseline(ts, mode, threads, policy="FP_DM"):
    """The oracle's Algorithm 1 over every set of the workload, on `threads` host threads."""
    from concurrent.futures import ThreadPoolExecutor

    import oracle
    t0 = time.perf_counter()
    with ThreadPoolExecutor(threads) as ex:
        v = list(ex.map(lambda s: oracle.alg1(ts.set(s), mode, policy=policy)["verdict"], range(ts.n_sets)))
    return {"seconds": time.perf_counter() - t0, "sets": ts.n_sets, "schedulable": int(sum(v))}


def alg1_main(args, eng, capart, workload, sync, threads, valu_ops):
    """Algorithm 1 with free partition sizes on the paper's workloads: fig4
    (n = 50 tasks, Figs. 4-5) or fig6 (n = 200 tasks, Figs. 6-8), M = 68
    units, U = 2..68 step 2, `--n-sets` sets per point (default 1000); one
    step = the whole batch through capart_alg1_async.  Also the analysis time
    per utilisation point (Fig. 8): each point's sets in a launch of their own."""
    import numpy as np
    import torch
    mode = args.mode
    pol = args.policy
    n = 50 if args.workload == "fig4" else 200
    fig = "Fig. 4" if n == 50 else "Figs. 6-8"
    per_point = args.n_sets or 1000
    ts = workload.config_paper_fig4(sets_per_point=per_point, n=n)
    S, N = ts.n_sets, ts.n_tasks
    desc = (f"paper {fig}: {S} task sets ({per_point} per point, U = 2..68 step 2), n={n}, M=68, "
            f"D=0.75T, T log-uniform 50..4000 us, Algorithm 1 {mode}" + (f", {pol} per partition" if pol != "FP_DM" else ""))
    log(f"[bench] workload {args.workload}: {desc}")
    dev = capart.device_tasksets(ts)
    out = capart.device_alg1_results(S, N)

    def step():
        capart.capart_alg1_async(eng.ctx, dev, mode, out, max_tasks=n, max_M=68, policy=pol)

    for i in range(args.warmup):
        step()
        sync()
        log(f"[bench] warmup {i + 1}/{args.warmup} done")
    st = out["status"][:S].cpu().numpy()
    if not (st == 0).all():
        raise SystemExit(f"bench: {int((st != 0).sum())} sets reported errors")
    ms_per_step = timed(step, args.steps, sync)
    value = S / (ms_per_step / 1000.0)
    log(f"[bench] {args.steps} steps: {ms_per_step:.3f} ms/step, {value:.4g} sets/s")
    capart.capart_timing_enable(eng.ctx, True)
    capart.capart_timing_read(eng.ctx)
    ms_timed = timed(step, args.steps, sync)
    ms_k, n_k = capart.capart_timing_read(eng.ctx)
    capart.capart_timing_enable(eng.ctx, False)
    k_ms = ms_k["eval"] / max(1, n_k["eval"])
    verdict = out["verdict"][:S].cpu().numpy()
    nparts = out["nparts"][:S].cpu().numpy()
    tried = out["tried"][:S].cpu().numpy()
    wl = out["workload"][:S].cpu().numpy().astype(np.float64) / 2.0 ** 32
    rate = verdict.reshape(-1, per_point).mean(axis=1)
    # the efficiency plot (Figs. 5 and 7): per point, over the schedulable sets,
    # the mean scheduled workload against the no-interference (best) and the
    # all-interference (worst) totals, one-unit utilisations
    best, worst = workload_bounds(ts)
    eff = {}
    for i in range(len(rate)):
        sl = slice(i * per_point, (i + 1) * per_point)
        ok = verdict[sl] == 1
        eff[str(2 * (i + 1))] = None if not ok.any() else {
            "best": float(best[sl][ok].mean()), "worst": float(worst[sl][ok].mean()),
            "scheduled": float(wl[sl][ok].mean())}
    # analysis time by utilisation (Fig. 8): one point's sets per launch, HIP
    # events on the launch stream, the mean of three launches after a warmup
    per_U = {}
    s_launch = torch.cuda.current_stream()
    for i in range(len(rate)):
        sub = workload.subset(ts, np.arange(i * per_point, (i + 1) * per_point))
        dsub = capart.device_tasksets(sub)
        osub = capart.device_alg1_results(sub.n_sets, sub.n_tasks)
        capart.capart_alg1_async(eng.ctx, dsub, mode, osub, max_tasks=n, max_M=68, policy=pol)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(s_launch)
        for _ in range(3):
            capart.capart_alg1_async(eng.ctx, dsub, mode, osub, max_tasks=n, max_M=68, policy=pol)
        e1.record(s_launch)
        e1.synchronize()
        ms = e0.elapsed_time(e1) / 3
        per_U[str(2 * (i + 1))] = {"ms_per_launch": ms, "us_per_set": 1000.0 * ms / per_point}
        del dsub, osub
    log("[bench] analysis time by U (us per set): " +
        ", ".join(f"{u}: {v['us_per_set']:.2f}" for u, v in per_U.items()))
    wout = capart.device_alg1_results(S, N)
    work = capart.capart_alg1_count_work(eng.ctx, dev, mode, wout, n, 68, policy=pol)
    del wout
    log(f"[bench] Algorithm 1 kernel {k_ms:.3f} ms/launch, counted work {work}")
    ops = work["terms"] * C_TERM + work["tests"] * C_TEST
    achieved = ops / (k_ms / 1000.0)
    kname = "alg1_kernel" if n <= 64 else "alg1_big_kernel"
    roof = {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_INT_LANE_OPS / 1e12, "unit": "TOP/s",
            "frac": achieved / PEAK_INT_LANE_OPS,
            "traffic": traffic_bytes(f"{kname}_{args.workload}_{mode.lower()}{'_edf' if pol == 'EDF' else ''}"
                                     f"_traffic.json"),
            "kernel": kname, "kernel_ms": k_ms, "ops_per_launch": ops, "work_per_launch": work,
            "ops_per_term": C_TERM, "ops_per_test": C_TEST,
            "other_kernels_ms": {"prep": ms_k["prep"] / max(1, n_k["prep"])},
            "step_ms_with_kernel_events": ms_timed,
            "peak_measured": valu_ops / 1e12, "frac_of_measured_peak": achieved / valu_ops}
    cpu = None
    if not args.no_cpu:
        # fig4: every set; fig6: every 10th set (about 20 ms of oracle work per
        # 200-task set keeps the leg near 10-30 s)
        stride = 1 if n <= 64 else 10
        pick = np.arange(0, S, stride)
        sample = ts if stride == 1 else workload.subset(ts, pick)
        log(f"[bench] CPU oracle (Algorithm 1) on {sample.n_sets} sets with {threads} threads")
        cb = alg1_cpu_baseline(sample, mode, threads, pol)
        if cb["schedulable"] != int(verdict[pick].sum()):
            raise SystemExit("bench: the oracle's schedulable count differs from the GPU's")
        one = alg1_cpu_baseline(workload.subset(ts, np.arange(0, S, max(1, S // (500 if n <= 64 else 100)))),
                                mode, 1, pol)
        what = f"all {cb['sets']} sets of the workload" if stride == 1 else \
            f"{cb['sets']} sets (every {stride}th of the workload)"
        cpu = {"value": cb["sets"] / cb["seconds"], "unit": "sets/s", "cores": threads, "kind": "oracle",
               "sample": f"{what}, {cb['seconds']:.2f} s wall",
               "single_core": {"value": one["sets"] / one["seconds"],
                               "sample": f"{one['sets']} sets spread over the workload, {one['seconds']:.2f} s"},
               "cpu_model": cpu_model(), "host_cpus": os.cpu_count()}
        log(f"[bench] CPU oracle: {cpu['value']:.4g} sets/s")
    res = {"metric": "Algorithm 1 task sets/sec (free partition sizes)", "value": value, "unit": "sets/s",
           "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_per_step,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "int64", "data": "synthetic",
           "config": {"workload": desc, "n_sets": S, "n_tasks": n, "alloc_mode": mode, "policy": pol,
                      "sets_per_point": per_point},
           "schedulability_by_U": {str(2 * (i + 1)): float(r) for i, r in enumerate(rate)},
           "efficiency_by_U": eff,
           "analysis_time_by_U": per_U,
           "mean_partitions_when_schedulable": float(nparts[verdict == 1].mean()) if verdict.any() else None,
           "mean_merges_tried": float(tried.mean()),
           "roofline": roof, "cpu_baseline": cpu}
    eng.close()
    print(json.dumps(res), flush=True)


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="c3", choices=["c2", "c3", "c4", "c5", "fig4", "fig6"],
                    help="fig4 / fig6: the paper's Algorithm 1 (free partition sizes) on its 50-task (Fig. 4) "
                         "or 200-task (Figs. 6-8) workload")
    ap.add_argument("--mode", default="BF_INA", choices=["BF_INA", "BF_ACT", "SMS_INA", "SMS_ACT"])
    ap.add_argument("--n-sets", type=int, default=0, help="override the workload's number of sets")
    ap.add_argument("--cpu-sample", type=int, default=0, help="task sets timed on the CPU oracle (0 = default)")
    ap.add_argument("--cpu-threads", type=int, default=0, help="0 = all host cores (at most 16)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle leg (counts from a small sample)")
    ap.add_argument("--no-compare", action="store_true", help="skip the plain and per-set path comparisons")
    ap.add_argument("--no-serving", action="store_true", help="skip the serving leg")
    ap.add_argument("--form", default="batched", choices=["batched", "plain"],
                    help="GPU form timed for `value` (c2, c3)")
    ap.add_argument("--tables", action="store_true",
                    help="give the sets explicit per-task time tables (saturating memory-intensive profiles) "
                         "instead of the parametric model; runs the plain path")
    ap.add_argument("--schedule", default="auto", choices=["auto", "direct", "persistent"],
                    help="batched form: the autotuner's choice, or a fixed schedule (persistent: 8 blocks per CU, "
                         "4096-evaluation items, loop form 1; for reproducible counter runs)")
    ap.add_argument("--policy", default="FP_DM", choices=["FP_DM", "EDF"],
                    help="per-partition scheduling: fixed-priority DM (default) or EDF")
    ap.add_argument("--admissible", default="",
                    help="comma-separated admissible partition sizes (MIG-like restriction; default: every size)")
    ap.add_argument("--rates", default="",
                    help="c5: comma-separated offered rates in queries/s (default 1e3, 3e3, .., 1e6)")
    ap.add_argument("--no-graph", action="store_true",
                    help="batched form without HIP graph capture (same kernels and arguments; for counter runs)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="BYTES",
                    help="only run a plain device-to-device copy of BYTES (counter calibration) and exit")
    args = ap.parse_args()
    if args.copy_calibration:
        import torch
        n = args.copy_calibration // 4
        src = torch.arange(n, dtype=torch.int32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": 4 * n}), flush=True)
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: task sets would shard independently across GPUs, but no "
              "multi-GPU configuration is measured (use --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2105_10312_amd import capart, workload

    sync = torch.cuda.synchronize
    threads = args.cpu_threads or min(16, os.cpu_count() or 1)
    eng = capart.Engine(0)
    K = 4
    mode = args.mode
    # the integer VALU peak as measured on this device (reported beside the
    # nominal 256 CUs x 64 lanes x 2.4 GHz that `frac` uses)
    valu_ops, valu_ms = capart.capart_measure_valu(eng.ctx)
    log(f"[bench] measured full-rate int32 VALU: {valu_ops / 1e12:.2f} T lane-ops/s (kernel {valu_ms:.2f} ms)")
    if args.workload == "c5":
        # below and above the capacity of this query mix (about 2.7e4 queries/s)
        rates = [float(x) for x in args.rates.split(",")] if args.rates else [1e3, 3e3, 1e4, 3e4, 1e5, 3e5, 1e6]
        legs = []
        for r in rates:
            n_q = int(min(200000, max(2000, r * 2.0)))
            log(f"[bench] serving at {r:g} q/s, {n_q} queries")
            legs.append(serving_leg(eng, capart, workload, r, n_q))
            log(f"[bench]   p50 {legs[-1]['p50_us']:.1f} us p99 {legs[-1]['p99_us']:.1f} us "
                f"{legs[-1]['qps']:.4g} q/s")
        best = max(legs, key=lambda x: x["evals_per_s"])
        res = {"metric": METRIC, "value": best["evals_per_s"], "unit": "evals/s", "n_gpus": 1, "steps": len(rates),
               "warmup": 1, "ms_per_step": None, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
               "dtype": "int64", "data": "synthetic",
               "config": {"workload": "serving: open-loop Poisson admission queries, n log-uniform 2..64, "
                                      "M in {16,48,80,108}, K=4, BF_INA"},
               "serving": legs, "roofline": None, "cpu_baseline": None}
        eng.close()
        print(json.dumps(res), flush=True)
        return

    if args.workload in ("fig4", "fig6"):
        alg1_main(args, eng, capart, workload, sync, threads, valu_ops)
        return

    if args.workload == "c2":
        ts = workload.config_c2(n_sets=args.n_sets or 100_000)
        max_tasks, max_M, desc = 10, 80, "n=10, M=80"
        cpu_sample, cpu_stride = args.cpu_sample or 100_000, 1  # the whole batch
    elif args.workload == "c3":
        ts = workload.config_c3(n_sets=args.n_sets or 1_000_000)
        max_tasks, max_M, desc = 32, 108, "n uniform 4..32, M in {16,48,80,108}, constrained deadlines"
        cpu_sample, cpu_stride = args.cpu_sample or 10_000, 100
    else:
        ts = workload.config_c4(n_sets=args.n_sets or 1000)
        max_tasks, max_M, desc = 12, 48, "n=12, M=48, exhaustive allocation"
        mode = "EXH"
        cpu_sample, cpu_stride = 0, 1
    adm = tuple(int(x) for x in args.admissible.split(",")) if args.admissible else None
    if adm:
        desc += f", admissible sizes {args.admissible}"
    pol = args.policy
    if pol != "FP_DM":
        desc += f", {pol} per partition"
    if args.tables:
        ts = workload.with_time_tables(ts)
        for key in ("C_seq", "C_par", "k_permille"):
            del ts[key]
        desc += ", explicit time tables"
        args.form = "plain"
    log(f"[bench] workload {args.workload}: {ts.n_sets} sets, {desc}, K={K}, {mode}")
    Pcount = {int(m): capart.capart_count_partitionings(int(m), K) for m in np.unique(ts["M"])}
    evals_per_step = int(sum(Pcount[int(m)] for m in ts["M"]))
    dev = capart.device_tasksets(ts)
    out = capart.device_results(ts.n_sets, ts.n_tasks, K)

    def plain_step():
        capart.capart_solve_async(eng.ctx, dev, K, mode, out, max_tasks=max_tasks, max_M=max_M, admissible=adm,
                                  policy=pol)

    plan = None
    if args.form == "batched" and mode != "EXH":
        t0 = time.perf_counter()
        if args.schedule == "persistent":
            capart.capart_set_tuning(eng.ctx, loop_form=1)
            plan = capart.Plan(eng.ctx, dev, K, mode, out, max_tasks, max_M, autotune=False, blocks_per_cu=8,
                               item_evals=4096, use_graph=not args.no_graph, admissible=adm, policy=pol)
            capart.capart_set_tuning(eng.ctx)
        else:
            plan = capart.Plan(eng.ctx, dev, K, mode, out, max_tasks, max_M, autotune=args.schedule == "auto",
                               blocks_per_cu=-1 if args.schedule == "direct" else 0, use_graph=not args.no_graph,
                               admissible=adm, policy=pol)
        plan_info = plan.info()
        log(f"[bench] plan: {plan_info} ({(time.perf_counter() - t0):.1f} s)")
        step = plan.run
        sched = "persistent work queue" if plan_info["blocks"] > 0 else "direct schedule"
        tuned = ", autotuned" if args.schedule == "auto" else ", fixed"
        form = f"batched ({sched}{tuned}" + (")" if args.no_graph else ", HIP graph)")
    else:
        plan_info = None
        step = plain_step
        form = "plain (one launch sequence over the batch)"

    for i in range(args.warmup):
        step()
        sync()
        log(f"[bench] warmup {i + 1}/{args.warmup} done")
    st = out["status"][: ts.n_sets].cpu().numpy()
    if not (st == 0).all():
        raise SystemExit(f"bench: {int((st != 0).sum())} sets reported errors")
    ms_per_step = timed(step, args.steps, sync)
    value = evals_per_step / (ms_per_step / 1000.0)
    verdicts = int(out["verdict"][: ts.n_sets].sum().item())
    log(f"[bench] {args.steps} steps: {ms_per_step:.2f} ms/step, {value:.4g} evals/s ({form})")
    # kernel durations: the same steps with HIP events around each kernel on
    # the launch stream (a plan then launches its kernels directly)
    capart.capart_timing_enable(eng.ctx, True)
    capart.capart_timing_read(eng.ctx)
    ms_timed = timed(step, args.steps, sync)
    ms_k, n_k = capart.capart_timing_read(eng.ctx)
    capart.capart_timing_enable(eng.ctx, False)
    eval_ms = ms_k["eval"] / max(1, n_k["eval"])
    log(f"[bench] kernels per step: {ms_k} over {n_k['eval']} steps")

    # the algorithm's own work, counted exactly by the counting variants of
    # the evaluation kernels (outside the timed region)
    wout = capart.device_results(ts.n_sets, ts.n_tasks, K)
    work = capart.capart_count_work(eng.ctx, dev, K, mode, wout, max_tasks, max_M, admissible=adm, policy=pol)
    del wout
    log(f"[bench] counted work per step: {work}")

    # end to end: host (pinned) inputs copied in, one step, results copied out;
    # reported beside `value`, which keeps the inputs resident
    pinned_in = {k: v.cpu().pin_memory() for k, v in dev.items()}
    pinned_out = {k: torch.empty(v.shape, dtype=v.dtype).pin_memory() for k, v in out.items()}

    def e2e_step():
        for k, v in pinned_in.items():
            dev[k].copy_(v, non_blocking=True)
        step()
        for k, v in out.items():
            pinned_out[k].copy_(v, non_blocking=True)

    e2e_step()
    sync()
    e2e_ms = timed(e2e_step, max(2, args.steps // 2), sync)
    in_bytes = sum(v.numel() * v.element_size() for v in pinned_in.values())
    out_bytes = sum(v.numel() * v.element_size() for v in pinned_out.values())
    end_to_end = {"ms_per_step": e2e_ms, "value": evals_per_step / (e2e_ms / 1000.0), "h2d_bytes": in_bytes,
                  "d2h_bytes": out_bytes}
    log(f"[bench] end to end with copies: {e2e_ms:.2f} ms/step")
    del pinned_in, pinned_out

    compare = {}
    if not args.no_compare and args.form == "batched" and plan is not None:
        plain_ms = timed(plain_step, max(2, args.steps // 2), sync)
        compare["plain_path"] = {"ms_per_step": plain_ms, "value": evals_per_step / (plain_ms / 1000.0),
                                 "batched_over_plain": plain_ms / ms_per_step}
        log(f"[bench] plain path: {plain_ms:.2f} ms/step")
        sub_n = min(2000, ts.n_sets)
        sub = workload.subset(ts, np.arange(sub_n))
        sdev = capart.device_tasksets(sub)
        sout = capart.device_results(sub.n_sets, sub.n_tasks, K)

        def per_set():
            capart.capart_solve_async(eng.ctx, sdev, K, mode, sout, max_tasks=max_tasks, max_M=max_M,
                                      flags=capart.CAPART_FLAG_PER_SET_LAUNCH, admissible=adm, policy=pol)

        per_set()
        ps_ms = timed(per_set, 1, sync)
        ps_evals = int(sum(Pcount[int(m)] for m in sub["M"]))
        compare["per_set_launch"] = {"sets": sub_n, "ms": ps_ms, "value": ps_evals / (ps_ms / 1000.0)}
        compare["per_set_launch"]["batched_over_per_set"] = value / compare["per_set_launch"]["value"]
        log(f"[bench] one launch per set: {compare['per_set_launch']['value']:.4g} evals/s")
        del sdev, sout
        if args.workload == "c3" and not adm and not args.tables:
            # the 100,000-set n = 10, M = 80 workload through its own batched plan
            c2 = workload.config_c2(n_sets=100_000)
            c2dev = capart.device_tasksets(c2)
            c2out = capart.device_results(c2.n_sets, c2.n_tasks, K)
            c2plan = capart.Plan(eng.ctx, c2dev, K, mode, c2out, 10, 80, autotune=True, use_graph=True, policy=pol)
            c2plan.run()
            sync()
            c2_ms = timed(c2plan.run, max(3, args.steps // 2), sync)
            c2_evals = c2.n_sets * capart.capart_count_partitionings(80, K)
            compare["c2_batched"] = {"workload": "100000 task sets, n=10, M=80, K=4", "ms_per_step": c2_ms,
                                     "value": c2_evals / (c2_ms / 1000.0), "plan": c2plan.info()}
            log(f"[bench] c2 batched: {c2_ms:.2f} ms/step, {compare['c2_batched']['value']:.4g} evals/s")
            c2plan.close()
            del c2dev, c2out

    serving = None
    if args.workload in ("c2", "c3") and not args.no_serving and not args.tables and pol == "FP_DM" and not adm:
        # the serving workload's lowest configured rate (10,000 queries/s) and two
        # above it, one second of arrivals each; the headline p99 is the first
        legs = []
        for rate in (1e4, 3e4, 1e5):
            leg = serving_leg(eng, capart, workload, rate, int(min(50000, rate)))
            legs.append(leg)
            log(f"[bench] serving at {rate:g} q/s: {leg['qps']:.4g} q/s served, p50 {leg['p50_us']:.1f} us, "
                f"p99 {leg['p99_us']:.1f} us, rejected {leg['rejected']}")
        serving = dict(legs[0])
        serving["sweep"] = legs
        serving["saturation_qps"] = max(x["qps"] for x in legs)

    cpu = None
    cflags = 0
    if mode == "EXH":
        # the oracle's memoised exhaustive search (every allocation of every
        # partitioning scored from a table of subset tests; the plain search
        # decodes every triple and would take hours per set)
        import oracle
        cflags = oracle.FLAG_EXH_FAST
        cpu_sample = args.cpu_sample or 10  # 10 sets x all 1,033 partitionings (about 45 s per set and thread)
        threads = min(threads, cpu_sample)
    if args.no_cpu:
        cb = None if mode == "EXH" else cpu_baseline(ts, K, mode, 200, threads, cpu_stride, adm, pol)
    else:
        log(f"[bench] CPU oracle on {cpu_sample} sets with {threads} threads")
        cb = cpu_baseline(ts, K, mode, cpu_sample, threads, cpu_stride, adm, pol, cflags)
        one = cpu_baseline(ts, K, mode, max(1, cpu_sample // threads), 1, cpu_stride, adm, pol, cflags) \
            if threads > 1 else cb
        cpu = {"value": cb["evals"] / cb["seconds"], "unit": "evals/s", "cores": threads, "kind": "oracle",
               "sample": f"{cb['sets']} of the {ts.n_sets} sets (every {cpu_stride}th from the first), "
                         f"{cb['evals']} evals, {cb['seconds']:.2f} s wall"
                         + (", memoised exhaustive search" if mode == "EXH" else ""),
               "single_core": {"value": one["evals"] / one["seconds"], "sample": f"the first {one['sets']} of "
                               f"those sets, {one['seconds']:.2f} s"},
               "cpu_model": cpu_model(), "host_cpus": os.cpu_count()}
        log(f"[bench] CPU oracle: {cpu['value']:.4g} evals/s ({cpu['single_core']['value']:.4g} on one core)")
    roof = None
    if work is not None:
        # the plan runs a persistent grid, or the direct schedule (blocks == 0);
        # the exhaustive search fills subset tables and searches them
        if mode == "EXH":
            kname = "subset_table_kernel + exh_dfs_kernel"
        else:
            kname = "eval_persistent_kernel" if plan is not None and plan_info["blocks"] > 0 else "eval_heur_kernel"
        ops = work["terms"] * C_TERM + work["tests"] * C_TEST + work["lookups"] * C_LOOK
        achieved = ops / (eval_ms / 1000.0)
        roof = {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_INT_LANE_OPS / 1e12, "unit": "TOP/s",
                "frac": achieved / PEAK_INT_LANE_OPS,
                "traffic": traffic_bytes(f"{kname}_{args.workload}_{mode.lower()}"
                                         f"{'_edf' if pol == 'EDF' else ''}_traffic.json"),
                "kernel": kname, "kernel_ms": eval_ms, "ops_per_launch": ops, "work_per_launch": work,
                "ops_per_term": C_TERM, "ops_per_test": C_TEST, "ops_per_lookup": C_LOOK,
                "other_kernels_ms": {"prep": ms_k["prep"] / max(1, n_k["prep"]),
                                     "final": ms_k["final"] / max(1, n_k["final"])},
                "step_ms_with_kernel_events": ms_timed,
                "peak_measured": valu_ops / 1e12, "frac_of_measured_peak": achieved / valu_ops}
        if pol == "EDF":
            roof["note"] = ("EDF terms (members x utilisation and density sums, busy-period steps, demand points) "
                            "are priced at the fixed-priority term cost")
        if mode == "EXH":
            roof["note"] = ("exhaustive search: terms and tests fill the subset tables, lookups are the table reads "
                            "of the pruned depth-first search (6 operations each, as a frontier lookup)")
        if cb is not None and mode != "EXH":
            # the same roofline priced on the oracle's plain-order work per
            # evaluation (no frontier, no memo, no skipped tests), measured on
            # the oracle's sample: the work the method defines, not the work
            # this kernel executes
            tpe, spe = cb["terms"] / cb["evals"], cb["tests"] / cb["evals"]
            plain = (tpe * C_TERM + spe * C_TEST) * evals_per_step / (eval_ms / 1000.0)
            roof["oracle_plain_order_terms_per_eval"] = tpe
            roof["oracle_plain_order_tests_per_eval"] = spe
            roof["plain_order"] = {"achieved": plain / 1e12, "frac": plain / PEAK_INT_LANE_OPS,
                                   "frac_of_measured_peak": plain / valu_ops,
                                   "sample_sets": cb["sets"], "sample_evals": cb["evals"]}
    res = {"metric": METRIC, "value": value, "unit": "evals/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": ms_per_step, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "int64", "data": "synthetic",
           "config": {"workload": f"{args.workload}: {ts.n_sets} task sets, {desc}, K={K}, {mode}, {form}",
                      "n_sets": ts.n_sets, "K": K, "alloc_mode": mode, "policy": pol, "evals_per_step": evals_per_step,
                      "schedulable_sets": verdicts, "lemma1_pruned_sets": lemma1_pruned(ts), "plan": plan_info},
           "end_to_end_with_copies": end_to_end, "compare": compare, "serving": serving, "roofline": roof, "cpu_baseline": cpu}
    if plan is not None:
        plan.close()
    eng.close()
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
