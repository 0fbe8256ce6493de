#!/usr/bin/env python3
"""Benchmark: tree-LQR factor + solve throughput on one MI355X.

A step is one whole pass of the hot path, rcr_solve (Algorithm 1, Steps 2-6:
condensation, quadratic contraction and expansion, local factors, affine
contraction and expansion, local affine solve, state contraction and
expansion, recovery), on one synthetic instance whose inputs are already
resident in HBM.  The workload is the single-tree FP64 configuration:
N = 65,536 nodes from the chain-probability generator (p = 0.95), n = 12,
m = 4, rank-6 PSD dual regularisation with eigenvalues U(0, 1e-2).

Output: one JSON line with nodes/s (whole job), p50/p99 per-step latency, the
KKT residual reached, the roofline of the dominant kernel class (HIP events
around each of its launches on the launch stream, algorithmic bytes per
launch from the plan's operation counts), and the FP64 CPU oracle timed on a
bounded sample on the host.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0


def algorithmic_words(st: dict, n: int, m: int) -> dict:
    """Algorithmic FP words moved per solve, per kernel class: every primitive
    reads each operand block once and writes each result block once (s = n^2,
    t = n m, v = m^2)."""
    s, t, v = n * n, n * m, m * m
    N = st["N"]
    E = N - 1
    R, B, A, C = st["n_rake"], st["n_combine"], st["n_absorb"], st["n_compress"]
    return {
        "condense": N * 2 * s + E * (5 * s + 2 * t + v),
        "quad_contract": R * 6 * s + B * 3 * s + A * 3 * s + C * 10 * s,
        "quad_expand": C * 6 * s,
        "local_factor": N * 4 * s + E * (3 * s + 3 * t + 2 * v),
        "tcompose": C * 3 * s,
        "rhs_init": N * 2 * n + E * (2 * s + t + 2 * n + m),
        "aff_contract": R * (s + 4 * n) + (B + A) * 3 * n + C * (s + 4 * n),
        "aff_expand": C * (s + 4 * n),
        "local_affine": N * (3 * s + t + v + 3 * n + 2 * m),
        "state_contract": C * (s + 3 * n),
        "state_expand": E * (s + 3 * n),
        "recover": N * (s + 4 * n) + E * (t + n + 2 * m),
    }


def kernel_source_sha() -> str:
    """Digest of every HIP/C++ source of the solver library (a traffic figure is
    only reported for the kernels it was measured on)."""
    import hashlib
    d = os.path.join(ROOT, "paper_2608_01332_amd", "csrc")
    h = hashlib.sha256()
    for f in sorted(os.listdir(d)):
        if f.endswith((".hip", ".hpp", ".cpp", ".h")):
            h.update(f.encode())
            h.update(open(os.path.join(d, f), "rb").read())
    return h.hexdigest()[:16]


def bench_copy(args) -> dict:
    """Plain device-to-device copy of a known size: the calibration kernel for
    the FETCH_SIZE / WRITE_SIZE counters, and the achievable HBM copy rate."""
    import torch
    nbytes = args.copy_mib << 20
    a = torch.empty(nbytes // 8, dtype=torch.float64, device="cuda:0").normal_()
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    reps = 10
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    return {"workload": "copy", "bytes_read_per_launch": nbytes, "bytes_written_per_launch": nbytes,
            "launches": reps + 3, "ms_per_copy": ms, "copy_GBps": 2 * nbytes / (ms / 1e3) / 1e9}


def read_traffic(kernel_class: str):
    """HBM traffic per launch from the committed rocprofv3 PMC summary, if it was
    taken on the current kernel source (else None)."""
    path = os.path.join(ROOT, "profiles", f"traffic_{kernel_class}.txt")
    if not os.path.exists(path):
        return None
    kv = {}
    for line in open(path):
        if "=" in line and not line.lstrip().startswith("#"):
            k, v = line.split("=", 1)
            kv[k.strip()] = v.strip()
    if kv.get("source_sha") != kernel_source_sha():
        return None
    try:
        return float(kv["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def cpu_baseline(parent, data, seconds: float) -> dict:
    from oracle import riccati as orc
    N = len(parent)
    runs, t0 = 0, time.perf_counter()
    while True:
        orc.tree_riccati(parent, data)
        runs += 1
        el = time.perf_counter() - t0
        if el >= seconds:
            break
    return {"value": N * runs / el, "unit": "nodes/s", "cores": 1, "kind": "oracle",
            "sample": f"{runs} sequential FP64 solves of the N={N}, n=12, m=4 instance on 1 thread "
                      f"({el:.1f} s)"}


def bench_batch(args) -> dict:
    """512 independent trees (N log-uniform in [256, 16384], p ~ U(0.8, 0.98), n = 8,
    m = 3), MIXED32 with one refinement step: one merged launch sequence for the whole
    batch against one solve per tree, both checked at KKT residual <= 1e-8."""
    import numpy as np
    import torch
    from paper_2608_01332_amd import rcr
    from paper_2608_01332_amd import workloads as w
    dev = torch.device("cuda:0")
    T = args.trees
    pars, datas = [], []
    for t in range(T):
        p_, d_, spec = w.config_instance(3, tree=t)
        pars.append(p_)
        datas.append(d_)
    n, m = spec.n, spec.m
    plans = [rcr.Plan(p_, n, m) for p_ in pars]
    t0 = time.perf_counter()
    B = rcr.Plan.batch(plans)
    merge_ms = (time.perf_counter() - t0) * 1e3
    Ntot = B.N
    big = rcr.to_device(rcr.concat_problems(datas), dev)
    out = rcr.alloc_solution(B, dev)
    stream = torch.cuda.current_stream(dev)
    kw = dict(precision=rcr.MIXED32, refine_steps=1, executor=rcr.EXEC_GRAPH)
    chk = rcr.solve(B, big, out=out, check=True, kkt_residual=True, **kw)
    for _ in range(args.warmup):
        rcr.solve(B, big, out=out, **kw)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(args.steps):
        rcr.solve(B, big, out=out, stream=stream, **kw)
    e1.record(stream)
    torch.cuda.synchronize()
    batched_ms = e0.elapsed_time(e1) / args.steps
    # one solve per tree, on views of the same device arrays
    offs = B.offsets
    views = []
    worst = 0.0
    for t, p_ in enumerate(plans):
        lo, hi = int(offs[t]), int(offs[t + 1])
        pv = {k: big[k][lo:hi] for k in rcr.PROBLEM_FIELDS}
        ov = {k: out[k][lo:hi] for k in rcr.SOLUTION_FIELDS}
        views.append((p_, pv, ov))
        r = rcr.solve(p_, pv, out=ov, check=True, kkt_residual=True, **kw)
        worst = max(worst, r["kkt_residual"])
    for p_, pv, ov in views:
        rcr.solve(p_, pv, out=ov, **kw)
    torch.cuda.synchronize()
    reps = max(1, args.steps // 4)
    e0.record(stream)
    for _ in range(reps):
        for p_, pv, ov in views:
            rcr.solve(p_, pv, out=ov, stream=stream, **kw)
    e1.record(stream)
    torch.cuda.synchronize()
    separate_ms = e0.elapsed_time(e1) / reps
    st = B.stats()
    rec = {
        "metric": "tree-LQR nodes/sec vs CPU Riccati at KKT res 1e-8; p50/p99 solve latency",
        "value": Ntot / (batched_ms / 1e3), "unit": "nodes/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": batched_ms, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32+f64-refine", "data": "synthetic",
        "config": {"workload": f"{T} trees, N log-uniform [256,16384], p~U(0.8,0.98), n=8, m=3, MIXED32 + 1 "
                               "refinement, one merged launch sequence", "trees": T, "nodes": int(Ntot),
                   "levels": st["levels"], "height_max": st["height"]},
        "kkt_residual_batched": chk["kkt_residual"], "kkt_residual_separate_max": worst,
        "separate_ms_per_step": separate_ms, "separate_nodes_per_s": Ntot / (separate_ms / 1e3),
        "batched_speedup": separate_ms / batched_ms, "merge_plan_ms": merge_ms,
    }
    if args.cpu_seconds > 0:
        from oracle import riccati as orc
        nth = min(16, os.cpu_count() or 1)
        tt0 = time.perf_counter()
        done, nodes = 0, 0
        while time.perf_counter() - tt0 < args.cpu_seconds and done < T:
            chunk = list(zip(pars[done:done + 32], datas[done:done + 32]))
            orc.tree_riccati_batch(chunk, nth)
            nodes += sum(len(p_) for p_, _ in chunk)
            done += len(chunk)
        el = time.perf_counter() - tt0
        rec["cpu_baseline"] = {"value": nodes / el, "unit": "nodes/s", "cores": nth, "kind": "oracle",
                               "sample": f"first {done} of the {T} trees ({nodes} nodes), FP64, {nth} threads, {el:.1f} s"}
    return rec


def bench_extreme(args) -> dict:
    """Shape-extreme trees at N = 1,048,576 (n = 6, m = 2, FP64): one plan per tree
    reused across 8 re-solves with fresh cost/dynamics data (copied to the device
    outside the timed region)."""
    import numpy as np
    import torch
    from paper_2608_01332_amd import rcr
    from paper_2608_01332_amd import workloads as w
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream(dev)
    res = {}
    for ti, kind in enumerate(["caterpillar", "star_heavy", "chainprob"]):
        par = w.shape_extreme(kind)
        t0 = time.perf_counter()
        plan = rcr.Plan(par, 6, 2)
        plan_ms = (time.perf_counter() - t0) * 1e3
        prob, out, times, kkt = None, None, [], 0.0
        for s_ in range(args.resolves):
            d = w.lqr_data(par, w.DataSpec(6, 2), np.random.default_rng(w.config_seed(4, s_, ti)))
            if prob is None:
                prob = rcr.to_device(d, dev)
                out = rcr.alloc_solution(plan, dev)
                rcr.solve(plan, prob, out=out, executor=rcr.EXEC_GRAPH)  # graph capture (untimed)
            else:
                for k in rcr.PROBLEM_FIELDS:
                    prob[k].copy_(torch.from_numpy(d[k]))
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            rcr.solve(plan, prob, out=out, executor=rcr.EXEC_GRAPH, stream=stream)
            e1.record(stream)
            torch.cuda.synchronize()
            times.append(e0.elapsed_time(e1))
            r = rcr.solve(plan, prob, out=out, executor=rcr.EXEC_GRAPH, kkt_residual=True)
            kkt = max(kkt, r["kkt_residual"])
        st = plan.stats()
        res[kind] = {"nodes_per_s": len(par) / (float(np.median(times)) / 1e3), "median_ms": float(np.median(times)),
                     "max_ms": float(np.max(times)), "resolves": args.resolves, "kkt_residual_max": kkt,
                     "plan_ms": plan_ms, "height": st["height"], "levels": st["levels"], "rounds": st["rounds"]}
        del prob, out
        torch.cuda.empty_cache()
    tot_ms = sum(v["median_ms"] for v in res.values())
    return {"metric": "tree-LQR nodes/sec vs CPU Riccati at KKT res 1e-8; p50/p99 solve latency",
            "value": 3 * 1048576 / (tot_ms / 1e3), "unit": "nodes/s", "n_gpus": 1, "steps": args.resolves,
            "warmup": 1, "ms_per_step": tot_ms / 3, "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None, "dtype": "f64", "data": "synthetic",
            "config": {"workload": "shape-extreme trees N=1,048,576 (caterpillar, star-heavy, chain-prob 0.9), "
                                   "n=6, m=2, FP64, plan reused across re-solves"},
            "trees": res}


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--executor", choices=["graph", "levels"], default="graph")
    ap.add_argument("--cpu-seconds", type=float, default=12.0, help="CPU oracle sample length; 0 skips it")
    ap.add_argument("--class-steps", type=int, default=5, help="steps of the per-launch event pass")
    ap.add_argument("--no-mixed", action="store_true", help="skip the MIXED32 + refinement leg")
    ap.add_argument("--copy-mib", type=int, default=1024)
    ap.add_argument("--workload", choices=["single", "batch", "extreme", "copy"], default="single",
                    help="single: the 65,536-node tree (default); batch: the 512-tree batched workload; "
                         "extreme: the 1M-node shape-extreme trees; copy: plain HBM copy (counter calibration)")
    ap.add_argument("--resolves", type=int, default=8)
    ap.add_argument("--trees", type=int, default=512)
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this build measures one GPU only; --gpus {args.gpus} is not supported "
              "(the solver shards by tree across GPUs with no communication, see DESIGN.md)", file=sys.stderr)
        return 2

    import numpy as np
    import torch
    from paper_2608_01332_amd import rcr
    from paper_2608_01332_amd import workloads as w

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        return 1
    if args.workload == "batch":
        print(json.dumps(bench_batch(args)), flush=True)
        return 0
    if args.workload == "extreme":
        print(json.dumps(bench_extreme(args)), flush=True)
        return 0
    if args.workload == "copy":
        print(json.dumps(bench_copy(args)), flush=True)
        return 0
    dev = torch.device("cuda:0")
    parent, data, spec = w.config_instance(2)
    N, n, m = len(parent), spec.n, spec.m
    t0 = time.perf_counter()
    plan = rcr.Plan(parent, n, m)
    plan_s = time.perf_counter() - t0
    st = plan.stats()
    prob = rcr.to_device(data, dev)
    out = rcr.alloc_solution(plan, dev)
    ex = rcr.EXEC_GRAPH if args.executor == "graph" else rcr.EXEC_LEVELS
    stream = torch.cuda.current_stream(dev)

    # accuracy at the measured configuration (outside the timed region)
    chk = rcr.solve(plan, prob, out=out, executor=ex, check=True, kkt_residual=True)
    kkt = chk["kkt_residual"]

    for _ in range(args.warmup):
        rcr.solve(plan, prob, out=out, executor=ex)
    torch.cuda.synchronize()
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
    torch.cuda.synchronize()
    t_wall = time.perf_counter()
    evs[0].record(stream)
    for k in range(args.steps):
        rcr.solve(plan, prob, out=out, executor=ex, stream=stream)
        evs[k + 1].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_wall
    step_ms = [evs[k].elapsed_time(evs[k + 1]) for k in range(args.steps)]
    total_ms = evs[0].elapsed_time(evs[-1])
    ms_per_step = total_ms / args.steps
    value = N * args.steps / (total_ms / 1e3)
    p50 = float(np.percentile(step_ms, 50))
    p99 = float(np.percentile(step_ms, 99))

    # per-launch HIP-event pass: device time and launch count per kernel class
    cls_ms, cls_n = {}, {}
    for _ in range(max(1, args.class_steps)):
        r = rcr.solve(plan, prob, out=out, executor=rcr.EXEC_LEVELS, kernel_ms=True, stream=stream)
        for k, v in r["kernel_ms"].items():
            cls_ms[k] = cls_ms.get(k, 0.0) + v
            cls_n[k] = cls_n.get(k, 0) + r["kernel_launches"][k]
    reps = max(1, args.class_steps)
    words = algorithmic_words(st, n, m)
    # The per-level quadratic contraction launches cover levels 1..k (k = their launch
    # count); the narrow levels after them run in the tail kernel.  Its algorithmic
    # bytes are those of the ops in its own levels.
    ops = plan.export_ops()
    k_q = cls_n.get("quad_contract", 0) // reps
    sel = ops[ops[:, 2] <= k_q]
    s_, per_kind = n * n, {0: 6, 1: 3, 2: 3, 3: 10}
    words_q = sum(int((sel[:, 0] == kind).sum()) * mult * s_ for kind, mult in per_kind.items())
    measured = dict(words)
    measured["quad_contract"] = words_q
    dom = max(measured, key=lambda k: cls_ms.get(k, 0.0))
    dom_ms = cls_ms[dom] / reps
    dom_launches = cls_n[dom] / reps
    bytes_per_solve = measured[dom] * 8
    achieved = bytes_per_solve / (dom_ms / 1e3) / 1e9
    traffic = read_traffic(dom)
    total_words = sum(words.values())
    class_sum_ms = sum(cls_ms.values()) / reps

    rec = {
        "metric": "tree-LQR nodes/sec vs CPU Riccati at KKT res 1e-8; p50/p99 solve latency",
        "value": value,
        "unit": "nodes/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "p50_ms": p50,
        "p99_ms": p99,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "single tree-LQR factor+solve, N=65536 chain-prob p=0.95 tree, n=12, m=4, "
                               "rank-6 PSD dual regularisation, FP64",
                   "N": N, "n": n, "m": m, "height": st["height"], "levels": st["levels"],
                   "rounds": st["rounds"], "executor": args.executor, "precision": "fp64"},
        "kkt_residual": kkt,
        "roofline": {"bound": "hbm", "kernel_class": dom, "achieved": achieved, "peak": PEAK_HBM_GBS,
                     "unit": "GB/s", "frac": achieved / PEAK_HBM_GBS,
                     "traffic": traffic,
                     "bytes_per_launch": bytes_per_solve / dom_launches,
                     "avg_launch_us": dom_ms * 1e3 / dom_launches,
                     "launches_per_step": dom_launches},
        "solve_alg_bytes": total_words * 8,
        "solve_alg_frac": total_words * 8 / (ms_per_step / 1e3) / 1e9 / PEAK_HBM_GBS,
        "kernel_ms_per_step": {k: round(v / reps, 4) for k, v in cls_ms.items()},
        "kernel_sum_ms_per_step": class_sum_ms,
        "plan_ms": plan_s * 1e3,
        "wall_ms_per_step": wall * 1e3 / args.steps,
    }
    if not args.no_mixed:
        # the same workload in MIXED32: float32 factor/solves (float64 R/G Cholesky and
        # compress solves), one refinement step on the float64 KKT residual
        mout = rcr.alloc_solution(plan, dev)
        chk = rcr.solve(plan, prob, out=mout, precision=rcr.MIXED32, refine_steps=1, executor=ex, check=True,
                        kkt_residual=True)
        for _ in range(args.warmup):
            rcr.solve(plan, prob, out=mout, precision=rcr.MIXED32, refine_steps=1, executor=ex)
        mev = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
        torch.cuda.synchronize()
        mev[0].record(stream)
        for k in range(args.steps):
            rcr.solve(plan, prob, out=mout, precision=rcr.MIXED32, refine_steps=1, executor=ex, stream=stream)
            mev[k + 1].record(stream)
        torch.cuda.synchronize()
        mms = [mev[k].elapsed_time(mev[k + 1]) for k in range(args.steps)]
        mtot = mev[0].elapsed_time(mev[-1])
        rel = {}
        for k in rcr.SOLUTION_FIELDS:
            a, b = mout[k], out[k]
            rel[k] = float((a - b).abs().max() / b.abs().max().clamp_min(1e-300))
        rec["mixed32"] = {"value": N * args.steps / (mtot / 1e3), "unit": "nodes/s",
                          "ms_per_step": mtot / args.steps, "p50_ms": float(np.percentile(mms, 50)),
                          "p99_ms": float(np.percentile(mms, 99)), "refine_steps": 1,
                          "kkt_residual": chk["kkt_residual"], "rel_err_vs_fp64": rel}
    if args.cpu_seconds > 0:
        cb = cpu_baseline(parent, data, args.cpu_seconds)
        rec["cpu_baseline"] = cb
        rec["speedup_vs_cpu_oracle"] = value / cb["value"]
    else:
        rec["cpu_baseline"] = None
    print(json.dumps(rec), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
