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
PEAK_FP64_TFLOPS = 78.6
METRIC = "tree-LQR nodes/sec vs CPU Riccati at KKT res 1e-8; p50/p99 solve latency"


def alg_words(st: dict, n: int, m: int) -> dict:
    """Algorithmic FP words of one factor + solve by primitive, the fixed model
    of the measurement plan: every primitive reads each operand block once and
    writes each result block once, symmetric blocks full (s = n^2, t = n m,
    v = m^2; N nodes, E = N - 1 edges; the plan's op counts)."""
    s, t, v = n * n, n * m, m * m
    N = st["N"]
    E = N - 1
    R, Cb, A, C = st["n_rake"], st["n_combine"], st["n_absorb"], st["n_compress"]
    return {
        # factor
        "condense": E * (5 * s + 2 * t + v),
        "rake": R * 5 * s, "combine": Cb * 3 * s, "absorb": A * 3 * s, "compress": C * 10 * s,
        "expand_rake": R * 2 * s, "expand_compress": C * 6 * s,
        "node_factor": N * 4 * s, "edge_factor": E * (4 * s + 3 * t + 2 * v),
        # solve
        "z": E * (2 * s + 2 * t + 2 * n + m),
        "aff_rake": R * (s + 3 * n), "aff_combine_absorb": (Cb + A) * 3 * n, "aff_compress": C * (3 * s + 4 * n),
        "aff_expand": R * 2 * n + C * (s + 4 * n),
        "local": N * (2 * s + 4 * n) + E * (s + t + v + 3 * n + 2 * m),
        "state_compress": C * (s + 3 * n), "state_expand": E * (s + 3 * n),
        "u": E * (t + n + 2 * m), "y": N * (s + 3 * n),
    }


def io_words(N: int, n: int, m: int) -> int:
    """Inputs read once and outputs written once: (4s + v + 3t + 4n + 2m) words per node."""
    s, t, v = n * n, n * m, m * m
    return N * (4 * s + v + 3 * t + 4 * n + 2 * m)


# words per primitive of the quadratic contraction, by op kind (rake, combine, absorb, compress)
CONTRACT_WORDS = {0: 5, 1: 3, 2: 3, 3: 10}


def host_cpu() -> dict:
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = os.cpu_count() or 1
    return {"cpu_model": model, "nproc": os.cpu_count() or 1, "cpus_available": avail}


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


def _csvs(d: str, suffix: str):
    import glob
    return sorted(glob.glob(os.path.join(d, "**", f"*{suffix}"), recursive=True))


def summarize_stats(d: str) -> str:
    """Kernel statistics table from a rocprofv3 --kernel-trace --stats run
    (its *kernel_stats.csv under directory d)."""
    import csv
    rows = []
    for f in _csvs(d, "kernel_stats.csv"):
        rows += list(csv.DictReader(open(f)))
    rows.sort(key=lambda r: -float(r["TotalDurationNs"]))
    import io
    buf = io.StringIO()
    wr = csv.writer(buf, lineterminator="\n")
    wr.writerow(["name", "calls", "total_us", "avg_us", "min_us", "max_us", "percent"])
    for r in rows:
        wr.writerow([r["Name"], r["Calls"], f'{float(r["TotalDurationNs"]) / 1e3:.1f}',
                     f'{float(r["AverageNs"]) / 1e3:.2f}', f'{float(r["MinNs"]) / 1e3:.2f}',
                     f'{float(r["MaxNs"]) / 1e3:.2f}', f'{float(r["Percentage"]):.2f}'])
    return buf.getvalue().rstrip("\n")


def summarize_timeline(d: str, which: int) -> str:
    """Per-launch timeline of one solve from a rocprofv3 --kernel-trace run (its
    *kernel_trace.csv under directory d): solves are split at the first-level
    kernel; for solve `which`, each launch's start (from the solve's first
    launch), duration and idle gap before it, in microseconds."""
    import csv
    import re
    rows = []
    for f in _csvs(d, "kernel_trace.csv"):
        rows += list(csv.DictReader(open(f)))
    rows.sort(key=lambda r: int(r["Start_Timestamp"]))
    starts = [i for i, r in enumerate(rows) if "k_level1_wide" in r["Kernel_Name"] or "k_condense_wide" in r["Kernel_Name"]]
    i0, i1 = starts[which], starts[which + 1] if which + 1 < len(starts) else len(rows)
    seq = rows[i0:i1]
    t0 = int(seq[0]["Start_Timestamp"])
    out = ["start_us,dur_us,gap_us,kernel"]
    prev = None
    busy = gaps = 0
    for r in seq:
        s_, e_ = int(r["Start_Timestamp"]), int(r["End_Timestamp"])
        gap = 0 if prev is None else max(0, s_ - prev)
        name = re.sub(r"\(.*", "", r["Kernel_Name"]).replace("void ", "")
        out.append(f"{(s_ - t0) / 1e3:.2f},{(e_ - s_) / 1e3:.2f},{gap / 1e3:.2f},\"{name}\"")
        busy += e_ - s_
        gaps += gap
        prev = e_
    out.append(f"# {len(seq)} launches: kernels {busy / 1e3:.1f} us, gaps {gaps / 1e3:.1f} us, "
               f"span {(prev - t0) / 1e3:.1f} us (the last row starts the next solve's graph)")
    return "\n".join(out)


def pmc_totals(d: str) -> dict:
    """Per kernel name: dispatches and the sum of each counter over them, from
    a rocprofv3 --pmc run (its *counter_collection.csv under directory d)."""
    import csv
    tot = {}
    for f in _csvs(d, "counter_collection.csv"):
        for r in csv.DictReader(open(f)):
            e = tot.setdefault(r["Kernel_Name"], {"dispatches": set()})
            e["dispatches"].add(r["Dispatch_Id"])
            c = r["Counter_Name"]
            e[c] = e.get(c, 0.0) + float(r["Counter_Value"])
    return {k: dict(v, dispatches=len(v["dispatches"])) for k, v in tot.items()}


# the dominant class: the first contraction level (fused with the condensation
# when the plan allows) and the later per-level quadratic contraction launches
DOMINANT_KERNELS = ("k_level1_wide<double, 12>", "k_quad_level_wide<double, 12>", "k_condense_wide<double, 12>")


def _dominant(tot: dict):
    sel = {k: v for k, v in tot.items() if any(x in k for x in DOMINANT_KERNELS)}
    solves = max((v["dispatches"] for k, v in sel.items() if "k_level1_wide" in k or "k_condense_wide" in k),
                 default=0)
    launches = sum(v["dispatches"] for k, v in sel.items() if "k_condense_wide" not in k)
    return sel, solves, launches


def summarize_pmc(kind: str, runs: dict, copy_dirs: dict) -> str:
    """Per-launch figures of the dominant kernel class from rocprofv3 --pmc runs:
    kind "traffic": HBM bytes from FETCH_SIZE and WRITE_SIZE (KiB per dispatch),
    each scaled by what the counter reads for a plain copy of known size;
    kind "flops": FP64 flops from the SQ instruction counters (64 lanes per VALU
    instruction, an FMA counting 2; MFMA as 512 per MOPS unit).  runs maps a
    quadratic tail setting q to {counter group: directory}."""
    lines = []
    if kind == "traffic":
        cal = {}
        for c, dirpath in copy_dirs.items():
            t = pmc_totals(dirpath)
            k = max(t, key=lambda x: t[x].get(c, 0.0) / max(t[x]["dispatches"], 1))
            per = t[k][c] / t[k]["dispatches"] * 1024.0  # bytes per copy launch
            known = float(os.environ.get("RCR_COPY_BYTES", 1 << 30))
            cal[c] = known / per
            lines.append(f"# copy: {c} reads {per / 1024:.0f} KiB for {known / 1024:.0f} KiB -> factor {cal[c]:.4f}")
        lines.append(f"fetch_factor={cal['FETCH_SIZE']:.4f}")
        lines.append(f"write_factor={cal['WRITE_SIZE']:.4f}")
    for q, dirs in sorted(runs.items()):
        tot = {}
        for dirpath in dirs.values():
            for k, v in pmc_totals(dirpath).items():
                e = tot.setdefault(k, {"dispatches": v["dispatches"]})
                e.update({c: x for c, x in v.items() if c != "dispatches"})
        sel, solves, launches = _dominant(tot)
        lpsolve = launches / max(solves, 1)
        lines.append(f"# quad_tail_rounds={q}: {solves} solves, {launches} launches of the class; per launch:")
        for k, v in sorted(sel.items()):
            vals = " ".join(f"{c}={x / v['dispatches']:.4g}" for c, x in sorted(v.items()) if c != "dispatches")
            lines.append(f"#   {k}: dispatches={v['dispatches']} {vals}")
        if kind == "traffic":
            fetch = sum(v.get("FETCH_SIZE", 0.0) for v in sel.values()) * 1024 * cal["FETCH_SIZE"] / max(launches, 1)
            write = sum(v.get("WRITE_SIZE", 0.0) for v in sel.values()) * 1024 * cal["WRITE_SIZE"] / max(launches, 1)
            lines += [f"qtr{q}.launches_per_solve={lpsolve:g}", f"qtr{q}.fetch_bytes_per_launch={fetch:.0f}",
                      f"qtr{q}.write_bytes_per_launch={write:.0f}", f"qtr{q}.hbm_bytes_per_launch={fetch + write:.0f}"]
        else:
            def c_(name):
                return sum(v.get(name, 0.0) for v in sel.values())
            valu = 64 * (c_("SQ_INSTS_VALU_ADD_F64") + c_("SQ_INSTS_VALU_MUL_F64") + c_("SQ_INSTS_VALU_TRANS_F64")
                         + 2 * c_("SQ_INSTS_VALU_FMA_F64"))
            mfma = 512 * c_("SQ_INSTS_VALU_MFMA_MOPS_F64")
            lines += [f"qtr{q}.launches_per_solve={lpsolve:g}",
                      f"qtr{q}.valu_fp64_flops_per_launch={valu / max(launches, 1):.0f}",
                      f"qtr{q}.mfma_fp64_flops_per_launch={mfma / max(launches, 1):.0f}",
                      f"qtr{q}.fp64_flops_per_launch={(valu + mfma) / max(launches, 1):.0f}"]
    lines.append(f"source_sha={kernel_source_sha()}")
    return "\n".join(lines)


def mapping_string(cfg) -> str:
    return ",".join(f"{k}={v}" for k, v in cfg.items()) if isinstance(cfg, dict) else "default"


def read_profile_value(name: str, mapping: str, key: str):
    """A per-launch figure (HBM bytes, FP64 flops) of the dominant kernel class
    from a committed rocprofv3 PMC summary, if it was taken on the current
    kernel source, for the quadratic tail setting of this run's launch mapping
    (it decides which levels the per-level launches cover; the summary holds one
    record per setting), else None."""
    path = os.path.join(ROOT, "profiles", f"{name}.txt")
    if not os.path.exists(path):
        return None
    kv = {}
    for line in open(path):
        if "=" in line and not line.lstrip().startswith("#"):
            k, v = line.split("=", 1)
            kv[k.strip()] = v.strip()
    if kv.get("source_sha") != kernel_source_sha():
        return None
    m = dict(x.split("=", 1) for x in mapping.split(",") if "=" in x)
    try:
        q = int(m["quad_tail_rounds"])
        return float(kv[f"qtr{1 if q == 0 else q}.{key}"])  # 0 selects the default, 1 at n = 12
    except (KeyError, ValueError):
        return None


def cpu_baseline(parent, data, seconds: float) -> dict:
    """The oracle (sequential FP64 tree Riccati, one thread) timed on a bounded
    sample: repeated whole solves of the same instance for about `seconds`."""
    from oracle import riccati as orc
    N = len(parent)
    n, m = data["Q"].shape[-1], data["R"].shape[-1]
    runs, t0 = 0, time.perf_counter()
    while True:
        orc.tree_riccati(parent, data)
        runs += 1
        el = time.perf_counter() - t0
        if el >= seconds:
            break
    rec = {"value": N * runs / el, "unit": "nodes/s", "cores": 1, "kind": "oracle",
           "sample": f"{runs} sequential FP64 solves of the N={N}, n={n}, m={m} instance on 1 thread "
                     f"({el:.1f} s)", "build": orc.BUILD_FLAGS}
    rec.update(host_cpu())
    return rec


def batch_record(args, steps: int, cpu_seconds: float) -> dict:
    """512 independent trees (N log-uniform in [256, 16384], p ~ U(0.8, 0.98), n = 8,
    m = 3), MIXED32 with one refinement step: rcr_batch_solve (each tree's own
    buffers, one merged launch sequence) against one rcr_solve per tree, both at
    KKT residual <= 1e-8, and the oracle on all host cores."""
    import numpy as np
    import torch
    from paper_2608_01332_amd import rcr
    from paper_2608_01332_amd import workloads as w
    dev = torch.device("cuda:0")
    T = args.trees
    t0 = time.perf_counter()
    pars, datas = [], []
    for t in range(T):
        p_, d_, spec = w.config_instance(3, tree=t)
        pars.append(p_)
        datas.append(d_)
    gen_s = time.perf_counter() - t0
    n, m = spec.n, spec.m
    t0 = time.perf_counter()
    plans = [rcr.Plan(p_, n, m) for p_ in pars]
    plan_ms = (time.perf_counter() - t0) * 1e3
    t0 = time.perf_counter()
    rcr.batch_prepare(plans)
    merge_ms = (time.perf_counter() - t0) * 1e3
    Ntot = sum(len(p_) for p_ in pars)
    probs = [rcr.to_device(d_, dev) for d_ in datas]
    outs = [rcr.alloc_solution(p_, dev) for p_ in plans]
    stream = torch.cuda.current_stream(dev)
    kw = dict(precision=rcr.MIXED32, refine_steps=1, executor=rcr.EXEC_GRAPH)
    chk = rcr.batch_solve(plans, probs, outs, check=True, kkt_residual=True, **kw)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    for _ in range(2):
        rcr.batch_solve(plans, probs, outs, **kw)
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(steps):
        rcr.batch_solve(plans, probs, outs, stream=stream, **kw)
    e1.record(stream)
    torch.cuda.synchronize()
    batched_ms = e0.elapsed_time(e1) / steps
    # one solve per tree (each tree's own plan, launch sequence and buffers)
    if getattr(args, "no_separate", False):
        for p_ in plans:
            p_.close()
        return {"workload": f"{T} trees, n=8, m=3, MIXED32 + 1 refinement (merged only)", "trees": T,
                "nodes": int(Ntot), "nodes_per_s": Ntot / (batched_ms / 1e3), "ms_per_batch": batched_ms,
                "kkt_residual_batched": chk["kkt_residual"], "steps": steps}
    worst = 0.0
    for p_, pr, ou in zip(plans, probs, outs):
        r = rcr.solve(p_, pr, out=ou, check=True, kkt_residual=True, **kw)
        worst = max(worst, r["kkt_residual"])
    torch.cuda.synchronize()
    reps = max(1, steps // 4)
    e0.record(stream)
    for _ in range(reps):
        for p_, pr, ou in zip(plans, probs, outs):
            rcr.solve(p_, pr, out=ou, stream=stream, **kw)
    e1.record(stream)
    torch.cuda.synchronize()
    separate_ms = e0.elapsed_time(e1) / reps
    rec = {"workload": f"{T} trees, N log-uniform [256,16384], p~U(0.8,0.98), n=8, m=3, MIXED32 + 1 refinement",
           "trees": T, "nodes": int(Ntot), "nodes_per_s": Ntot / (batched_ms / 1e3), "ms_per_batch": batched_ms,
           "separate_ms": separate_ms, "separate_nodes_per_s": Ntot / (separate_ms / 1e3),
           "speedup": separate_ms / batched_ms, "kkt_residual_batched": chk["kkt_residual"],
           "kkt_residual_separate_max": worst, "steps": steps, "merge_plan_ms": merge_ms, "plan_ms": plan_ms,
           "generate_s": gen_s}
    if cpu_seconds > 0:
        from oracle import riccati as orc
        nth = min(16, host_cpu()["cpus_available"])
        tt0 = time.perf_counter()
        done, nodes = 0, 0
        while time.perf_counter() - tt0 < cpu_seconds and done < T:
            chunk = list(zip(pars[done:done + 32], datas[done:done + 32]))
            orc.tree_riccati_batch(chunk, nth)
            nodes += sum(len(p_) for p_, _ in chunk)
            done += len(chunk)
        el = time.perf_counter() - tt0
        cb = {"value": nodes / el, "unit": "nodes/s", "cores": nth, "kind": "oracle",
              "sample": f"first {done} of the {T} trees ({nodes} nodes), FP64, {nth} threads, {el:.1f} s"}
        cb.update(host_cpu())
        rec["cpu_baseline"] = cb
    for p_ in plans:
        p_.close()
    del probs, outs
    torch.cuda.empty_cache()
    return rec


def bench_batch(args) -> dict:
    rec = batch_record(args, args.steps, args.cpu_seconds)
    out = {"metric": METRIC, "value": rec["nodes_per_s"], "unit": "nodes/s", "n_gpus": 1, "steps": args.steps,
           "warmup": 2, "ms_per_step": rec["ms_per_batch"], "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f32+f64-refine", "data": "synthetic",
           "config": {"workload": rec["workload"] + ", one rcr_batch_solve", "trees": rec["trees"],
                      "nodes": rec["nodes"]}}
    out.update({k: v for k, v in rec.items() if k not in ("workload", "trees", "nodes")})
    return out


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
        print(f"[bench] extreme {kind}", file=sys.stderr, flush=True)
        # the re-solves' data drawn ahead on host threads (numpy releases the
        # interpreter lock in its array work), each from its own seed as before
        import concurrent.futures as cf
        with cf.ThreadPoolExecutor(max_workers=4) as gen_pool:
            futs = [gen_pool.submit(w.lqr_data, par, w.DataSpec(6, 2),
                                    np.random.default_rng(w.config_seed(4, s_, ti))) for s_ in range(args.resolves)]
        for s_ in range(args.resolves):
            d = futs[s_].result()
            futs[s_] = None
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
            del d
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


def _serve_pool(specs, dev):
    """Device data blocks of every (n, m, variant) class a request stream uses."""
    import torch
    from paper_2608_01332_amd import rcr
    from paper_2608_01332_amd import workloads as w
    need = {}
    for e in specs:
        key = (e["n"], e["m"], e["variant"])
        need[key] = max(need.get(key, 0), e["N"])
    pool = {}
    for (n, m, var), Nmax in sorted(need.items()):
        d = w.serve_data_block(Nmax, n, m, var, seed=w.config_seed(5))
        pool[(n, m, var)] = {k: torch.from_numpy(d[k]).to(dev) for k in rcr.PROBLEM_FIELDS}
    return pool


def run_serving(specs, pars, pool, dev, slots: int, batching: bool, budget: int, planner_threads: int,
                sample_every: int = 0, device_planner: bool = False):
    """Drive a Server with the stream's arrival times in real time; returns the
    completed requests (outputs kept only for every sample_every-th) and the
    wall time from the first arrival to the last completion."""
    import numpy as np
    import torch
    from paper_2608_01332_amd import rcr
    from paper_2608_01332_amd import serve
    srv = serve.Server(dev, slots=slots, batching=batching, hbm_budget=budget, planner_threads=planner_threads,
                       device_planner=device_planner)
    # the planner and preparation threads run C code between short Python steps:
    # hand them the interpreter lock promptly
    old_switch = sys.getswitchinterval()
    sys.setswitchinterval(2e-4)
    reqs = [serve.Request(rid=e["rid"], parent=pars[e["topo"]], n=e["n"], m=e["m"],
                          prob={k: v[:e["N"]] for k, v in pool[(e["n"], e["m"], e["variant"])].items()},
                          topo=e["topo"]) for e in specs]
    # warm-up (not timed): a request of every (n, m) class of the stream, alone
    # and then in merged pairs, through the same server, so every kernel the
    # stream uses has been launched once (its code loaded) and the planner
    # threads and staging buffers exist before the first timed arrival; the
    # tree is large enough (WARM_N nodes) to need the per-level launches too
    WARM_N = min([32768] + [int(v["Q"].shape[0]) for v in pool.values()])
    from paper_2608_01332_amd import workloads as w
    classes = sorted({(e["n"], e["m"], e["variant"]) for e in specs})
    wpar = w.tree_chainprob(WARM_N, 0.9, np.random.default_rng(7))
    # slot workspaces and output blocks at the size of the largest group the
    # stream can form (a merged group of max_group_nodes of its largest class)
    big_ws, big_out = 0, 0
    for (n, m) in sorted({(c[0], c[1]) for c in classes}):
        p_ = rcr.Plan(wpar, n, m, single_thread=True)
        G = srv.max_group_nodes
        big_ws = max(big_ws, int(p_.workspace_size(srv.precision) / WARM_N * G) + serve.batch_staging_bytes([G], n, m))
        big_out = max(big_out, serve.io_words(G, n, m)[1] * 8)
        p_.close()
    srv.reserve(1 << max(big_ws - 1, 0).bit_length(), 1 << max(big_out - 1, 0).bit_length())
    wid = -1
    for pair in (1, 2):
        for (n, m, var) in classes:
            for _ in range(pair):
                srv.submit(serve.Request(rid=wid, parent=wpar, n=n, m=m,
                                         prob={k: v[:WARM_N] for k, v in pool[(n, m, var)].items()}))
                wid -= 1
        srv.drain()
    srv.done.clear()
    srv.groups = 0
    srv.stats = {k: 0.0 for k in srv.stats}
    torch.cuda.synchronize()
    # no cyclic garbage collection while the stream runs (a full collection over
    # the requests' objects stalls the loop for tens of milliseconds)
    import gc
    gc.collect()
    gc.disable()
    t0 = time.perf_counter()
    i, done, seen = 0, 0, 0
    while done < len(reqs):
        now = time.perf_counter() - t0
        while i < len(reqs) and specs[i]["arrival"] <= now:
            reqs[i].arrival = t0 + specs[i]["arrival"]
            srv.submit(reqs[i])
            i += 1
        got = srv.poll()
        done += got
        if not got:  # nothing completed: give the planner threads the CPU for up to 0.1 ms
            time.sleep(1e-4 if i >= len(reqs) else min(1e-4, max(0.0, specs[i]["arrival"] - (time.perf_counter() - t0))))
        while seen < len(srv.done):
            r = srv.done[seen]
            if not sample_every or r.rid % sample_every:
                r.out = {}
            seen += 1
    wall = max(r.t_done for r in reqs) - t0
    gc.enable()
    groups = srv.groups
    stats = dict(srv.stats)
    srv.close()
    sys.setswitchinterval(old_switch)
    return reqs, wall, groups, stats


def serve_rate(rate: float, specs, pool, dev, args, mode: str = "continuous", sample: int = 97) -> dict:
    """One rate of the serving stream: latency percentiles, throughput, grouping,
    and (continuous mode) sampled results checked against the same request
    solved alone."""
    import numpy as np
    import torch
    from paper_2608_01332_amd import rcr
    from paper_2608_01332_amd import workloads as w
    pars = {}
    for e in specs:
        if e["topo"] not in pars:
            pars[e["topo"]] = w.serve_tree(e)
    slots, batching = (4, True) if mode == "continuous" else (1, False)
    if mode != "continuous":
        sample = 0
    reqs, wall, groups, hstats = run_serving(specs, pars, pool, dev, slots, batching, args.hbm_budget_gib << 30,
                                             args.planner_threads, sample_every=sample,
                                             device_planner=getattr(args, "device_planner", False))
    lat = np.array([(r.t_done - r.arrival) * 1e3 for r in reqs])
    nodes = sum(r.N for r in reqs)
    row = {"rate_per_s": rate, "mode": mode, "slots": slots, "requests": len(reqs),
           "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
           "mean_ms": float(lat.mean()), "nodes_per_s": nodes / wall, "solves_per_s": len(reqs) / wall,
           "groups": groups, "mean_group": len(reqs) / max(groups, 1),
           "plan_cache_hits": float(np.mean([r.cache_hit for r in reqs])),
           "host_s": {k: round(v, 3) for k, v in hstats.items()}, "wall_s": wall,
           "planner": "device" if getattr(args, "device_planner", False) else "host"}
    if sample:
        torch.cuda.synchronize()
        torch.cuda.empty_cache()  # the run's cached group buffers
        worst_diff, worst_kkt = 0.0, 0.0
        for r in reqs:
            if not r.out:
                continue
            sel = rcr.SELECT_LIST_RANK if getattr(args, "device_planner", False) else rcr.SELECT_GREEDY_INDEX
            plan = rcr.Plan(r.parent, r.n, r.m, selection=sel)  # the selection the server's planner used
            alone = rcr.solve(plan, r.prob, precision=rcr.MIXED32, refine_steps=1, kkt_residual=True)
            for k in rcr.SOLUTION_FIELDS:
                worst_diff = max(worst_diff, float((alone[k] - r.out[k]).abs().max()))
            worst_kkt = max(worst_kkt, alone["kkt_residual"])
            r.out = {}
        row["sampled"] = sum(1 for r in reqs if r.rid % sample == 0)
        row["max_abs_diff_alone_vs_mix"] = worst_diff
        row["max_kkt_residual"] = worst_kkt
    del reqs
    torch.cuda.empty_cache()
    return row


def bench_serve(args) -> dict:
    """Serving stream: Poisson arrivals (rates swept) of tree-LQR solves with N
    log-uniform in [1k, 128k], n in {4, 8, 12, 16}, m in {2, 4}, p ~ U(0.85, 0.97),
    MIXED32 + one refinement step, 30% of requests resending an earlier topology
    with new data; admitted by HBM footprint into 4 stream slots with continuous
    batching.  Latency from arrival to completion, planning of cache misses
    included; the request data is resident in HBM when it arrives."""
    import torch
    from paper_2608_01332_amd import workloads as w
    dev = torch.device("cuda:0")
    rates = [float(x) for x in args.rates.split(",")]
    streams = []
    for ri, rate in enumerate(rates):
        count = args.requests if args.requests else (10000 if rate >= 500 else int(rate * 20))
        specs = w.serve_requests(count, rate, seed=w.config_seed(5, 0, ri))
        streams.append((rate, specs))
    t_gen = time.perf_counter()
    pool = _serve_pool([e for _, sp in streams for e in sp], dev)
    print(f"[serve] data pool {len(pool)} blocks in {time.perf_counter() - t_gen:.1f} s", file=sys.stderr, flush=True)
    rows = []
    for ri, (rate, specs) in enumerate(streams):
        modes = ["continuous"] + (["fifo"] if rate in args.fifo_rates else [])
        for mode in modes:
            row = serve_rate(rate, specs, pool, dev, args, mode)
            rows.append(row)
            print(f"[serve] {json.dumps(row)}", file=sys.stderr, flush=True)
    cont = [r for r in rows if r["mode"] == "continuous"]
    best = max(cont, key=lambda r: r["nodes_per_s"])
    return {"metric": METRIC,
            "value": best["nodes_per_s"], "unit": "nodes/s", "n_gpus": 1, "steps": sum(r["requests"] for r in cont),
            "warmup": 0, "ms_per_step": best["mean_ms"], "p50_ms": best["p50_ms"], "p99_ms": best["p99_ms"],
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32+f64-refine",
            "data": "synthetic",
            "config": {"workload": "serving: Poisson arrivals, N log-uniform [1k,128k], n in {4,8,12,16}, m in {2,4}, "
                                   "p ~ U(0.85,0.97), MIXED32 + 1 refinement, 30% plan reuse, 4 slots, "
                                   "continuous batching, HBM-footprint admission",
                       "hbm_budget_gib": args.hbm_budget_gib},
            "rates": rows}


def bench_lift(args) -> dict:
    """The node-control variant of the 65,536-node instance (n = 12, m = 4, one
    control per non-leaf node) solved through the exact lifting: device lift,
    rake-compress solve of the 127,970-node lifted tree (state 16), device
    projection."""
    import numpy as np
    import torch
    from paper_2608_01332_amd import rcr
    from paper_2608_01332_amd import workloads as w
    dev = torch.device("cuda:0")
    par, nd = w.config2_lift_instance()
    t0 = time.perf_counter()
    plan = rcr.Plan.lift(par, 12, 4)
    plan_ms = (time.perf_counter() - t0) * 1e3
    prob = rcr.to_device(nd, dev, fields=rcr.NATIVE_FIELDS)
    stream = torch.cuda.current_stream(dev)
    res = {}
    for name, prec in (("fp64", rcr.FP64), ("mixed32", rcr.MIXED32)):
        chk = rcr.lift_solve(plan, prob, precision=prec, refine_steps=1, executor=rcr.EXEC_GRAPH, check=True,
                             kkt_residual=True)
        out = {k: chk[k] for k in rcr.NATIVE_SOLUTION_FIELDS}
        for _ in range(args.warmup):
            rcr.lift_solve(plan, prob, out=out, precision=prec, refine_steps=1, executor=rcr.EXEC_GRAPH)
        evs = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
        torch.cuda.synchronize()
        evs[0].record(stream)
        for k in range(args.steps):
            rcr.lift_solve(plan, prob, out=out, precision=prec, refine_steps=1, executor=rcr.EXEC_GRAPH,
                           stream=stream)
            evs[k + 1].record(stream)
        torch.cuda.synchronize()
        ms = [evs[k].elapsed_time(evs[k + 1]) for k in range(args.steps)]
        res[name] = {"native_nodes_per_s": len(par) / (float(np.mean(ms)) / 1e3),
                     "lifted_nodes_per_s": plan.N / (float(np.mean(ms)) / 1e3),
                     "ms_per_step": float(np.mean(ms)), "p50_ms": float(np.percentile(ms, 50)),
                     "p99_ms": float(np.percentile(ms, 99)), "kkt_residual_lifted": chk["kkt_residual"]}
    return {"metric": "tree-LQR nodes/sec vs CPU Riccati at KKT res 1e-8; p50/p99 solve latency",
            "value": res["fp64"]["native_nodes_per_s"], "unit": "nodes/s", "n_gpus": 1, "steps": args.steps,
            "warmup": args.warmup, "ms_per_step": res["fp64"]["ms_per_step"], "higher_is_better": True,
            "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
            "config": {"workload": "node-control variant of the N=65536 p=0.95 tree, n=12, m=4, one control per "
                                   "non-leaf node, exact lifting to 127,970 nodes of state 16",
                       "lifted_N": plan.N, "plan_ms": plan_ms},
            "precisions": res}


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--executor", choices=["graph", "levels"], default="graph")
    ap.add_argument("--cpu-seconds", type=float, default=12.0, help="CPU oracle sample length; 0 skips it")
    ap.add_argument("--class-steps", type=int, default=5, help="steps of the per-launch event pass")
    ap.add_argument("--no-mixed", action="store_true", help="skip the MIXED32 + refinement leg")
    ap.add_argument("--no-tune", action="store_true", help="keep the default launch mapping (no autotuning)")
    ap.add_argument("--launch", default="", help="explicit launch mapping of the single workload, "
                    "'key=value,...' with the fields of rcr_launch_config (no autotuning)")
    ap.add_argument("--copy-mib", type=int, default=1024)
    ap.add_argument("--rates", default="100,200,500,1000,2000,5000")
    ap.add_argument("--requests", type=int, default=0, help="requests per rate (0: 10k, or 20 s of arrivals below 500/s)")
    ap.add_argument("--fifo-rates", type=lambda s: [float(x) for x in s.split(",") if x], default=[100.0, 500.0, 2000.0],
                    help="rates at which the one-slot FIFO queue (no batching) is also measured")
    ap.add_argument("--hbm-budget-gib", type=int, default=64)
    ap.add_argument("--planner-threads", type=int, default=12)
    ap.add_argument("--workload", choices=["single", "batch", "extreme", "copy", "serve", "lift"], default="single",
                    help="single: the 65,536-node tree (default); batch: the 512-tree batched workload; "
                         "extreme: the 1M-node shape-extreme trees; copy: plain HBM copy (counter calibration); "
                         "serve: the request stream at swept arrival rates; lift: the node-control variant through the lifting")
    ap.add_argument("--resolves", type=int, default=8)
    ap.add_argument("--trees", type=int, default=512)
    ap.add_argument("--no-batch", action="store_true", help="single workload: skip the batched sub-record")
    ap.add_argument("--no-serve", action="store_true", help="single workload: skip the serving sub-record")
    ap.add_argument("--serve-rate", type=float, default=1000.0, help="arrival rate of the serving sub-record")
    ap.add_argument("--serve-requests", type=int, default=10000, help="requests of the serving sub-record")
    ap.add_argument("--no-separate", action="store_true", help="batch workload: merged solves only (for profiling)")
    ap.add_argument("--device-planner", action="store_true", help="serve workload: plan cache misses on the GPU")
    ap.add_argument("--no-extreme", action="store_true", help="single workload: skip the shape-extreme sub-record")
    ap.add_argument("--no-lift", action="store_true", help="single workload: skip the lifted sub-record")
    ap.add_argument("--summarize-stats", default="", help="print the kernel statistics of a rocprofv3 run directory")
    ap.add_argument("--summarize-timeline", default="", help="print one solve's launches from a --kernel-trace run")
    ap.add_argument("--timeline-solve", type=int, default=10, help="which solve of the trace --summarize-timeline prints")
    ap.add_argument("--summarize-pmc", default="", choices=["", "traffic", "flops"],
                    help="print the dominant class's per-launch figures from rocprofv3 --pmc run directories")
    ap.add_argument("--pmc-run", action="append", default=[],
                    help="Q:DIR, a --pmc run directory of the single workload at quad_tail_rounds=Q")
    ap.add_argument("--pmc-copy", action="append", default=[],
                    help="COUNTER:DIR, a --pmc run directory of the copy workload for that counter")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: measures one GPU only; --gpus {args.gpus} is not supported "
              "(independent trees shard across GPUs with no communication: each GPU runs its own plans)",
              file=sys.stderr)
        return 2
    if args.summarize_stats:
        print(summarize_stats(args.summarize_stats))
        return 0
    if args.summarize_timeline:
        print(summarize_timeline(args.summarize_timeline, args.timeline_solve))
        return 0
    if args.summarize_pmc:
        runs = {}
        for spec in args.pmc_run:
            q, dirpath = spec.split(":", 1)
            runs.setdefault(int(q), {})[dirpath] = dirpath
        copies = dict(x.split(":", 1) for x in args.pmc_copy)
        print(summarize_pmc(args.summarize_pmc, runs, copies))
        return 0

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
    if args.workload == "serve":
        print(json.dumps(bench_serve(args)), flush=True)
        return 0
    if args.workload == "lift":
        print(json.dumps(bench_lift(args)), flush=True)
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

    tuned = None
    if args.launch:
        # an explicit launch mapping ("key=value,..."), no autotuning
        plan.set_launch({k: int(v) for k, v in (kv.split("=") for kv in args.launch.split(","))})
        tuned = plan.get_launch()
    elif not args.no_tune:
        # launch mapping of the narrow levels, autotuned on this instance (untimed)
        tuned, tuned_ms = plan.tune(prob, out=out)
    # accuracy at the measured configuration (outside the timed region)
    chk = rcr.solve(plan, prob, out=out, executor=ex, check=True, kkt_residual=True)
    kkt = chk["kkt_residual"]
    fp64_out = {k: v.cpu().numpy() for k, v in out.items()}

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

    # HIP-event pass on the executor that was timed: device time and launch count
    # per kernel class (graph: events only where the class changes, so a class's
    # launches run back to back as in the timed steps)
    cls_ms, cls_n = {}, {}
    for _ in range(max(1, args.class_steps)):
        r = rcr.solve(plan, prob, out=out, executor=ex, kernel_ms=True, stream=stream)
        for k, v in r["kernel_ms"].items():
            cls_ms[k] = cls_ms.get(k, 0.0) + v
            cls_n[k] = cls_n.get(k, 0) + r["kernel_launches"][k]
    reps = max(1, args.class_steps)
    words = alg_words(st, n, m)
    b_alg = sum(words.values()) * 8
    b_io = io_words(N, n, m) * 8
    # Dominant kernel class: the per-level quadratic contraction launches, which
    # cover levels 1..k (k = their launch count; the narrow levels after them run
    # in the tail kernel).  Its algorithmic bytes are those of the ops in its own
    # levels, at the fixed words per primitive (rake 5s, combine 3s, absorb 3s,
    # compress 10s; a rake's expansion P_j = U_j, fused into it, is not counted).
    # When the first level is fused with the condensation, that launch also
    # condenses every edge: the condensation's words E (5s + 2t + v) count too.
    ops = plan.export_ops()
    k_q = cls_n.get("quad_contract", 0) // reps
    sel = ops[ops[:, 2] <= k_q]
    words_q = sum(int((sel[:, 0] == kind).sum()) * mult * n * n for kind, mult in CONTRACT_WORDS.items())
    fused_condense = cls_n.get("condense", 0) == 0  # level 1 condenses every edge in its own launch
    if fused_condense:
        words_q += words["condense"]
    dom = "quad_contract"
    dom_ms = cls_ms[dom] / reps
    dom_launches = cls_n[dom] / reps
    bytes_per_solve = words_q * 8
    achieved = bytes_per_solve / (dom_ms / 1e3) / 1e9
    mapping = mapping_string(tuned)
    traffic = read_profile_value("traffic_quad_contract", mapping, "hbm_bytes_per_launch")
    flops = read_profile_value("flops_quad_contract", mapping, "fp64_flops_per_launch")
    class_sum_ms = sum(cls_ms.values()) / reps
    avg_launch_s = dom_ms / 1e3 / dom_launches

    rec = {
        "metric": METRIC,
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
                   "rounds": st["rounds"], "executor": args.executor, "precision": "fp64",
                   "launch_mapping": tuned if tuned is not None else "default"},
        "kkt_residual": kkt,
        "roofline": {"bound": "hbm", "kernel_class": dom, "achieved": achieved, "peak": PEAK_HBM_GBS,
                     "unit": "GB/s", "frac": achieved / PEAK_HBM_GBS,
                     "traffic": traffic,
                     "bytes_per_launch": bytes_per_solve / dom_launches,
                     "avg_launch_us": avg_launch_s * 1e6,
                     "launches_per_step": dom_launches,
                     "includes_condensation": fused_condense,
                     "fp64_tflops": (flops / avg_launch_s / 1e12) if flops is not None else None,
                     "fp64_peak_tflops": PEAK_FP64_TFLOPS,
                     "fp64_flop_frac": (flops / avg_launch_s / 1e12 / PEAK_FP64_TFLOPS) if flops is not None else None},
        "headline": {"B_alg_bytes": b_alg, "B_alg_frac": b_alg / (ms_per_step / 1e3) / 1e9 / PEAK_HBM_GBS,
                     "B_io_bytes": b_io, "B_io_frac": b_io / (ms_per_step / 1e3) / 1e9 / PEAK_HBM_GBS,
                     "dominant_class_frac": achieved / PEAK_HBM_GBS},
        "kernel_ms_per_step": {k: round(v / reps, 4) for k, v in cls_ms.items()},
        "kernel_launches_per_step": {k: v // reps for k, v in cls_n.items() if v},
        "kernel_sum_ms_per_step": class_sum_ms,
        "plan_ms": plan_s * 1e3,
        "wall_ms_per_step": wall * 1e3 / args.steps,
    }
    oracle_ref = None
    if args.cpu_seconds > 0:
        from oracle import riccati as orc
        oracle_ref = orc.tree_riccati(parent, data)
        rec["rel_err_vs_oracle"] = {k: float(np.abs(fp64_out[k] - oracle_ref[k]).max() /
                                             max(np.abs(oracle_ref[k]).max(), 1e-300)) for k in rcr.SOLUTION_FIELDS}
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
        mr = rcr.solve(plan, prob, out=mout, precision=rcr.MIXED32, refine_steps=1, executor=ex, kernel_ms=True,
                       stream=stream)
        mrec = {"value": N * args.steps / (mtot / 1e3), "unit": "nodes/s",
                "ms_per_step": mtot / args.steps, "p50_ms": float(np.percentile(mms, 50)),
                "p99_ms": float(np.percentile(mms, 99)), "refine_steps": 1,
                "kkt_residual": chk["kkt_residual"],
                "kernel_ms_per_step": {k: round(v, 4) for k, v in mr["kernel_ms"].items() if v},
                "kernel_launches_per_step": {k: v for k, v in mr["kernel_launches"].items() if v}}
        if oracle_ref is not None:
            mrec["rel_err_vs_oracle"] = {
                k: float(np.abs(mout[k].cpu().numpy() - oracle_ref[k]).max() / max(np.abs(oracle_ref[k]).max(), 1e-300))
                for k in rcr.SOLUTION_FIELDS}
        rec["mixed32"] = mrec
        del mout
    if args.cpu_seconds > 0:
        cb = cpu_baseline(parent, data, args.cpu_seconds)
        rec["cpu_baseline"] = cb
        rec["speedup_vs_cpu_oracle"] = value / cb["value"]
    else:
        rec["cpu_baseline"] = None
    del prob, out
    plan.close()
    torch.cuda.empty_cache()
    if not args.no_batch:
        print("[bench] batched workload", file=sys.stderr, flush=True)
        rec["batch"] = batch_record(args, max(3, args.steps // 4), min(args.cpu_seconds, 8.0))
    if not args.no_serve:
        print("[bench] serving workload", file=sys.stderr, flush=True)
        specs = w.serve_requests(args.serve_requests, args.serve_rate, seed=w.config_seed(5, 0, 3))
        t_gen = time.perf_counter()
        pool = _serve_pool(specs, dev)
        row = serve_rate(args.serve_rate, specs, pool, dev, args)
        row["data_pool_s"] = time.perf_counter() - t_gen - row["wall_s"]
        rec["serve"] = row
        del pool
        torch.cuda.empty_cache()
    if not args.no_extreme:
        # the shape-extreme trees at 1,048,576 nodes: one plan each, eight re-solves with fresh data
        print("[bench] shape-extreme workload", file=sys.stderr, flush=True)
        ex_rec = bench_extreme(args)
        rec["extreme"] = {"workload": ex_rec["config"]["workload"], "nodes_per_s": ex_rec["value"],
                          "ms_per_solve": ex_rec["ms_per_step"], "resolves": args.resolves,
                          "trees": {k: {kk: v[kk] for kk in ("median_ms", "max_ms", "kkt_residual_max", "plan_ms")}
                                    for k, v in ex_rec["trees"].items()}}
        torch.cuda.empty_cache()
    if not args.no_lift:
        print("[bench] lifted node-control workload", file=sys.stderr, flush=True)
        lf = bench_lift(args)
        rec["lift"] = {"workload": lf["config"]["workload"], "native_nodes_per_s": lf["value"],
                       "ms_per_step_fp64": lf["precisions"]["fp64"]["ms_per_step"],
                       "kkt_residual_fp64": lf["precisions"]["fp64"]["kkt_residual_lifted"],
                       "ms_per_step_mixed32": lf["precisions"]["mixed32"]["ms_per_step"],
                       "kkt_residual_mixed32": lf["precisions"]["mixed32"]["kkt_residual_lifted"]}
        torch.cuda.empty_cache()
    # the plan of the same tree built on the device (list-rank selection) against
    # the host planner's with that selection on one host thread: median of 5 builds
    par_d = torch.from_numpy(np.ascontiguousarray(parent, dtype=np.int64)).to(dev)
    t_dev, t_host, same = [], [], True
    for _ in range(5):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        pd = rcr.Plan.from_device(par_d, n, m)
        t_dev.append(time.perf_counter() - t0)
        t0 = time.perf_counter()
        ph = rcr.Plan(parent, n, m, selection=rcr.SELECT_LIST_RANK, single_thread=True)
        t_host.append(time.perf_counter() - t0)
        same = same and pd.digest() == ph.digest()
    rec["device_planner"] = {"tree": f"N={N} chain-prob p=0.95 (the single workload's)",
                             "device_ms": float(np.median(t_dev)) * 1e3, "host_ms": float(np.median(t_host)) * 1e3,
                             "host_threads": 1, "identical_plans": bool(same)}
    print(json.dumps(rec), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
