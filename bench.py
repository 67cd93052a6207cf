#!/usr/bin/env python3
"""Benchmark of the sliced tensor-network amplitude path on one MI355X.

Workload (default): 6x6-qubit grid random circuit of depth (1+14+1), the
contraction sliced on 8 wires (256 slices), a batch of 64 amplitudes (the
six qubits of the bottom row open, the other 30 bits seeded), complex64
arithmetic on FP32 matrix cores, FP64 slice sum.  One step = every slice of
the batch contracted and summed (one graph launch).

Prints one JSON line.  `value` is amplitudes per second with the circuit's
leaves and plan resident in HBM before the timed region starts.
"""
import argparse
import json
import math
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "amplitudes/s + contraction TFLOP/s vs plain FP32 path at stated error; p99 latency"
PEAK_MFMA_FP32 = 157.3   # TFLOP/s, MI355X dense FP32 matrix
PEAK_MFMA_16 = 2500.0    # TFLOP/s, MI355X dense FP16 / BF16 matrix
PEAK_HBM = 8000.0        # GB/s
# Kernel kinds of the timing probe: 0 generic SIMT, 1 FP32 MFMA, 2 rows,
# 3 16-bit MFMA (probe kind 1 also brackets kind 3; kind 4 brackets all).
KIND_NAMES = {0: "k_simt", 1: "k_mfma32", 2: "k_rows", 3: "k_mfma16"}
KIND_SOURCES = {0: "k_simt.hip", 1: "k_mfma32.hip", 2: "k_rows.hip", 3: "k_mfma16.hip"}
KIND_LABELS = {
    0: "k_simt (generic table-driven contraction, split-K)",
    1: "k_mfma32 (fused permute + complex GEMM, FP32 MFMA 32x32x2)",
    2: "k_rows (row-streaming stem step, FP32 MFMA 16x16x4, LDS-staged stores)",
    3: "k_mfma16 (fused permute + complex GEMM, FP16/BF16 MFMA 32x32x16)",
}
TIME_ALL = 4
GOLDEN_CONFIG2 = os.path.join(ROOT, "tests", "golden", "config2_amplitudes.txt")
# Counter summaries (FETCH_SIZE / WRITE_SIZE) of the kernels of the default
# amplitude workload, per (kernel kind, precision of the leg).
TRAFFIC_PROFILES = {(1, "f32"): "k_mfma32_config2_6x6x14_fp32_traffic.md",
                    (2, "f32"): "k_rows_config2_6x6x14_fp32_traffic.md",
                    (0, "f32"): "k_simt_config2_6x6x14_fp32_traffic.md",
                    (3, "f16"): "k_mfma16_config2_6x6x14_fp16_traffic.md",
                    (2, "f16"): "k_rows_config2_6x6x14_fp16_traffic.md",
                    (0, "f16"): "k_simt_config2_6x6x14_fp16_traffic.md"}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--mode", default="amplitudes",
                    choices=["amplitudes", "steps", "kernel", "serve", "copy", "share", "batch"],
                    help="amplitudes: the sliced circuit contraction (default); steps: "
                         "synthetic rank-24..32 pairwise contractions, fused vs permute+GEMM; "
                         "kernel: one plan-shaped contraction repeated; share: one GPU's "
                         "1024-slice share of a 10x10 (1+20+1) circuit in FP32, FP16, BF16")
    ap.add_argument("--mnk", default="15,10,13", help="kernel mode: m,n,k bits")
    ap.add_argument("--batch", type=int, default=8, help="kernel mode: copies per launch")
    ap.add_argument("--reps", type=int, default=5)
    ap.add_argument("--kprec", default="f32", choices=["f32", "f16", "bf16"],
                    help="kernel mode: arithmetic")
    ap.add_argument("--cases", type=int, default=12, help="steps mode: number of synthetic cases")
    ap.add_argument("--max-cases", type=int, default=0,
                    help="steps mode: 1 adds the (32,32,16) and (32,24,12) cases (32 GiB tensors)")
    ap.add_argument("--requests", type=int, default=600, help="serve mode: Poisson requests")
    ap.add_argument("--load", type=float, default=0.8, help="serve mode: rate / saturation rate")
    ap.add_argument("--budget-gb", type=float, default=192.0,
                    help="serve mode: device pool (plans, workspaces, outputs)")
    ap.add_argument("--share-bound", type=int, default=28,
                    help="share mode: per-slice bound, log2 elements")
    ap.add_argument("--share-local", type=int, default=10,
                    help="share mode: enumerated sliced wires (2^L slices)")
    ap.add_argument("--share-trials", type=int, default=256)
    ap.add_argument("--share-candidates", type=int, default=16,
                    help="share mode: plans searched (seeds from the circuit seed on)")
    ap.add_argument("--share-probe", type=int, default=4,
                    help="share mode: best-ranked plans timed on 8 slices")
    ap.add_argument("--share-bf16-min-log2", type=int, default=0,
                    help="share mode: smallest intermediate (log2 elements) stored in BF16; 0 = default")
    ap.add_argument("--share-precs", default="f32,f16,bf16", help="share mode: precisions to run")
    ap.add_argument("--share-f32-parts", type=int, default=2,
                    help="share mode: FP32 baseline calls (each prints a progress line)")
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--prec", default="f32", choices=["f32", "f16", "bf16"])
    ap.add_argument("--rows", type=int, default=6)
    ap.add_argument("--cols", type=int, default=6)
    ap.add_argument("--depth", type=int, default=14)
    ap.add_argument("--open", type=int, default=6)
    ap.add_argument("--sliced", type=int, default=8)
    ap.add_argument("--seed", type=int, default=2)
    ap.add_argument("--trials", type=int, default=1024)
    ap.add_argument("--plan-seed", type=int, default=2)
    ap.add_argument("--plan-candidates", type=int, default=256,
                    help="plans searched with seeds plan-seed.. (in parallel) and ranked by "
                         "the planner's cost (1 = no selection)")
    ap.add_argument("--probe-candidates", type=int, default=8,
                    help="best-ranked plans timed on a sample of slices; the fastest is "
                         "benchmarked")
    ap.add_argument("--probe-slices", type=int, default=32)
    ap.add_argument("--roofline-kernel", type=int, default=-1, choices=[-1, 0, 1, 2],
                    help="kernel kind bracketed in the timed region (0 simt, 1 mfma, 2 rows); "
                         "-1 = the one that takes longest in a probe step")
    ap.add_argument("--ws-fraction", type=float, default=0.85)
    ap.add_argument("--slices", type=int, default=0,
                    help="contract only the first N slice ids (profiling); 0 = all")
    ap.add_argument("--max-group", type=int, default=0,
                    help="bound on the slices per batched group (0 = workspace only)")
    ap.add_argument("--graph-steps", type=int, default=1)
    ap.add_argument("--lp-steps", type=int, default=1,
                    help="timed steps of the reduced-precision (f16) comparison, 0 = skip")
    ap.add_argument("--tune-cache", default="",
                    help="per-step kernel choices file read before tuning and written after "
                         "(runs that share it make the same choices)")
    ap.add_argument("--tune", type=int, default=1,
                    help="per-step kernel tuning of the benchmarked plan before timing (1 = on)")
    ap.add_argument("--serve-requests", type=int, default=200,
                    help="amplitude mode: requests of the serving leg (0 = skip)")
    ap.add_argument("--cpu-seconds", type=float, default=15.0,
                    help="budget of the oracle CPU baseline sample, 0 = skip")
    return ap.parse_args()


def _cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(circ, openq, bits, plan, budget_s):
    """The oracle timed on whole slices of the benchmarked plan: each slice
    contracted in complex128 along the plan's tree (oracle.contract_ordered,
    the order given as data); as many slices as fit ~70% of the budget on all
    host threads, then one slice on one thread; both extrapolated to every
    slice of the step."""
    import oracle
    sys.path.insert(0, os.path.join(ROOT, "tests"))
    from plan_order import oracle_order, oracle_wires_and_ids
    try:
        from threadpoolctl import threadpool_info, threadpool_limits
        threads = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
    except Exception:
        threadpool_limits = None
        threads = os.cpu_count() or 1
    e = plan.export()
    groups, pairs = oracle_order(circ, openq, e)
    n_sl = int(plan.info()["n_slices"])

    def one(sid):
        ow, oids = oracle_wires_and_ids(e, [sid])
        return oracle.slice_values_ordered(circ, openq, bits, ow, oids, groups, pairs)

    t0 = time.perf_counter()
    done = 0
    for sid in range(n_sl):
        one(sid)
        done += 1
        if time.perf_counter() - t0 > 0.7 * budget_s:
            break
    dt = time.perf_counter() - t0
    full = dt / done * n_sl
    n_amp = 1 << len(openq)
    res = {"value": n_amp / full, "unit": "amplitudes/s", "cores": int(threads), "kind": "oracle",
           "sample": f"{done} of the {n_sl} slices of the benchmarked plan, each contracted in "
                     f"complex128 along the plan's tree (oracle.contract_ordered), {dt:.1f} s on "
                     f"{threads} threads, extrapolated to all {n_sl} slices ({full:.1f} s)",
           "cpu_model": _cpu_model(), "host_cpus": os.cpu_count()}
    if threadpool_limits is not None:
        with threadpool_limits(1):
            t1 = time.perf_counter()
            one(done % n_sl)
            d1 = time.perf_counter() - t1
        res["one_thread"] = {"value": n_amp / (d1 * n_sl), "unit": "amplitudes/s",
                             "sample": f"1 slice on 1 thread, {d1:.1f} s, extrapolated to "
                                       f"{n_sl} slices ({d1 * n_sl:.0f} s)"}
    return res


def _norm_err(a, ref, n_qubits):
    """max |a - ref| in units of the RMS amplitude 2^(-n/2)."""
    import numpy as np
    return float(np.max(np.abs(np.asarray(a) - np.asarray(ref)))) * 2.0 ** (n_qubits / 2)


def _fidelity(a, ref):
    """Linear fidelity |<ref|a>|^2 / (<ref|ref><a|a>)."""
    import numpy as np
    a, ref = np.asarray(a).ravel(), np.asarray(ref).ravel()
    num = abs(np.vdot(ref, a)) ** 2
    return float(num / (np.vdot(ref, ref).real * np.vdot(a, a).real))


def kernel_source_hash(root, kind):
    """SHA-256 over the sources of one kernel kind and the shared headers."""
    import hashlib
    h = hashlib.sha256()
    for f in (KIND_SOURCES[kind], "kernels_dev.h", "kernels.h"):
        h.update(open(os.path.join(root, "paper_2110_14502_amd", "csrc", f), "rb").read())
    return h.hexdigest()


def _profile_traffic(kind, prec, launches):
    """Counter traffic over algorithmic bytes of a kernel kind's launches,
    from a committed counter summary: each launch takes the measured ratio of
    its shape (m, n, k, copies) in the summary's table, or the ratio of the
    summary's remaining small launches; None when the kernel sources changed
    since the counters were taken, or when launches of shapes the table does
    not hold carry more than 5% of the bytes (the tuner put a step the
    summary did not see on this kernel)."""
    root = os.path.dirname(os.path.abspath(__file__))
    try:
        text = open(os.path.join(root, "profiles", TRAFFIC_PROFILES[(kind, prec)])).read()
    except (OSError, KeyError):
        return None
    vals = dict(re.findall(r"^(\w+): (\S+)$", text, re.M))
    if vals.get("kernel_source_sha256") != kernel_source_hash(root, kind):
        return None
    shapes, others = {}, None
    for row in re.findall(r"^\| (\S+) \| (\S+) \| (\S+) \| \S+ \| \S+ \| (\S+) \| (\S+) \| \S+ \|$",
                          text, re.M):
        try:
            scaled, alg = float(row[3]), float(row[4])
        except ValueError:
            continue
        if row[0] == "others":
            others = (scaled, alg)
            continue
        key = (tuple(int(x) for x in row[1].split(",")), int(row[2]))
        s0, a0 = shapes.get(key, (0.0, 0.0))
        shapes[key] = (s0 + scaled, a0 + alg)
    total = covered = traffic = 0.0
    for L in launches:
        key = (tuple(L["mnk"]), L["copies"])
        total += L["bytes"]
        if key in shapes:
            covered += L["bytes"]
            traffic += L["bytes"] * shapes[key][0] / shapes[key][1]
        elif others is not None and others[1] > 0:
            traffic += L["bytes"] * others[0] / others[1]
        else:
            return None
    if total <= 0 or covered < 0.95 * total:
        return None
    return traffic / total


def plan_cost(plan):
    """The planner's time-like cost of a plan: per step max(complex
    multiply-adds, 20 x elements moved), summed over every slice for the
    steps that depend on the sliced wires and once for those that depend on
    the closed bits only."""
    n = plan.info()["n_slices"]
    cost = 0.0
    for s in plan.steps():
        c = max(s["flops"] / 8.0, 20.0 * s["bytes_c64"] / 8.0)
        if s["depends_on_slice"]:
            cost += n * c
        elif s["depends_on_bits"]:
            cost += c
    return cost


def select_plan(R, net, bits, a):
    """Plan autotuning: search plan-candidates plans (planner seeds
    plan-seed, plan-seed+1, ...) on host threads in parallel, rank them by
    the planner's time-like cost, time the probe-candidates best on the
    device on a sample of probe-slices slices (after a warm call), and return
    the seed and plan of the fastest with the measured times."""
    import torch
    from concurrent.futures import ThreadPoolExecutor
    seeds = [a.plan_seed + i for i in range(max(1, a.plan_candidates))]
    workers = max(1, min(len(seeds), 16, os.cpu_count() or 1))

    def make(sd):
        p = R.Plan(net, n_sliced=a.sliced, path_trials=a.trials, seed=sd)
        return plan_cost(p), sd, p

    t0 = time.perf_counter()
    with ThreadPoolExecutor(workers) as ex:  # the planner releases the GIL
        ranked = sorted(ex.map(make, seeds), key=lambda x: (x[0], x[1]))
    t_plan = time.perf_counter() - t0
    log(f"{len(seeds)} plans in {t_plan:.1f} s on {workers} threads")
    costs = {str(sd): c for c, sd, _ in ranked}
    ranked = ranked[:max(1, a.probe_candidates)]
    seeds = [sd for _, sd, _ in ranked]
    plans = [p for _, _, p in ranked]
    if len(seeds) == 1:
        return seeds[0], {"candidates": len(costs), "plan_seconds": round(t_plan, 2)}, plans[0], None
    # The reduced-precision run of the FP32 benchmark is autotuned the same
    # way, on its own precision.
    precs = [a.prec] + (["f16"] if a.lp_steps > 0 and a.prec == "f32" else [])
    times = {pr: {} for pr in precs}
    best = {pr: (None, None, float("inf")) for pr in precs}
    for i, sd in enumerate(seeds):
        p, plans[i] = plans[i], None
        n_ids = min(a.probe_slices, p.info()["n_slices"])
        p.bind("cuda:0")
        for pr in precs:
            lo, pref = p.workspace_bytes(n_ids, 1, R.PRECISIONS[pr])
            free, _ = torch.cuda.mem_get_info()
            ws = torch.empty(int(min(pref, max(lo, 0.5 * free))), dtype=torch.uint8, device="cuda:0")
            ids = list(range(n_ids))
            p.contract(bits, slice_ids=ids, prec=R.PRECISIONS[pr], workspace=ws)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            p.contract(bits, slice_ids=ids, prec=R.PRECISIONS[pr], workspace=ws)
            torch.cuda.synchronize()
            times[pr][sd] = 1000.0 * (time.perf_counter() - t1) / n_ids
            log(f"plan seed {sd} {pr}: {times[pr][sd]:.3f} ms per slice on {n_ids} slices")
            del ws
            if times[pr][sd] < best[pr][2]:  # keep only the fastest plans alive
                best[pr] = (sd, p, times[pr][sd])
        del p
    chosen, plan, _ = best[a.prec]
    info = {"candidates": len(costs), "probed": len(seeds), "probe_slices": a.probe_slices,
            "plan_seconds": round(t_plan, 2),
            "cost_rank_of_chosen": seeds.index(chosen),
            "ms_per_slice_by_seed": {str(k): round(v, 4) for k, v in times[a.prec].items()},
            "chosen_seed": chosen}
    lp_plan = None
    if len(precs) > 1:
        info["f16_ms_per_slice_by_seed"] = {str(k): round(v, 4) for k, v in times["f16"].items()}
        info["f16_chosen_seed"] = best["f16"][0]
        lp_plan = best["f16"][1]
    return chosen, info, plan, lp_plan


def roofline(kind, tim, a, flops_total, kind_ms, traffic_ratio=None):
    """Roofline entry of the dominant kernel kind from the timing probe."""
    n = max(1, tim["launches"])
    secs = tim["total_ms"] / 1000.0
    fpl, bpl = tim["flops"] / n, tim["bytes"] / n
    if kind == 1:
        peak = PEAK_MFMA_FP32 if a.prec == "f32" else PEAK_MFMA_16
        achieved = tim["flops"] / secs / 1e12 if secs > 0 else 0.0
        bound, unit = "mfma", "TFLOP/s"
    else:
        peak = PEAK_HBM
        achieved = tim["bytes"] / secs / 1e9 if secs > 0 else 0.0
        bound, unit = "hbm", "GB/s"
    label = KIND_LABELS[kind]
    if kind == 1 and a.prec != "f32":
        label = "k_mfma32 + k_mfma16 (fused permute + complex GEMM, FP32 and FP16/BF16 MFMA)"
    return {
        "bound": bound, "kernel": label, "achieved": achieved, "peak": peak, "unit": unit,
        "frac": achieved / peak,
        "traffic": (None if traffic_ratio is None else traffic_ratio * bpl),
        "algorithmic_bytes_per_launch": bpl,
        "flops_per_launch": fpl,
        "launches": tim["launches"],
        "avg_launch_ms": tim["total_ms"] / n,
        "achieved_tflops": tim["flops"] / secs / 1e12 if secs > 0 else 0.0,
        "share_of_step_flops": tim["flops"] / flops_total,
        "probe_ms_per_step_by_kernel": kind_ms,
    }


def launch_table(launches, n_reps=1, prec="f32"):
    """Per-launch roofline: t_min = max(F / P, B / 8 TB/s) with P the matrix
    peak of the launch's arithmetic (FP32 157.3 TFLOP/s; 16-bit matrix cores
    2.5 PFLOP/s), F and B the algorithmic flops and bytes; and per kernel
    kind the summed time, rates and roofline fraction (sum of t_min over
    sum of measured time)."""
    rows, kinds = [], {}
    for L in launches:
        # 16-bit matrix cores: the 16-bit GEMM kernel, and the row kernel on
        # a 16-bit stored A with sums of 16 or more.
        lp_mma = L["kernel"] == 3 or (L["kernel"] == 2 and L["store_a"] != 0 and L["k"] >= 4)
        peak = PEAK_MFMA_16 if lp_mma else PEAK_MFMA_FP32
        t_f = L["flops"] / (peak * 1e12) * 1e3
        t_b = L["bytes"] / (PEAK_HBM * 1e9) * 1e3
        t_min = max(t_f, t_b)
        ms = L["ms"] / n_reps
        rows.append({"step": L["step"], "kernel": KIND_NAMES.get(L["kernel"], str(L["kernel"])),
                     "mnk": [L["m"], L["n"], L["k"]], "copies": L["copies"],
                     "store": [L["store_a"], L["store_b"], L["store_c"]],
                     "variant": L["variant"],
                     "flops": L["flops"], "bytes": L["bytes"], "ms": round(ms, 5),
                     "t_min_ms": round(t_min, 5), "bound": "mfma" if t_f >= t_b else "hbm",
                     "frac": round(t_min / ms, 4) if ms > 0 else None})
        k = kinds.setdefault(L["kernel"], {"launches": 0, "ms": 0.0, "flops": 0.0, "bytes": 0.0,
                                           "t_min_ms": 0.0, "t_min_mfma_ms": 0.0})
        k["launches"] += 1
        k["ms"] += ms
        k["flops"] += L["flops"]
        k["bytes"] += L["bytes"]
        k["t_min_ms"] += t_min
        k["t_min_mfma_ms"] += t_min if t_f >= t_b else 0.0
    out = {}
    for kind, k in kinds.items():
        k["ratio"] = _profile_traffic(kind, prec, [r for r in rows if r["kernel"] == KIND_NAMES.get(kind)])
        secs = k["ms"] / 1e3
        mfma = k["t_min_mfma_ms"] >= 0.5 * k["t_min_ms"]
        peak = PEAK_MFMA_16 if kind == 3 else PEAK_MFMA_FP32
        out[KIND_NAMES.get(kind, str(kind))] = {
            "kernel": KIND_LABELS.get(kind, str(kind)),
            "bound": "mfma" if mfma else "hbm",
            "achieved": (k["flops"] / secs / 1e12) if mfma else (k["bytes"] / secs / 1e9),
            "peak": peak if mfma else PEAK_HBM,
            "unit": "TFLOP/s" if mfma else "GB/s",
            "frac": ((k["flops"] / secs / 1e12) / peak) if mfma else ((k["bytes"] / secs / 1e9) / PEAK_HBM),
            "roofline_frac": k["t_min_ms"] / k["ms"] if k["ms"] > 0 else None,
            "ms_per_step": k["ms"], "t_min_ms_per_step": k["t_min_ms"],
            "achieved_tflops": k["flops"] / secs / 1e12, "achieved_gbs": k["bytes"] / secs / 1e9,
            "launches": k["launches"],
            "traffic": (None if k["ratio"] is None else k["ratio"] * k["bytes"] / k["launches"]),
            "algorithmic_bytes_per_launch": k["bytes"] / k["launches"],
            "traffic_over_algorithmic": k["ratio"]}
    return rows, out


def read_golden(path):
    """(indices, complex128 values) of a stored oracle file."""
    import numpy as np
    idx, val = [], []
    with open(path) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            i, re_, im_ = line.split()
            idx.append(int(i))
            val.append(complex(float(re_), float(im_)))
    return np.array(idx), np.array(val, dtype=np.complex128)


def log(*msg):
    print("[bench]", *msg, file=sys.stderr, flush=True)


def _events_time(fn, reps):
    import torch
    fn()
    torch.cuda.synchronize()
    s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    s.record()
    for _ in range(reps):
        fn()
    e.record()
    torch.cuda.synchronize()
    return s.elapsed_time(e) / reps


def kernel_mode(a):
    """One plan-shaped contraction (summed labels lowest in A and B, random
    output order) repeated; reports TFLOP/s of the chosen kernel."""
    import numpy as np
    import torch
    import paper_2110_14502_amd as R
    m, n, k = [int(x) for x in a.mnk.split(",")]
    rng = np.random.default_rng(7)
    M, N, K = list(range(m)), list(range(100, 100 + n)), list(range(200, 200 + k))
    la = [M[i] for i in rng.permutation(m)] + K
    lb = [N[i] for i in rng.permutation(n)] + K
    lc = M + N
    lc = [lc[i] for i in rng.permutation(len(lc))]
    A = torch.randn(a.batch << (m + k), dtype=torch.complex64, device="cuda")
    B = torch.randn(a.batch << (n + k), dtype=torch.complex64, device="cuda")
    C = torch.empty(a.batch << (m + n), dtype=torch.complex64, device="cuda")
    res = {"mode": "kernel", "m": m, "n": n, "k": k, "batch": a.batch, "prec": a.kprec}
    kp = R.PRECISIONS[a.kprec]
    fl = 8.0 * a.batch * 2.0 ** (m + n + k)
    by = 8.0 * a.batch * (2.0 ** (m + k) + 2.0 ** (n + k) + 2.0 ** (m + n))
    if kp != R.F32 and m >= 7 and n >= 6 and k >= 4:
        # 16-bit matrix-core variants on the plan's storage (A and C in 16
        # bits, B in complex64): the tile walk and the streaming form.
        t16 = torch.float16 if kp == R.F16 else torch.bfloat16
        A16 = torch.randn((a.batch << (m + k), 2), dtype=torch.float32, device="cuda").to(t16)
        C16 = torch.empty((a.batch << (m + n), 2), dtype=t16, device="cuda")
        lp = R.ST_F16 if kp == R.F16 else R.ST_BF16
        for var, name in ((0, "lp_tiles"), (R.VAR_STREAM, "lp_stream")):
            ms = _events_time(lambda: R.pair_contract_stored(
                A16, B, C16, la, lb, lc, lp, R.ST_C64, lp, R.KERN_MFMA16, mma_prec=kp,
                batch=a.batch, stride_a=1 << (m + k), stride_b=1 << (n + k),
                stride_c=1 << (m + n), variant=var), a.reps)
            by16 = a.batch * (4.0 * 2 ** (m + k) + 8.0 * 2 ** (n + k) + 4.0 * 2 ** (m + n))
            res[name] = {"ms": ms, "tflops": fl / ms / 1e9, "gbs": by16 / ms / 1e6}
            log(f"variant {name}: {ms:.3f} ms, {by16 / ms / 1e6:.0f} GB/s")
    if kp == R.F32 and m >= 7 and n >= 6 and k >= 4:
        # FP32 matrix-core variants: 3M / 4M products, per-tile / persistent.
        for var, name in ((0, "3m_auto"), (1, "4m_auto"), (2, "3m_tiles"), (3, "4m_tiles"),
                          (4, "3m_persistent"), (5, "4m_persistent")):
            ms = _events_time(lambda: R.pair_contract_stored(
                A, B, C, la, lb, lc, R.ST_C64, R.ST_C64, R.ST_C64, R.KERN_MFMA, batch=a.batch,
                stride_a=1 << (m + k), stride_b=1 << (n + k), stride_c=1 << (m + n), variant=var),
                a.reps)
            res[name] = {"ms": ms, "tflops": fl / ms / 1e9, "gbs": by / ms / 1e6}
            log(f"variant {name}: {ms:.3f} ms, {fl / ms / 1e9:.1f} TFLOP/s")
    for kern in (-1, 0):
        ms = _events_time(lambda: R.pair_contract(A, B, la, lb, lc, C_out=C, kernel=kern,
                                                  batch=a.batch, stride_a=1 << (m + k),
                                                  stride_b=1 << (n + k), stride_c=1 << (m + n),
                                                  prec=kp),
                          a.reps)
        res["auto" if kern < 0 else "generic"] = {"ms": ms, "tflops": fl / ms / 1e9,
                                                 "gbs": by / ms / 1e6}
        log(f"kernel {kern}: {ms:.3f} ms, {fl / ms / 1e9:.1f} TFLOP/s")
    print(json.dumps(res), flush=True)


def steps_mode(a):
    """Synthetic pairwise contractions of complex64 tensors of rank 24..32
    with random index orders: the fused kernel (FP32, or FP16/BF16 matrix
    cores with --kprec) vs permute + our GEMM + permute and vs permute +
    the vendor complex GEMM (torch.matmul, rocBLAS/hipBLASLt) + permute;
    --max-cases adds the two largest cases, (32, 32, 16) and (32, 24, 12)."""
    import numpy as np
    import torch
    import rqcgen
    import paper_2110_14502_amd as R
    cases = rqcgen.synthetic_step_cases(3, n_cases=a.cases)
    if a.max_cases:
        cases += [rqcgen.synthetic_step(32, 32, 16, 71), rqcgen.synthetic_step(32, 24, 12, 72)]
    kp = R.PRECISIONS[a.kprec]
    peak = PEAK_MFMA_FP32 if kp == R.F32 else PEAK_MFMA_16
    out = []
    for st in cases:
        ra, rb, rc = len(st.labels_a), len(st.labels_b), len(st.labels_c)
        g = torch.Generator(device="cuda").manual_seed(st.seed)
        A = torch.randn(1 << ra, dtype=torch.complex64, device="cuda", generator=g)
        B = torch.randn(1 << rb, dtype=torch.complex64, device="cuda", generator=g)
        C = torch.empty(1 << rc, dtype=torch.complex64, device="cuda")
        K = [x for x in st.labels_a if x in st.labels_b]
        Mf = [x for x in st.labels_a if x not in K]
        Nf = [x for x in st.labels_b if x not in K]
        m, n, k = len(Mf), len(Nf), len(K)
        fl = 8.0 * 2.0 ** (m + n + k)
        reps = a.reps if m + n + k <= 40 else 1
        need = R.pair_workspace_bytes(st.labels_a, st.labels_b, st.labels_c, prec=kp)
        ws = torch.empty(need, dtype=torch.uint8, device="cuda") if need else None
        form = "two-phase (permute + convert, 16-bit GEMM)" if need else "fused"
        log(f"steps case mnk=({m},{n},{k}) prec={a.kprec}: {form}")
        t_f = _events_time(lambda: R.pair_contract(A, B, st.labels_a, st.labels_b, st.labels_c,
                                                   C_out=C, prec=kp, workspace=ws), reps)
        row = {"ranks": [ra, rb, rc], "mnk": [m, n, k], "prec": a.kprec, "form": form,
               "fused_ms": t_f, "fused_tflops": fl / t_f / 1e9,
               "fused_frac_of_peak": fl / t_f / 1e9 / peak}
        if kp == R.F32:
            A2, B2, C2 = torch.empty_like(A), torch.empty_like(B), torch.empty_like(C)

            def unfused():
                R.permute(A, st.labels_a, Mf + K, out=A2)
                R.permute(B, st.labels_b, K + Nf, out=B2)
                R.cgemm(A2, B2, 1 << m, 1 << n, 1 << k, out=C2)
                R.permute(C2, Mf + Nf, st.labels_c, out=C)

            def unfused_vendor():
                R.permute(A, st.labels_a, Mf + K, out=A2)
                R.permute(B, st.labels_b, K + Nf, out=B2)
                torch.matmul(A2.view(1 << m, 1 << k), B2.view(1 << k, 1 << n),
                             out=C2.view(1 << m, 1 << n))
                R.permute(C2, Mf + Nf, st.labels_c, out=C)
            log(f"  fused {t_f:.3f} ms; permute + our GEMM + permute")
            t_u = _events_time(unfused, reps)
            log(f"  {t_u:.3f} ms; permute + vendor GEMM + permute")
            t_v = _events_time(unfused_vendor, reps)
            log(f"  {t_v:.3f} ms; vendor GEMM alone")
            t_g = _events_time(lambda: torch.matmul(A2.view(1 << m, 1 << k), B2.view(1 << k, 1 << n),
                                                    out=C2.view(1 << m, 1 << n)), reps)
            row.update({"unfused_ms": t_u, "unfused_tflops": fl / t_u / 1e9, "speedup": t_u / t_f,
                        "unfused_vendor_ms": t_v, "speedup_vs_vendor_unfused": t_v / t_f,
                        "vendor_gemm_only_tflops": fl / t_g / 1e9})
            del A2, B2, C2
        log(json.dumps(row))
        out.append(row)
        del A, B, C, ws
        torch.cuda.empty_cache()
    res = {"mode": "steps", "prec": a.kprec, "cases": out,
           "median_fused_tflops": float(np.median([r["fused_tflops"] for r in out])),
           "median_frac_of_peak": float(np.median([r["fused_frac_of_peak"] for r in out]))}
    if kp == R.F32:
        res["geomean_speedup"] = float(np.exp(np.mean([np.log(r["speedup"]) for r in out])))
        res["geomean_speedup_vs_vendor_unfused"] = float(
            np.exp(np.mean([np.log(r["speedup_vs_vendor_unfused"]) for r in out])))
    print(json.dumps(res), flush=True)


def run_serving(n_requests, load, budget_gb, grids, depths, circuits_per_family, burst):
    """Continuous batching of amplitude requests over seeded circuits (grids x
    depths, circuits_per_family seeds each; families whose plan exceeds 2^42
    flops are rejected), 0-10 open qubits, FP16 or FP32 at 50/50; a burst
    measures the saturation rate, then n_requests Poisson arrivals at
    load x saturation; latency is submit to result."""
    import numpy as np
    import rqcgen
    import paper_2110_14502_amd as R
    rng = np.random.default_rng(5)
    fams, tried = [], 0
    t = time.perf_counter()
    for (r, c) in grids:
        for d in depths:
            tried += 1
            n = r * c
            circ = rqcgen.grid_rqc(r, c, d, 1)
            try:
                P = R.Plan(R.Network(R.Circuit.from_rqcgen(circ), list(range(n - 10, n))),
                           max_log2_elems=26, path_trials=64, seed=1)
                ok = P.info()["log2_total_flops"] <= 42
            except R.RqcError:
                ok = False
            if ok:
                fams.append((r, c, d))
    log(f"serve: {len(fams)}/{tried} circuit families accepted ({time.perf_counter() - t:.1f}s)")
    pool = {}
    for f in fams:
        for sd in range(circuits_per_family):
            pool[(f, sd)] = rqcgen.grid_rqc(f[0], f[1], f[2], 1000 + sd)

    def draw(i):
        f = fams[int(rng.integers(len(fams)))]
        sd = int(rng.integers(circuits_per_family))
        circ = pool[(f, sd)]
        n = circ.n_qubits
        n_open = int(rng.integers(0, 11))
        openq = list(range(n - n_open, n))
        bits = rqcgen.random_bits(n - n_open, 10000 + i)
        prec = R.F16 if rng.random() < 0.5 else R.F32
        return circ, openq, bits, prec

    srv = R.Server(int(budget_gb * (1 << 30)), max_inflight=8, n_streams=4, max_batch=32)

    def submit(q):
        circ, openq, bits, prec = q
        return srv.submit(circ.n_qubits, circ.gates, openq, bits, prec=prec, max_log2_elems=26)

    def collect(tickets):
        got = {}
        while len(got) < len(tickets):
            for r in srv.poll(1024):
                got[r["ticket"]] = r
            time.sleep(0.0005)
        return [got[t] for t in tickets]

    # Warm-up: one request per circuit builds and binds every plan.
    t = time.perf_counter()
    warm = [submit((c, list(range(c.n_qubits - 2, c.n_qubits)), rqcgen.random_bits(c.n_qubits - 2, 1),
                    R.F32)) for c in pool.values()]
    collect(warm)
    log(f"serve: warmed {len(warm)} plans ({time.perf_counter() - t:.1f}s)")
    # Saturation: a burst of requests at once.
    bq = [draw(i) for i in range(burst)]
    t0 = time.perf_counter()
    collect([submit(q) for q in bq])
    sat_rate = len(bq) / (time.perf_counter() - t0)
    log(f"serve: saturation {sat_rate:.1f} requests/s")
    # Poisson stream at `load` x saturation.
    lam = load * sat_rate
    arr = rqcgen.poisson_arrivals(lam, n_requests, 6)
    stream = [draw(10000 + i) for i in range(n_requests)]
    tickets = []
    t0 = time.perf_counter()
    for q, ta in zip(stream, arr):
        now = time.perf_counter() - t0
        if ta > now:
            time.sleep(ta - now)
        tickets.append(submit(q))
    res = collect(tickets)
    wall = time.perf_counter() - t0
    st = srv.stats()
    srv.close()
    ok = [r for r in res if r["status"] == 0]
    failed = {}
    for q, r in zip(stream, res):
        if r["status"] != 0:
            key = f"{q[0].n_qubits}q open{len(q[1])} prec{q[3]} status{r['status']}"
            failed[key] = failed.get(key, 0) + 1
    lat = np.array([r["t_done"] - r["t_submit"] for r in ok])
    n_amp = sum(1 << len(q[1]) for q, r in zip(stream, res) if r["status"] == 0)
    return {"requests": n_requests, "completed": len(ok),
            "families_accepted": f"{len(fams)}/{tried}", "circuits": len(pool),
            "saturation_req_s": sat_rate, "offered_req_s": lam, "load": load,
            "amplitudes_per_s": n_amp / wall, "requests_per_s": len(ok) / wall,
            "latency_ms": {"p50": 1000 * float(np.percentile(lat, 50)),
                           "p99": 1000 * float(np.percentile(lat, 99))},
            "max_inflight_seen": st["max_inflight_seen"], "plans_built": st["plans_built"],
            "plans_reused": st["plans_reused"], "peak_bytes": st["peak_bytes"],
            "budget_gb": budget_gb, "failed": failed}


def serve_mode(a):
    """Serving workload: grids 5x5 to 8x8, depths 10-20, 4 circuits per
    family."""
    out = run_serving(a.requests, a.load, a.budget_gb, ((5, 5), (6, 6), (7, 7), (8, 8)),
                      range(10, 21, 2), 4, min(200, a.requests))
    out["mode"] = "serve"
    print(json.dumps(out), flush=True)


def select_share_plan(R, net, bits, a, seed):
    """Share plans for planner seeds seed, seed+1, ... (share-candidates of
    them, in parallel), ranked by the planner's time-like cost; the
    share-probe best are timed in FP32 on 8 of their slices and the fastest
    is returned."""
    import torch
    from concurrent.futures import ThreadPoolExecutor
    seeds = [seed + i for i in range(max(1, a.share_candidates))]

    def make(sd):
        p = R.Plan(net, max_log2_elems=a.share_bound, path_trials=a.share_trials, seed=sd,
                   n_local_sliced=a.share_local, bf16_min_log2=a.share_bf16_min_log2)
        return plan_cost(p), sd, p

    with ThreadPoolExecutor(max(1, min(len(seeds), 16, os.cpu_count() or 1))) as ex:
        ranked = sorted(ex.map(make, seeds), key=lambda x: (x[0], x[1]))[:max(1, a.share_probe)]
    if len(ranked) == 1:
        return ranked[0][2], {"candidates": len(seeds), "chosen_seed": ranked[0][1]}
    times, best, best_t = {}, None, float("inf")
    for i in range(len(ranked)):
        _, sd, p = ranked[i]
        ranked[i] = None
        ids = list(range(min(8, p.info()["n_slices"])))
        p.bind("cuda:0")
        lo, pref = p.workspace_bytes(len(ids), 1, R.F32)
        free, _ = torch.cuda.mem_get_info()
        ws = torch.empty(int(min(pref, max(lo, 0.5 * free))), dtype=torch.uint8, device="cuda:0")
        p.contract(bits, slice_ids=ids, prec=R.F32, workspace=ws)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        p.contract(bits, slice_ids=ids, prec=R.F32, workspace=ws)
        torch.cuda.synchronize()
        times[sd] = 1000.0 * (time.perf_counter() - t1) / len(ids)
        log(f"share plan seed {sd}: {times[sd]:.2f} ms per slice")
        del ws
        if times[sd] < best_t:
            best, best_t = (sd, p), times[sd]
        del p
    return best[1], {"candidates": len(seeds), "probed": len(times),
                     "ms_per_slice_by_seed": {str(k): round(v, 3) for k, v in times.items()},
                     "chosen_seed": best[0]}


def share_mode(a):
    """One GPU's share of a 10x10 (1+20+1) circuit: 2^L slices of a plan
    whose other sliced wires are fixed, every intermediate within the bound.
    FP16 and BF16 each run the whole share as one call (one graph launch of
    every slice); the FP32 baseline runs the same slices in a few calls."""
    import numpy as np
    import torch
    import rqcgen
    import paper_2110_14502_amd as R

    torch.cuda.set_device(0)
    rows = cols = 10
    depth, seed = 20, 4
    n = rows * cols
    circ = rqcgen.grid_rqc(rows, cols, depth, seed)
    bits = rqcgen.random_bits(n, seed)
    t = time.perf_counter()
    net = R.Network(R.Circuit.from_rqcgen(circ), [])
    plan, selection = select_share_plan(R, net, bits, a, seed)
    t_plan = time.perf_counter() - t
    info = plan.info()
    n_sl = info["n_slices"]
    log(f"share plan: {t_plan:.1f}s, log2 flops/slice {math.log2(info['flops_per_slice']):.2f}, "
        f"width {info['max_log2_elems']}, {n_sl} slices, {len(plan.fixed_wires())} fixed, "
        f"{len(plan.pruned_wires())} pruned wires")
    t = time.perf_counter()
    plan.bind("cuda:0")
    torch.cuda.synchronize()
    t_bind = time.perf_counter() - t
    free, _ = torch.cuda.mem_get_info()
    lo, pref = plan.workspace_bytes(n_sl, 1, R.F32)
    ws = torch.empty(int(min(pref, max(lo, a.ws_fraction * free))), dtype=torch.uint8, device="cuda:0")
    share_flops = info["flops_per_slice"] * n_sl + info["flops_per_bitstring"]
    checked = sorted(int(x) for x in np.random.default_rng(seed).choice(n_sl, 32, replace=False))
    res = {"mode": "share", "n_gpus": 1, "data": "synthetic",
           "config": {"workload": f"{rows}x{cols} grid RQC depth 1+{depth}+1, fSim(pi/2,pi/6) ABCDCDAB, "
                                  f"circuit seed {seed}, one bitstring; share of {n_sl} slices "
                                  f"({a.share_local} enumerated sliced wires, "
                                  f"{len(plan.fixed_wires())} fixed), per-slice bound 2^{a.share_bound}",
                      "plan_log2_flops_per_slice": math.log2(info["flops_per_slice"]),
                      "plan_max_log2_elems": info["max_log2_elems"],
                      "plan_seconds": round(t_plan, 2), "bind_seconds": round(t_bind, 2),
                      "plan_selection": selection,
                      "invariant_log2_flops": math.log2(info["flops_invariant"] + 1.0)},
           "unit": "slices/s"}
    vals = {}
    precs = [p for p in ("f32", "f16", "bf16") if p in a.share_precs.split(",")]
    if "f32" not in precs:
        raise SystemExit("share mode needs f32 (the comparison baseline)")
    for prec in precs:
        pc = R.PRECISIONS[prec]
        parts = a.share_f32_parts if prec == "f32" else 1
        # Timed: the product path, each call one graph launch of its slices.
        plan.set_timing(-1)
        per_all = []
        total_ms = 0.0
        reruns = 0
        for part in range(parts):
            ids = list(range(part * n_sl // parts, (part + 1) * n_sl // parts))
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            _, per = plan.contract(bits, slice_ids=ids, per_slice=True, prec=pc, workspace=ws)
            torch.cuda.synchronize()
            ms = 1000 * (time.perf_counter() - t0)
            total_ms += ms
            reruns += plan.last_report["fp32_reruns"]
            per_all.append(R.to_complex(per)[:, 0, 0])
            log(f"share {prec} part {part + 1}/{parts}: {ms / 1000:.1f}s "
                f"(groups of {plan.last_report['slices_per_group']})")
        vals[prec] = np.concatenate(per_all)
        # MFMA rate: the same launches run directly with events around the
        # matrix-core steps, on the first eighth of the slices.
        plan.set_timing(1)
        plan.contract(bits, slice_ids=list(range(max(1, n_sl // 8))), prec=pc, workspace=ws)
        tim = plan.timing()
        log(f"share {prec} MFMA probe: {tim['launches']} launches")
        achieved = tim["flops"] / (tim["total_ms"] / 1000.0) / 1e12 if tim["total_ms"] > 0 else 0.0
        peak = PEAK_MFMA_FP32 if prec == "f32" else PEAK_MFMA_16
        res[prec] = {"seconds": total_ms / 1000, "slices_per_s": n_sl / (total_ms / 1000),
                     "tflops": share_flops / (total_ms / 1000) / 1e12, "calls": parts,
                     "fp32_reruns": reruns,
                     "mfma": {"achieved_tflops": achieved, "peak": peak, "frac": achieved / peak,
                              "launches": tim["launches"],
                              "share_of_flops": tim["flops"] / (info["flops_per_slice"] * max(1, n_sl // 8)
                                                                 + info["flops_per_bitstring"])}}
    plan.set_timing(-1)
    # Per-slice errors in units of the larger of the checked slices' RMS and
    # the natural scale of one slice, 2^-(n+S)/2 (S sliced wires in all).
    n_sliced_all = len(plan.sliced_wires()) + len(plan.fixed_wires())
    natural = 2.0 ** (-(n + n_sliced_all) / 2)
    for prec in [p for p in precs if p != "f32"]:
        ref, got = vals["f32"][checked], vals[prec][checked]
        rms = float(np.sqrt(np.mean(np.abs(ref) ** 2)))
        res[prec]["speedup_vs_f32"] = res["f32"]["seconds"] / res[prec]["seconds"]
        res[prec]["per_slice_error_vs_f32"] = float(np.max(np.abs(got - ref)) / max(rms, natural))
        res[prec]["fidelity_vs_f32"] = _fidelity(got, ref)
    res["slice_scale"] = {"checked_rms": float(np.sqrt(np.mean(np.abs(vals["f32"][checked]) ** 2))),
                          "natural": natural}
    lp_precs = [p for p in precs if p != "f32"] or ["f32"]
    best = max(lp_precs, key=lambda p: res[p]["slices_per_s"])
    res["metric"] = "share slices/s (reduced precision) and contraction TFLOP/s"
    res["value"] = res[best]["slices_per_s"]
    res["dtype"] = best
    res["share_sum_f32"] = [float(vals["f32"].sum().real), float(vals["f32"].sum().imag)]
    res["checked_slices"] = len(checked)
    print(json.dumps(res), flush=True)


def batch_mode(a):
    """A large correlated batch (Appendix A: fix some qubits, exhaust the
    rest): the 6x6 (1+12+1) circuit with qubits 15..35 open, 2^21 amplitudes
    from one sliced contraction, in FP32 and FP16; the linear cross-entropy
    statistics computed on the device; 64 entries checked against the stored
    oracle values."""
    import numpy as np
    import torch
    import rqcgen
    import paper_2110_14502_amd as R
    torch.cuda.set_device(0)
    circ = rqcgen.grid_rqc(6, 6, 12, 2)
    n, n_open = 36, 21
    openq = list(range(n - n_open, n))
    bits = rqcgen.random_bits(n - n_open, 3)
    t = time.perf_counter()
    plan = R.Plan(R.Network(R.Circuit.from_rqcgen(circ), openq), max_log2_elems=28,
                  path_trials=128, seed=1).bind("cuda:0")
    info = plan.info()
    t_plan = time.perf_counter() - t
    flops = info["flops_per_slice"] * info["n_slices"] + info["flops_per_bitstring"]
    pattern = rqcgen.random_bits(15, 4)
    entries = sum(int(b) << i for i, b in enumerate(pattern)) + (np.arange(64) << 15)
    golden = None
    gpath = os.path.join(ROOT, "tests", "golden", "batch6_amplitudes.txt")
    if os.path.exists(gpath):
        golden = read_golden(gpath)[1]
    res = {"mode": "batch", "n_gpus": 1, "data": "synthetic", "unit": "amplitudes/s",
           "config": {"workload": "6x6 grid RQC depth 1+12+1, circuit seed 2, qubits 15..35 open "
                                  "(2^21 amplitudes), qubits 0..14 closed at random_bits(15, 3)",
                      "n_slices": info["n_slices"], "plan_max_log2_elems": info["max_log2_elems"],
                      "plan_log2_flops": math.log2(flops), "plan_seconds": round(t_plan, 2)}}
    for prec in ("f32", "f16"):
        out = plan.contract(bits, prec=R.PRECISIONS[prec])  # warm (graph capture)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(a.reps):
            out = plan.contract(bits, prec=R.PRECISIONS[prec])
        torch.cuda.synchronize()
        secs = (time.perf_counter() - t0) / a.reps
        st = R.batch_xeb(out, n, samples=torch.from_numpy(entries.astype(np.int64)).cuda())
        row = {"seconds": secs, "amplitudes_per_s": (1 << n_open) / secs,
               "tflops": flops / secs / 1e12, "xeb": st,
               "fp32_reruns": plan.last_report["fp32_reruns"]}
        if golden is not None:
            got = R.to_complex(out)[0][entries]
            row["error_vs_oracle_64"] = _norm_err(got, golden, n)
            row["fidelity_vs_oracle_64"] = _fidelity(got, golden)
        res[prec] = row
        log(f"batch {prec}: {secs:.3f} s, xeb ideal-sampling {st['xeb_ideal_sampling']:.4f}")
    res["speedup_f16"] = res["f32"]["seconds"] / res["f16"]["seconds"]
    res["value"] = res["f16"]["amplitudes_per_s"]
    print(json.dumps(res), flush=True)


def copy_mode(a):
    """Plain device copies, reads and writes (calibration of the traffic
    counters and of the achievable HBM rate)."""
    import torch
    out = {"mode": "copy"}
    for gib in (1, 4):
        n = gib << 30
        x = torch.ones(n // 4, dtype=torch.float32, device="cuda")
        y = torch.empty_like(x)
        ms = _events_time(lambda: y.copy_(x), 5)
        out[f"copy_{gib}GiB"] = {"ms": ms, "gbs_read_plus_write": 2 * n / ms / 1e6}
        ms = _events_time(lambda: y.fill_(2.0), 5)
        out[f"fill_{gib}GiB"] = {"ms": ms, "gbs_write": n / ms / 1e6}
        ms = _events_time(lambda: torch.sum(x), 5)
        out[f"sum_{gib}GiB"] = {"ms": ms, "gbs_read": n / ms / 1e6}
        del x, y
    out["bytes_read"] = 1 << 30
    out["bytes_written"] = 1 << 30
    print(json.dumps(out), flush=True)


def main():
    a = parse()
    if a.gpus != 1:
        print(f"bench.py runs on one GPU only; --gpus {a.gpus} is not supported "
              "(the slices would shard across GPUs with one final reduction, not built here)",
              file=sys.stderr)
        sys.exit(2)
    if a.mode == "kernel":
        return kernel_mode(a)
    if a.mode == "steps":
        return steps_mode(a)
    if a.mode == "serve":
        return serve_mode(a)
    if a.mode == "copy":
        return copy_mode(a)
    if a.mode == "share":
        return share_mode(a)
    if a.mode == "batch":
        return batch_mode(a)
    import numpy as np
    import torch
    import rqcgen
    import paper_2110_14502_amd as R

    torch.cuda.set_device(0)
    n = a.rows * a.cols
    circ = rqcgen.grid_rqc(a.rows, a.cols, a.depth, a.seed)
    openq = list(range(n - a.open, n))
    bits = rqcgen.random_bits(n - a.open, a.seed)
    net = R.Network(R.Circuit.from_rqcgen(circ), openq)
    t = time.perf_counter()
    chosen, probe, plan, lp_plan = select_plan(R, net, bits, a)
    t_plan = time.perf_counter() - t
    info = plan.info()
    log(f"plan: {t_plan:.1f}s, log2 flops/slice {math.log2(max(info['flops_per_slice'], 1.0)):.2f}, "
        f"width {info['max_log2_elems']}, {info['n_slices']} slices")
    ids = None
    frac = 1.0
    if a.slices > 0:
        ids = list(range(min(a.slices, info["n_slices"])))
        frac = len(ids) / info["n_slices"]
    plan.bind("cuda:0")
    plan.set_group_limit(a.max_group)
    prec = R.PRECISIONS[a.prec]
    free, _ = torch.cuda.mem_get_info()
    lo, pref = plan.workspace_bytes(len(ids) if ids else 0, 1, prec)
    ws_bytes = int(min(pref, max(lo, a.ws_fraction * free)))
    ws = torch.empty(ws_bytes, dtype=torch.uint8, device="cuda:0")
    out = torch.empty(2 << a.open, dtype=torch.float64, device="cuda:0")
    tune = None
    if a.tune:
        t0 = time.perf_counter()
        tune = plan.autotune(prec, n_ids=len(ids) if ids else 0, workspace=ws,
                             cache_path=a.tune_cache or None)
        tune["seconds"] = round(time.perf_counter() - t0, 2)
        log(f"autotune {a.prec}: {tune}")
    def step(p, tag):
        ts = time.perf_counter()
        plan.contract(bits, slice_ids=ids, prec=p, workspace=ws, out=out, sync=False)
        r = plan.report()
        log(f"{tag}: {time.perf_counter() - ts:.2f}s (groups of {r['slices_per_group']} slices)")
        return r

    # One probe step with every launch bracketed by events (direct launches
    # on the caller's stream; it also warms up): the per-launch table, each
    # kernel kind's time and roofline.  The timed region then brackets the
    # launches of the kind that takes longest.
    step(prec, "warm")
    plan.set_timing(TIME_ALL)
    step(prec, "probe all kernels")
    table, by_kind = launch_table(plan.launch_timings(), prec=a.prec)
    kind_ms = {k: v["ms_per_step"] / frac for k, v in by_kind.items()}
    names = {v: k for k, v in KIND_NAMES.items()}
    dom = names[max(by_kind, key=lambda k: by_kind[k]["ms_per_step"])]
    if a.roofline_kernel >= 0:
        dom = a.roofline_kernel
    plan.set_timing(dom)
    for _ in range(a.warmup):
        step(prec, "warmup")
    torch.cuda.synchronize()
    lat = []
    tim = {"launches": 0, "total_ms": 0.0, "flops": 0.0, "bytes": 0.0}
    t0 = time.perf_counter()
    for _ in range(a.steps):
        ts = time.perf_counter()
        rep = step(prec, "timed")
        lat.append(time.perf_counter() - ts)
        for k, v in plan.timing().items():
            tim[k] += v
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ms = 1000.0 * elapsed / a.steps / frac
    ref_amps = out.clone()
    n_amp = 1 << a.open
    amps_s = n_amp / (ms / 1000.0)
    step_flops = info["flops_per_slice"] * info["n_slices"] + info["flops_per_bitstring"]
    lat = [x / frac for x in lat]
    res = {
        "metric": METRIC,
        "value": amps_s,
        "unit": "amplitudes/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": a.prec,
        "data": "synthetic",
        "config": {
            "workload": f"{a.rows}x{a.cols} grid RQC depth 1+{a.depth}+1, fSim(pi/2,pi/6) ABCDCDAB, "
                        f"{a.sliced} sliced wires ({info['n_slices']} slices), {n_amp} amplitudes "
                        f"({a.open} open qubits), circuit seed {a.seed}",
            "n_slices": info["n_slices"],
            "slices_run": len(ids) if ids else info["n_slices"],
            "slices_per_group": rep["slices_per_group"],
            "plan_log2_flops": math.log2(step_flops),
            "plan_max_log2_elems": info["max_log2_elems"],
            "plan_steps": info["n_steps"],
            "plan_seconds": round(t_plan, 2),
            "plan_selection": probe,
        },
        "tflops": step_flops / (ms / 1000.0) / 1e12,
        "latency_ms": {"p50": 1000 * float(np.percentile(lat, 50)),
                       "p99": 1000 * float(np.percentile(lat, 99))},
        "roofline": roofline(dom, tim, a, step_flops * frac * a.steps, kind_ms,
                             by_kind[KIND_NAMES[dom]].get("traffic_over_algorithmic")),
        "roofline_by_kernel": by_kind,
        "launch_table": table,
        "autotune": tune,
    }
    golden = None
    if (a.rows, a.cols, a.depth, a.seed, a.open, ids) == (6, 6, 14, 2, 6, None) and \
            os.path.exists(GOLDEN_CONFIG2):
        golden = read_golden(GOLDEN_CONFIG2)[1]
        got = R.to_complex(ref_amps.view(-1, 2))
        res["error_vs_oracle"] = _norm_err(got, golden, n)
        res["fidelity_vs_oracle"] = _fidelity(got, golden)
        res["oracle_reference"] = "tests/golden/config2_amplitudes.txt (complex128 oracle)"
    # The same call replayed as one captured graph launch (probe off).
    if a.graph_steps > 0:
        plan.set_timing(-1)
        step(prec, "graph capture")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(a.graph_steps):
            step(prec, "graph")
        torch.cuda.synchronize()
        res["graph_ms_per_step"] = 1000.0 * (time.perf_counter() - t0) / a.graph_steps / frac
    if a.lp_steps > 0 and a.prec == "f32":
        if lp_plan is not None and lp_plan is not plan:
            # The plan autotuned for FP16 (its own workspace).
            plan.set_timing(-1)
            del ws
            lp_plan.bind("cuda:0")
            free, _ = torch.cuda.mem_get_info()
            lo, pref = lp_plan.workspace_bytes(len(ids) if ids else 0, 1, R.F16)
            ws = torch.empty(int(min(pref, max(lo, a.ws_fraction * free))), dtype=torch.uint8,
                             device="cuda:0")
        else:
            lp_plan = plan

        def step16(tag):
            ts = time.perf_counter()
            lp_plan.contract(bits, slice_ids=ids, prec=R.F16, workspace=ws, out=out, sync=False)
            r = lp_plan.report()
            log(f"{tag}: {time.perf_counter() - ts:.2f}s (groups of {r['slices_per_group']} slices)")
            return r

        if a.tune:
            t0 = time.perf_counter()
            tune16 = lp_plan.autotune(R.F16, n_ids=len(ids) if ids else 0, workspace=ws,
                                      cache_path=a.tune_cache or None)
            tune16["seconds"] = round(time.perf_counter() - t0, 2)
            log(f"autotune f16: {tune16}")
        step16("f16 warmup")
        lp_plan.set_timing(TIME_ALL)
        step16("f16 probe all kernels")
        table16, by_kind16 = launch_table(lp_plan.launch_timings(), prec="f16")
        lp_plan.set_timing(-1)
        step16("f16 graph capture")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(a.lp_steps):
            rep16 = step16("f16")
        torch.cuda.synchronize()
        ms16 = 1000.0 * (time.perf_counter() - t0) / a.lp_steps / frac
        lp_amps = R.to_complex(out.view(-1, 2))
        f32_amps = R.to_complex(ref_amps.view(-1, 2))
        res["reduced_precision"] = {
            "dtype": "f16 (16-bit storage of large intermediates, FP16 MFMA, FP32 accumulate)",
            "ms_per_step": ms16, "value": n_amp / (ms16 / 1000.0), "speedup_vs_f32": ms / ms16,
            "plan_seed": probe.get("f16_chosen_seed", chosen),
            "fp32_reruns": rep16["fp32_reruns"],
            "normalized_error_vs_f32": _norm_err(lp_amps, f32_amps, n),
            "fidelity_vs_f32": _fidelity(lp_amps, f32_amps),
            "roofline_by_kernel": by_kind16, "launch_table": table16,
            "autotune": tune16 if a.tune else None}
        if golden is not None:
            res["reduced_precision"]["error_vs_oracle"] = _norm_err(lp_amps, golden, n)
            res["reduced_precision"]["fidelity_vs_oracle"] = _fidelity(lp_amps, golden)
    if a.serve_requests > 0:
        # Serving leg (continuous batching; p50 / p99 latency beside the
        # throughput): 5x5 and 6x6 grids at depths 10-14, 4 circuits each.
        plan.set_timing(-1)
        del ws
        torch.cuda.empty_cache()
        res["serving"] = run_serving(a.serve_requests, 0.8, 64.0, ((5, 5), (6, 6)), (10, 12, 14),
                                     4, 100)
        res["latency_ms"]["serving_p50"] = res["serving"]["latency_ms"]["p50"]
        res["latency_ms"]["serving_p99"] = res["serving"]["latency_ms"]["p99"]
    if a.cpu_seconds > 0:
        log("cpu baseline")
        res["cpu_baseline"] = cpu_baseline(circ, openq, bits, plan, a.cpu_seconds)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
