"""Benchmark: leaf evaluations per second of Batch-BFS search with the BCTS
correction on one MI355X.

Workload (one step = the whole hot path over one batch, inputs resident in
HBM): 256 root states, A = 18 actions, depth 3 (5,832 leaves per root,
1,492,992 per step), gamma = 0.99, correction on with c = 1.0, synthetic sprite
world and a random Kaiming-initialised Nature-DQN.  Each step expands 3
levels, scores every leaf (plus the root and depth-1 nodes the correction
needs), backs up and corrects all 256 roots.

Reported beside the headline (BF16, batched):
  * the FP8 batched form and the plain FP32 form that searches one root per
    launch sequence, at the same shape;
  * root-vector error and root-action agreement against the FP64 oracle (on a
    sample of roots) and against the FP32 GPU path (all 256 roots);
  * per-kernel durations from HIP events on the search stream, the roofline of
    the dominant kernel, p50/p99 step latency;
  * the FP64 oracle timed on the host cores over a bounded sample.

Two further workloads print their own JSON line:
  --workload mixed  1,024 roots with A in {4,6,18} and depth in {1,2,3}
                    (seeded) plus 8 roots at A=6, depth 4, BF16, the whole
                    batch as one captured HIP graph replayed per step;
  --workload serve  Poisson arrivals at 2000 requests/s for 60 s (A in
                    {4,6,18}, depth 1-4), BF16, continuous batching through
                    submit/progress/poll; p50/p99 request latency after a
                    5 s warm-up, plus a run under a 1 GB device budget and
                    one at 20,000 requests/s for 10 s;
  --workload mlp    the learned forward-model world (a fully connected
                    model with three hidden layers of width 100, A = 2 and
                    10): GPU time per search of one root against depth, the
                    FP64 oracle's depth-first search on the host beside it,
                    and the batched throughput of 64 roots;
  --workload beam   pruned search: 64 roots at A=18, depth 4, BF16,
                    exhaustive against beams of 4, 16 and 64 nodes per root
                    action: time per step, leaves scored, and root-action
                    agreement with the exhaustive search;
  --workload copy   a plain 1 GiB device-to-device copy, three times: the
                    calibration run for the HBM byte counters of a profiler.

    python bench.py [--steps K] [--warmup W] [--precision bf16|fp8|fp32]
                    [--workload headline|mixed|serve|mlp|beam|copy]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "leaf evals/sec at A=18,d=3 (BF16/FP8 vs FP32); p50/p99 search latency"
N_ROOTS, A, DEPTH, GAMMA, C = 256, 18, 3, 0.99, 1.0
INSTANCE_SEED, WEIGHT_SEED, CALIB_SEED = 1003, 7, 2003
PEAK_TFLOPS = {"fp32": 157.3, "bf16": 2500.0, "fp8": 5000.0}
HBM_PEAK_GBS = 8000.0
# algorithmic FLOPs per evaluated stack, by layer (2 * rows * N * K)
LAYER_FLOPS = {"conv1": 2 * 400 * 32 * 256, "conv2": 2 * 81 * 64 * 512, "conv3": 2 * 49 * 64 * 576,
               "fc1": 2 * 512 * 3136, "fc2": 2 * A * 512}
LAYER_KERNEL = {"conv1": "layer_kernel<0,P>", "conv2": "layer_kernel<1,P>", "conv3": "layer_kernel<2,P>",
                "fc1": "fc1_kernel<P>", "fc2": "layer_kernel<4,P>", "conv_fused": "conv_fused_kernel<P,T>"}
MIXED_SEED, SERVE_SEED, MLP_SEED = 1004, 1005, 1007
# algorithmic bytes per new node written by the expansion: frame, positions, return, reward
EXPAND_BYTES_PER_NODE = 7056 + 16 + 4 + 1
# committed autotune results (per precision and shape) and FP8 scales
TUNING_FILE = os.path.join(ROOT, "paper_2107_01715_amd", "tuning.json")


def _oracle_root(args):
    """One root of the workload through the FP64 oracle (CPU worker)."""
    r, = args
    from threadpoolctl import threadpool_limits
    from paper_2107_01715_amd import workload as W
    from oracle import qnet as Q, search as S
    with threadpool_limits(1):
        ep = W.env_params(INSTANCE_SEED)
        world = S.World(ep.delta, ep.vel, Q.prepare(W.qnet_weights(WEIGHT_SEED)))
        pos, st = W.roots(INSTANCE_SEED, r + 1)
        res = S.search(world, pos[r], st[r], DEPTH, A, GAMMA, correction=True, c=C)
        return r, res.q, res.action, res.ties


def oracle_pool():
    """A process pool for the oracle, one worker per core (at most 16),
    forked before any GPU use."""
    import multiprocessing as mp
    cores = min(len(os.sched_getaffinity(0)), 16)
    return mp.get_context("fork").Pool(cores), cores


def cpu_baseline(pool, cores, n_sample: int):
    """The oracle as it stands, timed on a bounded sample of roots."""
    t0 = time.perf_counter()
    out = pool.map(_oracle_root, [(r,) for r in range(n_sample)])
    dt = time.perf_counter() - t0
    leaves = n_sample * A ** DEPTH
    return {"value": leaves / dt, "unit": "leaf evals/s", "cores": min(cores, n_sample), "kind": "oracle",
            "sample": f"{n_sample} roots of the A=18,d=3 workload ({leaves} leaves), FP64, "
                      f"{dt:.1f} s wall"}, {r: (q, a, t) for r, q, a, t in out}


def agreement(act, q, ref):
    """Per-root error (|dQ|max / |Q|max) and tie-excused action agreement."""
    import numpy as np
    errs, agree = [], 0
    for r, (qo, ao, ties) in ref.items():
        errs.append(float(np.abs(q[r, :A] - qo).max() / np.abs(qo).max()))
        agree += int(act[r] == ao or act[r] in ties)
    return {"roots": len(ref), "agree": agree, "rate": agree / len(ref),
            "max_rel_err": max(errs), "mean_rel_err": float(np.mean(errs))}


TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "conv_fused_bf16_256roots_A18_d3_traffic.md")
COUNTER_PROFILE = os.path.join(ROOT, "profiles", "conv_fused_fc1_bf16_fp8_256roots_A18_d3_sq_counters.md")


def _profile_value(path, pattern):
    """A figure from a committed counter summary, only while the fused
    kernel's source (and the header that fixes its output layout) is the one
    it was measured on (else None)."""
    import hashlib
    import re
    csrc = os.path.join(ROOT, "paper_2107_01715_amd", "csrc")
    try:
        text = open(path).read()
        src = b"".join(open(os.path.join(csrc, f), "rb").read() for f in ("qnet_fused.hip", "bcts_internal.h"))
    except OSError:
        return None
    m = re.search(pattern, text)
    h = re.search(r"source_sha256 qnet_fused.hip\+bcts_internal.h:\s*([0-9a-f]{64})", text)
    if not m or not h or h.group(1) != hashlib.sha256(src).hexdigest():
        return None
    return float(m.group(1))


EXPAND_PROFILE = os.path.join(ROOT, "profiles", "expand_256roots_A18_d3_traffic.md")


def measured_expand_traffic():
    """HBM bytes per new node of the expansion (FETCH_SIZE + WRITE_SIZE,
    copy-calibrated) while its kernel's source is the one measured."""
    import hashlib
    import re
    try:
        text = open(EXPAND_PROFILE).read()
        src = open(os.path.join(ROOT, "paper_2107_01715_amd", "csrc", "expand.hip"), "rb").read()
    except OSError:
        return None
    m = re.search(r"traffic_bytes_per_node:\s*([0-9.]+)", text)
    h = re.search(r"source_sha256 expand.hip:\s*([0-9a-f]{64})", text)
    if not m or not h or h.group(1) != hashlib.sha256(src).hexdigest():
        return None
    return float(m.group(1))


def measured_traffic(kernel, precision, fused, tuned):
    """HBM bytes per stack of the dominant kernel (FETCH_SIZE + WRITE_SIZE,
    copy-calibrated), for the kernel and round size it was measured on.  The
    per-stack figure does not depend on how the stacks are chunked."""
    if kernel != "conv_fused" or precision != "bf16" or not fused or tuned.get("round") != 3:
        return None
    return _profile_value(TRAFFIC_PROFILE, r"traffic_bytes_per_stack:\s*([0-9.]+)")


def measured_executed_flops(kernel, precision, fused, tuned):
    """Matrix-core FLOP per stack the fused kernel executes (counter
    SQ_INSTS_VALU_MFMA_MOPS_* x 512), for the launch shape it was measured on."""
    if kernel != "conv_fused" or precision not in ("bf16", "fp8") or not fused or tuned.get("round") != 3:
        return None
    if precision == "fp8" and not tuned.get("fp8_k128"):
        return None
    return _profile_value(COUNTER_PROFILE, r"executed_flop_per_stack %s:\s*([0-9.]+)" % precision)


def _setup(seed, n_roots, budget=0):
    """Context with the workload's env, weights and FP8 calibration."""
    from paper_2107_01715_amd import bcts, workload as W
    ep = W.env_params(seed)
    ctx = bcts.Context(0, budget)
    ctx.set_env(ep.delta, ep.vel)
    ctx.set_qnet(W.qnet_blob(W.qnet_weights(WEIGHT_SEED)))
    _, cal = W.roots(CALIB_SEED, 64)
    ctx.calibrate_fp8(cal)
    return ctx


def run_mixed(args):
    """Mixed batch: 1,024 roots (A ~ U{4,6,18}, d ~ U{1,2,3}) + 8 roots at
    A=6, d=4, searched together as one captured HIP graph per step."""
    import numpy as np
    import torch
    from paper_2107_01715_amd import bcts, workload as W
    A_mix, d_mix = W.mixed_shapes(MIXED_SEED, 1024, (4, 6, 18), (1, 2, 3))
    Av = np.concatenate([A_mix, np.full(8, 6, np.int32)]).astype(np.int32)
    dv = np.concatenate([d_mix, np.full(8, 4, np.int32)]).astype(np.int32)
    n = len(Av)
    pos, st = W.roots(MIXED_SEED, n)
    leaves = int((Av.astype(np.int64) ** dv).sum())
    ctx = _setup(MIXED_SEED, n)
    ctx.set_precision({"bf16": bcts.BF16, "fp8": bcts.FP8, "fp32": bcts.FP32}[args.precision])
    dev = torch.device("cuda:0")
    pos_t = torch.from_numpy(pos).to(dev)
    st_t = torch.from_numpy(st).to(dev)
    act_t = torch.zeros(n, dtype=torch.int32, device=dev)
    q_t = torch.zeros(n, 18, dtype=torch.float32, device=dev)        # [n][18] rows (entries >= A are -inf)
    corr = bcts.correction(True, C)
    stream = torch.cuda.Stream()
    tuned = None
    if args.precision != "fp32":
        with torch.cuda.stream(stream):
            tuned = ctx.autotune(pos_t, st_t, dv, Av, GAMMA, corr, act_t, q_t, reps=2, stream=stream)
        torch.cuda.synchronize()
        print(f"# autotune mixed: {tuned}", file=sys.stderr, flush=True)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    with torch.cuda.stream(stream):
        # eager form (one launch sequence per step)
        for _ in range(args.warmup):
            ctx.search_batch_device(pos_t, st_t, dv, Av, GAMMA, corr, act_t, q_t, stream=stream)
        e0.record(stream)
        for _ in range(args.steps):
            ctx.search_batch_device(pos_t, st_t, dv, Av, GAMMA, corr, act_t, q_t, stream=stream)
        e1.record(stream)
        torch.cuda.synchronize()
        eager_ms = e0.elapsed_time(e1) / args.steps
        act_eager, q_eager = act_t.cpu().numpy().copy(), q_t.cpu().numpy().copy()
        # graph form: capture once (warm-up replays), then time `steps` replays
        ctx.search_batch_graph(pos_t, st_t, dv, Av, GAMMA, corr, act_t, q_t, replays=max(args.warmup, 1),
                               stream=stream)
        torch.cuda.synchronize()
        e0.record(stream)
        ctx.search_batch_graph(pos_t, st_t, dv, Av, GAMMA, corr, act_t, q_t, replays=args.steps, stream=stream)
        e1.record(stream)
        torch.cuda.synchronize()
        graph_ms = e0.elapsed_time(e1) / args.steps
    same = bool((act_t.cpu().numpy() == act_eager).all() and (q_t.cpu().numpy() == q_eager).all())
    ctx.close()
    out = {
        "metric": "leaf evals/sec, mixed-shape batch (graph replay)", "value": leaves / (graph_ms * 1e-3),
        "unit": "leaf evals/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": graph_ms,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": {"bf16": "bf16", "fp8": "fp8_e4m3", "fp32": "f32"}[args.precision],
        "data": "synthetic (seeded sprite world, random Kaiming-uniform Nature-DQN)",
        "config": {"workload": "1024 roots, A ~ U{4,6,18}, depth ~ U{1,2,3} + 8 roots A=6 depth 4, gamma 0.99, "
                               "BCTS c=1.0, one captured HIP graph per step", "roots": n,
                   "leaves_per_step": leaves, "precision": args.precision},
        "eager_ms_per_step": eager_ms, "eager_value": leaves / (eager_ms * 1e-3),
        "graph_equals_eager": same, "autotuned": tuned,
    }
    print(json.dumps(out))


def _serve_once(args, budget, duration, warm, rate):
    """Replay the Poisson request stream in real time; returns latency and
    throughput figures over the requests that arrive after `warm` seconds."""
    import numpy as np
    from paper_2107_01715_amd import bcts, workload as W
    t_arr, A_r, d_r = W.request_arrivals(SERVE_SEED, rate, duration)
    n = len(t_arr)
    pool = 4096                                 # distinct root states, cycled over the requests
    pos, st = W.roots(SERVE_SEED, pool)
    ctx = _setup(SERVE_SEED, pool, budget)
    ctx.set_precision({"bf16": bcts.BF16, "fp8": bcts.FP8, "fp32": bcts.FP32}[args.precision])
    corr = bcts.correction(True, C)
    # warm the engine (allocations, first launches) before the clock starts
    for i in range(8):
        tk = ctx.submit(pos[i], st[i], int(d_r[i]), int(A_r[i]), GAMMA, corr)
        while True:
            ctx.progress()
            r = ctx.poll(tk, int(A_r[i]))
            if r is not None:
                break
    lat = np.full(n, np.nan)
    pending = {}
    i = 0
    t0 = time.monotonic()
    max_pending = 0
    while i < n or pending:
        now = time.monotonic() - t0
        while i < n and t_arr[i] <= now:
            k = i % pool
            tk = ctx.submit(pos[k], st[k], int(d_r[i]), int(A_r[i]), GAMMA, corr)
            pending[tk] = i
            i += 1
        left = ctx.progress()                   # requests queued or on the GPU
        max_pending = max(max_pending, len(pending))
        if left < len(pending):                 # some finished: collect them
            for tk in list(pending):
                j = pending[tk]
                r = ctx.poll(tk, int(A_r[j]))
                if r is not None:
                    lat[j] = r[2] - (t0 + t_arr[j])
                    del pending[tk]
    wall = time.monotonic() - t0
    stats = ctx.serve_stats()
    ctx.close()
    sel = t_arr >= warm
    lm = lat[sel] * 1e3
    leaves = (A_r.astype(np.int64) ** d_r)
    return {"requests": int(n), "measured_requests": int(sel.sum()), "wall_s": wall,
            "p50_ms": float(np.percentile(lm, 50)), "p99_ms": float(np.percentile(lm, 99)),
            "mean_ms": float(lm.mean()), "max_ms": float(lm.max()),
            "requests_per_s": float(n / wall), "leaf_evals_per_s": float(leaves.sum() / wall),
            "max_pending": int(max_pending), "cohorts": stats["cohorts_done"],
            "requests_per_cohort": float(n / max(stats["cohorts_done"], 1)),
            "budget_bytes": budget if budget else "80% of free device memory"}


def run_serve(args):
    rate, duration, warm = 2000.0, args.serve_seconds, min(5.0, args.serve_seconds / 4)
    main_run = _serve_once(args, 0, duration, warm, rate)
    print(f"# serve (default budget): {main_run}", file=sys.stderr, flush=True)
    small = _serve_once(args, 1 << 30, min(duration, 20.0), min(warm, 5.0), rate)
    print(f"# serve (1 GB budget): {small}", file=sys.stderr, flush=True)
    # ten times the arrival rate, where batching and admission bind
    heavy = _serve_once(args, 0, min(duration, 10.0), min(warm, 2.0), 10 * rate)
    heavy["offered_requests_per_s"] = 10 * rate
    print(f"# serve (10x rate): {heavy}", file=sys.stderr, flush=True)
    out = {
        "metric": "serving request latency p50/p99 (Poisson 2000 req/s)", "value": main_run["p99_ms"],
        "unit": "ms (p99)", "n_gpus": 1, "steps": main_run["requests"], "warmup": 0,
        "ms_per_step": main_run["mean_ms"], "higher_is_better": False, "scaling": "weak", "vs_baseline": None,
        "dtype": {"bf16": "bf16", "fp8": "fp8_e4m3", "fp32": "f32"}[args.precision],
        "data": "synthetic (seeded sprite world, random Kaiming-uniform Nature-DQN)",
        "config": {"workload": f"Poisson arrivals 2000 req/s for {duration:g} s; A ~ U{{4,6,18}}, depth 1-4 "
                               "(p .50/.30/.15/.05, A=18 caps at 3); gamma 0.99, BCTS c=1.0; latency = completion "
                               f"- arrival after a {warm:g} s warm-up", "precision": args.precision},
        "serve": main_run, "serve_1gb_budget": small, "serve_10x_rate": heavy,
    }
    print(json.dumps(out))


def _oracle_mlp_time(A, d, budget_s):
    """Host time of one depth-first search of the FP64 oracle (one root),
    averaged over as many roots as fit the budget (at least one)."""
    import numpy as np
    from paper_2107_01715_amd import workload as W
    from oracle import mlp as M
    w = M.prepare(W.mlp_weights(WEIGHT_SEED, A))
    st = W.mlp_states(MLP_SEED, 16).astype(np.float64)
    t0, k = time.perf_counter(), 0
    while True:
        M.search(w, st[k % 16], d, A, GAMMA, correction=True, c=C)
        k += 1
        if time.perf_counter() - t0 > budget_s or k >= 16:
            break
    return (time.perf_counter() - t0) / k, k


def run_mlp(args):
    """Forward-model world: time per search (one root, as one action
    selection) against depth on the GPU, with the oracle's DFS on the host
    beside it for the depths it finishes, and the batched throughput."""
    import numpy as np
    import torch
    from paper_2107_01715_amd import bcts, workload as W
    dev = torch.device("cuda:0")
    stream = torch.cuda.Stream()
    corr = bcts.correction(True, C)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    rows, batched, crossover = [], {}, []
    cpu_rows = []
    for A, dmax in ((2, 14), (10, 6)):
        ctx = bcts.Context(0)
        ctx.set_mlp(A, W.mlp_blob(W.mlp_weights(WEIGHT_SEED, A), A))
        st = torch.from_numpy(W.mlp_states(MLP_SEED, 64)).to(dev)
        act = torch.zeros(64, dtype=torch.int32, device=dev)
        q = torch.zeros(64, A, dtype=torch.float32, device=dev)
        with torch.cuda.stream(stream):
            for d in range(1, dmax + 1):
                reps = 50 if A ** d < 10 ** 5 else 10
                for _ in range(3):
                    ctx.mlp_search_device(st[:1], d, GAMMA, corr, act[:1], q[:1], stream=stream)
                e0.record(stream)
                for i in range(reps):
                    ctx.mlp_search_device(st[i % 64:i % 64 + 1], d, GAMMA, corr, act[:1], q[:1], stream=stream)
                e1.record(stream)
                torch.cuda.synchronize()
                ms = e0.elapsed_time(e1) / reps
                rows.append({"A": A, "depth": d, "leaves": A ** d, "gpu_ms_per_search": ms,
                             "gpu_leaf_evals_per_s": A ** d / (ms * 1e-3)})
            # batched: 64 roots at the deepest depth
            d = dmax - 1 if A == 10 else dmax
            for _ in range(2):
                ctx.mlp_search_device(st, d, GAMMA, corr, act, q, stream=stream)
            e0.record(stream)
            for _ in range(args.steps):
                ctx.mlp_search_device(st, d, GAMMA, corr, act, q, stream=stream)
            e1.record(stream)
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / args.steps
            batched[A] = {"roots": 64, "depth": d, "leaves": 64 * A ** d, "ms_per_step": ms,
                          "leaf_evals_per_s": 64 * A ** d / (ms * 1e-3)}
        # CPU-to-GPU cross-over (Sec. 4.1): host-buffer searches of one root
        # (the state starts on the host, the result returns to it), levels
        # 1..k on the CPU and the rest on the GPU, against depth
        st_h = W.mlp_states(MLP_SEED, 64)
        for d in range(1, min(dmax, 8 if A == 2 else 5) + 1):
            row = {"A": A, "depth": d}
            ks = list(range(0, min(d - 1, 3) + 1))
            for k in ks:
                ctx.set_tuning(bcts.TUNE_MLP_CROSSOVER, k)
                for i in range(3):
                    ctx.mlp_search(st_h[i:i + 1], d, A, GAMMA, corr)
            # every search timed alone, the cross-over depths taken in turn;
            # the median per depth (a host hiccup moves one search, not it)
            reps = 40 if A ** d < 10 ** 4 else 10
            samples = {k: [] for k in ks}
            for i in range(reps):
                for k in ks:
                    ctx.set_tuning(bcts.TUNE_MLP_CROSSOVER, k)
                    t0 = time.perf_counter()
                    ctx.mlp_search(st_h[i % 64:i % 64 + 1], d, A, GAMMA, corr)
                    samples[k].append(time.perf_counter() - t0)
            for k in ks:
                row[f"host_levels_{k}_ms"] = float(np.median(samples[k])) * 1e3
            ctx.set_tuning(bcts.TUNE_MLP_CROSSOVER, 0)
            times = {k: v for k, v in row.items() if k.startswith("host_levels_")}
            row["best_crossover_depth"] = int(min(times, key=times.get).split("_")[2])
            # the whole search on the host CPU (the paper's CPU BFS), one core
            ctx.set_tuning(bcts.TUNE_MLP_HOST, 1)
            cpu = []
            for i in range(reps if A ** d < 10 ** 4 else 3):
                t0 = time.perf_counter()
                ctx.mlp_search(st_h[i % 64:i % 64 + 1], d, A, GAMMA, corr)
                cpu.append(time.perf_counter() - t0)
            ctx.set_tuning(bcts.TUNE_MLP_HOST, 0)
            row["cpu_bfs_ms"] = float(np.median(cpu)) * 1e3
            row["fastest"] = ("cpu_bfs" if row["cpu_bfs_ms"] < min(times.values())
                              else f"host_levels_{row['best_crossover_depth']}")
            crossover.append(row)
        ctx.close()
        print(f"# mlp A={A}: {[(r['depth'], round(r['gpu_ms_per_search'], 4)) for r in rows if r['A'] == A]}",
              file=sys.stderr, flush=True)
        print(f"# mlp A={A} cross-over: {[r for r in crossover if r['A'] == A]}", file=sys.stderr, flush=True)
    if args.cpu_sample > 0:
        for A, dmax in ((2, 10), (10, 4)):
            for d in range(1, dmax + 1):
                sec, k = _oracle_mlp_time(A, d, 2.0)
                cpu_rows.append({"A": A, "depth": d, "oracle_dfs_ms_per_search": sec * 1e3, "roots_timed": k})
    head = batched[10]
    out = {
        "metric": "leaf evals/sec, learned forward-model world (A=10, 64 roots)", "value": head["leaf_evals_per_s"],
        "unit": "leaf evals/s", "n_gpus": 1, "steps": args.steps, "warmup": 2, "ms_per_step": head["ms_per_step"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic (random fully connected forward model, uniform +-1/sqrt(fan_in))",
        "config": {"workload": f"64 root states, A=10, depth {head['depth']}, gamma 0.99, BCTS c=1.0; per-search "
                               "times: one root per search, A in {2, 10}, depth 1..14 / 1..6"},
        "batched": batched, "per_search": rows,
        "crossover": {"rows": crossover,
                      "what": "median ms per host-buffer search of one root (state in, action and root vector "
                              "out, PCIe included) with levels 1..k expanded on the host CPU and the rest on the "
                              "GPU; best_crossover_depth = the fastest k; cpu_bfs_ms = the whole search on one "
                              "host core (the CPU BFS, the same bits); fastest = the fastest of all"},
        "cpu_baseline": {"kind": "oracle", "cores": 1, "rows": cpu_rows,
                         "sample": "FP64 depth-first search of one root on one host core, averaged over up to "
                                   "16 roots within 2 s per depth"} if cpu_rows else None,
    }
    print(json.dumps(out))


def run_beam(args):
    """Pruned search against the exhaustive one at A=18, depth 4 (64 roots)."""
    import numpy as np
    import torch
    from paper_2107_01715_amd import bcts, workload as W
    n, A_, d = 64, 18, 4
    pos, st = W.roots(INSTANCE_SEED, n)
    ctx = _setup(INSTANCE_SEED, n)
    ctx.set_precision({"bf16": bcts.BF16, "fp8": bcts.FP8, "fp32": bcts.FP32}[args.precision])
    dev = torch.device("cuda:0")
    pos_t, st_t = torch.from_numpy(pos).to(dev), torch.from_numpy(st).to(dev)
    act_t = torch.zeros(n, dtype=torch.int32, device=dev)
    q_t = torch.zeros(n, 18, dtype=torch.float32, device=dev)
    dv, Av = np.full(n, d, np.int32), np.full(n, A_, np.int32)
    corr = bcts.correction(True, C)
    stream = torch.cuda.Stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    rows, ref = [], None
    for beam in (0, 64, 16, 4):
        ctx.set_beam(beam)
        with torch.cuda.stream(stream):
            for _ in range(2):
                ctx.search_batch_device(pos_t, st_t, dv, Av, GAMMA, corr, act_t, q_t, stream=stream)
            e0.record(stream)
            for _ in range(args.steps):
                ctx.search_batch_device(pos_t, st_t, dv, Av, GAMMA, corr, act_t, q_t, stream=stream)
            e1.record(stream)
            torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / args.steps
        act, q = act_t.cpu().numpy().copy(), q_t.cpu().numpy().copy()
        if beam == 0:
            ref = (act, q)
        per_a0 = 1
        for k in range(2, d):
            per_a0 = per_a0 * A_ if beam == 0 or per_a0 * A_ <= beam else beam
        leaves = n * A_ * per_a0 * A_
        agree = int((act == ref[0]).sum())
        rows.append({"beam": beam, "ms_per_step": ms, "leaves_scored": leaves,
                     "leaf_evals_per_s": leaves / (ms * 1e-3), "root_action_agreement": agree / n,
                     "max_root_q_drop": float((ref[1][:, :A_] - q[:, :A_]).max())})
        print(f"# beam {beam}: {ms:.2f} ms, {leaves} leaves, agreement {agree}/{n}", file=sys.stderr, flush=True)
    ctx.set_beam(0)
    ctx.close()
    b16 = [r for r in rows if r["beam"] == 16][0]
    out = {
        "metric": "pruned search time per step (A=18, depth 4, beam 16 per root action)", "value": b16["ms_per_step"],
        "unit": "ms", "n_gpus": 1, "steps": args.steps, "warmup": 2, "ms_per_step": b16["ms_per_step"],
        "higher_is_better": False, "scaling": "weak", "vs_baseline": None,
        "dtype": {"bf16": "bf16", "fp8": "fp8_e4m3", "fp32": "f32"}[args.precision],
        "data": "synthetic (seeded sprite world, random Kaiming-uniform Nature-DQN)",
        "config": {"workload": "64 roots, A=18, depth 4, gamma 0.99, BCTS c=1.0; beams 0 (exhaustive), 64, 16, 4 "
                               "nodes per root action at levels 2-3", "precision": args.precision},
        "beams": rows,
    }
    print(json.dumps(out))


def run_copy(args):
    """Calibration for HBM byte counters: 3 copies of 1 GiB (read 1 GiB,
    write 1 GiB each)."""
    import torch
    nbytes = 1 << 30
    src = torch.empty(nbytes, dtype=torch.uint8, device="cuda:0").fill_(1)
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(3):
        dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / 3
    print(json.dumps({"metric": "device copy bandwidth (counter calibration)", "value": 2 * nbytes / (ms * 1e-3) / 1e9,
                      "unit": "GB/s", "n_gpus": 1, "steps": 3, "warmup": 0, "ms_per_step": ms,
                      "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u8",
                      "data": "synthetic", "config": {"workload": "copy of 1 GiB, 3 times", "bytes": nbytes}}))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--precision", default="bf16", choices=["bf16", "fp8", "fp32"])
    ap.add_argument("--cpu-sample", type=int, default=64, help="roots timed through the oracle (0 = skip)")
    ap.add_argument("--oracle-all", type=int, default=1,
                    help="1 = also run the oracle (untimed) on the remaining roots, for agreement over all 256")
    ap.add_argument("--skip-fp32-single", action="store_true")
    ap.add_argument("--tune-cache", default=os.environ.get("BCTS_TUNE_CACHE", TUNING_FILE),
                    help="autotune results and FP8 scales (JSON); read unless --retune")
    ap.add_argument("--retune", action="store_true", help="autotune and calibrate again, write --tune-out")
    ap.add_argument("--tune-out", default=None, help="where --retune writes (default: --tune-cache)")
    ap.add_argument("--workload", default="headline", choices=["headline", "mixed", "serve", "mlp", "beam", "copy"])
    ap.add_argument("--serve-seconds", type=float, default=60.0)
    ap.add_argument("--quick", action="store_true",
                    help="headline precision only (no comparison forms, no accuracy): for profiler runs")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU: --gpus {args.gpus} is not supported (the search shards over roots "
              f"with no communication; see DESIGN.md for the multi-GPU layout)", file=sys.stderr)
        sys.exit(2)
    if args.workload == "mixed":
        return run_mixed(args)
    if args.workload == "serve":
        return run_serve(args)
    if args.workload == "mlp":
        return run_mlp(args)
    if args.workload == "beam":
        return run_beam(args)
    if args.workload == "copy":
        return run_copy(args)

    # CPU baseline first: the worker pool forks before the GPU is touched; it
    # stays open to run the oracle over the remaining roots (untimed) after
    # the GPU measurements
    cpu, oracle_ref, pool = None, {}, None
    if args.cpu_sample > 0 or args.oracle_all:
        pool, cores = oracle_pool()
    if args.cpu_sample > 0:
        cpu, oracle_ref = cpu_baseline(pool, cores, args.cpu_sample)
        print(f"# cpu baseline: {cpu['value']:.1f} leaf evals/s on {cpu['cores']} cores", file=sys.stderr, flush=True)

    import numpy as np
    import torch
    from paper_2107_01715_amd import bcts, workload as W

    ep = W.env_params(INSTANCE_SEED)
    pos, st = W.roots(INSTANCE_SEED, N_ROOTS)
    _, cal = W.roots(CALIB_SEED, 64)
    ctx = bcts.Context(0)
    ctx.set_env(ep.delta, ep.vel)
    ctx.set_qnet(W.qnet_blob(W.qnet_weights(WEIGHT_SEED)))
    cache = {}
    try:
        cache = json.load(open(args.tune_cache))
    except (OSError, ValueError):
        pass
    if "fp8_scales" in cache and not args.retune:
        ctx.set_fp8_scales(np.asarray(cache["fp8_scales"], np.float32))
    else:
        ctx.calibrate_fp8(cal)
        cache["fp8_scales"] = [float(v) for v in ctx.get_fp8_scales()]
    corr = bcts.correction(True, C)
    dev = torch.device("cuda:0")
    pos_t = torch.from_numpy(pos).to(dev)
    st_t = torch.from_numpy(st).to(dev)
    act_t = torch.zeros(N_ROOTS, dtype=torch.int32, device=dev)
    q_t = torch.zeros(N_ROOTS, 18, dtype=torch.float32, device=dev)
    depth = np.full(N_ROOTS, DEPTH, np.int32)
    Av = np.full(N_ROOTS, A, np.int32)
    stream = torch.cuda.Stream()
    leaves = N_ROOTS * A ** DEPTH
    prec_id = {"fp32": bcts.FP32, "bf16": bcts.BF16, "fp8": bcts.FP8}

    def batched(prec, steps, warmup, timed=True):
        set_prec(prec)
        with torch.cuda.stream(stream):
            for _ in range(warmup):
                ctx.search_batch_device(pos_t, st_t, depth, Av, GAMMA, corr, act_t, q_t, stream=stream)
            torch.cuda.synchronize()
            ctx.set_timing(timed)
            per_step, kern = [], np.zeros(24)
            t0 = time.perf_counter()
            for _ in range(steps):
                ctx.search_batch_device(pos_t, st_t, depth, Av, GAMMA, corr, act_t, q_t, stream=stream)
                if timed:
                    tm = ctx.get_timing()
                    per_step.append(tm[3])
                    kern += tm
            torch.cuda.synchronize()
            wall = time.perf_counter() - t0
            ctx.set_timing(False)
        return wall, per_step, kern / max(steps, 1), act_t.cpu().numpy().copy(), q_t.cpu().numpy().copy()

    # autotune the Q-network launch shape per precision (cached by shape)
    tuned_all = {}
    for prec in ((args.precision,) if args.quick else ("bf16", "fp8")):
        if prec == "fp32":
            continue
        ctx.set_precision(prec_id[prec])
        key = f"{prec}:{N_ROOTS}x{A}^{DEPTH}"
        if key in cache and not args.retune:
            best = cache[key]
            ctx.set_tuning(bcts.TUNE_FUSED, best["fused"])
            ctx.set_tuning(bcts.TUNE_FUSED_ROUND, best["round"])
            ctx.set_tuning(bcts.TUNE_FUSED_CHUNK, best["chunk"])
            ctx.set_tuning(bcts.TUNE_FP8_K128, best.get("fp8_k128", 1))
        else:
            with torch.cuda.stream(stream):
                best = ctx.autotune(pos_t, st_t, depth, Av, GAMMA, corr, act_t, q_t, reps=2, stream=stream)
            torch.cuda.synchronize()
            cache[key] = {k: int(best[k]) for k in ("fused", "round", "chunk", "fp8_k128")}
            cache[key]["us_per_search"] = best.get("us_per_search")
        tuned_all[prec] = {k: best.get(k, 1) for k in ("fused", "round", "chunk", "fp8_k128")}
        tuned_all[prec]["us_per_search"] = best.get("us_per_search")
        print(f"# autotune {prec}: {best}", file=sys.stderr, flush=True)
    tuned = tuned_all.get(args.precision, {})
    if args.retune:
        try:
            with open(args.tune_out or args.tune_cache, "w") as f:
                json.dump(cache, f, indent=1, sort_keys=True)
        except OSError as e:
            print(f"# could not write the tuning file: {e}", file=sys.stderr)

    def set_prec(prec):
        ctx.set_precision(prec_id[prec])
        if prec in tuned_all:
            t = tuned_all[prec]
            ctx.set_tuning(bcts.TUNE_FUSED, t["fused"])
            ctx.set_tuning(bcts.TUNE_FUSED_ROUND, t["round"])
            ctx.set_tuning(bcts.TUNE_FUSED_CHUNK, t["chunk"])
            ctx.set_tuning(bcts.TUNE_FP8_K128, t["fp8_k128"])

    print(f"# {args.precision} batched: warmup {args.warmup}, {args.steps} timed steps", file=sys.stderr, flush=True)
    # per-kernel HIP-event timing (each step waits for its events) ...
    wall_ev, per_step, kern, act_main, q_main = batched(args.precision, args.steps, args.warmup)
    # ... and the headline: the same steps back to back, the host planning
    # step i+1 while the device runs step i; synchronised before and after
    wall, _, _, act_bb, q_bb = batched(args.precision, args.steps, 1, timed=False)
    assert np.array_equal(act_bb, act_main) and np.array_equal(q_bb, q_main)
    ms_step = wall / args.steps * 1e3
    value = leaves / (wall / args.steps)

    results = {args.precision: (value, act_main, q_main, kern, per_step)}
    for prec in (() if args.quick else ("bf16", "fp8", "fp32")):
        if prec in results:
            continue
        if prec == "fp32":
            w2, ps2, k2, a2, q2 = batched(prec, 1, 1)
            results[prec] = (leaves / w2, a2, q2, k2, ps2)
        else:
            w2, ps2, k2, a2, q2 = batched(prec, max(3, args.steps // 2), 1)
            results[prec] = (leaves / (w2 / max(3, args.steps // 2)), a2, q2, k2, ps2)
        print(f"# {prec} batched: {results[prec][0]:.4g} leaf evals/s", file=sys.stderr, flush=True)

    # the plain form: FP32, one root per launch sequence
    single = None
    if not args.skip_fp32_single and not args.quick:
        ctx.set_precision(bcts.FP32)
        one_d, one_a = depth[:1], Av[:1]
        with torch.cuda.stream(stream):
            ctx.search_batch_device(pos_t[:1], st_t[:1], one_d, one_a, GAMMA, corr, act_t[:1], q_t[:1], stream=stream)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for r in range(N_ROOTS):
                ctx.search_batch_device(pos_t[r:r + 1], st_t[r:r + 1], one_d, one_a, GAMMA, corr,
                                        act_t[r:r + 1], q_t[r:r + 1], stream=stream)
            torch.cuda.synchronize()
            w1 = time.perf_counter() - t0
        single = {"value": leaves / w1, "ms_per_pass": w1 * 1e3, "dtype": "f32",
                  "form": "one root per launch sequence, 256 sequential searches"}
        print(f"# fp32 single-root: {single['value']:.4g} leaf evals/s", file=sys.stderr, flush=True)

    # the host-buffer entry point: root positions and stacks (7.2 MB) copied in
    # and the root vectors copied out inside every step (PCIe included); a
    # reported form, never the headline value
    host_form = None
    if not args.quick:
        set_prec(args.precision)
        ctx.search(pos, st, DEPTH, A, GAMMA, corr)                       # warm-up
        hsteps = 3
        t0 = time.perf_counter()
        for _ in range(hsteps):
            ha, hq = ctx.search(pos, st, DEPTH, A, GAMMA, corr)
        hw = (time.perf_counter() - t0) / hsteps
        host_form = {"value": leaves / hw, "unit": "leaf evals/s", "ms_per_step": hw * 1e3,
                     "form": "bcts_search with host buffers, inputs copied in and results out every step",
                     "same_results_as_device_form": bool(np.array_equal(ha, act_main) and
                                                         np.array_equal(hq, q_main[:, :A]))}
        print(f"# {args.precision} host buffers: {host_form['value']:.4g} leaf evals/s", file=sys.stderr, flush=True)

    # the oracle on the roots the timed sample left out (untimed): agreement
    # over all 256 roots
    if pool is not None and args.oracle_all and not args.quick:
        rest = [(r,) for r in range(N_ROOTS) if r not in oracle_ref]
        t0 = time.perf_counter()
        for r, q_, a_, t_ in pool.map(_oracle_root, rest):
            oracle_ref[r] = (q_, a_, t_)
        print(f"# oracle on {len(rest)} more roots: {time.perf_counter() - t0:.1f} s", file=sys.stderr, flush=True)
    if pool is not None:
        pool.close()
        pool.join()

    # accuracy: vs FP64 oracle, vs FP32 GPU path on all roots
    accuracy = {}
    if "fp32" not in results:
        results["fp32"] = results[args.precision]
    a32, q32 = results["fp32"][1], results["fp32"][2]
    gpu32_ref = {}
    for r in range(N_ROOTS):
        qq = q32[r, :A].astype(np.float64)
        m = qq.max()
        ties = [int(i) for i in np.flatnonzero(qq >= m - 1e-6 * max(1.0, abs(m)))]
        gpu32_ref[r] = (qq, int(a32[r]), ties)
    for prec in (() if args.quick else ("fp32", "bf16", "fp8")):
        _, a_, q_, _, _ = results[prec]
        accuracy[prec] = {}
        if oracle_ref:
            accuracy[prec]["vs_fp64_oracle"] = agreement(a_, q_, oracle_ref)
        if prec != "fp32":
            accuracy[prec]["vs_fp32_gpu"] = agreement(a_, q_, gpu32_ref)

    # per-kernel roofline of the headline precision; on the fused path the
    # root and depth-1 evaluations of the correction run in FP32 beside the
    # chunks, so the chunks' kernels see the leaves only
    n_items = kern[16]
    fused = kern[18] > 0.5
    main_items = n_items - N_ROOTS * (A + 1) if fused and kern[19] > 0 else n_items
    names = ("conv_fused", None, None, "fc1", "fc2") if fused else ("conv1", "conv2", "conv3", "fc1", "fc2")
    flops_of = dict(LAYER_FLOPS)
    flops_of["conv_fused"] = LAYER_FLOPS["conv1"] + LAYER_FLOPS["conv2"] + LAYER_FLOPS["conv3"]
    kernels = {}
    for i, name in enumerate(names):
        if name is None:
            continue
        ms = kern[4 + i]
        launches = kern[9]
        flops = flops_of[name] * main_items
        kernels[name] = {"ms_per_step": ms, "launches": launches, "avg_launch_ms": ms / max(launches, 1),
                         "tflops": flops / (ms * 1e-3) / 1e12 if ms > 0 else None,
                         "algorithmic_flop_per_stack": flops_of[name]}
        if name == "fc2" and fused:
            kernels[name]["note"] = ("fc2's matrix work runs in fc1's epilogue (BCTS_TUNE_FC2_FOLDED); this is the "
                                     "kernel that adds its two halves and writes V and the q0 rows")
        if name == "conv1" and kern[20] > 0 and kern[20] == launches and ms > 0:
            # every chunk's conv1 ran by sibling groups: the 6 stages of the
            # shared channels once per group of A, 2 per stack (of 8)
            ex = flops_of["conv1"] * (6.0 / A + 2.0) / 8.0
            kernels[name]["executed_flop_per_stack"] = ex
            kernels[name]["executed_tflops"] = ex * main_items / (ms * 1e-3) / 1e12
            kernels[name]["note"] = ("conv1 by sibling groups: channels 0..2 summed once per group, so the "
                                     "algorithmic rate (every stack's full conv1) can exceed the FP32 peak")
    dom = max(kernels, key=lambda k: kernels[k]["ms_per_step"])
    ach = kernels[dom]["tflops"]
    peak = PEAK_TFLOPS[args.precision]
    exp_nodes = kern[17]
    exp_ms = kern[0]
    exp_gbs = exp_nodes * EXPAND_BYTES_PER_NODE / (exp_ms * 1e-3) / 1e9 if exp_ms > 0 else None
    qnet_tflops = leaves * sum(LAYER_FLOPS.values()) / (kern[1] * 1e-3) / 1e12 if kern[1] > 0 else None
    per_stack = measured_traffic(dom, args.precision, fused, tuned)
    traffic = per_stack * main_items / max(kern[9], 1) if per_stack is not None else None
    ex_stack = measured_executed_flops(dom, args.precision, fused, tuned)
    ex_tflops = (ex_stack * main_items / (kernels[dom]["ms_per_step"] * 1e-3) / 1e12
                 if ex_stack is not None and kernels[dom]["ms_per_step"] > 0 else None)
    roofline = {"bound": "mfma", "kernel": LAYER_KERNEL[dom].replace("P", args.precision).replace("T", str(tuned.get("round", ""))),
                "layer": dom, "achieved": ach, "peak": peak, "unit": "TFLOP/s", "frac": ach / peak,
                "flop_per_launch": flops_of[dom] * main_items / max(kern[9], 1),
                "avg_launch_ms": kernels[dom]["avg_launch_ms"], "traffic": traffic,
                "traffic_unit": "bytes per launch (HBM, rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
                "achieved_is": "algorithmic FLOP (the three plain convolutions per stack) / HIP-event kernel time",
                "executed": ({"achieved": ex_tflops, "frac": ex_tflops / peak, "flop_per_stack": ex_stack,
                              "what": "matrix-core FLOP the kernel executes (rocprofv3 SQ_INSTS_VALU_MFMA_MOPS x 512: "
                                      "conv1 shared by siblings, padded rows) / the same kernel time"}
                             if ex_tflops is not None else None)}

    lat = np.array(per_step) if per_step else np.array([ms_step])
    out = {
        "metric": METRIC, "value": value, "unit": "leaf evals/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_step, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": {"bf16": "bf16", "fp8": "fp8_e4m3", "fp32": "f32"}[args.precision],
        "data": "synthetic (seeded sprite world, random Kaiming-uniform Nature-DQN)",
        "config": {"workload": "256 roots, A=18, depth 3 (5832 leaves/root), gamma 0.99, BCTS c=1.0, "
                               "all roots in one batched launch sequence", "roots": N_ROOTS, "A": A,
                   "depth": DEPTH, "leaves_per_step": leaves, "q_evals_per_step": int(n_items),
                   "precision": args.precision},
        "latency_ms": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99)),
                       "what": "whole-batch search latency per step (HIP events)"},
        "ms_per_step_event_timed": wall_ev / args.steps * 1e3,
        "timing": "value and ms_per_step: steps back to back (the host plans the next step while the device runs "
                  "the current one), synchronised before and after; kernel times and latency: a second pass whose "
                  "every step waits for its HIP events",
        "precisions": {p: {"value": results[p][0]} for p in results},
        "fp32_single_root": single,
        "host_buffers": host_form,
        "speedup_vs_fp32_single_root": (value / single["value"]) if single else None,
        "accuracy": accuracy,
        "autotuned": tuned_all,
        "stages_ms": {"expand": kern[0], "qnet": kern[1], "backup_correct": kern[2], "total": kern[3]},
        "kernels": kernels,
        "qnet_stage_tflops": qnet_tflops,
        "expand": {"bound": "hbm", "achieved": exp_gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                   "frac": exp_gbs / HBM_PEAK_GBS if exp_gbs else None, "nodes": exp_nodes,
                   "bytes_per_node": EXPAND_BYTES_PER_NODE,
                   "traffic_bytes_per_node": measured_expand_traffic(),
                   "achieved_is": "algorithmic bytes per node x new nodes / HIP-event time of the three launches; "
                                  "traffic_bytes_per_node from rocprofv3 FETCH_SIZE + WRITE_SIZE"},
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    ctx.close()
    print(json.dumps(out))


if __name__ == "__main__":
    main()
