"""Benchmark of the batched PGA hot path on one MI355X.

    python bench.py [--steps K] [--warmup W] [--workload NAME]

A "step" of this benchmark is one complete batched solve of the workload
(every round: reset, PGA steps, rounding, local search, exact evaluation,
acceptance) on synthetic inputs resident in HBM.  Prints ONE JSON line.

value      = edge updates per second of the whole solve, edge update =
             one stored CSR entry applied to one trajectory in one PGA step
plain      = the same trajectories one at a time (B = 1 kernels, captured
             step loops), whose incumbents must equal the batched ones
roofline   = the dominant kernel (the one that runs the PGA steps),
             algorithmic bytes per launch over its HIP-event launch time
cpu_baseline = the CPU oracle on a bounded sample of the same workload
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK = 8.0e12  # bytes/s, MI355X
# LDS read peak: 256 CUs x 256 bytes/clock x 2.4 GHz.  CDNA 4 doubles the
# LDS read bandwidth of CDNA 3 (128 bytes/clock/CU) along with its size
# (160 KiB); a plain 128-bit LDS read loop over all CUs measured 168
# bytes/clock/CU on MI355X, above the CDNA 3 figure, so 256 is the bound.
LDS_PEAK = 256 * 256 * 2.4e9
KERNEL_SOURCES = {"k_tile_round": "paper_2605_06921_amd/csrc/tile_kernel.hip",
                  "k_pga_step": "paper_2605_06921_amd/csrc/grid_kernels.hip",
                  "k_objective_grad": "paper_2605_06921_amd/csrc/grid_kernels.hip",
                  "k_flip2_best": "paper_2605_06921_amd/csrc/grid_kernels.hip",
                  "k_swap_propose": "paper_2605_06921_amd/csrc/grid_kernels.hip"}
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "hbm_traffic.json")


def source_sha256(path):
    import hashlib
    with open(os.path.join(ROOT, path), "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()


def measured_traffic(workload, kernel, tile=None):
    """HBM bytes per launch of `kernel` on `workload` from the committed
    calibrated FETCH_SIZE / WRITE_SIZE counter runs, or None when there is
    no record, the kernel source changed since the counters were taken, or
    the record was taken on another persistent-plan shape than `tile`."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    rec = json.load(open(TRAFFIC_FILE)).get(workload, {}).get(kernel)
    if not rec or rec.get("source_sha256") != source_sha256(KERNEL_SOURCES[kernel]):
        return None
    if tile is not None and rec.get("tile", tile) != tile:
        return None
    return rec["hbm_bytes_per_launch"]


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def with_measured_rate(res):
    """Beside the algorithmic rate: the measured HBM bytes of the kernel
    (the counters' `traffic`) over the same average launch time."""
    r = res.get("roofline", {})
    if r.get("traffic") and r.get("avg_launch_ms"):
        rate = r["traffic"] / (r["avg_launch_ms"] / 1e3)
        r["measured_rate"] = dict(achieved=rate / 1e9, unit="GB/s", frac=rate / HBM_PEAK,
                                  note="measured HBM bytes per launch over the average launch time")
    return res


def step_bytes(g, B, momentum=False):
    """Compulsory bytes of one PGA step over every graph: the CSR once,
    the iterate read once and written once (and the momentum)."""
    n, nnz = g.n, g.nnz
    b = 4 * (n + g.num_graphs) + 4 * nnz + 8 * n * B
    if g.weight is not None:
        b += 4 * nnz
    if momentum:
        b += 8 * n * B
    return b


def host_cores():
    """Cores this process may run on, capped at the 16 a one-GPU share of
    the machine provides, and the CPU model."""
    n = len(os.sched_getaffinity(0))
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return min(n, 16), n, model


def _oracle_params(wl, rounds, pool_k=0, final_search=False):
    from oracle import solver as osolver
    return osolver.Params(batch=wl.batch, steps_per_round=wl.steps_per_round, rounds=rounds, alpha=wl.alpha,
                          seed=wl.seed, gamma=wl.gamma, lam=wl.lam, rho=wl.rho, reset_mode=wl.reset_mode,
                          local_search=wl.local_search, pool_k=pool_k, final_search=final_search or wl.final_search,
                          mu=wl.momentum, check_every=wl.check_every, init_mode=wl.init_mode,
                          init_sigma=wl.init_sigma)


_WORKER = {}


def _worker_init(name):
    os.environ["OMP_NUM_THREADS"] = "1"
    from synth.workloads import WORKLOADS
    wl = WORKLOADS[name]
    _WORKER["wl"] = wl
    _WORKER["sub"] = wl.make_graph().subgraph(0)


def _worker_run(task):
    """One worker's share: trajectories `cols` of graph 0 for `rounds` rounds."""
    from oracle import solver as osolver
    cols, rounds = task
    wl, sub = _WORKER["wl"], _WORKER["sub"]
    t0 = time.perf_counter()
    osolver.solve_graph(wl.problem, sub, _oracle_params(wl, rounds), 0, cols=np.asarray(cols))
    return time.perf_counter() - t0


def cpu_baseline(wl, g, budget_s=15.0, pool_k=0, final_search=False):
    """The oracle (float32 replay, as used for parity) on a bounded sample of
    the workload, graph 0, run before the GPU is touched.  Independent
    trajectories: one oracle process per host core, each on its own
    trajectories for whole rounds (the pool couples every trajectory of the
    graph: then one process on all of them).  The sample is sized from
    single-process probes to take about budget_s / 2 of wall time."""
    import multiprocessing as mp
    from oracle import solver as osolver

    sub = g.subgraph(0)
    cores, visible, model = host_cores()
    coupled = pool_k > 0
    ncols = wl.batch if coupled else 1
    t0 = time.perf_counter()
    osolver.solve_graph(wl.problem, sub, _oracle_params(wl, 1, pool_k, final_search), 0, cols=np.arange(ncols))
    probe = time.perf_counter() - t0
    rounds = int(min(wl.rounds, max(1, budget_s / 2 // probe)))
    per = 1 if not coupled else wl.batch
    workers = 1 if coupled else min(cores, wl.batch)
    if not coupled:
        # columns per process: grow while one process stays under budget / 4
        while per * 2 * workers <= wl.batch:
            t0 = time.perf_counter()
            osolver.solve_graph(wl.problem, sub, _oracle_params(wl, rounds), 0, cols=np.arange(per))
            if time.perf_counter() - t0 >= budget_s / 4:
                break
            per *= 2
    reps = 1
    if workers == 1:
        def once():
            osolver.solve_graph(wl.problem, sub, _oracle_params(wl, rounds, pool_k, final_search), 0,
                                cols=np.arange(per))
        t0 = time.perf_counter()
        once()
        el = time.perf_counter() - t0
        if el < budget_s / 4:  # a small workload: repeat it to fill the sample
            reps = int(np.ceil(budget_s / 2 / max(el, 1e-4)))
            t0 = time.perf_counter()
            for _ in range(reps):
                once()
            el = time.perf_counter() - t0
        nt = per
    else:
        tasks = [(list(range(w * per, (w + 1) * per)), rounds) for w in range(workers)]
        ctx = mp.get_context("spawn")  # the GPU is not initialised yet
        with ctx.Pool(workers, initializer=_worker_init, initargs=(wl.name,)) as pool:
            pool.map(_worker_run, [([0], 1)] * workers)  # every process up and warm
            t0 = time.perf_counter()
            pool.map(_worker_run, tasks, chunksize=1)
            el = time.perf_counter() - t0
            if el < budget_s / 4:  # a small workload: repeat it to fill the sample
                reps = int(np.ceil(budget_s / 2 / max(el, 1e-4)))
                t0 = time.perf_counter()
                pool.map(_worker_run, tasks * reps, chunksize=1)
                el = time.perf_counter() - t0
        nt = per * workers
    eu = sub.nnz * nt * wl.steps_per_round * rounds * reps
    return dict(value=eu / el, unit="edge-updates/s", cores=workers, kind="oracle",
                cpu_model=model, cores_visible=visible,
                sample=f"graph 0 of {g.num_graphs} (n={sub.n}, nnz={sub.nnz}), trajectories 0..{nt - 1} of "
                       f"{wl.batch}, rounds 1..{rounds} of {wl.rounds} ({wl.steps_per_round} steps each, reset, "
                       f"1-flip search and evaluation included), {reps} time(s), float32 replay in numpy/scipy, "
                       f"{workers} process(es) of one thread each over disjoint trajectories, {el:.1f} s wall")


def pair_cpu_baseline(kind, wl, g, Z0, budget_s):
    """The oracle's pair search on graph 0, from the 1-flip optima that the
    oracle's own 1-flip search makes of the same rounded start (untimed),
    over as many trajectories as fit in about half the budget."""
    from oracle import discrete as odisc
    sub = g.subgraph(0)
    lo, hi = int(g.vtx_offset[0]), int(g.vtx_offset[1])
    ncols = 1
    while True:
        start, _ = odisc.local_search(kind, sub, Z0[lo:hi, :ncols], wl.seed, np.arange(ncols), 0)
        t0 = time.perf_counter()
        odisc.pair_search(kind, sub, start, wl.seed, np.arange(ncols), 0)
        el = time.perf_counter() - t0
        if ncols == wl.batch or el >= budget_s / 2:
            break
        ncols = int(min(wl.batch, max(2 * ncols, ncols * budget_s / 2 / max(el, 1e-3))))
    return dict(value=sub.nnz * ncols / el, unit="edge-trajectories/s", cores=1, kind="oracle",
                sample=f"graph 0 of {g.num_graphs} (n={sub.n}, nnz={sub.nnz}), trajectories 0..{ncols - 1} of "
                       f"{wl.batch}, one complete pair search each from the oracle's own 1-flip optima of the "
                       f"same rounded start, pure-Python loops with numpy, single-threaded, {el:.1f} s")


def plain_sample(G, B, per_graph=32, graphs=8):
    """Trajectory ids of the plain comparison: `per_graph` trajectories spread
    over the batch of each of `graphs` graphs spread over the workload (all
    of them when it is smaller)."""
    gs = np.unique(np.linspace(0, G - 1, min(G, graphs)).round().astype(np.int64))
    bs = np.unique(np.linspace(0, B - 1, min(B, per_graph)).round().astype(np.int64))
    return (gs[:, None] * B + bs[None, :]).ravel()


def same_trajectories(g, B, ids, a, b):
    """Incumbent values and sets of trajectories `ids` equal in both solves."""
    va, vb = a["traj_best_value"].cpu().numpy(), b["traj_best_value"].cpu().numpy()
    if not np.array_equal(va[ids], vb[ids]):
        return False
    xa, xb = a["traj_best_x"].cpu().numpy(), b["traj_best_x"].cpu().numpy()
    for t in ids:
        gi, c = divmod(int(t), B)
        lo, hi = int(g.vtx_offset[gi]), int(g.vtx_offset[gi + 1])
        if not np.array_equal(xa[lo:hi, c], xb[lo:hi, c]):
            return False
    return True


def bench_pair(args, wl):
    """The paper's own search (OneTwoSwap / OneTwoFlip) over the workload's
    batch, started from 1-flip optima (what the search meets after a solve
    with 1-flip search): the rounded uniform iterate of every trajectory
    after the 1-flip search, untimed.  A step is one complete search of every
    trajectory of every graph; value = stored CSR entries x trajectories
    searched per second."""
    import torch
    from synth import arrays
    from paper_2605_06921_amd import mqo

    g = wl.make_graph()
    dev = torch.device("cuda:0")
    dg = mqo.DeviceGraph(g, dev)
    B = wl.batch
    kind = "mis" if wl.problem == "mis" else "maxcut"
    lo, hi = (0.0, 1.0) if kind == "mis" else (-1.0, 1.0)  # the box of h (Eq. (3)) / f_B (Eq. (7))
    X = arrays.uniform((g.n, B), lo, hi, wl.seed)
    Zr = (X > 0.5).astype(np.int8) if kind == "mis" else np.where(X > 0, 1, -1).astype(np.int8)
    Z0 = torch.from_numpy(Zr).to(dev)
    ws = mqo.Workspace(dev)
    mqo.local_search(kind, dg, Z0, wl.seed, 0, workspace=ws)
    Z = torch.empty_like(Z0)
    alt = 0
    for i in range(args.warmup):
        Z.copy_(Z0)
        alt = mqo.pair_search(kind, dg, Z, wl.seed, 0, workspace=ws)
        torch.cuda.synchronize()
        log(f"[bench] pair warmup {i}: {alt} pair iterations")
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0.record()
    cand_ms, launches = 0.0, 0
    for _ in range(args.steps):
        Z.copy_(Z0)
        tm = {}
        alt = mqo.pair_search(kind, dg, Z, wl.seed, 0, workspace=ws, timing=tm)
        cand_ms += tm["candidate_kernel_ms"]
        launches += alt + 1
    e1.record()
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    gpu_s = e0.elapsed_time(e1) / 1e3
    improved = float((Z0 != Z).any(dim=0).float().mean())
    res = dict(metric="CSR entries x trajectories searched per second (OneTwoSwap / OneTwoFlip)",
               value=g.nnz * B * args.steps / el, unit="edge-trajectories/s", n_gpus=1, steps=args.steps,
               warmup=args.warmup, ms_per_step=1e3 * el / args.steps, higher_is_better=True, scaling="weak",
               vs_baseline=None, dtype="int32", data="synthetic",
               config=dict(workload=wl.name, mode="pair", description=wl.description, graphs=g.num_graphs, n=g.n,
                           nnz=g.nnz, batch=B, start="1-flip optima of the rounded uniform iterate",
                           pair_iterations=alt, trajectories_improved=improved, parallelism="dp1"),
               gpu_ms_per_step=1e3 * gpu_s / args.steps)
    # dominant kernel: the candidate launch of every pair iteration.
    # Compulsory bytes: the CSR once, the per-vertex state of every
    # trajectory once (MaxCut: s, t, priority read, best gain / hash /
    # position written; MIS: z and m read (every vertex outside a maximal
    # I neighbours it), the owner array cleared, the proposal pair written)
    csr = 4 * (g.n + 1) + 4 * g.nnz + (4 * g.nnz if g.weight is not None else 0)
    per_launch = csr + (21 if kind == "maxcut" else 17) * g.n * B
    avg_s = cand_ms / 1e3 / max(1, launches)
    kname = "k_flip2_best" if kind == "maxcut" else "k_swap_propose"
    res["roofline"] = dict(bound="hbm", achieved=per_launch / avg_s / 1e9, peak=HBM_PEAK / 1e9, unit="GB/s",
                           frac=per_launch / avg_s / HBM_PEAK, traffic=measured_traffic(f"{wl.name}:pair", kname),
                           kernel=kname if kind == "maxcut" else "k_fill_rows_i32 + k_tight_bits + k_swap_propose",
                           avg_launch_ms=avg_s * 1e3, algorithmic_bytes_per_launch=per_launch,
                           launches=launches)
    if not args.no_cpu_baseline:
        log("[bench] CPU oracle baseline (pair search)")
        res["cpu_baseline"] = pair_cpu_baseline(kind, wl, g, Zr, args.cpu_budget)
    return res


def bench_quality(args, wl):
    """Best value at fixed wall-time budgets: the workload's solve with as
    many rounds as fit in each budget (the outer loop of Alg. 1-4 runs
    while time remains; no round starts after the budget), then its own
    full run of `rounds` rounds.  Each budget is one solve; its best value,
    the rounds run and the wall time are reported."""
    import torch
    from paper_2605_06921_amd import mqo

    g = wl.make_graph()
    dev = torch.device("cuda:0")
    dg = mqo.DeviceGraph(g, dev)
    kw = dict(batch=wl.batch, steps_per_round=wl.steps_per_round, alpha=wl.alpha, gamma=wl.gamma, lam=wl.lam,
              rho=wl.rho, reset_mode=wl.reset_mode, local_search=wl.local_search, seed=wl.seed)
    ws = mqo.Workspace(dev)
    mqo.solve(wl.problem, dg, workspace=ws, rounds=1, **kw)  # tuning and warm-up
    torch.cuda.synchronize()
    runs = []
    for budget in [float(b) for b in args.budgets.split(",") if b] + [None]:
        rounds = wl.rounds if budget is None else 1 << 30
        t0 = time.perf_counter()
        out = mqo.solve(wl.problem, dg, workspace=ws, rounds=rounds, time_budget_s=budget or 0.0, **kw)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        runs.append(dict(budget_s=budget, wall_s=el, rounds=out["rounds_executed"],
                         steps=out["steps_executed"], best_value=int(out["best_value"][0]),
                         edge_updates_per_s=out["edge_updates"] / el, plan=out["plan"]))
        log(f"[bench] quality budget={budget}: best {runs[-1]['best_value']} after {out['rounds_executed']} rounds "
            f"in {el:.1f} s")
    return dict(metric="best MIS size / cut at fixed wall time", value=runs[0]["best_value"],
                unit="MIS size" if wl.problem == "mis" else "cut weight", n_gpus=1, steps=len(runs), warmup=1,
                ms_per_step=1e3 * runs[0]["wall_s"], higher_is_better=True, scaling="weak", vs_baseline=None,
                dtype="f32", data="synthetic",
                config=dict(workload=wl.name, mode="quality", description=wl.description, n=g.n, nnz=g.nnz,
                            batch=wl.batch, steps_per_round=wl.steps_per_round, rho=wl.rho, parallelism="dp1"),
                runs=runs)


def bench_toy(args):
    """Prop. 4.1's toy at n = 64: 2^20 independent trials of the
    single-coordinate global reset for R = ceil(2 log(n / delta)) rounds of n
    attempts (delta = 0.01), 128 descent steps per reset.  A step is one
    launch over every trial; value = reset attempts per second.  The full
    restart comparison runs once, untimed, at n = 12."""
    import math
    import torch
    from paper_2605_06921_amd import mqo

    n, delta, steps, trials = 64, 0.01, 128, 1 << 20
    R = math.ceil(2 * math.log(n / delta))
    m = R * n
    dev = torch.device("cuda:0")
    first = None
    for _ in range(args.warmup):
        first, _ = mqo.toy_reset(11, n, trials, m, steps=steps, device=dev, want_x=False)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record()
    for _ in range(args.steps):
        first, _ = mqo.toy_reset(11, n, trials, m, steps=steps, device=dev, want_x=False)
    e1.record()
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    gpu_s = e0.elapsed_time(e1) / 1e3
    f = first.cpu().numpy()
    rs, _ = mqo.toy_reset(12, 12, 1 << 16, 4096, mode="restart", steps=steps, device=dev)
    rs = rs.cpu().numpy()
    attempts = trials * m * args.steps
    res = dict(metric="reset attempts per second (Prop. 4.1 toy, single-coordinate global reset)",
               value=attempts / el, unit="attempts/s", n_gpus=1, steps=args.steps, warmup=args.warmup,
               ms_per_step=1e3 * el / args.steps, higher_is_better=True, scaling="weak", vs_baseline=None,
               dtype="f32", data="synthetic",
               config=dict(workload="prop41_toy_n64", mode="toy", n=n, trials=trials, rounds=R, attempts=m,
                           descent_steps=steps, alpha=0.5, beta=0.5, parallelism="dp1"),
               result=dict(success_fraction=float((f >= 0).mean()), failure_bound=float(n * math.exp(-R / 2.0)),
                           delta=delta, mean_attempts_to_hit=float(f[f >= 0].mean()),
                           full_restart_n12_success_fraction_within_4096=float((rs >= 0).mean()),
                           full_restart_n12_exact=float(1 - (1 - 2.0 ** -12) ** 4097)))
    # ALU-bound: 5 float32 operations per descent step (the clip is one
    # more instruction, not counted), 128 steps per attempt; Philox and the
    # float64 acceptance test are extra work not counted.  Peak for this
    # mix: every operation is rounded on its own (no fused multiply-add)
    # and packed float32 is not used, so each lane retires one flop per
    # clock: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz.  The published 157.3
    # TFLOP/s counts packed fused multiply-adds (4 flops per lane-clock).
    flops = 5.0 * steps * attempts
    alu_peak = 256 * 64 * 2.4e9
    res["roofline"] = dict(bound="alu", achieved=flops / gpu_s / 1e12, peak=alu_peak / 1e12, unit="TFLOP/s",
                           frac=flops / gpu_s / alu_peak, traffic=None, kernel="k_toy_global_reset",
                           avg_launch_ms=1e3 * gpu_s / args.steps, flops_per_launch=flops / args.steps,
                           published_peak=157.3, frac_of_published=flops / gpu_s / 157.3e12,
                           issue_slots_per_step=6,
                           note="peak = 256 CUs x 64 lanes x 2.4 GHz, one separately rounded float32 "
                                "operation per lane-clock; the clamp takes a sixth issue slot per step")
    if not args.no_cpu_baseline:
        from oracle import toy as otoy
        log("[bench] CPU oracle baseline (toy)")
        T = 256
        t0 = time.perf_counter()
        otoy.global_reset(11, n, T, m, steps=steps)
        cel = time.perf_counter() - t0
        while cel < args.cpu_budget / 2 and T < trials:
            T *= 2
            t0 = time.perf_counter()
            otoy.global_reset(11, n, T, m, steps=steps)
            cel = time.perf_counter() - t0
        res["cpu_baseline"] = dict(value=T * m / cel, unit="attempts/s", cores=1, kind="oracle",
                                   sample=f"trials 0..{T - 1} of {trials}, all {m} attempts each, numpy "
                                          f"vectorised over trials, single-threaded, {cel:.1f} s")
    return res


def bench_differentiation(args, wl):
    """Objective + gradient (grad) or the unrolled adjoint (unrolled) over the
    workload's batch.  EU = one stored CSR entry x one trajectory in one
    sparse-product pass; an unrolled forward + backward of K = 20 steps with
    checkpoints every 5 is 20 + 4 x (4 + 2 x 5) = 76 passes."""
    import torch
    from synth import arrays
    from paper_2605_06921_amd import mqo

    g = wl.make_graph()
    dev = torch.device("cuda:0")
    dg = mqo.DeviceGraph(g, dev)
    B = wl.batch
    param = wl.gamma if wl.problem == "mis" else wl.lam
    lo = 0.0 if wl.problem == "mis" else -1.0
    X = torch.from_numpy(arrays.uniform((g.n, B), lo, 1.0, wl.seed)).to(dev)
    K, c = 20, 5
    if args.mode == "grad":
        passes = 1
        kernel = "k_objective_grad"

        def run():
            return mqo.objective_grad(wl.problem, dg, X, param)
    else:
        passes = K + (K // c) * ((c - 1) + 2 * c)
        kernel = "k_adj_mu"
        dL = torch.ones_like(X)

        def run():
            XK, ckpt = mqo.unrolled_forward(wl.problem, dg, X, wl.alpha, K, c, param)
            return mqo.unrolled_backward(wl.problem, dg, ckpt, dL, wl.alpha, K, c, param)
    for _ in range(args.warmup):
        run()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record()
    for _ in range(args.steps):
        run()
    e1.record()
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    gpu_s = e0.elapsed_time(e1) / 1e3  # the library's launches run on the current stream
    kernel_s = None
    if args.mode == "grad":
        # the backward of the autograd Objective alone: dL/dX = scale_b (c + H x),
        # one launch of the SpMM-gradient kernel per call (no objective
        # partials, no reductions), timed on the same stream
        ones = torch.ones(g.num_graphs * B, dtype=torch.float32, device=dev)
        for _ in range(args.warmup):
            mqo.objective_grad(wl.problem, dg, X, param, scale=ones, want_f=False)
        torch.cuda.synchronize()
        e0.record()
        for _ in range(args.steps):
            mqo.objective_grad(wl.problem, dg, X, param, scale=ones, want_f=False)
        e1.record()
        torch.cuda.synchronize()
        kernel_s = e0.elapsed_time(e1) / 1e3 / args.steps
    eu = g.nnz * B * passes * args.steps
    res = dict(metric="edge-updates/s of the differentiation path; HBM GB/s", value=eu / el, unit="edge-updates/s",
               n_gpus=1, steps=args.steps, warmup=args.warmup, ms_per_step=1e3 * el / args.steps,
               higher_is_better=True, scaling="weak", vs_baseline=None, dtype="f32", data="synthetic",
               config=dict(workload=wl.name, objective=wl.problem, mode=args.mode, description=wl.description, n=g.n, nnz=g.nnz, batch=B,
                           sparse_product_passes=passes, hubs=dg.num_hubs, parallelism="dp1"))
    # algorithmic bytes per pass: CSR once, X read, output written (float64
    # objective partials are small); average over the timed region
    per_pass = step_bytes(g, B)
    if kernel_s is not None:
        achieved = per_pass / kernel_s
        res["roofline"] = dict(bound="hbm", achieved=achieved / 1e9, peak=HBM_PEAK / 1e9, unit="GB/s",
                               frac=achieved / HBM_PEAK, traffic=measured_traffic(wl.name, kernel),
                               kernel=kernel, avg_launch_ms=1e3 * kernel_s, algorithmic_bytes_per_launch=per_pass,
                               call_gpu_ms=1e3 * gpu_s / args.steps,
                               call_frac=per_pass * args.steps / gpu_s / HBM_PEAK,
                               note="avg_launch_ms: HIP events around gradient-only calls (the autograd "
                                    "backward: one k_objective_grad launch each); call_gpu_ms: whole calls "
                                    "with the float64 objective (the kernel with partials + 2 reductions)")
    else:
        achieved = per_pass * passes * args.steps / gpu_s
        res["roofline"] = dict(bound="hbm", achieved=achieved / 1e9, peak=HBM_PEAK / 1e9, unit="GB/s",
                               frac=achieved / HBM_PEAK, traffic=None, kernel=kernel,
                               algorithmic_bytes_per_pass=per_pass, gpu_ms_per_step=1e3 * gpu_s / args.steps,
                               note="HIP-event time of whole calls (every launch of the call, including the "
                                    "float64 reductions), so a lower bound on the sparse-product kernels' rate")
    print(json.dumps(with_measured_rate(res)), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="er_batch_mis")
    ap.add_argument("--plan", default="auto")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=15.0)
    ap.add_argument("--objective", default="", choices=["", "maxcut", "maxcut_fl", "maxcut_fp", "maxcut_fa"],
                    help="MaxCut workloads: the formulation of the steps (default f_B, Eq. (7); f_L, f_P, f_A are "
                         "Eq. (4)-(6))")
    ap.add_argument("--pool", type=int, default=0,
                    help="solve mode: pmQO pool of K solutions per graph (Alg. 3 / 4)")
    ap.add_argument("--final-search", action="store_true",
                    help="solve mode: the paper's own search on the incumbents (or the pool) after the rounds")
    ap.add_argument("--budgets", default="10,60",
                    help="quality mode: wall-time budgets in seconds, comma separated")
    ap.add_argument("--mode", default="solve", choices=["solve", "grad", "unrolled", "pair", "toy", "quality"],
                    help="solve: whole batched solves; grad: objective + SpMM gradient over the batch; "
                         "unrolled: K = 20 unrolled PGA steps forward and their adjoint (checkpoints every 5)")
    ap.add_argument("--tile", default="",
                    help="persistent plan shape T,threads,vec,csr,reg[,sb] (mqo_params tile_* fields; 0 = autotune)")
    ap.add_argument("--copy-calibration-mb", type=int, default=0,
                    help="first run a plain device copy of this many MiB (scale for HBM counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); trajectories are independent, "
              f"so N GPUs would each run B/N of them with no per-step communication", file=sys.stderr)
        sys.exit(2)

    import torch
    from synth.workloads import WORKLOADS
    from paper_2605_06921_amd import mqo

    wl = WORKLOADS[args.workload]
    if args.objective:
        if wl.problem == "mis":
            raise SystemExit("--objective selects a MaxCut formulation; the workload is MIS")
        import dataclasses
        if args.objective != wl.problem:
            # counter records are per workload and formulation
            wl = dataclasses.replace(wl, problem=args.objective, name=f"{wl.name}:{args.objective}")
    if args.copy_calibration_mb:
        # a plain device copy of known size: the scale of the HBM counters
        a = torch.empty(args.copy_calibration_mb << 18, dtype=torch.float32, device="cuda:0").fill_(1.0)
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        log(f"[bench] calibration copy of {args.copy_calibration_mb} MiB done")
        del a, b
    if args.mode == "toy":
        print(json.dumps(bench_toy(args)), flush=True)
        return
    if args.mode == "pair":
        print(json.dumps(with_measured_rate(bench_pair(args, wl))), flush=True)
        return
    if args.mode == "quality":
        print(json.dumps(bench_quality(args, wl)), flush=True)
        return
    if args.mode != "solve":
        return bench_differentiation(args, wl)
    if args.pool or args.final_search:
        import dataclasses
        tag = (f":pool{args.pool}" if args.pool else "") + (":final" if args.final_search else "")
        wl = dataclasses.replace(wl, name=wl.name + tag)
    log(f"[bench] building graph {wl.name}")
    g = wl.make_graph()
    cpu = None
    if not args.no_cpu_baseline:
        # before the GPU is touched: the oracle's worker processes are started fresh
        log("[bench] CPU oracle baseline")
        cpu = cpu_baseline(wl, g, args.cpu_budget, args.pool, args.final_search)
        log(f"[bench] cpu oracle {cpu['value']:.4e} EU/s on {cpu['cores']} cores")
    dev = torch.device("cuda:0")
    dg = mqo.DeviceGraph(g, dev)
    kw = dict(batch=wl.batch, steps_per_round=wl.steps_per_round, rounds=wl.rounds, alpha=wl.alpha, gamma=wl.gamma,
              lam=wl.lam, rho=wl.rho, reset_mode=wl.reset_mode, local_search=wl.local_search, seed=wl.seed,
              pool_k=args.pool, final_search=args.final_search or wl.final_search, momentum=wl.momentum,
              check_every=wl.check_every, init_mode=wl.init_mode, init_sigma=wl.init_sigma)
    if args.tile:
        t = [int(v) for v in args.tile.split(",")]
        kw.update(tile_cols=t[0], tile_threads=t[1], tile_vec=t[2], tile_csr=t[3], tile_reg=t[4])
        if len(t) > 5:
            kw.update(tile_sb=t[5])
    ws = mqo.Workspace(dev)
    for i in range(args.warmup):
        out = mqo.solve(wl.problem, dg, plan=args.plan, workspace=ws, **kw)
        torch.cuda.synchronize()
        log(f"[bench] warmup {i}: plan={out['plan']} T={out['tile_cols']} threads={out['tile_threads']} "
            f"best={out['best_value'][:4].tolist()}")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    eu = 0
    kms, klaunch = 0.0, 0
    for i in range(args.steps):
        out = mqo.solve(wl.problem, dg, plan=args.plan, workspace=ws, **kw)
        eu += out["edge_updates"]
        kms += out["step_kernel_ms"]
        klaunch += out["step_kernel_launches"]
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    value = eu / elapsed
    ms_per_step = 1e3 * elapsed / args.steps
    log(f"[bench] timed {args.steps} solves: {ms_per_step:.3f} ms/solve, {value:.4e} EU/s")

    res = dict(metric="edge-updates/s batched PGA vs plain at equal best MIS size / cut; HBM GB/s",
               value=value, unit="edge-updates/s", n_gpus=1, steps=args.steps, warmup=args.warmup,
               ms_per_step=ms_per_step, higher_is_better=True, scaling="weak", vs_baseline=None, dtype="f32",
               data="synthetic",
               config=dict(workload=wl.name, objective=wl.problem, description=wl.description, graphs=g.num_graphs,
                           n=g.n, nnz=g.nnz,
                           batch=wl.batch, steps_per_round=wl.steps_per_round, rounds=wl.rounds, alpha=wl.alpha,
                           rho=wl.rho, reset_mode=wl.reset_mode, plan=out["plan"], tile_cols=out["tile_cols"],
                           tile_threads=out["tile_threads"], tile_vec=out["tile_vec"],
                           tile_csr_lds=out["tile_csr_lds"], tile_reg_degree=out["tile_reg_degree"],
                           tile_single_buffer=out["tile_sb"], step_vec=out["step_vec"], step_lanes=out["step_lanes"],
                           pool_k=args.pool, final_search=bool(args.final_search or wl.final_search), parallelism="dp1"))

    # dominant kernel: the launches that run the PGA steps
    steps_per_launch = wl.steps_per_round * wl.rounds / max(1, out["step_kernel_launches"])
    per_launch_bytes = step_bytes(g, wl.batch) * steps_per_launch
    avg_launch_s = kms / 1e3 / max(1, klaunch)
    achieved = per_launch_bytes / avg_launch_s
    kernel = "k_tile_round" if out["plan"] == "persistent" else "k_pga_step"
    tile = None
    if out["plan"] == "persistent":
        tile = ",".join(str(out[k]) for k in ("tile_cols", "tile_threads", "tile_vec", "tile_csr_lds",
                                              "tile_reg_degree", "tile_sb"))
    traffic = measured_traffic(wl.name, kernel, tile)
    if out["plan"] == "persistent":
        res["roofline"] = dict(bound="hbm", achieved=achieved / 1e9, peak=HBM_PEAK / 1e9, unit="GB/s",
                               frac=achieved / HBM_PEAK, traffic=traffic, kernel=kernel,
                               avg_launch_ms=avg_launch_s * 1e3, algorithmic_bytes_per_launch=per_launch_bytes,
                               steps_per_launch=steps_per_launch)
    else:
        # a captured step loop is steps_per_launch back-to-back dispatches of
        # the step kernel: report per dispatch (the unit of the counters)
        res["roofline"] = dict(bound="hbm", achieved=achieved / 1e9, peak=HBM_PEAK / 1e9, unit="GB/s",
                               frac=achieved / HBM_PEAK, traffic=traffic, kernel=kernel,
                               avg_launch_ms=avg_launch_s * 1e3 / steps_per_launch,
                               algorithmic_bytes_per_launch=per_launch_bytes / steps_per_launch,
                               graph_launch_ms=avg_launch_s * 1e3, steps_per_graph_launch=steps_per_launch,
                               note="per dispatch of the step kernel: the HIP-event time of each captured "
                                    "step loop over its steps")
    if out["plan"] == "persistent":
        # The persistent kernel keeps the iterate in LDS: its bound is the
        # LDS, where every edge update gathers 4 bytes and every element is
        # read and written once per step.  What a streaming step would move
        # through HBM is kept beside it as the HBM-equivalent rate.
        lds_bytes = (4 * g.nnz * wl.batch + 8 * g.n * wl.batch) * steps_per_launch
        hbm_eq = res["roofline"]
        res["roofline"] = dict(bound="lds", achieved=lds_bytes / avg_launch_s / 1e9, peak=LDS_PEAK / 1e9,
                               unit="GB/s", frac=lds_bytes / avg_launch_s / LDS_PEAK, traffic=traffic, kernel=kernel,
                               avg_launch_ms=avg_launch_s * 1e3, algorithmic_bytes_per_launch=lds_bytes,
                               steps_per_launch=steps_per_launch,
                               note="LDS peak = 256 CUs x 256 bytes/clock x 2.4 GHz (CDNA 4 LDS reads); "
                                    "traffic = measured HBM bytes per launch")
        res["hbm_equivalent"] = dict(rate=hbm_eq["achieved"], unit="GB/s", bytes_per_launch=per_launch_bytes,
                                     note="the bytes a streaming step would move through HBM (CSR once, X read "
                                          "once, X' written once), over the same launch time; the persistent "
                                          "kernel keeps X in LDS, so this is no fraction of an HBM peak")

    if not args.no_plain and args.pool:
        log("[bench] no plain comparison: the pool runs on the batched plan only")
    if not args.no_plain and not args.pool:
        ids = plain_sample(g.num_graphs, wl.batch)
        log(f"[bench] plain per-trajectory solve of {len(ids)} trajectories")
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        pout = mqo.solve(wl.problem, dg, plan="plain", workspace=ws, trajectories=ids, **kw)
        torch.cuda.synchronize()
        pel = time.perf_counter() - t1
        equal = same_trajectories(g, wl.batch, ids, pout, out)
        pval = pout["edge_updates"] / pel
        res["plain"] = dict(value=pval, unit="edge-updates/s", seconds=pel, trajectories=len(ids),
                            graphs=len(np.unique(ids // wl.batch)), equal_best=equal,
                            batched_over_plain=value / pval,
                            note="the same kernels one trajectory at a time (captured step loops), on a sample "
                                 "of the batched run's trajectories; equal_best: their incumbent values and "
                                 "sets are identical to the batched run's")
        log(f"[bench] plain {pval:.4e} EU/s, batched/plain = {value / pval:.1f}x, equal best: {equal}")
        if not equal:
            raise SystemExit("plain and batched incumbents differ")
    res["best_value"] = out["best_value"].cpu().tolist()[:8]
    if cpu is not None:
        res["cpu_baseline"] = cpu
    print(json.dumps(with_measured_rate(res)), flush=True)


if __name__ == "__main__":
    main()
