"""Benchmark: round-synchronous speculative colouring on one MI355X.

    python bench.py [--steps K] [--warmup W] [--workload NAME] [--gpus 1]

A step is one whole colouring (every round: speculate, detect/commit, until
no vertex is left) of the workload's graph through the C ABI (gc_color),
with the CSR already resident in HBM.  Prints one JSON line.

value        GTEPS = m / t_step (m = undirected edges, each counted once)
roofline     the dominant round kernel (speculate or detect, by measured
             time): algorithmic bytes of its launches / their total time
             measured with HIP events around each launch in a second timed
             region, against 8 TB/s HBM
cpu_baseline the oracle (plain single-thread C) on the same graph
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "GTEPS + vertices colored/s vs HBM roofline; colors used; batched p99 latency"


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=50)
    p.add_argument("--warmup", type=int, default=3)
    p.add_argument("--workload", default="er_1m_16m")
    p.add_argument("--mode", default="graph")
    p.add_argument("--algorithm", default="auto",
                   choices=["auto", "pull", "push", "seq", "blocks"],
                   help="seq: the sequential First-Fit colouring computed in rounds; "
                        "blocks: Algorithm 1 read literally with the recorded number of "
                        "blocks (p = 16384)")
    p.add_argument("--lanes", type=int, default=0,
                   help="fixed lanes per light vertex (turns the autotuner off)")
    p.add_argument("--no-autotune", action="store_true",
                   help="keep the library's automatic settings instead of tuning them "
                        "(untimed) on the workload first")
    p.add_argument("--tune-budget", type=float, default=20.0)
    p.add_argument("--order", default="natural", choices=["natural", "largest_first", "random"],
                   help="vertex order (relabelled on the device, seed 0 for random); "
                        "checked against the oracle's colouring in that order")
    p.add_argument("--rounds-per-step", type=int, default=4,
                   help="served path: rounds each server step advances every resident job")
    p.add_argument("--batch-only", action="store_true",
                   help="batched workload: time the one-launch batch only (no per-graph "
                        "or served comparison); for profiling runs")
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--copy-calibration", action="store_true",
                   help="only run a plain 1 GiB device copy three times (scales the "
                        "FETCH_SIZE / WRITE_SIZE counters to bytes)")
    return p.parse_args()


def copy_calibration():
    import torch
    nbytes = 1 << 30
    src = torch.randint(0, 255, (nbytes,), dtype=torch.uint8, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read": nbytes, "copy_bytes_written": nbytes, "copies": 3}))


def kernel_source_hash():
    """Hash of the kernel sources and of the engine that picks their launch
    shape; a committed counter summary is used only while it matches."""
    h = hashlib.sha256()
    for f in ("gc_kernels.hip", "gc_batch.hip", "gc_device.h", "gc_internal.h", "gc_api.hip"):
        with open(os.path.join(ROOT, "paper_1509_08267_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(workload, kernel):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 PMC
    summary (``key: value`` lines), if it was taken on the current kernel
    source."""
    path = os.path.join(ROOT, "profiles", f"{kernel}_{workload}_pmc.txt")
    if not os.path.exists(path):
        return None
    rec = {}
    with open(path) as f:
        for line in f:
            if ":" in line and not line.startswith((" ", "#", "|")):
                k, v = line.split(":", 1)
                rec[k.strip()] = v.strip()
    if rec.get("kernel_source_sha") != kernel_source_hash():
        return None
    return int(rec["bytes_per_launch"]) if "bytes_per_launch" in rec else None


def main():
    args = parse()
    if args.copy_calibration:
        copy_calibration()
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}); the colouring of "
              "one graph is not sharded across GPUs by this library", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    import graphgen
    from paper_1509_08267_amd import gc

    with open(os.path.join(ROOT, "tests", "golden", "workloads.json")) as f:
        golden = json.load(f)[args.workload]
    if args.workload == "er_batch_4096":
        return run_batch(args, golden)
    g = graphgen.workload(args.workload)
    if g.sha256() != golden["input_sha256"]:
        raise SystemExit("generated input does not match the recorded workload")
    rp64 = g.nnz > 2**31 - 1 or args.workload == "rmat22_ef16"
    dev = torch.device("cuda:0")
    rp = torch.from_numpy(g.rowptr.astype(np.int64 if rp64 else np.int32)).to(dev)
    ci = torch.from_numpy(g.colidx).to(dev)
    out = torch.empty(g.n, dtype=torch.int32, device=dev)

    extra = {"partitions": golden["blocks_p"]} if args.algorithm == "blocks" else {}
    G = gc.Graph(rp, ci, mode=args.mode, algorithm=args.algorithm, lanes=args.lanes, **extra)
    if args.order != "natural":
        if args.algorithm not in ("auto", "push", "pull"):
            raise SystemExit("--order is recorded for the speculative colouring only")
        G.set("order", args.order)
    tuned = None
    # (the p-block colouring has none of the tuned knobs but the grid)
    if not args.no_autotune and args.lanes == 0 and args.algorithm != "blocks":
        from paper_1509_08267_amd import autotune
        res = autotune.tune(G, budget_s=args.tune_budget)
        tuned = dict(res.setting, cached=res.cached, measurements=len(res.table),
                     ms_start=None if res.cached else round(res.baseline_seconds * 1e3, 4),
                     ms_best=round(res.seconds * 1e3, 4))
    t0 = time.perf_counter()
    G.color(out)
    rounds, ncolors = G.stats()
    t_first = time.perf_counter() - t0
    for _ in range(args.warmup):
        G.color(out)
    G.stats()
    got = hashlib.sha256(out.cpu().numpy().astype(np.int32).tobytes()).hexdigest()
    if args.algorithm == "seq":
        parity = got == golden["seq_colors_sha256"] and rounds == golden["seq_rounds"]
    elif args.algorithm == "blocks":
        parity = got == golden["blocks_colors_sha256"] and rounds == golden["blocks_rounds"]
    elif args.order != "natural":
        parity = (got == golden[f"order_{args.order}_colors_sha256"]
                  and rounds == golden[f"order_{args.order}_rounds"])
    else:
        parity = got == golden["colors_sha256"] and rounds == golden["rounds"]

    # timed region 1: the library's default path, K back-to-back colourings
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        G.color(out)
    G.stats()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0

    # timed region 2: the same K colourings with a HIP event around every
    # kernel on the launch stream (rounds launched directly, not as a graph)
    G.set("profile", 1)
    G.color(out)
    G.stats()
    G.profile(reset=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        G.color(out)
    G.stats()
    torch.cuda.synchronize()
    elapsed_prof = time.perf_counter() - t0
    prof = G.profile()
    G.set("profile", 0)
    sbytes = G.get(gc.GC_OPT_STATE_BYTES)
    algo = {gc.GC_ALGO_PUSH: "push", gc.GC_ALGO_PULL: "pull", gc.GC_ALGO_SEQ: "seq",
            gc.GC_ALGO_BLOCKS: "blocks"}[G.get(gc.GC_OPT_ALGORITHM)]
    lanes = G.get(gc.GC_OPT_LANES)
    G_medium = G.get(gc.GC_OPT_MEDIUM_DEGREE)
    G_heavy = G.get(gc.GC_OPT_HEAVY_DEGREE)
    G_bpc = G.get(gc.GC_OPT_BLOCKS_PER_CU)
    G.close()

    t_step = elapsed / args.steps
    gteps = g.m / t_step / 1e9

    # Algorithmic bytes per colouring of the two round kernels (rounds 2..R;
    # round 1 has its own kernel).  Units come from the oracle's per-round
    # totals recorded for this workload (tests/golden/workloads.json):
    #   speculate, pull: per neighbour visit a 4-byte colidx entry and one
    #     state gather; per uncoloured vertex its rowptr pair, its own state
    #     read and the tentative-colour write;
    #   speculate, push: per uncoloured vertex its 32 flag bytes, state read
    #     and write;
    #   detect: per lower neighbour the early-stopping scan must visit, a
    #     colidx entry and a state gather; per uncoloured vertex the rowptr
    #     pair and state read/write; with push, the row entries of a vertex
    #     made final that may still need a push are read with one state read
    #     each, plus one flag byte per entry whose neighbour is still
    #     uncoloured.  With sorted rows the scan and the pushes need not
    #     revisit the leading run of lower neighbours already final (the
    #     oracle-derived lower bounds "*_skip*"); otherwise whole prefixes
    #     and whole rows are counted.
    rp_b = 8 if rp64 else 4
    verts2 = golden["sum_active"] - g.n
    visits2 = golden["sum_active_deg"] - g.nnz
    skip = bool(golden.get("rows_sorted")) and "sum_active_scan_skip" in golden
    if skip:
        scan2 = golden["sum_active_scan_skip"]
        push_rows = golden["push_rows_skip_after_round1"]
    else:
        # round 1 (every tentative colour 0) stops each scan at the first
        # lower neighbour: one entry per vertex that has one, i.e. |U_2|
        sizes = golden["round_sizes"]
        scan2 = golden["sum_active_scan"] - (sizes[1] if len(sizes) > 1 else 0)
        push_rows = golden["push_rows_after_round1"]
    per_vertex = 2 * rp_b + 2 * sbytes
    if algo == "push":
        spec_bytes = verts2 * (32 + 2 * sbytes)
    else:
        spec_bytes = visits2 * (4 + sbytes) + verts2 * per_vertex
    det_bytes = scan2 * (4 + sbytes) + verts2 * per_vertex
    if algo == "push":
        det_bytes += push_rows * (4 + sbytes) \
            + golden["push_useful_after_round1"]
    if algo == "seq":
        # pick (speculate kernel), rounds 2..R: per visit the rowptr pair and
        # the vertex's state; per waiting visit at least one lower-neighbour
        # entry and its state; per vertex coloured, its row once (entry +
        # state gather) and the state write.  Commit (detect kernel): per
        # visit a state read, per vertex coloured a state write.
        sv = golden["seq_visits_after_round1"]
        sc = golden["seq_coloured_after_round1"]
        spec_bytes = (sv * (2 * rp_b + sbytes) + golden["seq_waiting_visits_after_round1"]
                      * (4 + sbytes) + golden["seq_rows_after_round1"] * (4 + sbytes)
                      + sc * sbytes)
        det_bytes = sv * sbytes + sc * sbytes
    # rounds whose kernels are timed per colouring (round 1 has its own launch
    # except in the p-block colouring)
    timed_rounds = rounds if algo == "blocks" else rounds - 1
    if algo == "blocks":
        # phase 1 ("speculate"): per pending vertex its rowptr pair, todo byte
        # and colour write, per row entry the neighbour id and its slot or
        # colour; phase 2 ("detect"): the same reads, per entry also the slot
        # write (entries whose neighbour is in another block: all but ~0.2%
        # at p = 16384), per pending vertex the todo write
        sa, sd = golden["blocks_sum_active"], golden["blocks_sum_active_deg"]
        spec_bytes = sd * 8 + sa * (2 * rp_b + 1 + 4)
        det_bytes = sd * 12 + sa * (2 * rp_b + 1 + 4 + 1)
    spec_ms, spec_launches = prof["speculate"]
    det_ms, det_launches = prof["detect"]
    kernel = "detect" if det_ms > spec_ms else "speculate"
    k_ms, k_launches, k_bytes = ((det_ms, det_launches, det_bytes) if kernel == "detect"
                                 else (spec_ms, spec_launches, spec_bytes))
    calls = max(1, k_launches // max(1, timed_rounds))
    achieved = k_bytes * calls / (k_ms / 1e3) / 1e9 if k_ms > 0 else None
    traffic = measured_traffic(args.workload, kernel)
    roofline = {
        "kernel": ({"speculate": "k_blk_phase1", "detect": "k_blk_phase2"}[kernel]
                   if algo == "blocks" else kernel),
        "bound": "hbm",
        "achieved": round(achieved, 1) if achieved else None,
        "peak": HBM_PEAK_GBS,
        "unit": "GB/s",
        "frac": round(achieved / HBM_PEAK_GBS, 4) if achieved else None,
        "traffic": traffic,
        "alg_bytes_per_launch": k_bytes // max(1, timed_rounds),
        "avg_launch_us": round(k_ms * 1e3 / max(1, k_launches), 2),
        "launches": k_launches,
        "other_kernel": {"kernel": "speculate" if kernel == "detect" else "detect",
                         "achieved": round((spec_bytes if kernel == "detect" else det_bytes) * calls
                                           / ((spec_ms if kernel == "detect" else det_ms) / 1e3)
                                           / 1e9, 1) if min(spec_ms, det_ms) > 0 else None},
    }
    if traffic:
        # bytes the counters saw per launch over the measured launch time
        roofline["traffic_gbs"] = round(traffic / (k_ms / 1e3 / max(1, k_launches)) / 1e9, 1)
        roofline["traffic_frac"] = round(roofline["traffic_gbs"] / HBM_PEAK_GBS, 4)
    kernels_ms_per_step = {k: round(v[0] / max(1, calls), 4) for k, v in prof.items()}
    # The whole colouring priced with the pull-based per-unit byte figures
    # (8 B per neighbour visit in speculate and per lower-neighbour visit in
    # detect, plus per uncoloured vertex two rowptr pairs, worklist and state
    # bytes), i.e. what a pull implementation of the same rounds must move,
    # over the timed step.
    pull_bytes = (8 * golden["sum_active_deg"] + 8 * golden["sum_active_lower_deg"]
                  + golden["sum_active"] * (2 * (4 + 2 * rp_b + 4) + 4))
    step_roofline = None if algo in ("seq", "blocks") else {"definition": "pull-equivalent bytes per colouring",
                     "bytes": pull_bytes,
                     "achieved": round(pull_bytes / t_step / 1e9, 1), "unit": "GB/s",
                     "peak": HBM_PEAK_GBS,
                     "frac": round(pull_bytes / t_step / 1e9 / HBM_PEAK_GBS, 4)}

    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        ts = []
        budget = 20.0
        tstart = time.perf_counter()
        while len(ts) < 3 and (time.perf_counter() - tstart) < budget:
            t = time.perf_counter()
            if algo == "seq":
                oracle.seq(g.rowptr, g.colidx)
            elif algo == "blocks":
                oracle.blocks(g.rowptr, g.colidx, golden["blocks_p"])
            elif args.order != "natural":
                from oracle import ordering
                ordering.colour_in_order(g.rowptr, g.colidx, args.order, 0,
                                         lambda rp_, ci_: oracle.rsc(rp_, ci_).colors)
            else:
                oracle.rsc(g.rowptr, g.colidx)
            ts.append(time.perf_counter() - t)
        tb = min(ts)
        cpu = {"value": round(g.m / tb / 1e9, 5), "unit": "GTEPS", "cores": 1, "kind": "oracle",
               "sample": f"whole {args.workload} graph, oracle "
                         f"{algo if algo in ('seq', 'blocks') else 'rsc'}"
                         f"{'' if args.order == 'natural' else ' after relabelling in the ' + args.order + ' order (numpy)'}"
                         f", best of {len(ts)} single-thread runs "
                         f"({tb:.2f} s each)",
               "seconds": round(tb, 3)}

    rec = {
        "metric": METRIC,
        "value": round(gteps, 3),
        "unit": "GTEPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(t_step * 1e3, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic",
        "config": {"workload": args.workload, "n": g.n, "m": g.m, "nnz": g.nnz, "seed": 0,
                   "mode": args.mode, "algorithm": algo, "lanes": lanes, "state_bytes": sbytes,
                   "medium_degree": G_medium, "heavy_degree": G_heavy,
                   "blocks_per_cu": G_bpc, "autotuned": tuned, "order": args.order},
        "vertices_per_s": round(g.n / t_step, 1),
        "colors": ncolors,
        "colors_seq": golden.get("seq_num_colors"),
        "rounds_seq": golden.get("seq_rounds"),
        "partitions": golden["blocks_p"] if algo == "blocks" else None,
        "rounds": rounds,
        "parity_vs_oracle": parity,
        "first_call_ms": round(t_first * 1e3, 3),
        "profiled_ms_per_step": round(elapsed_prof / args.steps * 1e3, 4),
        "kernel_ms_per_step": kernels_ms_per_step,
        # the byte counts are those of the natural order
        "roofline": roofline if args.order == "natural" else None,
        "step_roofline_pull_equivalent": step_roofline if args.order == "natural" else None,
        "cpu_baseline": cpu,
    }
    print(json.dumps(rec), flush=True)


def run_batch(args, golden):
    """The batched workload: 4,096 independent ER graphs.

    value        GTEPS of one gc_color_batch launch over the whole batch
                 (CSR resident in HBM), summed edges / time
    per-graph    the same graphs coloured one gc_color call each
    served       the continuous-batching server fed the graphs as requests
                 staged on the device, burst and Poisson arrivals
    """
    import numpy as np
    import torch

    import graphgen
    from paper_1509_08267_amd import gc, serve

    b = graphgen.workload(args.workload)
    if b.sha256() != golden["input_sha256"]:
        raise SystemExit("generated input does not match the recorded workload")
    G = b.num_graphs
    dev = torch.device("cuda:0")
    d = lambda a, dt: torch.from_numpy(np.ascontiguousarray(a, dtype=dt)).to(dev)
    voff, eoff = d(b.voff, np.int64), d(b.eoff, np.int64)
    rpl, cil = d(b.rowptr_local, np.int32), d(b.colidx_local, np.int32)
    m = int(b.eoff[-1]) // 2
    n = int(b.voff[-1])
    nbytes = gc.gc_batch_workspace_bytes(G, b.voff, b.eoff)
    ws = torch.empty(nbytes, dtype=torch.uint8, device=dev)
    colors = torch.empty(n, dtype=torch.int32, device=dev)
    rounds = torch.empty(G, dtype=torch.int32, device=dev)

    def launch():
        gc.gc_color_batch(G, voff, eoff, rpl, cil, colors, rounds, ws, nbytes)

    for _ in range(max(1, args.warmup)):
        launch()
    torch.cuda.synchronize()
    parity = (hashlib.sha256(colors.cpu().numpy().astype(np.int32).tobytes()).hexdigest()
              == golden["colors_sha256"]
              and hashlib.sha256(rounds.cpu().numpy().astype(np.int64).tobytes()).hexdigest()
              == golden["rounds_sha256"])
    start, end = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    steps = max(1, args.steps // 5)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    start.record()
    for _ in range(steps):
        launch()
    end.record()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    kernel_ms = start.elapsed_time(end) / steps
    t_step = elapsed / steps

    t_pergraph = None
    served = None
    if args.batch_only:
        return batch_record(args, golden, b, G, m, n, t_step, kernel_ms, steps, parity,
                            t_pergraph, served)

    # per-graph path on the same graphs (handles made untimed, rounds known)
    handles = []
    for gi in range(G):
        a0, a1 = int(b.voff[gi]) + gi, int(b.voff[gi + 1]) + gi + 1
        e0, e1 = int(b.eoff[gi]), int(b.eoff[gi + 1])
        H = gc.Graph(rpl[a0:a1], cil[e0:e1] if e1 > e0 else cil[:1])
        out = colors[int(b.voff[gi]):int(b.voff[gi + 1])]
        H.color(out)
        H.stats()
        handles.append((H, out))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for H, out in handles:
        H.color(out)
    for H, _ in handles:
        H.stats()
    torch.cuda.synchronize()
    t_pergraph = time.perf_counter() - t0
    for H, _ in handles:
        H.close()

    # served: requests staged on the device, burst and Poisson arrivals
    class Req:
        def __init__(self, gi):
            a0, a1 = int(b.voff[gi]) + gi, int(b.voff[gi + 1]) + gi + 1
            self.rowptr = rpl[a0:a1]
            self.colidx = cil[int(b.eoff[gi]):int(b.eoff[gi + 1])]

    reqs = [Req(gi) for gi in range(G)]
    K = args.rounds_per_step
    srv = serve.Server(budget_bytes=12 << 30, max_slots=G, rounds_per_step=K, keep_colors=False)
    t0 = time.perf_counter()
    jobs = srv.serve(reqs, np.zeros(G))
    burst_rate = G / (time.perf_counter() - t0)
    served = {"requests": "device-staged CSR, copied into the server arena on admission",
              "rounds_per_step": K, "burst_graphs_per_s": round(burst_rate, 1),
              "burst": serve.latency_summary(jobs), "poisson": []}
    for frac in (0.5, 0.8, 0.95):
        lam = frac * burst_rate
        arr = graphgen.poisson_arrivals(G, lam, seed=1)
        srv = serve.Server(budget_bytes=12 << 30, max_slots=G, rounds_per_step=K,
                           keep_colors=False)
        t0 = time.perf_counter()
        jobs = srv.serve(reqs, arr)
        dt = time.perf_counter() - t0
        rec = {"load": frac, "rate_per_s": round(lam, 1), "achieved_per_s": round(G / dt, 1)}
        rec.update({k: round(v, 3) for k, v in serve.latency_summary(jobs).items()})
        served["poisson"].append(rec)
    return batch_record(args, golden, b, G, m, n, t_step, kernel_ms, steps, parity,
                        t_pergraph, served)


def batch_record(args, golden, b, G, m, n, t_step, kernel_ms, steps, parity, t_pergraph, served):

    # HBM roofline of the batch kernel: colidx entries the rounds read
    # (speculate: every neighbour of every uncoloured vertex of rounds >= 2;
    # detect: the lower-id prefix, an upper bound because the scan stops at
    # the first conflict) plus each uncoloured vertex's rowptr pair; the
    # state is in LDS and is not HBM traffic.
    alg = 4 * (golden["sum_active_deg"] - int(b.eoff[-1]) + golden["sum_active_lower_deg"]) \
        + 8 * golden["sum_active"]
    achieved = alg / (kernel_ms / 1e3) / 1e9
    traffic = measured_traffic(args.workload, "batch")
    roofline = {"kernel": "gc_color_batch (k_batch_color)", "bound": "hbm",
                "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                "alg_bytes_per_launch": alg, "avg_launch_us": round(kernel_ms * 1e3, 1),
                "launches": steps}
    if traffic:
        roofline["traffic_gbs"] = round(traffic / (kernel_ms / 1e3) / 1e9, 1)
        roofline["traffic_frac"] = round(roofline["traffic_gbs"] / HBM_PEAK_GBS, 4)
    rec = {
        "metric": METRIC,
        "value": round(m / t_step / 1e9, 3),
        "unit": "GTEPS",
        "n_gpus": 1,
        "steps": steps,
        "warmup": args.warmup,
        "ms_per_step": round(t_step * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic",
        "config": {"workload": args.workload, "graphs": G, "n": n, "m": m, "nnz": int(b.eoff[-1]),
                   "seed": 0},
        "graphs_per_s": round(G / t_step, 1),
        "vertices_per_s": round(n / t_step, 1),
        "parity_vs_oracle": parity,
        "colors_max": golden["num_colors_max"],
        "rounds_max": golden["rounds_max"],
        "per_graph_path": None if t_pergraph is None else {
            "ms": round(t_pergraph * 1e3, 2), "GTEPS": round(m / t_pergraph / 1e9, 3),
            "graphs_per_s": round(G / t_pergraph, 1)},
        "batch_gain_over_per_graph": None if t_pergraph is None else round(t_pergraph / t_step, 2),
        "served": served,
        "roofline": roofline,
        "cpu_baseline": None if args.no_cpu_baseline else batch_cpu_baseline(b),
    }
    print(json.dumps(rec), flush=True)


def batch_cpu_baseline(b, budget=15.0):
    """The oracle on the batch's first graphs, one at a time in order, until
    `budget` seconds of single-thread work; GTEPS over the graphs done."""
    import oracle
    t_total, edges, done = 0.0, 0, 0
    while done < b.num_graphs and t_total < budget:
        g = b.graph(done)
        t = time.perf_counter()
        oracle.rsc(g.rowptr, g.colidx)
        t_total += time.perf_counter() - t
        edges += g.nnz // 2
        done += 1
    return {"value": round(edges / t_total / 1e9, 5), "unit": "GTEPS", "cores": 1,
            "kind": "oracle",
            "sample": f"the first {done} of {b.num_graphs} graphs of the batch, each coloured by "
                      f"the single-thread oracle ({t_total:.1f} s, {edges} edges)",
            "seconds": round(t_total, 3)}


if __name__ == "__main__":
    main()
