"""Benchmark: randomized BP (RnBP) on the 1000 x 1000 Ising grid on one MI355X.

A step is one complete solve through the C ABI: bp_run (messages reset to
uniform, RnBP with the EdgeRatio rule, eps = 1e-4, at most 10000 iterations)
followed by Eq. (3) beliefs into device memory.  Every iteration of a solve runs
the whole hot path: node aggregates, Eq. (2) for every directed message, the
residual of Eq. (4), the count / max reduction, the p schedule, the eps and
random filters and the commit.  The graph (h ~ U[-1, 1], J ~ U[-C, C]) is built
and uploaded before the timed region; each step uses a different RNG seed.

Prints one JSON line.  ``value`` is message updates (Eq. (2) evaluations) per
second over the timed steps.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK = 8.0e12  # MI355X HBM3E, bytes/s


def _log(msg):
    print(msg, file=sys.stderr, flush=True)


def iteration_bytes(N, E, K=2, K_unary=1):
    """Algorithmic bytes of one dense iteration (the workload's definition):
    every message read once and written once as K FP32 values, the pairwise
    parameter of every undirected edge (4), K_unary FP32 unary values per node,
    the slot offsets (N + 1 int32) and two int32 indices per message:
    2 E K 4 + (E / 2) 4 + N K_unary 4 + (N + 1) 4 + 2 E 4.
    1000 x 1000 Ising: 111.9 MB (28.0 B per message)."""
    return 2 * E * K * 4 + (E // 2) * 4 + N * K_unary * 4 + (N + 1) * 4 + 2 * E * 4


def eval_kernel_bytes(N, E, two_outputs=True, rev_bytes=2):
    """Bytes the K = 2 log-odds evaluation kernel must move, each array element
    once: per directed message the in-slot log-odds (4), the reverse slot
    (rev_bytes: a 16-bit offset from the slot on graphs where every offset fits,
    such as the grids here, else a 4-byte index), the coupling (4) and the
    committed value (4), and in RnBP mode the committed value under the second
    keep threshold (4); per node the slot offset (4) and the unary log-odds (4).
    (The stored layout keeps one value per K = 2 message, hence fewer bytes than
    iteration_bytes.)"""
    return ((16 if two_outputs else 12) + rev_bytes) * E + 8 * N


def ragged_iteration_bytes(problem):
    """Algorithmic bytes of one dense iteration with per-variable state counts:
    every message i -> j read once and written once (K_j FP32 values each), its
    K_i x K_j table once, every unary once, and the topology (node offsets, two
    int32 per message, the message and table offsets)."""
    import numpy as np
    kv = np.asarray(problem["var_states"], dtype=np.int64)
    ed = np.asarray(problem["edges"], dtype=np.int64).reshape(-1, 2)
    ka, kb = kv[ed[:, 0]], kv[ed[:, 1]]
    E, N = 2 * len(ed), len(kv)
    msg = 2 * int((ka + kb).sum()) * 4
    tab = 2 * int((ka * kb).sum()) * 4
    return msg + tab + int(kv.sum()) * 4 + (N + 1) * 4 + 2 * E * 4 + 2 * (E + 1) * 4


def paper_ratios(bp, inputs, srbp, torch, eps, time_limit_s=20.0):
    """The paper's speedup protocol restated on this host: serial residual BP
    (SRBP, one host core, its own indexed heap) against RnBP, frontier RBP and
    residual splash on the GPU, on the paper's own parameterisation (unaries
    U(0, 1] per state, J = lambda C, lambda ~ U[-1/2, 1/2]; C is the paper's),
    with the LowP settings and frontier sizes the paper reports.  Times are
    wall clock to convergence (graph resident on the GPU)."""
    cases = [("ising100_C2", (100, 100, 2.0), 0.7), ("ising100_C2.5", (100, 100, 2.5), 0.7),
             ("ising100_C3", (100, 100, 3.0), 0.1), ("ising200_C2.5", (200, 200, 2.5), 0.7),
             ("chain100000_C10", (1, 100000, 10.0), 0.7)]
    out = {}
    for name, (H, W, C), low in cases:
        pr = inputs.paper_ising_grid(H, W, C, 0)
        s = srbp.srbp_solve(pr, eps=eps, time_limit_s=time_limit_s)
        row = {"srbp_s": s["seconds"], "srbp_converged": s["converged"],
               "srbp_updates": s["updates"], "low_p": low}
        p_rbp = 1 / 16 if H == 1 else 1 / 256
        with bp.Graph(pr) as g:
            for key, sched, p in (("rnbp", "rnbp", low), ("rbp", "rbp", p_rbp),
                                  ("rs", "rs", p_rbp), ("lbp", "lbp", 1.0)):
                g.run(sched, eps=eps, p=p, seed=1, max_iters=50)  # warm the launch path
                torch.cuda.synchronize()
                a = time.perf_counter()
                r = g.run(sched, eps=eps, p=p, seed=1, max_iters=10000, check_every=16)
                torch.cuda.synchronize()
                dt = time.perf_counter() - a
                row[key] = {"s": dt, "converged": r["converged"], "iterations": r["iterations"],
                            "p": p, "speedup_vs_srbp": (s["seconds"] / dt
                                                        if r["converged"] and s["converged"]
                                                        else None)}
        out[name] = row
        _log(f"bench: paper ratio {name} {row}")
    return out


def host_cpu():
    """Host cores and CPU model (for the CPU baseline)."""
    model = None
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count()
    return {"nproc": usable, "logical_cpus": os.cpu_count(), "model": model}


def counter_traffic(path, kernel_src):
    """Bytes per launch from the committed FETCH_SIZE / WRITE_SIZE summary, or
    None when the kernel source has changed since the counters were taken."""
    import hashlib
    try:
        kv = dict(line.strip().split("=", 1) for line in open(path)
                  if "=" in line and not line.startswith("#"))
        sha = hashlib.sha256(open(kernel_src, "rb").read()).hexdigest()
    except OSError:
        return None
    if kv.get("kernel_source_sha256") != sha:
        return None
    return float(kv["traffic_bytes_per_launch"])


def serving_mix(inputs, np, n, seed=0):
    """The serving workload: Ising grids with side ~ U{32..512} and Erdos-Renyi
    graphs with n ~ U[1k, 50k], average degree ~ U{4..8}; C ~ U[1, 3]."""
    rng = np.random.default_rng(seed)
    mix = []
    for i in range(n):
        C = float(rng.uniform(1.0, 3.0))
        if rng.random() < 0.5:
            side = int(rng.integers(32, 513))
            mix.append(inputs.ising_grid(side, side, C, 1000 + i))
        else:
            mix.append(inputs.er_graph(int(rng.integers(1000, 50001)), float(rng.integers(4, 9)), C,
                                       1000 + i))
    return mix


def serving_bench(bp, inputs, np, torch, args, n=1000, max_iters=2000, p=0.5,
                  rates=(100.0,), launches=16):
    """Batched serving (one launch per iteration for every resident graph,
    recorded HIP graphs, autotuned grid) against one graph per bp_run, on the
    same n requests (RnBP, eps = 1e-4, at most 2000 iterations each) and the same
    arrival times, both legs replayed on the wall clock: a burst (all at time 0)
    and Poisson processes at each of `rates` requests/s.  Latency = completion -
    arrival; submission (the host builds and validates the layout) is inside it."""
    mix = serving_mix(inputs, np, n)
    msgs = sum(2 * len(pr["edges"]) for pr in mix)
    out = {"requests": n, "messages_total": msgs, "max_iters": max_iters,
           "poisson_rates": list(rates), "launches_per_step": launches}
    rng = np.random.default_rng(7)
    gaps = rng.exponential(1.0, n)  # one unit-rate draw, scaled per rate
    arrivals = {"burst": np.zeros(n)}
    for rate in rates:
        arrivals[f"poisson_{rate:g}/s"] = np.cumsum(gaps / rate)

    def stats(lat, makespan):
        lat = np.asarray(lat)
        return {"graphs_per_s": n / makespan, "p50_ms": float(np.percentile(lat, 50) * 1e3),
                "p99_ms": float(np.percentile(lat, 99) * 1e3), "makespan_s": makespan}

    for name, arr in arrivals.items():
        # one graph per run: a single worker takes requests in arrival order
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        lat = []
        for i, pr in enumerate(mix):
            now = time.perf_counter() - t0
            if arr[i] > now:
                time.sleep(arr[i] - now)
            with bp.Graph(pr) as g:
                g.run("rnbp", eps=args.eps, p=p, seed=i, max_iters=max_iters, check_every=64)
                g.marginals()
            lat.append(time.perf_counter() - t0 - arr[i])
        out.setdefault(name, {})["one_graph_per_run"] = stats(lat, time.perf_counter() - t0)
        _log(f"bench: serving {name} one graph per run {out[name]['one_graph_per_run']}")
        # batched serving
        with bp.Server(4 << 30, max_graphs=128, graphs=True, autotune=True) as srv:
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            ids, done, nxt = {}, {}, 0
            while len(done) < n:
                now = time.perf_counter() - t0
                while nxt < n and arr[nxt] <= now:
                    ids[srv.submit(mix[nxt], "rnbp", eps=args.eps, p=p, seed=nxt,
                                   max_iters=max_iters)] = nxt
                    nxt += 1
                if ids:
                    srv.step(launches)
                    now = time.perf_counter() - t0
                    for rid, k in list(ids.items()):
                        if srv.result(rid) is not None:
                            done[k] = now
                            del ids[rid]
                else:
                    time.sleep(max(0.0, min(arr[nxt] - now, 0.001)))
            makespan = time.perf_counter() - t0
            out[name]["batched"] = stats([done[k] - arr[k] for k in range(n)], makespan)
            out[name]["batched"]["autotuner"] = srv.config()
        _log(f"bench: serving {name} batched {out[name]['batched']}")
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--size", type=int, default=1000)
    ap.add_argument("--C", type=float, default=2.5)
    ap.add_argument("--p", type=float, default=0.5)
    ap.add_argument("--eps", type=float, default=1e-4)
    ap.add_argument("--max-iters", type=int, default=10000)
    ap.add_argument("--check-every", type=int, default=64)
    ap.add_argument("--profile-every", type=int, default=16,
                    help="time one evaluation launch in this many with HIP events")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-iters", type=int, default=20)
    ap.add_argument("--no-ttc", action="store_true")
    ap.add_argument("--no-extra", action="store_true")
    ap.add_argument("--copy-probe", action="store_true",
                    help="run one 256 MiB device-to-device copy kernel first (a known-size "
                         "reference for hardware byte counters)")
    ap.add_argument("--ttc-seeds", type=int, default=3)
    ap.add_argument("--ttc-seeds-c1", type=int, default=50,
                    help="graphs of the C = 1 time-to-convergence study for LBP and RnBP p = 0.5")
    ap.add_argument("--cpu-omp-iters", type=int, default=100)
    ap.add_argument("--er-seeds", type=int, default=0,
                    help="time to convergence on this many 200k-node ER graphs (RnBP p = 0.3 "
                         "vs LBP, C = 2.5); 0 = skip")
    ap.add_argument("--extras", default="rbp,er,potts,ising4000,splash,protein,paper_ratios,serving",
                    help="comma-separated extras to run (unless --no-extra)")
    ap.add_argument("--serving-requests", type=int, default=1000,
                    help="requests of the serving mix")
    ap.add_argument("--ttc-check-every", type=int, default=16,
                    help="convergence poll interval of the time-to-convergence runs")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path; "
              "use --gpus 1", file=sys.stderr)
        sys.exit(2)

    lib = os.path.join(ROOT, "paper_1909_11469_amd", "libbp.so")
    if not os.path.exists(lib):
        import __graft_entry__
        __graft_entry__.build()

    import numpy as np
    import torch

    from paper_1909_11469_amd import bp, inputs

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    S = args.size
    _log(f"bench: building Ising {S}x{S} C={args.C}")
    prob = inputs.ising_grid(S, S, args.C, 0)
    N, E = prob["N"], 2 * len(prob["edges"])
    g = bp.Graph(prob)
    marg = torch.empty((N, 2), dtype=torch.float32, device="cuda")
    run_kw = dict(eps=args.eps, p=args.p, max_iters=args.max_iters,
                  check_every=args.check_every)

    if args.copy_probe:
        src = torch.ones(64 << 20, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    for w in range(args.warmup):
        r = g.run("rnbp", seed=1000 + w, **run_kw)
        g.marginals_device(marg)
        _log(f"bench: warmup {w} iterations={r['iterations']} converged={r['converged']}")
    torch.cuda.synchronize()

    evaluated = committed = iters = conv = 0
    kern_ms = 0.0
    kern_n = 0
    t0 = time.perf_counter()
    for k in range(args.steps):
        r = g.run("rnbp", seed=k, profile=args.profile_every, **run_kw)
        g.marginals_device(marg)
        evaluated += r["evaluated"]
        committed += r["committed"]
        iters += r["iterations"]
        conv += int(r["converged"])
        kern_ms += r["eval_kernel_ms"]
        kern_n += r["eval_kernel_launches"]
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    elapsed = t1 - t0
    _log(f"bench: timed {args.steps} steps in {elapsed:.3f} s, {iters} iterations, "
         f"{conv} converged")

    avg_kernel_s = kern_ms / max(kern_n, 1) / 1e3
    # algorithmic bytes per launch: 28.0 B per directed message (the workload's
    # definition, iteration_bytes) x E messages per launch
    nbytes = iteration_bytes(N, E)
    achieved = nbytes / avg_kernel_s if avg_kernel_s > 0 else 0.0
    stored = eval_kernel_bytes(N, E)
    traffic = counter_traffic(
        os.path.join(ROOT, "profiles", "k_eval_logodds_rnbp_ising1000_counters.txt"),
        os.path.join(ROOT, "paper_1909_11469_amd", "csrc", "bp_kernels.hip"))
    roofline = {"bound": "hbm", "kernel": "k_eval_logodds<RnBP>",
                "achieved": achieved / 1e9, "peak": HBM_PEAK / 1e9, "unit": "GB/s",
                "frac": achieved / HBM_PEAK, "traffic": traffic,
                "bytes_per_launch": nbytes, "bytes_per_message": nbytes / E,
                "bytes_definition": "2EK4 + (E/2)4 + N4 + (N+1)4 + 2E4 (each message read and "
                                    "written once as K = 2 FP32 values, parameters, topology)",
                "frac_stored_layout": (stored / avg_kernel_s / HBM_PEAK
                                       if avg_kernel_s > 0 else None),
                "stored_layout_bytes_per_launch": stored,
                "frac_counter_traffic": (traffic / avg_kernel_s / HBM_PEAK
                                         if traffic and avg_kernel_s > 0 else None),
                "avg_kernel_us": avg_kernel_s * 1e6, "launches": kern_n}

    out = {
        "metric": "message updates/s (1000x1000 Ising, RnBP)",
        "value": evaluated / elapsed,
        "unit": "message updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"ising_{S}x{S}", "C": args.C, "schedule": "rnbp",
                   "low_p": args.p, "high_p": 1.0, "eps": args.eps,
                   "max_iters": args.max_iters, "messages": E, "variables": N,
                   "iterations_timed": iters, "converged_steps": conv,
                   "committed_updates_per_s": committed / elapsed},
        "roofline": roofline,
    }

    if not args.no_ttc:
        # time to convergence, LBP vs RnBP at several low settings p, and RnBP
        # with sparse re-evaluation once n_t <= E / 16 (bitwise the same run),
        # per coupling scale (graph resident; the paper's C is twice this C).
        # At C = 1 (where schedules converge) LBP and RnBP p = 0.5 run on
        # --ttc-seeds-c1 graphs, the other schedules on the first --ttc-seeds.
        ttc = {}
        scheds_all = ([("lbp", 1.0, 0)] + [("rnbp", q, 0) for q in (0.1, 0.3, 0.5, 1.0)] +
                      [("rnbp", 0.5, 2)] + [("rbp", q, 0) for q in (0.1, 0.3, 0.5)])
        scheds_core = [("lbp", 1.0, 0), ("rnbp", 0.5, 0), ("rnbp", 0.5, 2)]
        for C in (1.0, 2.5, 4.0):
            rows = {}
            nseeds = max(args.ttc_seeds, args.ttc_seeds_c1) if C == 1.0 else args.ttc_seeds
            for s in range(nseeds):
                scheds = scheds_all if s < args.ttc_seeds else scheds_core
                pr = inputs.ising_grid(S, S, C, 100 + s)
                with bp.Graph(pr) as gg:
                    for sched, q, sp in scheds:
                        torch.cuda.synchronize()
                        a = time.perf_counter()
                        rr = gg.run(sched, eps=args.eps, p=q, seed=s, max_iters=args.max_iters,
                                    check_every=args.ttc_check_every, sparse=sp)
                        torch.cuda.synchronize()
                        key = sched if sched == "lbp" else f"{sched}_p={q:g}"
                        key += "_sparse" if sp else ""
                        rows.setdefault(key, []).append(
                            (rr["converged"], time.perf_counter() - a, rr["iterations"],
                             rr["evaluated"]))
                _log(f"bench: ttc C={C} seed={100 + s} " +
                     " ".join(f"{k}={v[-1][0]}/{v[-1][2]}" for k, v in rows.items()))
            ttc[f"C={C}"] = {
                k: {"converged": sum(r[0] for r in v), "graphs": len(v),
                    "mean_s_converged": (float(np.mean([r[1] for r in v if r[0]]))
                                         if any(r[0] for r in v) else None),
                    "mean_iterations": float(np.mean([r[2] for r in v])),
                    "mean_evaluated": float(np.mean([r[3] for r in v]))}
                for k, v in rows.items()}
        out["time_to_convergence"] = ttc

    if args.er_seeds > 0:
        rows = {}
        for s in range(args.er_seeds):
            pr = inputs.er_graph(200000, 6.0, 2.5, 100 + s)
            with bp.Graph(pr) as gg:
                for sched, q in (("lbp", 1.0), ("rnbp", 0.3)):
                    torch.cuda.synchronize()
                    a = time.perf_counter()
                    rr = gg.run(sched, eps=args.eps, p=q, seed=s, max_iters=args.max_iters,
                                check_every=args.ttc_check_every)
                    torch.cuda.synchronize()
                    rows.setdefault(sched, []).append(
                        (rr["converged"], time.perf_counter() - a, rr["iterations"]))
            _log(f"bench: er ttc seed={100 + s} " +
                 " ".join(f"{k}={v[-1][0]}/{v[-1][2]}" for k, v in rows.items()))
        out["er_time_to_convergence"] = {
            k: {"converged": sum(r[0] for r in v), "graphs": len(v),
                "mean_s_converged": (float(np.mean([r[1] for r in v if r[0]]))
                                     if any(r[0] for r in v) else None),
                "mean_iterations": float(np.mean([r[2] for r in v]))}
            for k, v in rows.items()}

    if not args.no_extra:
        extra = {}
        wanted = set(x.strip() for x in args.extras.split(",") if x.strip())
        # frontier residual BP on the same graph: share of the iteration spent
        # outside the evaluation kernel (top-k selection and commit)
        for p_rbp in ((1 / 256, 1 / 16) if "rbp" in wanted else ()):
            r = g.run("rbp", eps=args.eps, p=p_rbp, max_iters=200, check_every=args.check_every,
                      profile=1)
            it_us = r["device_ms"] * 1e3 / (r["iterations"] + 1)
            ev_us = r["eval_kernel_ms"] * 1e3 / max(r["eval_kernel_launches"], 1)
            extra[f"rbp_p={p_rbp:.6g}"] = {
                "iteration_us": it_us, "eval_kernel_us": ev_us,
                "selection_share": max(0.0, 1.0 - ev_us / it_us),
                "committed_per_iteration": r["committed"] / max(r["iterations"], 1)}
            _log(f"bench: rbp p={p_rbp:.6g} {extra[f'rbp_p={p_rbp:.6g}']}")
        # the irregular and the K = 32 workloads (parity-tested).  Throughput is
        # taken over launches that all evaluate (eps = 0: no launch is a no-op
        # after convergence); convergence at eps is reported from its own run.
        for name, pr, p_, iters in (
                (("er_200k_deg6_C2.5", inputs.er_graph(200000, 6.0, 2.5, 0), 0.3, 1000),)
                if "er" in wanted else ()) + (
                (("potts_500x500_K32", inputs.potts_grid(500, 500, 32, 1.0, 0), 0.5, 100),)
                if "potts" in wanted else ()):
            E_, N_, K_ = 2 * len(pr["edges"]), pr["N"], pr["K"]
            # the workload's algorithmic bytes per iteration (iteration_bytes)
            nb = iteration_bytes(N_, E_, K_, 1 if K_ == 2 else K_)
            row = {"schedule": "rnbp", "p": p_, "messages": E_, "bytes_per_launch": nb}
            # Potts: the matrix-core product and the FP32 vector path (flag 2)
            # and BF16 operands on the matrix cores (flag 16)
            variants = (("", 0),) if K_ == 2 else (("", 0), ("vector_path_", 2), ("bf16_", 16))
            margs = []
            for tag, flags in variants:
                with bp.Graph(pr, flags=flags) as gg:
                    t0 = time.perf_counter()
                    rc = gg.run("rnbp", eps=args.eps, p=p_, seed=1, max_iters=iters, check_every=1)
                    t_conv = time.perf_counter() - t0
                    margs.append(gg.marginals())
                    gg.run("rnbp", eps=0.0, p=p_, seed=1, max_iters=5)
                    rr = gg.run("rnbp", eps=0.0, p=p_, seed=2, max_iters=min(iters, 50),
                                check_every=args.check_every, profile=args.profile_every)
                    us = rr["eval_kernel_ms"] * 1e3 / max(rr["eval_kernel_launches"], 1)
                    row.update({
                        tag + "iterations_at_eps": rc["iterations"],
                        tag + "converged_at_eps": rc["converged"], tag + "solve_s": t_conv,
                        tag + "message_updates_per_s": rr["evaluated"] / (rr["device_ms"] / 1e3),
                        tag + "eval_kernel_us": us,
                        tag + "hbm_frac": nb / (us * 1e-6) / HBM_PEAK if us > 0 else None})
                    if K_ == 2:
                        # the LBP baseline on the same graph
                        t0 = time.perf_counter()
                        rl = gg.run("lbp", eps=args.eps, max_iters=iters, check_every=16)
                        row["lbp_iterations_at_eps"] = rl["iterations"]
                        row["lbp_converged_at_eps"] = rl["converged"]
                        row["lbp_solve_s"] = time.perf_counter() - t0
                        rl = gg.run("lbp", eps=0.0, max_iters=50, check_every=args.check_every,
                                    profile=args.profile_every)
                        row["lbp_eval_kernel_us"] = (rl["eval_kernel_ms"] * 1e3 /
                                                     max(rl["eval_kernel_launches"], 1))
            if len(margs) == 3:
                row["max_abs_marginal_diff_matrix_vs_vector"] = float(
                    np.max(np.abs(margs[0] - margs[1])))
                row["max_abs_marginal_diff_bf16_vs_fp32_matrix"] = float(
                    np.max(np.abs(margs[2] - margs[0])))
            extra[name] = row
            _log(f"bench: {name} {extra[name]}")
        # a working set far beyond the 256 MB Infinity Cache: every byte of a
        # sweep comes from HBM (16M variables, 64M messages)
        if "ising4000" in wanted:
            pr = inputs.ising_grid(4000, 4000, args.C, 0)
            N4, E4 = pr["N"], 2 * len(pr["edges"])
            with bp.Graph(pr) as gg:
                del pr
                row = {"messages": E4}
                # the graph's first long run tunes its launch shape: keep those
                # launches out of the timed runs
                gg.run("rnbp", eps=0.0, p=args.p, seed=0, max_iters=40)
                for sched in ("lbp", "rnbp"):
                    rr = gg.run(sched, eps=args.eps, p=args.p, seed=1, max_iters=60,
                                check_every=args.check_every, profile=args.profile_every)
                    us = rr["eval_kernel_ms"] * 1e3 / max(rr["eval_kernel_launches"], 1)
                    nb = iteration_bytes(N4, E4)
                    row[sched] = {"eval_kernel_us": us, "bytes_per_launch": nb,
                                  "hbm_frac": nb / (us * 1e-6) / HBM_PEAK if us > 0 else None,
                                  "message_updates_per_s": rr["evaluated"] / (rr["device_ms"] / 1e3)}
            extra["ising_4000x4000_C%g" % args.C] = row
            _log(f"bench: ising 4000x4000 {row}")
        if "splash" in wanted:
            # residual splash (the paper's strongest prior GPU baseline, h = 2) on
            # the 1000 x 1000 grid: iteration time at C = 2.5, convergence at C = 1
            rs_row = {}
            for p_rs in (1 / 256, 1 / 16):
                r = g.run("rs", eps=args.eps, p=p_rs, max_iters=100, check_every=args.check_every,
                          profile=1)
                it_us = r["device_ms"] * 1e3 / (r["iterations"] + 1)
                ev_us = r["eval_kernel_ms"] * 1e3 / max(r["eval_kernel_launches"], 1)
                rs_row[f"p={p_rs:.6g}"] = {
                    "iteration_us": it_us, "eval_kernel_us": ev_us,
                    "share_outside_evaluation": max(0.0, 1.0 - ev_us / it_us),
                    "committed_per_iteration": r["committed"] / max(r["iterations"], 1)}
            conv = []
            for sd in range(3):
                pr = inputs.ising_grid(S, S, 1.0, 100 + sd)
                with bp.Graph(pr) as gg:
                    torch.cuda.synchronize()
                    a = time.perf_counter()
                    rr = gg.run("rs", eps=args.eps, p=1 / 256, max_iters=args.max_iters,
                                check_every=args.ttc_check_every)
                    torch.cuda.synchronize()
                    conv.append((rr["converged"], time.perf_counter() - a, rr["iterations"]))
            rs_row["ttc_C=1_p=1/256"] = {
                "converged": sum(c[0] for c in conv), "graphs": len(conv),
                "mean_s_converged": (float(np.mean([c[1] for c in conv if c[0]]))
                                     if any(c[0] for c in conv) else None),
                "mean_iterations": float(np.mean([c[2] for c in conv]))}
            extra["residual_splash_1000x1000_h2"] = rs_row
            _log(f"bench: residual splash {rs_row}")
        # variables with their own numbers of states (2..81, a contact graph):
        # the stand-in for the paper's side-chain models
        for n_pl in ((2000, 50000) if "protein" in wanted else ()):
            pr = inputs.protein_like_graph(n_pl, 8.0, 0)
            nb = ragged_iteration_bytes(pr)
            with bp.Graph(pr) as gg:
                t0 = time.perf_counter()
                rc = gg.run("rnbp", eps=args.eps, p=0.4, high_p=0.9, seed=1, max_iters=2000,
                            check_every=16)
                t_conv = time.perf_counter() - t0
                rl = gg.run("lbp", eps=0.0, max_iters=50, check_every=args.check_every,
                            profile=args.profile_every)
                us = rl["eval_kernel_ms"] * 1e3 / max(rl["eval_kernel_launches"], 1)
            extra[f"protein_like_{n_pl}_deg8_K2-81"] = {
                "messages": 2 * len(pr["edges"]), "bytes_per_iteration": nb,
                "rnbp_low0.4_high0.9_converged": rc["converged"],
                "rnbp_iterations": rc["iterations"], "rnbp_solve_s": t_conv,
                "lbp_eval_kernel_us": us,
                "lbp_message_updates_per_s": rl["evaluated"] / (rl["device_ms"] / 1e3),
                "hbm_frac": nb / (us * 1e-6) / HBM_PEAK if us > 0 else None}
            _log(f"bench: protein-like {n_pl} {extra[f'protein_like_{n_pl}_deg8_K2-81']}")
        if "paper_ratios" in wanted:
            from paper_1909_11469_amd import srbp
            extra["paper_ratios_vs_srbp"] = paper_ratios(bp, inputs, srbp, torch, args.eps)
        if "serving" in wanted:
            extra["serving"] = serving_bench(bp, inputs, np, torch, args, n=args.serving_requests)
            _log(f"bench: serving {extra['serving']}")
        out["extra"] = extra

    if not args.no_cpu_baseline:
        # the oracle as it is, on the host's cores: the parity build (one
        # thread) and the same loop split over OpenMP threads
        import oracle
        host = host_cpu()
        _log(f"bench: cpu baseline, {args.cpu_iters} oracle iterations (1 thread), "
             f"{args.cpu_omp_iters} (OpenMP), host {host}")
        a = time.perf_counter()
        rr = oracle.run(prob, oracle.RNBP, eps=args.eps, p=args.p, seed=0,
                        max_iters=args.cpu_iters)
        dt = time.perf_counter() - a
        single = {"value": rr["evaluated"] / dt, "unit": "message updates/s", "cores": 1,
                  "sample": f"{args.cpu_iters} RnBP iterations ({rr['evaluated']} Eq. (2) "
                            f"evaluations) of the same {S}x{S} grid, FP64, {dt:.1f} s"}
        omp = oracle.load_openmp()
        threads = oracle.num_threads(omp)
        a = time.perf_counter()
        ro = oracle.run(prob, oracle.RNBP, eps=args.eps, p=args.p, seed=0,
                        max_iters=args.cpu_omp_iters, lib=omp)
        dto = time.perf_counter() - a
        out["cpu_baseline"] = {
            "value": ro["evaluated"] / dto, "unit": "message updates/s", "cores": threads,
            "kind": "oracle",
            "sample": f"{args.cpu_omp_iters} RnBP iterations ({ro['evaluated']} Eq. (2) "
                      f"evaluations) of the same {S}x{S} grid, FP64, evaluation loop over "
                      f"{threads} OpenMP threads, {dto:.1f} s wall",
            "single_thread": single, "host": host}
    g.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
