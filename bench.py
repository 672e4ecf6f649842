"""Benchmark of the MI355X RLGL solver.

A "step" of this benchmark is one whole solve: step 0 of Algorithm 1, the
green-light steps, the stop test and the normalisation pi_hat = H / (H 1),
on a graph already resident in HBM.  The default workload is the R-MAT graph
of scale 24 (16.8M nodes, 268M links, (a, b, c) = (0.57, 0.19, 0.19), damping
0.85) with FP32 link values stored per link, FP32 cash and FP64 history.  Its
green-light schedule is the one with the shortest time to solution on these
kernels: the all-green schedule (power iteration as RLGL's special case),
measured beside the threshold schedule (r = 1) in the same run.  Also timed:
the Chung-Lu 2^20 graph under both schedules, the CPU oracle, the batched
engines and the serving pool.

The solve stops at ||C_t||_1 / |H_t 1| < (1 - c) * 1e-6, which bounds the L1
distance to pi* by 1e-6 (contraction of the Google matrix); the result is
then checked against the FP64 reference (power iteration of the oracle) and
by the FP64 residual of the returned vector.

Printed: one JSON line (the contract of the build driver).
"""
import argparse
import hashlib
import json
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "edge-pushes/s (GTEPS) to L1≤1e-6 vs FP64; batched solves/s + p99 latency"


def source_hash():
    """Hash of the device code (kernels and their shared definitions)."""
    h = hashlib.sha256()
    for f in ("rlgl_kernels.hip", "rlgl_device.h"):
        with open(os.path.join(ROOT, "paper_2008_02710_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def read_traffic(kernel: str, workload: str):
    """HBM bytes per launch from a committed rocprofv3 counter summary, if it
    was taken on the current kernel sources."""
    path = os.path.join(ROOT, "profiles", f"{kernel}_{workload}_pmc.txt")
    if not os.path.exists(path):
        return None
    kv = {}
    for line in open(path):
        if "=" in line and not line.startswith("#"):
            k, v = line.split("=", 1)
            kv[k.strip()] = v.strip()
    if kv.get("source_hash") != source_hash():
        return None
    try:
        return float(kv["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


# Per workload: the generator, the schedule timed for the headline, the
# schedules timed beside it, and how the link values are held.
WORKLOADS = {
    # R-MAT scale 24 with FP32 P values stored per link.  All-green takes 21
    # steps (5.9G edge-pushes) where the threshold rule takes 198 (46.6G): the
    # threshold's green nodes are the hubs (about 80% of the links per step)
    # and the equal cash of the nodes without in-links keeps the residual up
    "rmat_s24": dict(sched="all", alt=["threshold"], link_values="stored"),
    # Chung-Lu 2^20: the threshold schedule is the workload's own
    "chung_lu_2p20": dict(sched="threshold", alt=["all"], link_values="implicit"),
    "scc_c1_2p20": dict(sched="threshold", alt=[], link_values="implicit"),
    "poisson_1e4": dict(sched="all", alt=["maxc"], link_values="stored"),
}


def make_workload(name: str):
    import workloads
    if name == "chung_lu_2p20":
        return workloads.chung_lu(1 << 20, 2.1, 16.0, 0.05, 0.85, seed=0, name=name)
    if name == "rmat_s24":
        g = workloads.rmat(24, 16, 0.57, 0.19, 0.19, 0.85, seed=0)
        g.name = name
        return g
    if name == "scc_c1_2p20":
        # the undamped chain (c = 1) on the largest strongly connected component
        base = workloads.chung_lu(1 << 20, 2.1, 16.0, 0.0, 1.0, seed=0, name="chung_lu_2p20_nodangle")
        return workloads.largest_scc(base, c=1.0, name=name)
    if name == "poisson_1e4":
        g = workloads.poisson_uniform(10000, 8.0, 0.85, seed=0)
        g.name = name
        return g
    raise SystemExit(f"unknown workload {name}")


def host_cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or platform.machine()


def log(*a):
    print("#", *a, file=sys.stderr, flush=True)


def time_solves(rl, torch, s, eps, max_steps, steps, warmup, stream):
    """Warm-up solves, then `steps` timed solves (reset + solve each), with a
    device synchronisation on both sides of the timed region."""
    def one():
        s.reset()
        st, info = s.solve(eps, max_steps)
        return info

    for _ in range(warmup):
        one()
    torch.cuda.synchronize()
    infos, wall = [], []
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    ev0.record(stream)
    t0 = time.perf_counter()
    for _ in range(steps):
        a = time.perf_counter()
        infos.append(one())
        wall.append(time.perf_counter() - a)
    ev1.record(stream)
    torch.cuda.synchronize()
    total = time.perf_counter() - t0
    return infos, wall, total, ev0.elapsed_time(ev1)


def roofline_of(prof, copy_gbps, traffic):
    """Roofline of the dominant kernel from one profiled solve: algorithmic
    bytes (links of green nodes that moved cash and the per-node terms, the
    work the method does) over the launches' event-timed duration, against
    the 8 TB/s HBM peak; the bytes its access pattern touches beside them."""
    dom_name, st = max(prof.items(), key=lambda kv: kv[1]["ms"])
    launches = max(st["launches"], 1)
    achieved = st["bytes"] / (st["ms"] * 1e-3) / 1e9
    touched = st["bytes_touched"] / (st["ms"] * 1e-3) / 1e9
    return {"bound": "hbm", "kernel": f"k_{dom_name}", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
            "algorithmic_bytes_per_launch": round(st["bytes"] / launches),
            "touched_bytes_per_launch": round(st["bytes_touched"] / launches),
            "touched_GBps": round(touched, 1), "touched_frac": round(touched / HBM_PEAK_GBS, 4),
            "green_links_per_launch": round(st["green_links"] / launches),
            "avg_launch_us": round(1000.0 * st["ms"] / launches, 2), "launches_per_solve": st["launches"],
            "stream_copy_GBps": round(copy_gbps, 1), "frac_of_copy": round(achieved / copy_gbps, 4),
            "kernels": {k: {"launches": v["launches"], "ms": round(v["ms"], 4),
                            "GBps": round(v["bytes"] / max(v["ms"], 1e-9) / 1e6, 1),
                            "touched_GBps": round(v["bytes_touched"] / max(v["ms"], 1e-9) / 1e6, 1)}
                        for k, v in prof.items()}}


def schedule_leg(rl, torch, oracle, g, dg, sched_name, args, prec, route, stream, eps, steps, warmup, r=1.0):
    """Times one schedule on a resident graph and certifies its result."""
    import numpy as np
    sched = SCHED_IDS[sched_name]
    relabel = args.relabel if sched not in (rl.SCHED_PC, rl.SCHED_TOPK) else 0
    max_steps = 100000 if sched != rl.SCHED_MAXC else 10_000_000
    s = rl.Solver(dg, stream=stream, sched=sched, r=r, route=route, precision=prec, relabel=relabel)
    infos, wall, total, _ = time_solves(rl, torch, s, eps, max_steps, steps, warmup, stream)
    last = infos[-1]
    pi = s.pi.detach().cpu().numpy()
    s.close()
    ch = oracle.Chain(g.rowptr, g.col, g.val(), g.c)
    resid = oracle.residual(ch, pi)
    ms = 1000.0 * total / steps
    out = {"ms_per_solve": round(ms, 4), "solve_ms_min": round(1000 * min(wall), 4),
           "steps": last["t"] - 1, "edge_pushes": last["edges_pushed"],
           "normalized_iterations": round(last["edges_pushed"] / g.nnz, 3),
           "gteps": round(sum(i["edges_pushed"] for i in infos) / total / 1e9, 3),
           "fp64_residual": resid, "l1_certified_bound": resid / (1.0 - g.c) if g.c < 1.0 else None}
    log(f"schedule {sched_name} on {g.name}: {json.dumps(out)}")
    return out


def batched_leg(args, rl, torch, oracle):
    """Independent chains: n log-uniform in [1e3, 2e5], Chung-Lu exponent 2.3,
    mean degree 10, damping uniform in [0.8, 0.95]; FP32 cash with compensated
    history; each chain stops at ||C||_1/|H.1| < tol (1 - c_k), tol = 1e-6.
    The step-synchronous engine runs with the launch shape the autotuner
    picks, under the all-green and the threshold schedule, in the relabelled
    layout and (for the faster schedule) in the caller's numbering; the
    fastest is the leg's figure.  The plain single-chain path solving the same
    chains one after another is reported beside them."""
    import numpy as np
    import workloads
    t0 = time.time()
    gs = workloads.batch_chains(args.batch, seed=4, with_csc=True)
    tot_n = sum(g.n for g in gs)
    tot_e = sum(g.nnz for g in gs)
    print(f"# batched workload: {len(gs)} chains, {tot_n} nodes, {tot_e} links, gen {time.time() - t0:.1f}s",
          file=sys.stderr, flush=True)
    tol = 1e-6
    db = rl.DeviceBatch(gs, precision=rl.FP32C_KAHANH, tol_l1=tol)
    bs = rl.BatchSolver(db, max_steps=100000)
    tuned = bs.autotune()
    bs.close()
    shapes = {}
    wg, per_cu = tuned["wg_size"], tuned["wg_per_cu"]
    scheds = {"all": rl.SCHED_ALL, "threshold": rl.SCHED_THRESHOLD}

    def run(name, sched, relabel):
        b2 = rl.BatchSolver(db, max_steps=100000, wg_size=wg, wg_per_cu=per_cu, sched=scheds[sched],
                            relabel=relabel)
        b2.solve()  # warm-up
        runs = []
        for _ in range(max(1, min(args.steps, 5))):
            st, res, ms = b2.solve()
            runs.append((ms, res))
        ms_best, res = min(runs, key=lambda x: x[0])
        lat = np.array([r["end_us"] for r in res]) / 1000.0
        pushes = sum(r["edges_pushed"] for r in res)
        # algorithmic bytes (per link of a green node that moved cash: source
        # index and gathered send value, 8 B with implied weights; per node and
        # step: column pointer, cash read and write, send value, 16 B)
        alg = sum(8.0 * r["edges_pushed"] + 16.0 * g.n * r["t"] for r, g in zip(res, gs))
        worst = 0.0
        pi = b2.pi.detach().cpu().numpy()
        for k, g in enumerate(gs):
            ch = oracle.Chain(g.rowptr, g.col, g.val(), g.c)
            r = oracle.residual(ch, pi[db.node_off[k]:db.node_off[k + 1]])
            worst = max(worst, r / (1.0 - g.c))
        b2.close()
        gbps = alg / (ms_best * 1e-3) / 1e9
        shapes[name] = {"solves_per_s": round(len(gs) / (ms_best / 1000.0), 1), "batch_ms": round(ms_best, 3),
                        "p50_ms": round(float(np.percentile(lat, 50)), 3),
                        "p99_ms": round(float(np.percentile(lat, 99)), 3),
                        "gteps": round(pushes / (ms_best / 1000.0) / 1e9, 2), "worst_certified_l1": worst,
                        "algorithmic_GBps": round(gbps, 1), "hbm_frac": round(gbps / HBM_PEAK_GBS, 4),
                        "sched": sched, "relabel": relabel, "wg_size": wg, "wg_per_cu": per_cu,
                        "mean_steps": round(float(np.mean([r["t"] for r in res])), 1),
                        "max_steps": int(max(r["t"] for r in res))}
        log(f"batched {name}: {json.dumps(shapes[name])}")

    run("all_relabelled", "all", 1)
    run("threshold_relabelled", "threshold", 1)
    fast = min(("all", "threshold"), key=lambda x: shapes[x + "_relabelled"]["batch_ms"])
    run(fast + "_caller_numbering", fast, 0)
    # the plain single-chain path on the same chains, one after another (same
    # schedule, relabelled layout)
    plain = []
    plain_push = 0
    for g in gs:
        eps = tol * (1.0 - g.c)
        dg = rl.DeviceGraph.from_workload(g, precision=rl.FP32C_KAHANH, explicit_val=False)
        s = rl.Solver(dg, sched=scheds[fast], precision=rl.FP32C_KAHANH, relabel=1)
        s.reset()
        s.solve(eps)
        torch.cuda.synchronize()
        a = time.perf_counter()
        s.reset()
        stp, info = s.solve(eps)
        torch.cuda.synchronize()
        plain.append(1000.0 * (time.perf_counter() - a))
        plain_push += info["edges_pushed"]
        s.close()
        del dg
    plain = np.array(plain)
    seq_lat = np.cumsum(plain)
    print(f"# plain path: {plain.sum():.1f} ms for {len(gs)} solves back to back", file=sys.stderr, flush=True)
    best = min(shapes.values(), key=lambda x: x["batch_ms"])
    return {"workload": f"chung_lu_batch{len(gs)}", "chains": len(gs), "nodes": tot_n, "links": tot_e,
            "precision": "fp32c_kahanh", "tol_l1": tol, "stop": "resid < tol_l1 * (1 - c_k)",
            "tuned": {"engine": "lockstep", "wg_size": tuned["wg_size"], "wg_per_cu": tuned["wg_per_cu"]},
            "sched": best["sched"], "relabel": best["relabel"], "batch_ms": best["batch_ms"],
            "solves_per_s": best["solves_per_s"], "p50_ms": best["p50_ms"], "p99_ms": best["p99_ms"],
            "gteps": best["gteps"], "hbm_frac": best["hbm_frac"], "runs": shapes,
            "plain_single_chain": {"sched": fast, "relabel": 1,
                                   "solves_per_s": round(len(gs) / (plain.sum() / 1000.0), 1),
                                   "solve_ms_p50": round(float(np.percentile(plain, 50)), 3),
                                   "solve_ms_p99": round(float(np.percentile(plain, 99)), 3),
                                   "p50_ms_back_to_back": round(float(np.percentile(seq_lat, 50)), 3),
                                   "p99_ms_back_to_back": round(float(np.percentile(seq_lat, 99)), 3),
                                   "gteps": round(plain_push / (plain.sum() / 1000.0) / 1e9, 2)}}


def serving_leg(args, rl, torch, oracle):
    """Poisson arrivals at 500 requests/s; each request is a chain drawn
    uniformly from a pool of pre-generated chains (n log-uniform in
    [1e3, 1e6], Chung-Lu exponent 2.3, mean degree 12, damping 0.85) held in
    page-locked host memory, tolerance 1e-6 L1.  The upload counts toward the
    latency.  The first seconds of requests warm the pool up; the measured
    requests follow.  Run under an arena budget that never binds and under
    one of 1.25 times the largest request's footprint, where a large request
    holds most of the arena and the admissions after it wait for memory."""
    import numpy as np
    import workloads
    from paper_2008_02710_amd.serving import serve
    t0 = time.time()
    pool_graphs = workloads.serving_pool(args.serve_pool, seed=5)
    hcs = [rl.HostChain(g, tol_l1=1e-6) for g in pool_graphs]
    log(f"serving pool: {len(hcs)} chains, {sum(g.n for g in pool_graphs)} nodes, "
        f"{sum(g.nnz for g in pool_graphs)} links, gen {time.time() - t0:.1f}s")
    total = args.serve_requests + int(args.serve_rate * args.serve_warmup_s * 1.5) + 16
    arrivals = workloads.poisson_arrivals(total, args.serve_rate, seed=5)
    warm = int(np.searchsorted(arrivals, args.serve_warmup_s))
    total = warm + args.serve_requests
    arrivals = list(arrivals[:total])
    draws = workloads.request_draws(total, len(hcs), seed=5)
    reqs = [hcs[d] for d in draws]
    sample = set(range(warm, total, max(1, args.serve_requests // 16)))
    probe = rl.Pool(1 << 20, max_chains=1, precision=rl.FP32C_KAHANH)
    foot = [probe.footprint(h.n, h.nnz) for h in hcs]
    probe.close()
    tight = int(1.25 * max(foot))
    out = {}
    for label, arena in (("unbounded", 48 << 30), ("tight", tight)):
        pool = rl.Pool(arena, max_chains=256, precision=rl.FP32C_KAHANH)
        kept = {}

        def on_result(i, res, pi):
            if i in sample:
                kept[i] = pi.detach().cpu().numpy().copy()

        recs = serve(pool, reqs, arrivals, iterations=args.serve_iters, on_result=on_result)
        pool.close()
        meas = recs[warm:]
        lat = np.array([r["latency"] for r in meas]) * 1000.0
        wait = np.array([r["admitted"] - r["arrival"] for r in meas]) * 1000.0
        span = max(r["finished"] for r in meas) - min(r["arrival"] for r in meas)
        pushes = sum(r["edges_pushed"] for r in meas)
        bad = sum(r["status"] != rl.RLGL_OK for r in meas)
        worst = 0.0
        for i, pi in kept.items():
            g = pool_graphs[draws[i]]
            ch = oracle.Chain(g.rowptr, g.col, g.val(), g.c)
            worst = max(worst, oracle.residual(ch, pi) / (1.0 - g.c))
        # requests and arena bytes in flight over time, from the admission and finish times
        ev = sorted([(r["admitted"], 1, foot[draws[warm + k]]) for k, r in enumerate(meas)] +
                    [(r["finished"], -1, -foot[draws[warm + k]]) for k, r in enumerate(meas)])
        cur = cur_b = peak = peak_b = 0
        for _, d, fb in ev:
            cur += d
            cur_b += fb
            peak = max(peak, cur)
            peak_b = max(peak_b, cur_b)
        out[label] = {"arena_bytes": arena, "requests": len(meas), "failed": bad,
                      "p50_ms": round(float(np.percentile(lat, 50)), 3),
                      "p99_ms": round(float(np.percentile(lat, 99)), 3),
                      "mean_ms": round(float(lat.mean()), 3),
                      "admission_wait_p50_ms": round(float(np.percentile(wait, 50)), 3),
                      "admission_wait_p99_ms": round(float(np.percentile(wait, 99)), 3),
                      "admissions_that_waited": int(sum(r["blocked"] for r in meas)),
                      "completed_per_s": round(len(meas) / span, 1),
                      "served_gteps": round(pushes / span / 1e9, 3),
                      "peak_in_flight": peak, "peak_resident_bytes": int(peak_b),
                      "worst_certified_l1_sampled": worst, "sampled": len(kept)}
        log(f"serving {label}: {json.dumps(out[label])}")
    return {"workload": "chung_lu_serving", "rate_per_s": args.serve_rate, "pool_chains": len(hcs),
            "warmup_s": args.serve_warmup_s, "warmup_requests": warm, "tol_l1": 1e-6,
            "largest_footprint_bytes": int(max(foot)), "iterations_per_poll": args.serve_iters, "budgets": out}


def _csv_rows(folder, suffix):
    import csv
    import glob
    rows = []
    for f in sorted(glob.glob(os.path.join(folder, "**", f"*{suffix}"), recursive=True)):
        rows.extend(csv.DictReader(open(f)))
    return rows


def pmc_summary(folder: str, workload: str, kernel: str, commands: list) -> str:
    """Summary text of the rocprofv3 runs under `folder` (trace/, pmc_FETCH_SIZE/,
    pmc_WRITE_SIZE/, copy_FETCH_SIZE/, copy_WRITE_SIZE/): the dominant kernel's
    mean launch duration and its HBM bytes per launch, the counters scaled by
    what they read for a plain 1 GiB device copy."""
    def per_dispatch(sub, name_part):
        vals = {}
        for r in _csv_rows(os.path.join(folder, sub), "counter_collection.csv"):
            if name_part in r["Kernel_Name"]:
                vals[r["Dispatch_Id"]] = vals.get(r["Dispatch_Id"], 0.0) + float(r["Counter_Value"])
        return list(vals.values())

    fetch = per_dispatch("pmc_FETCH_SIZE", f"k_{kernel}")
    write = per_dispatch("pmc_WRITE_SIZE", f"k_{kernel}")
    cf = max(per_dispatch("copy_FETCH_SIZE", "copyBuffer"))
    cw = max(per_dispatch("copy_WRITE_SIZE", "copyBuffer"))
    gib_kib = float(1 << 20)  # a 1 GiB copy moves 2^20 KiB each way
    ff, wf = gib_kib / cf, gib_kib / cw
    durs = [(int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1000.0
            for r in _csv_rows(os.path.join(folder, "trace"), "kernel_trace.csv") if f"k_{kernel}" in r["Kernel_Name"]]
    # launches of steps that ran (those enqueued after the stop return at once)
    durs = [x for x in durs if x >= 0.25 * max(durs)]
    pairs = [(f, w) for f, w in zip(fetch, write) if f >= 0.25 * max(fetch)]
    fetch, write = [f for f, _ in pairs], [w for _, w in pairs]
    hbm = [1024.0 * (f * ff + w * wf) for f, w in zip(fetch, write)]
    lines = [f"# rocprofv3 summary of k_{kernel} on the {workload} workload (MI355X)", "# commands, from the repository root:"]
    lines += [f"#   {c}" for c in commands]
    lines += [f"# calibration: a plain 1 GiB device copy reads {cf:.0f} KiB (FETCH_SIZE) and writes {cw:.0f} KiB "
              f"(WRITE_SIZE) per launch for {gib_kib:.0f} KiB each way",
              f"kernel = {kernel}", f"workload = {workload}", f"source_hash = {source_hash()}",
              f"fetch_factor = {ff:.4f}", f"write_factor = {wf:.4f}",
              "# launches of steps that ran (a launch enqueued after the stop returns at once and is left out)",
              f"launches_counted = {len(hbm)}",
              f"fetch_size_kib_mean = {sum(fetch) / max(len(fetch), 1):.1f}",
              f"write_size_kib_mean = {sum(write) / max(len(write), 1):.1f}",
              f"hbm_bytes_per_launch = {sum(hbm) / max(len(hbm), 1):.0f}",
              f"trace_launches = {len(durs)}",
              f"trace_avg_duration_us = {sum(durs) / max(len(durs), 1):.2f}"]
    return "\n".join(lines) + "\n"


def fixed_step_leg(rl, torch, dg, args, prec, route, stream, nsteps: int = 20, reps: int = 7):
    """A top-k step beside a threshold step (with about as many green nodes:
    k = N/4 on the Chung-Lu graphs) in the same, the caller's, numbering:
    nsteps steps from step 0, best of reps, and the per-kernel event times
    of one more run (rlgl_profile)."""
    out = {}
    for name, opts in (("threshold", dict(sched=rl.SCHED_THRESHOLD)), ("topk", dict(sched=rl.SCHED_TOPK, k=args.k))):
        s = rl.Solver(dg, stream=stream, route=route, precision=prec, relabel=0, **opts)
        s.reset()
        s.step(nsteps)
        best = 1e30
        for _ in range(reps):
            torch.cuda.synchronize()
            a = time.perf_counter()
            s.reset()
            info = s.step(nsteps)
            torch.cuda.synchronize()
            best = min(best, time.perf_counter() - a)
        rl.rlgl_profile_enable(s.ctx, True)
        s.reset()
        s.step(nsteps)
        torch.cuda.synchronize()
        prof = rl.rlgl_profile_read(s.ctx)
        rl.rlgl_profile_enable(s.ctx, False)
        out[name] = {"us_per_step": round(best / nsteps * 1e6, 1), "green_last_step": info["green"],
                     "kernel_us_per_step": {k: round(1000.0 * v["ms"] / nsteps, 1) for k, v in prof.items()}}
        s.close()
    out["ratio"] = round(out["topk"]["us_per_step"] / out["threshold"]["us_per_step"], 3)
    out["steps"] = nsteps
    log(f"top-k beside threshold, {nsteps} steps from step 0: {json.dumps(out)}")
    return out


def trace_summary(folder: str, workload: str, commands: list, label: str = None) -> str:
    """Markdown table of rocprofv3 --stats kernel statistics under `folder`."""
    rows = _csv_rows(folder, "kernel_stats.csv")
    what = label or f"the {workload} workload"
    out = [f"# rocprofv3 kernel statistics: bench.py on {what} (MI355X)", "",
           "Commands (from the repository root):", "", "```"] + commands + ["```", "",
           "| kernel | calls | total ms | avg us | min us | max us | % |", "|---|---|---|---|---|---|---|"]
    for r in rows[:16]:
        out.append(f"| `{r['Name'][:72]}` | {r['Calls']} | {float(r['TotalDurationNs']) / 1e6:.3f} | "
                   f"{float(r['AverageNs']) / 1e3:.2f} | {float(r['MinNs']) / 1e3:.2f} | "
                   f"{float(r['MaxNs']) / 1e3:.2f} | {float(r['Percentage']):.2f} |")
    out += lockstep_iterations(folder)
    return "\n".join(out) + "\n"


def lockstep_iterations(folder: str) -> list:
    """Per batched (lockstep) solve in the trace: its iterations (one select,
    route and control launch each), the mean kernel times of the iterations
    in which every chain is still in the launch grids, and the time of the
    later ones (from the per-dispatch timestamps)."""
    try:
        rows = _csv_rows(folder, "kernel_trace.csv")
    except (OSError, StopIteration, IndexError):
        return []
    rows.sort(key=lambda r: int(r["Start_Timestamp"]))
    starts = [i for i, r in enumerate(rows) if "k_batch_start" in r["Kernel_Name"]]
    if not starts:
        return []
    out = ["", "Lockstep solves in the trace (per-dispatch timestamps; a full iteration has every chain in the "
           "launch grids):", "",
           "| solve | ms | iterations | full iterations | select / route / control per full iteration, us | "
           "later iterations: kernel ms | later iterations: idle ms |", "|---|---|---|---|---|---|---|"]
    for q, a in enumerate(starts):
        b = starts[q + 1] if q + 1 < len(starts) else len(rows)
        its = []
        for r in rows[a:b]:
            name = r["Kernel_Name"]
            dur = int(r["End_Timestamp"]) - int(r["Start_Timestamp"])
            if "k_ls_select" in name:
                its.append({"start": int(r["Start_Timestamp"]), "grid": int(r["Grid_Size_X"]), "k": {}, "busy": 0})
            if its and "k_ls_" in name:
                kind = "select" if "select" in name else "route" if "route" in name else "control"
                its[-1]["k"][kind] = its[-1]["k"].get(kind, 0) + dur
                its[-1]["busy"] += dur
        if not its:
            continue
        # the solve ends at the last lockstep launch
        end = max(int(r["End_Timestamp"]) for r in rows[a:b] if "k_ls_" in r["Kernel_Name"])
        full = [it for it in its if it["grid"] == its[0]["grid"]]
        later = its[len(full):]
        mean = lambda kind: sum(it["k"].get(kind, 0) for it in full) / len(full) / 1e3
        span_later = (end - later[0]["start"]) / 1e6 if later else 0.0
        busy_later = sum(it["busy"] for it in later) / 1e6
        out.append(f"| {q} | {(end - int(rows[a]['Start_Timestamp'])) / 1e6:.2f} | {len(its)} | {len(full)} | "
                   f"{mean('select'):.1f} / {mean('route'):.1f} / {mean('control'):.1f} | {busy_later:.2f} | "
                   f"{span_later - busy_later:.2f} |")
    return out


SCHED_IDS = {}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10, help="timed solves")
    ap.add_argument("--warmup", type=int, default=3, help="untimed solves")
    ap.add_argument("--workload", default="rmat_s24", choices=sorted(WORKLOADS))
    ap.add_argument("--route", default="auto", choices=["auto", "push", "pull"])
    ap.add_argument("--precision", default="fp32c_fp64h", choices=["fp64", "fp32c_fp64h", "fp32c_kahanh"])
    ap.add_argument("--tol", type=float, default=1e-6, help="certified L1 target")
    ap.add_argument("--sched", default=None, choices=["all", "threshold", "topk", "maxc", "pc"],
                    help="green-light schedule (default: the workload's)")
    ap.add_argument("--k", type=int, default=262144, help="green nodes per step of the top-k schedule")
    ap.add_argument("--r", type=float, default=None, help="threshold power-mean order (default 1)")
    ap.add_argument("--theta-period", type=int, default=1, help="steps between threshold refreshes")
    ap.add_argument("--seed", type=int, default=1, help="seed of the PC draws")
    ap.add_argument("--link-values", default=None, choices=["implicit", "stored"],
                    help="link weights 1/outdeg implied by the CSR row pointers, or stored per link "
                         "(default: the workload's)")
    ap.add_argument("--relabel", type=int, default=1, choices=[0, 1],
                    help="renumber the states by decreasing out-degree inside the library (layout step)")
    ap.add_argument("--small", action="store_true",
                    help="solve with the one-workgroup solver (rlgl_solve_small; small chains)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU-baseline leg")
    ap.add_argument("--no-ref", action="store_true", help="skip the FP64 power-iteration reference")
    ap.add_argument("--no-legs", action="store_true", help="skip the schedule and Chung-Lu comparison legs")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a plain 1 GiB device copy (HBM counter calibration) and exit")
    ap.add_argument("--pmc-summary", default=None, metavar="FOLDER",
                    help="print the summary of the rocprofv3 runs under FOLDER (no GPU) and exit")
    ap.add_argument("--kernel", default="complete", help="kernel of --pmc-summary")
    ap.add_argument("--trace-summary", default=None, metavar="FOLDER",
                    help="print the kernel statistics of the rocprofv3 trace under FOLDER (no GPU) and exit")
    ap.add_argument("--commands", default="", help="--pmc-summary: the commands that made the runs, ';'-separated")
    ap.add_argument("--label", default=None, help="--trace-summary: what the run measured (title of the table)")
    ap.add_argument("--batch", type=int, default=512,
                    help="chains of the batched workload (0 skips the batched leg)")
    ap.add_argument("--serve-requests", type=int, default=20000,
                    help="measured requests of the serving leg (0 skips it)")
    ap.add_argument("--serve-warmup-s", type=float, default=2.0, help="seconds of requests before the measured ones")
    ap.add_argument("--serve-rate", type=float, default=500.0, help="Poisson arrival rate (requests/s)")
    ap.add_argument("--serve-pool", type=int, default=512, help="pre-generated chains requests draw from")
    ap.add_argument("--serve-iters", type=int, default=4, help="lockstep iterations between host polls")
    args = ap.parse_args()

    if args.trace_summary:
        print(trace_summary(args.trace_summary, args.workload,
                            [c.strip() for c in args.commands.split(";") if c.strip()], args.label), end="")
        return

    if args.pmc_summary:
        print(pmc_summary(args.pmc_summary, args.workload, args.kernel,
                          [c.strip() for c in args.commands.split(";") if c.strip()]), end="")
        return

    if args.calibrate_copy:
        import torch
        src = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": src.numel() * 4, "copy_bytes_written": dst.numel() * 4, "launches": 3}))
        return

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path (run with --gpus 1)",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2008_02710_amd as rl

    SCHED_IDS.update({"threshold": rl.SCHED_THRESHOLD, "all": rl.SCHED_ALL, "maxc": rl.SCHED_MAXC,
                      "pc": rl.SCHED_PC, "topk": rl.SCHED_TOPK})
    prec = {"fp64": rl.FP64, "fp32c_fp64h": rl.FP32C_FP64H, "fp32c_kahanh": rl.FP32C_KAHANH}[args.precision]
    route = {"auto": rl.ROUTE_AUTO, "push": rl.ROUTE_PUSH, "pull": rl.ROUTE_PULL}[args.route]
    wl = dict(WORKLOADS[args.workload])
    if args.sched:
        wl["sched"] = args.sched
        wl["alt"] = [x for x in ("all", "threshold") if x != args.sched]
    if args.link_values:
        wl["link_values"] = args.link_values
    r = 1.0 if args.r is None else args.r
    t0 = time.time()
    g = make_workload(args.workload)
    sched = SCHED_IDS[wl["sched"]]
    if sched in (rl.SCHED_PC, rl.SCHED_TOPK) and args.relabel:
        args.relabel = 0  # the PC draws and the top-k ties are keyed by the caller's node ids
    log(f"workload {g.name}: n={g.n} nnz={g.nnz} dangling={g.n_dangling} gen={time.time() - t0:.1f}s")

    dev = torch.device("cuda:0")
    stored = wl["link_values"] == "stored"
    dg = rl.DeviceGraph.from_workload(g, precision=prec, with_csc=True, explicit_val=stored, device=dev)
    stream = torch.cuda.current_stream(dev)
    # c < 1: the residual certifies the L1 error through 1/(1-c); c = 1 has no
    # such bound, so the stop is a tenth of the target and the error is
    # measured against FP64 power iteration
    eps = (1.0 - g.c) * args.tol if g.c < 1.0 else 0.1 * args.tol
    max_steps = 100000 if sched != rl.SCHED_MAXC else 10_000_000

    if args.small:
        s = rl.SmallSolver(dg, stream=stream, sched=sched, r=r, precision=prec, theta_period=args.theta_period,
                           seed=args.seed)
        s.reset = lambda: None  # every one-workgroup solve starts from step 0
    else:
        s = rl.Solver(dg, stream=stream, sched=sched, r=r, route=route, precision=prec, relabel=args.relabel,
                      theta_period=args.theta_period, seed=args.seed, k=args.k)
    infos, wall, t_total, ev_ms = time_solves(rl, torch, s, eps, max_steps, args.steps, args.warmup, stream)
    pushes = sum(i["edges_pushed"] for i in infos)
    gteps = pushes / t_total / 1e9
    ms_per_solve = 1000.0 * t_total / args.steps
    last = infos[-1]
    pi = s.pi.detach().cpu().numpy()
    log(f"timed {args.steps} solves: {ms_per_solve:.3f} ms/solve (events {ev_ms / args.steps:.3f}), "
        f"steps={last['t'] - 1} pushes/solve={last['edges_pushed']} GTEPS={gteps:.1f}")

    # ---- a plain device copy on the same GPU (STREAM-copy style): 2 x 1 GiB moved
    cbuf = torch.empty(1 << 28, dtype=torch.float32, device=dev)
    cdst = torch.empty_like(cbuf)
    cdst.copy_(cbuf)
    ce0 = torch.cuda.Event(enable_timing=True)
    ce1 = torch.cuda.Event(enable_timing=True)
    ce0.record()
    for _ in range(5):
        cdst.copy_(cbuf)
    ce1.record()
    torch.cuda.synchronize()
    copy_gbps = 5 * 2 * cbuf.numel() * 4 / (ce0.elapsed_time(ce1) * 1e-3) / 1e9
    del cbuf, cdst

    # ---- roofline of the dominant kernel: one more solve, HIP events around each launch
    roofline = None
    if not args.small:
        rl.rlgl_profile_enable(s.ctx, True)
        s.reset()
        s.solve(eps, max_steps)
        torch.cuda.synchronize()
        prof = rl.rlgl_profile_read(s.ctx)
        rl.rlgl_profile_enable(s.ctx, False)
        dom = max(prof.items(), key=lambda kv: kv[1]["ms"])[0]
        roofline = roofline_of(prof, copy_gbps, read_traffic(dom, g.name))
        log(f"profile: {json.dumps(roofline['kernels'])}")
    s.close() if hasattr(s, "close") else None
    del s

    # ---- accuracy against FP64
    import oracle
    ch = oracle.Chain(g.rowptr, g.col, g.val(), g.c)
    t_res = time.time()
    true_resid = oracle.residual(ch, pi)
    l1_bound = true_resid / (1.0 - g.c) if g.c < 1.0 else None
    log(f"FP64 residual of pi_hat {true_resid:.3e} -> certified L1 <= {l1_bound} ({time.time() - t_res:.1f}s)")
    l1_ref = None
    if not args.no_ref:
        t_ref = time.time()
        tol_pi = 1e-10 * (1.0 - g.c) if g.c < 1.0 else 1e-13
        pst, x, it, _ = oracle.power_iteration_omp(ch, tol_pi, 100000)
        if pst != oracle.OK:
            raise SystemExit("power iteration reference did not converge")
        l1_ref = float(np.abs(pi - x).sum())
        del x
        log(f"L1 vs FP64 power iteration ({it} iterations, {time.time() - t_ref:.1f}s): {l1_ref:.3e}")

    # ---- the other schedules on the same resident graph, and the Chung-Lu 2^20 graph under both
    schedules = {wl["sched"]: {"ms_per_solve": round(ms_per_solve, 4), "steps": last["t"] - 1,
                               "edge_pushes": last["edges_pushed"],
                               "normalized_iterations": round(last["edges_pushed"] / g.nnz, 3),
                               "gteps": round(gteps, 3), "fp64_residual": true_resid,
                               "l1_certified_bound": l1_bound, "headline": True}}
    chung_lu = None
    if not args.no_legs and not args.small:
        for alt in wl["alt"]:
            schedules[alt] = schedule_leg(rl, torch, oracle, g, dg, alt, args, prec, route, stream, eps,
                                          steps=max(1, min(args.steps, 3)), warmup=1, r=r)
        if args.workload != "chung_lu_2p20":
            g2 = make_workload("chung_lu_2p20")
            dg2 = rl.DeviceGraph.from_workload(g2, precision=prec, with_csc=True, explicit_val=False, device=dev)
            eps2 = (1.0 - g2.c) * args.tol
            chung_lu = {"workload": g2.name, "n": g2.n, "nnz": g2.nnz, "link_values": "implicit",
                        "schedules": {x: schedule_leg(rl, torch, oracle, g2, dg2, x, args, prec, route, stream,
                                                      eps2, steps=max(1, min(args.steps, 5)), warmup=1)
                                      for x in ("threshold", "all")}}
            del dg2, g2
            torch.cuda.empty_cache()

    # ---- top-k: fixed steps beside the threshold rule in the same numbering
    topk_steps = None
    if sched == rl.SCHED_TOPK and not args.small:
        topk_steps = fixed_step_leg(rl, torch, dg, args, prec, route, stream)

    # ---- CPU baseline: the oracle's own serial solve loop (C, FP64, one core)
    # on the same graph, schedule and eps: whole solves while they fit the time
    # budget, else its first steps (step 0 included)
    cpu = None
    if not args.no_cpu:
        osched = {rl.SCHED_THRESHOLD: oracle.THRESHOLD, rl.SCHED_ALL: oracle.ALL, rl.SCHED_MAXC: oracle.MAXC,
                  rl.SCHED_PC: oracle.PC, rl.SCHED_TOPK: oracle.TOPK}[sched]
        ok = {"r": r, "seed": args.seed, "k": args.k}
        a = time.perf_counter()
        ost, _, oinfo = oracle.solve(ch, osched, eps=eps, max_steps=1, **ok)
        probe = time.perf_counter() - a
        per_step = probe / 2.0
        if ost == oracle.OK:
            solves, opushes, tcpu = 0, 0, 0.0
            while tcpu < args.cpu_seconds:
                a = time.perf_counter()
                ost, _, oinfo = oracle.solve(ch, osched, eps=eps, max_steps=10_000_000, **ok)
                tcpu += time.perf_counter() - a
                opushes += oinfo["edges_pushed"]
                solves += 1
            sample = f"{solves} full solves of the serial FP64 oracle (C) on the same graph, schedule and eps"
        else:
            k = max(1, int(args.cpu_seconds / max(per_step, 1e-9)) - 1)
            a = time.perf_counter()
            ost, _, oinfo = oracle.solve(ch, osched, eps=eps, max_steps=k, **ok)
            tcpu = time.perf_counter() - a
            opushes = oinfo["edges_pushed"]
            sample = (f"{'a full solve' if ost == oracle.OK else 'the first ' + str(oinfo['steps']) + ' steps'} "
                      f"(step 0 included) of the serial FP64 oracle's solve loop (C) on the same graph and schedule")
        cpu = {"value": round(opushes / tcpu / 1e9, 5), "unit": "GTEPS", "cores": 1, "kind": "oracle",
               "sample": f"{sample} ({tcpu:.1f} s)", "host": host_cpu_model(), "host_cpus": os.cpu_count()}
        log(f"cpu oracle: {cpu}")
        # all host cores: FP64 power iteration (pull by columns, OpenMP) to the same L1 target
        if g.c < 1.0:
            a = time.perf_counter()
            pst, _, pit, threads = oracle.power_iteration_omp(ch, (1.0 - g.c) * args.tol, 100000)
            tpi = time.perf_counter() - a
            cpu["power_iteration_all_cores"] = {
                "value": round(pit * int(g.nnz) / tpi / 1e9, 5), "unit": "GTEPS", "cores": threads,
                "kind": "OpenMP FP64 power iteration", "iterations": pit, "seconds": round(tpi, 3),
                "sample": "one full solve to the same L1 target, transpose built inside the timed region"}
            log(f"cpu power iteration, all cores: {cpu['power_iteration_all_cores']}")
    del ch, dg
    torch.cuda.empty_cache()

    batched = batched_leg(args, rl, torch, oracle) if args.batch > 0 else None
    serving = serving_leg(args, rl, torch, oracle) if args.serve_requests > 0 else None

    out = {
        "metric": METRIC,
        "value": round(gteps, 3),
        "unit": "GTEPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_solve, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if prec != rl.FP64 else "f64",
        "data": "synthetic",
        "config": {"workload": g.name, "n": g.n, "nnz": g.nnz, "dangling": g.n_dangling, "damping": g.c,
                   "schedule": wl["sched"], "r": r, "precision": args.precision, "route": args.route,
                   "relabel": args.relabel, "link_values": wl["link_values"], "theta_period": args.theta_period,
                   "solver": "one-workgroup" if args.small else "multi-launch",
                   **({"k": args.k} if wl["sched"] == "topk" else {}),
                   "eps_resid": eps, "tol_l1": args.tol, "generator": g.params.get("generator"),
                   "seed": g.params.get("seed")},
        "time_to_solution_ms": round(ms_per_solve, 4),
        "steps_per_solve": last["t"] - 1,
        "edge_pushes_per_solve": last["edges_pushed"],
        "normalized_iterations": round(last["edges_pushed"] / g.nnz, 3),
        "solve_ms_min": round(1000 * min(wall), 4),
        "solve_ms_max": round(1000 * max(wall), 4),
        "l1_vs_fp64_power_iteration": l1_ref,
        "fp64_residual": true_resid,
        "l1_certified_bound": l1_bound,
        "schedules": schedules,
        "chung_lu_2p20": chung_lu,
        "topk_vs_threshold": topk_steps,
        "roofline": roofline,
        "cpu_baseline": cpu,
        "batched": batched,
        "serving": serving,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
