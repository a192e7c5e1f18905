"""Benchmark: simulated-annealing iterations/s and accepted-swap Delta-updates/s
of the HIP path on one MI355X, single chain vs batched chains, with the CPU
oracle timed beside it.

    python bench.py [--steps K] [--warmup W] [--sections single,batched,update,serve,random,tabu]

Headline (``value``): one step is one whole annealing run of the single-chain
workload -- set-up of B', Delta, cost and schedule, then all I iterations -- on
inputs already resident in device memory.  The workload is the N=150
asymmetric instance (sparse flows on a 10 x 15 Manhattan grid), I = 1e8,
geometric cooling from T0 = mean |Delta_0| to 1e-3 T0.

Further sections, reported in the same JSON line:
  batched  512 chains over 64 instances of N in [20, 200], I = 1e7 each, in one
           persistent launch; aggregate iterations/s and the ratio to the
           single-chain rate.
  update   the Delta update at N = 2000 (symmetric, Euclidean distances) with
           every proposal accepted (T = +inf): updates/s and the roofline of
           the multi-workgroup kernel against HBM (algorithmic int32 bytes per
           update: 4N(N-1) for Delta read + write, 8N^2 for A and B' read once).
  serve    a prefix of the served trace (Poisson 200 req/s, N log-uniform in
           [32, 512], I = 1e7): p50/p99 latency and aggregate iterations/s.
  random   the single-chain workload with the pairs proposed at random instead
           of in row-major order: iterations/s, parity against the oracle's
           stored full run, and the oracle timed on a prefix of the same run.
  tabu     tabu search on the single-chain instance (tenure N): iterations/s
           (one swap each), the first iterations checked against the oracle's
           tabu search, which is timed on them.
Prints one JSON line.
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

HBM_PEAK_GBS = 8000.0
TRAFFIC_JSON = os.path.join(ROOT, "profiles", "k_chain_dist_update_n2000_traffic.json")
DIST_SOURCE = os.path.join(ROOT, "paper_1208_2675_amd", "csrc", "qapsa_chain_dist.hip")


def source_hash(path: str) -> str:
    import hashlib
    with open(path, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def measured_traffic(per_update_bytes: int):
    """HBM bytes per Delta update from the committed counter summary, if it was
    taken on the current source of the kernel; else None."""
    if not os.path.exists(TRAFFIC_JSON):
        return None
    with open(TRAFFIC_JSON) as f:
        t = json.load(f)
    if t.get("source_sha256_16") != source_hash(DIST_SOURCE):
        return None
    return {"fetch_bytes_per_update": t["fetch_bytes_per_update"], "write_bytes_per_update": t["write_bytes_per_update"],
            "bytes_per_update": t["fetch_bytes_per_update"] + t["write_bytes_per_update"],
            "vs_algorithmic": (t["fetch_bytes_per_update"] + t["write_bytes_per_update"]) / per_update_bytes,
            "copy_scale": t["copy_scale"], "summary": os.path.relpath(TRAFFIC_JSON, ROOT)}


def update_bytes(n: int, symmetric: bool) -> int:
    """Algorithmic bytes of one Delta update, int32 entries: read and write the
    n(n-1)/2 packed entries; read A and B' once (rows and columns when asymmetric)."""
    return 4 * n * (n - 1) + (8 if symmetric else 16) * n * n


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def cpu_baseline(ch, iters_sample: int, order: int = 0) -> dict:
    import oracle
    oracle.build()
    s = oracle.schedule(ch.A, ch.B, ch.p0, ch.iters)
    t0 = time.perf_counter()
    r = oracle.sa_run(ch.A, ch.B, ch.p0, ch.iters, s["T0"], s["alpha"], ch.philox_seed, ch.chain_id,
                      t_end=iters_sample, order=order)
    dt = time.perf_counter() - t0
    return {"value": iters_sample / dt, "unit": "iterations/s", "cores": 1, "kind": "oracle",
            "sample": f"first {iters_sample:.0e} iterations of the same schedule, single thread "
                      f"({r['accepts']} accepts, {dt:.1f} s); the oracle computes every proposal's swap cost "
                      f"from scratch, so its cost per iteration does not depend on the acceptance rate"}


def section_tabu(Q, W, torch, args):
    """Tabu search on the single-chain instance: a prefix checked against the
    oracle (and timed there), then the timed search."""
    ch = W.single_chain(args.workload)
    iters, check = args.tabu_iters, args.tabu_check
    log(f"tabu: workload={args.workload} n={ch.n} iters={iters} tenure={ch.n}")
    c = Q.Chain(ch.A, ch.B, ch.p0, iters, ch.philox_seed, ch.chain_id).init()
    c.tabu(check, ch.n)
    st_check = c.state()
    c2 = Q.Chain(ch.A, ch.B, ch.p0, iters, ch.philox_seed, ch.chain_id).init()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    c2.tabu(iters, ch.n)
    st = c2.state()
    wall = time.perf_counter() - t0
    import oracle
    oracle.build()
    t1 = time.perf_counter()
    ref = oracle.tabu_run(ch.A, ch.B, ch.p0, check, ch.n)
    dt = time.perf_counter() - t1
    parity = all(int(getattr(st_check, k)) == ref[k] for k in ("accepts", "hash", "cost", "best_cost", "best_iter"))
    return {"value": iters / wall, "unit": "iterations/s", "iters": iters, "tenure": ch.n, "wall_s": wall,
            "final_cost": int(st.cost), "best_cost": int(st.best_cost),
            "parity_vs_oracle": parity, "parity_prefix_iters": check,
            "timed": "one search of all iterations on resident inputs (set-up excluded)",
            "cpu_baseline": {"value": check / dt, "unit": "iterations/s", "cores": 1, "kind": "oracle",
                             "sample": f"first {check} iterations of the same search, single thread ({dt:.1f} s); "
                                       f"every swap cost recomputed in O(N) per iteration"}}


def section_random(Q, W, torch, args):
    """The single-chain workload with random proposal order: one timed run."""
    ch = W.single_chain(args.workload)
    log(f"random: workload={args.workload} n={ch.n} iters={ch.iters}")
    c = Q.Chain(ch.A, ch.B, ch.p0, ch.iters, ch.philox_seed, ch.chain_id, flags=Q.QAP_FLAG_RANDOM_ORDER).init()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    c.run()
    st = c.state()
    wall = time.perf_counter() - t0
    parity = None
    gold_path = os.path.join(ROOT, "tests", "golden", "oracle_runs.json")
    g = json.load(open(gold_path)).get(f"{args.workload}@{ch.iters}:random") if os.path.exists(gold_path) else None
    if g:
        parity = all(int(getattr(st, k)) == g[k] for k in ("accepts", "hash", "cost", "best_cost")) and \
            c.p.cpu().numpy().tolist() == g["p"]
    out = {"value": ch.iters / wall, "unit": "iterations/s", "wall_s": wall, "accepts": int(st.accepts),
           "delta_updates_per_s": int(st.accepts) / wall, "final_cost": int(st.cost),
           "parity_vs_oracle": parity, "timed": "one run of all I iterations on resident inputs (set-up excluded)"}
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(ch, min(args.cpu_sample // 3, ch.iters), order=1)
    return out


def section_single(Q, W, torch, args):
    ch = W.single_chain(args.workload)
    log(f"single: workload={args.workload} n={ch.n} iters={ch.iters}")
    c = Q.Chain(ch.A, ch.B, ch.p0, ch.iters, ch.philox_seed, ch.chain_id)
    p0 = c.p.clone()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)

    def step():
        c.p.copy_(p0)
        c.init()                      # B', Delta_0, cost, T0, cooling tables (syncs to read T0)
        ev0.record()
        c.run()
        ev1.record()
        st = c.state()                # syncs
        return st, ev0.elapsed_time(ev1)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    results = [step() for _ in range(args.steps)]
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    st = results[-1][0]
    parity = None
    gold_path = os.path.join(ROOT, "tests", "golden", "oracle_runs.json")
    key = f"{args.workload}@{ch.iters}"
    if os.path.exists(gold_path):
        g = json.load(open(gold_path)).get(key)
        if g:
            parity = all(int(getattr(st, k)) == g[k] for k in ("accepts", "hash", "cost", "best_cost")) and \
                c.p.cpu().numpy().tolist() == g["p"]
    # phase split from one profiled run (not timed)
    cp = Q.Chain(ch.A, ch.B, ch.p0, ch.iters, ch.philox_seed, ch.chain_id, profile=True).init().run()
    phases = cp.phases()
    return {
        "ch": ch, "wall": wall, "iters_total": ch.iters * args.steps,
        "accepts_total": sum(int(r[0].accepts) for r in results), "state": st,
        "kernel_ms": sum(r[1] for r in results) / len(results), "parity": parity, "phases": phases,
        "symmetric": bool(c.info.symmetric),
    }


def section_batched(Q, W, torch, args):
    from paper_1208_2675_amd import tune
    chains = W.batched_mix(iters=args.batch_iters)
    fits = [ch for ch in chains
            if Q.fits_one_workgroup(ch.n, ch.symmetric, int(ch.A.max() - ch.A.min()), int(ch.B.max() - ch.B.min()))]
    log(f"batched: {len(fits)} of {len(chains)} chains, I={args.batch_iters:.0e}")
    t_tune = time.perf_counter()
    table = tune.load_or_tune(iters=args.batch_iters, log=log)
    t_tune = time.perf_counter() - t_tune
    b = Q.Batch(fits).init(switch_permille=lambda n, sym: tune.switch_for(table, n, sym))
    # largest expected work first
    import numpy as np
    order = torch.tensor(np.argsort([-(ch.n * ch.n) for ch in fits]).astype(np.int32), device="cuda")
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev0.record()
    b.run(threads=args.batch_threads, order=order)
    ev1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    sts = b.states()
    iters = sum(ch.iters for ch in fits)
    acc = sum(s["accepts"] for s in sts)
    parity = None
    gold_path = os.path.join(ROOT, "tests", "golden", "oracle_runs.json")
    if os.path.exists(gold_path) and len(fits) == len(chains) and args.batch_iters == 10**7:
        gold = json.load(open(gold_path)).get("mix512", {}).get("chains")
        if gold and len(gold) == len(sts):
            parity = all(all(st[k] == g[k] for k in ("accepts", "hash", "cost", "best_cost", "best_iter"))
                         for st, g in zip(sts, gold))
    return {"chains": len(fits), "chains_total": len(chains), "iters": iters, "wall_s": wall,
            "kernel_ms": ev0.elapsed_time(ev1), "value": iters / wall, "delta_updates_per_s": acc / wall,
            "unsupported_chains": len(chains) - len(fits), "tuning_s": round(t_tune, 2),
            "parity_vs_oracle": parity,
            "switch_permille": {f"{x['lo']}-{x['hi']}{'s' if x['symmetric'] else 'a'}": x["switch_permille"]
                                for x in table["buckets"]}}


def calibrate_copy(torch, mib: int = 256):
    """A plain device copy of known size, for scaling the FETCH_SIZE and
    WRITE_SIZE counters (run under rocprofv3 --pmc beside the update)."""
    x = torch.ones(mib << 18, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    torch.cuda.synchronize()
    y.copy_(x)
    torch.cuda.synchronize()
    return {"copy_bytes": mib << 20}


def section_update(Q, W, torch, args):
    """R equal launches of the multi-workgroup kernel, each making K/R forced
    accepts (T = +inf) on the N=2000 chain, after one untimed launch of the
    same size; per-launch durations from HIP events on the stream the kernel
    runs on."""
    ch = W.single_chain("n2000_sym")
    n = ch.n
    launches = args.update_launches
    per = args.update_accepts // launches
    log(f"update: n={n} forced accepts={per * launches} in {launches} launches")
    # one untimed launch of the same size first (first-launch set-up of the
    # cooperative kernel), then the timed ones
    c = Q.Chain(ch.A, ch.B, ch.p0, per * (launches + 1), ch.philox_seed, ch.chain_id, T0=math.inf)
    c.init()
    c.run(per)
    torch.cuda.synchronize()
    ms = []
    for i in range(launches):
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ev0.record()
        c.run((i + 2) * per)
        ev1.record()
        torch.cuda.synchronize()
        ms.append(ev0.elapsed_time(ev1))
    st = c.state()
    avg_ms = sum(ms) / len(ms)
    ups = per / (avg_ms * 1e-3)
    bytes_per = update_bytes(n, True)
    achieved = bytes_per * ups / 1e9
    return {"n": n, "launches": launches, "updates_per_launch": per, "launch_ms": ms, "avg_launch_ms": avg_ms,
            "updates_per_s": ups, "us_per_update": 1e6 / ups, "bytes_per_update": bytes_per,
            "bytes_per_launch": bytes_per * per, "achieved_GBs": achieved, "accepts": int(st.accepts),
            "status": int(st.status)}


def section_serve(Q, W, torch, args):
    from paper_1208_2675_amd.serve import Server
    reqs = W.served_trace(n_requests=args.serve_requests, iters=args.serve_iters)
    log(f"serve: {len(reqs)} requests, I={args.serve_iters:.0e}, slice={args.serve_slice}")
    srv = Server(max_slots=args.serve_slots, memory_budget=args.serve_budget, slice_iters=args.serve_slice)
    st = srv.run_trace(reqs, time_limit=args.serve_time_limit)
    import numpy as np
    lat = np.array([r.latency for r in st.results]) if st.results else np.array([float("nan")])
    return {"requests": len(reqs), "completed": len(st.results), "wall_s": st.wall_s,
            "iterations_per_s": st.iterations / st.wall_s, "p50_latency_s": float(np.percentile(lat, 50)),
            "p99_latency_s": float(np.percentile(lat, 99)), "slices": st.slices,
            "mean_resident": st.resident_sum / max(st.slices, 1), "waits_for_memory": st.waits_for_memory,
            "offered_iterations_per_s": 200.0 * args.serve_iters}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="n150_asym")
    ap.add_argument("--sections", default="single,batched,update,serve,random,tabu")
    ap.add_argument("--tabu-iters", type=int, default=100_000)
    ap.add_argument("--tabu-check", type=int, default=1500)
    ap.add_argument("--cpu-sample", type=int, default=30_000_000)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--batch-iters", type=int, default=10**7)
    ap.add_argument("--batch-threads", type=int, default=256)
    ap.add_argument("--update-accepts", type=int, default=20_000)
    ap.add_argument("--update-launches", type=int, default=4)
    ap.add_argument("--serve-requests", type=int, default=400)
    ap.add_argument("--serve-iters", type=int, default=10**7)
    ap.add_argument("--serve-slice", type=int, default=500_000)
    ap.add_argument("--serve-slots", type=int, default=512)
    ap.add_argument("--serve-budget", type=int, default=64 << 30)
    ap.add_argument("--serve-time-limit", type=float, default=120.0)
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(independent chains shard across GPUs without communication, see the design notes)",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1208_2675_amd import qapsa as Q
    from paper_1208_2675_amd import workloads as W

    sections = set(args.sections.split(","))
    if "single" not in sections:   # partial run (profiling): no headline value
        line = {"metric": "SA iterations/s + Delta-updates/s, 1 GPU: single chain vs batched chains", "value": None,
                "unit": "iterations/s", "n_gpus": 1, "sections": sorted(sections)}
        if "update" in sections:
            line["update_n2000"] = section_update(Q, W, torch, args)
        if "calib" in sections:
            line["copy_calibration"] = calibrate_copy(torch)
        if "batched" in sections:
            line["batched"] = section_batched(Q, W, torch, args)
        if "random" in sections:
            line["random_order"] = section_random(Q, W, torch, args)
        if "tabu" in sections:
            line["tabu"] = section_tabu(Q, W, torch, args)
        print(json.dumps(line))
        return
    s = section_single(Q, W, torch, args)
    ch = s["ch"]
    value = s["iters_total"] / s["wall"]
    line = {
        "metric": "SA iterations/s + Delta-updates/s, 1 GPU: single chain vs batched chains",
        "value": value,
        "unit": "iterations/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": s["wall"] / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32 swap costs, int64 costs, Eq. 2 in f64",
        "data": "synthetic",
        "config": {"workload": f"{args.workload}: single chain, N={ch.n}, I={ch.iters:.0e}, "
                               f"geometric cooling T0=mean|Delta0| -> 1e-3*T0",
                   "n": ch.n, "iters": ch.iters, "symmetric": s["symmetric"], "instance_sha256": ch.meta["sha256"]},
        "delta_updates_per_s": s["accepts_total"] / s["wall"],
        "acceptance_rate": int(s["state"].accepts) / ch.iters,
        "single_chain": {"kernel_ms": s["kernel_ms"], "parity_vs_oracle": s["parity"],
                         "phase_cycles": s["phases"], "clock_hz": 2.4e9},
    }
    if "batched" in sections:
        b = section_batched(Q, W, torch, args)
        b["ratio_vs_single_chain"] = b["value"] / value
        line["batched"] = b
    if "update" in sections:
        u = section_update(Q, W, torch, args)
        line["update_n2000"] = u
        tr = measured_traffic(u["bytes_per_update"])
        line["roofline"] = {"bound": "hbm", "achieved": u["achieved_GBs"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                            "frac": u["achieved_GBs"] / HBM_PEAK_GBS,
                            "traffic": tr["bytes_per_update"] * u["updates_per_s"] / 1e9 if tr else None,
                            "traffic_detail": tr,
                            "kernel": "k_chain_dist (N=2000, every proposal accepted)",
                            "per_unit": f"{u['bytes_per_update']} B per Delta update (int32 algorithmic), "
                                        f"{u['updates_per_launch']} updates per launch",
                            "avg_launch_ms": u["avg_launch_ms"]}
    if "serve" in sections:
        line["serve"] = section_serve(Q, W, torch, args)
    if "random" in sections:
        line["random_order"] = section_random(Q, W, torch, args)
    if "tabu" in sections:
        line["tabu"] = section_tabu(Q, W, torch, args)
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(ch, min(args.cpu_sample, ch.iters))
    print(json.dumps(line))


if __name__ == "__main__":
    main()
