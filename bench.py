"""Benchmark: simulated-annealing iterations/s and accepted-swap Delta-updates/s
of the HIP path on one MI355X, single chain vs batched chains, with CPU
baselines timed on the host in the same run.

    python bench.py [--steps K] [--warmup W] [--sections single,batched,update,serve,random,tabu]
    python bench.py --sections config2 [--c2-budget S] [--c2-state PATH]   # the N=2000 schedule

Headline (``value``): one step is one whole annealing run of the single-chain
workload -- set-up of B', Delta, cost and schedule, then all I iterations -- on
inputs already resident in device memory.  The workload is the N=150
asymmetric instance (sparse flows on a 10 x 15 Manhattan grid), I = 1e8,
geometric cooling from T0 = mean |Delta_0| to 1e-3 T0.

Further sections, reported in the same JSON line:
  batched  512 chains over 64 instances of N in [20, 200], I = 1e7 each, in one
           persistent launch; aggregate iterations/s, and the ratio to the
           same mix's chains run one at a time (a sample of 8 chains, each on
           the single-chain path).
  update   the Delta update at N = 2000 (symmetric, Euclidean distances) with
           every proposal accepted (T = +inf): updates/s and the roofline of
           the multi-workgroup kernel against HBM (algorithmic int32 bytes per
           update: 4N(N-1) for Delta read + write, 8N^2 for A and B' read once);
           parity against the closed form of T = +inf and Eq. (1).
  serve    the served trace (2000 requests, Poisson 200 req/s, N log-uniform
           in [32, 512], I = 1e7): p50/p99 latency, aggregate iterations/s,
           and whether the offered load exceeds what the server sustains.
  random   the single-chain workload with the pairs proposed at random instead
           of in row-major order: iterations/s, parity against the oracle's
           stored full run.
  tabu     tabu search on the single-chain instance (tenure N): iterations/s
           (one swap each), the first iterations checked against the oracle's
           tabu search.
  prefix   (not in the default set) the first --prefix-iters iterations of a
           single-chain workload (--prefix-workload) with chain flags
           --prefix-flags (default 2, scratch mode only), one call: seconds,
           iterations/s and scratch rounds (the run that SQ counters are
           taken on).
  config2  (not in the default set) the N = 2000 symmetric chain over its whole
           schedule of 1e9 iterations in slices of 1e7, resumable across calls
           through a state file: iterations/s, Delta-updates/s and acceptance
           per slice, phase cycles, parity with the oracle's stored run at
           2e7 iterations and the end-of-run invariants (Eq. (1), Delta by
           definition on sampled pairs, B' = B[p][p]).
CPU baselines (single thread for single chains: the plain oracle and the
paper's comparator type, a Delta-matrix SA; one oracle chain per host thread
for the batched and served forms) run during the untimed warm-up steps.
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


def cpu_threads() -> int:
    """Host threads for the all-core CPU baselines: the host's CPU share for one
    GPU (16 threads), less one for the thread that drives the GPU."""
    return max(1, min(16, os.cpu_count() or 1) - 1)


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


def cpu_comparator_baseline(ch) -> dict:
    """The paper's comparator type on one core: the whole schedule of the
    single-chain workload with the CPU Delta-matrix SA (from-scratch swap costs
    while acceptance is high, the Delta matrix afterwards); same trajectory as
    the oracle (tested), so its final state is checked against it here too."""
    import cpu_comparator
    import oracle
    cpu_comparator.build()
    oracle.build()
    s = oracle.schedule(ch.A, ch.B, ch.p0, ch.iters)
    num, den = cpu_comparator.default_switch(ch.n)
    t0 = time.perf_counter()
    r = cpu_comparator.sa_run(ch.A, ch.B, ch.p0, ch.iters, s["T0"], s["alpha"], ch.philox_seed, ch.chain_id)
    dt = time.perf_counter() - t0
    return {"value": ch.iters / dt, "unit": "iterations/s", "cores": 1, "kind": "delta_matrix_comparator",
            "delta_updates_per_s": r["accepts"] / dt, "accepts": r["accepts"], "hash": r["hash"],
            "sample": f"the whole schedule ({ch.iters:.0e} iterations, {dt:.1f} s), single thread; Delta matrix "
                      f"from iteration {r['delta_mode_at']} (acceptance under {num}/{den} over 8192 iterations)"}


def _oracle_chain_prefix(ch, t_end):
    import oracle
    s = oracle.schedule(ch.A, ch.B, ch.p0, ch.iters)
    oracle.sa_run(ch.A, ch.B, ch.p0, ch.iters, s["T0"], s["alpha"], ch.philox_seed, ch.chain_id, t_end=t_end)
    return t_end


def cpu_baseline_many(chains, prefix: int, what: str) -> dict:
    """Independent chains on all host threads: one oracle chain per thread at a
    time (ctypes releases the interpreter lock during each run), each chain run
    over the first ``prefix`` iterations of its schedule; aggregate
    iterations/s over the wall time of the whole sample."""
    import oracle
    from concurrent.futures import ThreadPoolExecutor
    oracle.build()
    k = cpu_threads()
    t0 = time.perf_counter()
    with ThreadPoolExecutor(k) as ex:
        total = sum(ex.map(lambda ch: _oracle_chain_prefix(ch, min(prefix, ch.iters)), chains))
    dt = time.perf_counter() - t0
    return {"value": total / dt, "unit": "iterations/s", "cores": k, "kind": "oracle",
            "sample": f"{what}: {len(chains)} chains, the first {prefix:.0e} iterations of each, one chain per "
                      f"thread on {k} threads ({dt:.1f} s); the oracle's cost per iteration does not depend "
                      f"on the acceptance rate, so a prefix measures its rate"}


def _comparator_chain(ch):
    import cpu_comparator
    import oracle
    s = oracle.schedule(ch.A, ch.B, ch.p0, ch.iters)
    cpu_comparator.sa_run(ch.A, ch.B, ch.p0, ch.iters, s["T0"], s["alpha"], ch.philox_seed, ch.chain_id)
    return ch.iters


def cpu_comparator_many(chains, what: str) -> dict:
    """The paper's comparator type on all host threads: one CPU Delta-matrix
    chain per thread at a time, each over its whole schedule (its cost per
    iteration changes along the schedule, so a prefix would not measure it);
    aggregate iterations/s over the wall time of the sample."""
    import cpu_comparator
    import oracle
    from concurrent.futures import ThreadPoolExecutor
    cpu_comparator.build()
    oracle.build()
    k = cpu_threads()
    t0 = time.perf_counter()
    with ThreadPoolExecutor(k) as ex:
        total = sum(ex.map(_comparator_chain, chains))
    dt = time.perf_counter() - t0
    return {"value": total / dt, "unit": "iterations/s", "cores": k, "kind": "delta_matrix_comparator",
            "sample": f"{what}: {len(chains)} chains, whole schedules (T0 from the oracle's Delta_0, inside "
                      f"the timing), one chain per thread on {k} threads ({dt:.1f} s)"}


class CpuJobs:
    """CPU baselines run one after another on a background thread (each one
    single- or multi-threaded as it states), so that they overlap the untimed
    warm-up steps of the single-chain section instead of adding to the run."""

    def __init__(self):
        import threading
        self.results = {}
        self.jobs = []
        self._threading = threading
        self.thread = None

    def add(self, name, fn):
        self.jobs.append((name, fn))

    def start(self):
        def work():
            for name, fn in self.jobs:
                t0 = time.perf_counter()
                try:
                    self.results[name] = fn()
                except Exception as e:   # reported in the JSON line, never hides a GPU result
                    self.results[name] = {"error": repr(e)}
                log(f"cpu baseline {name}: {time.perf_counter() - t0:.1f} s")
        self.thread = self._threading.Thread(target=work, daemon=True)
        self.thread.start()

    def join(self) -> dict:
        if self.thread is not None:
            self.thread.join()
        return self.results


def tabu_oracle_prefix(ch, check: int) -> dict:
    import oracle
    oracle.build()
    t1 = time.perf_counter()
    ref = oracle.tabu_run(ch.A, ch.B, ch.p0, check, ch.n)
    ref = {k: ref[k] for k in ("accepts", "hash", "cost", "best_cost", "best_iter")}
    return {"ref": ref, "seconds": time.perf_counter() - t1}


def section_tabu(Q, W, torch, args, jobs=None):
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
    job = jobs.get("tabu_oracle") if jobs else None
    if job is None or "error" in job:
        job = tabu_oracle_prefix(ch, check)
    ref, dt = job["ref"], job["seconds"]
    parity = all(int(getattr(st_check, k)) == ref[k] for k in ("accepts", "hash", "cost", "best_cost", "best_iter"))
    return {"value": iters / wall, "unit": "iterations/s", "iters": iters, "tenure": ch.n, "wall_s": wall,
            "final_cost": int(st.cost), "best_cost": int(st.best_cost),
            "parity_vs_oracle": parity, "parity_prefix_iters": check,
            "timed": "one search of all iterations on resident inputs (set-up excluded)",
            "cpu_baseline": {"value": check / dt, "unit": "iterations/s", "cores": 1, "kind": "oracle",
                             "sample": f"first {check} iterations of the same search, single thread ({dt:.1f} s); "
                                       f"every swap cost recomputed in O(N) per iteration"}}


def section_random(Q, W, torch, args, jobs=None):
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
    if jobs and "random_oracle" in jobs:
        out["cpu_baseline"] = jobs["random_oracle"]
    return out


def section_single(Q, W, torch, args, cpu_jobs=None):
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

    for i in range(args.warmup):
        step()
        log(f"single: warm-up step {i + 1}/{args.warmup}")
    torch.cuda.synchronize()
    if cpu_jobs is not None:   # the CPU baselines ran during the warm-up; the timed steps run alone
        cpu_jobs.join()
    t0 = time.perf_counter()
    results = []
    for i in range(args.steps):
        results.append(step())
        log(f"single: step {i + 1}/{args.steps}: {results[-1][1] / 1e3:.3f} s")
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
    phases = None
    if args.phases:   # phase split from one more, profiled run (not timed)
        cp = Q.Chain(ch.A, ch.B, ch.p0, ch.iters, ch.philox_seed, ch.chain_id, profile=True).init().run()
        phases = cp.phases()
    return {
        "ch": ch, "wall": wall, "iters_total": ch.iters * args.steps,
        "accepts_total": sum(int(r[0].accepts) for r in results), "state": st,
        "kernel_ms": sum(r[1] for r in results) / len(results), "parity": parity, "phases": phases,
        "symmetric": bool(c.info.symmetric),
    }


def section_batched(Q, W, torch, args, jobs=None):
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
    out = {"chains": len(fits), "chains_total": len(chains), "iters": iters, "wall_s": wall,
           "kernel_ms": ev0.elapsed_time(ev1), "value": iters / wall, "delta_updates_per_s": acc / wall,
           "unsupported_chains": len(chains) - len(fits), "tuning_s": round(t_tune, 2),
           "parity_vs_oracle": parity,
           "switch_permille": {f"{x['lo']}-{x['hi']}{'s' if x['symmetric'] else 'a'}": x["switch_permille"]
                               for x in table["buckets"]}}
    # the same mix one chain at a time: a sample of chains, each alone on the
    # single-chain path (qap_sa_run with its default kernel choice)
    sample = [fits[i] for i in range(0, len(fits), max(1, len(fits) // args.batch_single_sample))]
    sample = sample[: args.batch_single_sample]
    t_single = 0.0
    for ch in sample:
        sw = tune.switch_for(table, ch.n, ch.symmetric)
        c = Q.Chain(ch.A, ch.B, ch.p0, ch.iters, ch.philox_seed, ch.chain_id, switch_permille=sw).init()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        c.run()
        c.state()
        t_single += time.perf_counter() - t1
    single_rate = sum(ch.iters for ch in sample) / t_single
    out["single_chain_same_mix"] = {
        "value": single_rate, "unit": "iterations/s", "chains": len(sample),
        "n": [ch.n for ch in sample], "symmetric": [bool(ch.symmetric) for ch in sample],
        "how": "each sampled chain of the mix run alone through qap_sa_run (whole schedule, set-up excluded); "
               "iterations over the summed run times"}
    out["ratio_vs_single_chain"] = out["value"] / single_rate
    if jobs and "batched_cpu" in jobs:
        out["cpu_baseline"] = jobs["batched_cpu"]
    if jobs and "batched_cpu_comparator" in jobs:
        out["cpu_baseline_comparator"] = jobs["batched_cpu_comparator"]
    return out


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
    # Delta mode throughout: the update of Sec. 3 is what is timed (scratch mode
    # would otherwise run the whole forced-accept schedule)
    c = Q.Chain(ch.A, ch.B, ch.p0, per * (launches + 1), ch.philox_seed, ch.chain_id, T0=math.inf,
                flags=Q.QAP_FLAG_DELTA_ONLY)
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
    parity = update_parity(ch, c, st, per * (launches + 1))
    out = {"n": n, "launches": launches, "updates_per_launch": per, "launch_ms": ms, "avg_launch_ms": avg_ms,
           "updates_per_s": ups, "us_per_update": 1e6 / ups, "bytes_per_update": bytes_per,
           "bytes_per_launch": bytes_per * per, "achieved_GBs": achieved, "accepts": int(st.accepts),
           "status": int(st.status), "parity": parity}
    if args.phases:   # one more launch of the same size with the phase clock of workgroup 0 (untimed)
        cp = Q.Chain(ch.A, ch.B, ch.p0, per, ch.philox_seed, ch.chain_id, T0=math.inf, profile=True,
                     flags=Q.QAP_FLAG_DELTA_ONLY).init()
        cp.run(per)
        ph = cp.phases()
        out["phase_cycles_per_update"] = {k: round(ph[k] / per, 1) for k in
                                          ("total", "delta_scan", "grid_sync", "delta_update")}
    return out


def _eq1(A, B, p):
    """Eq. (1) by its definition, in int64 (numpy)."""
    import numpy as np
    return int((A.astype(np.int64) * B.astype(np.int64)[np.ix_(p, p)]).sum())


def update_parity(ch, c, st, k):
    """Checks of the forced-accept run: at T = +inf every proposal is accepted,
    so after k iterations p is p0 composed with the first k row-major
    transpositions (closed form); the tracked cost equals Eq. (1) at that p;
    B' equals B[p][p]; sampled Delta entries equal C(p o (r s)) - C(p)."""
    import numpy as np
    n = ch.n
    p = ch.p0.copy()
    r, s = 0, 1
    for _ in range(k):
        p[r], p[s] = p[s], p[r]
        s += 1
        if s == n:
            r += 1
            if r == n - 1:
                r = 0
            s = r + 1
    got = c.result(with_delta=True)
    cost = _eq1(ch.A, ch.B, p)
    rng = np.random.default_rng(5)
    ok_delta = True
    for _ in range(8):
        a, b = sorted(int(x) for x in rng.choice(n, 2, replace=False))
        q = p.copy()
        q[a], q[b] = q[b], q[a]
        idx = a * (2 * n - a - 1) // 2 + b - a - 1
        ok_delta = ok_delta and int(got["delta"][idx]) == _eq1(ch.A, ch.B, q) - cost
    return {"accepts_all": int(st.accepts) == k, "p_closed_form": bool(np.array_equal(got["p"], p)),
            "cost_eq1": int(st.cost) == cost, "bprime": bool(np.array_equal(got["Bp"], ch.B[np.ix_(p, p)])),
            "delta_sampled_8": bool(ok_delta)}


def section_serve(Q, W, torch, args, jobs=None):
    from paper_1208_2675_amd.serve import Server
    reqs = W.served_trace(n_requests=args.serve_requests, iters=args.serve_iters)
    log(f"serve: {len(reqs)} requests, I={args.serve_iters:.0e}, slice={args.serve_slice}")
    srv = Server(max_slots=args.serve_slots, memory_budget=args.serve_budget, slice_iters=args.serve_slice)
    st = srv.run_trace(reqs, time_limit=args.serve_time_limit)
    import numpy as np
    lat = np.array([r.latency for r in st.results]) if st.results else np.array([float("nan")])
    rate = st.iterations / st.wall_s
    offered = 200.0 * args.serve_iters
    arrivals_s = reqs[-1].arrival_s if reqs else 0.0
    out = {"requests": len(reqs), "completed": len(st.results), "wall_s": st.wall_s,
           "iterations_per_s": rate, "p50_latency_s": float(np.percentile(lat, 50)),
           "p99_latency_s": float(np.percentile(lat, 99)), "slices": st.slices,
           "mean_resident": st.resident_sum / max(st.slices, 1), "max_resident": st.max_resident,
           "waits_for_memory": st.waits_for_memory, "waits_for_slot": st.waits_for_slot,
           "offered_iterations_per_s": offered, "arrival_span_s": arrivals_s,
           # the queue grows while arrivals last when the server sustains less
           # than the offered load: latencies are then those of a finite trace
           # served by a saturated server, not a steady state
           "saturated": rate < offered,
           "latency_note": "completion minus arrival over the whole trace; with saturated true they grow "
                           "with the request's position in the trace"}
    if jobs and "serve_cpu" in jobs:
        out["cpu_baseline"] = jobs["serve_cpu"]
    if jobs and "serve_cpu_comparator" in jobs:
        out["cpu_baseline_comparator"] = jobs["serve_cpu_comparator"]
    return out


def section_prefix(Q, W, torch, args):
    """A prefix of one single-chain run with the given flags, one call; the
    phase counters come from a second, identical run (they cost a little)."""
    ch = W.single_chain(args.prefix_workload)
    t_end = min(args.prefix_iters, ch.iters)
    log(f"prefix: workload={args.prefix_workload} n={ch.n} t_end={t_end} flags={args.prefix_flags}")
    c = Q.Chain(ch.A, ch.B, ch.p0, ch.iters, ch.philox_seed, ch.chain_id, flags=args.prefix_flags).init()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    c.run(t_end)
    st = c.state()
    dt = time.perf_counter() - t0
    cp = Q.Chain(ch.A, ch.B, ch.p0, ch.iters, ch.philox_seed, ch.chain_id, flags=args.prefix_flags,
                 profile=True).init()
    cp.run(t_end)
    ph = cp.phases()
    return {"workload": args.prefix_workload, "n": ch.n, "t_end": t_end, "flags": args.prefix_flags, "s": dt,
            "iterations_per_s": t_end / dt, "accepts": int(st.accepts), "hash": int(st.hash),
            "status": int(st.status), "phase_cycles": ph}


def section_config2(Q, W, torch, args):
    """The N = 2000 symmetric chain over its whole schedule (I = 1e9) in
    slices of args.c2_slice iterations, as many as fit args.c2_budget seconds
    in this call.  After every slice p, the chain state and the phase counters
    go to args.c2_state, and a later call given that file (--c2-resume)
    continues from it: qap_delta_init rebuilds B' and Delta at the saved p and
    the saved state is put back, so the run is the one an unbroken call makes."""
    import numpy as np
    ch = W.single_chain("n2000_sym")
    n = ch.n
    c = Q.Chain(ch.A, ch.B, ch.p0, ch.iters, ch.philox_seed, ch.chain_id, profile=True, tie_cap=1024).init()
    slices = []
    if args.c2_resume and os.path.exists(args.c2_resume):
        z = np.load(args.c2_resume)
        c.p.copy_(torch.from_numpy(z["p"].astype(np.int32)).to(c.p.device))
        Q._check(Q.qap_delta_init(n, c.A, c.B, c.p, c.Bp, c.delta, c.info_d, None), "qap_delta_init")
        c.state_d.copy_(torch.from_numpy(z["state"].astype(np.uint8)).to(c.p.device))
        c.prof.copy_(torch.from_numpy(z["prof"].astype(np.int64)).to(c.p.device))
        slices = json.loads(str(z["slices"]))
        torch.cuda.synchronize()
    gold_path = os.path.join(ROOT, "tests", "golden", "oracle_runs.json")
    gold = json.load(open(gold_path)) if os.path.exists(gold_path) else {}
    prefix_keys = sorted((int(k.split("@")[1]), k) for k in gold
                         if k.startswith("n2000_sym@") and ":" not in k)
    t = int(c.state().t)
    log(f"config2: n={n} I={ch.iters:.0e} from t={t}, budget {args.c2_budget:.0f} s")
    T = time.perf_counter()
    prev = c.phases()
    prev_acc = int(c.state().accepts)
    prefix_parity = {}
    while t < ch.iters and time.perf_counter() - T < args.c2_budget:
        t_end = min(t + args.c2_slice, ch.iters)
        for tp, key in prefix_keys:   # stop at a stored oracle prefix to compare with it
            if t < tp < t_end:
                t_end = tp
                break
        t0 = time.perf_counter()
        c.run(t_end)
        st = c.state()
        dt = time.perf_counter() - t0
        if st.status != 0:
            raise Q.QapError(st.status, f"config2 slice ending at {t_end}")
        ph = c.phases()
        d = {k: ph[k] - prev[k] for k in ph}
        prev = ph
        acc = int(st.accepts) - prev_acc
        prev_acc = int(st.accepts)
        slices.append({"t_end": t_end, "iters": t_end - t, "s": round(dt, 4), "accepts": acc,
                       "acceptance": acc / (t_end - t), "cost": int(st.cost),
                       "scan_steps": d["n_scan_steps"], "scanned": d["n_scanned"],
                       "cycles_scan": d["delta_scan"], "cycles_sync": d["grid_sync"],
                       "cycles_update": d["delta_update"], "scratch_windows": d["n_rounds"],
                       "scratch_accepts": d["n_scratch_acc"], "cycles_scratch_eval": d["scratch_eval"],
                       "cycles_scratch_accept": d["scratch_accept"]})
        t = t_end
        for tp, key in prefix_keys:
            if t == tp:
                g = gold[key]
                r = c.result()
                prefix_parity[key] = all(int(getattr(st, k)) == g[k] for k in
                                         ("accepts", "hash", "cost", "best_cost", "best_iter", "near_ties")) \
                    and r["p"].tolist() == g["p"]
                log(f"config2: parity with the oracle at t={tp}: {prefix_parity[key]}")
        log(f"config2: t={t:.3e} {dt:.2f} s accepts={acc} ({acc / slices[-1]['iters']:.4f}) cost={int(st.cost)}")
        if args.c2_state:
            os.makedirs(os.path.dirname(os.path.abspath(args.c2_state)), exist_ok=True)
            tmp = args.c2_state + ".tmp.npz"
            np.savez(tmp, p=c.p.cpu().numpy(), state=c.state_d.cpu().numpy(), prof=c.prof.cpu().numpy(),
                     slices=json.dumps(slices))
            os.replace(tmp, args.c2_state)
    st = c.state()
    secs = sum(x["s"] for x in slices)
    iters_done = sum(x["iters"] for x in slices)
    out = {"n": n, "iters": ch.iters, "t": int(st.t), "complete": int(st.t) == ch.iters,
           "seconds": secs, "iterations_per_s": iters_done / secs if secs else None,
           "delta_updates_per_s": sum(x["accepts"] for x in slices) / secs if secs else None,
           "accepts": int(st.accepts), "acceptance_rate": int(st.accepts) / max(int(st.t), 1),
           "cost": int(st.cost), "best_cost": int(st.best_cost), "near_ties": int(st.near_ties),
           "prefix_parity": prefix_parity, "phase_cycles": c.phases(), "slices": slices}
    if int(st.t) == ch.iters:   # end-of-run invariants
        r = c.result(with_delta=True)
        p = r["p"]
        cost = _eq1(ch.A, ch.B, p)
        rng = np.random.default_rng(9)
        ok = True
        for _ in range(16):
            a, b = sorted(int(x) for x in rng.choice(n, 2, replace=False))
            q = p.copy()
            q[a], q[b] = q[b], q[a]
            ok = ok and int(r["delta"][a * (2 * n - a - 1) // 2 + b - a - 1]) == _eq1(ch.A, ch.B, q) - cost
        out["final_checks"] = {"cost_eq1": int(st.cost) == cost, "delta_sampled_16": bool(ok),
                               "bprime": bool(np.array_equal(r["Bp"], ch.B[np.ix_(p, p)])),
                               "perm": sorted(p.tolist()) == list(range(n))}
    return out


def make_cpu_jobs(W, args, sections) -> CpuJobs:
    """The CPU baselines of the sections asked for (none with --no-cpu-baseline)."""
    jobs = CpuJobs()
    if args.no_cpu_baseline:
        return jobs
    ch = W.single_chain(args.workload)
    if "single" in sections:
        jobs.add("single_oracle", lambda: cpu_baseline(ch, min(args.cpu_sample, ch.iters)))
        if not args.no_comparator:
            jobs.add("single_comparator", lambda: cpu_comparator_baseline(ch))
    if "random" in sections:
        jobs.add("random_oracle", lambda: cpu_baseline(ch, min(args.cpu_sample // 3, ch.iters), order=1))
    if "tabu" in sections:
        jobs.add("tabu_oracle", lambda: tabu_oracle_prefix(ch, args.tabu_check))
    if "batched" in sections:
        mix = W.batched_mix(iters=args.batch_iters)
        sample = mix[:: max(1, len(mix) // 64)][:64]   # one chain per instance
        jobs.add("batched_cpu", lambda: cpu_baseline_many(sample, args.cpu_prefix_batched,
                                                          "one chain of each of the mix's 64 instances"))
        if not args.no_comparator:
            jobs.add("batched_cpu_comparator", lambda: cpu_comparator_many(
                sample, "one chain of each of the mix's 64 instances"))
    if "serve" in sections:
        reqs = W.served_trace(n_requests=args.serve_requests, iters=args.serve_iters)
        sample = [q.chain for q in reqs[:: max(1, len(reqs) // 64)][:64]]
        jobs.add("serve_cpu", lambda: cpu_baseline_many(sample, args.cpu_prefix_serve,
                                                        "every k-th request of the served trace"))
        if not args.no_comparator:
            jobs.add("serve_cpu_comparator", lambda: cpu_comparator_many(
                sample, "every k-th request of the served trace"))
    return jobs


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="n150_asym")
    ap.add_argument("--sections", default="single,batched,update,serve,random,tabu")
    ap.add_argument("--phases", action="store_true", help="one more single-chain run with phase counters")
    ap.add_argument("--tabu-iters", type=int, default=100_000)
    ap.add_argument("--tabu-check", type=int, default=1500)
    ap.add_argument("--cpu-sample", type=int, default=30_000_000)
    ap.add_argument("--cpu-prefix-batched", type=int, default=2_000_000)
    ap.add_argument("--cpu-prefix-serve", type=int, default=400_000)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-comparator", action="store_true")
    ap.add_argument("--batch-iters", type=int, default=10**7)
    ap.add_argument("--batch-threads", type=int, default=256)
    ap.add_argument("--batch-single-sample", type=int, default=8)
    ap.add_argument("--update-accepts", type=int, default=20_000)
    ap.add_argument("--update-launches", type=int, default=4)
    ap.add_argument("--serve-requests", type=int, default=2000)
    ap.add_argument("--serve-iters", type=int, default=10**7)
    ap.add_argument("--serve-slice", type=int, default=500_000)
    ap.add_argument("--serve-slots", type=int, default=512)
    ap.add_argument("--serve-budget", type=int, default=64 << 30)
    ap.add_argument("--serve-time-limit", type=float, default=150.0)
    ap.add_argument("--c2-budget", type=float, default=900.0, help="seconds of config2 slices in this call")
    ap.add_argument("--c2-state", default="gpurun_out/config2_state.npz", help="state file written after each slice")
    ap.add_argument("--c2-resume", default=None, help="state file of an earlier call to continue from")
    ap.add_argument("--c2-slice", type=int, default=10_000_000)
    ap.add_argument("--prefix-workload", default="n150_asym")
    ap.add_argument("--prefix-iters", type=int, default=2_000_000)
    ap.add_argument("--prefix-flags", type=int, default=2)
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
    jobs = make_cpu_jobs(W, args, sections)
    jobs.start()
    if "single" not in sections:   # partial run (profiling): no headline value
        line = {"metric": "SA iterations/s + Delta-updates/s, 1 GPU: single chain vs batched chains", "value": None,
                "unit": "iterations/s", "n_gpus": 1, "sections": sorted(sections)}
        res = jobs.join()
        if "update" in sections:
            line["update_n2000"] = section_update(Q, W, torch, args)
        if "calib" in sections:
            line["copy_calibration"] = calibrate_copy(torch)
        if "batched" in sections:
            line["batched"] = section_batched(Q, W, torch, args, res)
        if "serve" in sections:
            line["serve"] = section_serve(Q, W, torch, args, res)
        if "random" in sections:
            line["random_order"] = section_random(Q, W, torch, args, res)
        if "tabu" in sections:
            line["tabu"] = section_tabu(Q, W, torch, args, res)
        if "prefix" in sections:
            line["prefix"] = section_prefix(Q, W, torch, args)
        if "config2" in sections:
            line["config2"] = section_config2(Q, W, torch, args)
        print(json.dumps(line))
        return
    s = section_single(Q, W, torch, args, jobs)
    res = jobs.join()
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
        line["batched"] = section_batched(Q, W, torch, args, res)
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
        line["serve"] = section_serve(Q, W, torch, args, res)
    if "random" in sections:
        line["random_order"] = section_random(Q, W, torch, args, res)
    if "tabu" in sections:
        line["tabu"] = section_tabu(Q, W, torch, args, res)
    if "single_oracle" in res:
        line["cpu_baseline"] = res["single_oracle"]
    if "single_comparator" in res:
        cmpb = res["single_comparator"]
        if "error" not in cmpb and s["parity"] is not None:
            cmpb["same_trajectory_as_gpu"] = cmpb.pop("hash") == int(s["state"].hash)
        line["cpu_baseline_comparator"] = cmpb
        if "value" in cmpb and "value" in line.get("cpu_baseline", {}):
            line["cpu_baseline_fastest"] = max(("oracle", line["cpu_baseline"]["value"]),
                                               ("delta_matrix_comparator", cmpb["value"]), key=lambda x: x[1])
    print(json.dumps(line))


if __name__ == "__main__":
    main()
