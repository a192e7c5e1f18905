"""Write tests/golden/oracle_runs.json: expected results of full-size runs,
computed by the CPU oracle only (nothing here touches the device library).

    python tests/golden/make_golden.py                 # single-chain workloads
    python tests/golden/make_golden.py --only n150_asym@100000000:random   # some of them
    python tests/golden/make_golden.py --mix --no-single   # the 512-chain mix (minutes, all cores)

Each entry records the schedule (T0 = mean |Delta_0|, alpha), the final state
(accepts, trajectory hash of the accepted swaps, cost, best cost and its
iteration), the final permutation (single chains) and the near ties of Eq. (2).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time
from concurrent.futures import ProcessPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_1208_2675_amd import workloads as W  # noqa: E402

OUT = os.path.join(HERE, "oracle_runs.json")

# (workload, t_end or None for the whole schedule, proposal order: 0 row-major, 1 random)
SINGLE = [("n32_sym", None, 0), ("n150_asym", None, 0), ("n150_asym", 3_000_000, 0), ("n2000_sym", 2_000_000, 0),
          ("n150_asym", None, 1), ("n2000_sym", 300_000, 1), ("n2000_sym", 20_000_000, 0),
          ("n2000_asym", 300_000, 0)]


def key_of(name, t_end, order) -> str:
    return f"{name}@{t_end}" + (":random" if order else "")


def run_chain(A, B, p0, iters, seed, chain_id, t_end=None, order=0) -> dict:
    s = oracle.schedule(A, B, p0, iters)
    t0 = time.time()
    r = oracle.sa_run(A, B, p0, iters, s["T0"], s["alpha"], seed, chain_id, t_end=t_end, tie_cap=1024, order=order)
    assert r["cost"] == oracle.cost(A, B, r["p"])
    return {"iters": iters, "t_end": r["t"], "T0": s["T0"], "alpha": s["alpha"], "sum_abs_delta0": s["sum_abs"],
            "cost0": oracle.cost(A, B, p0), "accepts": r["accepts"], "hash": r["hash"], "cost": r["cost"],
            "best_cost": r["best_cost"], "best_iter": r["best_iter"], "near_ties": r["near_ties"],
            "near_tie_t": [int(x) for x in r["near_tie_t"]], "p": [int(x) for x in r["p"]],
            "oracle_seconds": round(time.time() - t0, 2)}


def _single(item):
    name, t_end, order = item
    ch = W.single_chain(name)
    res = run_chain(ch.A, ch.B, ch.p0, ch.iters, ch.philox_seed, ch.chain_id, t_end, order)
    res["sha256"] = ch.meta["sha256"]
    res["order"] = "random" if order else "row-major"
    return key_of(name, res["t_end"], order), res


def _mix_chain(c):
    ch = _MIX[c]
    res = run_chain(ch.A, ch.B, ch.p0, ch.iters, ch.philox_seed, ch.chain_id)
    res.pop("p")
    return c, res


_MIX = None


def main():
    global _MIX
    ap = argparse.ArgumentParser()
    ap.add_argument("--mix", action="store_true")
    ap.add_argument("--no-single", action="store_true")
    ap.add_argument("--jobs", type=int, default=min(8, os.cpu_count() or 1))
    ap.add_argument("--only", nargs="*", default=None, help="keys of the single-chain entries to (re)compute")
    args = ap.parse_args()
    oracle.build()
    data = json.load(open(OUT)) if os.path.exists(OUT) else {}
    with ProcessPoolExecutor(args.jobs) as ex:
        todo = [] if args.no_single else [
            it for it in SINGLE
            if args.only is None or key_of(it[0], it[1] or W.single_chain(it[0]).iters, it[2]) in args.only]
        for key, res in ex.map(_single, todo):
            data[key] = res
            print(key, res["accepts"], res["cost"], res["oracle_seconds"], flush=True)
    if args.mix:
        _MIX = W.batched_mix()
        with ProcessPoolExecutor(args.jobs) as ex:
            mix = dict(ex.map(_mix_chain, range(len(_MIX)), chunksize=4))
        data["mix512"] = {"chains": [mix[c] for c in range(len(_MIX))]}
        print("mix512 done", flush=True)
    with open(OUT, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)


if __name__ == "__main__":
    main()
