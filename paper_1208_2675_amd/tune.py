"""Autotuners: the scratch-to-Delta switch threshold of a batched chain, and
the kernel and scan window of a single chain, per instance size and symmetry.

A chain computes each proposal's swap cost from scratch (O(N) per proposal,
nothing to update after a swap) while its acceptance rate is high, and keeps
the Delta matrix of Sec. 2.2 (O(1) per proposal, O(N^2) per accepted swap)
once the rate over a window of 8192 iterations falls below a threshold given
in per mille.  Where the crossover lies depends on N and on symmetry (the
asymmetric form has twice the dot products per swap cost).  The tuner runs,
for every bucket, one representative chain per candidate threshold through a
whole schedule on the device, keeps the fastest and caches the table as JSON
next to the library, keyed by device name and schedule length.  The
threshold changes the time of a run, never its result.

The dispatch tuner covers single chains past the size where one workgroup
holds everything in LDS: it times one workgroup (QAP_FLAG_SINGLE_WG, the byte
matrices in device memory) against the multi-workgroup kernel
(QAP_FLAG_MULTI_WG), each with several scan windows (the adjustable subset
size of Sec. 3 (ii)), over a whole schedule of a representative chain of each
size and symmetry, and keeps the fastest (kernel, window) per entry in
``tuned_dispatch.json``, keyed like the threshold table.  These choices too
change only the time of a run.
"""
from __future__ import annotations

import json
import os
import time

from . import qapsa as Q
from . import workloads as W

BUCKETS = ((20, 60), (60, 100), (100, 140), (140, 200))
CANDIDATES = (5, 10, 20, 40, 80)
CACHE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuned_switch.json")
DISPATCH_CACHE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuned_dispatch.json")
DISPATCH_SIZES = (200, 300, 450, 700, 1000)
DISPATCH_WINDOWS = (1024, 4096, 16384)
FLAG_SINGLE_WG, FLAG_MULTI_WG = 16, 4   # qap_schedule.flags


def _representative(lo: int, hi: int, symmetric: bool, iters: int) -> W.Chain:
    n = (lo + hi) // 2
    if symmetric:
        A, B = W.sym_uniform(n, (90, n))
    else:
        A, B = W.asym_sparse_grid(n, (91, n))
    return W.Chain(f"tune{n}{'s' if symmetric else 'a'}", A, B, W.random_perm(n, (92, n)), iters,
                   W.philox_key(93, n), 0, symmetric, {})


def _time_run(ch: W.Chain, switch_permille: int) -> float:
    import torch
    c = Q.Chain(ch.A, ch.B, ch.p0, ch.iters, ch.philox_seed, ch.chain_id, switch_permille=switch_permille).init()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    c.run()
    torch.cuda.synchronize()
    return time.perf_counter() - t0


def tune(iters: int = 10**7, buckets=BUCKETS, candidates=CANDIDATES, log=None) -> dict:
    """Time every candidate on every bucket; returns the table."""
    table = {"iters": iters, "buckets": []}
    for lo, hi in buckets:
        for sym in (True, False):
            ch = _representative(lo, hi, sym, iters)
            times = {c: _time_run(ch, c) for c in candidates}
            best = min(times, key=times.get)
            table["buckets"].append({"lo": lo, "hi": hi, "symmetric": sym, "switch_permille": best,
                                     "seconds": {str(k): round(v, 4) for k, v in times.items()}})
            if log:
                log(f"tune: n in [{lo},{hi}) sym={sym}: {best} permille ({times[best]:.3f} s)")
    return table


def _device_key(iters: int) -> str:
    """Architecture (e.g. gfx950) and schedule length: the marketing name a
    device reports can change with the runtime's environment, the ISA cannot."""
    import torch
    props = torch.cuda.get_device_properties(0)
    arch = getattr(props, "gcnArchName", "") or torch.cuda.get_device_name(0)
    return f"{arch.split(':')[0]}|{iters}"


def load_or_tune(iters: int = 10**7, path: str = CACHE, log=None, retune: bool = False) -> dict:
    """The cached table for this device and schedule length, tuning on a miss."""
    key = _device_key(iters)
    cache = {}
    if os.path.exists(path):
        with open(path) as f:
            cache = json.load(f)
    if key in cache and not retune:
        return cache[key]
    table = tune(iters, log=log)
    cache[key] = table
    with open(path, "w") as f:
        json.dump(cache, f, indent=1, sort_keys=True)
    return table


def switch_for(table: dict | None, n: int, symmetric: bool, default: int = 10) -> int:
    """Threshold for a chain of size n (the nearest bucket's)."""
    if not table:
        return default
    best, dist = default, None
    for b in table["buckets"]:
        if b["symmetric"] != symmetric:
            continue
        d = -1 if b["lo"] <= n < b["hi"] else min(abs(n - b["lo"]), abs(n - b["hi"]))
        if dist is None or d < dist:
            best, dist = b["switch_permille"], d
    return best


# ----------------------------------------------------------------- dispatch

def _dispatch_chain(n: int, symmetric: bool, iters: int) -> W.Chain:
    if symmetric:
        A, B = W.sym_uniform(n, (94, n))
    else:
        A, B = W.asym_sparse_grid(n, (95, n))
    return W.Chain(f"disp{n}{'s' if symmetric else 'a'}", A, B, W.random_perm(n, (96, n)), iters,
                   W.philox_key(97, n), 0, symmetric, {})


def _time_dispatch(ch: W.Chain, flags: int, window: int) -> tuple[float, int]:
    import torch
    c = Q.Chain(ch.A, ch.B, ch.p0, ch.iters, ch.philox_seed, ch.chain_id, flags=flags, scan_window=window).init()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    c.run()
    st = c.state()
    return time.perf_counter() - t0, int(st.hash)


def tune_dispatch(iters: int = 2 * 10**6, sizes=DISPATCH_SIZES, windows=DISPATCH_WINDOWS, log=None) -> dict:
    """Time (kernel, window) for a representative chain of every size and
    symmetry over a whole schedule of ``iters`` iterations; every option must
    give the same run (the hash is compared)."""
    table = {"iters": iters, "entries": []}
    for n in sizes:
        for sym in (True, False):
            ch = _dispatch_chain(n, sym, iters)
            secs, hashes = {}, set()
            for kind, flags in (("single", FLAG_SINGLE_WG), ("multi", FLAG_MULTI_WG)):
                for w in windows:
                    dt, h = _time_dispatch(ch, flags, w)
                    secs[f"{kind}:{w}"] = round(dt, 4)
                    hashes.add(h)
            if len(hashes) != 1:
                raise RuntimeError(f"dispatch options disagree at n={n} sym={sym}")
            best = min(secs, key=secs.get)
            kind, w = best.split(":")
            table["entries"].append({"n": n, "symmetric": sym, "seconds": secs,
                                     "flags": FLAG_SINGLE_WG if kind == "single" else FLAG_MULTI_WG,
                                     "scan_window": int(w), "kernel": kind})
            if log:
                log(f"tune dispatch: n={n} sym={sym}: {best} ({secs[best]:.3f} s)")
    return table


def load_or_tune_dispatch(iters: int = 2 * 10**6, path: str = DISPATCH_CACHE, log=None, retune: bool = False) -> dict:
    key = _device_key(iters)
    cache = {}
    if os.path.exists(path):
        with open(path) as f:
            cache = json.load(f)
    if key in cache and not retune:
        return cache[key]
    table = tune_dispatch(iters, log=log)
    cache[key] = table
    with open(path, "w") as f:
        json.dump(cache, f, indent=1, sort_keys=True)
    return table


def dispatch_for(table: dict | None, n: int, symmetric: bool) -> tuple[int, int]:
    """(qap_schedule.flags bits, scan_window) for a chain of size n: the
    measured entry of the same symmetry nearest in size; (0, 0), the
    library's own choice, without a table or below the smallest measured size
    (where one workgroup holds the chain in LDS)."""
    if not table or not table.get("entries"):
        return 0, 0
    same = [e for e in table["entries"] if e["symmetric"] == symmetric]
    if not same or n < min(e["n"] for e in same) * 3 // 4:
        return 0, 0
    e = min(same, key=lambda e: (abs(e["n"] - n), e["n"]))
    return int(e["flags"]), int(e["scan_window"])
