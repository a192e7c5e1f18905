"""Autotuner of the batched form: the scratch-to-Delta switch threshold of a
chain, per instance-size bucket and symmetry.

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
