"""Serving loop: continuous batching of annealing requests in iteration slices.

Requests (an instance, a start permutation, a schedule length I and a seed)
arrive over time.  The server keeps every admitted request's A, B, B', Delta, p,
cooling tables and chain state resident in device memory and advances all of
them together, one slice of iterations per launch:

* admission: a waiting request is admitted when a slot is free and its device
  footprint fits the memory budget; admission runs step (a) of Sec. 2.2 for it
  (B', Delta, cost, T0, cooling tables) and adds it to the resident set;
* slice: one ``qap_sa_run_batch`` launch advances every resident chain that a
  single workgroup can hold by ``slice_iters`` iterations; larger symmetric
  requests advance by the same slice through ``qap_sa_run`` (one cooperative
  multi-workgroup launch each) on the same stream;
* retire: chains that reached I are read back, their latency (completion
  minus arrival) recorded, and their memory and slot released.

Because a chain's trajectory depends only on (instance, p0, I, seed) -- the
random draw and temperature of iteration t are functions of t -- a request's
result is the same whether it runs alone or in any mix and whatever the slice
boundaries.  That is the tolerance: zero.
"""
from __future__ import annotations

import ctypes as C
import time
from dataclasses import dataclass, field

import numpy as np

from . import qapsa as Q


def footprint_bytes(n: int, iters: int) -> int:
    """Device bytes one resident request holds."""
    m = n * (n - 1) // 2
    return (3 * n * n * 4 + 4 * max(m, 1) + 4 * n + Q.INFO_BYTES + Q.STATE_BYTES
            + 8 * Q.qap_temp_table_len(iters) + Q.qap_workspace_bytes(n))


@dataclass
class Resident:
    rid: int
    chain: object
    arrival: float
    admitted: float
    bufs: dict
    desc: Q.ChainDesc
    wide: bool          # needs the multi-workgroup kernel
    sched: Q.Schedule | None = None
    info: Q.InstanceInfo | None = None


@dataclass
class Result:
    rid: int
    n: int
    arrival: float
    admitted: float
    done: float
    state: dict
    p: np.ndarray

    @property
    def latency(self) -> float:
        return self.done - self.arrival


@dataclass
class ServerStats:
    slices: int = 0
    iterations: int = 0
    busy_s: float = 0.0
    resident_sum: int = 0
    max_resident: int = 0
    admitted: int = 0
    waits_for_memory: int = 0
    waits_for_slot: int = 0
    results: list = field(default_factory=list)


class Server:
    def __init__(self, max_slots: int = 512, memory_budget: int = 8 << 30, slice_iters: int = 250_000,
                 threads: int = 256, device: str = "cuda", ratio: float = 1e-3):
        import torch
        self.torch = torch
        self.dev = torch.device(device)
        self.max_slots = max_slots
        self.budget = memory_budget
        self.slice = slice_iters
        self.threads = threads
        self.ratio = ratio
        self.waiting: list = []          # (arrival, rid, chain)
        self.resident: list[Resident] = []
        self.used = 0
        self.stats = ServerStats()
        self.ws = torch.zeros(Q.qap_batch_workspace_bytes(), dtype=torch.uint8, device=self.dev)
        self._descs_dirty = True
        self._descs_host = None
        self._descs_dev = None

    # -------------------------------------------------------------- requests
    def submit(self, rid: int, chain, arrival: float):
        self.waiting.append((arrival, rid, chain))

    def _admit_one(self, arrival: float, rid: int, ch, now: float) -> Resident:
        torch = self.torch
        n, dev = ch.n, self.dev
        m = max(n * (n - 1) // 2, 1)
        b = {
            "A": torch.from_numpy(np.ascontiguousarray(ch.A, dtype=np.int32)).to(dev),
            "B": torch.from_numpy(np.ascontiguousarray(ch.B, dtype=np.int32)).to(dev),
            "Bp": torch.empty(n * n, dtype=torch.int32, device=dev),
            "p": torch.from_numpy(np.ascontiguousarray(ch.p0, dtype=np.int32)).to(dev),
            "delta": torch.empty(m, dtype=torch.int32, device=dev),
            "info": torch.zeros(Q.INFO_BYTES, dtype=torch.uint8, device=dev),
            "state": torch.zeros(Q.STATE_BYTES, dtype=torch.uint8, device=dev),
            "temps": torch.empty(Q.qap_temp_table_len(ch.iters), dtype=torch.float64, device=dev),
            "ws": torch.zeros(Q.qap_workspace_bytes(n), dtype=torch.uint8, device=dev),
            "ties": torch.zeros(16 * Q.TIE_BYTES, dtype=torch.uint8, device=dev),
        }
        Q._check(Q.qap_delta_init(n, b["A"], b["B"], b["p"], b["Bp"], b["delta"], b["info"], b["state"]),
                 "qap_delta_init")
        torch.cuda.synchronize()
        info = Q._struct_from(b["info"], Q.InstanceInfo)
        if info.status != Q.QAP_OK:
            raise Q.QapError(info.status, f"request {rid}")
        sched = Q.schedule_for(n, info, ch.iters, self.ratio)
        sched.t_end = 0
        sched.seed = ch.philox_seed & (2**64 - 1)
        sched.chain_id = ch.chain_id
        T0 = sched.T0
        Q._check(Q.qap_schedule_tables(ch.iters, sched.alpha, b["temps"]), "qap_schedule_tables")
        ra, rb = info.a_max - info.a_min, info.b_max - info.b_min
        wide = not Q.fits_one_workgroup(n, bool(info.symmetric), ra, rb)
        scr = b["ws"].data_ptr() if Q.needs_scratch(n, bool(info.symmetric), ra, rb) else None
        desc = Q.ChainDesc(n, info.symmetric, info.a_min, info.a_max, info.b_min, info.b_max, 0, 0,
                           b["A"].data_ptr(), b["Bp"].data_ptr(), b["p"].data_ptr(), b["delta"].data_ptr(),
                           b["state"].data_ptr(), b["temps"].data_ptr(), b["ties"].data_ptr(), 16,
                           ch.chain_id, ch.iters, ch.iters, T0, ch.philox_seed & (2**64 - 1), scr)
        r = Resident(rid, ch, arrival, now, b, desc, wide)
        r.info = info
        r.sched = sched
        return r

    def admit(self, now: float):
        self.waiting.sort(key=lambda x: x[0])
        keep = []
        for arrival, rid, ch in self.waiting:
            if arrival > now:
                keep.append((arrival, rid, ch))
                continue
            need = footprint_bytes(ch.n, ch.iters)
            if len(self.resident) >= self.max_slots:
                self.stats.waits_for_slot += 1
                keep.append((arrival, rid, ch))
                continue
            if self.used + need > self.budget:
                self.stats.waits_for_memory += 1
                keep.append((arrival, rid, ch))
                continue
            self.resident.append(self._admit_one(arrival, rid, ch, now))
            self.used += need
            self.stats.admitted += 1
            self._descs_dirty = True
        self.waiting = keep

    # ----------------------------------------------------------------- slices
    def _narrow(self):
        return [r for r in self.resident if not r.wide]

    def step(self):
        """Advance every resident chain by one slice (one batched launch plus
        one launch per wide chain), then retire finished chains."""
        torch = self.torch
        narrow = self._narrow()
        if self._descs_dirty:
            arr = (Q.ChainDesc * max(len(narrow), 1))()
            for i, r in enumerate(narrow):
                arr[i] = r.desc
            self._descs_host = arr
            self._descs_dev = torch.from_numpy(np.frombuffer(bytes(arr), dtype=np.uint8).copy()).to(self.dev)
            self._descs_dirty = False
        t0 = time.perf_counter()
        if narrow:
            cfg = Q.BatchConfig(self.threads, 0, self.slice, None)
            Q._check(Q.qap_sa_run_batch(len(narrow), self._descs_host, self._descs_dev, None, cfg, self.ws),
                     "qap_sa_run_batch")
        for r in self.resident:
            if r.wide:
                b = r.bufs
                st = Q._struct_from(b["state"], Q.ChainState)
                r.sched.t_end = min(st.t + self.slice, r.chain.iters)
                bufs = Q.RunBuffers(b["temps"].data_ptr(), b["ties"].data_ptr(), 16, 0, None, 0, None,
                                    b["ws"].data_ptr(), b["ws"].numel())
                Q._check(Q.qap_sa_run(r.chain.n, b["A"], b["B"], b["Bp"], b["p"], b["delta"], b["state"],
                                      r.sched, r.info, bufs), "qap_sa_run")
        torch.cuda.synchronize()
        self.stats.busy_s += time.perf_counter() - t0
        self.stats.slices += 1
        self.stats.resident_sum += len(self.resident)
        self.stats.max_resident = max(self.stats.max_resident, len(self.resident))
        return self.retire()

    def retire(self) -> list[Result]:
        if not self.resident:
            return []
        raw = [Q._struct_from(r.bufs["state"], Q.ChainState) for r in self.resident]
        now = time.perf_counter()
        done, keep = [], []
        for r, st in zip(self.resident, raw):
            if st.status != Q.QAP_OK:
                raise Q.QapError(st.status, f"request {r.rid}")
            if st.t >= r.chain.iters:
                state = {k: int(getattr(st, k)) for k, _ in Q.ChainState._fields_}
                res = Result(r.rid, r.chain.n, r.arrival, r.admitted, now, state, r.bufs["p"].cpu().numpy())
                done.append(res)
                self.used -= footprint_bytes(r.chain.n, r.chain.iters)
                self.stats.iterations += r.chain.iters
                self._descs_dirty = True
            else:
                keep.append(r)
        self.resident = keep
        self.stats.results.extend(done)
        return done

    # ------------------------------------------------------------------ trace
    def run_trace(self, requests, time_limit: float | None = None) -> ServerStats:
        """Serve ``requests`` (objects with rid, arrival_s, chain) arriving on
        the wall clock, from the first call, until all are done (or the limit)."""
        start = time.perf_counter()
        for q in requests:
            self.submit(q.rid, q.chain, start + q.arrival_s)
        while self.waiting or self.resident:
            now = time.perf_counter()
            if time_limit is not None and now - start > time_limit:
                break
            self.admit(now)
            if self.resident:
                self.step()
            else:
                nxt = min(a for a, _, _ in self.waiting)
                time.sleep(max(0.0, min(nxt - time.perf_counter(), 0.01)))
        self.stats.wall_s = time.perf_counter() - start
        return self.stats
