"""Python binding of libqapsa (ctypes).

The functions named ``qap_*`` mirror the C ABI in ``include/qapsa.h`` one to
one and only marshal arguments: device buffers are torch tensors on a ROCm
device (or raw integer addresses), streams are ``torch.cuda.Stream`` objects
(or raw handles).  Every step of the annealing runs in the HIP kernels.

``Chain`` is a convenience holder for one chain's device buffers that calls
those functions in the order the method needs (set-up, schedule, run).
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libqapsa.so")

QAP_OK, QAP_E_INVAL, QAP_E_NOT_PERM, QAP_E_RANGE = 0, -1, -2, -3
QAP_E_NOMEM, QAP_E_DEVICE, QAP_E_UNSUPPORTED, QAP_E_STATE, QAP_E_TIMEOUT = -4, -5, -6, -7, -8
QAP_E_TIE_OVERFLOW = -9
QAP_MODE_SCRATCH, QAP_MODE_DELTA, QAP_MODE_SCRATCH_STALE = 0, 1, 2
QAP_FLAG_DELTA_ONLY, QAP_FLAG_SCRATCH_ONLY, QAP_FLAG_MULTI_WG, QAP_FLAG_RANDOM_ORDER = 1, 2, 4, 8
QAP_FLAG_SINGLE_WG = 16


class QapError(RuntimeError):
    def __init__(self, status: int, where: str):
        super().__init__(f"{where}: {qap_strerror(status)} ({status})")
        self.status = status


class InstanceInfo(C.Structure):
    _fields_ = [("cost", C.c_int64), ("sum_abs_delta", C.c_int64),
                ("a_min", C.c_int32), ("a_max", C.c_int32), ("b_min", C.c_int32), ("b_max", C.c_int32),
                ("symmetric", C.c_int32), ("status", C.c_int32)]


class ChainState(C.Structure):
    _fields_ = [("t", C.c_uint64), ("accepts", C.c_uint64), ("near_ties", C.c_uint64),
                ("hash", C.c_uint64), ("cost", C.c_int64), ("best_cost", C.c_int64),
                ("best_iter", C.c_uint64), ("status", C.c_int32), ("mode", C.c_int32)]


class NearTie(C.Structure):
    _fields_ = [("t", C.c_uint64), ("delta", C.c_int64), ("z", C.c_double)]


class Schedule(C.Structure):
    _fields_ = [("iters", C.c_uint64), ("t_end", C.c_uint64), ("T0", C.c_double), ("alpha", C.c_double),
                ("seed", C.c_uint64), ("chain_id", C.c_uint32), ("flags", C.c_uint32),
                ("switch_permille", C.c_uint32), ("scan_window", C.c_uint32)]


class TabuSchedule(C.Structure):
    _fields_ = [("iters", C.c_uint64), ("t_end", C.c_uint64), ("tenure", C.c_int32), ("reserved", C.c_uint32)]


class RunBuffers(C.Structure):
    _fields_ = [("temps", C.c_void_p), ("ties", C.c_void_p), ("tie_cap", C.c_uint32),
                ("reserved", C.c_uint32), ("accept_log", C.c_void_p), ("accept_cap", C.c_uint64),
                ("phase_cycles", C.c_void_p), ("workspace", C.c_void_p), ("workspace_bytes", C.c_uint64)]


PHASES = ["total", "scratch_thresh", "scratch_eval", "scratch_accept", "delta_scan", "delta_update", "build",
          "io", "n_rounds", "n_scratch_acc", "n_scan_steps", "n_delta_acc", "n_thresh", "switch_t", "n_scanned",
          "grid_sync"]


STATE_BYTES = C.sizeof(ChainState)
INFO_BYTES = C.sizeof(InstanceInfo)
TIE_BYTES = C.sizeof(NearTie)


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_1208_2675_amd.build`")
    # torch brings its own HIP runtime.  Loading it first makes this library bind
    # to that same runtime; loaded the other way round, the process would hold
    # two runtimes, and torch's streams and memory would be foreign to ours.
    import torch  # noqa: F401
    L = C.CDLL(LIB_PATH)
    vp, i32, u64, i64 = C.c_void_p, C.c_int32, C.c_uint64, C.c_int64
    L.qap_strerror.argtypes = [C.c_int]
    L.qap_strerror.restype = C.c_char_p
    L.qap_cost.argtypes = [i32, vp, vp, vp, vp, vp]
    L.qap_cost.restype = C.c_int
    L.qap_delta_init.argtypes = [i32, vp, vp, vp, vp, vp, vp, vp, vp]
    L.qap_delta_init.restype = C.c_int
    L.qap_temp_table_len.argtypes = [u64]
    L.qap_temp_table_len.restype = u64
    L.qap_schedule_tables.argtypes = [u64, C.c_double, vp, vp]
    L.qap_schedule_tables.restype = C.c_int
    L.qap_schedule_init.argtypes = [i32, C.POINTER(InstanceInfo), u64, C.c_double, C.POINTER(Schedule)]
    L.qap_schedule_init.restype = C.c_int
    L.qap_workspace_bytes.argtypes = [i32]
    L.qap_workspace_bytes.restype = u64
    L.qap_sa_run.argtypes = [i32, vp, vp, vp, vp, vp, vp, C.POINTER(Schedule), C.POINTER(InstanceInfo),
                             C.POINTER(RunBuffers), vp]
    L.qap_sa_run.restype = C.c_int
    L.qap_sa_run_static.argtypes = L.qap_sa_run.argtypes
    L.qap_sa_run_static.restype = C.c_int
    L.qap_static_scratch_bytes.argtypes = []
    L.qap_static_scratch_bytes.restype = u64
    L.qap_tabu_run.argtypes = [i32, vp, vp, vp, vp, vp, C.POINTER(TabuSchedule), C.POINTER(InstanceInfo), vp,
                               C.POINTER(RunBuffers), vp]
    L.qap_tabu_run.restype = C.c_int
    return L


_lib = _load()


def _ptr(x) -> int | None:
    if x is None:
        return None
    if isinstance(x, int):
        return x
    return x.data_ptr()


def _stream(s) -> int | None:
    if s is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    if isinstance(s, int):
        return s
    return s.cuda_stream


def _check(rc: int, where: str):
    if rc != QAP_OK:
        raise QapError(rc, where)


# ----------------------------------------------------------- the C ABI, 1:1

def qap_strerror(status: int) -> str:
    return _lib.qap_strerror(status).decode()


def qap_cost(n, A, B, p, cost, stream=None) -> int:
    return _lib.qap_cost(n, _ptr(A), _ptr(B), _ptr(p), _ptr(cost), _stream(stream))


def qap_delta_init(n, A, B, p, Bp, delta, info, state=None, stream=None) -> int:
    return _lib.qap_delta_init(n, _ptr(A), _ptr(B), _ptr(p), _ptr(Bp), _ptr(delta), _ptr(info),
                               _ptr(state), _stream(stream))


def qap_temp_table_len(iters: int) -> int:
    return int(_lib.qap_temp_table_len(iters))


def qap_schedule_tables(iters, alpha, temps, stream=None) -> int:
    return _lib.qap_schedule_tables(iters, alpha, _ptr(temps), _stream(stream))


def qap_schedule_init(n, info: InstanceInfo, iters, final_ratio, sched: Schedule) -> int:
    return _lib.qap_schedule_init(n, C.byref(info), iters, final_ratio, C.byref(sched))


def qap_workspace_bytes(n: int) -> int:
    return int(_lib.qap_workspace_bytes(n))


def qap_sa_run(n, A, B, Bp, p, delta, state, sched: Schedule, info: InstanceInfo, bufs: RunBuffers,
               stream=None) -> int:
    return _lib.qap_sa_run(n, _ptr(A), _ptr(B), _ptr(Bp), _ptr(p), _ptr(delta), _ptr(state), C.byref(sched),
                           C.byref(info), C.byref(bufs), _stream(stream))


def qap_sa_run_static(n, A, B, Bp, p, delta, state, sched: Schedule, info: InstanceInfo, bufs: RunBuffers,
                      stream=None) -> int:
    return _lib.qap_sa_run_static(n, _ptr(A), _ptr(B), _ptr(Bp), _ptr(p), _ptr(delta), _ptr(state),
                                  C.byref(sched), C.byref(info), C.byref(bufs), _stream(stream))


def qap_static_scratch_bytes() -> int:
    return int(_lib.qap_static_scratch_bytes())


def qap_tabu_run(n, A, Bp, p, delta, state, sched: TabuSchedule, info: InstanceInfo, tabu, bufs: RunBuffers,
                 stream=None) -> int:
    return _lib.qap_tabu_run(n, _ptr(A), _ptr(Bp), _ptr(p), _ptr(delta), _ptr(state), C.byref(sched),
                             C.byref(info), _ptr(tabu), C.byref(bufs), _stream(stream))


# ------------------------------------------------------------- conveniences

def schedule_for(n: int, info: InstanceInfo, iters: int, ratio: float = 1e-3, T0: float | None = None) -> Schedule:
    """The library's geometric schedule (qap_schedule_init) for an instance
    whose facts ``info`` came back from qap_delta_init; ``T0`` overrides the
    start temperature (e.g. +inf, every proposal accepted)."""
    sched = Schedule()
    if T0 is not None and info.sum_abs_delta <= 0:
        # the library refuses T0 = mean |Delta| = 0; an explicit T0 needs only alpha
        info = InstanceInfo.from_buffer_copy(bytes(info))
        info.sum_abs_delta = 1
    _check(qap_schedule_init(n, info, iters, ratio, sched), "qap_schedule_init")
    if T0 is not None:
        sched.T0 = float(T0)
    return sched


def _struct_from(t, cls):
    buf = t.cpu().numpy().tobytes()
    return cls.from_buffer_copy(buf)


class Chain:
    """Device buffers of one chain plus the calls of a full run.

    A, B, p0: host arrays (numpy) copied to `device`.  After ``init()`` the
    instance facts are on the host in ``self.info``; ``run(t_end)`` advances the
    chain; ``result()`` copies the state, p and (optionally) Delta back.
    """

    def __init__(self, A, B, p0, iters: int, seed: int, chain_id: int = 0, ratio: float = 1e-3,
                 T0: float | None = None, device: str = "cuda", stream=None, tie_cap: int = 64,
                 accept_cap: int = 0, flags: int = 0, switch_permille: int = 0, profile: bool = False,
                 scan_window: int = 0):
        import torch
        self.torch = torch
        A = np.ascontiguousarray(A, dtype=np.int32)
        B = np.ascontiguousarray(B, dtype=np.int32)
        self.n = n = int(A.shape[0])
        self.m = n * (n - 1) // 2
        self.iters = int(iters)
        self.seed, self.chain_id, self.ratio, self.T0_override = int(seed), int(chain_id), ratio, T0
        self.flags, self.switch_permille, self.scan_window = int(flags), int(switch_permille), int(scan_window)
        self.stream = stream
        dev = torch.device(device)
        self.A = torch.from_numpy(A).to(dev)
        self.B = torch.from_numpy(B).to(dev)
        self.p = torch.from_numpy(np.ascontiguousarray(p0, dtype=np.int32)).to(dev)
        self.Bp = torch.empty((n, n), dtype=torch.int32, device=dev)
        self.delta = torch.empty(max(self.m, 1), dtype=torch.int32, device=dev)
        self.info_d = torch.zeros(INFO_BYTES, dtype=torch.uint8, device=dev)
        self.state_d = torch.zeros(STATE_BYTES, dtype=torch.uint8, device=dev)
        self.temps = torch.empty(qap_temp_table_len(self.iters), dtype=torch.float64, device=dev)
        self.tie_cap = tie_cap
        self.ties = torch.zeros(max(tie_cap, 1) * TIE_BYTES, dtype=torch.uint8, device=dev)
        self.accept_cap = accept_cap
        self.accept_log = torch.zeros((max(accept_cap, 1), 4), dtype=torch.int64, device=dev)
        self.prof = torch.zeros(len(PHASES), dtype=torch.int64, device=dev) if profile else None
        self.workspace = torch.zeros(qap_workspace_bytes(n), dtype=torch.uint8, device=dev)
        self.info = None
        self.sched = None

    def init(self):
        n = self.n
        _check(qap_delta_init(n, self.A, self.B, self.p, self.Bp, self.delta, self.info_d, self.state_d,
                              self.stream), "qap_delta_init")
        self.torch.cuda.synchronize()
        self.info = _struct_from(self.info_d, InstanceInfo)
        if self.info.status != QAP_OK:
            raise QapError(self.info.status, "qap_delta_init (device)")
        self.sched = schedule_for(n, self.info, self.iters, self.ratio, self.T0_override)
        self.sched.t_end = 0
        self.sched.seed = self.seed & (2**64 - 1)
        self.sched.chain_id = self.chain_id
        self.sched.flags = self.flags
        self.sched.switch_permille = self.switch_permille
        self.sched.scan_window = self.scan_window
        _check(qap_schedule_tables(self.iters, self.sched.alpha, self.temps, self.stream), "qap_schedule_tables")
        return self

    def buffers(self) -> RunBuffers:
        return RunBuffers(self.temps.data_ptr(), self.ties.data_ptr(), self.tie_cap, 0,
                          self.accept_log.data_ptr() if self.accept_cap else None, self.accept_cap,
                          self.prof.data_ptr() if self.prof is not None else None,
                          self.workspace.data_ptr(), self.workspace.numel())

    def phases(self) -> dict:
        """Phase counters of the runs so far (cycles of the shader clock, counts)."""
        v = self.prof.cpu().numpy().tolist()
        return {k: int(x) for k, x in zip(PHASES, v)}

    def run(self, t_end: int | None = None, static: bool = False):
        """Advance the chain to t_end; ``static`` runs through qap_sa_run_static
        (the library's own device scratch instead of this chain's workspace)."""
        self.sched.t_end = self.iters if t_end is None else int(t_end)
        if static:
            bufs = self.buffers()
            bufs.workspace, bufs.workspace_bytes = None, 0
            _check(qap_sa_run_static(self.n, self.A, self.B, self.Bp, self.p, self.delta, self.state_d, self.sched,
                                     self.info, bufs, self.stream), "qap_sa_run_static")
            return self
        _check(qap_sa_run(self.n, self.A, self.B, self.Bp, self.p, self.delta, self.state_d, self.sched,
                          self.info, self.buffers(), self.stream), "qap_sa_run")
        return self

    def tabu(self, t_end: int | None = None, tenure: int | None = None):
        """Tabu search instead of annealing: iterations state.t .. t_end-1 of a
        search of ``iters`` iterations (tenure defaults to n).  The tabu table
        lives on the device between calls."""
        if getattr(self, "tabu_table", None) is None:
            self.tabu_table = self.torch.zeros(self.n * self.n, dtype=self.torch.int32, device=self.p.device)
            self.tenure = self.n if tenure is None else int(tenure)
        ts = TabuSchedule(self.iters, self.iters if t_end is None else int(t_end), self.tenure, 0)
        _check(qap_tabu_run(self.n, self.A, self.Bp, self.p, self.delta, self.state_d, ts, self.info,
                            self.tabu_table, self.buffers(), self.stream), "qap_tabu_run")
        return self

    def state(self) -> ChainState:
        self.torch.cuda.synchronize()
        return _struct_from(self.state_d, ChainState)

    def result(self, with_delta: bool = False) -> dict:
        st = self.state()
        if st.status != QAP_OK:
            raise QapError(st.status, "qap_sa_run (device)")
        out = {k: int(getattr(st, k)) for k, _ in ChainState._fields_}
        out["p"] = self.p.cpu().numpy()
        nt = min(st.near_ties, self.tie_cap)
        ties = np.frombuffer(self.ties.cpu().numpy().tobytes(), dtype=np.dtype(
            [("t", "<u8"), ("delta", "<i8"), ("z", "<f8")]))[:nt]
        order = np.argsort(ties["t"], kind="stable")
        out["near_tie_t"] = ties["t"][order]
        out["near_tie_z"] = ties["z"][order]
        out["near_tie_delta"] = ties["delta"][order]
        out["T0"], out["alpha"] = self.sched.T0, self.sched.alpha
        if with_delta:
            out["delta"] = self.delta.cpu().numpy().astype(np.int64)[: self.m]
            out["Bp"] = self.Bp.cpu().numpy()
        if self.accept_cap:
            out["accept_log"] = self.accept_log.cpu().numpy()[: min(st.accepts, self.accept_cap)]
        return out


# ------------------------------------------------------------------ batches

class ChainDesc(C.Structure):
    _fields_ = [("n", C.c_int32), ("symmetric", C.c_int32), ("a_min", C.c_int32), ("a_max", C.c_int32),
                ("b_min", C.c_int32), ("b_max", C.c_int32), ("flags", C.c_uint32), ("switch_permille", C.c_uint32),
                ("A", C.c_void_p), ("Bp", C.c_void_p), ("p", C.c_void_p), ("delta", C.c_void_p),
                ("state", C.c_void_p), ("temps", C.c_void_p), ("ties", C.c_void_p), ("tie_cap", C.c_uint32),
                ("chain_id", C.c_uint32), ("iters", C.c_uint64), ("t_end", C.c_uint64), ("T0", C.c_double),
                ("seed", C.c_uint64), ("scratch", C.c_void_p)]


class BatchConfig(C.Structure):
    _fields_ = [("threads", C.c_int32), ("groups", C.c_int32), ("slice", C.c_uint64),
                ("phase_cycles", C.c_void_p)]


_lib.qap_batch_workspace_bytes.argtypes = []
_lib.qap_batch_workspace_bytes.restype = C.c_uint64
_lib.qap_sa_run_batch.argtypes = [C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p, C.POINTER(BatchConfig),
                                  C.c_void_p, C.c_void_p]
_lib.qap_sa_run_batch.restype = C.c_int


_lib.qap_single_workgroup.argtypes = [C.c_int32, C.c_int32, C.c_int64, C.c_int64]
_lib.qap_single_workgroup.restype = C.c_int


def qap_single_workgroup(n: int, symmetric: int, a_range: int, b_range: int) -> int:
    return int(_lib.qap_single_workgroup(n, symmetric, a_range, b_range))


def fits_one_workgroup(n: int, symmetric: bool, a_range: int, b_range: int) -> bool:
    """True if one workgroup can hold the chain (in LDS, or with a per-chain scratch)."""
    return qap_single_workgroup(n, int(symmetric), a_range, b_range) != 0


def needs_scratch(n: int, symmetric: bool, a_range: int, b_range: int) -> bool:
    return qap_single_workgroup(n, int(symmetric), a_range, b_range) == 2


_lib.qap_chain_scratch_bytes.argtypes = [C.c_int32, C.c_int32]
_lib.qap_chain_scratch_bytes.restype = C.c_uint64


def qap_chain_scratch_bytes(n: int, symmetric: int) -> int:
    return int(_lib.qap_chain_scratch_bytes(n, symmetric))


def qap_batch_workspace_bytes() -> int:
    return int(_lib.qap_batch_workspace_bytes())


def qap_sa_run_batch(n_chains, host_descs, dev_descs, order, cfg: BatchConfig, workspace, stream=None) -> int:
    return _lib.qap_sa_run_batch(n_chains, C.cast(host_descs, C.c_void_p) if host_descs is not None else None,
                                 _ptr(dev_descs), _ptr(order), C.byref(cfg), _ptr(workspace), _stream(stream))


class Batch:
    """Device buffers of many independent chains and one batched run.

    ``chains`` are workload chains (A, B, p0, iters, philox_seed, chain_id);
    chains that share the same A array object share its device copy.
    """

    def __init__(self, chains, device: str = "cuda", tie_cap: int = 16, profile: bool = False):
        import torch
        self.torch = torch
        dev = torch.device(device)
        self.chains = chains
        self.k = len(chains)
        inst = {}
        self.views = []
        for ch in chains:
            key = (id(ch.A), id(ch.B))
            if key not in inst:
                inst[key] = (torch.from_numpy(np.ascontiguousarray(ch.A, dtype=np.int32)).to(dev),
                             torch.from_numpy(np.ascontiguousarray(ch.B, dtype=np.int32)).to(dev))
            self.views.append(inst[key])
        n_tot = sum(ch.n for ch in chains)
        m_tot = sum(max(ch.n * (ch.n - 1) // 2, 1) for ch in chains)
        self.p = torch.empty(n_tot, dtype=torch.int32, device=dev)
        self.Bp = torch.empty(sum(ch.n * ch.n for ch in chains), dtype=torch.int32, device=dev)
        self.delta = torch.empty(m_tot, dtype=torch.int32, device=dev)
        self.info_d = torch.zeros((self.k, INFO_BYTES), dtype=torch.uint8, device=dev)
        self.state_d = torch.zeros((self.k, STATE_BYTES), dtype=torch.uint8, device=dev)
        t_tot = sum(qap_temp_table_len(ch.iters) for ch in chains)
        self.temps = torch.empty(t_tot, dtype=torch.float64, device=dev)
        self.tie_cap = tie_cap
        self.ties = torch.zeros((self.k, max(tie_cap, 1) * TIE_BYTES), dtype=torch.uint8, device=dev)
        self.ws = torch.zeros(qap_batch_workspace_bytes(), dtype=torch.uint8, device=dev)
        self.prof = torch.zeros(len(PHASES), dtype=torch.int64, device=dev) if profile else None
        self.off = []
        po = bo = do = to = 0
        for ch in chains:
            self.off.append((po, bo, do, to))
            po += ch.n; bo += ch.n * ch.n; do += max(ch.n * (ch.n - 1) // 2, 1); to += qap_temp_table_len(ch.iters)
        self.p.copy_(torch.from_numpy(np.concatenate([np.asarray(ch.p0, dtype=np.int32) for ch in chains])).to(dev))
        self.descs = None
        self.scratch = {}

    def init(self, ratio: float = 1e-3, flags: int = 0, switch_permille=0, T0=None):
        """Step (a) of Sec. 2.2 for every chain and the descriptors of the batch.
        ``switch_permille`` is a number or a function (n, symmetric) -> number
        (a tuned table, see tune.py); 0 means the library default.  ``T0``
        (None, a number or a function of the chain index) overrides the start
        temperature of the library's schedule."""
        torch = self.torch
        i4, i8, f8 = 4, 8, 8
        for i, ch in enumerate(self.chains):
            A, B = self.views[i]
            po, bo, do, _ = self.off[i]
            _check(qap_delta_init(ch.n, A, B, self.p.data_ptr() + i4 * po, self.Bp.data_ptr() + i4 * bo,
                                  self.delta.data_ptr() + i4 * do, self.info_d[i], self.state_d[i]),
                   "qap_delta_init")
        torch.cuda.synchronize()
        raw = self.info_d.cpu().numpy()
        self.infos = [InstanceInfo.from_buffer_copy(raw[i].tobytes()) for i in range(self.k)]
        descs = (ChainDesc * self.k)()
        for i, ch in enumerate(self.chains):
            inf = self.infos[i]
            if inf.status != QAP_OK:
                raise QapError(inf.status, f"qap_delta_init (device), chain {i}")
            po, bo, do, to = self.off[i]
            T0_i = T0(i) if callable(T0) else T0
            sc = schedule_for(ch.n, inf, ch.iters, ratio, T0_i)
            temps = self.temps.data_ptr() + f8 * to
            _check(qap_schedule_tables(ch.iters, sc.alpha, temps), "qap_schedule_tables")
            A, _ = self.views[i]
            scr = None
            if needs_scratch(ch.n, bool(inf.symmetric), inf.a_max - inf.a_min, inf.b_max - inf.b_min):
                self.scratch[i] = torch.empty(qap_chain_scratch_bytes(ch.n, inf.symmetric), dtype=torch.uint8,
                                              device=self.p.device)
                scr = self.scratch[i].data_ptr()
            sw = switch_permille(ch.n, bool(inf.symmetric)) if callable(switch_permille) else switch_permille
            descs[i] = ChainDesc(ch.n, inf.symmetric, inf.a_min, inf.a_max, inf.b_min, inf.b_max, flags,
                                 int(sw), A.data_ptr(), self.Bp.data_ptr() + i4 * bo,
                                 self.p.data_ptr() + i4 * po, self.delta.data_ptr() + i4 * do,
                                 self.state_d[i].data_ptr(), temps, self.ties[i].data_ptr(), self.tie_cap,
                                 ch.chain_id, ch.iters, ch.iters, sc.T0, ch.philox_seed & (2**64 - 1), scr)
        self.descs = descs
        raw = np.frombuffer(bytes(descs), dtype=np.uint8).copy()
        self.descs_d = torch.from_numpy(raw).to(self.p.device)
        return self

    def run(self, threads: int = 256, groups: int = 0, slice_iters: int = 0, order=None, stream=None):
        cfg = BatchConfig(threads, groups, slice_iters, self.prof.data_ptr() if self.prof is not None else None)
        _check(qap_sa_run_batch(self.k, self.descs, self.descs_d, order, cfg, self.ws, stream), "qap_sa_run_batch")
        return self

    def capture(self, slices: int, slice_iters: int, groups: int = 0, order=None):
        """Record `slices` consecutive slice launches into one HIP graph
        (torch.cuda.CUDAGraph).  Each replay advances every chain by up to
        slices * slice_iters iterations from wherever its state stands, so the
        steady loop costs one graph launch per `slices` slices.  One eager slice
        must have run first (it sets up the library's side streams)."""
        torch = self.torch
        g = torch.cuda.CUDAGraph()
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.graph(g, stream=s):
            for _ in range(slices):
                self.run(groups=groups, slice_iters=slice_iters, order=order, stream=s.cuda_stream)
        torch.cuda.current_stream().wait_stream(s)
        return g

    def states(self) -> list[dict]:
        self.torch.cuda.synchronize()
        raw = self.state_d.cpu().numpy()
        out = []
        for i in range(self.k):
            st = ChainState.from_buffer_copy(raw[i].tobytes())
            out.append({k: int(getattr(st, k)) for k, _ in ChainState._fields_})
        return out

    def perm(self, i: int) -> np.ndarray:
        po = self.off[i][0]
        return self.p[po: po + self.chains[i].n].cpu().numpy()

    def done(self) -> bool:
        return all(s["t"] >= ch.iters for s, ch in zip(self.states(), self.chains))

    def phases(self) -> dict:
        v = self.prof.cpu().numpy().tolist()
        return {k: int(x) for k, x in zip(PHASES, v)}
