"""CPU oracle for Delta-matrix simulated annealing on the QAP (ctypes over
``qap_oracle.c``).

TEST INFRASTRUCTURE ONLY: the test-suite, the smoke check and the benchmark's
CPU-baseline leg are its only users.  The device library never imports it and
it never imports the device library.

Every function cites the passage of the paper it follows in ``qap_oracle.c``.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "qap_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

CFLAGS = ["-O2", "-std=c11", "-fPIC", "-shared", "-ffp-contract=off", "-fno-fast-math",
          "-Wall", "-Wextra"]


def build(force: bool = False) -> str:
    """Compile ``qap_oracle.c`` into ``liboracle.so`` with gcc."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.run(["gcc", *CFLAGS, "-o", tmp, _SRC, "-lm"], check=True)
        os.replace(tmp, _LIB)
    return _LIB


class State(C.Structure):
    _fields_ = [("t", C.c_uint64), ("accepts", C.c_uint64), ("near_ties", C.c_uint64),
                ("hash", C.c_uint64), ("cost", C.c_int64), ("best_cost", C.c_int64),
                ("best_iter", C.c_uint64)]

    def as_dict(self) -> dict:
        return {k: int(getattr(self, k)) for k, _ in self._fields_}


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        L = C.CDLL(_LIB)
        i32p = np.ctypeslib.ndpointer(np.int32, flags="C_CONTIGUOUS")
        i64p = np.ctypeslib.ndpointer(np.int64, flags="C_CONTIGUOUS")
        f64p = np.ctypeslib.ndpointer(np.float64, flags="C_CONTIGUOUS")
        u32p = np.ctypeslib.ndpointer(np.uint32, flags="C_CONTIGUOUS")
        L.orc_cost.argtypes = [C.c_int32, i32p, i32p, i32p]
        L.orc_cost.restype = C.c_int64
        for f in (L.orc_swap_cost, L.orc_swap_cost_by_definition):
            f.argtypes = [C.c_int32, i32p, i32p, i32p, C.c_int32, C.c_int32]
            f.restype = C.c_int64
        L.orc_delta_matrix.argtypes = [C.c_int32, i32p, i32p, i32p, i64p]
        L.orc_delta_matrix.restype = None
        L.orc_mean_abs_delta.argtypes = [C.c_int32, i64p, C.POINTER(C.c_int64)]
        L.orc_mean_abs_delta.restype = C.c_double
        L.orc_check_bounds.argtypes = [C.c_int32, i32p, i32p]
        L.orc_check_bounds.restype = C.c_int
        L.orc_philox4x32_10.argtypes = [u32p, u32p, u32p]
        L.orc_philox4x32_10.restype = None
        L.orc_uniform.argtypes = [C.c_uint64, C.c_uint32, C.c_uint64]
        L.orc_uniform.restype = C.c_double
        L.orc_geometric_alpha.argtypes = [C.c_uint64, C.c_double]
        L.orc_geometric_alpha.restype = C.c_double
        L.orc_temperature_table_len.argtypes = [C.c_uint64]
        L.orc_temperature_table_len.restype = C.c_uint64
        L.orc_temperature_tables.argtypes = [C.c_double, C.c_uint64, f64p, f64p, f64p]
        L.orc_temperature_tables.restype = None
        L.orc_temperature.argtypes = [C.c_double, f64p, f64p, f64p, C.c_uint64]
        L.orc_temperature.restype = C.c_double
        L.orc_accept_fingerprint.argtypes = [C.c_uint64, C.c_int32, C.c_int32, C.c_int64]
        L.orc_accept_fingerprint.restype = C.c_uint64
        L.orc_state_init.argtypes = [C.c_int32, i32p, i32p, i32p, C.POINTER(State)]
        L.orc_state_init.restype = None
        L.orc_sa_run.argtypes = [C.c_int32, i32p, i32p, i32p, C.POINTER(State),
                                 C.c_uint64, C.c_uint64, C.c_double, C.c_double,
                                 C.c_uint64, C.c_uint32,
                                 C.c_void_p, C.c_uint64, C.c_void_p, C.c_void_p, C.c_uint64]
        L.orc_sa_run.restype = C.c_int
        L.orc_sa_run_order.argtypes = [C.c_int32, i32p, i32p, i32p, C.POINTER(State),
                                       C.c_uint64, C.c_uint64, C.c_double, C.c_double,
                                       C.c_uint64, C.c_uint32, C.c_int32,
                                       C.c_void_p, C.c_uint64, C.c_void_p, C.c_void_p, C.c_uint64]
        L.orc_sa_run_order.restype = C.c_int
        L.orc_random_pair_index.argtypes = [C.c_uint64, C.c_uint32, C.c_uint64, C.c_uint64]
        L.orc_random_pair_index.restype = C.c_uint64
        L.orc_tabu_run.argtypes = [C.c_int32, i32p, i32p, i32p, C.POINTER(State), C.c_uint64, C.c_int64,
                                   i64p, C.c_void_p, C.c_uint64]
        L.orc_tabu_run.restype = C.c_int
        L.orc_brute_force.argtypes = [C.c_int32, i32p, i32p, i32p, C.POINTER(C.c_uint64)]
        L.orc_brute_force.restype = C.c_int64
        _lib = L
    return _lib



def _mats(A, B):
    A = np.ascontiguousarray(A, dtype=np.int32)
    B = np.ascontiguousarray(B, dtype=np.int32)
    assert A.ndim == 2 and A.shape[0] == A.shape[1] == B.shape[0] == B.shape[1]
    return A, B


def cost(A, B, p) -> int:
    """Eq. (1)."""
    A, B = _mats(A, B)
    return int(lib().orc_cost(A.shape[0], A, B, np.ascontiguousarray(p, dtype=np.int32)))


def swap_cost(A, B, p, r, s) -> int:
    """O(N) swap cost (Eq. (1) differenced)."""
    A, B = _mats(A, B)
    return int(lib().orc_swap_cost(A.shape[0], A, B, np.ascontiguousarray(p, dtype=np.int32), r, s))


def swap_cost_by_definition(A, B, p, r, s) -> int:
    """C(p o (r s)) - C(p), two evaluations of Eq. (1)."""
    A, B = _mats(A, B)
    return int(lib().orc_swap_cost_by_definition(A.shape[0], A, B,
                                                 np.ascontiguousarray(p, dtype=np.int32), r, s))


def delta_matrix(A, B, p) -> np.ndarray:
    """Step (a): packed row-major swap costs of all pairs r < s (int64)."""
    A, B = _mats(A, B)
    n = A.shape[0]
    out = np.empty(n * (n - 1) // 2, dtype=np.int64)
    lib().orc_delta_matrix(n, A, B, np.ascontiguousarray(p, dtype=np.int32), out)
    return out


def mean_abs_delta(n: int, delta: np.ndarray) -> tuple[float, int]:
    """T0 of the schedule: (mean |Delta|, sum |Delta|)."""
    s = C.c_int64(0)
    T0 = lib().orc_mean_abs_delta(n, np.ascontiguousarray(delta, dtype=np.int64), C.byref(s))
    return float(T0), int(s.value)


def check_bounds(A, B) -> int:
    A, B = _mats(A, B)
    return int(lib().orc_check_bounds(A.shape[0], A, B))


def philox4x32_10(ctr, key) -> np.ndarray:
    out = np.zeros(4, dtype=np.uint32)
    lib().orc_philox4x32_10(np.asarray(ctr, dtype=np.uint32), np.asarray(key, dtype=np.uint32), out)
    return out


def uniform(seed: int, chain: int, t: int) -> float:
    return float(lib().orc_uniform(seed, chain, t))


def geometric_alpha(iters: int, ratio: float = 1e-3) -> float:
    return float(lib().orc_geometric_alpha(iters, ratio))


def temperature_tables(alpha: float, iters: int):
    nh = int(lib().orc_temperature_table_len(iters))
    L = np.zeros(1024); M = np.zeros(1024); H = np.zeros(nh)
    lib().orc_temperature_tables(alpha, iters, L, M, H)
    return L, M, H


def temperatures(T0: float, alpha: float, iters: int, ts) -> np.ndarray:
    L, M, H = temperature_tables(alpha, iters)
    f = lib().orc_temperature
    return np.array([f(T0, L, M, H, int(t)) for t in ts])


def accept_fingerprint(t: int, r: int, s: int, delta: int) -> int:
    return int(lib().orc_accept_fingerprint(t, r, s, delta))


def schedule(A, B, p, iters: int, ratio: float = 1e-3) -> dict:
    """The schedule parameters a run uses: T0 = mean |Delta_0|, alpha geometric."""
    d = delta_matrix(A, B, p)
    T0, sabs = mean_abs_delta(np.asarray(A).shape[0], d)
    return {"T0": T0, "alpha": geometric_alpha(iters, ratio), "iters": int(iters), "sum_abs": sabs}


def random_pair_index(seed: int, chain: int, t: int, m: int) -> int:
    """Pair number proposed at iteration t under random order."""
    return int(lib().orc_random_pair_index(seed, chain, t, m))


def sa_run(A, B, p0, iters: int, T0: float, alpha: float, seed: int, chain: int = 0,
           t_end: int | None = None, state: State | None = None, acc_cap: int = 0,
           tie_cap: int = 64, order: int = 0) -> dict:
    """Steps (b)-(e) of the Delta-matrix approach as a from-scratch SA run over
    iterations [state.t, t_end); order 0 proposes the pairs in row-major order,
    order 1 at random.  Returns the final p, the state and the logs."""
    A, B = _mats(A, B)
    n = A.shape[0]
    p = np.ascontiguousarray(p0, dtype=np.int32).copy()
    L = lib()
    if state is None:
        state = State()
        L.orc_state_init(n, A, B, p, C.byref(state))
    t_end = iters if t_end is None else int(t_end)
    acc = np.zeros((max(acc_cap, 1), 4), dtype=np.int64)
    tie_t = np.zeros(max(tie_cap, 1), dtype=np.uint64)
    tie_z = np.zeros(max(tie_cap, 1), dtype=np.float64)
    rc = L.orc_sa_run_order(n, A, B, p, C.byref(state), iters, t_end, T0, alpha, seed, chain, order,
                            acc.ctypes.data if acc_cap else None, acc_cap,
                            tie_t.ctypes.data, tie_z.ctypes.data, tie_cap)
    if rc != 0:
        raise ValueError(f"orc_sa_run failed with status {rc}")
    nacc = min(state.accepts, acc_cap)
    nt = min(state.near_ties, tie_cap)
    return {"p": p, "state": state, **state.as_dict(),
            "accept_log": acc[:nacc] if acc_cap else None,
            "near_tie_t": tie_t[:nt].copy(), "near_tie_z": tie_z[:nt].copy()}


def tabu_run(A, B, p0, t_end: int, tenure: int, state: State | None = None, tabu=None,
             acc_cap: int = 0) -> dict:
    """Tabu search over iterations [state.t, t_end) (rules in qap_oracle.c).
    ``tabu`` (n*n int64) carries the tabu table between calls."""
    A, B = _mats(A, B)
    n = A.shape[0]
    p = np.ascontiguousarray(p0, dtype=np.int32).copy()
    L = lib()
    if state is None:
        state = State()
        L.orc_state_init(n, A, B, p, C.byref(state))
    tabu = np.zeros(n * n, dtype=np.int64) if tabu is None else np.ascontiguousarray(tabu, dtype=np.int64).copy()
    acc = np.zeros((max(acc_cap, 1), 4), dtype=np.int64)
    rc = L.orc_tabu_run(n, A, B, p, C.byref(state), int(t_end), int(tenure), tabu,
                        acc.ctypes.data if acc_cap else None, acc_cap)
    if rc != 0:
        raise ValueError(f"orc_tabu_run failed with status {rc}")
    nacc = min(state.accepts, acc_cap)
    return {"p": p, "state": state, "tabu": tabu, **state.as_dict(),
            "accept_log": acc[:nacc] if acc_cap else None}


def brute_force(A, B) -> tuple[int, np.ndarray, int]:
    A, B = _mats(A, B)
    n = A.shape[0]
    pb = np.zeros(n, dtype=np.int32)
    vis = C.c_uint64(0)
    c = lib().orc_brute_force(n, A, B, pb, C.byref(vis))
    return int(c), pb, int(vis.value)
