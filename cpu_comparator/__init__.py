"""CPU Delta-matrix simulated annealing, the paper's comparator type (ctypes
over ``qap_delta_sa.c``): a single-threaded run that computes swap costs from
scratch while acceptance is high and keeps the Delta matrix afterwards.

A TIMING BASELINE ONLY: the benchmark times it on the host beside the GPU and
the tests check that it walks the oracle's trajectory.  It is not the oracle
and not part of the device library.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "qap_delta_sa.c")
_LIB = os.path.join(_HERE, "libcmp.so")
CFLAGS = ["-O3", "-march=native", "-std=c11", "-fPIC", "-shared", "-ffp-contract=off", "-fno-fast-math",
          "-Wall", "-Wextra"]


def build(force: bool = False) -> str:
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.run(["gcc", *CFLAGS, "-o", tmp, _SRC, "-lm"], check=True)
        os.replace(tmp, _LIB)
    return _LIB


class State(C.Structure):
    _fields_ = [("t", C.c_uint64), ("accepts", C.c_uint64), ("near_ties", C.c_uint64), ("hash", C.c_uint64),
                ("cost", C.c_int64), ("best_cost", C.c_int64), ("best_iter", C.c_uint64),
                ("delta_mode_at", C.c_uint64)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = C.CDLL(_LIB)
        i32p = np.ctypeslib.ndpointer(np.int32, flags="C_CONTIGUOUS")
        L.cmp_state_init.argtypes = [C.c_int32, i32p, i32p, i32p, C.POINTER(State)]
        L.cmp_state_init.restype = None
        L.cmp_sa_run.argtypes = [C.c_int32, i32p, i32p, i32p, C.POINTER(State), C.c_uint64, C.c_uint64,
                                 C.c_double, C.c_double, C.c_uint64, C.c_uint32, C.c_int32, C.c_int32]
        L.cmp_sa_run.restype = C.c_int
        _lib = L
    return _lib


# acceptance below 4 proposals in N (over 8192 iterations) moves the chain to
# the Delta matrix: an accepted swap then costs O(N^2) instead of O(N) per
# proposal, so the matrix pays once accepts are rarer than about 1 in N/4
def default_switch(n: int) -> tuple[int, int]:
    return 4, max(n, 4)


def sa_run(A, B, p0, iters: int, T0: float, alpha: float, seed: int, chain: int = 0, t_end: int | None = None,
           switch: tuple[int, int] | None = None, state: State | None = None) -> dict:
    """Iterations [state.t, t_end) of the run; ``switch`` = (num, den): move to
    the Delta matrix when acceptance over 8192 iterations falls below num/den
    ((0, 1): never; (-1, 1): from the start)."""
    A = np.ascontiguousarray(A, dtype=np.int32)
    B = np.ascontiguousarray(B, dtype=np.int32)
    n = A.shape[0]
    p = np.ascontiguousarray(p0, dtype=np.int32).copy()
    L = lib()
    if state is None:
        state = State()
        L.cmp_state_init(n, A, B, p, C.byref(state))
    num, den = switch if switch is not None else default_switch(n)
    rc = L.cmp_sa_run(n, A, B, p, C.byref(state), iters, iters if t_end is None else int(t_end), T0, alpha,
                      seed, chain, num, den)
    if rc != 0:
        raise ValueError("cmp_sa_run failed")
    out = {k: int(getattr(state, k)) for k, _ in State._fields_}
    out["p"] = p
    out["state"] = state
    return out
