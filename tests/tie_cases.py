"""Constructed near ties of Eq. (2), built with the CPU oracle only.

A near tie is an evaluation of Eq. (2) with |z| < 1e-12, z = fl(fl(delta / T_t)
+ fl(log r_t)).  Random instances essentially never produce one, so these
cases choose the temperature that puts a chosen iteration t* at a chosen z:
under a constant schedule (final ratio 1, so T_t = T0 for every t) the state
at t* depends on T0 only through earlier Eq. (2) decisions, so the fixed
point T0 = delta*(T0) / (eps - log r_t*) is found in a few steps, where
delta*(T0) is the swap cost the sequential run meets at t*.

With eps = -1e-13 or +1e-13 the decision at t* is an acceptance or a
rejection by a margin far larger than a last-bit difference of log between
two libraries (under 1e-14 for |log r| < 37), so every implementation of the
method must take it the same way and log the tie; eps = 0 makes the decision
itself depend on the last bit.
"""
from __future__ import annotations

import math

import numpy as np


def pair_at(n: int, t: int) -> tuple[int, int]:
    """Pair proposed at iteration t in row-major cyclic order."""
    idx = t % (n * (n - 1) // 2)
    r = 0
    while idx >= n - 1 - r:
        idx -= n - 1 - r
        r += 1
    return r, r + 1 + idx


def tie_T0(orc, A, B, p0, seed: int, chain: int, t_star: int, eps: float, iters: int,
           T_start: float | None = None, max_rounds: int = 40) -> float | None:
    """T0 of a constant schedule (alpha = 1) under which the oracle's run meets
    a near tie at iteration t_star with z = eps (up to rounding); None if the
    swap cost met at t_star is not positive or no fixed point is found.
    T_start is the first guess (the run up to t_star is taken at it)."""
    n = A.shape[0]
    r, s = pair_at(n, t_star)
    y = math.log(orc.uniform(seed, chain, t_star))
    if not eps - y > 0:
        return None
    if t_star == 0:
        d = orc.swap_cost(A, B, np.asarray(p0, dtype=np.int32), r, s)
        return d / (eps - y) if d > 0 else None
    T = T_start if T_start is not None else orc.schedule(A, B, p0, iters)["T0"]
    for _ in range(max_rounds):
        p = orc.sa_run(A, B, p0, iters, T, 1.0, seed, chain, t_end=t_star)["p"]
        d = orc.swap_cost(A, B, p, r, s)
        if d <= 0:
            return None
        T_new = d / (eps - y)
        if T_new == T:
            return T
        T = T_new
    return None


def identical_pair_instance(n: int, seed: int, sym: bool, lo: int = 0, hi: int = 60):
    """Instance whose facilities 0 and 1 have identical rows and columns of A:
    the swap (0, 1) always costs 0, so it is accepted whenever it is proposed,
    and it leaves the swap cost of every pair disjoint from {0, 1} unchanged
    (a first acceptance early in a scan window, followed by unchanged costs)."""
    rng = np.random.default_rng(seed)
    A = rng.integers(lo, hi + 1, (n, n)).astype(np.int64)
    B = rng.integers(lo, hi + 1, (n, n)).astype(np.int64)
    if sym:
        A = np.triu(A, 1); A = A + A.T
        B = np.triu(B, 1); B = B + B.T
    A[1, :] = A[0, :]
    A[:, 1] = A[:, 0]
    A[1, 1] = A[0, 0]
    A[0, 1] = A[1, 0]
    if sym:
        np.fill_diagonal(A, 0)
    return A.astype(np.int32), B.astype(np.int32), rng.permutation(n).astype(np.int32)


def find_tie(orc, A, B, p0, iters: int, eps: float, t_candidates, seeds, chain: int = 0,
             T_start: float | None = None):
    """First (seed, t*, T0) among the candidates whose constructed tie the
    oracle then logs at t* with the wanted sign of z."""
    for seed in seeds:
        for t_star in t_candidates:
            T0 = tie_T0(orc, A, B, p0, seed, chain, t_star, eps, iters, T_start)
            if T0 is None:
                continue
            ref = orc.sa_run(A, B, p0, iters, T0, 1.0, seed, chain, t_end=t_star + 1, tie_cap=64)
            hit = [float(z) for t, z in zip(ref["near_tie_t"], ref["near_tie_z"]) if int(t) == t_star]
            if hit and (eps == 0.0 or (hit[0] < 0) == (eps < 0)):
                return seed, t_star, T0
    return None
