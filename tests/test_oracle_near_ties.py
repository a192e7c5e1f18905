"""Pins of the oracle's near-tie branch of Eq. (2): ties constructed so that
z = delta / T + log r is known in advance (tests/tie_cases.py), checked for
being logged, for the logged z, for the decision taken and for the edges of
the |z| < 1e-12 band."""
import math
import sys
import os

import numpy as np
import pytest

sys.path.insert(0, os.path.dirname(__file__))
import tie_cases as TC  # noqa: E402


def _inst(n, seed, sym=False, lo=0, hi=60):
    rng = np.random.default_rng(seed)
    A = rng.integers(lo, hi + 1, (n, n)).astype(np.int32)
    B = rng.integers(lo, hi + 1, (n, n)).astype(np.int32)
    if sym:
        A = np.triu(A, 1); A = (A + A.T).astype(np.int32)
        B = np.triu(B, 1); B = (B + B.T).astype(np.int32)
    return A, B, rng.permutation(n).astype(np.int32)


def _first_tie_inst(orc, eps, inst_seed=1, n=12):
    """An instance whose first proposal (0, 1) has a positive swap cost, and
    the generator seed and T0 that put a tie of value eps at iteration 0."""
    for k in range(inst_seed, inst_seed + 100):
        A, B, p0 = _inst(n, k)
        T0 = TC.tie_T0(orc, A, B, p0, 3, 0, 0, eps, 100)
        if T0 is not None:
            return A, B, p0, 3, T0
    raise AssertionError("no positive first swap cost")


@pytest.mark.parametrize("eps", [-1e-13, 1e-13, -5e-13, 5e-13])
def test_tie_at_first_proposal(orc, eps):
    A, B, p0, seed, T0 = _first_tie_inst(orc, eps)
    d = orc.swap_cost_by_definition(A, B, p0, 0, 1)
    y = math.log(orc.uniform(seed, 0, 0))
    # by construction delta / T0 = eps - log r up to rounding, so z = eps up to
    # the rounding of the two additions (a few ulp of |log r| < 37)
    res = orc.sa_run(A, B, p0, 100, T0, 1.0, seed, 0, t_end=1, tie_cap=8, acc_cap=1)
    assert res["near_ties"] == 1 and res["near_tie_t"].tolist() == [0]
    z = float(res["near_tie_z"][0])
    assert abs(z - eps) < 16 * math.ulp(abs(y)) + 1e-3 * abs(eps)
    assert d > 0 and T0 == d / (eps - y)
    # Eq. (2): the swap is made iff z < 0
    assert res["accepts"] == (1 if eps < 0 else 0)
    if eps < 0:
        assert res["accept_log"][0].tolist() == [0, 0, 1, d]


@pytest.mark.parametrize("eps", [-2e-12, 2e-12, -1e-11])
def test_outside_the_band_is_not_logged(orc, eps):
    A, B, p0, seed, T0 = _first_tie_inst(orc, eps)
    res = orc.sa_run(A, B, p0, 100, T0, 1.0, seed, 0, t_end=1, tie_cap=8)
    assert res["near_ties"] == 0
    assert res["accepts"] == (1 if eps < 0 else 0)


def test_exact_tie_is_logged_and_decided_by_its_sign(orc):
    """eps = 0: z is 0 or a few ulp either side; whichever it is, it is logged
    and the decision is z < 0."""
    A, B, p0, seed, T0 = _first_tie_inst(orc, 0.0, inst_seed=7)
    y = math.log(orc.uniform(seed, 0, 0))
    res = orc.sa_run(A, B, p0, 100, T0, 1.0, seed, 0, t_end=1, tie_cap=8)
    assert res["near_ties"] == 1
    z = float(res["near_tie_z"][0])
    assert abs(z) <= 4 * math.ulp(abs(y))
    assert res["accepts"] == (1 if z < 0 else 0)


@pytest.mark.parametrize("sym", [False, True])
def test_tie_in_mid_run_is_logged_once(orc, sym):
    """A tie at a later iteration t* of a constant-temperature run, on an
    instance whose swap (0, 1) always costs 0 (accepted at the start of every
    sweep, leaving the other pairs' costs unchanged): logged exactly once, at
    t*, and the run is the same as before t* with the tie evaluated on."""
    A, B, p0 = TC.identical_pair_instance(14, 5, sym)
    n, iters = 14, 3000
    T_start = orc.schedule(A, B, p0, iters)["T0"] / 30
    found = None
    for seed in range(1, 60):
        cands = [t for t in range(270, 600) if not {0, 1} & set(TC.pair_at(n, t))
                 and math.log(orc.uniform(seed, 0, t)) < -5]
        found = TC.find_tie(orc, A, B, p0, iters, -1e-13, cands[:5], [seed], T_start=T_start)
        if found:
            break
    assert found
    seed, t_star, T0 = found
    res = orc.sa_run(A, B, p0, iters, T0, 1.0, seed, 0, tie_cap=64, acc_cap=iters)
    assert res["near_tie_t"].tolist() == [t_star]
    assert abs(float(res["near_tie_z"][0]) + 1e-13) < 1e-14
    assert t_star in res["accept_log"][:, 0]
    # the swap (0, 1) is accepted every time it is proposed
    m = n * (n - 1) // 2
    zero_swaps = [tuple(x) for x in res["accept_log"] if x[1] == 0 and x[2] == 1]
    assert len(zero_swaps) == (iters + m - 1) // m and all(x[3] == 0 for x in zero_swaps)
    # splitting the run at t* changes nothing, and the tie is counted once
    a = orc.sa_run(A, B, p0, iters, T0, 1.0, seed, 0, t_end=t_star, tie_cap=64)
    b = orc.sa_run(A, B, a["p"], iters, T0, 1.0, seed, 0, state=a["state"], tie_cap=64)
    assert b["near_ties"] == 1 and b["hash"] == res["hash"] and np.array_equal(b["p"], res["p"])
