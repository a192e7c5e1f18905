"""The CPU Delta-matrix comparator (the paper's comparator type, timed by the
benchmark) walks the oracle's trajectory in every mode: from-scratch costs
throughout, the Delta matrix throughout, and the switch between them."""
import math

import numpy as np
import pytest


@pytest.fixture(scope="module")
def cmp():
    import cpu_comparator
    cpu_comparator.build()
    return cpu_comparator


def _inst(n, seed, sym):
    rng = np.random.default_rng(seed)
    A = rng.integers(-4, 60, (n, n)).astype(np.int32)
    B = rng.integers(-4, 60, (n, n)).astype(np.int32)
    if sym:
        A = np.triu(A, 1); A = (A + A.T).astype(np.int32)
        B = np.triu(B, 1); B = (B + B.T).astype(np.int32)
    return A, B, rng.permutation(n).astype(np.int32)


@pytest.mark.parametrize("switch", [(0, 1), (-1, 1), None, (1, 2)])
@pytest.mark.parametrize("n,sym,seed,iters", [(2, False, 1, 300), (5, True, 2, 4000), (12, False, 3, 30000),
                                              (31, True, 4, 60000), (47, False, 5, 80000)])
def test_same_trajectory_as_the_oracle(orc, cmp, n, sym, seed, iters, switch):
    A, B, p0 = _inst(n, seed, sym)
    s = orc.schedule(A, B, p0, iters)
    ref = orc.sa_run(A, B, p0, iters, s["T0"], s["alpha"], 9, 2)
    got = cmp.sa_run(A, B, p0, iters, s["T0"], s["alpha"], 9, 2, switch=switch)
    for k in ("t", "accepts", "hash", "cost", "best_cost", "best_iter", "near_ties"):
        assert got[k] == ref[k], (k, got[k], ref[k])
    assert np.array_equal(got["p"], ref["p"])
    if switch == (-1, 1):
        assert got["delta_mode_at"] == 0


def test_infinite_temperature_and_slices(orc, cmp):
    A, B, p0 = _inst(20, 6, False)
    ref = orc.sa_run(A, B, p0, 5000, math.inf, 1.0, 3, 0)
    got = cmp.sa_run(A, B, p0, 5000, math.inf, 1.0, 3, 0, switch=(-1, 1))
    assert got["accepts"] == 5000 and got["hash"] == ref["hash"] and np.array_equal(got["p"], ref["p"])
    s = orc.schedule(A, B, p0, 40000)
    ref = orc.sa_run(A, B, p0, 40000, s["T0"], s["alpha"], 3, 0)
    a = cmp.sa_run(A, B, p0, 40000, s["T0"], s["alpha"], 3, 0, t_end=12345)
    b = cmp.sa_run(A, B, a["p"], 40000, s["T0"], s["alpha"], 3, 0, state=a["state"])
    assert b["hash"] == ref["hash"] and b["cost"] == ref["cost"] and np.array_equal(b["p"], ref["p"])
