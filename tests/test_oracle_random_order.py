"""Pins of the oracle's random proposal order (Sec. 2.1 lets the next swap be
picked at random instead of in sequence): the pair draw covers every pair
evenly and is independent of the Metropolis draw of the same iteration; at
infinite and zero temperature the run has a closed form; an independent
re-simulation over Eq. (1) gives the same run; runs resume seamlessly and
never beat the brute-force optimum."""
import math

import numpy as np
import pytest

from test_oracle_sa import M64, _fp, _inst


def _pairs(n):
    # row-major r < s enumeration, built independently of the oracle's walk
    r, s = np.triu_indices(n, 1)
    return list(zip(r.tolist(), s.tolist()))


def test_pair_draw_is_even_and_in_range(orc):
    n = 10
    m = n * (n - 1) // 2
    T = 90_000
    idx = np.array([orc.random_pair_index(123, 4, t, m) for t in range(T)])
    assert idx.min() == 0 and idx.max() == m - 1
    counts = np.bincount(idx, minlength=m)
    chi2 = float(((counts - T / m) ** 2 / (T / m)).sum())
    # 44 degrees of freedom: mean 44, sd ~9.4; a shifted or truncated map fails by far
    assert 15 < chi2 < 90, chi2


def test_pair_draw_uses_its_own_word(orc):
    """The pair comes from the third output word; r_t from the first two, so the
    two draws of one iteration are uncorrelated."""
    m = 1999 * 1000
    T = 20_000
    idx = np.array([orc.random_pair_index(9, 0, t, m) for t in range(T)], dtype=np.float64)
    u = np.array([orc.uniform(9, 0, t) for t in range(T)])
    for t in (0, 1, 2**32 + 5):
        x = orc.philox4x32_10([t & 0xFFFFFFFF, t >> 32, 0, 0], [9, 0])
        assert orc.random_pair_index(9, 0, t, m) == (int(x[2]) * m) >> 32
    assert abs(np.corrcoef(idx, u)[0, 1]) < 0.05
    # the extremes of the word map to the first and the last pair
    assert orc.random_pair_index(9, 0, 0, 1) == 0


def test_infinite_temperature_applies_every_drawn_swap(orc):
    n, iters = 7, 400
    A, B, p0 = _inst(n, 11)
    res = orc.sa_run(A, B, p0, iters, math.inf, 1.0, seed=21, chain=2, acc_cap=iters, order=1)
    pairs = _pairs(n)
    m = len(pairs)
    p = p0.copy()
    h = 0
    for t in range(iters):
        r, s = pairs[orc.random_pair_index(21, 2, t, m)]
        d = orc.swap_cost_by_definition(A, B, p, r, s)
        assert tuple(res["accept_log"][t]) == (t, r, s, d)
        h = (h + _fp(t, r, s, d)) & M64
        p[[r, s]] = p[[s, r]]
    assert res["accepts"] == iters
    assert np.array_equal(res["p"], p)
    assert res["hash"] == h
    assert res["cost"] == orc.cost(A, B, p)


def test_zero_temperature_is_random_descent(orc):
    n, iters = 8, 1500
    A, B, p0 = _inst(n, 12)
    res = orc.sa_run(A, B, p0, iters, 1e-300, 1.0, seed=3, acc_cap=iters, order=1)
    pairs = _pairs(n)
    p = p0.copy()
    log = []
    for t in range(iters):
        r, s = pairs[orc.random_pair_index(3, 0, t, len(pairs))]
        d = orc.swap_cost_by_definition(A, B, p, r, s)
        if d <= 0:
            log.append((t, r, s, d))
            p[[r, s]] = p[[s, r]]
    assert [tuple(x) for x in res["accept_log"]] == log
    assert np.array_equal(res["p"], p)
    assert all(x[3] <= 0 for x in log)


@pytest.mark.parametrize("n,sym,seed", [(2, False, 3), (6, True, 4), (9, False, 5)])
def test_independent_resimulation(orc, n, sym, seed):
    iters = 3000
    A, B, p0 = _inst(n, seed, sym)
    sched = orc.schedule(A, B, p0, iters)
    T0, alpha = sched["T0"], sched["alpha"]
    res = orc.sa_run(A, B, p0, iters, T0, alpha, seed=78, chain=5, acc_cap=iters, order=1)
    temps = orc.temperatures(T0, alpha, iters, range(iters))
    pairs = _pairs(n)
    p = p0.copy()
    log = []
    c = orc.cost(A, B, p)
    for t in range(iters):
        r, s = pairs[orc.random_pair_index(78, 5, t, len(pairs))]
        q = p.copy()
        q[[r, s]] = q[[s, r]]
        d = orc.cost(A, B, q) - c
        if d <= 0 or (d / temps[t] + math.log(orc.uniform(78, 5, t))) < 0:
            log.append((t, r, s, d))
            p = q
            c += d
    assert [tuple(x) for x in res["accept_log"]] == log
    assert np.array_equal(res["p"], p)
    assert res["cost"] == c == orc.cost(A, B, p)
    assert 0 < res["accepts"] < iters


def test_resume_is_seamless(orc):
    A, B, p0 = _inst(12, 13)
    iters = 40_000
    s = orc.schedule(A, B, p0, iters)
    full = orc.sa_run(A, B, p0, iters, s["T0"], s["alpha"], 17, order=1)
    half = orc.sa_run(A, B, p0, iters, s["T0"], s["alpha"], 17, t_end=12_345, order=1)
    rest = orc.sa_run(A, B, half["p"], iters, s["T0"], s["alpha"], 17, state=half["state"], order=1)
    for k in ("accepts", "hash", "cost", "best_cost", "best_iter", "t"):
        assert rest[k] == full[k], k
    assert np.array_equal(rest["p"], full["p"])
    row = orc.sa_run(A, B, p0, iters, s["T0"], s["alpha"], 17)
    assert row["hash"] != full["hash"]


def test_never_beats_brute_force(orc):
    for seed in range(3):
        A, B, p0 = _inst(8, 60 + seed)
        best, _, _ = orc.brute_force(A, B)
        s = orc.schedule(A, B, p0, 20000)
        res = orc.sa_run(A, B, p0, 20000, s["T0"], s["alpha"], seed=seed, order=1)
        assert res["best_cost"] >= best and res["cost"] >= best


def test_unknown_order_is_refused(orc):
    A, B, p0 = _inst(5, 9)
    with pytest.raises(ValueError):
        orc.sa_run(A, B, p0, 10, 1.0, 1.0, seed=0, order=2)
