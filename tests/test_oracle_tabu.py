"""Pins of the oracle's tabu search (the heuristic named in Sec. 2.2 and 2.4
as the origin of the Delta bookkeeping; the rules are this implementation's
reading): an independent re-simulation over Eq. (1), the closed-form first
move and descent without a tabu list, the no-return property of a long tabu
list, resumption, the cost invariant and the brute-force bound."""
import numpy as np
import pytest

from test_oracle_sa import M64, _fp, _inst


def _cost(A, B, p):
    # Eq. (1) written with numpy fancy indexing, independent of the oracle
    return int((A.astype(np.int64) * B.astype(np.int64)[np.ix_(p, p)]).sum())


def _resimulate(A, B, p0, iters, tenure):
    n = A.shape[0]
    p = p0.copy()
    tabu = np.zeros((n, n), dtype=np.int64)
    cost = _cost(A, B, p)
    best = cost
    log = []
    for t in range(iters):
        cands = []
        for r in range(n):
            for s in range(r + 1, n):
                q = p.copy()
                q[[r, s]] = q[[s, r]]
                d = _cost(A, B, q) - cost
                is_tabu = tabu[r, p[s]] > t and tabu[s, p[r]] > t
                cands.append((d, r, s, (not is_tabu) or cost + d < best))
        adm = [c for c in cands if c[3]]
        d, r, s, _ = min(adm or cands, key=lambda c: (c[0], c[1], c[2]))
        tabu[r, p[r]] = t + tenure
        tabu[s, p[s]] = t + tenure
        p[[r, s]] = p[[s, r]]
        cost += d
        best = min(best, cost)
        log.append((t, r, s, d))
    return p, cost, best, log


@pytest.mark.parametrize("n,sym,seed,tenure", [(2, False, 1, 3), (5, True, 2, 4), (6, False, 3, 6), (7, False, 4, 2)])
def test_independent_resimulation(orc, n, sym, seed, tenure):
    A, B, p0 = _inst(n, 500 + seed, sym)
    iters = 60
    res = orc.tabu_run(A, B, p0, iters, tenure, acc_cap=iters)
    p, cost, best, log = _resimulate(A, B, p0, iters, tenure)
    assert [tuple(x) for x in res["accept_log"]] == log
    assert np.array_equal(res["p"], p)
    assert res["cost"] == cost and res["best_cost"] == best
    assert res["accepts"] == iters
    assert res["hash"] == sum(_fp(*x) for x in log) & M64


def test_without_tabu_list_is_steepest_descent(orc):
    n = 9
    A, B, p0 = _inst(n, 601)
    iters = 40
    res = orc.tabu_run(A, B, p0, iters, 0, acc_cap=iters)
    p = p0.copy()
    for t, r, s, d in (tuple(x) for x in res["accept_log"]):
        D = orc.delta_matrix(A, B, p)          # packed row-major, pinned against Eq. (1) elsewhere
        iu = np.triu_indices(n, 1)
        k = int(np.argmin(D))                   # first minimum in row-major order
        assert (r, s, d) == (int(iu[0][k]), int(iu[1][k]), int(D[k]))
        p[[r, s]] = p[[s, r]]
    # a local minimum is reached, after which the least-cost swap is taken anyway
    ds = res["accept_log"][:, 3]
    first_up = np.argmax(ds >= 0)
    assert np.all(ds[:first_up] < 0) and first_up > 0


def test_long_tabu_list_never_returns(orc):
    """With a tenure longer than the run, a swap that puts both facilities
    back on locations they left is made only if it beats the best cost seen so
    far, or if every swap is of that kind."""
    n = 8
    A, B, p0 = _inst(n, 602)
    iters = 150
    res = orc.tabu_run(A, B, p0, iters, 10**6, acc_cap=iters)
    p = p0.copy()
    left = set()
    cost = _cost(A, B, p)
    best = cost
    forced = 0
    for t, r, s, d in (tuple(x) for x in res["accept_log"]):
        back = (r, p[s]) in left and (s, p[r]) in left
        if back and not cost + d < best:
            for a in range(n):
                for b in range(a + 1, n):
                    q = p.copy()
                    q[[a, b]] = q[[b, a]]
                    assert ((a, p[b]) in left and (b, p[a]) in left and
                            not _cost(A, B, q) < best), (t, a, b)
            forced += 1
        left.add((r, p[r]))
        left.add((s, p[s]))
        p[[r, s]] = p[[s, r]]
        cost += d
        best = min(best, cost)
    assert res["cost"] == cost == _cost(A, B, res["p"])
    assert forced < iters


def test_resume_carries_the_tabu_table(orc):
    A, B, p0 = _inst(12, 603)
    full = orc.tabu_run(A, B, p0, 300, 9)
    half = orc.tabu_run(A, B, p0, 123, 9)
    rest = orc.tabu_run(A, B, half["p"], 300, 9, state=half["state"], tabu=half["tabu"])
    for k in ("accepts", "hash", "cost", "best_cost", "best_iter", "t"):
        assert rest[k] == full[k], k
    assert np.array_equal(rest["p"], full["p"])
    assert np.array_equal(rest["tabu"], full["tabu"])


def test_never_beats_brute_force(orc):
    for seed in range(3):
        A, B, p0 = _inst(8, 610 + seed)
        best, _, _ = orc.brute_force(A, B)
        res = orc.tabu_run(A, B, p0, 400, 8)
        assert res["best_cost"] >= best and res["cost"] >= best
        assert res["cost"] == _cost(A, B, res["p"])


def test_invalid_inputs(orc):
    A, B, p0 = _inst(5, 9)
    with pytest.raises(ValueError):
        orc.tabu_run(A, B, p0, 10, -1)
    with pytest.raises(ValueError):
        orc.tabu_run(A, B, np.array([0, 0, 1, 2, 3], dtype=np.int32), 10, 3)
