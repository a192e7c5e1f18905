"""Pins of the oracle's Eq. (1) and swap costs against things other than itself:
a hand-worked example, a library QAP routine, a linear-algebra identity and
exhaustive enumeration."""
import itertools
import os

import numpy as np
import pytest

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _read_golden(name):
    d = {}
    with open(os.path.join(GOLD, name)) as f:
        for line in f:
            line = line.split("#", 1)[0].strip()
            if line:
                k, *v = line.split()
                d.setdefault(k, []).append([int(x) for x in v])
    return d


def _rand_inst(rng, n, lo=-5, hi=9):
    A = rng.integers(lo, hi + 1, (n, n)).astype(np.int32)
    B = rng.integers(lo, hi + 1, (n, n)).astype(np.int32)
    return A, B


def test_eq1_hand_worked_example(orc):
    g = _read_golden("eq1_hand_n3.txt")
    n = g["n"][0][0]
    A = np.array(g["A"][0], dtype=np.int32).reshape(n, n)
    B = np.array(g["B"][0], dtype=np.int32).reshape(n, n)
    p = np.array(g["p"][0], dtype=np.int32)
    assert orc.cost(A, B, p) == g["cost"][0][0]
    r, s, d = g["swap"][0]
    assert orc.swap_cost_by_definition(A, B, p, r, s) == d
    assert orc.swap_cost(A, B, p, r, s) == d


def test_eq1_orientation_matches_scipy_qap(orc):
    """scipy's quadratic_assignment reports the objective trace(A^T P B P^T) of the
    permutation col_ind it returns; with asymmetric A and B this fixes that p(i)
    is the location of facility i, not its inverse."""
    so = pytest.importorskip("scipy.optimize")
    rng = np.random.default_rng(11)
    inverse_differs = 0
    for n in (4, 6, 9, 12):
        for _ in range(3):
            A, B = _rand_inst(rng, n)
            res = so.quadratic_assignment(A, B, method="2opt",
                                          options={"rng": np.random.default_rng(int(rng.integers(1 << 30)))})
            assert orc.cost(A, B, res.col_ind) == int(round(res.fun))
            inverse_differs += orc.cost(A, B, np.argsort(res.col_ind)) != int(round(res.fun))
    # the check has teeth: the inverse permutation would usually fail it
    assert inverse_differs > 0


def test_eq1_trace_identity(orc):
    rng = np.random.default_rng(3)
    for n in (2, 3, 7, 20, 41):
        A, B = _rand_inst(rng, n, -50, 99)
        p = rng.permutation(n).astype(np.int32)
        P = np.zeros((n, n), dtype=np.int64)
        P[np.arange(n), p] = 1
        ref = int(np.trace(A.T.astype(np.int64) @ P @ B.astype(np.int64) @ P.T))
        assert orc.cost(A, B, p) == ref


@pytest.mark.parametrize("n", [2, 3, 4, 5, 6])
def test_swap_cost_exhaustive(orc, n):
    """Every permutation, every pair: the O(N) form equals two evaluations of Eq. (1)."""
    rng = np.random.default_rng(100 + n)
    A, B = _rand_inst(rng, n)
    for perm in itertools.permutations(range(n)):
        p = np.array(perm, dtype=np.int32)
        for r in range(n):
            for s in range(r + 1, n):
                assert orc.swap_cost(A, B, p, r, s) == orc.swap_cost_by_definition(A, B, p, r, s)


def test_swap_cost_sampled_large(orc):
    rng = np.random.default_rng(7)
    for n in (10, 23, 40):
        A, B = _rand_inst(rng, n, -1000, 1000)
        for _ in range(30):
            p = rng.permutation(n).astype(np.int32)
            r, s = sorted(rng.choice(n, 2, replace=False))
            assert orc.swap_cost(A, B, p, r, s) == orc.swap_cost_by_definition(A, B, p, r, s)


def test_delta_matrix_order_and_properties(orc):
    rng = np.random.default_rng(8)
    n = 9
    A, B = _rand_inst(rng, n)
    p = rng.permutation(n).astype(np.int32)
    d = orc.delta_matrix(A, B, p)
    assert d.shape == (n * (n - 1) // 2,)
    k = 0
    for r in range(n):
        for s in range(r + 1, n):
            assert d[k] == orc.swap_cost_by_definition(A, B, p, r, s)
            # swapping back undoes the change: the swap cost negates
            q = p.copy(); q[[r, s]] = q[[s, r]]
            assert orc.swap_cost(A, B, q, r, s) == -d[k]
            k += 1


def test_symmetric_zero_diagonal_gives_even_delta(orc):
    rng = np.random.default_rng(9)
    n = 15
    A = rng.integers(0, 100, (n, n)); A = np.triu(A, 1); A = (A + A.T).astype(np.int32)
    B = rng.integers(0, 100, (n, n)); B = np.triu(B, 1); B = (B + B.T).astype(np.int32)
    p = rng.permutation(n).astype(np.int32)
    assert np.all(orc.delta_matrix(A, B, p) % 2 == 0)


def test_brute_force_enumerates_all_and_is_optimal(orc):
    rng = np.random.default_rng(12)
    for n in (1, 2, 3, 5, 6, 7):
        A, B = _rand_inst(rng, n)
        best, pb, visited = orc.brute_force(A, B)
        assert visited == int(np.prod(range(1, n + 1)))
        assert orc.cost(A, B, pb) == best
        ref = min(
            int(sum(int(A[i, j]) * int(B[perm[i], perm[j]]) for i in range(n) for j in range(n)))
            for perm in itertools.permutations(range(n)))
        assert best == ref


def test_bounds_check(orc):
    A = np.full((4, 4), 2**30, dtype=np.int32)
    B = np.full((4, 4), 2**30, dtype=np.int32)
    assert orc.check_bounds(A, B) == -3
    A = np.arange(16, dtype=np.int32).reshape(4, 4)
    assert orc.check_bounds(A, A) == 0


def test_bounds_check_swap_cost_branch_alone(orc):
    """Values that keep the cost bound n^2 max|A| max|B| < 2^62 but break the
    swap-cost bound (2n + 8) range(A) range(B) < 2^62: entries of both signs,
    so the range is twice the magnitude.  With n = 4: 16 m^2 < 2^62 while
    16 (2m)^2 >= 2^62 for m = 2^28.5 (rounded down)."""
    m = 379625062
    A = np.array([[m if (i + j) % 2 else -m for j in range(4)] for i in range(4)], dtype=np.int32)
    n = 4
    assert n * n * m * m < 2**62 <= (2 * n + 8) * (2 * m) * (2 * m)
    assert orc.check_bounds(A, A) == -3
    # halving the magnitude keeps both bounds
    assert orc.check_bounds(A // 2, A // 2) == 0
    # one sign only: the range equals the magnitude, both bounds hold
    assert orc.check_bounds(np.abs(A), np.abs(A)) == 0


@pytest.mark.parametrize("n,sym,seed", [(2, False, 1), (5, True, 2), (9, False, 3), (23, True, 4)])
def test_mean_abs_delta_by_definition(orc, n, sym, seed):
    """T0 of the schedule is the mean of |C(p o (r s)) - C(p)| over the
    n(n-1)/2 pairs r < s, each swap cost taken from two evaluations of Eq. (1)
    (numpy here), averaged with one binary64 division of the integer sum."""
    rng = np.random.default_rng(seed)
    A = rng.integers(-5, 30, (n, n)).astype(np.int32)
    B = rng.integers(-5, 30, (n, n)).astype(np.int32)
    if sym:
        A = np.triu(A, 1); A = (A + A.T).astype(np.int32)
        B = np.triu(B, 1); B = (B + B.T).astype(np.int32)
    p = rng.permutation(n).astype(np.int32)

    def eq1(q):
        return int((A.astype(np.int64) * B.astype(np.int64)[np.ix_(q, q)]).sum())

    total = 0
    pairs = 0
    for r in range(n):
        for s in range(r + 1, n):
            q = p.copy()
            q[[r, s]] = q[[s, r]]
            total += abs(eq1(q) - eq1(p))
            pairs += 1
    assert pairs == n * (n - 1) // 2
    T0, sabs = orc.mean_abs_delta(n, orc.delta_matrix(A, B, p))
    assert sabs == total
    assert T0 == total / pairs
    sched = orc.schedule(A, B, p, 1000)
    assert sched["T0"] == total / pairs and sched["sum_abs"] == total
    if total:   # a wrong divisor would show: n(n-1) or n^2 pairs instead of n(n-1)/2
        assert T0 != total / (n * (n - 1)) and T0 != total / (n * n)
