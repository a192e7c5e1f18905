"""Value ranges wider than a byte on the multi-workgroup kernel: A and B' kept
as 16-bit or 32-bit words (value minus minimum), all sums modulo 2^32, exact
because the Delta bound keeps every swap cost inside int32.  Parity with the
oracle, symmetric and asymmetric, with slices, at the sizes where one CU
cannot hold the chain and at small sizes forced onto the kernel."""
import math

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def Q():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1208_2675_amd import qapsa
    return qapsa


def _inst(n, seed, sym, a_lo, a_hi, b_lo, b_hi):
    rng = np.random.default_rng(seed)
    A = rng.integers(a_lo, a_hi + 1, (n, n)).astype(np.int64)
    B = rng.integers(b_lo, b_hi + 1, (n, n)).astype(np.int64)
    if sym:
        A = np.triu(A, 1); A = A + A.T
        B = np.triu(B, 1); B = B + B.T
    return A.astype(np.int32), B.astype(np.int32), rng.permutation(n).astype(np.int32)


def _compare(orc, Q, A, B, p0, iters, seed, flags=0, slices=(), T0=None, acc_cap=512):
    n = A.shape[0]
    print(f"[case] wide n={n} A=[{A.min()},{A.max()}] B=[{B.min()},{B.max()}] iters={iters} flags={flags}",
          flush=True)
    assert orc.check_bounds(A, B) == 0
    s = orc.schedule(A, B, p0, iters)
    T0o = s["T0"] if T0 is None else T0
    ref = orc.sa_run(A, B, p0, iters, T0o, s["alpha"], seed, 0, acc_cap=acc_cap, tie_cap=64)
    c = Q.Chain(A, B, p0, iters, seed, 0, T0=T0, accept_cap=acc_cap, flags=flags).init()
    for t_end in list(slices) + [iters]:
        c.run(t_end)
    got = c.result(with_delta=True)
    assert got["status"] == 0
    for k in ("t", "accepts", "hash", "cost", "best_cost", "best_iter", "near_ties"):
        assert got[k] == ref[k], (k, got[k], ref[k])
    assert np.array_equal(got["p"], ref["p"])
    assert np.array_equal(got["accept_log"], ref["accept_log"])
    assert np.array_equal(got["Bp"], B[np.ix_(got["p"], got["p"])])
    if n <= 400:
        assert np.array_equal(got["delta"], orc.delta_matrix(A, B, got["p"]))
    else:
        rng = np.random.default_rng(n)
        for _ in range(200):
            a_, b_ = sorted(rng.choice(n, 2, replace=False))
            idx = a_ * (2 * n - a_ - 1) // 2 + b_ - a_ - 1
            assert got["delta"][idx] == orc.swap_cost(A, B, got["p"], int(a_), int(b_))
    return got


# (n, symmetric, A range, B range): 16-bit words for ranges up to 65535, 32-bit beyond
CASES = [(300, False, (0, 999), (0, 999)), (300, True, (0, 999), (0, 999)),
         (300, False, (0, 29999), (0, 60)), (300, True, (-15000, 14999), (0, 60)),
         (1000, True, (0, 999), (0, 999)), (1000, False, (0, 999), (0, 999)),
         (300, False, (-50000, 49999), (0, 20)), (260, True, (0, 99999), (-10, 9))]


@pytest.mark.parametrize("n,sym,ar,br", CASES)
def test_wide_values_match_oracle(orc, Q, n, sym, ar, br):
    A, B, p0 = _inst(n, 7000 + n, sym, *ar, *br)
    _compare(orc, Q, A, B, p0, 20000 if n >= 1000 else 40000, seed=3 + n, slices=(1, 5000))


@pytest.mark.parametrize("sym", [False, True])
@pytest.mark.parametrize("ar", [(0, 999), (0, 70000)])
def test_wide_values_small_forced_multi_workgroup(orc, Q, sym, ar):
    A, B, p0 = _inst(37, 31, sym, *ar, 0, 30)
    _compare(orc, Q, A, B, p0, 30000, seed=4, flags=Q.QAP_FLAG_MULTI_WG)


def test_wide_values_infinite_and_low_temperature(orc, Q):
    A, B, p0 = _inst(280, 33, False, 0, 4999, 0, 499)
    got = _compare(orc, Q, A, B, p0, 3000, seed=1, T0=math.inf, acc_cap=3000)
    assert got["accepts"] == 3000
    _compare(orc, Q, A, B, p0, 100000, seed=2, T0=1.0)


# odd n with 16-bit words: the general form's own rows and columns of A do not
# fit the LDS of the Delta rows in scratch mode and are read from device memory
MODE_CASES = [(301, False, (0, 999), (0, 999)), (300, False, (0, 999), (0, 999)),
              (300, False, (-50000, 49999), (0, 20)), (260, True, (0, 99999), (-10, 9))]


@pytest.mark.parametrize("mode", ["scratch", "delta"])
@pytest.mark.parametrize("n,sym,ar,br", MODE_CASES)
def test_wide_values_scratch_and_delta_modes(orc, Q, n, sym, ar, br, mode):
    A, B, p0 = _inst(n, 7100 + n, sym, *ar, *br)
    flags = Q.QAP_FLAG_MULTI_WG | (Q.QAP_FLAG_SCRATCH_ONLY if mode == "scratch" else Q.QAP_FLAG_DELTA_ONLY)
    _compare(orc, Q, A, B, p0, 20000, seed=5 + n, flags=flags, slices=(1, 5000))
