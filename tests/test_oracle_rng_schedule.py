"""Pins of the oracle's random numbers (Eq. (2)'s r) and cooling schedule.

The generator is checked against rocRAND's Philox-4x32-10, an independent
published implementation that is compiled and run here (host side only), not
copied.  The temperature tables are checked against closed forms."""
import math
import os
import shutil
import subprocess

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def rocrand_probe(tmp_path_factory):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc) or not os.path.exists("/opt/rocm/include/rocrand"):
        pytest.skip("hipcc / rocRAND headers not available")
    exe = str(tmp_path_factory.mktemp("probe") / "rocrand_philox_probe")
    subprocess.run([hipcc, "-O1", "-x", "hip", "--cuda-host-only", "-o", exe,
                    os.path.join(HERE, "probes", "rocrand_philox_probe.cpp")],
                   check=True, capture_output=True)
    return exe


def test_philox_matches_rocrand(orc, rocrand_probe):
    rng = np.random.default_rng(2024)
    cases = [(0, 0, 0), (2**64 - 1, 2**64 - 1, 2**62 - 1), (1234567, 3, 99)]
    for _ in range(200):
        cases.append((int(rng.integers(0, 2**63)) * 2 + int(rng.integers(0, 2)),
                      int(rng.integers(0, 2**32)), int(rng.integers(0, 2**40))))
    inp = "".join(f"{s} {q} {b}\n" for s, q, b in cases)
    out = subprocess.run([rocrand_probe], input=inp, capture_output=True, text=True, check=True)
    lines = out.stdout.split("\n")
    for (seed, subseq, block), line in zip(cases, lines):
        ref = [int(w, 16) for w in line.split()]
        ctr = [block & 0xFFFFFFFF, (block >> 32) & 0xFFFFFFFF, subseq & 0xFFFFFFFF, (subseq >> 32) & 0xFFFFFFFF]
        key = [seed & 0xFFFFFFFF, (seed >> 32) & 0xFFFFFFFF]
        assert orc.philox4x32_10(ctr, key).tolist() == ref, (seed, subseq, block)


def test_uniform_is_the_stated_dyadic_map(orc):
    """r_t = (2u + 1) 2^-53 with u = (x0 << 20) | (x1 >> 12), counter (t lo, t hi, chain, 0)."""
    for seed, chain, t in [(0, 0, 0), (12, 0, 5), (2**40 + 3, 7, 2**33 + 9), (2**64 - 1, 2**32 - 1, 2**64 - 1)]:
        x = orc.philox4x32_10([t & 0xFFFFFFFF, t >> 32, chain, 0], [seed & 0xFFFFFFFF, seed >> 32])
        u = (int(x[0]) << 20) | (int(x[1]) >> 12)
        expect = (2 * u + 1) / 2.0**53
        r = orc.uniform(seed, chain, t)
        assert r == expect and 0.0 < r < 1.0


def test_uniform_distribution(orc):
    scipy_stats = pytest.importorskip("scipy.stats")
    r = np.array([orc.uniform(2, 0, t) for t in range(20000)])
    assert r.min() > 0.0 and r.max() < 1.0
    assert scipy_stats.kstest(r, "uniform").pvalue > 1e-3
    # distinct chains give distinct streams
    r1 = np.array([orc.uniform(2, 1, t) for t in range(2000)])
    assert not np.array_equal(r[:2000], r1)


def test_uniform_extremes_bound_log(orc):
    # the smallest and largest values the map can produce
    assert math.log((2 * 0 + 1) / 2.0**53) > -36.75
    assert (2 * (2**52 - 1) + 1) / 2.0**53 < 1.0


def test_temperature_tables_closed_form(orc):
    for iters in (1, 2, 1000, 10**6, 3 * 2**20 + 17, 10**9):
        alpha = orc.geometric_alpha(iters, 1e-3)
        if iters == 1:
            assert alpha == 1.0
            continue
        # alpha carries one rounding (2^-53 relative); raised to the power I - 1
        # that becomes about I * 2^-53
        tol_alpha = 1e-12 + iters * 2.3e-16
        assert abs(alpha ** (iters - 1) / 1e-3 - 1.0) < tol_alpha
        T0 = 1234.5
        ts = sorted(t for t in {0, 1, 1023, 1024, 1025, 2**20 - 1, 2**20, iters // 3, iters - 1} if t < iters)
        T = orc.temperatures(T0, alpha, iters, ts)
        assert T[0] == T0
        for t, Tt in zip(ts, T):
            exact = T0 * math.exp(t * math.log(alpha))
            assert abs(Tt / exact - 1.0) < 1e-8, (iters, t)
        assert abs(T[-1] / T0 / 1e-3 - 1.0) < 1e-8 + tol_alpha
        assert np.all(np.diff(T) <= 0)


def test_temperature_table_recurrence(orc):
    alpha = orc.geometric_alpha(5 * 2**20, 1e-3)
    L, M, H = orc.temperature_tables(alpha, 5 * 2**20)
    assert L[0] == M[0] == H[0] == 1.0 and H.size == 5
    for j in range(1, 1024):
        assert L[j] == L[j - 1] * alpha
    s1 = L[1023] * alpha
    for j in range(1, 1024):
        assert M[j] == M[j - 1] * s1
    s2 = M[1023] * s1
    for j in range(1, 5):
        assert H[j] == H[j - 1] * s2
