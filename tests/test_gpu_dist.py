"""Parity of the multi-workgroup chain kernel (instances too large for one CU,
and smaller ones sent there by QAP_FLAG_MULTI_WG), symmetric and general
(asymmetric) forms, with the CPU oracle, and at N=2000 against stored oracle
results."""
import json
import math
import os

import numpy as np
import pytest

from paper_1208_2675_amd import workloads as W

pytestmark = pytest.mark.gpu
GOLD = os.path.join(os.path.dirname(__file__), "golden", "oracle_runs.json")


@pytest.fixture(scope="module")
def Q():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1208_2675_amd import qapsa
    return qapsa


def _sym(n, seed, hi=99):
    rng = np.random.default_rng(seed)
    A = np.triu(rng.integers(0, hi + 1, (n, n)), 1)
    B = np.triu(rng.integers(0, hi + 1, (n, n)), 1)
    return (A + A.T).astype(np.int32), (B + B.T).astype(np.int32), rng.permutation(n).astype(np.int32)


def _run_compare(orc, Q, A, B, p0, iters, seed, T0=None, slices=(), acc_cap=512, check_delta=True):
    n = A.shape[0]
    print(f"[case] dist n={n} iters={iters} seed={seed} T0={T0} slices={slices}", flush=True)
    s = orc.schedule(A, B, p0, iters)
    T0o = s["T0"] if T0 is None else T0
    ref = orc.sa_run(A, B, p0, iters, T0o, s["alpha"], seed, 0, acc_cap=acc_cap, tie_cap=64)
    c = Q.Chain(A, B, p0, iters, seed, 0, T0=T0, accept_cap=acc_cap, flags=Q.QAP_FLAG_MULTI_WG).init()
    for t_end in list(slices) + [iters]:
        c.run(t_end)
    got = c.result(with_delta=True)
    assert got["status"] == 0 and got["mode"] == Q.QAP_MODE_DELTA
    for k in ("t", "accepts", "hash", "cost", "best_cost", "best_iter", "near_ties"):
        assert got[k] == ref[k], (k, got[k], ref[k])
    assert np.array_equal(got["p"], ref["p"])
    assert np.array_equal(got["accept_log"], ref["accept_log"])
    assert np.array_equal(got["Bp"], B[np.ix_(got["p"], got["p"])])
    if check_delta:
        assert np.array_equal(got["delta"], orc.delta_matrix(A, B, got["p"]))
    return got


@pytest.mark.parametrize("n,iters", [(201, 30000), (260, 40000), (333, 40000), (517, 30000)])
def test_dist_matches_oracle(orc, Q, n, iters):
    A, B, p0 = _sym(n, 500 + n)
    _run_compare(orc, Q, A, B, p0, iters, seed=7 + n)


def test_dist_infinite_temperature(orc, Q):
    A, B, p0 = _sym(300, 61)
    got = _run_compare(orc, Q, A, B, p0, 3000, seed=1, T0=math.inf, acc_cap=3000)
    assert got["accepts"] == 3000


def test_dist_slices(orc, Q):
    A, B, p0 = _sym(280, 62)
    _run_compare(orc, Q, A, B, p0, 30000, seed=2, slices=(1, 999, 15000, 15001))


def test_dist_low_temperature(orc, Q):
    A, B, p0 = _sym(240, 63)
    _run_compare(orc, Q, A, B, p0, 200000, seed=3, T0=1.0)


def test_dist_n2000_prefix_golden(orc, Q):
    with open(GOLD) as f:
        g = json.load(f)["n2000_sym@2000000"]
    ch = W.single_chain("n2000_sym")
    c = Q.Chain(ch.A, ch.B, ch.p0, ch.iters, ch.philox_seed, ch.chain_id).init()
    assert c.sched.T0 == g["T0"] and c.sched.alpha == g["alpha"]
    assert c.info.sum_abs_delta == g["sum_abs_delta0"] and c.info.cost == g["cost0"]
    c.run(2_000_000)
    r = c.result(with_delta=True)
    for k in ("accepts", "hash", "cost", "best_cost", "best_iter", "near_ties"):
        assert r[k] == g[k], (k, r[k], g[k])
    assert r["t"] == g["t_end"]
    assert r["p"].tolist() == g["p"]
    # sampled Delta entries equal the definition at the final p
    rng = np.random.default_rng(1)
    n = ch.n
    for _ in range(300):
        a_, b_ = sorted(rng.choice(n, 2, replace=False))
        idx = a_ * (2 * n - a_ - 1) // 2 + b_ - a_ - 1
        assert r["delta"][idx] == orc.swap_cost(ch.A, ch.B, r["p"], int(a_), int(b_))


def test_dist_refuses_stale_delta(Q):
    """A chain that stopped in scratch mode mid-schedule leaves Delta stale; the
    multi-workgroup kernel, which needs Delta, reports QAP_E_STATE."""
    A, B, p0 = _sym(220, 64)
    c = Q.Chain(A, B, p0, 50000, 5, 0, flags=Q.QAP_FLAG_SCRATCH_ONLY).init()
    c.run(1000)
    st = c.state()
    assert st.mode == Q.QAP_MODE_SCRATCH_STALE and st.status == 0
    c.sched.flags = Q.QAP_FLAG_MULTI_WG
    c.run(2000)
    assert c.state().status == Q.QAP_E_STATE


def _asym(n, seed, hi=99):
    rng = np.random.default_rng(seed)
    A = rng.integers(0, hi + 1, (n, n)).astype(np.int32)
    B = rng.integers(0, hi + 1, (n, n)).astype(np.int32)
    np.fill_diagonal(A, rng.integers(0, hi + 1, n))   # the diagonal terms of Eq. (1) count too
    return A, B, rng.permutation(n).astype(np.int32)


@pytest.mark.parametrize("n,iters", [(9, 20000), (64, 30000), (300, 30000), (517, 20000)])
def test_dist_general_form_matches_oracle(orc, Q, n, iters):
    """Asymmetric A and B (non-zero diagonals): the general Taillard correction
    (rows and columns u, v staged) and the general touched-pair recomputation."""
    A, B, p0 = _asym(n, 900 + n)
    _run_compare(orc, Q, A, B, p0, iters, seed=11 + n)


def test_dist_general_form_slices_and_infinite_temperature(orc, Q):
    A, B, p0 = _asym(280, 71)
    _run_compare(orc, Q, A, B, p0, 30000, seed=2, slices=(1, 999, 15000, 15001))
    got = _run_compare(orc, Q, A, B, p0, 3000, seed=1, T0=math.inf, acc_cap=3000)
    assert got["accepts"] == 3000


def test_dist_general_form_low_temperature(orc, Q):
    A, B, p0 = _asym(240, 73)
    _run_compare(orc, Q, A, B, p0, 200000, seed=3, T0=1.0)


def test_dist_general_form_sparse_grid(orc, Q):
    """The workload family of the asymmetric single chain (sparse flows on a
    Manhattan grid) at a size past one CU's LDS."""
    A, B = W.asym_sparse_grid(333, 5)
    p0 = W.random_perm(333, 6)
    _run_compare(orc, Q, A, B, p0, 40000, seed=4)


def test_dist_general_form_n2000_prefix_golden(orc, Q):
    with open(GOLD) as f:
        g = json.load(f)["n2000_asym@300000"]
    ch = W.single_chain("n2000_asym")
    c = Q.Chain(ch.A, ch.B, ch.p0, ch.iters, ch.philox_seed, ch.chain_id).init()
    assert c.sched.T0 == g["T0"] and c.sched.alpha == g["alpha"]
    c.run(100_000)
    c.run(300_000)
    r = c.result(with_delta=True)
    for k in ("accepts", "hash", "cost", "best_cost", "best_iter", "near_ties"):
        assert r[k] == g[k], (k, r[k], g[k])
    assert r["t"] == g["t_end"] and r["p"].tolist() == g["p"]
    rng = np.random.default_rng(2)
    n = ch.n
    for _ in range(100):
        a_, b_ = sorted(rng.choice(n, 2, replace=False))
        idx = a_ * (2 * n - a_ - 1) // 2 + b_ - a_ - 1
        assert r["delta"][idx] == orc.swap_cost(ch.A, ch.B, r["p"], int(a_), int(b_))


@pytest.mark.parametrize("sym", [True, False])
@pytest.mark.parametrize("flags,window", [(16, 0), (16, 256), (16, 16384), (4, 16), (4, 1024), (4, 65536)])
def test_dispatch_choices_do_not_change_the_run(orc, Q, sym, flags, window):
    """Every (kernel, scan window) the dispatch tuner may pick gives the
    oracle's run: QAP_FLAG_SINGLE_WG (16) or QAP_FLAG_MULTI_WG (4), windows
    from 16 proposals to 65536."""
    n, iters = 230, 40000
    A, B, p0 = _sym(n, 77) if sym else _asym(n, 78)
    s = orc.schedule(A, B, p0, iters)
    ref = orc.sa_run(A, B, p0, iters, s["T0"], s["alpha"], 6, 0, tie_cap=16)
    print(f"[case] dispatch n={n} sym={sym} flags={flags} window={window}", flush=True)
    c = Q.Chain(A, B, p0, iters, 6, 0, flags=flags, scan_window=window).init()
    c.run(15000)
    c.run()
    got = c.result(with_delta=True)
    for k in ("t", "accepts", "hash", "cost", "best_cost", "best_iter", "near_ties"):
        assert got[k] == ref[k], (k, got[k], ref[k])
    assert np.array_equal(got["p"], ref["p"])
    assert np.array_equal(got["delta"], orc.delta_matrix(A, B, got["p"]))
