"""Parity of the HIP path with the CPU oracle: element by element on small and
ragged instances, and on the standard workloads at full size against stored
oracle results (tests/golden/oracle_runs.json, written by make_golden.py from
the oracle alone).  Everything integer must match bit for bit; the trajectory
(accepted swaps, their hash, p, cost, best cost) must be identical."""
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


@pytest.fixture(scope="module")
def golden():
    with open(GOLD) as f:
        return json.load(f)


def _inst(n, seed, sym=False, lo=-3, hi=40):
    rng = np.random.default_rng(seed)
    A = rng.integers(lo, hi + 1, (n, n)).astype(np.int32)
    B = rng.integers(lo, hi + 1, (n, n)).astype(np.int32)
    if sym:
        A = np.triu(A, 1); A = (A + A.T).astype(np.int32)
        B = np.triu(B, 1); B = (B + B.T).astype(np.int32)
    return A, B, rng.permutation(n).astype(np.int32)


def _compare_run(orc, Q, A, B, p0, iters, seed, chain=0, T0=None, acc_cap=256, slices=None, flags=0,
                 switch_permille=0):
    print(f"[case] n={A.shape[0]} iters={iters} seed={seed} chain={chain} T0={T0} flags={flags} "
          f"switch={switch_permille}", flush=True)
    sched = orc.schedule(A, B, p0, iters)
    T0o = sched["T0"] if T0 is None else T0
    ref = orc.sa_run(A, B, p0, iters, T0o, sched["alpha"], seed, chain, acc_cap=acc_cap, tie_cap=256)
    ch = Q.Chain(A, B, p0, iters, seed, chain, T0=T0, accept_cap=acc_cap, tie_cap=256, flags=flags,
                 switch_permille=switch_permille).init()
    assert ch.sched.T0 == T0o and ch.sched.alpha == sched["alpha"]
    for t_end in (slices or []) + [iters]:
        ch.run(t_end)
    got = ch.result(with_delta=True)
    for k in ("t", "accepts", "hash", "cost", "best_cost", "best_iter", "near_ties"):
        assert got[k] == ref[k], (k, got[k], ref[k])
    assert np.array_equal(got["p"], ref["p"])
    if acc_cap:
        assert np.array_equal(got["accept_log"], ref["accept_log"])
    assert np.array_equal(got["near_tie_t"], np.sort(ref["near_tie_t"]))
    # final Delta and B' equal their definitions at the final p
    assert np.array_equal(got["delta"], orc.delta_matrix(A, B, got["p"]))
    assert np.array_equal(got["Bp"], B[np.ix_(got["p"], got["p"])])
    return got, ref


# ---------------------------------------------------------------- set-up path

@pytest.mark.parametrize("n,sym", [(2, False), (3, True), (7, False), (33, True), (65, False), (100, True)])
def test_delta_init_matches_oracle(orc, Q, n, sym):
    import torch
    A, B, p = _inst(n, 1000 + n, sym)
    ch = Q.Chain(A, B, p, 1000, 1).init()
    info = ch.info
    assert info.status == 0
    assert info.cost == orc.cost(A, B, p)
    ref = orc.delta_matrix(A, B, p)
    got = ch.delta.cpu().numpy().astype(np.int64)[: n * (n - 1) // 2]
    assert np.array_equal(got, ref)
    assert info.sum_abs_delta == int(np.abs(ref).sum())
    assert (info.a_min, info.a_max, info.b_min, info.b_max) == (A.min(), A.max(), B.min(), B.max())
    assert info.symmetric == int(sym or (np.array_equal(A, A.T) and np.array_equal(B, B.T)))
    assert np.array_equal(ch.Bp.cpu().numpy(), B[np.ix_(p, p)])
    c = torch.zeros(1, dtype=torch.int64, device="cuda")
    assert Q.qap_cost(n, ch.A, ch.B, ch.p, c) == 0
    assert int(c.item()) == orc.cost(A, B, p)


@pytest.mark.parametrize("name", ["n32_sym", "n150_asym"])
def test_delta_init_standard_workloads(orc, Q, name):
    ch = W.single_chain(name)
    c = Q.Chain(ch.A, ch.B, ch.p0, ch.iters, ch.philox_seed).init()
    ref = orc.delta_matrix(ch.A, ch.B, ch.p0)
    assert np.array_equal(c.delta.cpu().numpy().astype(np.int64), ref)
    T0, sabs = orc.mean_abs_delta(ch.n, ref)
    assert c.info.sum_abs_delta == sabs and c.sched.T0 == T0


def test_delta_init_reports_bad_inputs(Q):
    A, B, p = _inst(6, 5)
    with pytest.raises(Q.QapError) as e:
        Q.Chain(A, B, np.array([0, 1, 2, 3, 3, 5], dtype=np.int32), 10, 1).init()
    assert e.value.status == Q.QAP_E_NOT_PERM
    with pytest.raises(Q.QapError) as e:
        Q.Chain(A, B, np.array([0, 1, 2, 3, 9, 5], dtype=np.int32), 10, 1).init()
    assert e.value.status == Q.QAP_E_NOT_PERM
    big = np.full((6, 6), 2**24, dtype=np.int32)
    big[0, 1] = 0
    with pytest.raises(Q.QapError) as e:
        Q.Chain(big, big, p, 10, 1).init()
    assert e.value.status == Q.QAP_E_RANGE


# -------------------------------------------------------------- chain runs

MODES = [(0, 0), (1, 0), (2, 0), (0, 1000), (0, 300)]   # (flags, switch_permille)


@pytest.mark.parametrize("flags,switch", MODES)
@pytest.mark.parametrize("n,sym,iters", [(2, False, 500), (3, True, 700), (5, False, 3000), (8, True, 5000),
                                         (13, False, 20000), (31, True, 30000), (64, False, 40000),
                                         (97, False, 60000), (130, True, 60000), (150, False, 60000),
                                         (190, True, 50000)])
def test_chain_matches_oracle_small(orc, Q, n, sym, iters, flags, switch):
    A, B, p0 = _inst(n, 2000 + n, sym)
    _compare_run(orc, Q, A, B, p0, iters, seed=123 + n, chain=n % 5, flags=flags, switch_permille=switch)


@pytest.mark.parametrize("n,sym", [(9, False), (40, True), (77, False)])
def test_chain_wide_values_16bit_kernel(orc, Q, n, sym):
    """Value ranges above a byte take the 16-bit kernel (Delta mode throughout)."""
    A, B, p0 = _inst(n, 3000 + n, sym, lo=-300, hi=900)
    _compare_run(orc, Q, A, B, p0, 20000, seed=5)


@pytest.mark.parametrize("flags", [0, 1])
def test_chain_infinite_temperature(orc, Q, flags):
    A, B, p0 = _inst(40, 77)
    got, _ = _compare_run(orc, Q, A, B, p0, 5000, seed=9, T0=math.inf, acc_cap=5000, flags=flags)
    assert got["accepts"] == 5000


@pytest.mark.parametrize("n,sym", [(40, False), (41, True), (6, False)])
def test_lookahead_rounds_make_two_swaps(orc, Q, n, sym):
    """Scratch rounds that also test the proposals after the window's first
    one: at T = +inf every proposal is accepted, so nearly every round makes two
    swaps (its first proposal and the next one, in the state after the first
    swap), except at the ends of rows of the cyclic order, where plain rounds
    run; the run equals the oracle's swap by swap."""
    A, B, p0 = _inst(n, 80 + n, sym)
    iters = 3000
    sched = orc.schedule(A, B, p0, iters)
    ref = orc.sa_run(A, B, p0, iters, math.inf, sched["alpha"], 4, 0, acc_cap=iters, tie_cap=16)
    ch = Q.Chain(A, B, p0, iters, 4, 0, T0=math.inf, accept_cap=iters, flags=Q.QAP_FLAG_SCRATCH_ONLY,
                 profile=True).init()
    ch.run(1234)
    ch.run()
    got = ch.result(with_delta=True)
    for k in ("t", "accepts", "hash", "cost", "best_cost", "best_iter"):
        assert got[k] == ref[k], (k, got[k], ref[k])
    assert np.array_equal(got["accept_log"], ref["accept_log"])
    assert np.array_equal(got["Bp"], B[np.ix_(got["p"], got["p"])])
    ph = ch.phases()
    assert ph["n_scratch_acc"] == iters
    if n >= 40:   # rows of the cyclic order long enough for the look-ahead to run in most rounds
        assert ph["n_rounds"] < 0.7 * iters, ph["n_rounds"]


def test_chain_near_zero_temperature(orc, Q):
    A, B, p0 = _inst(25, 78, True)
    _compare_run(orc, Q, A, B, p0, 20000, seed=9, T0=1e-300)


@pytest.mark.parametrize("switch", [0, 200])
def test_chain_slices_are_seamless(orc, Q, switch):
    A, B, p0 = _inst(45, 79)
    _compare_run(orc, Q, A, B, p0, 50000, seed=3, slices=[1, 777, 20000, 20001, 49999], switch_permille=switch)


def test_stale_delta_between_scratch_slices(orc, Q):
    """A call that stops in scratch mode leaves Delta stale (and says so); a
    later call that needs Delta rebuilds it, so the trajectory and the final
    Delta are unchanged."""
    A, B, p0 = _inst(60, 81)
    s = orc.schedule(A, B, p0, 40000)
    ref = orc.sa_run(A, B, p0, 40000, s["T0"], s["alpha"], 4, 0)
    c = Q.Chain(A, B, p0, 40000, 4, 0, flags=Q.QAP_FLAG_SCRATCH_ONLY).init()
    c.run(10000)
    assert c.state().mode == Q.QAP_MODE_SCRATCH_STALE
    c.sched.flags = Q.QAP_FLAG_DELTA_ONLY
    c.run(25000)
    assert c.state().mode == Q.QAP_MODE_DELTA
    c.sched.flags = Q.QAP_FLAG_SCRATCH_ONLY
    c.run()
    got = c.result(with_delta=True)
    assert got["mode"] == Q.QAP_MODE_SCRATCH
    for k in ("t", "accepts", "hash", "cost", "best_cost", "best_iter", "near_ties"):
        assert got[k] == ref[k], k
    assert np.array_equal(got["p"], ref["p"])
    assert np.array_equal(got["delta"], orc.delta_matrix(A, B, got["p"]))


def test_chain_n32_full(orc, Q, golden):
    ch = W.single_chain("n32_sym")
    _compare_run(orc, Q, ch.A, ch.B, ch.p0, ch.iters, ch.philox_seed, acc_cap=1000)


def _check_golden(Q, ch, g, t_end=None):
    c = Q.Chain(ch.A, ch.B, ch.p0, ch.iters, ch.philox_seed, ch.chain_id).init()
    assert c.sched.T0 == g["T0"] and c.sched.alpha == g["alpha"]
    assert c.info.sum_abs_delta == g["sum_abs_delta0"] and c.info.cost == g["cost0"]
    c.run(t_end)
    r = c.result()
    for k in ("t", "accepts", "hash", "cost", "best_cost", "best_iter", "near_ties"):
        key = "t_end" if k == "t" else k
        assert r[k] == g[key], (k, r[k], g[key])
    assert r["p"].tolist() == g["p"]
    assert r["near_tie_t"].tolist() == sorted(g["near_tie_t"])
    return c


def test_chain_n150_prefix_golden(Q, golden):
    ch = W.single_chain("n150_asym")
    _check_golden(Q, ch, golden["n150_asym@3000000"], 3_000_000)


@pytest.mark.slow
def test_chain_n150_full_golden(orc, Q, golden):
    ch = W.single_chain("n150_asym")
    c = _check_golden(Q, ch, golden["n150_asym@100000000"])
    r = c.result(with_delta=True)
    # sampled final Delta entries equal the definition at the final p
    rng = np.random.default_rng(0)
    for idx in rng.choice(c.m, 200, replace=False):
        r_, s_ = _pair(ch.n, int(idx))
        assert r["delta"][idx] == orc.swap_cost(ch.A, ch.B, r["p"], r_, s_)


def _pair(n, idx):
    r = 0
    while idx >= n - 1 - r:
        idx -= n - 1 - r
        r += 1
    return r, r + 1 + idx
