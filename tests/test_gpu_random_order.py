"""Parity of the random proposal order (QAP_FLAG_RANDOM_ORDER) with the CPU
oracle's random-order run, on every kernel that runs a chain: the
one-workgroup kernel in each mode and placement, the 16-bit kernel, the
multi-workgroup kernel and batches.  The trajectory and the final Delta and B'
must match bit for bit."""
import math

import numpy as np
import pytest

from paper_1208_2675_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def Q():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1208_2675_amd import qapsa
    return qapsa


def _inst(n, seed, sym=False, lo=-3, hi=40):
    rng = np.random.default_rng(seed)
    A = rng.integers(lo, hi + 1, (n, n)).astype(np.int32)
    B = rng.integers(lo, hi + 1, (n, n)).astype(np.int32)
    if sym:
        A = np.triu(A, 1); A = (A + A.T).astype(np.int32)
        B = np.triu(B, 1); B = (B + B.T).astype(np.int32)
    return A, B, rng.permutation(n).astype(np.int32)


def _compare(orc, Q, A, B, p0, iters, seed, chain=0, T0=None, flags=0, switch=0, slices=(), acc_cap=256):
    n = A.shape[0]
    flags |= Q.QAP_FLAG_RANDOM_ORDER
    print(f"[case] random order n={n} iters={iters} seed={seed} T0={T0} flags={flags} switch={switch} "
          f"slices={slices}", flush=True)
    s = orc.schedule(A, B, p0, iters)
    T0o = s["T0"] if T0 is None else T0
    ref = orc.sa_run(A, B, p0, iters, T0o, s["alpha"], seed, chain, acc_cap=acc_cap, tie_cap=256, order=1)
    c = Q.Chain(A, B, p0, iters, seed, chain, T0=T0, accept_cap=acc_cap, tie_cap=256, flags=flags,
                switch_permille=switch).init()
    for t_end in list(slices) + [iters]:
        c.run(t_end)
    got = c.result(with_delta=True)
    assert got["status"] == 0
    for k in ("t", "accepts", "hash", "cost", "best_cost", "best_iter", "near_ties"):
        assert got[k] == ref[k], (k, got[k], ref[k])
    assert np.array_equal(got["p"], ref["p"])
    if acc_cap:
        assert np.array_equal(got["accept_log"], ref["accept_log"])
    assert np.array_equal(got["near_tie_t"], np.sort(ref["near_tie_t"]))
    assert np.array_equal(got["delta"], orc.delta_matrix(A, B, got["p"]))
    assert np.array_equal(got["Bp"], B[np.ix_(got["p"], got["p"])])
    return got, ref


MODES = [(0, 0), (1, 0), (2, 0), (0, 1000), (0, 300)]   # (flags, switch_permille)


@pytest.mark.parametrize("flags,switch", MODES)
@pytest.mark.parametrize("n,sym,iters", [(2, False, 500), (3, True, 700), (7, False, 5000), (33, True, 30000),
                                         (65, False, 40000), (150, False, 60000), (190, True, 40000)])
def test_one_workgroup_matches_oracle(orc, Q, n, sym, iters, flags, switch):
    A, B, p0 = _inst(n, 7000 + n, sym)
    _compare(orc, Q, A, B, p0, iters, seed=31 + n, chain=n % 3, flags=flags, switch=switch)


@pytest.mark.parametrize("n,sym", [(170, False), (230, False), (300, True)])
def test_device_memory_placements(orc, Q, n, sym):
    """Chains that keep Delta (and A, B') in device memory."""
    A, B = W.sym_uniform(n, (410, n)) if sym else W.asym_sparse_grid(n, (410, n))
    p0 = W.random_perm(n, (411, n))
    _compare(orc, Q, A, B, p0, 30000, seed=W.philox_key(412, n))


@pytest.mark.parametrize("n,sym", [(9, False), (40, True)])
def test_16bit_kernel(orc, Q, n, sym):
    A, B, p0 = _inst(n, 7100 + n, sym, lo=-300, hi=900)
    _compare(orc, Q, A, B, p0, 20000, seed=6)


@pytest.mark.parametrize("flags", [0, 1])
def test_infinite_temperature(orc, Q, flags):
    A, B, p0 = _inst(40, 7200)
    got, _ = _compare(orc, Q, A, B, p0, 5000, seed=8, T0=math.inf, flags=flags, acc_cap=5000)
    assert got["accepts"] == 5000


def test_near_zero_temperature(orc, Q):
    A, B, p0 = _inst(25, 7201, True)
    _compare(orc, Q, A, B, p0, 20000, seed=9, T0=1e-300)


@pytest.mark.parametrize("switch", [0, 200])
def test_slices_are_seamless(orc, Q, switch):
    A, B, p0 = _inst(45, 7202)
    _compare(orc, Q, A, B, p0, 50000, seed=3, slices=(1, 777, 20000, 20001, 49999), switch=switch)


def _sym(n, seed, hi=99):
    rng = np.random.default_rng(seed)
    A = np.triu(rng.integers(0, hi + 1, (n, n)), 1)
    B = np.triu(rng.integers(0, hi + 1, (n, n)), 1)
    return (A + A.T).astype(np.int32), (B + B.T).astype(np.int32), rng.permutation(n).astype(np.int32)


@pytest.mark.parametrize("n,iters", [(201, 20000), (333, 20000)])
def test_multi_workgroup_matches_oracle(orc, Q, n, iters):
    A, B, p0 = _sym(n, 7300 + n)
    got, _ = _compare(orc, Q, A, B, p0, iters, seed=11 + n, flags=Q.QAP_FLAG_MULTI_WG, slices=(4321,))
    assert got["mode"] in (Q.QAP_MODE_SCRATCH, Q.QAP_MODE_DELTA)


def test_multi_workgroup_infinite_temperature(orc, Q):
    A, B, p0 = _sym(260, 7400)
    got, _ = _compare(orc, Q, A, B, p0, 3000, seed=12, T0=math.inf, flags=Q.QAP_FLAG_MULTI_WG, acc_cap=3000)
    assert got["accepts"] == 3000


def test_batch_matches_oracle_per_chain(orc, Q):
    chains = W.batched_mix(n_instances=8, chains_per_instance=2, iters=20000, n_lo=20, n_hi=200, seed=91)
    refs = []
    for ch in chains:
        s = orc.schedule(ch.A, ch.B, ch.p0, ch.iters)
        refs.append(orc.sa_run(ch.A, ch.B, ch.p0, ch.iters, s["T0"], s["alpha"], ch.philox_seed, ch.chain_id,
                               tie_cap=16, order=1))
    b = Q.Batch(chains).init(flags=Q.QAP_FLAG_RANDOM_ORDER)
    b.run(slice_iters=7777)
    b.run()
    for i, (ch, st, ref) in enumerate(zip(b.chains, b.states(), refs)):
        for k in ("t", "accepts", "hash", "cost", "best_cost", "best_iter", "near_ties"):
            assert st[k] == ref[k], (i, ch.name, k, st[k], ref[k])
        assert np.array_equal(b.perm(i), ref["p"]), (i, ch.name)


# ------------------------------------------------------- full-size workloads

def _golden(key):
    import json
    import os
    with open(os.path.join(os.path.dirname(__file__), "golden", "oracle_runs.json")) as f:
        return json.load(f)[key]


def _check_state(r, g):
    for k in ("accepts", "hash", "cost", "best_cost", "best_iter", "near_ties"):
        assert r[k] == g[k], (k, r[k], g[k])
    assert r["t"] == g["t_end"]
    assert r["p"].tolist() == g["p"]


def _sampled_delta(orc, ch, r, k, seed):
    rng = np.random.default_rng(seed)
    n = ch.n
    for _ in range(k):
        a_, b_ = sorted(rng.choice(n, 2, replace=False))
        idx = a_ * (2 * n - a_ - 1) // 2 + b_ - a_ - 1
        assert r["delta"][idx] == orc.swap_cost(ch.A, ch.B, r["p"], int(a_), int(b_))


@pytest.mark.slow
def test_n150_full_schedule_against_stored_oracle_run(orc, Q):
    """N = 150 asymmetric, I = 1e8, random order, against the oracle's full run."""
    g = _golden("n150_asym@100000000:random")
    ch = W.single_chain("n150_asym")
    c = Q.Chain(ch.A, ch.B, ch.p0, ch.iters, ch.philox_seed, ch.chain_id, flags=Q.QAP_FLAG_RANDOM_ORDER).init()
    assert c.sched.T0 == g["T0"] and c.sched.alpha == g["alpha"]
    c.run()
    r = c.result(with_delta=True)
    _check_state(r, g)
    _sampled_delta(orc, ch, r, 200, 2)


@pytest.mark.parametrize("flags", [0, 1])   # the library's choice (scratch mode first); Delta mode throughout
def test_n2000_prefix_against_stored_oracle_run(orc, Q, flags):
    """N = 2000 symmetric on the multi-workgroup kernel, random order, first 3e5
    iterations of the I = 1e9 schedule."""
    g = _golden("n2000_sym@300000:random")
    ch = W.single_chain("n2000_sym")
    print(f"[case] n2000_sym random order prefix flags={flags}", flush=True)
    c = Q.Chain(ch.A, ch.B, ch.p0, ch.iters, ch.philox_seed, ch.chain_id,
                flags=Q.QAP_FLAG_RANDOM_ORDER | flags).init()
    assert c.sched.T0 == g["T0"] and c.sched.alpha == g["alpha"]
    c.run(300_000)
    r = c.result(with_delta=True)
    _check_state(r, g)
    rows = np.random.default_rng(4).choice(ch.n, 4, replace=False)
    for row in rows:
        assert np.array_equal(r["Bp"][row], ch.B[r["p"][row]][r["p"]])
    if r["mode"] != Q.QAP_MODE_SCRATCH_STALE:   # Delta is not kept in scratch mode
        _sampled_delta(orc, ch, r, 300, 3)


@pytest.mark.parametrize("flags,switch", [(2, 0), (0, 1000), (1, 0)])
@pytest.mark.parametrize("sym", [True, False])
def test_multi_workgroup_modes_random_order(orc, Q, flags, switch, sym):
    """Random proposal order over many workgroups in scratch mode, across the
    switch, and in Delta mode."""
    n = 240
    if sym:
        A, B, p0 = _sym(n, 7500)
    else:
        rng = np.random.default_rng(7501)
        A = rng.integers(0, 100, (n, n)).astype(np.int32)
        B = rng.integers(0, 100, (n, n)).astype(np.int32)
        p0 = rng.permutation(n).astype(np.int32)
    _compare(orc, Q, A, B, p0, 30000, seed=13, flags=Q.QAP_FLAG_MULTI_WG | flags, switch=switch,
             slices=(3, 9000, 9001))
