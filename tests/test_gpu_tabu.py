"""Parity of the tabu search on the device (qap_tabu_run: the one-workgroup
kernel's Delta update with a best-admissible-swap selection) with the
oracle's tabu search, swap by swap, in every placement of the chain state,
across calls, and after an annealing run."""
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


def _compare(orc, Q, A, B, p0, iters, tenure, slices=()):
    n = A.shape[0]
    print(f"[case] tabu n={n} iters={iters} tenure={tenure} slices={slices}", flush=True)
    ref = orc.tabu_run(A, B, p0, iters, tenure, acc_cap=iters)
    c = Q.Chain(A, B, p0, iters, 1, accept_cap=iters).init()
    for t_end in list(slices) + [iters]:
        c.tabu(t_end, tenure)
    got = c.result(with_delta=True)
    assert got["status"] == 0 and got["mode"] == Q.QAP_MODE_DELTA
    for k in ("t", "accepts", "hash", "cost", "best_cost", "best_iter"):
        assert got[k] == ref[k], (k, got[k], ref[k])
    assert np.array_equal(got["accept_log"], ref["accept_log"])
    assert np.array_equal(got["p"], ref["p"])
    assert np.array_equal(c.tabu_table.cpu().numpy().astype(np.int64), ref["tabu"])
    assert np.array_equal(got["delta"], orc.delta_matrix(A, B, got["p"]))
    assert np.array_equal(got["Bp"], B[np.ix_(got["p"], got["p"])])
    return got


@pytest.mark.parametrize("n,sym,iters,tenure", [(2, False, 20, 1), (3, True, 30, 2), (7, False, 200, 5),
                                                (20, True, 600, 20), (33, False, 800, 0), (64, False, 1000, 64),
                                                (100, True, 400, 10**6), (150, False, 200, 150)])
def test_tabu_matches_oracle(orc, Q, n, sym, iters, tenure):
    A, B, p0 = _inst(n, 8000 + n, sym)
    _compare(orc, Q, A, B, p0, iters, tenure)


def test_tabu_slices_are_seamless(orc, Q):
    A, B, p0 = _inst(40, 8100)
    _compare(orc, Q, A, B, p0, 500, 30, slices=(1, 37, 250, 251))


@pytest.mark.parametrize("n,sym", [(170, False), (230, False), (300, True)])
def test_tabu_device_memory_placements(orc, Q, n, sym):
    """Chains that keep Delta (and A, B') in device memory."""
    A, B = W.sym_uniform(n, (420, n)) if sym else W.asym_sparse_grid(n, (420, n))
    p0 = W.random_perm(n, (421, n))
    _compare(orc, Q, A, B, p0, 40, n)


def test_tabu_after_annealing(orc, Q):
    """A search started from an annealing chain's state (stale Delta after a
    scratch-mode call) continues its counters and rebuilds Delta first."""
    A, B, p0 = _inst(50, 8200)
    iters = 6000
    s = orc.schedule(A, B, p0, iters)
    sa = orc.sa_run(A, B, p0, iters, s["T0"], s["alpha"], 5, 0, t_end=4000)
    ref = orc.tabu_run(A, B, sa["p"], 4300, 25, state=sa["state"], acc_cap=0)
    c = Q.Chain(A, B, p0, iters, 5, 0, flags=Q.QAP_FLAG_SCRATCH_ONLY).init()
    c.run(4000)
    assert c.state().mode == Q.QAP_MODE_SCRATCH_STALE
    c.iters = 4300
    c.tabu(4300, 25)
    got = c.result(with_delta=True)
    for k in ("t", "accepts", "hash", "cost", "best_cost", "best_iter"):
        assert got[k] == ref[k], (k, got[k], ref[k])
    assert np.array_equal(got["p"], ref["p"])
    assert np.array_equal(got["delta"], orc.delta_matrix(A, B, got["p"]))
