"""Batched chains of uneven size in one persistent launch: every chain equals
the oracle's run of that chain alone, whatever the batch and the slicing."""
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


def _mix(iters, k_inst=10, per=3, seed=77, n_hi=150):
    return W.batched_mix(n_instances=k_inst, chains_per_instance=per, iters=iters, n_lo=20, n_hi=n_hi, seed=seed)


def _oracle(orc, ch):
    s = orc.schedule(ch.A, ch.B, ch.p0, ch.iters)
    return orc.sa_run(ch.A, ch.B, ch.p0, ch.iters, s["T0"], s["alpha"], ch.philox_seed, ch.chain_id, tie_cap=16)


def _check(orc, Q, b, refs):
    sts = b.states()
    for i, (ch, st, ref) in enumerate(zip(b.chains, sts, refs)):
        for k in ("t", "accepts", "hash", "cost", "best_cost", "best_iter", "near_ties"):
            assert st[k] == ref[k], (i, ch.name, k, st[k], ref[k])
        assert np.array_equal(b.perm(i), ref["p"]), (i, ch.name)


@pytest.mark.parametrize("groups", [0, 5])
def test_batch_matches_oracle_per_chain(orc, Q, groups):
    chains = _mix(30000)
    refs = [_oracle(orc, ch) for ch in chains]
    b = Q.Batch(chains).init()
    b.run(groups=groups)
    _check(orc, Q, b, refs)


def test_batch_slices_and_order_do_not_change_results(orc, Q):
    chains = _mix(20000, k_inst=8, per=2, seed=78)
    refs = [_oracle(orc, ch) for ch in chains]
    b = Q.Batch(chains).init()
    import torch
    order = torch.arange(len(chains) - 1, -1, -1, dtype=torch.int32, device="cuda")
    k = 0
    while not b.done():
        b.run(slice_iters=3333, order=order if k % 2 else None, groups=3 + k % 4)
        k += 1
        assert k < 100
    _check(orc, Q, b, refs)


def test_batch_alone_equals_mixed(Q):
    chains = _mix(15000, k_inst=6, per=2, seed=79)
    mixed = Q.Batch(chains).init()
    mixed.run()
    sm = mixed.states()
    for i in (0, 5, 11):
        alone = Q.Batch([chains[i]]).init()
        alone.run(groups=1)
        assert alone.states()[0] == sm[i]
        assert np.array_equal(alone.perm(0), mixed.perm(i))
