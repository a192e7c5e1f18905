"""The serving loop: requests admitted by footprint into slots, advanced in
iteration slices together, retired when done.  Each served result must equal
the same request run alone (tolerance zero) and the oracle's run."""
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


def _trace(k, iters, n_lo=32, n_hi=300, rate=2000.0, seed=41, force=()):
    """Served trace; ``force`` maps request positions to instance sizes so that
    each kind of kernel (whole chain in LDS, chain with device scratch,
    multi-workgroup) is sure to take part."""
    reqs = W.served_trace(n_requests=k, rate=rate, iters=iters, n_lo=n_lo, n_hi=n_hi, seed=seed)
    for j, n in force:
        ch = reqs[j].chain
        A, B = W.sym_uniform(n, 7000 + j)
        reqs[j].chain = W.Chain(f"req{j}", A, B, W.random_perm(n, 7001 + j), ch.iters, ch.philox_seed,
                                ch.chain_id, True, {"kind": "sym_uniform"})
    return reqs


def test_served_equals_alone_and_oracle(orc, Q):
    from paper_1208_2675_amd.serve import Server
    reqs = _trace(16, 60000, force=((3, 470), (5, 260), (6, 90)))
    # chains wholly in LDS and chains with matrices in device scratch both take
    # part (n = 470: A and B' both in scratch)
    kinds = {Q.qap_single_workgroup(q.chain.n, 1, 99, 99) for q in reqs}
    assert kinds == {1, 2}, kinds
    srv = Server(max_slots=6, slice_iters=7000)
    st = srv.run_trace(reqs, time_limit=300)
    assert len(st.results) == len(reqs)
    by = {r.rid: r for r in st.results}
    for q in reqs:
        ch = q.chain
        alone = Q.Chain(ch.A, ch.B, ch.p0, ch.iters, ch.philox_seed, ch.chain_id).init().run().result()
        got = by[q.rid]
        for k in ("t", "accepts", "hash", "cost", "best_cost", "best_iter"):
            assert got.state[k] == alone[k], (q.rid, k)
        assert np.array_equal(got.p, alone["p"])
        if ch.n <= 64:
            s = orc.schedule(ch.A, ch.B, ch.p0, ch.iters)
            ref = orc.sa_run(ch.A, ch.B, ch.p0, ch.iters, s["T0"], s["alpha"], ch.philox_seed, ch.chain_id)
            assert got.state["hash"] == ref["hash"] and np.array_equal(got.p, ref["p"])


def test_admission_waits_for_memory(Q):
    from paper_1208_2675_amd.serve import Server, footprint_bytes
    reqs = _trace(6, 20000, n_lo=60, n_hi=120, seed=42)
    budget = max(footprint_bytes(q.chain.n, q.chain.iters) for q in reqs) + 1
    srv = Server(max_slots=8, memory_budget=budget, slice_iters=5000)
    st = srv.run_trace(reqs, time_limit=120)
    assert len(st.results) == 6
    assert st.waits_for_memory > 0
    assert max(st.resident_sum, 1) >= 1
