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


def _trace(k, iters, n_lo=32, n_hi=300, rate=2000.0, seed=41):
    return W.served_trace(n_requests=k, rate=rate, iters=iters, n_lo=n_lo, n_hi=n_hi, seed=seed)


def test_served_equals_alone_and_oracle(orc, Q):
    from paper_1208_2675_amd.serve import Server
    reqs = _trace(16, 60000)
    assert any(not Q.fits_one_workgroup(q.chain.n, True, 99, 99) for q in reqs)   # both kernels take part
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
