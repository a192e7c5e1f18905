"""qap_sa_run_static, the entry point that allocates nothing (its workspace is
a device array inside the library), against qap_sa_run with a caller
workspace: the same chain through both, bit for bit, on the kernels that use
a workspace (the multi-workgroup kernel and a one-workgroup chain whose byte
matrices live in device scratch), two static calls in a row with the second
one smaller, so that it runs on what the first left in the shared array."""
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


def _inst(n, seed, sym):
    rng = np.random.default_rng(seed)
    A = rng.integers(0, 99, (n, n)).astype(np.int32)
    B = rng.integers(0, 99, (n, n)).astype(np.int32)
    if sym:
        A = np.triu(A, 1); A = (A + A.T).astype(np.int32)
        B = np.triu(B, 1); B = (B + B.T).astype(np.int32)
    return A, B, rng.permutation(n).astype(np.int32)


def _result(c):
    r = c.result(with_delta=True)
    return {k: (v.tolist() if isinstance(v, np.ndarray) else v) for k, v in r.items()}


def _pair(Q, n, sym, flags, seed, iters, slices):
    A, B, p0 = _inst(n, seed, sym)
    print(f"[case] static n={n} sym={sym} flags={flags} iters={iters} slices={slices}", flush=True)
    ref = Q.Chain(A, B, p0, iters, seed, 1, flags=flags, accept_cap=2048).init()
    got = Q.Chain(A, B, p0, iters, seed, 1, flags=flags, accept_cap=2048).init()
    for t_end in list(slices) + [iters]:
        ref.run(t_end)
        got.run(t_end, static=True)
    return _result(ref), _result(got)


# (n, symmetric, flags): the multi-workgroup kernel (exchange area in the
# scratch) and one-workgroup chains with byte matrices in device scratch
CASES = [((300, True, 4), (220, True, 4)),      # QAP_FLAG_MULTI_WG, larger then smaller
         ((240, False, 0), (205, False, 0)),    # asymmetric, placement 2
         ((420, True, 16), (300, True, 16))]    # QAP_FLAG_SINGLE_WG: symmetric placement 2 / 3


@pytest.mark.parametrize("first,second", CASES)
def test_static_run_matches_workspace_run(Q, first, second):
    for k, (n, sym, flags) in enumerate((first, second)):
        ref, got = _pair(Q, n, sym, flags, seed=40 + n, iters=30000, slices=(7, 12000))
        assert got["status"] == 0
        for key in ref:
            assert got[key] == ref[key], (k, n, key)


def test_static_rejects_what_it_cannot_hold(Q):
    import torch
    A, B, p0 = _inst(640, 3, False)   # asymmetric placement 3 needs about 1.6 MB of scratch
    c = Q.Chain(A, B, p0, 1000, 1, 0).init()
    with pytest.raises(Q.QapError) as e:
        c.run(10, static=True)
    assert e.value.status == Q.QAP_E_NOMEM
    assert c.state().t == 0   # nothing ran
    bufs = c.buffers()   # a workspace given to the no-allocation entry point is an error
    assert Q.qap_sa_run_static(c.n, c.A, c.B, c.Bp, c.p, c.delta, c.state_d, c.sched, c.info, bufs) == Q.QAP_E_INVAL
    assert Q.qap_static_scratch_bytes() == 1 << 20
    torch.cuda.synchronize()
