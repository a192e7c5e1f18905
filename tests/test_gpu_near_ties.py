"""Near ties of Eq. (2) on every kernel: ties built with the oracle
(tests/tie_cases.py) at the first proposal and in mid-run, run through the
one-workgroup kernel in scratch mode and in Delta mode, the 16-bit kernel, the
multi-workgroup kernel and a batch.  Each path must log the same iterations
as the oracle and make the same decisions (the constructed z is +-1e-13, far
from 0 compared with a last-bit difference of log), so the whole trajectory
stays bit-exact.  The exact tie (z within a few ulp of 0) is checked for being
logged on both sides and decided by the sign of each side's own z."""
import math
import os
import sys

import numpy as np
import pytest

sys.path.insert(0, os.path.dirname(__file__))
import tie_cases as TC  # noqa: E402
from paper_1208_2675_amd import workloads as W  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def Q():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1208_2675_amd import qapsa
    return qapsa


def _inst(n, seed, sym, lo, hi):
    rng = np.random.default_rng(seed)
    A = rng.integers(lo, hi + 1, (n, n)).astype(np.int32)
    B = rng.integers(lo, hi + 1, (n, n)).astype(np.int32)
    if sym:
        A = np.triu(A, 1); A = (A + A.T).astype(np.int32)
        B = np.triu(B, 1); B = (B + B.T).astype(np.int32)
    return A, B, rng.permutation(n).astype(np.int32)


# path name -> (instance symmetric, value range, chain flags)
PATHS = {
    "wg_scratch": (False, (0, 60), 2),      # QAP_FLAG_SCRATCH_ONLY
    "wg_delta": (False, (0, 60), 1),        # QAP_FLAG_DELTA_ONLY
    "wg_scratch_sym": (True, (0, 60), 2),
    "lds16": (False, (0, 600), 0),          # value range above a byte: 16-bit kernel
    "dist": (True, (0, 60), 4),             # QAP_FLAG_MULTI_WG
    "batch": (False, (0, 60), 0),
}


def _first_tie_case(orc, sym, lohi, eps, n=24):
    for k in range(1, 200):
        A, B, p0 = _inst(n, 100 + k, sym, *lohi)
        T0 = TC.tie_T0(orc, A, B, p0, 3, 0, 0, eps, 400)
        if T0 is not None:
            return A, B, p0, 3, T0
    raise AssertionError("no instance with a positive first swap cost")


def _mid_tie_case(orc, sym, lohi, n=24, iters=4000):
    A, B, p0 = TC.identical_pair_instance(n, 5, sym, *lohi)
    T_start = orc.schedule(A, B, p0, iters)["T0"] / 30
    for seed in range(1, 80):
        cands = [t for t in range(600, 1500) if not {0, 1} & set(TC.pair_at(n, t))
                 and math.log(orc.uniform(seed, 0, t)) < -5]
        found = TC.find_tie(orc, A, B, p0, iters, -1e-13, cands[:5], [seed], T_start=T_start)
        if found:
            seed, t_star, T0 = found
            return A, B, p0, seed, T0, t_star
    raise AssertionError("no mid-run tie found")


def _run_path(Q, path, A, B, p0, iters, seed, T0, t_end=None, tie_cap=64, acc_cap=0):
    """Run one chain on the named path; returns the result dict of the chain."""
    sym, _, flags = PATHS[path]
    if path == "batch":
        ch = W.Chain("tie", A, B, p0, iters, seed, 0, sym)
        b = Q.Batch([ch], tie_cap=tie_cap).init(ratio=1.0, T0=T0)
        if t_end is not None:
            b.descs[0].t_end = t_end
            b.descs_d.copy_(__import__("torch").from_numpy(np.frombuffer(bytes(b.descs), dtype=np.uint8).copy()))
        b.run()
        st = b.states()[0]
        raw = b.ties[0].cpu().numpy().tobytes()
        ties = np.frombuffer(raw, dtype=np.dtype([("t", "<u8"), ("delta", "<i8"), ("z", "<f8")]))
        ties = ties[: min(st["near_ties"], tie_cap)]
        o = np.argsort(ties["t"], kind="stable")
        st.update(p=b.perm(0), near_tie_t=ties["t"][o], near_tie_z=ties["z"][o])
        return st
    c = Q.Chain(A, B, p0, iters, seed, 0, ratio=1.0, T0=T0, tie_cap=tie_cap, accept_cap=acc_cap,
                flags=flags).init()
    c.run(t_end)
    return c.result()


def _check_same(got, ref):
    for k in ("t", "accepts", "hash", "cost", "best_cost", "best_iter", "near_ties"):
        assert got[k] == ref[k], (k, got[k], ref[k])
    assert np.array_equal(got["p"], ref["p"])
    assert got["near_tie_t"].tolist() == sorted(int(x) for x in ref["near_tie_t"])


@pytest.mark.parametrize("path", list(PATHS))
@pytest.mark.parametrize("eps", [-1e-13, 1e-13])
def test_tie_at_first_proposal(orc, Q, path, eps):
    sym, lohi, _ = PATHS[path]
    A, B, p0, seed, T0 = _first_tie_case(orc, sym, lohi, eps)
    iters = 400
    print(f"[case] path={path} eps={eps} n={A.shape[0]} T0={T0!r} seed={seed}", flush=True)
    ref = orc.sa_run(A, B, p0, iters, T0, 1.0, seed, 0, tie_cap=64)
    assert 0 in ref["near_tie_t"].tolist()
    got = _run_path(Q, path, A, B, p0, iters, seed, T0)
    _check_same(got, ref)
    z = dict(zip(got["near_tie_t"].tolist(), got["near_tie_z"].tolist()))[0]
    assert abs(z - eps) < 1e-14 and (z < 0) == (eps < 0)


@pytest.mark.parametrize("path", list(PATHS))
def test_tie_in_mid_run(orc, Q, path):
    sym, lohi, _ = PATHS[path]
    A, B, p0, seed, T0, t_star = _mid_tie_case(orc, sym, lohi)
    iters = 4000
    print(f"[case] path={path} mid-run tie t*={t_star} n={A.shape[0]} T0={T0!r} seed={seed}", flush=True)
    ref = orc.sa_run(A, B, p0, iters, T0, 1.0, seed, 0, tie_cap=64)
    assert ref["near_tie_t"].tolist() == [t_star]
    got = _run_path(Q, path, A, B, p0, iters, seed, T0)
    _check_same(got, ref)


@pytest.mark.parametrize("path", list(PATHS))
def test_exact_tie_logged_on_both_sides(orc, Q, path):
    """z = 0 up to the last bits: host and device log may round differently,
    so only one iteration is compared: both log the tie at t = 0, their z
    agree to a few ulp of |log r|, and each decides by the sign of its own z."""
    sym, lohi, _ = PATHS[path]
    A, B, p0, seed, T0 = _first_tie_case(orc, sym, lohi, 0.0)
    y = math.log(orc.uniform(seed, 0, 0))
    print(f"[case] path={path} exact tie n={A.shape[0]} T0={T0!r}", flush=True)
    ref = orc.sa_run(A, B, p0, 400, T0, 1.0, seed, 0, t_end=1, tie_cap=8)
    got = _run_path(Q, path, A, B, p0, 400, seed, T0, t_end=1, tie_cap=8)
    assert ref["near_ties"] == 1 and got["near_ties"] == 1
    assert got["near_tie_t"].tolist() == [0]
    z_ref, z_got = float(ref["near_tie_z"][0]), float(got["near_tie_z"][0])
    assert abs(z_got - z_ref) <= 4 * math.ulp(abs(y))
    assert ref["accepts"] == (1 if z_ref < 0 else 0)
    assert got["accepts"] == (1 if z_got < 0 else 0)
    print(f"[exact tie] path={path} z_host={z_ref!r} z_device={z_got!r} same={z_ref == z_got}", flush=True)
