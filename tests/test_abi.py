"""CPU checks of the C ABI: the library loads, exports every function the
header declares, its structs have the layout the binding assumes, and argument
errors are reported before any device work."""
import ctypes as C
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "qapsa.h")


def _declared():
    text = open(HEADER).read()
    return re.findall(r"QAP_API\s+[\w\s\*]+?\b(qap_\w+)\s*\(", text)


@pytest.fixture(scope="module")
def qlib():
    path = os.path.join(ROOT, "paper_1208_2675_amd", "libqapsa.so")
    if not os.path.exists(path):
        from paper_1208_2675_amd import build
        build.build()
    return C.CDLL(path)


def test_header_declares_the_boundary():
    names = set(_declared())
    assert {"qap_strerror", "qap_cost", "qap_delta_init", "qap_temp_table_len", "qap_workspace_bytes",
            "qap_schedule_tables", "qap_schedule_init", "qap_sa_run", "qap_batch_workspace_bytes",
            "qap_sa_run_batch", "qap_tabu_run", "qap_sa_run_static", "qap_static_scratch_bytes"} <= names


def test_every_declared_symbol_is_exported(qlib):
    for name in _declared():
        assert hasattr(qlib, name), name


def test_struct_layout_matches_binding(tmp_path):
    from paper_1208_2675_amd import qapsa as Q
    src = tmp_path / "sz.c"
    src.write_text('#include "qapsa.h"\n#include <stdio.h>\n#include <stddef.h>\n'
                   "int main(void){printf(\"%zu %zu %zu %zu %zu %zu %zu %zu %zu %zu\\n\","
                   "sizeof(qap_instance_info), sizeof(qap_chain_state), sizeof(qap_near_tie),"
                   "sizeof(qap_schedule), sizeof(qap_run_buffers), offsetof(qap_chain_state, status),"
                   "offsetof(qap_run_buffers, workspace), sizeof(qap_chain_desc), offsetof(qap_chain_desc, T0),"
                   "sizeof(qap_batch_config));return 0;}\n")
    exe = tmp_path / "sz"
    subprocess.run(["gcc", "-D__HIP_PLATFORM_AMD__", "-I", os.path.join(ROOT, "include"),
                    "-I", "/opt/rocm/include", str(src), "-o", str(exe)], check=True)
    got = [int(x) for x in subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split()]
    assert got == [C.sizeof(Q.InstanceInfo), C.sizeof(Q.ChainState), C.sizeof(Q.NearTie),
                   C.sizeof(Q.Schedule), C.sizeof(Q.RunBuffers), Q.ChainState.status.offset,
                   Q.RunBuffers.workspace.offset, C.sizeof(Q.ChainDesc), Q.ChainDesc.T0.offset,
                   C.sizeof(Q.BatchConfig)]


def test_host_side_argument_errors(qlib):
    """These calls must fail in argument checking, before touching any device."""
    from paper_1208_2675_amd import qapsa as Q
    assert Q.qap_strerror(Q.QAP_E_RANGE).startswith("instance values")
    assert Q.qap_temp_table_len(10**9) == 2048 + 954
    assert Q.qap_temp_table_len(1) == 2049
    q = lambda n: (((n + 3) // 4) | 1) * 4
    for n in (2, 150):   # everything in LDS: the multi-workgroup area (asymmetric, 32-bit values) is the larger
        head = (64 + 2 * 1024 * 8 + 32 * (n + 1024) + 2 * 1024 * 16 * 8 + 255) // 256 * 256
        assert Q.qap_workspace_bytes(n) == head + 3 * n * 4 * n
    # n = 2000: A, A^T, B', B'^T as bytes in device scratch (asymmetric chain)
    assert Q.qap_workspace_bytes(2000) == 4 * 2000 * q(2000)
    assert Q.qap_single_workgroup(150, 0, 99, 23) == 1 and Q.qap_single_workgroup(195, 1, 99, 99) == 1
    assert Q.qap_single_workgroup(200, 0, 99, 27) == 2 and Q.qap_single_workgroup(2000, 1, 99, 141) == 2
    assert Q.qap_single_workgroup(20000, 1, 99, 99) == 0
    assert Q.qap_chain_scratch_bytes(200, 0) == 2 * 200 * 204
    assert Q.qap_chain_scratch_bytes(150, 0) == 0 and Q.qap_chain_scratch_bytes(512, 1) == 2 * 512 * q(512)
    assert Q.qap_single_workgroup(100, 1, 300, 9) == 0
    fake = 0x1000  # never dereferenced: every call below is rejected first
    assert Q.qap_sa_run(8, fake, None, fake, fake, fake, fake, Q.Schedule(100, 100, 1.0, 0.99, 1, 0, 0, 0, 0),
                        Q.InstanceInfo(0, 0, 0, 9, 0, 9, 1, 0), Q.RunBuffers(fake, None, 0, 0, None, 0), 0) == Q.QAP_E_INVAL
    info = Q.InstanceInfo(0, 0, 0, 9, 0, 9, 1, 0)
    bufs = Q.RunBuffers(fake, None, 0, 0, None, 0)
    ok = Q.Schedule(100, 100, 1.0, 0.99, 1, 0, 0, 0, 0)
    assert Q.qap_sa_run(1, fake, fake, fake, fake, fake, fake, ok, info, bufs, 0) == Q.QAP_E_INVAL
    for bad in (Q.Schedule(100, 101, 1.0, 0.99, 1, 0, 0, 0, 0), Q.Schedule(100, 100, 0.0, 0.99, 1, 0, 0, 0, 0),
                Q.Schedule(100, 100, float("nan"), 0.99, 1, 0, 0, 0, 0),
                Q.Schedule(100, 100, 1.0, 1.5, 1, 0, 0, 0, 0), Q.Schedule(0, 0, 1.0, 0.5, 1, 0, 0, 0, 0),
                Q.Schedule(100, 100, 1.0, 0.5, 1, 0, 7, 0, 0), Q.Schedule(100, 100, 1.0, 0.5, 1, 0, 3, 0, 0),
                Q.Schedule(100, 100, 1.0, 0.5, 1, 0, 32, 0, 0), Q.Schedule(100, 100, 1.0, 0.5, 1, 0, 4 | 16, 0, 0),
                Q.Schedule(100, 100, 1.0, 0.5, 1, 0, 0, 1001, 0), Q.Schedule(100, 100, 1.0, 0.5, 1, 0, 0, 0, 1)):
        assert Q.qap_sa_run(8, fake, fake, fake, fake, fake, fake, bad, info, bufs, 0) == Q.QAP_E_INVAL
    assert Q.qap_sa_run(8, fake, fake, None, fake, fake, fake, ok, info, bufs, 0) == Q.QAP_E_INVAL
    assert Q.qap_sa_run(8, fake, fake, fake, fake, fake, fake, ok, info, Q.RunBuffers(None, None, 0, 0, None, 0),
                        0) == Q.QAP_E_INVAL
    # a device-reported error in the instance facts is passed through
    bad_info = Q.InstanceInfo(0, 0, 0, 9, 0, 9, 1, Q.QAP_E_RANGE)
    assert Q.qap_sa_run(8, fake, fake, fake, fake, fake, fake, ok, bad_info, bufs, 0) == Q.QAP_E_RANGE
    # values outside the 16-bit working range have no single-workgroup kernel
    wide = Q.InstanceInfo(0, 0, 0, 70000, 0, 9, 1, 0)
    single = Q.Schedule(100, 100, 1.0, 0.5, 1, 0, Q.QAP_FLAG_SINGLE_WG, 0, 0)
    assert Q.qap_sa_run(8, fake, fake, fake, fake, fake, fake, single, wide, bufs, 0) == Q.QAP_E_UNSUPPORTED
    # batches run four waves per chain: other workgroup sizes are refused
    one = (Q.ChainDesc * 1)()
    assert Q.qap_sa_run_batch(1, one, fake, None, Q.BatchConfig(128, 0, 0, None), fake, 0) == Q.QAP_E_INVAL
    assert Q.qap_sa_run_batch(-1, one, fake, None, Q.BatchConfig(256, 0, 0, None), fake, 0) == Q.QAP_E_INVAL
    # tabu search: schedule limits, the table, and the byte-valued one-workgroup kernel only
    ts = Q.TabuSchedule(10, 10, 5, 0)
    assert Q.qap_tabu_run(8, fake, fake, fake, fake, fake, Q.TabuSchedule(10, 10, -1, 0), info, fake, bufs, 0) == Q.QAP_E_INVAL
    assert Q.qap_tabu_run(8, fake, fake, fake, fake, fake, Q.TabuSchedule(10, 11, 5, 0), info, fake, bufs, 0) == Q.QAP_E_INVAL
    assert Q.qap_tabu_run(8, fake, fake, fake, fake, fake, Q.TabuSchedule(2**31 - 5, 9, 5, 0), info, fake, bufs,
                          0) == Q.QAP_E_INVAL
    assert Q.qap_tabu_run(8, fake, fake, fake, fake, fake, ts, info, None, bufs, 0) == Q.QAP_E_INVAL
    assert Q.qap_tabu_run(8, fake, fake, fake, fake, fake, ts, wide, fake, bufs, 0) == Q.QAP_E_UNSUPPORTED
    assert Q.qap_tabu_run(8, fake, fake, fake, fake, fake, ts, bad_info, fake, bufs, 0) == Q.QAP_E_RANGE
    assert Q.qap_cost(0, fake, fake, fake, fake, 0) == Q.QAP_E_INVAL
    assert Q.qap_delta_init(1, fake, fake, fake, fake, fake, fake, None, 0) == Q.QAP_E_INVAL
    assert Q.qap_schedule_tables(0, 0.5, fake, 0) == Q.QAP_E_INVAL
    assert Q.qap_schedule_tables(10, 1.5, fake, 0) == Q.QAP_E_INVAL


@pytest.mark.parametrize("n,sym,seed,iters", [(2, False, 1, 1), (9, True, 2, 1000), (40, False, 3, 10**8),
                                              (150, False, 4, 10**9)])
def test_schedule_init_matches_the_oracle(orc, n, sym, seed, iters):
    """qap_schedule_init (host code of the library) gives the oracle's T0 and
    alpha bit for bit from the instance facts qap_delta_init reports."""
    import numpy as np
    from paper_1208_2675_amd import qapsa as Q
    rng = np.random.default_rng(seed)
    A = rng.integers(0, 50, (n, n)).astype(np.int32)
    B = rng.integers(0, 50, (n, n)).astype(np.int32)
    if sym:
        A = np.triu(A, 1); A = (A + A.T).astype(np.int32)
        B = np.triu(B, 1); B = (B + B.T).astype(np.int32)
    p = rng.permutation(n).astype(np.int32)
    ref = orc.schedule(A, B, p, iters)
    if ref["sum_abs"] == 0:
        pytest.skip("all swap costs are 0")
    info = Q.InstanceInfo(orc.cost(A, B, p), ref["sum_abs"], 0, 49, 0, 49, int(sym), 0)
    sched = Q.Schedule()
    sched.seed, sched.chain_id, sched.flags = 77, 5, 8
    assert Q.qap_schedule_init(n, info, iters, 1e-3, sched) == Q.QAP_OK
    assert sched.T0 == ref["T0"] and sched.alpha == ref["alpha"]
    assert sched.iters == iters and sched.t_end == iters
    assert (sched.seed, sched.chain_id, sched.flags) == (77, 5, 8)   # left as the caller set them
    # argument errors
    assert Q.qap_schedule_init(1, info, iters, 1e-3, sched) == Q.QAP_E_INVAL
    assert Q.qap_schedule_init(n, info, 0, 1e-3, sched) == Q.QAP_E_INVAL
    assert Q.qap_schedule_init(n, info, iters, 0.0, sched) == Q.QAP_E_INVAL
    assert Q.qap_schedule_init(n, info, iters, 1.5, sched) == Q.QAP_E_INVAL
    bad = Q.InstanceInfo(0, ref["sum_abs"], 0, 49, 0, 49, 0, Q.QAP_E_RANGE)
    assert Q.qap_schedule_init(n, bad, iters, 1e-3, sched) == Q.QAP_E_RANGE
    zero = Q.InstanceInfo(0, 0, 0, 0, 0, 0, 1, 0)
    assert Q.qap_schedule_init(n, zero, iters, 1e-3, sched) == Q.QAP_E_INVAL
