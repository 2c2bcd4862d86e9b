"""The serving form (spamm_server_*) through the C ABI.

A request solved by the server, among other requests of mixed size and
precision, runs the same kernels on the same task lists in the same order
as sp2_solve on that request alone, so the server's P and iteration history
must equal sp2_solve's bit for bit.  sp2_solve itself is held to the oracle
by test_gpu_parity.py; one case here is also checked against the oracle
directly.
"""
import time

import numpy as np
import pytest

from oracle import sp2_oracle as sp2o
from watergen import water_cluster

pytestmark = pytest.mark.gpu

# (molecules, decay, seed, precision, tau); 1 molecule = n 25 (one tier:
# the one-wave-per-block kernels), 16 molecules = n 400 (depth 4).
CASES = [
    (8, 1.5, 1, "fp32", 1e-6),
    (12, 2.0, 2, "fp64", 1e-8),
    (6, 1.2, 3, "bf16x3", 1e-5),
    (10, 1.8, 4, "fp32", 1e-5),
    (1, 1.5, 5, "fp32", 1e-6),
    (16, 1.5, 6, "fp16x3", 1e-6),
    (5, 2.5, 7, "fp64", 0.0),
    (14, 1.3, 8, "fp32", 1e-6),
    (3, 2.0, 9, "bf16", 1e-4),
]


@pytest.fixture(scope="module")
def sp():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_1403_7458_amd as lib
    lib.load()
    return lib


@pytest.fixture(scope="module")
def inputs():
    return [water_cluster(m, decay=d, seed=s) for (m, d, s, _, _) in CASES]


@pytest.fixture(scope="module")
def alone(sp, inputs):
    out = []
    for wc, (_, _, _, prec, tau) in zip(inputs, CASES):
        out.append(sp.sp2_solve(wc.f, wc.n_occ, tau, precision=prec))
    return out


def same(res, ref):
    p, st = res
    p0, st0 = ref
    assert np.array_equal(p, p0)
    for key in ("status", "iterations", "stop", "branches", "traces", "errors", "n_exec",
                "n_blocks", "eps_min", "eps_max", "trace_final", "n_exec_total"):
        assert st[key] == st0[key], key


def test_mixed_requests_match_solo_solves_bitwise(sp, inputs, alone):
    with sp.Sp2Server(8 << 30) as srv:
        ids = [srv.submit(wc.f, wc.n_occ, tau, precision=prec)
               for wc, (_, _, _, prec, tau) in zip(inputs, CASES)]
        for rid, ref in zip(ids, alone):
            same(srv.wait(rid), ref)
        info = srv.stats()
    assert info["submitted"] == info["completed"] == len(CASES)
    assert info["failed"] == 0 and info["queued"] == 0 and info["active"] == 0
    assert info["used_bytes"] == 0
    assert info["used_bytes"] + info["cached_bytes"] <= info["budget_bytes"]
    # Batched: one leaf-product launch per precision and step, so fewer
    # launches than the requests' iterations added up.
    assert info["gemm_launches"] < info["solve_iterations"]
    assert info["solve_iterations"] == sum(r[1]["iterations"] for r in alone)


def test_device_inputs_unbatched_launches_and_device_outputs(sp, inputs, alone):
    import torch
    dev = torch.device("cuda:0")
    fs = [torch.from_numpy(wc.f).to(dev) for wc in inputs]
    outs = [torch.empty_like(f) for f in fs]
    with sp.Sp2Server(8 << 30, batch_gemm=False) as srv:
        ids = [srv.submit(f, wc.n_occ, tau, precision=prec)
               for f, wc, (_, _, _, prec, tau) in zip(fs, inputs, CASES)]
        res = [srv.wait(rid, out=o) for rid, o in zip(ids, outs)]
        info = srv.stats()
    torch.cuda.synchronize()
    for (o, st), ref in zip(res, alone):
        same((o.cpu().numpy(), st), ref)
    assert info["gemm_launches"] == info["solve_iterations"]


def test_fill_limit_runs_requests_one_at_a_time(sp, inputs, alone):
    """fill_products = 1: any running request fills the device, so requests
    run one after another (one launch per SP2 iteration), same results."""
    with sp.Sp2Server(8 << 30, fill_products=1) as srv:
        ids = [srv.submit(wc.f, wc.n_occ, tau, precision=prec)
               for wc, (_, _, _, prec, tau) in zip(inputs, CASES)]
        for rid, ref in zip(ids, alone):
            same(srv.wait(rid), ref)
        info = srv.stats()
    assert info["gemm_launches"] == info["solve_iterations"] == info["steps"]


def test_small_budget_queues_requests_and_stays_within_it(sp, inputs, alone):
    """A budget a little above the largest request admits one request at a
    time (plus nothing else while its result is held), in FIFO order."""
    need = max(sp.sp2_footprint_bytes(wc.n, prec) for wc, (_, _, _, prec, _) in zip(inputs, CASES))
    budget = int(need * 1.05)
    with sp.Sp2Server(budget) as srv:
        ids = [srv.submit(wc.f, wc.n_occ, tau, precision=prec)
               for wc, (_, _, _, prec, tau) in zip(inputs, CASES)]
        got = {}
        deadline = time.time() + 120
        while len(got) < len(ids):
            assert time.time() < deadline, "server made no progress"
            for rid in ids:
                if rid in got:
                    continue
                r = srv.poll(rid)
                if r is not None:
                    got[rid] = r
            time.sleep(0.001)
        info = srv.stats()
    for rid, ref in zip(ids, alone):
        same(got[rid], ref)
    assert info["peak_used_bytes"] <= budget
    assert info["completed"] == len(CASES)


def test_server_result_against_oracle(sp):
    wc = water_cluster(6, decay=1.5, seed=21)
    ref = sp2o.sp2(wc.f, wc.n_occ, 1e-7, tol=1e-8)
    with sp.Sp2Server(1 << 30) as srv:
        p, st = srv.wait(srv.submit(wc.f, wc.n_occ, 1e-7, precision="fp64"))
    assert st["iterations"] == ref.iterations
    assert st["branches"] == ref.branches
    np.testing.assert_allclose(p, ref.p, rtol=0, atol=1e-10)


def test_request_errors(sp, inputs):
    wc = inputs[0]
    bad = wc.f.copy()
    bad[0, 1] += 1.0  # not symmetric: found when the request starts
    with sp.Sp2Server(1 << 30) as srv:
        with pytest.raises(sp.SpammError) as e:
            srv.submit(wc.f, wc.n + 1, 1e-6)           # n_occ > n: at submit
        assert e.value.code == -1
        with pytest.raises(sp.SpammError) as e:
            srv.submit(wc.f, wc.n_occ, -1.0)           # tau < 0
        assert e.value.code == -1
        r_bad = srv.submit(bad, wc.n_occ, 1e-6)
        r_ok = srv.submit(wc.f, wc.n_occ, 1e-6)
        with pytest.raises(sp.SpammError) as e:
            srv.wait(r_bad)
        assert e.value.code == -3
        p, st = srv.wait(r_ok)
        assert st["status"] in (0, 1) and np.isfinite(p).all()
        with pytest.raises(sp.SpammError) as e:
            srv.wait(r_ok)                             # already collected
        assert e.value.code == -1
        info = srv.stats()
        assert info["failed"] == 1 and info["completed"] == 2
    with sp.Sp2Server(1 << 20) as srv:                 # 1 MiB: too small for anything
        with pytest.raises(sp.SpammError) as e:
            srv.submit(wc.f, wc.n_occ, 1e-6)
        assert e.value.code == -4


def test_destroy_with_requests_in_flight(sp, inputs):
    srv = sp.Sp2Server(8 << 30)
    for wc, (_, _, _, prec, tau) in zip(inputs, CASES):
        srv.submit(wc.f, wc.n_occ, tau, precision=prec)
    srv.close()  # stops after the current step; nothing left behind
    # The library still works afterwards.
    wc = inputs[0]
    p, st = sp.sp2_solve(wc.f, wc.n_occ, 1e-6)
    assert np.isfinite(p).all()
