"""Batches of problems and the request server, through the C ABI.

Every problem's homogenization inside a batch or the server runs the same
launches as qp_homogenized on that problem alone, on its own stream, so the
results must be bitwise equal to the standalone ones (also for a request
served alone versus in a mix of other requests).  Standalone results are
themselves checked against the oracle by the parity tests; here a few small
instances are also compared with the oracle directly.
"""
from __future__ import annotations

import sys
import time

import numpy as np
import pytest

import oracle
from paper_2404_06841_amd import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover - CPU container
    pytest.skip("no GPU", allow_module_level=True)

from paper_2404_06841_amd import qp  # noqa: E402


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def mixed_problems():
    return [W.eightfold_random(8, 1), W.eightfold_random(12, 2), W.eightfold_random(16, 3),
            W.eightfold_random(24, 4), W.icosahedral(6), W.eightfold_diagonal(10, 0),
            W.periodic_2d_diagonal(40)]


@pytest.mark.parametrize("prec", ["fp64", "fp32ir"])
def test_batch_equals_standalone(prec):
    probs = mixed_problems()
    alone = []
    for pr in probs:
        gp = qp.Problem(pr, precision=prec)
        r = gp.homogenized(tol=1e-12, energy=False)
        alone.append((r.A.copy(), [i.iters for i in r.infos]))
        gp.close()
    streams = [torch.cuda.Stream() for _ in probs]
    gps = [qp.Problem(pr, precision=prec, stream=s) for pr, s in zip(probs, streams)]
    t = time.perf_counter()
    As, infos, st = qp.homogenized_batch(gps, tol=1e-12)
    say("batch", prec, len(probs), "problems", round((time.perf_counter() - t) * 1e3, 2), "ms")
    assert st == qp.QP_OK
    for pr, (A0, it0), A, inf in zip(probs, alone, As, infos):
        assert np.array_equal(A, A0), (pr.name, pr.N, A, A0)
        assert [i.iters for i in inf] == it0
    for gp in gps:
        gp.close()


def test_batch_small_instances_match_oracle():
    probs = [W.eightfold_random(8, 5), W.eightfold_random(12, 6), W.laminate(8)]
    gps = [qp.Problem(pr, precision="fp32ir", stream=torch.cuda.Stream()) for pr in probs]
    As, _, st = qp.homogenized_batch(gps, tol=1e-12)
    assert st == qp.QP_OK
    for pr, A in zip(probs, As):
        ref = oracle.homogenize(pr, tol=1e-12)
        assert np.abs(A - ref.A).max() <= 1e-10 * np.abs(ref.A).max(), pr.name
    for gp in gps:
        gp.close()


def test_batch_rejects_repeated_problem():
    gp = qp.Problem(W.eightfold(6))
    with pytest.raises(qp.QPError):
        qp.homogenized_batch([gp, gp], tol=1e-12)
    gp.close()


def _alone(pr, prec):
    gp = qp.Problem(pr, precision=prec)
    r = gp.homogenized(tol=1e-12, energy=False)
    gp.close()
    return r.A.copy()


def _drain(srv, tickets, limit_s=120.0):
    left = set(tickets)
    t0 = time.perf_counter()
    while left:
        for t in srv.progress(wait_us=2000):
            left.discard(t)
        assert time.perf_counter() - t0 < limit_s, "server did not finish"


@pytest.mark.parametrize("prec", ["fp64", "fp32ir"])
def test_server_alone_equals_mix(prec):
    probs = mixed_problems()
    target = probs[2]
    srv = qp.Server(64 << 30, precision=prec)
    t = srv.submit(target, tol=1e-12)
    _drain(srv, [t])
    A_alone, _, st = srv.result(t)
    assert st == qp.QP_OK
    assert np.array_equal(A_alone, _alone(target, prec))
    srv.close()
    # the same request in a mix (other problems, and the same problem twice)
    srv = qp.Server(64 << 30, precision=prec)
    tickets = [srv.submit(pr, tol=1e-12) for pr in probs] + [srv.submit(target, tol=1e-12)]
    _drain(srv, tickets)
    for pr, tk in zip(probs + [target], tickets):
        A, infos, st = srv.result(tk)
        assert st == qp.QP_OK, (pr.name, st)
        assert np.array_equal(A, _alone(pr, prec)), (pr.name, pr.N)
    assert np.array_equal(srv.result(tickets[2])[0], A_alone)
    assert np.array_equal(srv.result(tickets[-1])[0], A_alone)
    srv.close()


def test_server_budget_evicts_idle_problems():
    probs = [W.eightfold_random(16, 7), W.eightfold_random(16, 8), W.eightfold_random(16, 9)]
    need = qp.qp_workspace_bytes(2, 4, 16, probs[0].g)
    srv = qp.Server(need + need // 2)  # room for one problem at a time
    tickets = [srv.submit(pr, tol=1e-12) for pr in probs]
    left = set(tickets)
    t0 = time.perf_counter()
    while left:
        for t in srv.progress(wait_us=2000):
            left.discard(t)
        assert srv.bytes() <= need + need // 2
        assert time.perf_counter() - t0 < 120
    for pr, tk in zip(probs, tickets):
        A, _, st = srv.result(tk)
        assert st == qp.QP_OK and np.array_equal(A, _alone(pr, "fp64"))
    srv.close()


def test_server_request_errors():
    srv = qp.Server(8 << 30)
    bad = W.eightfold(8, amplitude=1.0)  # literal amplitude: negative somewhere on the grid
    tb = srv.submit(bad, tol=1e-12)
    good = W.eightfold_random(8, 3)
    tg = srv.submit(good, tol=1e-12)
    _drain(srv, [tb, tg])
    assert srv.result(tb)[2] == qp.QP_ENOTELLIPTIC
    assert srv.result(tg)[2] == qp.QP_OK
    huge = W.icosahedral(40)  # 40^6 unknowns: far beyond the budget
    with pytest.raises(qp.QPError):
        srv.submit(huge, tol=1e-12)
    srv.close()
