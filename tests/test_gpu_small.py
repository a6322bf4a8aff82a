"""FP64 solves of small problems in one launch (qp_options.small_dim): one
workgroup per right-hand side runs the whole C-PCG loop (Alg. 2).

The one-launch loop takes the same recurrences as the three-launch
iteration, with its sums formed in another order, so the two agree to
rounding: the same statuses, iteration counts within one, solutions and A*
to the tolerance.  Both are also held against the oracle (the oracle parity
tests of test_gpu_parity.py run every FP64 problem of at most 2048 unknowns
through this path by default).
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


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to(device="cuda", dtype=torch.complex128)


CASES = {
    "c1_1d_n2_N32": lambda: W.one_d_two_mode(32, 2.0),          # d = 1, degenerate field
    "random_N6": lambda: W.eightfold_random(6, 1),              # d = 2, 1296 unknowns
    "icosa_N3": lambda: W.icosahedral(3),                        # d = 3, n = 6, odd N
    "paper2d_N6_complex": lambda: W.paper_four_mode_2d(6),      # complex coefficient
    "periodic_cubic_d4_N6": lambda: W.periodic_cubic(4, 6),     # d = 4
}


@pytest.mark.parametrize("name", sorted(CASES))
def test_one_launch_matches_three_launch_loop_and_oracle(name):
    prob = CASES[name]()
    say(f"[case] one launch {name} D={prob.D}")
    one = qp.Problem(prob)            # default small_dim covers it
    many = qp.Problem(prob, small_dim=0)
    assert prob.D <= qp.qp_default_options().small_dim
    r1 = one.homogenized(tol=1e-12)
    rm = many.homogenized(tol=1e-12)
    ref = oracle.homogenize(prob, tol=1e-12)
    scale = max(np.abs(ref.A).max(), 1.0)
    for r in (r1, rm):
        assert all(i.status == qp.QP_OK and i.rel_resid <= 1e-12 for i in r.infos)
        assert np.abs(r.A - ref.A).max() <= 1e-10 * scale, (name, r.A, ref.A)
    for a, b in zip(r1.infos, rm.infos):
        assert abs(a.iters - b.iters) <= max(1, int(0.02 * b.iters)), (name, a.iters, b.iters)
        assert abs(a.kappa_est - b.kappa_est) <= 1e-3 * b.kappa_est, (name, a.kappa_est,
                                                                      b.kappa_est)
        assert a.bytes_moved == b.bytes_moved or a.iters != b.iters
    # a user right-hand side, against the oracle's PCG solution
    F = W.random_vector(prob.D, seed=31)
    U, info = one.solve_d(dev(F), tol=1e-12)
    Ur, st, it, rr = oracle.pcg(prob, F, tol=1e-12)
    U = U.cpu().numpy()
    assert info.status == 0 and info.rel_resid <= 1e-12 and U[0] == 0
    if name != "c1_1d_n2_N32":  # the degenerate field: see test_gpu_parity.py
        assert abs(info.iters - it) <= 2
        assert np.linalg.norm(U - Ur) <= 1e-9 * np.linalg.norm(Ur)
    one.close()
    many.close()


def test_one_launch_limits_and_breakdown():
    prob = W.eightfold_random(6, 1)
    # iteration limit: QP_ENOCONV after exactly maxit updates on both paths
    for sd in (2048, 0):
        gp = qp.Problem(prob, maxit=5, small_dim=sd)
        r = gp.homogenized(tol=1e-12, check=False)
        assert [i.status for i in r.infos] == [qp.QP_ENOCONV] * 2
        assert [i.iters for i in r.infos] == [5, 5]
        gp.close()
    # indefinite coefficient: the same breakdown step as the three-launch loop
    bad = W.eightfold(6, amplitude=1.0)
    res = []
    for sd in (2048, 0):
        gp = qp.Problem(bad, allow_indefinite=True, small_dim=sd)
        F = W.random_vector(bad.D, seed=3)
        _, info = gp.solve_d(dev(F), tol=1e-12, check=False)
        res.append((info.status, info.iters))
        gp.close()
    say("  breakdown one launch / three launches:", res)
    assert res[0][0] == res[1][0]
    if res[1][0] == qp.QP_ENOTSPD:
        assert abs(res[0][1] - res[1][1]) <= 1
    # a zero right-hand side finishes at the start
    gp = qp.Problem(prob)
    U, info = gp.solve_d(torch.zeros(prob.D, dtype=torch.complex128, device="cuda"), tol=1e-12)
    assert info.status == 0 and info.iters == 0 and not bool(U.abs().any())
    gp.close()


def test_one_launch_batch_equals_standalone():
    probs = [W.eightfold_random(6, i) for i in range(4)] + [W.icosahedral(3), W.eightfold(6)]
    alone = []
    for pr in probs:
        gp = qp.Problem(pr)
        alone.append(gp.homogenized(tol=1e-12, energy=False).A.copy())
        gp.close()
    gps = [qp.Problem(pr, stream=torch.cuda.Stream()) for pr in probs]
    As, infos, st = qp.homogenized_batch(gps, tol=1e-12)
    assert st == qp.QP_OK
    assert all(np.array_equal(a, b) for a, b in zip(As, alone))
    for gp in gps:
        gp.close()


def test_one_launch_is_faster_on_the_degenerate_field():
    prob = W.one_d_two_mode(32, 2.0)
    rates = {}
    for sd in (2048, 0):
        gp = qp.Problem(prob, small_dim=sd)
        gp.homogenized(tol=1e-12, energy=False)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(20):
            gp.homogenized(tol=1e-12, energy=False)
        rates[sd] = 20 / (time.perf_counter() - t0)
        gp.close()
    say("  C1 homogenizations/s, one launch / three launches per iteration:",
        round(rates[2048], 1), round(rates[0], 1))
    assert rates[2048] > rates[0]
