"""qp_homogenized_grouped_noalloc through the C ABI: the grouped homogenization
whose group table lives in the library's static device array.  Its results
must equal qp_homogenized_grouped's on the same problems bitwise (the same
launches), on two calls in a row, the second with fewer and smaller problems
(the array keeps the first call's contents), and meet the oracle's A*."""
from __future__ import annotations

import sys

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


def run_both(probs):
    gps = [qp.Problem(pr, precision="fp32ir", stream=torch.cuda.Stream()) for pr in probs]
    A0, I0, s0 = qp.homogenized_batch(gps, tol=1e-12, grouped=True)
    A1, I1, s1 = qp.homogenized_batch(gps, tol=1e-12, grouped=True, noalloc=True)
    for gp in gps:
        gp.close()
    return (A0, I0, s0), (A1, I1, s1)


def check_equal(probs, ref, got):
    (A0, I0, s0), (A1, I1, s1) = ref, got
    assert s0 == s1 == qp.QP_OK
    for pr, a0, a1, i0, i1 in zip(probs, A0, A1, I0, I1):
        assert np.array_equal(a0, a1), (pr.name, pr.N, a0, a1)
        assert [x.iters for x in i0] == [x.iters for x in i1], (pr.name, pr.N)
        assert [x.outer_iters for x in i0] == [x.outer_iters for x in i1], (pr.name, pr.N)
        assert [x.status for x in i1] == [0] * pr.d
        assert [x.kappa_est for x in i0] == [x.kappa_est for x in i1]


def test_noalloc_equals_grouped_on_two_calls():
    first = [W.eightfold_random(32, 0), W.eightfold_random(8, 1), W.eightfold_random(24, 2),
             W.eightfold(10)]
    say("[case] noalloc call 1", [(p.name, p.N) for p in first])
    ref, got = run_both(first)
    check_equal(first, ref, got)
    # the second call: fewer and smaller problems
    second = [W.eightfold_random(8, 5), W.eightfold(6)]
    say("[case] noalloc call 2", [(p.name, p.N) for p in second])
    ref2, got2 = run_both(second)
    check_equal(second, ref2, got2)
    for pr, A in zip(second, got2[0]):
        oref = oracle.homogenize(pr, tol=1e-12)
        assert np.abs(A - oref.A).max() <= 1e-10 * np.abs(oref.A).max(), pr.name


def test_noalloc_three_dimensional_group():
    probs = [W.icosahedral(8), W.icosahedral(6), W.periodic_cubic(3, 7)]
    say("[case] noalloc d=3", [(p.name, p.N) for p in probs])
    ref, got = run_both(probs)
    check_equal(probs, ref, got)


def test_noalloc_rejects_more_problems_than_its_limit():
    hs = (qp.C.c_void_p * 4097)()
    A = np.zeros(4 * 4097)
    st = qp.lib().qp_homogenized_grouped_noalloc(hs, 4097, A.ctypes.data_as(qp.C.POINTER(qp.C.c_double)),
                                                1e-12, None)
    assert st == qp.QP_EINVAL and "group limit" in qp.qp_last_error()
