"""Grouped homogenization (one launch per solver step for a whole batch),
through the C ABI.

Each workgroup of a grouped launch computes what the same workgroup of its
problem's own launch computes, and a paused right-hand side is frozen until
its replacement, so the grouped A* and iteration counts must equal the
standalone ones bitwise, whatever the mix of sizes.  A few small groups are
also compared with the oracle directly.
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


def standalone(probs, **kw):
    out = []
    for pr in probs:
        gp = qp.Problem(pr, precision="fp32ir", **kw)
        r = gp.homogenized(tol=1e-12, energy=False, check=False)
        out.append((r.A.copy(), [i.iters for i in r.infos], [i.status for i in r.infos],
                    [i.outer_iters for i in r.infos]))
        gp.close()
    return out


def _many_modes(N: int):
    # 31 seeded +-mode pairs and the mean (g = 63: 64 padded mode records)
    rng = np.random.default_rng(2404)
    modes, coef, amps = W.random_modes(4, 31, 2, rng, 0.05, 2.5, 3.0)
    return W.Problem("eightfold_many_modes", 2, 4, int(N), W.eightfold_P(), modes, coef,
                     {"amplitudes": amps.tolist()})


GROUPS = {
    # d = 2, real coefficients, sizes from 125 to 331,776 unknowns (grids
    # below 8 workgroups, odd N, several workgroup counts)
    "eightfold_mixed": lambda: [W.eightfold_random(8, 1), W.eightfold_random(12, 2),
                                W.eightfold_random(16, 3), W.eightfold_random(24, 4),
                                W.eightfold_random(5, 5), W.eightfold(6), W.eightfold(10)],
    # d = 3, real coefficients, n = 3 and n = 6
    "d3_mixed": lambda: [W.icosahedral(6), W.periodic_cubic(3, 7), W.icosahedral(8),
                         W.periodic_cubic(3, 12)],
    # d = 2, complex coefficients
    "complex": lambda: [W.paper_four_mode_2d(6), W.paper_four_mode_2d(9)],
    # the largest batch size (N = 32: 1,048,576 unknowns, chunks above 1024
    # entries, so the vector steps load eight rows per thread) beside small ones
    "eightfold_N32_mixed": lambda: [W.eightfold_random(32, 0), W.eightfold_random(8, 1),
                                    W.eightfold_random(24, 2)],
    # 63 coefficient modes beside 17 (the grouped product's records at 64)
    "many_modes_mixed": lambda: [_many_modes(12), W.eightfold_random(8, 1), _many_modes(6)],
}
# groups whose problems are also created with the layout autotuner (as the
# batch benchmark does): the grouped launches must use each problem's tuned
# layouts and partial counts
AUTOTUNED = {"eightfold_N32_mixed"}
CASES = sorted(GROUPS) + [n + "+autotune" for n in sorted(AUTOTUNED)]


@pytest.mark.parametrize("case", CASES)
def test_grouped_equals_standalone(case):
    name = case.split("+")[0]
    kw = {"autotune": True} if case.endswith("+autotune") else {}
    probs = GROUPS[name]()
    say("[case] grouped", case, [(pr.name, pr.N) for pr in probs])
    alone = standalone(probs, **kw)
    gps = [qp.Problem(pr, precision="fp32ir", stream=torch.cuda.Stream(), **kw) for pr in probs]
    t = time.perf_counter()
    As, infos, st = qp.homogenized_batch(gps, tol=1e-12, grouped=True)
    say("  grouped", len(probs), "problems", round((time.perf_counter() - t) * 1e3, 2), "ms")
    assert st == qp.QP_OK
    for pr, (A0, it0, st0, out0), A, inf in zip(probs, alone, As, infos):
        assert all(s == 0 for s in st0)
        assert np.array_equal(A, A0), (pr.name, pr.N, A, A0)
        assert [i.iters for i in inf] == it0, (pr.name, pr.N)
        assert [i.outer_iters for i in inf] == out0, (pr.name, pr.N)
        assert all(i.status == 0 and i.rel_resid <= 1e-12 for i in inf)
    # a second call on the same problems repeats the result
    As2, _, st2 = qp.homogenized_batch(gps, tol=1e-12, grouped=True)
    assert st2 == qp.QP_OK and all(np.array_equal(a, b) for a, b in zip(As, As2))
    for gp in gps:
        gp.close()


def test_grouped_small_instances_match_oracle():
    probs = [W.eightfold_random(8, 5), W.eightfold_random(12, 6), W.eightfold(10)]
    gps = [qp.Problem(pr, precision="fp32ir") for pr in probs]
    As, _, st = qp.homogenized_batch(gps, tol=1e-12, grouped=True)
    assert st == qp.QP_OK
    for pr, A in zip(probs, As):
        ref = oracle.homogenize(pr, tol=1e-12)
        assert np.abs(A - ref.A).max() <= 1e-10 * np.abs(ref.A).max(), pr.name
    for gp in gps:
        gp.close()


def test_grouped_iteration_limit_matches_standalone():
    probs = [W.eightfold_random(12, 2), W.eightfold_random(16, 3)]
    alone = standalone(probs, maxit=6)
    gps = [qp.Problem(pr, precision="fp32ir", maxit=6) for pr in probs]
    As, infos, st = qp.homogenized_batch(gps, tol=1e-12, grouped=True, check=False)
    assert st == qp.QP_ENOCONV
    for (A0, it0, st0, _), A, inf in zip(alone, As, infos):
        assert st0 == [qp.QP_ENOCONV] * 2
        assert [i.status for i in inf] == st0
        assert [i.iters for i in inf] == it0
        assert np.array_equal(A, A0)
    for gp in gps:
        gp.close()


def test_grouped_rejects_what_cannot_join():
    a = qp.Problem(W.eightfold(6), precision="fp32ir")
    cases = [
        [a, a],                                                       # repeated
        [a, qp.Problem(W.eightfold(8))],                              # FP64
        [a, qp.Problem(W.icosahedral(6), precision="fp32ir")],        # d = 3 beside d = 2
        [a, qp.Problem(W.eightfold_diagonal(8, 0), precision="fp32ir")],  # diagonal
        [a, qp.Problem(W.periodic_1d(40), precision="fp32ir")],       # d = 1, line tiles
        [a, qp.Problem(W.paper_four_mode_2d(6), precision="fp32ir")],  # complex beside real
        [a, qp.Problem(W.eightfold(8), precision="fp32ir", maxit=50)],  # other maxit
    ]
    for grp in cases:
        with pytest.raises(qp.QPError) as e:
            qp.homogenized_batch(grp, tol=1e-12, grouped=True)
        assert e.value.status == qp.QP_EINVAL
    a.close()


def test_mixed_batch_equals_standalone():
    """qp_homogenized_batch_mixed: the small FP32-IR d = 2 real problems
    (at most 12^4 unknowns) form the group; the larger ones and those that
    cannot join it (FP64, d = 3, complex coefficient) run on their own
    streams; every result equals the standalone one bitwise."""
    spec = [(W.eightfold_random(32, 0), "fp32ir"), (W.eightfold_random(8, 1), "fp32ir"),
            (W.icosahedral(6), "fp32ir"), (W.eightfold(8), "fp64"),
            (W.eightfold_random(12, 2), "fp32ir"), (W.eightfold_random(24, 4), "fp32ir"),
            (W.eightfold(10), "fp32ir"), (W.paper_four_mode_2d(6), "fp32ir")]
    say("[case] mixed batch", [(pr.name, pr.N, prec) for pr, prec in spec])
    alone = []
    for pr, prec in spec:
        gp = qp.Problem(pr, precision=prec)
        r = gp.homogenized(tol=1e-12, energy=False)
        alone.append((r.A.copy(), [i.iters for i in r.infos], [i.outer_iters for i in r.infos]))
        gp.close()
    gps = [qp.Problem(pr, precision=prec, stream=torch.cuda.Stream()) for pr, prec in spec]
    for limit in (12 ** 4, 0):
        t = time.perf_counter()
        As, infos, st = qp.homogenized_batch(gps, tol=1e-12, group_max_dim=limit)
        say("  mixed, limit", limit, round((time.perf_counter() - t) * 1e3, 2), "ms")
        assert st == qp.QP_OK
        for (pr, _), (A0, it0, out0), A, inf in zip(spec, alone, As, infos):
            assert np.array_equal(A, A0), (pr.name, pr.N, limit)
            assert [i.iters for i in inf] == it0, (pr.name, pr.N, limit)
            assert [i.outer_iters for i in inf] == out0, (pr.name, pr.N, limit)
            assert all(i.status == 0 and i.rel_resid <= 1e-12 for i in inf)
    for gp in gps:
        gp.close()


def test_mixed_batch_reports_the_first_failure_in_problem_order():
    # the grouped problems stop at their iteration limit; the large one converges
    small = [qp.Problem(W.eightfold_random(8, 1), precision="fp32ir", maxit=6,
                        stream=torch.cuda.Stream()),
             qp.Problem(W.eightfold_random(12, 2), precision="fp32ir", maxit=6,
                        stream=torch.cuda.Stream())]
    big = qp.Problem(W.eightfold_random(24, 4), precision="fp32ir", stream=torch.cuda.Stream())
    As, infos, st = qp.homogenized_batch([big] + small, tol=1e-12, group_max_dim=12 ** 4,
                                         check=False)
    assert st == qp.QP_ENOCONV
    assert all(i.status == 0 for i in infos[0])
    assert all(i.status == qp.QP_ENOCONV for inf in infos[1:] for i in inf)
    for gp in small + [big]:
        gp.close()
