"""Diagonal coefficient A = diag(a_1..a_d) (App. D) on the GPU, through the C ABI.

Parity with the oracle (same seeded inputs, same tolerances as the scalar
coefficient: FP64 products 1e-13, FP32 products 2e-5, A* 1e-10 relative) on
plane tiles (n = 4, N <= 32; real and complex Fourier coefficients), line
tiles (n = 2, N = 40, and n = 4, N = 34) and the 64-bit gathers; plus the
closed forms the oracle tests pin: A*_22 = 7 and A*_12 = A*_21 = 0 for the
paper's example, the grid harmonic mean for a laminate.
"""
from __future__ import annotations

import sys

import numpy as np
import pytest

import oracle
from paper_2404_06841_amd import workloads as W
from tests import independent as ind

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover - CPU container
    pytest.skip("no GPU", allow_module_level=True)

from paper_2404_06841_amd import qp  # noqa: E402


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def dev(x: np.ndarray, dtype=torch.complex128):
    return torch.from_numpy(np.ascontiguousarray(x)).to(device="cuda", dtype=dtype)


def host(t) -> np.ndarray:
    return t.detach().cpu().numpy()


def _many_modes_diag(N: int):
    # both diagonal entries on the same 31 seeded +-mode pairs and the mean
    # (g = 63: 64 padded records), with their own amplitudes and means
    rng = np.random.default_rng(2405)
    modes, coef, _ = W.random_modes(4, 31, 2, rng, 0.05, 2.5, 3.0)
    coef2 = coef * 0.8
    coef2[np.all(modes == 0, axis=1)] = 4.0
    return W.diagonal("eightfold_diag_many_modes", 2, 4, int(N), W.eightfold_P(),
                      [(modes, coef), (modes, coef2)])


CASES = {
    "many_modes_g63_N12": lambda: _many_modes_diag(12),
    "paper_example_N6": lambda: W.paper_homogenization(6),
    "paper_example_N18": lambda: W.paper_homogenization(18),
    "laminate_N8": lambda: W.laminate(8),
    "eightfold_diag_N12": lambda: W.eightfold_diagonal(12, 0),
    "eightfold_diag_complex_N10": lambda: W.eightfold_diagonal(10, 1, complex_phase=True),
    "eightfold_diag_N5_odd": lambda: W.eightfold_diagonal(5, 2),
    "periodic_2d_N40_lines": lambda: W.periodic_2d_diagonal(40),
}


@pytest.fixture(scope="module", params=sorted(CASES))
def case(request):
    prob = CASES[request.param]()
    say(f"[case] {request.param} d={prob.d} n={prob.n} N={prob.N} D={prob.D} g={prob.g}")
    gp = qp.Problem(prob)
    yield request.param, prob, gp
    gp.close()


def test_diag_products_match_oracle(case):
    name, prob, gp = case
    u = W.random_vector(prob.D, seed=31)
    ref = oracle.matvec(prob, u)
    y = host(gp.matvec_d(dev(u)))
    assert np.abs(y - ref).max() <= 1e-13 * np.abs(ref).max(), name
    u32 = u.astype(np.complex64)
    ref32 = oracle.matvec(prob, u32.astype(np.complex128))
    y32 = host(gp.matvec32_d(dev(u32, torch.complex64)))
    assert np.abs(y32 - ref32).max() <= 2e-5 * np.abs(ref32).max(), name


def test_diag_setup_matches_oracle(case):
    name, prob, gp = case
    M = host(gp.precond_d())
    ref = oracle.precond(prob, 0)
    assert np.abs(M - ref).max() <= 1e-13 * np.abs(ref).max(), name
    lo, hi = gp.coef_extrema()
    rlo, rhi = oracle.coef_extrema(prob)
    assert lo == pytest.approx(rlo, abs=1e-12) and hi == pytest.approx(rhi, abs=1e-12)
    for j in range(prob.d):
        F = host(gp.corrector_rhs_d(j))
        R = oracle.corrector_rhs(prob, j)
        assert np.abs(F - R).max() <= 1e-15 * max(1.0, np.abs(R).max()), (name, j)


@pytest.mark.parametrize("prec", ["fp64", "fp32ir"])
def test_diag_homogenized_matches_oracle(case, prec):
    name, prob, gp = case
    ref = oracle.homogenize(prob, tol=1e-12)
    gp.set_precision(prec)
    try:
        r = gp.homogenized(tol=1e-12)
    finally:
        gp.set_precision("fp64")
    scale = max(np.abs(ref.A).max(), 1.0)
    say(f"  {prec} A* {r.A.ravel().tolist()} iters {[i.iters for i in r.infos]}")
    assert np.abs(r.A - ref.A).max() <= 1e-10 * scale, (name, r.A, ref.A)
    if prec == "fp64":
        assert np.abs(r.A_energy - ref.A_energy).max() <= 1e-10 * scale, name


@pytest.mark.parametrize("prec", ["fp64", "fp32ir"])
def test_paper_example_closed_forms(prec):
    prob = W.paper_homogenization(12)
    gp = qp.Problem(prob, precision=prec)
    r = gp.homogenized(tol=1e-12)
    say("paper example", prec, r.A.ravel().tolist())
    # f_2 = d_x2 beta = 0: the second corrector vanishes and A*_22 = mean(beta)
    assert abs(r.A[1, 1] - 7.0) <= 1e-14 * 7.0
    assert r.A[0, 1] == 0.0 and abs(r.A[1, 0]) <= 1e-14
    alpha = ind.coefficient_on_grid_l(prob, 0).real
    assert 1.0 / np.mean(1.0 / alpha) < r.A[0, 0] < 4.0
    gp.close()


@pytest.mark.parametrize("prec", ["fp64", "fp32ir"])
def test_laminate_harmonic_mean(prec):
    prob = W.laminate(16)
    gp = qp.Problem(prob, precision=prec)
    r = gp.homogenized(tol=1e-12)
    a1 = ind.coefficient_on_grid_l(prob, 0).real
    harm = 1.0 / np.mean(1.0 / a1)
    say("laminate", prec, r.A.ravel().tolist(), harm)
    assert r.A[0, 0] == pytest.approx(harm, rel=1e-10)
    assert abs(r.A[1, 1] - 5.0) <= 1e-14 * 5.0
    assert abs(r.A[0, 1]) <= 1e-14 and abs(r.A[1, 0]) <= 1e-14
    gp.close()


def test_diag_line_tiles_n4_products():
    prob = W.eightfold_diagonal(34, 3)  # N > 32: line tiles
    gp = qp.Problem(prob)
    u = W.random_vector(prob.D, seed=41)
    ref = oracle.matvec(prob, u)
    y = host(gp.matvec_d(dev(u)))
    assert np.abs(y - ref).max() <= 1e-13 * np.abs(ref).max()
    y32 = host(gp.matvec32_d(dev(u.astype(np.complex64), torch.complex64)))
    assert np.abs(y32 - ref).max() <= 2e-5 * np.abs(ref).max()
    gp.close()


@pytest.mark.parametrize("name", ["eightfold_diag_N12", "eightfold_diag_complex_N10"])
def test_diag_gather64_equals_default(name):
    prob = CASES[name]()
    a = qp.Problem(prob)
    b = qp.Problem(prob, gather64=True)
    u = dev(W.random_vector(prob.D, seed=51))
    assert torch.equal(a.matvec_d(u), b.matvec_d(u))
    ra = a.homogenized(tol=1e-12)
    rb = b.homogenized(tol=1e-12)
    assert np.abs(ra.A - rb.A).max() <= 1e-12 * np.abs(ra.A).max()
    a.close()
    b.close()


def test_diag_scalar_entries_equal_scalar_problem():
    base = W.eightfold_random(12, 4)
    dp = W.Problem(base.name + "_diag", base.d, base.n, base.N, base.P.copy(), base.modes.copy(),
                   base.coef.copy(), dict(base.meta), np.tile(base.coef, (base.d, 1)))
    a = qp.Problem(base)
    b = qp.Problem(dp)
    u = W.random_vector(base.D, seed=61)
    ya, yb = host(a.matvec_d(dev(u))), host(b.matvec_d(dev(u)))
    assert np.abs(ya - yb).max() <= 1e-13 * np.abs(ya).max()
    ra, rb = a.homogenized(tol=1e-12), b.homogenized(tol=1e-12)
    assert np.abs(ra.A - rb.A).max() <= 1e-10 * np.abs(ra.A).max()
    a.close()
    b.close()


def test_diag_not_elliptic_rejected():
    prob = W.laminate(8)
    coefs = prob.coefs.copy()
    zero = [i for i, m in enumerate(prob.modes) if not any(m)][0]
    coefs[1, zero] = 0.3  # a_2 = 0.3 + sin y3 - cos(y4)/2 < 0 somewhere
    st, h = qp.qp_create_diag(prob.d, prob.n, prob.P, prob.modes, coefs, prob.N)
    assert st == qp.QP_ENOTELLIPTIC and h is None, (st, qp.qp_last_error())
