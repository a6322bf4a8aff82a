"""Pins of the oracle's diagonal-coefficient path A = diag(a_1..a_d) (App. D).

Checks against an entry-by-entry assembly of Q = sum_l A^l o W^l, the
pseudo-spectral form of the same operator, the reduction to the scalar
coefficient when all entries are equal, and closed forms of A*: for the
paper's homogenization example f_2 = d_x2 beta = 0 gives A*_22 = mean(beta)
= 7 and A*_12 = A*_21 = 0 exactly; for a laminate whose entries depend on
x_1 only, A*_11 is the grid harmonic mean of a_1 over the (y_3, y_4) grid and
A*_22 the mean of a_2, exactly.
"""
from __future__ import annotations

import numpy as np
import pytest

import oracle
from paper_2404_06841_amd import workloads as W
from tests import independent as ind

SMALL = [
    W.paper_homogenization(5),
    W.laminate(4),
    W.eightfold_diagonal(5, 0),
    W.eightfold_diagonal(5, 1, complex_phase=True),
    W.periodic_2d_diagonal(8),
]
ids = lambda p: f"{p.name}_N{p.N}_{p.g}"  # noqa: E731


@pytest.mark.parametrize("prob", SMALL, ids=ids)
def test_diagonal_matvec_equals_dense_app_d(prob):
    Q = ind.dense_Q_diagonal(prob)
    assert np.abs(Q - Q.conj().T).max() <= 1e-12 * np.abs(Q).max()  # Hermitian
    u = W.random_vector(prob.D, seed=21)
    y = oracle.matvec(prob, u)
    ref = Q @ u
    np.testing.assert_allclose(y, ref, rtol=0, atol=1e-12 * np.abs(ref).max())
    # positive definite on k != 0
    assert np.linalg.eigvalsh(Q[1:, 1:]).min() > 0


@pytest.mark.parametrize("prob", SMALL + [W.eightfold_diagonal(9, 2), W.paper_homogenization(8),
                                          W.laminate(7)], ids=ids)
def test_diagonal_matvec_equals_pseudospectral(prob):
    u = W.random_vector(prob.D, seed=5)
    y = oracle.matvec(prob, u)
    z = ind.fft_apply_Q_diagonal(prob, u)
    assert np.abs(y - z).max() <= 1e-12 * np.abs(z).max()


def _as_diagonal(prob):
    return W.Problem(prob.name + "_diag", prob.d, prob.n, prob.N, prob.P.copy(), prob.modes.copy(),
                     prob.coef.copy(), dict(prob.meta), np.tile(prob.coef, (prob.d, 1)))


@pytest.mark.parametrize("prob", [W.eightfold_random(6, 1), W.icosahedral(3), W.paper_four_mode_2d(5)],
                         ids=ids)
def test_equal_entries_reduce_to_scalar_coefficient(prob):
    dp = _as_diagonal(prob)
    u = W.random_vector(prob.D, seed=2)
    y0 = oracle.matvec(prob, u)
    assert np.abs(oracle.matvec(dp, u) - y0).max() <= 1e-12 * np.abs(y0).max()
    np.testing.assert_allclose(oracle.precond(dp), oracle.precond(prob), rtol=1e-12, atol=0)
    r0 = oracle.homogenize(prob, tol=1e-13)
    r1 = oracle.homogenize(dp, tol=1e-13)
    assert np.abs(r1.A - r0.A).max() <= 1e-10 * np.abs(r0.A).max()


@pytest.mark.parametrize("prob", [W.paper_homogenization(5), W.eightfold_diagonal(5, 1, complex_phase=True)],
                         ids=ids)
def test_diagonal_precond_is_frobenius_optimal(prob):
    Q = ind.dense_Q_diagonal(prob)
    M = oracle.precond(prob, kind=0)
    colsq = np.sum(np.abs(Q) ** 2, axis=0)
    expect = np.where(colsq > 0, np.real(np.diag(Q)) / np.where(colsq > 0, colsq, 1), 0.0)
    np.testing.assert_allclose(M, expect, rtol=1e-13, atol=0)
    Mj = oracle.precond(prob, kind=1)
    dq = np.real(np.diag(Q))
    np.testing.assert_allclose(Mj, np.where(dq > 0, 1 / np.where(dq > 0, dq, 1), 0), rtol=1e-13, atol=0)


@pytest.mark.parametrize("prob", [W.laminate(4), W.eightfold_diagonal(5, 0)], ids=ids)
def test_diagonal_pcg_matches_dense_solve(prob):
    Q = ind.dense_Q_diagonal(prob)[1:, 1:]
    F = W.random_vector(prob.D, seed=4)
    x = np.linalg.solve(Q, F[1:])
    U, st, it, rr = oracle.pcg(prob, F, tol=1e-13)
    assert st == oracle.PCG_OK
    assert np.linalg.norm(U[1:] - x) <= 1e-10 * np.linalg.norm(x)


@pytest.mark.parametrize("N", [6, 8, 9])
def test_paper_homogenization_example_pins(N):
    prob = W.paper_homogenization(N)
    r = oracle.homogenize(prob, tol=1e-13)
    A = r.A
    assert A[1, 1] == 7.0 and A[0, 1] == 0.0 and A[1, 0] == 0.0
    # A*_11 between the grid harmonic and arithmetic means of alpha
    alpha = ind.coefficient_on_grid_l(prob, 0).real
    assert 1.0 / np.mean(1.0 / alpha) < A[0, 0] < 4.0
    assert r.A_energy[0, 0] == pytest.approx(A[0, 0], rel=1e-10)


@pytest.mark.parametrize("N", [4, 6, 7, 8])
def test_laminate_closed_forms(N):
    prob = W.laminate(N)
    r = oracle.homogenize(prob, tol=1e-13)
    a1 = ind.coefficient_on_grid_l(prob, 0).real  # depends on (y_3, y_4) only
    assert np.abs(a1 - a1[:1, :1]).max() <= 1e-12 * a1.max()
    harm = 1.0 / np.mean(1.0 / a1)
    assert r.A[0, 0] == pytest.approx(harm, rel=1e-11)
    assert r.A[1, 1] == 5.0
    assert r.A[0, 1] == 0.0 and r.A[1, 0] == 0.0
