"""Stiffness product on Hermitian half storage (qp_matvec_half_d) against the
FP64 oracle's full product.

A real coefficient (Ahat_{-m} = conj(Ahat_m)) and a vector with
u_{-k} = conj(u_k) give a product with the same symmetry (Sec. 2.3 and
eq. n-discrete: W is real), so the half layout holds everything at odd N.
The layout is rebuilt here from its definition (position 0: k = 0; then for
t = n, ..., 1 the C(k) index range [N^(n-t), (N+1)/2 N^(n-t))).  Tolerance:
|gpu - oracle| <= 1e-13 max|oracle| (summation order differs only).
"""
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


def half_indices(n: int, N: int) -> np.ndarray:
    parts = [np.zeros(1, dtype=np.int64)]
    for t in range(n, 0, -1):
        S = N ** (n - t)
        parts.append(np.arange(S, (N + 1) // 2 * S, dtype=np.int64))
    return np.concatenate(parts)


def negated(n: int, N: int, idx: np.ndarray) -> np.ndarray:
    """C(-k) for the entries idx = C(k)."""
    out = np.zeros_like(idx)
    rest = idx.copy()
    for t in range(n - 1, -1, -1):
        a = rest % N
        rest //= N
        out += ((N - a) % N) * N ** (n - 1 - t)
    return out


def hermitian_pair(prob, seed: int):
    """A random half vector and the full vector it stands for."""
    n, N, D = prob.n, prob.N, prob.D
    idx = half_indices(n, N)
    assert idx.size == (D + 1) // 2
    rng = np.random.default_rng(seed)
    uh = rng.standard_normal(idx.size) + 1j * rng.standard_normal(idx.size)
    uh[0] = 0.0
    full = np.zeros(D, dtype=np.complex128)
    full[idx] = uh
    full[negated(n, N, idx[1:])] = np.conj(uh[1:])
    return idx, uh, full


CASES = {
    "icosa_N7": lambda: W.icosahedral(7),
    "eightfold_random_N9": lambda: W.eightfold_random(9, 3),
    "three_mode_1d_N9": lambda: W.one_d_three_mode(9),
    "paper2d_complex_coef_N7": lambda: W.paper_four_mode_2d(7),
    "ex1_N33_lines": lambda: W.one_d_two_mode(33, 6.0, 2 * np.pi),
}


@pytest.mark.parametrize("name", sorted(CASES))
def test_half_product_matches_oracle(name):
    prob = CASES[name]()
    say(f"[case] {name} n={prob.n} N={prob.N} D={prob.D} g={prob.g}")
    idx, uh, full = hermitian_pair(prob, seed=prob.N)
    ref = oracle.matvec(prob, full)
    # the full product keeps the symmetry: y_{-k} = conj(y_k)
    neg = negated(prob.n, prob.N, idx[1:])
    assert np.abs(ref[neg] - np.conj(ref[idx[1:]])).max() <= 1e-13 * np.abs(ref).max()
    gp = qp.Problem(prob)
    yh = gp.matvec_half_d(torch.from_numpy(uh).cuda()).cpu().numpy()
    assert yh[0] == 0
    err = np.abs(yh - ref[idx]).max() / np.abs(ref).max()
    say(f"  rel err {err:.2e}")
    assert err <= 1e-13
    # the full-storage GPU product agrees on the stored half
    yf = gp.matvec_d(torch.from_numpy(full).cuda()).cpu().numpy()
    assert np.abs(yf[idx] - yh).max() <= 1e-13 * np.abs(ref).max()
    gp.close()


def test_half_product_large_sampled_rows():
    """Icosahedral N = 15: 11,390,625 unknowns, 5,695,313 stored; sampled rows."""
    prob = W.icosahedral(15)
    say(f"[case] icosahedral N=15 D={prob.D}")
    idx, uh, full = hermitian_pair(prob, seed=15)
    gp = qp.Problem(prob)
    yh = gp.matvec_half_d(torch.from_numpy(uh).cuda()).cpu().numpy()
    rng = np.random.default_rng(5)
    pos = np.unique(np.concatenate([rng.integers(1, idx.size, 4000),
                                    [1, idx.size - 1], np.arange(1, 200)]))
    ref = oracle.matvec_rows(prob, full, idx[pos])
    err = np.abs(yh[pos] - ref).max() / np.abs(ref).max()
    say(f"  sampled rel err {err:.2e}")
    assert err <= 1e-13
    gp.close()


def test_half_product_rejects_even_N_and_diagonal_coefficients():
    gp = qp.Problem(W.eightfold(8))
    u = torch.zeros((gp.D + 1) // 2, dtype=torch.complex128, device="cuda")
    with pytest.raises(qp.QPError) as e:
        gp.matvec_half_d(u)
    assert e.value.status == qp.QP_EINVAL and "odd N" in str(e.value)
    gp.close()
    gp = qp.Problem(W.eightfold_diagonal(9, 1))
    u = torch.zeros((gp.D + 1) // 2, dtype=torch.complex128, device="cuda")
    with pytest.raises(qp.QPError) as e:
        gp.matvec_half_d(u)
    assert e.value.status == qp.QP_EINVAL
    gp.close()
