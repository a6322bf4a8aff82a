"""Sampled-function inputs (Sec. 2.3): coefficient modes and right-hand sides
from values on the collocation grid.

CPU: qp_modes_from_spectrum (host code) recovers the modes of sampled
cosine and random fields (spectrum by numpy's FFT, a library primitive), and
the oracle's A* of the recovered problem equals that of the analytic one.
GPU: qp_dft_d equals the oracle's direct-sum transform in both directions
(the oracle's transform is pinned against numpy's FFT, closed forms and
Parseval in the oracle tests), and the whole sampled pipeline (samples ->
qp_dft_d -> modes -> problem -> A*; samples of f -> qp_dft_d -> solve) gives
the oracle's A* of the analytic inputs.
"""
from __future__ import annotations

import numpy as np
import pytest

import oracle
from paper_2404_06841_amd import qp
from paper_2404_06841_amd import workloads as W


def grid_samples(prob, table=None):
    """A(y_j) on T_N^n (storage order) from a mode table (default: the problem's)."""
    n, N = prob.n, prob.N
    ax = [2 * np.pi * np.arange(N) / N] * n
    Y = np.meshgrid(*ax, indexing="ij")
    out = np.zeros((N,) * n, dtype=np.complex128)
    items = table.items() if table is not None else zip(map(tuple, prob.modes), prob.coef)
    for m, c in items:
        ph = sum(int(m[t]) * Y[t] for t in range(n))
        out += c * np.exp(1j * ph)
    return out.reshape(-1)


def spectrum(samples, n, N):
    return np.fft.fftn(samples.reshape((N,) * n)).reshape(-1) / N ** n


def as_table(modes, coef):
    return {tuple(int(x) for x in m): complex(c) for m, c in zip(modes, coef)}


@pytest.mark.parametrize("prob", [W.eightfold(8), W.eightfold_random(9, 2), W.icosahedral(5),
                                  W.one_d_two_mode(12), W.paper_four_mode_2d(6)],
                         ids=lambda p: f"{p.name}_N{p.N}")
def test_modes_recovered_from_samples(prob):
    spec = spectrum(grid_samples(prob), prob.n, prob.N)
    modes, coef = qp.modes_from_spectrum(spec, prob.n, prob.N, rel_tol=1e-10)
    got, want = as_table(modes, coef), as_table(prob.modes, prob.coef)
    assert set(got) == set(want)
    for m in want:
        assert abs(got[m] - want[m]) <= 1e-13 * max(1.0, abs(want[m]))
        neg = tuple(-x for x in m)
        assert got[neg] == np.conj(got[m])  # exactly Hermitian


def test_sampled_problem_has_the_analytic_astar():
    prob = W.eightfold_random(8, 4)
    spec = spectrum(grid_samples(prob), prob.n, prob.N)
    modes, coef = qp.modes_from_spectrum(spec, prob.n, prob.N, rel_tol=1e-10)
    sp = W.Problem("sampled", prob.d, prob.n, prob.N, prob.P, modes, coef)
    a = oracle.homogenize(prob, tol=1e-13)
    b = oracle.homogenize(sp, tol=1e-13)
    assert np.abs(a.A - b.A).max() <= 1e-11 * np.abs(a.A).max()


def test_modes_from_spectrum_rejections():
    N, n = 8, 2
    spec = np.zeros(N ** n, dtype=np.complex128)
    spec[0] = 3.0
    spec[4 * N] = 0.5  # (4, 0): on the N/2 face
    with pytest.raises(qp.QPError):
        qp.modes_from_spectrum(spec, n, N, rel_tol=1e-3)
    noisy = np.random.default_rng(0).standard_normal(N ** n) + 0j
    with pytest.raises(qp.QPError):
        qp.modes_from_spectrum(noisy, n, N, rel_tol=1e-3, max_modes=16)
    with pytest.raises(qp.QPError):
        qp.modes_from_spectrum(np.zeros(N ** n, complex), n, N)


def _dft_rows_to_check(D: int) -> np.ndarray | None:
    """Every entry for small grids; else the first and last entries and a
    seeded sample (the oracle's direct sum costs O(D) per output)."""
    if D <= 4096:
        return None
    rng = np.random.default_rng(D)
    return np.unique(np.concatenate([np.arange(8), [D - 1], rng.integers(0, D, 56)]))


@pytest.mark.gpu
@pytest.mark.parametrize("n,N", [(1, 100), (2, 9), (4, 8), (6, 6), (4, 32), (3, 33), (1, 1024),
                                 (6, 16)])
def test_dft_matches_oracle(n, N):
    """qp_dft_d against the oracle's direct sum of the Sec. 2.3 definition
    (entrywise for small grids, sampled outputs for large ones), both
    directions; error bound: a few N eps per axis."""
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    D = N ** n
    x = W.random_vector(D, seed=n * 100 + N)
    xd = torch.from_numpy(x).cuda()
    rows = _dft_rows_to_check(D)
    f = qp.dft_d(xd, n, N).cpu().numpy()
    ref = oracle.dft_rows(n, N, x, rows=rows)
    got = f if rows is None else f[rows]
    # Forward outputs are of size ||x|| / D, inverse ones of size ||x||.  The
    # oracle sums D terms in sequence, so its own rounding grows like
    # eps sqrt(D) relative to the output; the GPU's per-axis sums like
    # n sqrt(N) eps.
    rel = 1e-13 + 4e-16 * np.sqrt(D)
    scale = np.linalg.norm(x) / D
    assert np.abs(got - ref).max() <= rel * scale, np.abs(got - ref).max() / scale
    b = qp.dft_d(xd, n, N, inverse=True).cpu().numpy()
    refb = oracle.dft_rows(n, N, x, rows=rows, inverse=True)
    gotb = b if rows is None else b[rows]
    assert np.abs(gotb - refb).max() <= rel * np.linalg.norm(x), \
        np.abs(gotb - refb).max() / np.linalg.norm(x)
    if D > (1 << 20):
        return
    # in place, and the round trip
    y = xd.clone()
    qp.dft_d(y, n, N, out=y)
    qp.dft_d(y, n, N, inverse=True, out=y)
    assert np.abs(y.cpu().numpy() - x).max() <= 1e-13 * np.abs(x).max()


@pytest.mark.gpu
def test_sampled_pipeline_on_gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    prob = W.eightfold_random(16, 6)
    n, N = prob.n, prob.N
    s = torch.from_numpy(grid_samples(prob)).cuda()
    spec = qp.dft_d(s, n, N).cpu().numpy()
    modes, coef = qp.modes_from_spectrum(spec, n, N, rel_tol=1e-10)
    sp = W.Problem("sampled", prob.d, n, N, prob.P, modes, coef)
    a = qp.Problem(prob)
    b = qp.Problem(sp)
    ra, rb = a.homogenized(tol=1e-12), b.homogenized(tol=1e-12)
    assert np.abs(ra.A - rb.A).max() <= 1e-11 * np.abs(ra.A).max()
    # the sampled problem's A* against the oracle's A* of the analytic one
    ref = oracle.homogenize(prob, tol=1e-12)
    assert np.abs(rb.A - ref.A).max() <= 1e-10 * np.abs(ref.A).max()
    # a right-hand side from samples of f = d_x1 of the coefficient
    F_exact = a.corrector_rhs_d(0)
    f_samples = qp.dft_d(F_exact, n, N, inverse=True)
    F = qp.dft_d(f_samples, n, N)
    assert (F - F_exact).abs().max().item() <= 1e-13 * F_exact.abs().max().item()
    u1, i1 = a.solve_d(F_exact, tol=1e-12)
    u2, i2 = a.solve_d(F, tol=1e-12)
    assert (u1 - u2).abs().max().item() <= 1e-9 * u1.abs().max().item()
    a.close()
    b.close()
