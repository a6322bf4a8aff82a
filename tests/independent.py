"""Independent second implementations used only to pin the oracle.

Each function restates a definition from the paper in a different form from
the oracle's C code, so that a mistake in one is caught by the other:

* ``dense_Q``: the stiffness matrix assembled entry by entry as in Alg. 1
  (A_ij = Ahat_{k_V -_N k_U}, W_ij = (P k_V).(P k_U), Q_ij = A_ij W_ij).
* ``fft_apply_Q``: Q u evaluated pseudo-spectrally on the collocation grid
  via discrete orthogonality (Sec. 2.3): multiply each component of the lifted
  gradient by the sampled coefficient and transform back.
* ``continuum_rhs``: -div(a grad u) for a finite Fourier series u, with no
  truncation or aliasing (the continuous operator in frequency space).
"""
from __future__ import annotations

import itertools

import numpy as np


def signed_indices(n: int, N: int) -> np.ndarray:
    """Rows: the signed k of every vector entry, in storage order (D x n).

    Built from numpy's FFT frequency convention (which is exactly the paper's
    per-dimension order 0, 1, ..., N/2-1, -N/2, ..., -1)."""
    f = np.fft.fftfreq(N, d=1.0 / N).astype(np.int64)
    grids = np.meshgrid(*([f] * n), indexing="ij")
    return np.stack([g.reshape(-1) for g in grids], axis=1)


def coef_table(prob) -> dict:
    return {tuple(int(x) for x in m): complex(c) for m, c in zip(prob.modes, prob.coef)}


def dense_Q(prob) -> np.ndarray:
    """Q = A o W assembled entry by entry (Alg. 1): for the pair (k_V, k_U),
    A_ij = Ahat at k_A = (k_V - k_U) mod N and W_ij = (P k_V).(P k_U)."""
    n, N = prob.n, prob.N
    K = signed_indices(n, N)
    PK = K @ np.asarray(prob.P, dtype=np.float64).T  # (D, d)
    D = K.shape[0]
    ahat = np.zeros(D, dtype=np.complex128)  # Ahat indexed by the class of k mod N
    weights = N ** np.arange(n - 1, -1, -1)
    for m, c in coef_table(prob).items():
        ahat[int(np.mod(np.array(m), N) @ weights)] += c
    Q = np.zeros((D, D), dtype=np.complex128)
    for i in range(D):
        kA = np.mod(K[i][None, :] - K, N)
        Q[i, :] = ahat[kA @ weights] * (PK @ PK[i])
    return Q


def coefficient_on_grid(prob) -> np.ndarray:
    """A(y_j) on the collocation grid T_N^n, shape (N,)*n."""
    n, N = prob.n, prob.N
    spec = np.zeros((N,) * n, dtype=np.complex128)
    for m, c in coef_table(prob).items():
        spec[tuple(int(x) % N for x in m)] += c
    return np.fft.ifftn(spec) * N ** n


def fft_apply_Q(prob, u) -> np.ndarray:
    n, N, d = prob.n, prob.N, prob.d
    K = signed_indices(n, N).astype(np.float64)
    PK = K @ np.asarray(prob.P, dtype=np.float64).T
    a = coefficient_on_grid(prob)
    y = np.zeros(N ** n, dtype=np.complex128)
    for l in range(d):
        g = np.fft.ifftn((PK[:, l] * u).reshape((N,) * n)) * N ** n   # l-th lifted derivative / i
        y += PK[:, l] * (np.fft.fftn(a * g) / N ** n).reshape(-1)
    return y


# ---- diagonal coefficient A = diag(a_1..a_d) (App. D) ----

def coef_table_l(prob, l: int) -> dict:
    """a_l's Fourier coefficients as {mode: Ahat} (the scalar a when the
    problem has no diagonal coefficient)."""
    coefs = getattr(prob, "coefs", None)
    row = prob.coef if coefs is None else np.asarray(coefs)[l]
    return {tuple(int(x) for x in m): complex(c) for m, c in zip(prob.modes, row) if c != 0}


def dense_Q_diagonal(prob) -> np.ndarray:
    """Q = sum_l A^l o W^l assembled entry by entry (App. D): for the pair
    (k_V, k_U), A^l_ij = Ahat of a_l at (k_V - k_U) mod N and
    W^l_ij = (P k_V)_l (P k_U)_l."""
    n, N, d = prob.n, prob.N, prob.d
    K = signed_indices(n, N)
    PK = K @ np.asarray(prob.P, dtype=np.float64).T
    D = K.shape[0]
    weights = N ** np.arange(n - 1, -1, -1)
    Q = np.zeros((D, D), dtype=np.complex128)
    for l in range(d):
        ahat = np.zeros(D, dtype=np.complex128)
        for m, c in coef_table_l(prob, l).items():
            ahat[int(np.mod(np.array(m), N) @ weights)] += c
        for i in range(D):
            kA = np.mod(K[i][None, :] - K, N)
            Q[i, :] += ahat[kA @ weights] * (PK[:, l] * PK[i, l])
    return Q


def coefficient_on_grid_l(prob, l: int) -> np.ndarray:
    """a_l(y_j) on the collocation grid T_N^n, shape (N,)*n."""
    n, N = prob.n, prob.N
    spec = np.zeros((N,) * n, dtype=np.complex128)
    for m, c in coef_table_l(prob, l).items():
        spec[tuple(int(x) % N for x in m)] += c
    return np.fft.ifftn(spec) * N ** n


def fft_apply_Q_diagonal(prob, u) -> np.ndarray:
    """Q u = sum_l (P k)_l DFT[a_l(y) IDFT[(P k)_l u]] (discrete orthogonality,
    one coefficient per component of the lifted gradient)."""
    n, N, d = prob.n, prob.N, prob.d
    K = signed_indices(n, N).astype(np.float64)
    PK = K @ np.asarray(prob.P, dtype=np.float64).T
    y = np.zeros(N ** n, dtype=np.complex128)
    for l in range(d):
        a = coefficient_on_grid_l(prob, l)
        g = np.fft.ifftn((PK[:, l] * u).reshape((N,) * n)) * N ** n
        y += PK[:, l] * (np.fft.fftn(a * g) / N ** n).reshape(-1)
    return y


def rayleigh_quotient(prob, u) -> float:
    """(1/D) sum_y a(y) |sum_j (P j) u_j e^{i j.y}|^2."""
    n, N, d = prob.n, prob.N, prob.d
    K = signed_indices(n, N).astype(np.float64)
    PK = K @ np.asarray(prob.P, dtype=np.float64).T
    a = coefficient_on_grid(prob).real
    tot = 0.0
    for l in range(d):
        g = np.fft.ifftn((PK[:, l] * u).reshape((N,) * n)) * N ** n
        tot += float(np.sum(a * np.abs(g) ** 2))
    return tot / N ** n


def continuum_rhs(prob, u: dict) -> dict:
    """f = -div(a grad u) for u = sum_k u_k e^{i (P k).x}: f_k = sum_m Ahat_m (P k).(P(k-m)) u_{k-m}."""
    P = np.asarray(prob.P, dtype=np.float64)
    out = {}
    for k, uk in u.items():
        for m, am in coef_table(prob).items():
            kv = tuple(a + b for a, b in zip(k, m))
            w = float((P @ np.array(kv, dtype=np.float64)) @ (P @ np.array(k, dtype=np.float64)))
            out[kv] = out.get(kv, 0.0) + am * w * uk
    return {k: v for k, v in out.items() if any(k)}


def fits_strictly(keys, n: int, N: int) -> bool:
    lo, hi = -(N // 2) if N % 2 == 0 else -((N - 1) // 2), (N - 1) // 2 if N % 2 else N // 2 - 1
    return all(lo <= x <= hi for k in keys for x in k)


def all_signed(n: int, N: int):
    lo = -(N // 2)
    return itertools.product(range(lo, lo + N), repeat=n)


def sparse_vector(n: int, N: int, table: dict) -> np.ndarray:
    """Dense vector of the grid K_N^n holding table[k] at signed index k
    (storage position from numpy's row-major raveling of k mod N, the FFT
    order of every axis)."""
    v = np.zeros(N ** n, dtype=np.complex128)
    for k, val in table.items():
        v[np.ravel_multi_index(tuple(int(x) % N for x in k), (N,) * n)] += val
    return v


def sine_source(n: int, N: int, axes) -> np.ndarray:
    """F for f = sum_{t in axes} sin(y_t): Fhat_{+e_t} = -i/2, Fhat_{-e_t} = +i/2."""
    table = {}
    for t in axes:
        e = [0] * n
        e[t] = 1
        table[tuple(e)] = -0.5j
        e[t] = -1
        table[tuple(e)] = 0.5j
    return sparse_vector(n, N, table)
