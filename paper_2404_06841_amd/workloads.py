"""Seeded synthetic inputs for the projection-method solver.

This module produces *inputs only*: projection matrices P, coefficient modes
m with their Fourier coefficients, grid sizes N and right-hand sides.  It does
none of the method's arithmetic (no stiffness products, preconditioner, Krylov
solve or homogenized coefficient), so the GPU path and the CPU reference can
both consume exactly the same arrays.  It imports only numpy.

Conventions (Sec. 2.1 and Sec. 3.1 of the paper):

* A quasiperiodic coefficient is a(x) = A(P^T x) with a parent function A on
  the n-torus, A(y) = sum_m Ahat_m exp(i m.y).  A problem is given by P (d x n,
  row-major), the integer mode list m (g x n) and the complex coefficients
  Ahat_m (g,).  A real coefficient needs Ahat_{-m} = conj(Ahat_m).
* A diagonal coefficient diag(a_1, ..., a_d) (App. D) shares one mode list;
  ``coefs`` (d x g) then holds a_l's Ahat per mode (0 where a_l has no such
  mode), and ``coef`` repeats row 0.
* Vectors of unknowns have D = N^n complex entries in the tensor-to-vector
  order of Sec. 3.1.2: row-major, k_1 slowest, each index stored as k mod N
  (FFT order).

Every random draw is made from ``numpy.random.default_rng(seed)``.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

SQRT2 = float(np.sqrt(2.0))
SQRT3 = float(np.sqrt(3.0))
SQRT5 = float(np.sqrt(5.0))
TAU = float((1.0 + np.sqrt(5.0)) / 2.0)
TWO_PI = float(2.0 * np.pi)

#: base seed of the random-coefficient workloads (the arXiv id followed by 0)
BASE_SEED = 2404068410


@dataclass
class Problem:
    """One quasiperiodic elliptic problem: P, coefficient modes and N."""

    name: str
    d: int
    n: int
    N: int
    P: np.ndarray  # (d, n) float64, row-major
    modes: np.ndarray  # (g, n) int32
    coef: np.ndarray  # (g,) complex128
    meta: dict = field(default_factory=dict)
    coefs: np.ndarray | None = None  # (d, g) complex128: diagonal coefficient

    @property
    def D(self) -> int:
        return int(self.N) ** int(self.n)

    @property
    def g(self) -> int:
        return int(self.modes.shape[0])

    def with_N(self, N: int) -> "Problem":
        return Problem(self.name, self.d, self.n, int(N), self.P.copy(),
                       self.modes.copy(), self.coef.copy(), dict(self.meta),
                       None if self.coefs is None else self.coefs.copy())


def _modes_from_dict(n: int, table: dict) -> tuple[np.ndarray, np.ndarray]:
    keys = sorted(table.keys())
    modes = np.array(keys, dtype=np.int32).reshape(len(keys), n)
    coef = np.array([table[k] for k in keys], dtype=np.complex128)
    return modes, coef


def _unit(n: int, t: int, s: int = 1) -> tuple:
    v = [0] * n
    v[t] = s
    return tuple(v)


def cosine_field(n: int, mean: float, amplitudes) -> tuple[np.ndarray, np.ndarray]:
    """A(y) = mean + sum_t amplitudes[t] cos(y_t): Ahat_{+-e_t} = amplitudes[t]/2."""
    table = {tuple([0] * n): complex(mean)}
    for t, c in enumerate(amplitudes):
        if c == 0.0:
            continue
        table[_unit(n, t, +1)] = complex(c / 2.0)
        table[_unit(n, t, -1)] = complex(c / 2.0)
    return _modes_from_dict(n, table)


# --------------------------------------------------------------------------
# Projection matrices
# --------------------------------------------------------------------------

def eightfold_P() -> np.ndarray:
    """Columns (1,0), (0,1), (cos pi/4, sin pi/4), (cos 3pi/4, sin 3pi/4)."""
    c = SQRT2 / 2.0
    return np.array([[1.0, 0.0, c, -c],
                     [0.0, 1.0, c, c]], dtype=np.float64)


def icosahedral_P() -> np.ndarray:
    """Columns (1,tau,0), (-1,tau,0), (0,1,tau), (0,-1,tau), (tau,0,1), (tau,0,-1)."""
    t = TAU
    cols = [(1.0, t, 0.0), (-1.0, t, 0.0), (0.0, 1.0, t), (0.0, -1.0, t),
            (t, 0.0, 1.0), (t, 0.0, -1.0)]
    return np.array(cols, dtype=np.float64).T.copy()


# --------------------------------------------------------------------------
# Named workloads
# --------------------------------------------------------------------------

def one_d_two_mode(N: int = 32, mean: float = 2.0, scale: float = 1.0) -> Problem:
    """d=1, n=2, P = scale*(1, sqrt2), A = mean + cos y1 + cos y2.

    mean=2, scale=1 is the 1024-unknown configuration at N=32 (degenerate: A
    touches 0 at y=(pi,pi)); mean=6, scale=2*pi is the paper's first example
    (Sec. 5.1.1).
    """
    P = np.array([[1.0, SQRT2]], dtype=np.float64) * scale
    modes, coef = cosine_field(2, mean, [1.0, 1.0])
    return Problem("1d_n2", 1, 2, int(N), P, modes, coef,
                   {"mean": mean, "scale": scale})


def one_d_three_mode(N: int = 16, mean: float = 6.0) -> Problem:
    """d=1, n=3, P = 2*pi*(1, sqrt2, sqrt3), A = mean + cos y1 + cos y2 + cos y3 (Sec. 5.1.3)."""
    P = np.array([[1.0, SQRT2, SQRT3]], dtype=np.float64) * TWO_PI
    modes, coef = cosine_field(3, mean, [1.0, 1.0, 1.0])
    return Problem("1d_n3", 1, 3, int(N), P, modes, coef, {"mean": mean})


def paper_four_mode_2d(N: int = 6) -> Problem:
    """d=2, n=4 example of Sec. 5.1.5: A = 12 + cos y1 + cos y2 + cos y3 + sin y4.

    P = 2*pi*[[1, 0, sqrt3, 0], [0, sqrt2, 0, sqrt5]].  The sine term gives a
    purely imaginary Hermitian pair, Ahat_{+-e4} = -+ i/2.
    """
    P = TWO_PI * np.array([[1.0, 0.0, SQRT3, 0.0],
                           [0.0, SQRT2, 0.0, SQRT5]], dtype=np.float64)
    n = 4
    table = {tuple([0] * n): 12.0 + 0j}
    for t in range(3):
        table[_unit(n, t, 1)] = 0.5 + 0j
        table[_unit(n, t, -1)] = 0.5 + 0j
    table[_unit(n, 3, 1)] = -0.5j
    table[_unit(n, 3, -1)] = 0.5j
    modes, coef = _modes_from_dict(n, table)
    return Problem("paper_2d_n4", 2, 4, int(N), P, modes, coef)


def periodic_1d(N: int = 100, mean: float = 2.0, amp: float = 1.0) -> Problem:
    """d = n = 1 (periodic): P = [1], A = mean + amp cos y."""
    modes, coef = cosine_field(1, mean, [amp])
    return Problem("periodic_1d", 1, 1, int(N), np.ones((1, 1)), modes, coef)


def eightfold(N: int = 16, amplitude: float = 0.5, mean: float = 3.0) -> Problem:
    """d=2, n=4 eightfold: A = mean + amplitude * sum_{j=1..4} cos(y_j).

    amplitude=1 is the literal (indefinite) field 3 + sum cos; the measured
    runs use amplitude 1/2 so that 1 <= a <= 5.
    """
    modes, coef = cosine_field(4, mean, [amplitude] * 4)
    return Problem("eightfold", 2, 4, int(N), eightfold_P(), modes, coef,
                   {"amplitude": amplitude, "mean": mean})


def random_modes(n: int, pairs: int, radius: int, rng: np.random.Generator,
                 max_amp: float, amp_cap: float, mean: float):
    """Draw `pairs` distinct +-m pairs from {-radius..radius}^n \\ {0} (modulo sign)
    with amplitudes c ~ U(0, max_amp), redrawing the amplitudes while their sum
    exceeds amp_cap; Ahat_{+-m} = c/2, Ahat_0 = mean."""
    side = 2 * radius + 1
    reps = []
    for flat in range(side ** n):
        v = []
        x = flat
        for _ in range(n):
            v.append(x % side - radius)
            x //= side
        v = tuple(reversed(v))
        if any(v):
            neg = tuple(-c for c in v)
            if v > neg:  # one representative of each +-pair
                reps.append(v)
    idx = rng.choice(len(reps), size=pairs, replace=False)
    chosen = [reps[i] for i in sorted(idx)]
    amps = rng.uniform(0.0, max_amp, size=pairs)
    while amps.sum() > amp_cap:
        amps = rng.uniform(0.0, max_amp, size=pairs)
    table = {tuple([0] * n): complex(mean)}
    for v, c in zip(chosen, amps):
        table[v] = complex(c / 2.0)
        table[tuple(-x for x in v)] = complex(c / 2.0)
    modes, coef = _modes_from_dict(n, table)
    return modes, coef, amps


def eightfold_random(N: int = 32, instance: int = 0, pairs: int = 8) -> Problem:
    """Eightfold P with `pairs` seeded random +-mode pairs around mean 3.

    Mode pairs come from {-2..2}^4 \\ {0}; amplitudes c_r ~ U(0, 0.4) redrawn
    while sum c_r > 2.5, so a >= 0.5.  Seed = BASE_SEED + instance.
    """
    rng = np.random.default_rng(BASE_SEED + int(instance))
    modes, coef, amps = random_modes(4, pairs, 2, rng, 0.4, 2.5, 3.0)
    return Problem("eightfold_random", 2, 4, int(N), eightfold_P(), modes, coef,
                   {"instance": int(instance), "amplitudes": amps.tolist()})


def eightfold_batch(count: int = 64, seed: int = BASE_SEED,
                    sizes=(8, 12, 16, 24, 32)) -> list:
    """`count` eightfold_random instances with N drawn uniformly from `sizes`."""
    rng = np.random.default_rng(int(seed))
    Ns = rng.choice(np.array(sizes), size=count, replace=True)
    return [eightfold_random(int(Ns[i]), instance=i) for i in range(count)]


def icosahedral(N: int = 8, amplitude: float = 0.5, mean: float = 4.0) -> Problem:
    """d=3, n=6 icosahedral: A = mean + amplitude * sum_{j=1..6} cos(y_j)."""
    modes, coef = cosine_field(6, mean, [amplitude] * 6)
    return Problem("icosahedral", 3, 6, int(N), icosahedral_P(), modes, coef,
                   {"amplitude": amplitude, "mean": mean})


def periodic_cubic(d: int = 4, N: int = 6, amplitude: float = 0.5, mean: float = 3.0) -> Problem:
    """Periodic d = n problem (P = identity): A = mean + amplitude * sum_t cos(y_t)."""
    modes, coef = cosine_field(d, mean, [amplitude] * d)
    return Problem("periodic_cubic", d, d, int(N), np.eye(d, dtype=np.float64), modes, coef,
                   {"amplitude": amplitude, "mean": mean})


def anisotropic_paper_example():
    """Appendix D / Sec. 5.2 homogenization example, as two parent fields on T^4.

    P = 2*pi*[[1, sqrt2, 1, sqrt2], [1, sqrt2, 0, 0]];
    alpha(x) = 4 + cos(2*pi(x1+x2)) + cos(2*pi*sqrt2(x1+x2)) -> parent 4 + cos y1 + cos y2,
    beta(x)  = 6 + sin^2(2*pi x1) + sin^2(2*pi*sqrt2 x1)       -> parent 7 - cos(2 y3)/2 - cos(2 y4)/2.
    Returns (P, (modes_alpha, coef_alpha), (modes_beta, coef_beta)).
    """
    P = TWO_PI * np.array([[1.0, SQRT2, 1.0, SQRT2],
                           [1.0, SQRT2, 0.0, 0.0]], dtype=np.float64)
    n = 4
    ta = {tuple([0] * n): 4.0 + 0j,
          _unit(n, 0, 1): 0.5 + 0j, _unit(n, 0, -1): 0.5 + 0j,
          _unit(n, 1, 1): 0.5 + 0j, _unit(n, 1, -1): 0.5 + 0j}
    tb = {tuple([0] * n): 7.0 + 0j,
          _unit(n, 2, 2): -0.25 + 0j, _unit(n, 2, -2): -0.25 + 0j,
          _unit(n, 3, 2): -0.25 + 0j, _unit(n, 3, -2): -0.25 + 0j}
    return P, _modes_from_dict(n, ta), _modes_from_dict(n, tb)


def diagonal(name: str, d: int, n: int, N: int, P: np.ndarray, fields, meta=None) -> Problem:
    """Diagonal coefficient diag(a_1..a_d) from d (modes, coef) fields with a
    common P: the union of the modes, coefs[l] = a_l's Ahat on it."""
    if len(fields) != d:
        raise ValueError("one field per physical axis")
    tables = []
    for modes, coef in fields:
        tables.append({tuple(int(x) for x in m): complex(c) for m, c in zip(modes, coef)})
    keys = sorted(set().union(*[t.keys() for t in tables]))
    modes = np.array(keys, dtype=np.int32).reshape(len(keys), n)
    coefs = np.array([[t.get(k, 0j) for k in keys] for t in tables], dtype=np.complex128)
    return Problem(name, int(d), int(n), int(N), np.asarray(P, dtype=np.float64).reshape(d, n),
                   modes, coefs[0].copy(), dict(meta or {}), coefs)


def paper_homogenization(N: int = 8) -> Problem:
    """The homogenization example of Sec. 5.2 / App. D: A = diag(alpha, beta)."""
    P, fa, fb = anisotropic_paper_example()
    return diagonal("paper_homogenization", 2, 4, N, P, [fa, fb])


def laminate(N: int = 8) -> Problem:
    """A = diag(a_1(x_1), a_2(x_1)) on the P of the homogenization example:
    a_1 = 6 + cos(2 pi x_1) + cos(2 pi sqrt2 x_1) / 2 -> parent 6 + cos y3 + cos(y4)/2,
    a_2 = 5 + sin(2 pi x_1) - cos(2 pi sqrt2 x_1) / 2 -> parent 5 + sin y3 - cos(y4)/2
    (a_2 has imaginary Fourier coefficients)."""
    P, _, _ = anisotropic_paper_example()
    n = 4
    t1 = {tuple([0] * n): 6.0 + 0j,
          _unit(n, 2, 1): 0.5 + 0j, _unit(n, 2, -1): 0.5 + 0j,
          _unit(n, 3, 1): 0.25 + 0j, _unit(n, 3, -1): 0.25 + 0j}
    t2 = {tuple([0] * n): 5.0 + 0j,
          _unit(n, 2, 1): -0.5j, _unit(n, 2, -1): 0.5j,
          _unit(n, 3, 1): -0.25 + 0j, _unit(n, 3, -1): -0.25 + 0j}
    return diagonal("laminate", 2, 4, N, P, [_modes_from_dict(n, t1), _modes_from_dict(n, t2)])


def eightfold_diagonal(N: int = 16, instance: int = 0, pairs: int = 6,
                       complex_phase: bool = False) -> Problem:
    """Eightfold P with an independent seeded random field per diagonal entry
    (as eightfold_random, means 3 and 4).  complex_phase: each +-pair's
    coefficients get a seeded phase, Ahat_{+-m} = (c/2) exp(+-i phi)."""
    rng = np.random.default_rng(BASE_SEED + 1000 + int(instance))
    fields = []
    for mean in (3.0, 4.0):
        modes, coef, _ = random_modes(4, pairs, 2, rng, 0.4, 2.5, mean)
        if complex_phase:
            coef = coef.copy()
            table = {tuple(int(x) for x in m): i for i, m in enumerate(modes)}
            for i, m in enumerate(modes):
                key = tuple(int(x) for x in m)
                neg = tuple(-x for x in key)
                if any(key) and key > neg:
                    phi = rng.uniform(0.0, 2.0 * np.pi)
                    coef[i] *= np.exp(1j * phi)
                    coef[table[neg]] *= np.exp(-1j * phi)
        fields.append((modes, coef))
    return diagonal("eightfold_diagonal", 2, 4, N, eightfold_P(), fields,
                    {"instance": int(instance), "complex_phase": bool(complex_phase)})


def periodic_2d_diagonal(N: int = 40) -> Problem:
    """d = n = 2 (periodic), A = diag(4 + cos y1 + cos y2 / 2, 3 + sin y2 / 2)."""
    n = 2
    P = np.array([[1.0, 0.0], [0.0, 1.0]], dtype=np.float64)
    t1 = {(0, 0): 4.0 + 0j, (1, 0): 0.5 + 0j, (-1, 0): 0.5 + 0j,
          (0, 1): 0.25 + 0j, (0, -1): 0.25 + 0j}
    t2 = {(0, 0): 3.0 + 0j, (0, 1): -0.25j, (0, -1): 0.25j}
    return diagonal("periodic_2d_diagonal", 2, n, N, P,
                    [_modes_from_dict(n, t1), _modes_from_dict(n, t2)])


# --------------------------------------------------------------------------
# Right-hand sides and vectors
# --------------------------------------------------------------------------

def random_vector(D: int, seed: int, dtype=np.complex128) -> np.ndarray:
    """Complex standard-normal vector of length D."""
    rng = np.random.default_rng(int(seed))
    v = rng.standard_normal(D) + 1j * rng.standard_normal(D)
    return v.astype(dtype)


def exponential_solution_modes(n_axes: int = 2, half: int = 32) -> dict:
    """Coefficients uhat_k = exp(-(|k1|+|k2|)) for -half <= k1,k2 < half (Sec. 5.1.2)."""
    out = {}
    for a in range(-half, half):
        for b in range(-half, half):
            out[(a, b)] = complex(np.exp(-(abs(a) + abs(b))))
    return out
