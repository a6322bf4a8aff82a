"""CPU reference (oracle) for the projection-method solver.

TEST INFRASTRUCTURE ONLY: the slow, plain FP64 implementation the GPU library is
checked against.  Only the tests, the smoke check and the benchmark's CPU
baseline use it; the product never imports it.  It shares no code with the GPU
library.  The arithmetic lives in ``qp_oracle.c`` (compiled by ``build.py``);
this module only marshals numpy arrays.

A problem is any object with attributes d, n, N, P (d x n), modes (g x n int)
and coef (g complex), e.g. the inputs made by the workload generator; an
optional attribute coefs (d x g complex, not None) makes the coefficient the
diagonal matrix diag(a_1..a_d) of App. D, row l holding a_l's Fourier
coefficients on the shared mode list.
"""
from __future__ import annotations

import ctypes as C
import os
from types import SimpleNamespace

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

PCG_OK, PCG_NOCONV, PCG_NOTSPD = 0, 1, 2


class _Problem(C.Structure):
    _fields_ = [("d", C.c_int), ("n", C.c_int), ("N", C.c_int), ("g", C.c_int),
                ("P", C.POINTER(C.c_double)), ("modes", C.POINTER(C.c_int)),
                ("coef", C.POINTER(C.c_double)), ("coefs", C.POINTER(C.c_double))]


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        from . import build as _b
        _b.build()
    lib = C.CDLL(_LIB_PATH)
    dp = C.POINTER(C.c_double)
    pp = C.POINTER(_Problem)
    lib.qo_set_threads.restype = None
    lib.qo_set_threads.argtypes = [C.c_int]
    lib.qo_max_threads.restype = C.c_int
    lib.qo_max_threads.argtypes = []
    lib.qo_size.restype = C.c_long
    lib.qo_size.argtypes = [C.c_int, C.c_int]
    lib.qo_rep.restype = C.c_int
    lib.qo_rep.argtypes = [C.c_int, C.c_long]
    lib.qo_index.restype = C.c_long
    lib.qo_index.argtypes = [C.c_int, C.c_int, C.POINTER(C.c_int)]
    lib.qo_multi_index.restype = None
    lib.qo_multi_index.argtypes = [C.c_int, C.c_int, C.c_long, C.POINTER(C.c_int)]
    lib.qo_matvec.restype = None
    lib.qo_matvec.argtypes = [pp, dp, dp]
    lib.qo_matvec_rows.restype = None
    lib.qo_matvec_rows.argtypes = [pp, dp, C.c_long, C.POINTER(C.c_long), dp]
    lib.qo_precond.restype = None
    lib.qo_precond.argtypes = [pp, C.c_int, dp]
    lib.qo_pcg.restype = C.c_int
    lib.qo_pcg.argtypes = [pp, C.c_int, dp, dp, C.c_double, C.c_int,
                           C.POINTER(C.c_int), dp]
    lib.qo_pcg_ex.restype = C.c_int
    lib.qo_pcg_ex.argtypes = [pp, C.c_int, dp, dp, C.c_double, C.c_int,
                              C.POINTER(C.c_int), dp, dp]
    lib.qo_dft_rows.restype = None
    lib.qo_dft_rows.argtypes = [C.c_int, C.c_int, C.c_int, dp, C.c_long, C.POINTER(C.c_long), dp]
    lib.qo_corrector_rhs.restype = None
    lib.qo_corrector_rhs.argtypes = [pp, C.c_int, dp]
    lib.qo_astar_flux.restype = C.c_double
    lib.qo_astar_flux.argtypes = [pp, C.c_int, C.c_int, dp, dp]
    lib.qo_astar_energy.restype = C.c_double
    lib.qo_astar_energy.argtypes = [pp, C.c_int, C.c_int, dp, dp, dp]
    lib.qo_coef_extrema.restype = None
    lib.qo_coef_extrema.argtypes = [pp, dp, dp]
    _lib = lib
    return lib


class _Bound:
    """Keeps the numpy buffers alive while the C struct points at them."""

    def __init__(self, prob):
        if prob.n > 8:
            raise ValueError("oracle supports n <= 8")
        self.P = np.ascontiguousarray(prob.P, dtype=np.float64).reshape(prob.d, prob.n)
        self.modes = np.ascontiguousarray(prob.modes, dtype=np.int32).reshape(-1, prob.n)
        g = int(self.modes.shape[0])
        coefs = getattr(prob, "coefs", None)
        if coefs is not None:
            # diagonal coefficient diag(a_1..a_d): row l holds a_l's Ahat per mode
            cs = np.ascontiguousarray(coefs, dtype=np.complex128).reshape(int(prob.d), g)
            self.coefs = cs.reshape(-1).view(np.float64).copy()
            coef = cs[0]
        else:
            self.coefs = None
            coef = np.ascontiguousarray(prob.coef, dtype=np.complex128).reshape(-1)
        self.coef = coef.view(np.float64).copy()
        self.struct = _Problem(int(prob.d), int(prob.n), int(prob.N), g,
                               self.P.ctypes.data_as(C.POINTER(C.c_double)),
                               self.modes.ctypes.data_as(C.POINTER(C.c_int)),
                               self.coef.ctypes.data_as(C.POINTER(C.c_double)),
                               None if self.coefs is None
                               else self.coefs.ctypes.data_as(C.POINTER(C.c_double)))
        self.D = int(prob.N) ** int(prob.n)

    @property
    def ref(self):
        return C.byref(self.struct)


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _cvec(v, D) -> np.ndarray:
    a = np.ascontiguousarray(v, dtype=np.complex128).reshape(-1)
    if a.shape[0] != D:
        raise ValueError(f"vector has {a.shape[0]} entries, expected {D}")
    return a


def index(n: int, N: int, k) -> int:
    """Tensor-to-vector conversion C(k)."""
    arr = (C.c_int * n)(*[int(x) for x in k])
    return int(_load().qo_index(n, N, arr))


def multi_index(n: int, N: int, i: int) -> tuple:
    """Inverse conversion C^{-1}(i) -> signed k in K_N^n."""
    arr = (C.c_int * n)()
    _load().qo_multi_index(n, N, int(i), arr)
    return tuple(int(x) for x in arr)


def rep(N: int, x: int) -> int:
    return int(_load().qo_rep(N, int(x)))


def matvec(prob, u) -> np.ndarray:
    """y = Q u (row and column of the zero frequency excluded)."""
    b = _Bound(prob)
    u = _cvec(u, b.D)
    y = np.empty(b.D, dtype=np.complex128)
    _load().qo_matvec(b.ref, _dptr(u.view(np.float64)), _dptr(y.view(np.float64)))
    return y


def matvec_rows(prob, u, rows) -> np.ndarray:
    """(Q u) at the given storage indices only (for vectors too large for a
    full CPU product)."""
    b = _Bound(prob)
    u = _cvec(u, b.D)
    rows = np.ascontiguousarray(rows, dtype=np.int64).reshape(-1)
    if rows.size and (rows.min() < 0 or rows.max() >= b.D):
        raise ValueError("row index out of range")
    y = np.empty(rows.size, dtype=np.complex128)
    _load().qo_matvec_rows(b.ref, _dptr(u.view(np.float64)), int(rows.size),
                           rows.ctypes.data_as(C.POINTER(C.c_long)), _dptr(y.view(np.float64)))
    return y


def precond(prob, kind: int = 0) -> np.ndarray:
    """Diagonal M: kind 0 = Frobenius-optimal (the paper's), 1 = Jacobi."""
    b = _Bound(prob)
    M = np.empty(b.D, dtype=np.float64)
    _load().qo_precond(b.ref, int(kind), _dptr(M))
    return M


def pcg(prob, F, tol: float = 1e-12, maxit: int = 10000, kind: int = 0):
    """C-PCG from U_0 = 0.  Returns (U, status, iters, relres)."""
    b = _Bound(prob)
    F = _cvec(F, b.D).copy()
    U = np.empty(b.D, dtype=np.complex128)
    it = C.c_int(0)
    rr = C.c_double(0.0)
    st = _load().qo_pcg(b.ref, int(kind), _dptr(F.view(np.float64)), _dptr(U.view(np.float64)),
                        float(tol), int(maxit), C.byref(it), C.byref(rr))
    return U, int(st), int(it.value), float(rr.value)


def pcg_lanczos(prob, F, tol: float = 1e-12, maxit: int = 10000, kind: int = 0):
    """C-PCG as pcg(), also returning the scalars of every step: alpha[j] and
    the beta[j] that follows step j (beta has iters - 1 entries)."""
    b = _Bound(prob)
    F = _cvec(F, b.D).copy()
    U = np.empty(b.D, dtype=np.complex128)
    ab = np.zeros(2 * max(1, int(maxit)), dtype=np.float64)
    it = C.c_int(0)
    rr = C.c_double(0.0)
    st = _load().qo_pcg_ex(b.ref, int(kind), _dptr(F.view(np.float64)), _dptr(U.view(np.float64)),
                           float(tol), int(maxit), C.byref(it), C.byref(rr), _dptr(ab))
    m = int(it.value)
    return U, int(st), m, float(rr.value), ab[0:2 * m:2].copy(), ab[1:2 * m - 1:2].copy()


def lanczos_kappa(alpha, beta) -> float:
    """Condition estimate of the preconditioned operator M^(1/2) Q M^(1/2)
    from C-PCG's scalars: PCG is the Lanczos process in disguise, whose
    tridiagonal matrix has diagonal 1/alpha_j + beta_(j-1)/alpha_(j-1) and
    off-diagonal sqrt(beta_j)/alpha_j; the ratio of its extreme eigenvalues
    (a library eigensolver) approaches the operator's from below."""
    from scipy.linalg import eigvalsh_tridiagonal
    alpha = np.asarray(alpha, dtype=np.float64)
    beta = np.asarray(beta, dtype=np.float64)[: max(0, alpha.size - 1)]
    if alpha.size == 0:
        return 0.0
    diag = 1.0 / alpha
    diag[1:] += beta / alpha[:-1]
    off = np.sqrt(beta) / alpha[:-1]
    ev = eigvalsh_tridiagonal(diag, off) if alpha.size > 1 else diag
    return float(ev.max() / ev.min())


def dft_rows(n: int, N: int, x, rows=None, inverse: bool = False) -> np.ndarray:
    """Discrete Fourier-Bohr transform on T_N^n (Sec. 2.3) at the given storage
    indices (all D when rows is None), straight from the definition:
    forward (1/D) sum_j x_j exp(-i k.y_j), inverse sum_k x_k exp(i k.y_j)."""
    D = int(N) ** int(n)
    x = _cvec(x, D)
    rows = np.arange(D, dtype=np.int64) if rows is None else \
        np.ascontiguousarray(rows, dtype=np.int64).reshape(-1)
    if rows.size and (rows.min() < 0 or rows.max() >= D):
        raise ValueError("row index out of range")
    out = np.empty(rows.size, dtype=np.complex128)
    _load().qo_dft_rows(int(n), int(N), 1 if inverse else 0, _dptr(x.view(np.float64)),
                        int(rows.size), rows.ctypes.data_as(C.POINTER(C.c_long)),
                        _dptr(out.view(np.float64)))
    return out


def corrector_rhs(prob, j: int) -> np.ndarray:
    b = _Bound(prob)
    F = np.empty(b.D, dtype=np.complex128)
    _load().qo_corrector_rhs(b.ref, int(j), _dptr(F.view(np.float64)))
    return F


def astar_flux(prob, chis) -> tuple:
    """(A*, imaginary parts) in the flux form from the d correctors."""
    b = _Bound(prob)
    d = prob.d
    A = np.zeros((d, d))
    Ai = np.zeros((d, d))
    im = C.c_double(0.0)
    cs = [_cvec(c, b.D) for c in chis]
    for i in range(d):
        for j in range(d):
            A[i, j] = _load().qo_astar_flux(b.ref, i, j, _dptr(cs[j].view(np.float64)), C.byref(im))
            Ai[i, j] = im.value
    return A, Ai


def astar_energy(prob, chis) -> tuple:
    b = _Bound(prob)
    d = prob.d
    A = np.zeros((d, d))
    Ai = np.zeros((d, d))
    im = C.c_double(0.0)
    cs = [_cvec(c, b.D) for c in chis]
    for i in range(d):
        for j in range(d):
            A[i, j] = _load().qo_astar_energy(b.ref, i, j, _dptr(cs[i].view(np.float64)),
                                              _dptr(cs[j].view(np.float64)), C.byref(im))
            Ai[i, j] = im.value
    return A, Ai


def coef_extrema(prob) -> tuple:
    b = _Bound(prob)
    lo = C.c_double(0.0)
    hi = C.c_double(0.0)
    _load().qo_coef_extrema(b.ref, C.byref(lo), C.byref(hi))
    return float(lo.value), float(hi.value)


def homogenize(prob, tol: float = 1e-12, maxit: int = 10000, kind: int = 0):
    """Solve the d corrector problems and evaluate A* (flux and energy forms)."""
    chis, infos = [], []
    for j in range(prob.d):
        F = corrector_rhs(prob, j)
        U, st, it, rr = pcg(prob, F, tol=tol, maxit=maxit, kind=kind)
        chis.append(U)
        infos.append(SimpleNamespace(status=st, iters=it, relres=rr))
    A_flux, A_flux_im = astar_flux(prob, chis)
    A_energy, _ = astar_energy(prob, chis)
    return SimpleNamespace(chi=chis, infos=infos, A=A_flux, A_imag=A_flux_im,
                           A_energy=A_energy)


def set_threads(n: int) -> None:
    """Set the OpenMP thread count of the oracle's routines (timing only)."""
    _load().qo_set_threads(int(n))


def max_threads() -> int:
    """The OpenMP thread count the oracle's routines use."""
    return int(_load().qo_max_threads())
