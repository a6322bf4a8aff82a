"""ctypes binding of libqp.so (the C ABI in include/qp.h).

Argument marshalling only: every step of the solver runs in the library's
gfx950 kernels.  Functions keep the C names; device arguments are torch CUDA
tensors (complex128 / complex64 / float64 / int32), host arguments are numpy
arrays.  PyTorch supplies device memory and the stream, nothing else.

Loading fails loudly when the library has not been built: there is no
fallback implementation.
"""
from __future__ import annotations

import ctypes as C
import os
from types import SimpleNamespace

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libqp.so")

QP_OK = 0
QP_EINVAL = -1
QP_ENOTELLIPTIC = -2
QP_ENOTSPD = -3
QP_ENOCONV = -4
QP_ENOMEM = -5
QP_EDEVICE = -6
QP_ENONFINITE = -7

QP_PREC_FP64 = 0
QP_PREC_FP32_IR = 1
QP_PRECOND_PAPER = 0
QP_PRECOND_JACOBI = 1
QP_FLAG_DEGENERATE = 1
QP_FLAG_F0_IGNORED = 2
QP_FLAG_INDEFINITE = 4

MAX_N, MAX_D, MAX_MODES = 8, 4, 64

#: every symbol include/qp.h declares
EXPORTED = (
    "qp_default_options", "qp_workspace_bytes", "qp_create", "qp_create_diag", "qp_destroy",
    "qp_dim",
    "qp_set_options", "qp_product_layout", "qp_set_product_layout", "qp_solve", "qp_solve_d", "qp_solve_multi_d", "qp_corrector",
    "qp_corrector_d",
    "qp_homogenized", "qp_homogenized_ex", "qp_homogenized_batch", "qp_homogenized_grouped",
    "qp_homogenized_grouped_noalloc", "qp_homogenized_batch_mixed", "qp_server_create",
    "qp_server_submit", "qp_server_progress", "qp_server_pending", "qp_server_bytes",
    "qp_server_destroy", "qp_coo_entries", "qp_coo_build_d", "qp_coo_matvec_d", "qp_dft_d",
    "qp_modes_from_spectrum", "qp_matvec_d", "qp_matvec32_d", "qp_matvec_half_d", "qp_last_product_ms", "qp_precond_d",
    "qp_corrector_rhs_d", "qp_multi_index_d", "qp_astar_d", "qp_coef_extrema",
    "qp_synchronize", "qp_strerror", "qp_last_error",
)


class qp_options(C.Structure):
    _fields_ = [("precision", C.c_int), ("precond", C.c_int), ("maxit", C.c_int),
                ("inner_tol", C.c_double), ("poll_every", C.c_int),
                ("profile", C.c_int), ("stream", C.c_void_p), ("workspace", C.c_void_p),
                ("workspace_bytes", C.c_size_t), ("graphs", C.c_int),
                ("gather64", C.c_int), ("autotune", C.c_int), ("allow_indefinite", C.c_int),
                ("half_storage", C.c_int), ("small_dim", C.c_int)]


class qp_layout(C.Structure):
    _fields_ = [("item_tiles", C.c_int), ("workgroups", C.c_int), ("xcd_front", C.c_int),
                ("tuned", C.c_int), ("candidates", C.c_int), ("default_us", C.c_double),
                ("best_us", C.c_double), ("item_tiles64", C.c_int), ("workgroups64", C.c_int),
                ("xcd_front64", C.c_int), ("default64_us", C.c_double), ("best64_us", C.c_double)]

    def as_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_}


class qp_solve_info(C.Structure):
    _fields_ = [("status", C.c_int), ("iters", C.c_int), ("outer_iters", C.c_int),
                ("flags", C.c_int), ("rel_resid", C.c_double), ("seconds", C.c_double),
                ("matvec_launches", C.c_int), ("matvec_ms", C.c_double),
                ("matvec32_launches", C.c_int), ("matvec32_ms", C.c_double),
                ("matvec_rhs", C.c_int), ("matvec32_rhs", C.c_int),
                ("kappa_est", C.c_double), ("bytes_moved", C.c_double)]

    def as_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_}


class QPError(RuntimeError):
    def __init__(self, status: int, where: str, message: str):
        super().__init__(f"{where}: {message} (status {status})")
        self.status = status


_lib = None


def lib():
    """Load libqp.so; raise if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with "
                          "`python -m paper_2404_06841_amd.build` (no fallback exists)")
    L = C.CDLL(LIB_PATH)
    vp, dp, ip = C.c_void_p, C.POINTER(C.c_double), C.POINTER(C.c_int32)
    sig = {
        "qp_default_options": (None, [C.POINTER(qp_options)]),
        "qp_workspace_bytes": (C.c_size_t, [C.c_int, C.c_int, C.c_int, C.c_int]),
        "qp_create": (C.c_int, [C.POINTER(vp), C.c_int, C.c_int, dp, C.c_int, ip, dp, C.c_int,
                                C.POINTER(qp_options)]),
        "qp_create_diag": (C.c_int, [C.POINTER(vp), C.c_int, C.c_int, dp, C.c_int, ip, dp,
                                     C.c_int, C.POINTER(qp_options)]),
        "qp_destroy": (None, [vp]),
        "qp_dim": (C.c_int64, [vp]),
        "qp_set_options": (C.c_int, [vp, C.POINTER(qp_options)]),
        "qp_solve": (C.c_int, [vp, dp, dp, C.c_double, C.POINTER(qp_solve_info)]),
        "qp_solve_d": (C.c_int, [vp, vp, vp, C.c_double, C.POINTER(qp_solve_info)]),
        "qp_solve_multi_d": (C.c_int, [vp, C.c_int, vp, vp, C.c_double, C.POINTER(qp_solve_info)]),
        "qp_corrector": (C.c_int, [vp, C.c_int, dp, C.c_double, C.POINTER(qp_solve_info)]),
        "qp_corrector_d": (C.c_int, [vp, C.c_int, vp, C.c_double, C.POINTER(qp_solve_info)]),
        "qp_homogenized": (C.c_int, [vp, dp, C.c_double, C.POINTER(qp_solve_info)]),
        "qp_homogenized_ex": (C.c_int, [vp, dp, dp, C.c_double, C.POINTER(qp_solve_info)]),
        "qp_homogenized_batch": (C.c_int, [C.POINTER(vp), C.c_int, dp, C.c_double,
                                           C.POINTER(qp_solve_info)]),
        "qp_homogenized_grouped": (C.c_int, [C.POINTER(vp), C.c_int, dp, C.c_double,
                                           C.POINTER(qp_solve_info)]),
        "qp_homogenized_grouped_noalloc": (C.c_int, [C.POINTER(vp), C.c_int, dp, C.c_double,
                                                   C.POINTER(qp_solve_info)]),
        "qp_homogenized_batch_mixed": (C.c_int, [C.POINTER(vp), C.c_int, dp, C.c_double,
                                               C.POINTER(qp_solve_info), C.c_int64]),
        "qp_server_create": (C.c_int, [C.POINTER(vp), C.c_size_t, C.POINTER(qp_options)]),
        "qp_server_submit": (C.c_int, [vp, C.c_int, C.c_int, dp, C.c_int, ip, dp, dp, C.c_int,
                                       C.c_double, dp, C.POINTER(qp_solve_info),
                                       C.POINTER(C.c_int64)]),
        "qp_server_progress": (C.c_int, [vp, C.c_int, C.POINTER(C.c_int64), C.POINTER(C.c_int),
                                         C.c_int, C.POINTER(C.c_int)]),
        "qp_server_pending": (C.c_int, [vp]),
        "qp_server_bytes": (C.c_size_t, [vp]),
        "qp_server_destroy": (None, [vp]),
        "qp_coo_entries": (C.c_int64, [vp]),
        "qp_dft_d": (C.c_int, [C.c_int, C.c_int, vp, vp, C.c_int, vp]),
        "qp_modes_from_spectrum": (C.c_int, [C.c_int, C.c_int, dp, C.c_double, C.c_int, ip, dp,
                                             C.POINTER(C.c_int)]),
        "qp_coo_build_d": (C.c_int, [vp, vp, vp, vp]),
        "qp_coo_matvec_d": (C.c_int, [vp, vp, vp, vp, vp]),
        "qp_matvec_d": (C.c_int, [vp, vp, vp]),
        "qp_matvec32_d": (C.c_int, [vp, vp, vp]),
        "qp_last_product_ms": (C.c_int, [vp, dp]),
        "qp_matvec_half_d": (C.c_int, [vp, vp, vp]),
        "qp_precond_d": (C.c_int, [vp, vp]),
        "qp_corrector_rhs_d": (C.c_int, [vp, C.c_int, vp]),
        "qp_multi_index_d": (C.c_int, [vp, vp]),
        "qp_astar_d": (C.c_int, [vp, vp, dp]),
        "qp_coef_extrema": (C.c_int, [vp, dp, dp]),
        "qp_product_layout": (C.c_int, [vp, C.POINTER(qp_layout)]),
        "qp_set_product_layout": (C.c_int, [vp, C.POINTER(qp_layout)]),
        "qp_synchronize": (C.c_int, [vp]),
        "qp_strerror": (C.c_char_p, [C.c_int]),
        "qp_last_error": (C.c_char_p, []),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L


def _check(status: int, where: str) -> int:
    if status != QP_OK:
        msg = lib().qp_last_error().decode() or lib().qp_strerror(status).decode()
        raise QPError(status, where, msg)
    return status


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _tensor_ptr(t, dtype=None, numel=None):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError("expected a CUDA tensor")
    if not t.is_contiguous():
        raise ValueError("tensor must be contiguous")
    if dtype is not None and t.dtype != dtype:
        raise TypeError(f"expected {dtype}, got {t.dtype}")
    if numel is not None and t.numel() != numel:
        raise ValueError(f"expected {numel} elements, got {t.numel()}")
    return C.c_void_p(t.data_ptr())


# --------------------------------------------------------------------------
# Thin wrappers with the C names
# --------------------------------------------------------------------------

def qp_default_options() -> qp_options:
    o = qp_options()
    lib().qp_default_options(C.byref(o))
    return o


def qp_workspace_bytes(d: int, n: int, N: int, g: int) -> int:
    return int(lib().qp_workspace_bytes(d, n, N, g))


def qp_create(d, n, P, modes, coef, N, opt: qp_options | None = None):
    """Returns (status, handle); handle is None on failure."""
    P = np.ascontiguousarray(P, dtype=np.float64).reshape(-1)
    modes = np.ascontiguousarray(modes, dtype=np.int32).reshape(-1)
    coef = np.ascontiguousarray(np.asarray(coef, dtype=np.complex128).reshape(-1)).view(np.float64)
    g = coef.shape[0] // 2
    h = C.c_void_p()
    st = lib().qp_create(C.byref(h), int(d), int(n), _dptr(P), int(g),
                         modes.ctypes.data_as(C.POINTER(C.c_int32)), _dptr(coef), int(N),
                         C.byref(opt) if opt is not None else None)
    return st, (h if st == QP_OK else None)


def qp_create_diag(d, n, P, modes, coefs, N, opt: qp_options | None = None):
    """Diagonal coefficient diag(a_1..a_d): coefs is d x g complex (row l = a_l's
    Ahat per mode).  Returns (status, handle); handle is None on failure."""
    P = np.ascontiguousarray(P, dtype=np.float64).reshape(-1)
    modes = np.ascontiguousarray(modes, dtype=np.int32).reshape(-1)
    g = modes.size // int(n) if int(n) > 0 else 0
    flat = np.ascontiguousarray(np.asarray(coefs, dtype=np.complex128).reshape(-1)).view(np.float64)
    h = C.c_void_p()
    st = lib().qp_create_diag(C.byref(h), int(d), int(n), _dptr(P), int(g),
                              modes.ctypes.data_as(C.POINTER(C.c_int32)), _dptr(flat), int(N),
                              C.byref(opt) if opt is not None else None)
    return st, (h if st == QP_OK else None)


def qp_last_error() -> str:
    return lib().qp_last_error().decode()


def qp_strerror(status: int) -> str:
    return lib().qp_strerror(int(status)).decode()


# --------------------------------------------------------------------------
# Convenience object
# --------------------------------------------------------------------------

class Problem:
    """One qp_problem with a torch-allocated workspace on the current stream.

    `prob` is any object with d, n, N, P, modes, coef (e.g. a workload); a
    non-None attribute `coefs` (d x g) makes it a diagonal coefficient."""

    def __init__(self, prob, precision: str = "fp64", precond: str = "paper",
                 maxit: int = 10000, inner_tol: float = 1e-5,
                 profile: bool = False, stream=None, poll_every: int = 0,
                 graphs: bool = True, gather64: bool = False, autotune: bool = False,
                 allow_indefinite: bool = False, half_storage: bool = False,
                 small_dim=None):
        import torch
        self.d, self.n, self.N = int(prob.d), int(prob.n), int(prob.N)
        self.Dgrid = self.N ** self.n
        # entries of every vector: the grid, or its Hermitian half
        self.D = (self.Dgrid + 1) // 2 if half_storage else self.Dgrid
        self.half = bool(half_storage)
        modes = np.asarray(prob.modes, dtype=np.int32).reshape(-1, self.n)
        self.g = modes.shape[0]
        opt = qp_default_options()
        opt.precision = QP_PREC_FP32_IR if precision == "fp32ir" else QP_PREC_FP64
        opt.precond = QP_PRECOND_JACOBI if precond == "jacobi" else QP_PRECOND_PAPER
        opt.maxit = int(maxit)
        opt.inner_tol = float(inner_tol)
        opt.profile = 1 if profile else 0
        opt.poll_every = int(poll_every)
        opt.graphs = 1 if graphs else 0
        opt.gather64 = 1 if gather64 else 0
        opt.autotune = 1 if autotune else 0
        opt.allow_indefinite = 1 if allow_indefinite else 0
        opt.half_storage = 1 if half_storage else 0
        if small_dim is not None:
            opt.small_dim = int(small_dim)
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        opt.stream = C.c_void_p(self.stream.cuda_stream)
        nbytes = qp_workspace_bytes(self.d, self.n, self.N, self.g)
        if nbytes <= 0:
            raise QPError(QP_EINVAL, "qp_workspace_bytes", "unsupported shape")
        # 256-byte aligned torch allocation
        self._ws = torch.empty(nbytes + 256, dtype=torch.uint8, device="cuda")
        base = self._ws.data_ptr()
        opt.workspace = C.c_void_p((base + 255) // 256 * 256)
        opt.workspace_bytes = nbytes
        self.opt = opt
        coefs = getattr(prob, "coefs", None)
        if coefs is not None:
            st, h = qp_create_diag(self.d, self.n, prob.P, modes, coefs, self.N, opt)
            _check(st, "qp_create_diag")
        else:
            st, h = qp_create(self.d, self.n, prob.P, modes, prob.coef, self.N, opt)
            _check(st, "qp_create")
        self.h = h

    def close(self):
        if getattr(self, "h", None) is not None:
            lib().qp_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- options
    def set_precision(self, precision: str):
        self.opt.precision = QP_PREC_FP32_IR if precision == "fp32ir" else QP_PREC_FP64
        _check(lib().qp_set_options(self.h, C.byref(self.opt)), "qp_set_options")

    def set_options(self, **kw):
        for k, v in kw.items():
            setattr(self.opt, k, v)
        _check(lib().qp_set_options(self.h, C.byref(self.opt)), "qp_set_options")

    # -- solves (device tensors)
    def solve_d(self, rhs, out=None, tol: float = 1e-12, check: bool = True):
        import torch
        if out is None:
            out = torch.empty(self.D, dtype=torch.complex128, device="cuda")
        info = qp_solve_info()
        st = lib().qp_solve_d(self.h, _tensor_ptr(rhs, torch.complex128, self.D),
                              _tensor_ptr(out, torch.complex128, self.D), float(tol), C.byref(info))
        if check:
            _check(st, "qp_solve_d")
        return out, info

    def solve_multi_d(self, rhs, out=None, tol: float = 1e-12, check: bool = True):
        """K solves at once: rhs is a (K, D) complex128 device tensor."""
        import torch
        K = int(rhs.shape[0])
        if out is None:
            out = torch.empty((K, self.D), dtype=torch.complex128, device="cuda")
        infos = (qp_solve_info * K)()
        st = lib().qp_solve_multi_d(self.h, K, _tensor_ptr(rhs, torch.complex128, K * self.D),
                                    _tensor_ptr(out, torch.complex128, K * self.D), float(tol),
                                    infos)
        if check:
            _check(st, "qp_solve_multi_d")
        return out, list(infos)

    def solve(self, rhs: np.ndarray, tol: float = 1e-12, check: bool = True):
        rhs = np.ascontiguousarray(rhs, dtype=np.complex128).reshape(-1)
        out = np.empty(self.D, dtype=np.complex128)
        info = qp_solve_info()
        st = lib().qp_solve(self.h, _dptr(rhs.view(np.float64)), _dptr(out.view(np.float64)),
                            float(tol), C.byref(info))
        if check:
            _check(st, "qp_solve")
        return out, info

    def corrector_d(self, j: int, out=None, tol: float = 1e-12, check: bool = True):
        import torch
        if out is None:
            out = torch.empty(self.D, dtype=torch.complex128, device="cuda")
        info = qp_solve_info()
        st = lib().qp_corrector_d(self.h, int(j), _tensor_ptr(out, torch.complex128, self.D),
                                  float(tol), C.byref(info))
        if check:
            _check(st, "qp_corrector_d")
        return out, info

    def homogenized(self, tol: float = 1e-12, energy: bool = True, check: bool = True):
        A = np.zeros(self.d * self.d)
        E = np.zeros(self.d * self.d)
        infos = (qp_solve_info * self.d)()
        st = lib().qp_homogenized_ex(self.h, _dptr(A), _dptr(E) if energy else None, float(tol),
                                     infos)
        if check:
            _check(st, "qp_homogenized_ex")
        return SimpleNamespace(A=A.reshape(self.d, self.d),
                               A_energy=E.reshape(self.d, self.d) if energy else None,
                               infos=[infos[j] for j in range(self.d)], status=st)

    # -- single steps
    def matvec_d(self, u, out=None):
        import torch
        if out is None:
            out = torch.empty(self.D, dtype=torch.complex128, device="cuda")
        _check(lib().qp_matvec_d(self.h, _tensor_ptr(u, torch.complex128, self.D),
                                 _tensor_ptr(out, torch.complex128, self.D)), "qp_matvec_d")
        return out

    def matvec32_d(self, u, out=None):
        import torch
        if out is None:
            out = torch.empty(self.D, dtype=torch.complex64, device="cuda")
        _check(lib().qp_matvec32_d(self.h, _tensor_ptr(u, torch.complex64, self.D),
                                   _tensor_ptr(out, torch.complex64, self.D)), "qp_matvec32_d")
        return out

    def last_product_ms(self) -> float:
        """Kernel time of the last matvec_d / matvec32_d call (profile option
        on; -1 otherwise), from the launch's own event pair."""
        ms = C.c_double()
        _check(lib().qp_last_product_ms(self.h, C.byref(ms)), "qp_last_product_ms")
        return ms.value

    def matvec_half_d(self, u, out=None):
        """y = Q u on Hermitian half storage: (D+1)//2 complex128 entries each
        (real coefficient, odd N; the layout of qp_matvec_half_d)."""
        import torch
        H = (self.Dgrid + 1) // 2
        if out is None:
            out = torch.empty(H, dtype=torch.complex128, device="cuda")
        _check(lib().qp_matvec_half_d(self.h, _tensor_ptr(u, torch.complex128, H),
                                      _tensor_ptr(out, torch.complex128, H)), "qp_matvec_half_d")
        return out

    def coo_build_d(self):
        """The compressed matrix of Alg. 1 as device tensors (rows, cols, vals)."""
        import torch
        n = int(lib().qp_coo_entries(self.h))
        rows = torch.empty(n, dtype=torch.int32, device="cuda")
        cols = torch.empty(n, dtype=torch.int32, device="cuda")
        vals = torch.empty(n, dtype=torch.complex128, device="cuda")
        _check(lib().qp_coo_build_d(self.h, _tensor_ptr(rows, torch.int32, n),
                                    _tensor_ptr(cols, torch.int32, n),
                                    _tensor_ptr(vals, torch.complex128, n)), "qp_coo_build_d")
        return rows, cols, vals

    def coo_matvec_d(self, coo, u, out=None):
        import torch
        _, cols, vals = coo
        if out is None:
            out = torch.empty(self.D, dtype=torch.complex128, device="cuda")
        _check(lib().qp_coo_matvec_d(self.h, _tensor_ptr(cols, torch.int32), _tensor_ptr(vals, torch.complex128),
                                     _tensor_ptr(u, torch.complex128, self.D),
                                     _tensor_ptr(out, torch.complex128, self.D)), "qp_coo_matvec_d")
        return out

    def precond_d(self):
        import torch
        out = torch.empty(self.D, dtype=torch.float64, device="cuda")
        _check(lib().qp_precond_d(self.h, _tensor_ptr(out, torch.float64, self.D)), "qp_precond_d")
        return out

    def corrector_rhs_d(self, j: int):
        import torch
        out = torch.empty(self.D, dtype=torch.complex128, device="cuda")
        _check(lib().qp_corrector_rhs_d(self.h, int(j), _tensor_ptr(out, torch.complex128, self.D)),
               "qp_corrector_rhs_d")
        return out

    def multi_index_d(self):
        import torch
        out = torch.empty(self.D * self.n, dtype=torch.int32, device="cuda")
        _check(lib().qp_multi_index_d(self.h, _tensor_ptr(out, torch.int32, self.D * self.n)),
               "qp_multi_index_d")
        return out.view(self.D, self.n)

    def astar_d(self, chis):
        import torch
        A = np.zeros(self.d * self.d)
        _check(lib().qp_astar_d(self.h, _tensor_ptr(chis, torch.complex128, self.d * self.D),
                                _dptr(A)), "qp_astar_d")
        return A.reshape(self.d, self.d)

    def layout(self) -> dict:
        """The stiffness product's work layout (qp_product_layout)."""
        out = qp_layout()
        _check(lib().qp_product_layout(self.h, C.byref(out)), "qp_product_layout")
        return out.as_dict()

    def set_layout(self, item_tiles: int, workgroups: int, xcd_front: int,
                   item_tiles64: int = 0, workgroups64: int = 0, xcd_front64: int = 0):
        """Set the stiffness product's work layouts (qp_set_product_layout);
        the FP64 launches take the float layout unless workgroups64 > 0."""
        L = qp_layout(item_tiles=int(item_tiles), workgroups=int(workgroups),
                      xcd_front=int(xcd_front), item_tiles64=int(item_tiles64),
                      workgroups64=int(workgroups64), xcd_front64=int(xcd_front64))
        _check(lib().qp_set_product_layout(self.h, C.byref(L)), "qp_set_product_layout")

    def coef_extrema(self):
        lo, hi = C.c_double(), C.c_double()
        _check(lib().qp_coef_extrema(self.h, C.byref(lo), C.byref(hi)), "qp_coef_extrema")
        return lo.value, hi.value

    def synchronize(self):
        _check(lib().qp_synchronize(self.h), "qp_synchronize")


# --------------------------------------------------------------------------
# Batches and serving
# --------------------------------------------------------------------------

def homogenized_batch(problems, tol: float = 1e-12, check: bool = True, grouped: bool = False,
                      noalloc: bool = False, group_max_dim: int = 0):
    """qp_homogenized_batch over Problem objects (each should own a distinct
    stream for the solves to overlap), or with grouped=True
    qp_homogenized_grouped (one launch per solver step for all of them), or
    with noalloc=True as well qp_homogenized_grouped_noalloc, or with
    group_max_dim > 0 qp_homogenized_batch_mixed (the problems with at most
    that many unknowns grouped, the others on their streams).
    Returns (list of d x d A*, list of per-problem info lists, status)."""
    count = len(problems)
    ds = [pr.d for pr in problems]
    A = np.zeros(sum(d * d for d in ds))
    infos = (qp_solve_info * sum(ds))()
    hs = (C.c_void_p * count)(*[pr.h for pr in problems])
    if group_max_dim and not grouped:
        name = "qp_homogenized_batch_mixed"
        st = lib().qp_homogenized_batch_mixed(hs, count, _dptr(A), float(tol), infos,
                                              int(group_max_dim))
    else:
        name = ("qp_homogenized_grouped_noalloc" if noalloc else "qp_homogenized_grouped") \
            if grouped else "qp_homogenized_batch"
        st = getattr(lib(), name)(hs, count, _dptr(A), float(tol), infos)
    if check:
        _check(st, name)
    outA, outI, ao, io = [], [], 0, 0
    for d in ds:
        outA.append(A[ao:ao + d * d].reshape(d, d).copy())
        outI.append([infos[io + j] for j in range(d)])
        ao += d * d
        io += d
    return outA, outI, st


class Server:
    """qp_server: homogenization requests over a cache of problems bounded by
    an HBM budget.  submit() returns a ticket; progress() returns the finished
    tickets; result(ticket) gives (A*, infos, status) once finished."""

    def __init__(self, hbm_budget: int, precision: str = "fp64", maxit: int = 10000,
                 inner_tol: float = 1e-5, autotune: bool = False):
        opt = qp_default_options()
        opt.autotune = 1 if autotune else 0
        opt.precision = QP_PREC_FP32_IR if precision == "fp32ir" else QP_PREC_FP64
        opt.maxit = int(maxit)
        opt.inner_tol = float(inner_tol)
        self.opt = opt
        h = C.c_void_p()
        _check(lib().qp_server_create(C.byref(h), int(hbm_budget), C.byref(opt)), "qp_server_create")
        self.h = h
        self._out = {}     # ticket -> (A buffer, infos buffer, d)
        self._status = {}  # finished ticket -> status

    def submit(self, prob, tol: float = 1e-12) -> int:
        d, n, N = int(prob.d), int(prob.n), int(prob.N)
        P = np.ascontiguousarray(prob.P, dtype=np.float64).reshape(-1)
        modes = np.ascontiguousarray(prob.modes, dtype=np.int32).reshape(-1)
        g = modes.size // n
        coefs = getattr(prob, "coefs", None)
        if coefs is not None:
            c = np.ascontiguousarray(np.asarray(coefs, dtype=np.complex128).reshape(-1)).view(np.float64)
            coef_p, coefs_p = None, _dptr(c)
        else:
            c = np.ascontiguousarray(np.asarray(prob.coef, dtype=np.complex128).reshape(-1)).view(np.float64)
            coef_p, coefs_p = _dptr(c), None
        A = np.zeros(d * d)
        infos = (qp_solve_info * d)()
        t = C.c_int64(0)
        st = lib().qp_server_submit(self.h, d, n, _dptr(P), g,
                                    modes.ctypes.data_as(C.POINTER(C.c_int32)), coef_p, coefs_p,
                                    N, float(tol), _dptr(A), infos, C.byref(t))
        _check(st, "qp_server_submit")
        self._out[t.value] = (A, infos, d)
        return t.value

    def progress(self, wait_us: int = 1000, max_done: int = 64):
        done = (C.c_int64 * max_done)()
        stat = (C.c_int * max_done)()
        nd = C.c_int(0)
        _check(lib().qp_server_progress(self.h, int(wait_us), done, stat, max_done, C.byref(nd)),
               "qp_server_progress")
        out = []
        for i in range(nd.value):
            self._status[done[i]] = stat[i]
            out.append(done[i])
        return out

    def result(self, ticket: int):
        A, infos, d = self._out[ticket]
        return A.reshape(d, d), [infos[j] for j in range(d)], self._status.get(ticket)

    def pending(self) -> int:
        return int(lib().qp_server_pending(self.h))

    def bytes(self) -> int:
        return int(lib().qp_server_bytes(self.h))

    def close(self):
        if getattr(self, "h", None) is not None:
            lib().qp_server_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def dft_d(x, n: int, N: int, inverse: bool = False, out=None):
    """qp_dft_d on a complex128 CUDA tensor of N^n entries (torch's current stream)."""
    import torch
    D = N ** n
    if out is None:
        out = torch.empty(D, dtype=torch.complex128, device="cuda")
    _check(lib().qp_dft_d(int(n), int(N), _tensor_ptr(x, torch.complex128, D),
                          _tensor_ptr(out, torch.complex128, D), 1 if inverse else 0,
                          C.c_void_p(torch.cuda.current_stream().cuda_stream)), "qp_dft_d")
    return out


def modes_from_spectrum(spec: np.ndarray, n: int, N: int, rel_tol: float = 1e-12,
                        max_modes: int = MAX_MODES):
    """qp_modes_from_spectrum: (modes (g x n int32), coef (g complex))."""
    sp = np.ascontiguousarray(np.asarray(spec, dtype=np.complex128).reshape(-1)).view(np.float64)
    modes = np.zeros(max_modes * n, dtype=np.int32)
    coef = np.zeros(2 * max_modes)
    g = C.c_int(0)
    _check(lib().qp_modes_from_spectrum(int(n), int(N), _dptr(sp), float(rel_tol), int(max_modes),
                                        modes.ctypes.data_as(C.POINTER(C.c_int32)), _dptr(coef),
                                        C.byref(g)), "qp_modes_from_spectrum")
    k = g.value
    return modes[:k * n].reshape(k, n).copy(), coef[:2 * k].view(np.complex128).copy()
