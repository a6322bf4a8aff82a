"""Host-side checks of the C ABI: the library loads, exports every declared
symbol, and rejects invalid problems on the host before any device call."""
from __future__ import annotations

import os
import re

import numpy as np
import pytest

from paper_2404_06841_amd import qp
from paper_2404_06841_amd import workloads as W

HEADER = os.path.join(os.path.dirname(os.path.dirname(__file__)), "include", "qp.h")


def declared_symbols():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(qp_[a-z0-9_]+)\s*\(", text)))


def test_header_and_binding_agree():
    assert declared_symbols() == sorted(qp.EXPORTED)


def test_library_exports_every_declared_symbol():
    L = qp.lib()
    for name in declared_symbols():
        assert hasattr(L, name), name


def test_default_options_and_strings():
    o = qp.qp_default_options()
    assert o.precision == qp.QP_PREC_FP64 and o.precond == qp.QP_PRECOND_PAPER
    assert o.maxit == 10000 and o.inner_tol == pytest.approx(1e-5) and o.poll_every == 0
    assert o.graphs == 1
    assert o.gather64 == 0
    assert o.small_dim == 2048
    assert o.stream is None and o.workspace is None
    for s in range(0, -8, -1):
        assert qp.qp_strerror(s)
    assert qp.qp_strerror(-99) == "unknown status"


def test_workspace_bytes():
    a = qp.qp_workspace_bytes(2, 4, 16, 9)
    b = qp.qp_workspace_bytes(2, 4, 32, 17)
    assert a > 0 and b > 15 * a  # grows with D = N^n
    assert b >= (16 * 5 + 12 + 32 + 32) * 32 ** 4
    assert qp.qp_workspace_bytes(2, 4, 1, 9) == 0
    assert qp.qp_workspace_bytes(1, 9, 4, 3) == 0
    assert qp.qp_workspace_bytes(1, 8, 16, 3) == 0  # 16^8 = 2^32 overflows int32 indexing


def _create(prob, **over):
    args = dict(d=prob.d, n=prob.n, P=prob.P, modes=prob.modes, coef=prob.coef, N=prob.N)
    args.update(over)
    return qp.qp_create(args["d"], args["n"], args["P"], args["modes"], args["coef"], args["N"])


BASE = W.eightfold(8)


@pytest.mark.parametrize("case", [
    "d_gt_n", "d_zero", "n_too_big", "N_small", "alias", "dup", "no_mean", "neg_mean",
    "not_hermitian", "no_partner", "nan_P", "inf_coef", "too_many_modes", "overflow",
])
def test_invalid_problems_rejected_on_host(case):
    p = BASE
    over = {}
    if case == "d_gt_n":
        over = dict(d=5, n=4, P=np.zeros((5, 4)))
    elif case == "d_zero":
        over = dict(d=0)
    elif case == "n_too_big":
        over = dict(n=9, modes=np.zeros((1, 9), np.int32), coef=np.array([1.0]), P=np.ones((2, 9)))
    elif case == "N_small":
        over = dict(N=1)
    elif case == "alias":
        over = dict(N=2)  # |m| = 1 >= N/2
    elif case == "dup":
        over = dict(modes=np.vstack([p.modes, p.modes[:1]]), coef=np.concatenate([p.coef, p.coef[:1]]))
    elif case == "no_mean":
        keep = [i for i, m in enumerate(p.modes) if any(m)]
        over = dict(modes=p.modes[keep], coef=p.coef[keep])
    elif case == "neg_mean":
        c = p.coef.copy()
        c[[i for i, m in enumerate(p.modes) if not any(m)][0]] = -3.0
        over = dict(coef=c)
    elif case == "not_hermitian":
        c = p.coef.copy()
        c[[i for i, m in enumerate(p.modes) if any(m)][0]] += 0.1j
        over = dict(coef=c)
    elif case == "no_partner":
        keep = [i for i, m in enumerate(p.modes) if tuple(m) != (0, 0, 0, -1)]
        over = dict(modes=p.modes[keep], coef=p.coef[keep])
    elif case == "nan_P":
        P = p.P.copy()
        P[0, 1] = np.nan
        over = dict(P=P)
    elif case == "inf_coef":
        c = p.coef.copy()
        c[0] = np.inf
        over = dict(coef=c)
    elif case == "too_many_modes":
        m = np.zeros((65, 4), np.int32)
        over = dict(modes=m, coef=np.ones(65, complex))
    elif case == "overflow":
        over = dict(N=300, n=4)
    st, h = _create(p, **over)
    assert st == qp.QP_EINVAL and h is None, (st, qp.qp_last_error())
    assert qp.qp_last_error()


def test_invalid_options_rejected_on_host():
    o = qp.qp_default_options()
    o.small_dim = -1
    st, h = qp.qp_create(BASE.d, BASE.n, BASE.P, BASE.modes, BASE.coef, BASE.N, o)
    assert st == qp.QP_EINVAL and h is None and "small_dim" in qp.qp_last_error()


def test_valid_problem_without_device_reports_device_error():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    st, h = _create(BASE)
    assert st == qp.QP_EDEVICE and h is None


DIAG = W.paper_homogenization(6)


@pytest.mark.parametrize("case", ["null_coefs", "row1_not_hermitian", "row1_neg_mean",
                                  "row0_zero_mean", "alias", "d_zero"])
def test_invalid_diagonal_problems_rejected_on_host(case):
    p = DIAG
    coefs = p.coefs.copy()
    N, d = p.N, p.d
    zero = [i for i, m in enumerate(p.modes) if not any(m)][0]
    other = [i for i, m in enumerate(p.modes) if any(m) and coefs[1, i] != 0][0]
    if case == "null_coefs":
        h = qp.C.c_void_p()
        P = np.ascontiguousarray(p.P, dtype=np.float64).reshape(-1)
        modes = np.ascontiguousarray(p.modes, dtype=np.int32).reshape(-1)
        st = qp.lib().qp_create_diag(qp.C.byref(h), d, p.n, qp._dptr(P), p.g,
                                     modes.ctypes.data_as(qp.C.POINTER(qp.C.c_int32)), None, N, None)
        assert st == qp.QP_EINVAL and qp.qp_last_error()
        return
    if case == "row1_not_hermitian":
        coefs[1, other] += 0.1j
    elif case == "row1_neg_mean":
        coefs[1, zero] = -1.0
    elif case == "row0_zero_mean":
        coefs[0, zero] = 0.0
    elif case == "alias":
        N = 4  # beta has |m_t| = 2 = N/2
    elif case == "d_zero":
        d = 0
    st, h = qp.qp_create_diag(d, p.n, p.P, p.modes, coefs if d else coefs[:1], N)
    assert st == qp.QP_EINVAL and h is None, (case, st, qp.qp_last_error())
    assert qp.qp_last_error()


def test_valid_diagonal_problem_without_device_reports_device_error():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    st, h = qp.qp_create_diag(DIAG.d, DIAG.n, DIAG.P, DIAG.modes, DIAG.coefs, DIAG.N)
    assert st == qp.QP_EDEVICE and h is None


def test_server_and_batch_argument_checks_on_host():
    h = qp.C.c_void_p()
    assert qp.lib().qp_server_create(qp.C.byref(h), 0, None) == qp.QP_EINVAL
    srv = qp.Server(1 << 30)  # creating a server touches no device
    with pytest.raises(qp.QPError):
        srv.submit(W.eightfold(8), tol=-1.0)
    bad = W.eightfold(8)
    bad = W.Problem(bad.name, bad.d, bad.n, 2, bad.P, bad.modes, bad.coef)  # |m| >= N/2
    with pytest.raises(qp.QPError):
        srv.submit(bad, tol=1e-12)
    with pytest.raises(qp.QPError):
        srv.submit(W.icosahedral(16), tol=1e-12)  # needs more than the 1 GiB budget
    assert srv.pending() == 0 and srv.bytes() == 0
    srv.close()
    assert qp.lib().qp_homogenized_batch(None, 0, None, 1e-12, None) == qp.QP_EINVAL
    assert qp.lib().qp_homogenized_batch_mixed(None, 0, None, 1e-12, None, 1024) == qp.QP_EINVAL
    # the size limit is checked before any problem is read
    A = np.zeros(4)
    dummy = (qp.C.c_void_p * 1)(1)
    assert qp.lib().qp_homogenized_batch_mixed(dummy, 1, qp._dptr(A), 1e-12, None, -1) == qp.QP_EINVAL
    assert "group_max_dim" in qp.qp_last_error()


def test_coo_entry_count_without_problem():
    assert qp.lib().qp_coo_entries(None) == 0
    assert qp.lib().qp_coo_build_d(None, None, None, None) == qp.QP_EINVAL
