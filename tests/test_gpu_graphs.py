"""Batches of PCG iterations replayed as HIP graphs (through the C ABI).

Graph replays must give exactly what direct launches give: the kernels, their
arguments and the fixed-order reductions are the same, so FP64 and FP32-IR
solves are compared bitwise.  Every cached graph is replayed several times
with unrelated eager work and synchronisations between the replays.
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


def dev(x: np.ndarray):
    return torch.from_numpy(np.ascontiguousarray(x)).to(device="cuda", dtype=torch.complex128)


@pytest.mark.parametrize("prec", ["fp64", "fp32ir"])
def test_graph_replays_equal_direct_launches(prec):
    prob = W.eightfold_random(12, 2)
    say("graphs vs direct", prec, prob.N)
    F = dev(W.random_vector(prob.D, seed=8))
    direct = qp.Problem(prob, precision=prec, graphs=False)
    ref, iref = direct.solve_d(F, tol=1e-12)
    ref = ref.clone()
    gp = qp.Problem(prob, precision=prec)
    out = torch.empty_like(ref)
    for rep in range(4):
        out.fill_(7.0)
        u, info = gp.solve_d(F, out=out, tol=1e-12)
        assert info.iters == iref.iters and info.outer_iters == iref.outer_iters
        assert torch.equal(u, ref), f"replay {rep} differs"
        # unrelated eager work and a synchronisation between replays
        x = torch.randn(1 << 16, device="cuda")
        assert float((x * x).sum()) > 0
        torch.cuda.synchronize()
    Fh = F.cpu().numpy()
    uo, *_ = oracle.pcg(prob, Fh, tol=1e-12)
    assert np.linalg.norm(ref.cpu().numpy() - uo) <= 1e-9 * np.linalg.norm(uo)
    direct.close()
    gp.close()


# The FP64 tests below keep small problems on the multi-launch loop
# (small_dim 0): its batches are what they test.
def test_graph_cache_follows_the_output_buffer():
    prob = W.eightfold(8)
    F = dev(W.random_vector(prob.D, seed=3))
    gp = qp.Problem(prob, small_dim=0)
    outs = [torch.empty(prob.D, dtype=torch.complex128, device="cuda") for _ in range(3)]
    res = []
    for rep in range(2):
        for o in outs:
            o.zero_()
            u, _ = gp.solve_d(F, out=o, tol=1e-12)
            res.append(u.clone())
    for r in res[1:]:
        assert torch.equal(r, res[0])
    gp.close()


def test_partial_last_batch_stops_at_the_limit():
    prob = W.eightfold(8)
    F = W.random_vector(prob.D, seed=1)
    ref, st, it, rr = oracle.pcg(prob, F, tol=1e-14, maxit=11)
    for graphs in (True, False):
        gp = qp.Problem(prob, maxit=11, graphs=graphs, small_dim=0)
        u, info = gp.solve_d(dev(F), tol=1e-14, check=False)
        assert info.status == qp.QP_ENOCONV and info.iters == 11
        assert np.linalg.norm(u.cpu().numpy() - ref) <= 1e-12 * np.linalg.norm(ref)
        gp.close()


def test_batch_length_does_not_change_fp64_iterates():
    prob = W.eightfold_random(8, 1)
    F = dev(W.random_vector(prob.D, seed=2))
    a = qp.Problem(prob, small_dim=0)
    b = qp.Problem(prob, poll_every=5, small_dim=0)  # rounded up to 6
    ua, ia = a.solve_d(F, tol=1e-12)
    ub, ib = b.solve_d(F, tol=1e-12)
    assert ia.iters == ib.iters and torch.equal(ua, ub)
    a.close()
    b.close()


def test_profiled_solves_time_every_product():
    # profiling launches batches directly whatever `graphs` says, so both
    # settings must time the same launches
    prob = W.eightfold_random(16, 4)
    counts = {}
    for graphs in (True, False):
        gp = qp.Problem(prob, precision="fp32ir", profile=True, graphs=graphs)
        r = gp.homogenized(tol=1e-12)
        i0 = r.infos[0]  # the correctors are solved together: shared launch totals
        iters = sum(i.iters for i in r.infos)
        say("profiled", graphs, i0.matvec32_launches, i0.matvec32_rhs, i0.matvec_launches,
            i0.matvec32_ms, iters)
        assert i0.matvec32_rhs == iters
        assert i0.matvec_rhs >= sum(i.outer_iters for i in r.infos)
        assert i0.matvec32_ms > 0
        counts[graphs] = (i0.matvec32_launches, i0.matvec32_rhs, i0.matvec_launches)
        gp.close()
    assert counts[True] == counts[False]


@pytest.mark.parametrize("prec", ["fp64", "fp32ir"])
@pytest.mark.parametrize("prob", [W.one_d_two_mode(128, 6.0, 2 * np.pi), W.eightfold_diagonal(12, 1),
                                  W.paper_four_mode_2d(6)],
                         ids=["line_kernel_1d_N128", "diagonal_N12", "paper2d_complex_N6"])
def test_profiled_launches_time_and_match_unprofiled(prob, prec):
    """A profiled product launch records its own event pair; the line kernel,
    the diagonal-coefficient and complex-coefficient plane kernels all take
    that launch path.  The timed solve gives bitwise the same A* as the
    unprofiled one on the same path (small_dim 0: a profiled FP64 solve never
    takes the one-launch loop of small problems)."""
    plain = qp.Problem(prob, precision=prec, small_dim=0)
    timed = qp.Problem(prob, precision=prec, profile=True)
    ra = plain.homogenized(tol=1e-12)
    rb = timed.homogenized(tol=1e-12)
    i0 = rb.infos[0]
    n64, ms64 = i0.matvec_launches, i0.matvec_ms
    n32, ms32 = i0.matvec32_launches, i0.matvec32_ms
    say("profiled", prec, n64, ms64, n32, ms32)
    assert np.array_equal(ra.A, rb.A)
    assert [i.iters for i in ra.infos] == [i.iters for i in rb.infos]
    if prec == "fp64":
        assert n64 > 0 and ms64 > 0 and n32 == 0
    else:
        assert n32 > 0 and ms32 > 0 and n64 > 0 and ms64 > 0
    assert 0 < ms64 / max(n64, 1) < 100 and (n32 == 0 or 0 < ms32 / n32 < 100)
    plain.close()
    timed.close()


@pytest.mark.parametrize("prob", [W.eightfold_random(12, 2), W.icosahedral(6), W.paper_four_mode_2d(6)],
                         ids=["eightfold_random_N12", "icosa_N6", "paper2d_complex_N6"])
def test_multi_rhs_fp64_equals_separate_solves(prob):
    K = prob.d
    F = torch.stack([dev(W.random_vector(prob.D, seed=20 + r)) for r in range(K)])
    gp = qp.Problem(prob)
    U, infos = gp.solve_multi_d(F, tol=1e-12)
    for r in range(K):
        u, info = gp.solve_d(F[r].contiguous(), tol=1e-12)
        assert info.iters == infos[r].iters
        err = float((U[r] - u).abs().max() / u.abs().max())
        say("multi vs single", prob.name, r, info.iters, err)
        assert err <= 1e-14
        ref, *_ = oracle.pcg(prob, F[r].cpu().numpy(), tol=1e-12)
        assert np.linalg.norm(U[r].cpu().numpy() - ref) <= 1e-9 * np.linalg.norm(ref)
    gp.close()


def test_multi_rhs_fp32ir_matches_oracle_and_counts_products():
    prob = W.eightfold_random(16, 3)
    K = 2
    F = torch.stack([dev(W.random_vector(prob.D, seed=40 + r)) for r in range(K)])
    gp = qp.Problem(prob, precision="fp32ir", profile=True)
    U, infos = gp.solve_multi_d(F, tol=1e-12)
    for r in range(K):
        ref, *_ = oracle.pcg(prob, F[r].cpu().numpy(), tol=1e-12)
        assert np.linalg.norm(U[r].cpu().numpy() - ref) <= 1e-9 * np.linalg.norm(ref)
    # one launch serves every unfinished right-hand side
    i0 = infos[0]
    assert all(i.matvec32_launches == i0.matvec32_launches for i in infos)
    assert i0.matvec32_rhs == sum(i.iters for i in infos)
    assert max(i.iters for i in infos) <= i0.matvec32_launches <= sum(i.iters for i in infos)
    gp.close()


def test_multi_rhs_rejects_bad_counts():
    prob = W.eightfold(6)
    gp = qp.Problem(prob)
    F = torch.zeros((3, prob.D), dtype=torch.complex128, device="cuda")
    with pytest.raises(qp.QPError):
        gp.solve_multi_d(F, tol=1e-12)  # K = 3 > d = 2
    gp.close()


@pytest.mark.parametrize("K", [1, 2])
def test_fp32ir_iteration_limit_folds_the_float_increment(K):
    # the limit stops the float iterations mid-way; the forced final
    # replacement must fold them into X and report X's true residual
    prob = W.eightfold_random(12, 6)
    F = torch.stack([dev(W.random_vector(prob.D, seed=60 + r)) for r in range(K)])
    gp = qp.Problem(prob, precision="fp32ir", maxit=5)
    U, infos = gp.solve_multi_d(F, tol=1e-12, check=False)
    for r in range(K):
        info = infos[r]
        assert info.status == qp.QP_ENOCONV and info.iters == 5
        Fh = F[r].cpu().numpy().copy()
        Fh[0] = 0
        res = Fh - oracle.matvec(prob, U[r].cpu().numpy())
        rel = np.linalg.norm(res) / np.linalg.norm(Fh)
        say("ir maxit", K, r, info.rel_resid, rel)
        assert rel < 0.9  # progress was kept
        assert abs(info.rel_resid - rel) <= 1e-6 * rel
    gp.close()
