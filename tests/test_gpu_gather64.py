"""The stiffness product with 64-bit neighbour addresses (through the C ABI).

The default plane-tile gathers index records with 32-bit indices that the
address unit scales by the entry size in 32 bits, so vectors of 2^28 entries
or more switch to 64-bit addresses (one right-hand side per launch).  The
option gather64 forces that path at small sizes, where it must equal the
default path and the oracle; one case above the switch point (icosahedral
n=6, N=26: 308,915,776 entries, 4.9 GB per FP64 vector) is checked at sampled
rows, most of them beyond entry 2^28, against the oracle evaluated row by row.
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


def dev(x: np.ndarray, dtype=torch.complex128):
    return torch.from_numpy(np.ascontiguousarray(x)).to(device="cuda", dtype=dtype)


CASES = {
    "eightfold_random_N12": lambda: W.eightfold_random(12, 2),
    "eightfold_random_N5": lambda: W.eightfold_random(5, 7),
    "icosa_N6": lambda: W.icosahedral(6),
    "paper2d_complex_N6": lambda: W.paper_four_mode_2d(6),
}


@pytest.mark.parametrize("name", sorted(CASES))
def test_gather64_products_equal_default_path(name):
    prob = CASES[name]()
    say("[case] gather64 products", name, prob.D, prob.g)
    a = qp.Problem(prob)
    b = qp.Problem(prob, gather64=True)
    u = W.random_vector(prob.D, seed=71)
    ya = a.matvec_d(dev(u))
    yb = b.matvec_d(dev(u))
    assert torch.equal(ya, yb)
    ref = oracle.matvec(prob, u)
    assert np.abs(yb.cpu().numpy() - ref).max() <= 1e-13 * np.abs(ref).max()
    u32 = dev(u.astype(np.complex64), torch.complex64)
    za = a.matvec32_d(u32)
    zb = b.matvec32_d(u32)
    assert torch.equal(za, zb)
    assert np.abs(zb.cpu().numpy() - ref).max() <= 2e-5 * np.abs(ref).max()
    a.close()
    b.close()


@pytest.mark.parametrize("prec", ["fp64", "fp32ir"])
@pytest.mark.parametrize("name", ["eightfold_random_N12", "icosa_N6"])
def test_gather64_homogenized_matches_oracle(name, prec):
    prob = CASES[name]()
    say("[case] gather64 homogenized", name, prec)
    ref = oracle.homogenize(prob, tol=1e-12)
    gp = qp.Problem(prob, precision=prec, gather64=True)
    r = gp.homogenized(tol=1e-12)
    err = np.abs(r.A - ref.A).max() / np.abs(ref.A).max()
    say("  A* rel err", err, [i.iters for i in r.infos])
    assert err <= 1e-10
    gp.close()


def test_vectors_beyond_4gib_sampled_rows():
    prob = W.icosahedral(26)
    D = prob.D
    assert D >= 1 << 28
    need = qp.qp_workspace_bytes(prob.d, prob.n, prob.N, prob.g) + 3 * 16 * D
    free, _ = torch.cuda.mem_get_info()
    if free < need + (8 << 30):
        pytest.skip(f"needs {need / 2**30:.0f} GiB of device memory, {free / 2**30:.0f} free")
    say("[case] icosahedral N=26 D", D, "workspace GiB", need / 2**30)
    u = W.random_vector(D, seed=91)
    gp = qp.Problem(prob)
    rng = np.random.default_rng(5)
    rows = np.concatenate([rng.integers(1 << 28, D, size=192), rng.integers(0, D, size=64),
                           np.arange(D - 8, D), np.arange(1, 9)])
    ud = dev(u)
    y = gp.matvec_d(ud)[torch.from_numpy(rows).cuda()].cpu().numpy()
    say("  fp64 product done")
    ref = oracle.matvec_rows(prob, u, rows)
    scale = np.abs(ref).max()
    err = np.abs(y - ref).max() / scale
    say("  fp64 sampled rel err", err)
    assert err <= 1e-13
    del ud
    u32 = dev(u.astype(np.complex64), torch.complex64)
    y32 = gp.matvec32_d(u32)[torch.from_numpy(rows).cuda()].cpu().numpy()
    err32 = np.abs(y32 - ref).max() / scale
    say("  fp32 sampled rel err", err32)
    assert err32 <= 2e-5
    gp.close()
