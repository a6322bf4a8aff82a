"""The stiffness product's work layout: explicit layouts and the autotuner.

The layout (plane tiles per wave work item, workgroups, XCD-front or plain
item order) decides only which waves compute which outputs and which
workgroup sums which partial dot product.  Every product value must therefore
be bitwise the same under every layout, and a solve under any layout must
meet the oracle's A* as the default layout does.
"""
from __future__ import annotations

import json
import os
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

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")

# (item_tiles, workgroups, xcd_front): grids below, at and above one item per
# wave, grids that are and are not multiples of 8
LAYOUTS = [(it, nb, x) for it in (1, 2, 4) for nb in (8, 24, 256, 1024) for x in (0, 1)]
LAYOUTS += [(1, 1, 0), (4, 3, 1), (2, 1000, 1)]
# slab order (xcd_front 2): the slowest axis innermost inside each XCD's eighth
# (identity where the eighths are not whole slabs, as for N = 6 here)
LAYOUTS += [(4, 1024, 2), (1, 256, 2), (2, 24, 2), (1, 1, 2)]
# blocked slab order (xcd_front 3; as the slab order below five axes)
LAYOUTS += [(4, 1024, 3), (1, 256, 3), (2, 8, 3)]


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def dev(x: np.ndarray, dtype=torch.complex128):
    return torch.from_numpy(np.ascontiguousarray(x)).to(device="cuda", dtype=dtype)


def key(L: dict) -> tuple:
    return L["item_tiles"], L["workgroups"], L["xcd_front"]


def key64(L: dict) -> tuple:
    return L["item_tiles64"], L["workgroups64"], L["xcd_front64"]


def _many_modes(N: int):
    # 31 seeded +-mode pairs and the mean (g = 63: 64 padded mode records)
    rng = np.random.default_rng(2404)
    modes, coef, amps = W.random_modes(4, 31, 2, rng, 0.05, 2.5, 3.0)
    return W.Problem("eightfold_many_modes", 2, 4, int(N), W.eightfold_P(), modes, coef,
                     {"amplitudes": amps.tolist()})


@pytest.mark.parametrize("make", [lambda: W.eightfold_random(16, 3), lambda: W.icosahedral(6),
                                  lambda: _many_modes(12)],
                         ids=["eightfold_random_N16", "icosa_N6", "many_modes_g63_N12"])
def test_every_layout_gives_bitwise_equal_products(make):
    prob = make()
    say("[case] layouts", prob.D, prob.g)
    a = qp.Problem(prob)
    u = W.random_vector(prob.D, seed=5)
    u32 = dev(u.astype(np.complex64), torch.complex64)
    y64 = a.matvec_d(dev(u))
    y32 = a.matvec32_d(u32)
    ref = oracle.matvec(prob, u)
    assert np.abs(y64.cpu().numpy() - ref).max() <= 1e-13 * np.abs(ref).max()
    for L in LAYOUTS:
        a.set_layout(*L)
        got = a.layout()
        assert key(got) == L and key64(got) == L and got["tuned"] == 0
        assert torch.equal(a.matvec_d(dev(u)), y64), L
        assert torch.equal(a.matvec32_d(u32), y32), L
    a.close()


def _large_rows(prob, count: int = 1500) -> np.ndarray:
    """Rows of the icosahedral N = 16 grid to check against the oracle: the
    first and last planes' corners, entries on the +-N/2 faces of every axis
    (where the neighbours wrap), and a seeded uniform sample."""
    D, N, n = prob.D, prob.N, prob.n
    rng = np.random.default_rng(16)
    rows = [np.arange(64), np.arange(D - 64, D), rng.integers(0, D, count)]
    for t in range(n):
        stride = N ** (n - 1 - t)
        base = rng.integers(0, D, 40)
        digit = (base // stride) % N
        rows.append(base + (N // 2 - digit) * stride)        # digit N/2: k_t = -N/2
        rows.append(base + (N // 2 - 1 - digit) * stride)    # digit N/2 - 1: k_t = N/2 - 1
    return np.unique(np.concatenate(rows))


def test_large_icosahedral_products_against_the_oracle():
    """16,777,216 unknowns (the largest serving request and the HBM-sized
    product shape): the FP64 and float products at sampled rows against the
    oracle evaluated row by row, under the default layout and the slab orders
    (each XCD's eighth is two values of the slowest axis), bitwise equal
    across layouts."""
    prob = W.icosahedral(16)
    a = qp.Problem(prob)
    say("[case] icosahedral N=16 products, layout", a.layout())
    gen = torch.Generator(device="cuda")
    gen.manual_seed(3)
    u = torch.randn(prob.D, dtype=torch.complex128, device="cuda", generator=gen)
    u32 = u.to(torch.complex64)
    y64, y32 = a.matvec_d(u), a.matvec32_d(u32)
    rows = _large_rows(prob)
    ix = torch.from_numpy(rows).cuda()
    ref = oracle.matvec_rows(prob, u.cpu().numpy(), rows)
    ref32 = oracle.matvec_rows(prob, u32.cpu().numpy().astype(np.complex128), rows)
    scale = np.abs(ref).max()
    e64 = np.abs(y64[ix].cpu().numpy() - ref).max() / scale
    e32 = np.abs(y32[ix].cpu().numpy() - ref32).max() / np.abs(ref32).max()
    say(f"  {rows.size} rows: FP64 rel err {e64:.2e}, float {e32:.2e}")
    assert e64 <= 1e-13 and e32 <= 2e-5
    for L in [(2, 1024, 2), (4, 1024, 2), (1, 512, 2), (1, 1024, 1), (4, 1024, 3), (2, 1024, 3),
              (1, 512, 3)]:
        a.set_layout(*L)
        assert torch.equal(a.matvec_d(u), y64), L
        assert torch.equal(a.matvec32_d(u32), y32), L
    a.close()


def test_solves_under_other_layouts_meet_the_oracle():
    gold = json.load(open(os.path.join(GOLDEN, "oracle_astar.json")))["c2_eightfold_N16"]
    A_ref = np.array(gold["A"])
    prob = W.eightfold(16)
    a = qp.Problem(prob)
    # grids whose partial sums do not fill whole rounds of a workgroup (600
    # and 1000: some threads of the next kernel reduce one more partial)
    for L in [(1, 24, 0), (4, 1024, 1), (2, 8, 1), (4, 1024, 2), (1, 256, 2), (1, 600, 1),
              (2, 1000, 0)]:
        a.set_layout(*L)
        for prec in ("fp64", "fp32ir"):
            a.set_precision(prec)
            r = a.homogenized(tol=1e-12)
            err = np.abs(r.A - A_ref).max() / np.abs(A_ref).max()
            say(f"  layout {L} {prec}: iters {[i.iters for i in r.infos]} rel err {err:.2e}")
            assert all(i.status == 0 for i in r.infos)
            assert err <= 1e-10, (L, prec, err)
    a.close()


def test_autotune_chooses_a_layout_and_reuses_it_for_the_shape():
    gold = json.load(open(os.path.join(GOLDEN, "oracle_astar.json")))["c2_eightfold_N16"]
    A_ref = np.array(gold["A"])
    prob = W.eightfold(16)
    plain = qp.Problem(prob, precision="fp32ir")
    a = qp.Problem(prob, precision="fp32ir", autotune=True)
    La = a.layout()
    say("  tuned layout", La)
    assert La["tuned"] in (1, 2)
    if La["tuned"] == 1:
        assert La["candidates"] >= 2
        assert 0 < La["best_us"] <= La["default_us"]
    b = qp.Problem(prob, precision="fp32ir", autotune=True)
    Lb = b.layout()
    assert Lb["tuned"] == 2 and key(Lb) == key(La) and key64(Lb) == key64(La)
    u = W.random_vector(prob.D, seed=9)
    assert torch.equal(a.matvec_d(dev(u)), plain.matvec_d(dev(u)))
    r = a.homogenized(tol=1e-12)
    err = np.abs(r.A - A_ref).max() / np.abs(A_ref).max()
    assert all(i.status == 0 for i in r.infos) and err <= 1e-10, err
    # the same layouts set explicitly repeat the tuned problem's A* bitwise
    plain.set_layout(*key(La), *key64(La))
    r2 = plain.homogenized(tol=1e-12)
    assert np.array_equal(r2.A, r.A)
    for p in (plain, a, b):
        p.close()


def test_separate_fp64_layout():
    # float and FP64 launches on different layouts: both products unchanged,
    # and an FP32-IR solve (float iterations, FP64 replacements) meets the oracle
    gold = json.load(open(os.path.join(GOLDEN, "oracle_astar.json")))["c2_eightfold_N16"]
    A_ref = np.array(gold["A"])
    prob = W.eightfold(16)
    a = qp.Problem(prob, precision="fp32ir")
    u = W.random_vector(prob.D, seed=11)
    u32 = dev(u.astype(np.complex64), torch.complex64)
    y64, y32 = a.matvec_d(dev(u)), a.matvec32_d(u32)
    a.set_layout(4, 256, 1, 1, 1000, 2)
    assert key(a.layout()) == (4, 256, 1) and key64(a.layout()) == (1, 1000, 2)
    assert torch.equal(a.matvec_d(dev(u)), y64) and torch.equal(a.matvec32_d(u32), y32)
    r = a.homogenized(tol=1e-12)
    err = np.abs(r.A - A_ref).max() / np.abs(A_ref).max()
    assert all(i.status == 0 for i in r.infos) and err <= 1e-10, err
    with pytest.raises(qp.QPError):
        a.set_layout(4, 256, 1, 3, 64, 0)  # item_tiles64 not 1, 2 or 4
    a.close()


def test_invalid_layouts_are_rejected():
    a = qp.Problem(W.eightfold(8))
    for L in [(3, 8, 0), (1, 0, 0), (1, 1025, 0), (1, 8, 4)]:
        with pytest.raises(qp.QPError) as e:
            a.set_layout(*L)
        assert e.value.status == qp.QP_EINVAL
    line = qp.Problem(W.periodic_1d(100))  # line tiles: one item size
    assert line.layout()["item_tiles"] == 1
    with pytest.raises(qp.QPError):
        line.set_layout(2, 8, 1)
    u = W.random_vector(line.D, seed=3)
    y = line.matvec_d(dev(u))
    line.set_layout(1, 16, 0)
    assert torch.equal(line.matvec_d(dev(u)), y)
    a.close()
    line.close()
