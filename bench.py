"""Benchmark: corrector solves per second of the projection-method hot path on
one MI355X.

Workload: the eightfold d=2, n=4 problem at N=32 per axis (1,048,576 complex
unknowns) with 8 seeded random +-mode pairs around mean 3 (17 modes).  One step
is one homogenization: the two corrector solves to relative residual 1e-12
and the 2x2 homogenized coefficient A*.  The headline precision is FP32-IR
(float stiffness product and preconditioner inside FP64 refinement); the same
steps in plain FP64 are timed beside it.  A* of both is checked against the
CPU oracle's value (tests/golden/oracle_astar.json).

Prints one JSON line.  Inputs are resident in HBM before the timed region.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "corrector solves/s + matvec HBM GB/s, FP32-IR vs FP64 @1e-10; p99 latency"
HBM_PEAK_GBS = 8000.0
TOL = 1e-12
# batch instances with at most this many unknowns run grouped beside the
# per-problem streams of the larger ones (qp_homogenized_batch_mixed)
MIXED_GROUP_DIM = 1 << 15
LATENCY_SAMPLES = 200  # homogenizations behind the latency percentiles
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_matvec_fp32_eightfold_n4_N32.txt")
TRAFFIC_FILE_HBM = os.path.join(ROOT, "profiles", "matvec_icosahedral_n6_N16_dram.txt")
# sources of the stiffness-product kernels (the product and its device helpers)
MATVEC_SRC = [os.path.join(ROOT, "paper_2404_06841_amd", "csrc", f)
              for f in ("qp_matvec.hip", "qp_matvec_half.hip", "qp_matvec_kernels.h",
                        "qp_chunk_walk.h", "qp_device.h")]


def parse_args():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-probe", action="store_true",
                    help="only run a plain device copy of known size (counter calibration)")
    ap.add_argument("--product-probe", action="store_true",
                    help="only run the HBM-sized stiffness products (icosahedral N=16, FP64 and "
                         "float; icosahedral N=15 FP64 on full and on half storage; seven "
                         "launches each) and the plain copies of --copy-probe, for counter runs")
    ap.add_argument("--headline-only", action="store_true",
                    help="only run the headline FP32-IR homogenizations (warm-up and timed "
                         "steps) and print their rate, for counter runs")
    ap.add_argument("--layout", type=str, default=None,
                    help="with --headline-only: IT,WG,XF,IT64,WG64,XF64, the product layouts "
                         "to use instead of the autotuner's choice (counter runs perturb the "
                         "tuner's timings, so they pin the layout the timed run chose)")
    ap.add_argument("--config-table", action="store_true",
                    help="only time every workload configuration on the GPU (FP32-IR and "
                         "FP64) beside the oracle on all host threads, one line each")
    ap.add_argument("--small-sweep", action="store_true",
                    help="only compare FP64 homogenizations of small problems in one launch "
                         "(small_dim) with the three-launch loop, one line per problem")
    ap.add_argument("--batch-breakdown", action="store_true",
                    help="only time the 64-instance FP32-IR batch by size class (instances "
                         "alone, on streams, grouped) and print one line per class")
    return ap.parse_args()


def batch_breakdown():
    """The FP32-IR batch of batch_instances split by instance size: for all
    instances, the N = 32 ones and the smaller ones, the sum of the times each
    instance takes alone, the time on per-problem streams and the time grouped;
    then the whole batch with the instances up to several size limits grouped
    beside the streams of the others (median of three runs after a warm-up)."""
    import torch

    from paper_2404_06841_amd import qp
    from paper_2404_06841_amd import workloads as W
    probs = W.eightfold_batch(64)
    gps = [qp.Problem(pr, precision="fp32ir", stream=torch.cuda.Stream(), autotune=True)
           for pr in probs]
    alone = []
    for gp in gps:
        gp.homogenized(tol=TOL, energy=False)
        ts = []
        for _ in range(3):
            t0 = time.perf_counter()
            gp.homogenized(tol=TOL, energy=False)
            ts.append(time.perf_counter() - t0)
        alone.append(sorted(ts)[1])

    def timed(sub, grouped):
        qp.homogenized_batch(sub, tol=TOL, grouped=grouped)
        torch.cuda.synchronize()
        ts = []
        for _ in range(3):
            t0 = time.perf_counter()
            qp.homogenized_batch(sub, tol=TOL, grouped=grouped)
            ts.append(time.perf_counter() - t0)
        return sorted(ts)[1]

    for name, keep in (("all", lambda N: True), ("N=32", lambda N: N == 32),
                       ("N<=24", lambda N: N <= 24), ("N<=16", lambda N: N <= 16)):
        idx = [i for i, pr in enumerate(probs) if keep(pr.N)]
        sub = [gps[i] for i in idx]
        print(json.dumps({"batch_breakdown": name, "instances": len(idx),
                          "unknowns": int(sum(probs[i].D for i in idx)),
                          "alone_sum_ms": round(sum(alone[i] for i in idx) * 1e3, 2),
                          "streams_ms": round(timed(sub, False) * 1e3, 2),
                          "grouped_ms": round(timed(sub, True) * 1e3, 2)}), flush=True)
    # the whole batch with the instances up to a size limit grouped
    for limit in (4096, 20736, 1 << 15, 65536, 331776):
        qp.homogenized_batch(gps, tol=TOL, group_max_dim=limit)
        torch.cuda.synchronize()
        ts = []
        for _ in range(3):
            t0 = time.perf_counter()
            qp.homogenized_batch(gps, tol=TOL, group_max_dim=limit)
            ts.append(time.perf_counter() - t0)
        print(json.dumps({"batch_breakdown": "mixed", "group_max_dim": limit,
                          "grouped_instances": sum(1 for pr in probs if pr.D <= limit),
                          "ms": round(sorted(ts)[1] * 1e3, 2)}), flush=True)
    for gp in gps:
        gp.close()


def config_table():
    """Corrector solves per second for every workload configuration: on the
    GPU (FP32-IR and FP64 homogenizations, autotuned layouts, at least five
    runs or one second after a warm-up) and by the oracle on all host threads
    (its corrector solves, A* excluded): the degenerate one-dimensional field
    at N = 32 (d = 1, n = 2), the eightfold field at N = 16 and the seeded
    eightfold field at N = 32 in full; the 64-instance batch as the sum over
    its instances (GPU: the mixed batch); the icosahedral field at N = 6, 8,
    12 in full and at N = 16 from three oracle iterations per corrector,
    scaled to the GPU's FP64 iteration counts.  First, the paper's first
    example at N = 32, 64, 128: the FP64 solve of a manufactured solution,
    its time and relative error."""
    import numpy as np
    import torch

    import oracle
    from paper_2404_06841_amd import qp
    from paper_2404_06841_amd import workloads as W

    def gpu_rate(prob, prec):
        gp = qp.Problem(prob, precision=prec, autotune=True)
        r = gp.homogenized(tol=TOL, energy=False)
        torch.cuda.synchronize()
        n, t0 = 0, time.perf_counter()
        while n < 5 or time.perf_counter() - t0 < 1.0:
            r = gp.homogenized(tol=TOL, energy=False)
            n += 1
        dt = time.perf_counter() - t0
        gp.close()
        return prob.d * n / dt, [int(i.iters) for i in r.infos]

    def oracle_solves(prob, maxit=10000):
        t0 = time.perf_counter()
        its = []
        for j in range(prob.d):
            _, _, it, _ = oracle.pcg(prob, oracle.corrector_rhs(prob, j), tol=TOL, maxit=maxit)
            its.append(it)
        return time.perf_counter() - t0, its

    threads = oracle.max_threads()
    # the paper's first example (Sec. 5.1.1): a = 6 + cos y1 + cos y2 on
    # P = 2 pi (1, sqrt 2), manufactured solution u = sin y1 + sin y2 (its
    # coefficients -i/2 at +e_t and +i/2 at -e_t lie in the grid), F = Q U
    for N in (32, 64, 128):
        prob = W.one_d_two_mode(N, 6.0, 2 * np.pi)
        Ux = torch.zeros(prob.D, dtype=torch.complex128, device="cuda")
        for stride in (N, 1):  # the two axes of the grid
            Ux[1 * stride] = -0.5j
            Ux[(N - 1) * stride] = 0.5j
        gp = qp.Problem(prob)
        F = gp.matvec_d(Ux).clone()
        U, info = gp.solve_d(F, tol=TOL)
        ts = []
        for _ in range(5):
            t0 = time.perf_counter()
            U, info = gp.solve_d(F, tol=TOL)
            ts.append(time.perf_counter() - t0)
        err = float(torch.linalg.vector_norm(U - Ux) / torch.linalg.vector_norm(Ux))
        print(json.dumps({"config": f"paper example 1 (d=1 n=2, a = 6 + cos + cos) N={N}",
                          "unknowns": int(prob.D), "gpu_fp64_solve_ms": round(sorted(ts)[2] * 1e3, 3),
                          "iters": int(info.iters), "relative_error": err}), flush=True)
        gp.close()
    cases = [("C1 one-dimensional degenerate d=1 n=2 N=32", W.one_d_two_mode(32, 2.0)),
             ("C2 eightfold d=2 n=4 N=16", W.eightfold(16)),
             ("C3 seeded eightfold d=2 n=4 N=32", W.eightfold_random(32, 0)),
             ("C5 icosahedral d=3 n=6 N=6", W.icosahedral(6)),
             ("C5 icosahedral d=3 n=6 N=8", W.icosahedral(8)),
             ("C5 icosahedral d=3 n=6 N=12", W.icosahedral(12))]
    for name, prob in cases:
        r32, it32 = gpu_rate(prob, "fp32ir")
        r64, it64 = gpu_rate(prob, "fp64")
        dt, its = oracle_solves(prob)
        print(json.dumps({"config": name, "unknowns": int(prob.D), "gpu_fp32ir_solves_per_s": round(r32, 2),
                          "gpu_fp64_solves_per_s": round(r64, 2), "gpu_iters_fp64": it64,
                          "oracle_solves_per_s": round(prob.d / dt, 4), "oracle_iters": its,
                          "oracle_threads": threads,
                          "gpu_fp32ir_over_oracle": round(r32 * dt / prob.d, 1)}), flush=True)
    # icosahedral N = 16: three oracle iterations per corrector, scaled
    prob = W.icosahedral(16)
    r32, it32 = gpu_rate(prob, "fp32ir")
    r64, it64 = gpu_rate(prob, "fp64")
    dt3, _ = oracle_solves(prob, maxit=3)
    est = dt3 * (sum(it64) / (3.0 * prob.d))
    print(json.dumps({"config": "C5 icosahedral d=3 n=6 N=16", "unknowns": int(prob.D),
                      "gpu_fp32ir_solves_per_s": round(r32, 2), "gpu_fp64_solves_per_s": round(r64, 2),
                      "gpu_iters_fp64": it64,
                      "oracle_solves_per_s": round(prob.d / est, 5),
                      "oracle_sample": f"3 iterations per corrector in {dt3:.2f} s, scaled to "
                                       f"{sum(it64)} iterations",
                      "oracle_threads": threads,
                      "gpu_fp32ir_over_oracle": round(r32 * est / prob.d, 1)}), flush=True)
    # the 64-instance batch: GPU mixed batch; oracle summed over the instances
    probs = W.eightfold_batch(64)
    gps = [qp.Problem(pr, precision="fp32ir", stream=torch.cuda.Stream(), autotune=True)
           for pr in probs]
    qp.homogenized_batch(gps, tol=TOL, group_max_dim=MIXED_GROUP_DIM)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(3):
        qp.homogenized_batch(gps, tol=TOL, group_max_dim=MIXED_GROUP_DIM)
    dtg = (time.perf_counter() - t0) / 3
    for gp in gps:
        gp.close()
    solves = sum(pr.d for pr in probs)
    tot = 0.0
    for i, pr in enumerate(probs):
        dt, _ = oracle_solves(pr)
        tot += dt
        if i % 16 == 15:
            print(json.dumps({"config_progress": f"oracle over batch instances {i + 1}/64",
                              "seconds": round(tot, 1)}), flush=True)
    print(json.dumps({"config": "C4 64 seeded eightfold instances, N in {8, 12, 16, 24, 32}",
                      "unknowns": int(sum(pr.D for pr in probs)),
                      "gpu_fp32ir_solves_per_s": round(solves / dtg, 2),
                      "gpu_path": "qp_homogenized_batch_mixed",
                      "oracle_solves_per_s": round(solves / tot, 4), "oracle_threads": threads,
                      "gpu_fp32ir_over_oracle": round(tot / dtg, 1)}), flush=True)


def small_sweep():
    """FP64 homogenizations of problems of at most 2048 unknowns with the
    whole PCG loop in one launch (the default small_dim) and with three
    launches per iteration (small_dim 0): corrector solves per second and
    microseconds per iteration (at least ten homogenizations or half a
    second each, after a warm-up)."""
    import numpy as np
    import torch

    from paper_2404_06841_amd import qp
    from paper_2404_06841_amd import workloads as W
    cases = [("one-dimensional degenerate N=32", W.one_d_two_mode(32, 2.0)),
             ("one-dimensional periodic N=100", W.periodic_1d(100)),
             ("one-dimensional N=45", W.one_d_two_mode(45, 6.0, 2 * np.pi)),
             ("eightfold N=6", W.eightfold(6)), ("seeded eightfold N=5", W.eightfold_random(5, 7)),
             ("seeded eightfold N=6", W.eightfold_random(6, 2)), ("icosahedral N=3", W.icosahedral(3)),
             ("cubic d=3 N=7", W.periodic_cubic(3, 7)), ("cubic d=3 N=12", W.periodic_cubic(3, 12)),
             ("cubic d=4 N=6", W.periodic_cubic(4, 6))]
    for name, prob in cases:
        out = {"small_sweep": name, "unknowns": int(prob.D), "modes": int(prob.g)}
        for label, sd in (("one_launch", None), ("three_launches", 0)):
            gp = qp.Problem(prob, small_dim=sd)
            r = gp.homogenized(tol=TOL, energy=False)
            torch.cuda.synchronize()
            n, t0 = 0, time.perf_counter()
            while n < 10 or time.perf_counter() - t0 < 0.5:
                r = gp.homogenized(tol=TOL, energy=False)
                n += 1
            dt = (time.perf_counter() - t0) / n
            it = max(int(i.iters) for i in r.infos)
            out[label] = {"solves_per_s": round(prob.d / dt, 1), "iters": it,
                          "us_per_iteration": round(dt * 1e6 / it, 2)}
            gp.close()
        print(json.dumps(out), flush=True)


def copy_probe():
    """Plain copies of known size, five times each, for scaling the FETCH_SIZE /
    WRITE_SIZE counters to bytes: the runtime's device-to-device copy and an
    elementwise torch kernel (y = x * 1) over 512 MiB."""
    import torch
    n = 512 * 1024 * 1024 // 4
    x = torch.ones(n, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    for _ in range(5):
        y.copy_(x)
    for _ in range(5):
        torch.mul(x, 1.0, out=y)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_bytes_per_copy": 4 * n, "copies": 5,
                      "kernels": ["runtime copy", "elementwise mul"]}), flush=True)


def product_probe():
    """The launches that the HBM-sized roofline is taken on: the icosahedral
    N = 16 products (one right-hand side, FP64 then float, the default
    layout, as hbm_products times them), seven of each; then the FP64
    products of icosahedral N = 15 on full and on half storage (default
    layouts, as half_storage times them); then the copies of copy_probe.
    The layouts are fixed because a counter run perturbs the autotuner's
    timings."""
    import torch

    from paper_2404_06841_amd import qp
    from paper_2404_06841_amd import workloads as W
    prob = W.icosahedral(16)
    gp = qp.Problem(prob)
    gen = torch.Generator(device="cuda")
    gen.manual_seed(16)
    for dtype, fn in ((torch.complex128, gp.matvec_d), (torch.complex64, gp.matvec32_d)):
        u = torch.randn(prob.D, dtype=dtype, device="cuda", generator=gen)
        y = torch.empty_like(u)
        for _ in range(7):
            fn(u, y)
        del u, y
    torch.cuda.synchronize()
    print(json.dumps({"product_probe": prob.D, "layout": gp.layout(), "launches": 7}), flush=True)
    gp.close()
    # Hermitian half storage at odd N: the FP64 product on the full and on the
    # half problem
    prob = W.icosahedral(15)
    for half in (False, True):
        gp = qp.Problem(prob, half_storage=half)
        u = torch.randn(gp.D, dtype=torch.complex128, device="cuda", generator=gen)
        y = torch.empty_like(u)
        for _ in range(7):
            gp.matvec_d(u, y)
        torch.cuda.synchronize()
        print(json.dumps({"product_probe": gp.D, "half_storage": half, "layout": gp.layout(),
                          "launches": 7}), flush=True)
        del u, y
        gp.close()
    copy_probe()


def kernel_hash() -> str:
    h = hashlib.sha256()
    for path in MATVEC_SRC:
        with open(path, "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def measured_traffic(path: str = TRAFFIC_FILE, key: str = "hbm_bytes_per_launch",
                     layout=None):
    """Memory-side bytes per stiffness-product launch from a committed
    rocprofv3 counter summary (sized read and write requests), or None when
    it was taken on another kernel version or, given `layout` (item tiles,
    workgroups, XCD order of the product), on another work layout."""
    if not os.path.exists(path):
        return None
    kv = {}
    for line in open(path):
        if "=" in line and not line.startswith("#"):
            k, v = line.split("=", 1)
            kv[k.strip()] = v.strip()
    if kv.get("kernel_hash") != kernel_hash():
        return None
    if layout is not None and kv.get("layout") != ",".join(str(int(v)) for v in layout):
        return None
    try:
        return float(kv[key])
    except (KeyError, ValueError):
        return None


def run_steps(gp, steps: int, torch):
    """Time `steps` homogenizations; returns (seconds, per-step latencies in ms,
    result of the last step, (float product ms, launches, right-hand sides served))."""
    lat = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    r = None
    mv_ms, mv_n, mv_rhs = 0.0, 0, 0
    for _ in range(steps):
        ts = time.perf_counter()
        r = gp.homogenized(tol=TOL, energy=False)
        lat.append((time.perf_counter() - ts) * 1e3)
        i0 = r.infos[0]  # the correctors are solved together: shared launch totals
        mv_ms += i0.matvec32_ms
        mv_n += i0.matvec32_launches
        mv_rhs += i0.matvec32_rhs
    torch.cuda.synchronize()
    return time.perf_counter() - t0, lat, r, (mv_ms, mv_n, mv_rhs)


def hbm_products(torch, qp, W):
    """Stiffness products on a vector far larger than the caches: icosahedral
    d=3, n=6 at N=16 (16,777,216 unknowns; 268 MB per FP64 vector), one
    right-hand side per launch, default layout, each launch timed by the HIP
    event pair it records itself on the library's stream (the profile
    option).  Algorithmic bytes: read x once, write y once.
    Each figure is given against the nominal HBM peak and against a measured
    512 MiB device copy (2 x 512 MiB moved per copy)."""
    prob = W.icosahedral(16)
    gp = qp.Problem(prob)  # the default layout, as in the counter runs of --product-probe
    D = prob.D
    gen = torch.Generator(device="cuda")
    gen.manual_seed(16)
    out = {"workload": "icosahedral d=3 n=6 N=16 (16,777,216 unknowns, 13 modes)",
           "layout": gp.layout()}
    # second denominator: plain copies of 512 MiB (read + write): the runtime's
    # device-to-device copy and an elementwise kernel (y = x * 1); the faster
    xc = torch.ones(1 << 27, dtype=torch.float32, device="cuda")
    yc = torch.empty_like(xc)
    rates = {}
    for name, fn in (("runtime_copy", lambda: yc.copy_(xc)),
                     ("elementwise", lambda: torch.mul(xc, 1.0, out=yc))):
        for _ in range(2):
            fn()
        c0, c1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        c0.record()
        for _ in range(5):
            fn()
        c1.record()
        torch.cuda.synchronize()
        rates[name] = round(2.0 * xc.numel() * 4 * 5 / (c0.elapsed_time(c1) * 1e-3) / 1e9, 1)
    del xc, yc
    copy_gbs = max(rates.values())
    out["copy_GBs"] = copy_gbs
    out["copy_GBs_by_kind"] = rates
    for name, dtype, fn, per in (("fp64", torch.complex128, gp.matvec_d, 32.0),
                                 ("fp32", torch.complex64, gp.matvec32_d, 16.0)):
        u = torch.randn(D, dtype=dtype, device="cuda", generator=gen)
        y = torch.empty_like(u)
        # kernel time from the event pair each launch records itself
        us = per_launch_us(torch, lambda: fn(u, y), gp=gp)
        gbs = per * D / (us * 1e-6) / 1e9
        out[name] = {"avg_launch_us": round(us, 2), "algorithmic_bytes": int(per * D),
                     "achieved_GBs": round(gbs, 1), "frac_of_hbm_peak": round(gbs / HBM_PEAK_GBS, 4),
                     "frac_of_copy": round(gbs / copy_gbs, 4)}
        del u, y
    gp.close()
    return out


def half_storage(torch, np, qp, W, gold, steps: int = 5):
    """Hermitian half storage at odd N (icosahedral d=3, n=6, N=15:
    11,390,625 unknowns, 5,695,313 stored): the stiffness products of a
    half-storage problem against the full-storage ones (each call bracketed
    by HIP events on the library's stream; algorithmic bytes 32 B FP64 / 16 B
    float per stored entry), and homogenizations on both storages in both
    precisions, A* against the oracle's stored value."""
    prob = W.icosahedral(15)
    A_ref = np.array(gold["icosa_N15"]["A"])
    D, H = prob.D, (prob.D + 1) // 2
    gen = torch.Generator(device="cuda")
    gen.manual_seed(15)
    out = {"workload": "icosahedral d=3 n=6 N=15 (11,390,625 unknowns; 5,695,313 stored in "
                       "half storage), three correctors per homogenization"}
    for storage in ("full", "half"):
        res = {}
        # the products (the FP64 and float kernels of this storage), in the
        # default layout as in the counter runs of --product-probe
        gp = qp.Problem(prob, half_storage=(storage == "half"))
        for name, dtype, fn, per in (("fp64", torch.complex128, gp.matvec_d, 32.0),
                                     ("fp32", torch.complex64, gp.matvec32_d, 16.0)):
            u = torch.randn(gp.D, dtype=dtype, device="cuda", generator=gen)
            y = torch.empty_like(u)
            us = per_launch_us(torch, lambda: fn(u, y), gp=gp)
            res["product_" + name] = {
                "avg_launch_us": round(us, 2), "algorithmic_bytes": int(per * gp.D),
                "achieved_GBs": round(per * gp.D / (us * 1e-6) / 1e9, 1),
                "frac_of_hbm_peak": round(per * gp.D / (us * 1e-6) / 1e9 / HBM_PEAK_GBS, 4)}
            del u, y
        res["product_layout"] = gp.layout()
        gp.close()
        # the homogenizations, each on a problem with the autotuner's layouts
        for prec in ("fp32ir", "fp64"):
            gp = qp.Problem(prob, precision=prec, autotune=True, half_storage=(storage == "half"))
            if prec == "fp32ir":
                res["layout"] = gp.layout()
            gp.homogenized(tol=TOL, energy=False)  # warm-up
            dt, _, r, _ = run_steps(gp, steps, torch)
            res[prec] = {"value": round(prob.d * steps / dt, 2), "unit": "corrector solves/s",
                         "ms_per_step": round(dt / steps * 1e3, 3),
                         "astar_rel_err": float(np.abs(r.A - A_ref).max() / np.abs(A_ref).max()),
                         "iters": [i.iters for i in r.infos]}
            gp.close()
        out[storage] = res
    f, h = out["full"], out["half"]
    out["half_over_full_product_time_fp64"] = round(
        h["product_fp64"]["avg_launch_us"] / f["product_fp64"]["avg_launch_us"], 3)
    out["half_over_full_product_time_fp32"] = round(
        h["product_fp32"]["avg_launch_us"] / f["product_fp32"]["avg_launch_us"], 3)
    out["half_speedup_fp32ir_solves"] = round(h["fp32ir"]["value"] / f["fp32ir"]["value"], 3)
    out["half_speedup_fp64_solves"] = round(h["fp64"]["value"] / f["fp64"]["value"], 3)
    return out


def per_launch_us(torch, fn, reps: int = 20, warm: int = 3, gp=None) -> float:
    """Average duration of fn() (an entry point that returns after its launch
    completed).  With gp (the problem whose matvec_d / matvec32_d fn calls):
    the kernel time from the event pair the launch itself records (profile
    option on), which excludes the host's dispatch gap.  Otherwise each call
    is bracketed by its own HIP events on torch's current stream (the
    library's stream), gap included."""
    for _ in range(warm):
        fn()
    if gp is not None:
        gp.set_options(profile=1)
        total = 0.0
        for _ in range(reps):
            fn()
            total += gp.last_product_ms()
        gp.set_options(profile=0)
        return total * 1e3 / reps
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(reps)]
    for e0, e1 in ev:
        e0.record()
        fn()
        e1.record()
    torch.cuda.synchronize()
    return sum(e0.elapsed_time(e1) for e0, e1 in ev) * 1e3 / reps


def stored_matrix(torch, qp, W):
    """The paper's compressed matrix (Alg. 1: D * g stored triples (i, j,
    Q_ij), int32 indices and FP64 complex values) against the matrix-free
    product, FP64, one right-hand side per launch."""
    out = {}
    gen = torch.Generator(device="cuda")
    gen.manual_seed(7)
    for name, prob in (("eightfold d=2 n=4 N=32", W.eightfold_random(32, 0)),
                       ("icosahedral d=3 n=6 N=16", W.icosahedral(16))):
        gp = qp.Problem(prob)
        t0 = time.perf_counter()
        coo = gp.coo_build_d()
        build_ms = (time.perf_counter() - t0) * 1e3
        D, g = prob.D, prob.g
        u = torch.randn(D, dtype=torch.complex128, device="cuda", generator=gen)
        y = torch.empty_like(u)
        t_coo = per_launch_us(torch, lambda: gp.coo_matvec_d(coo, u, y))
        # both per call (dispatch gap included), so that the two compare alike
        t_mf = per_launch_us(torch, lambda: gp.matvec_d(u, y))
        entries = D * g
        out[name] = {"unknowns": D, "entries": entries, "stored_bytes": entries * 24,
                     "build_ms": round(build_ms, 2),
                     "stored_product_us": round(t_coo, 2), "matrix_free_product_us": round(t_mf, 2),
                     "stored_over_matrix_free": round(t_coo / t_mf, 2),
                     "stored_GBs_read": round((entries * 20 + 32 * D) / (t_coo * 1e-6) / 1e9, 1)}
        del coo, u, y
        gp.close()
    return out


def sampled_inputs(torch, qp):
    """Forward DFT of grid samples (qp_dft_d: the discrete Fourier-Bohr
    coefficients of a sampled coefficient or right-hand side), FP64 complex,
    on the eightfold N=32 and icosahedral N=16 grids."""
    out = {}
    gen = torch.Generator(device="cuda")
    gen.manual_seed(3)
    for name, n, N in (("n=4 N=32", 4, 32), ("n=6 N=16", 6, 16)):
        D = N ** n
        x = torch.randn(D, dtype=torch.complex128, device="cuda", generator=gen)
        y = torch.empty_like(x)
        us = per_launch_us(torch, lambda: qp.dft_d(x, n, N, out=y), reps=10, warm=2)
        out[name] = {"points": D, "us": round(us, 1),
                     "GBs_per_pass": round(32.0 * D * n / (us * 1e-6) / 1e9, 1)}
        del x, y
    return out


def diagonal_workload(torch, np, qp, W, gold, steps: int, warmup: int):
    """The diagonal coefficient diag(a_1, a_2) of App. D on the eightfold P at
    N=32 (an independent seeded random field per entry): homogenizations in
    FP32-IR and FP64, A* checked against the oracle's stored value."""
    prob = W.eightfold_diagonal(32, 0)
    A_ref = np.array(gold["diag_eightfold_N32"]["A"])
    res = {"workload": "eightfold d=2 n=4 N=32, A = diag(a_1, a_2), 6 seeded random mode "
                       f"pairs per entry ({prob.g} modes)"}
    gp = qp.Problem(prob, precision="fp32ir", autotune=True)
    for prec in ("fp32ir", "fp64"):
        gp.set_options(precision=qp.QP_PREC_FP32_IR if prec == "fp32ir" else qp.QP_PREC_FP64)
        for _ in range(warmup):
            gp.homogenized(tol=TOL, energy=False)
        dt, lat, r, _ = run_steps(gp, steps, torch)
        res[prec] = {"value": round(prob.d * steps / dt, 2), "unit": "corrector solves/s",
                     "ms_per_step": round(dt / steps * 1e3, 4),
                     "p99_ms": round(float(np.percentile(np.array(lat), 99)), 4),
                     "astar_rel_err": float(np.abs(r.A - A_ref).max() / np.abs(A_ref).max()),
                     "iters": [i.iters for i in r.infos]}
    gp.close()
    return res


def batch_instances(torch, np, qp, W, reps: int = 3):
    """64 seeded eightfold instances with N drawn from {8, 12, 16, 24, 32}
    (16.2M unknowns for the default seed), two correctors each.  FP32-IR:
    homogenized together by qp_homogenized_grouped (one launch per solver
    step for all 64), by qp_homogenized_batch (each problem on its own
    stream), and one after another, on the same problems.  FP64 (the
    comparison leg): the same instances by qp_homogenized_batch and one after
    another.  Grouped and stream results are compared with the sequential
    ones bitwise, and the instances with N <= 12 with the oracle.  The work
    bound is the time of all instances' iterations at the best rate (per
    unknown and iteration) that an instance reaches when solved alone."""
    import oracle
    probs = W.eightfold_batch(64)
    solves = sum(pr.d for pr in probs)
    out = {}
    for prec in ("fp32ir", "fp64"):
        gps = [qp.Problem(pr, precision=prec, stream=torch.cuda.Stream(), autotune=True)
               for pr in probs]
        qp.homogenized_batch(gps, tol=TOL)  # warm-up (graphs, caches)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            As, _, st = qp.homogenized_batch(gps, tol=TOL)
        dt_b = (time.perf_counter() - t0) / reps
        if prec == "fp32ir":
            qp.homogenized_batch(gps, tol=TOL, grouped=True)  # warm-up (group tables)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(reps):
                Ag, _, stg = qp.homogenized_batch(gps, tol=TOL, grouped=True)
            dt_g = (time.perf_counter() - t0) / reps
            # the instances up to MIXED_GROUP_DIM unknowns grouped, the rest on streams
            qp.homogenized_batch(gps, tol=TOL, group_max_dim=MIXED_GROUP_DIM)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(reps):
                Am, _, stm = qp.homogenized_batch(gps, tol=TOL, group_max_dim=MIXED_GROUP_DIM)
            dt_m = (time.perf_counter() - t0) / reps
        seq = [gp.homogenized(tol=TOL, energy=False).A.copy() for gp in gps]
        # one after another, each homogenization timed on its own (it returns
        # A* to the host, so it has finished when the call returns)
        per = [0.0] * len(gps)
        iters = [0] * len(gps)
        for _ in range(reps):
            for i, gp in enumerate(gps):
                t1 = time.perf_counter()
                r = gp.homogenized(tol=TOL, energy=False)
                per[i] += time.perf_counter() - t1
                iters[i] = max(int(x.iters) for x in r.infos)
        dt_s = sum(per) / reps
        # work bound: every instance's iterations at the best rate per
        # unknown and iteration that any instance reaches alone
        rate = min(per[i] / reps / (probs[i].D * iters[i]) for i in range(len(gps)))
        bound = sum(probs[i].D * iters[i] for i in range(len(gps))) * rate
        leg = {"streams_value": round(solves / dt_b, 2), "streams_ms": round(dt_b * 1e3, 3),
               "streams_status": int(st),
               "streams_results_equal_sequential": all(np.array_equal(a, b) for a, b in zip(As, seq)),
               "sequential_value": round(solves / dt_s, 2), "sequential_ms": round(dt_s * 1e3, 3),
               "streams_speedup_vs_sequential": round(dt_s / dt_b, 3),
               "iterations_min_max": [min(iters), max(iters)],
               "work_bound_ms": round(bound * 1e3, 3),
               "streams_time_over_work_bound": round(dt_b / bound, 3)}
        if prec == "fp32ir":
            diff = max(float(np.abs(a - b).max() / np.abs(b).max()) for a, b in zip(Ag, seq))
            leg.update({"grouped_value": round(solves / dt_g, 2), "grouped_ms": round(dt_g * 1e3, 3),
                        "grouped_status": int(stg),
                        "grouped_results_equal_sequential": all(np.array_equal(a, b)
                                                                for a, b in zip(Ag, seq)),
                        "grouped_max_rel_diff_vs_sequential": diff,
                        "grouped_speedup_vs_sequential": round(dt_s / dt_g, 3),
                        "mixed_group_max_dim": MIXED_GROUP_DIM,
                        "mixed_grouped_instances": sum(1 for pr in probs
                                                       if pr.D <= MIXED_GROUP_DIM),
                        "mixed_value": round(solves / dt_m, 2), "mixed_ms": round(dt_m * 1e3, 3),
                        "mixed_status": int(stm),
                        "mixed_results_equal_sequential": all(np.array_equal(a, b)
                                                              for a, b in zip(Am, seq)),
                        "mixed_speedup_vs_sequential": round(dt_s / dt_m, 3),
                        "mixed_time_over_work_bound": round(dt_m / bound, 3)})
            leg["value"] = round(solves / min(dt_g, dt_b, dt_m), 2)
            leg["what"] = "the fastest of grouped_value, streams_value and mixed_value"
            # the grouped A* against the oracle for the small instances
            small = [i for i, pr in enumerate(probs) if pr.N <= 12][:6]
            errs = []
            for i in small:
                ref = oracle.homogenize(probs[i], tol=TOL).A
                errs.append(float(np.abs(Ag[i] - ref).max() / np.abs(ref).max()))
            leg["grouped_astar_rel_err_vs_oracle"] = {
                "instances": [f"#{i} N={probs[i].N}" for i in small], "max": max(errs)}
        else:
            leg["value"] = leg["streams_value"]
            leg["what"] = "streams_value"
        for gp in gps:
            gp.close()
        out[prec] = leg
    Ns = sorted(set(int(pr.N) for pr in probs))
    res = {"workload": f"64 seeded eightfold d=2 n=4 instances, N in {Ns} "
                       f"({sum(pr.D for pr in probs):,} unknowns), 2 correctors each",
           "unit": "corrector solves/s"}
    res.update(out["fp32ir"])
    res["fp64"] = out["fp64"]
    res["fp32ir_over_fp64"] = round(out["fp32ir"]["value"] / out["fp64"]["value"], 3)
    return res


def serving(torch, np, qp, W, requests: int = 400, load: float = 0.8):
    """Homogenization requests served by qp_server: icosahedral d=3 n=6
    problems at N = 6, 8, 12, 16 mixed with eightfold n=4 problems at
    N = 16, 24, 32, drawn uniformly (seeded).  For each precision (FP32-IR,
    then FP64 as the comparison leg): capacity with all requests queued at
    once, then the same mix as a seeded Poisson stream at `load` times that
    capacity, with each request's latency (arrival to result); then FP32-IR
    again under an HBM budget that holds only a few of the problems, so that
    admission waits for idle problems to be evicted."""
    kinds = [W.icosahedral(6), W.icosahedral(8), W.icosahedral(12), W.icosahedral(16),
             W.eightfold_random(16, 11), W.eightfold_random(24, 12),
             W.eightfold_random(32, 13)]
    rng = np.random.default_rng(W.BASE_SEED + 77)
    mix = [int(i) for i in rng.integers(0, len(kinds), size=requests)]
    gaps01 = rng.exponential(1.0, size=requests)  # unit-rate arrivals, scaled per run
    solves = sum(kinds[i].d for i in mix)

    def run(precision: str, budget: int, capacity=None):
        srv = qp.Server(budget, precision=precision, autotune=True)

        def drain(tickets):
            left, fin = set(tickets), {}
            while left:
                for t in srv.progress(wait_us=1000):
                    if t in left:
                        left.discard(t)
                        fin[t] = time.perf_counter()
            return fin

        drain([srv.submit(c, tol=TOL) for c in kinds])  # every problem created once
        if capacity is None:
            t0 = time.perf_counter()
            drain([srv.submit(kinds[i], tol=TOL) for i in mix])
            capacity = requests / (time.perf_counter() - t0)
        arrive = np.cumsum(gaps01 / (load * capacity))
        submitted, finish, tickets = {}, {}, []
        t0 = time.perf_counter()
        k = 0
        while len(finish) < requests:
            now = time.perf_counter() - t0
            while k < requests and arrive[k] <= now:
                t = srv.submit(kinds[mix[k]], tol=TOL)
                submitted[t] = t0 + arrive[k]
                tickets.append(t)
                k += 1
            wait = 1000 if k >= requests else int(max(50.0, min(1000.0, (arrive[k] - now) * 1e6)))
            for t in srv.progress(wait_us=wait):
                finish[t] = time.perf_counter()
        span = max(finish.values()) - t0
        lat = np.array([(finish[t] - submitted[t]) * 1e3 for t in tickets])
        bad = sum(1 for t in tickets if srv.result(t)[2] != qp.QP_OK)
        cached = srv.bytes()
        srv.close()
        return {"capacity_requests_per_s": round(capacity, 2),
                "capacity_solves_per_s": round(solves / requests * capacity, 2),
                "offered_requests_per_s": round(load * capacity, 2),
                "value": round(solves / span, 2), "unit": "corrector solves/s",
                "latency_ms": {"p50": round(float(np.percentile(lat, 50)), 3),
                               "p99": round(float(np.percentile(lat, 99)), 3),
                               "max": round(float(lat.max()), 3), "samples": int(lat.size)},
                "failed": bad, "cached_problem_bytes": int(cached)}

    res = {"workload": f"{requests} homogenization requests, icosahedral N 6/8/12/16 and eightfold "
                       "N 16/24/32 mixed uniformly; Poisson arrivals (seeded) at "
                       f"{load} x the measured capacity of each precision"}
    r32 = run("fp32ir", 96 << 30)
    res.update(r32)
    res["fp64"] = run("fp64", 96 << 30)
    res["fp32ir_over_fp64_capacity"] = round(r32["capacity_requests_per_s"] /
                                             res["fp64"]["capacity_requests_per_s"], 3)
    # a budget of 7 GiB holds the icosahedral N = 16 problem (6.8 GB of
    # workspace) and the small ones, not all seven at once: requests wait for
    # idle problems to be evicted
    budget = 7 << 30
    tight = run("fp32ir", budget, capacity=r32["capacity_requests_per_s"])
    tight["hbm_budget_bytes"] = budget
    res["tight_budget"] = tight
    return res


def cpu_baseline(prob):
    """The oracle, unmodified, on this host's cores: FP64 homogenizations of the
    same workload (two corrector solves at tol 1e-12 each), repeated until at
    least 10 s of CPU work have run; then one corrector solve on one thread."""
    import oracle
    threads = oracle.max_threads()
    reps, iters = 0, None
    t0 = time.perf_counter()
    while True:
        r = oracle.homogenize(prob, tol=TOL)
        reps += 1
        iters = [i.iters for i in r.infos]
        dt = time.perf_counter() - t0
        if dt >= 10.0 or reps >= 20:
            break
    # effective bandwidth: 32 B per unknown per stiffness product (FP64), one
    # product per PCG iteration
    gbs = 32.0 * prob.D * sum(iters) * reps / dt / 1e9
    oracle.set_threads(1)
    F = oracle.corrector_rhs(prob, 0)
    t1 = time.perf_counter()
    _, _, it1, _ = oracle.pcg(prob, F, tol=TOL)
    dt1 = time.perf_counter() - t1
    oracle.set_threads(threads)
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            model = next((ln.split(":", 1)[1].strip() for ln in f if ln.startswith("model name")), "")
    except OSError:
        pass
    return {"value": round(prob.d * reps / dt, 4), "unit": "corrector solves/s", "cores": threads,
            "kind": "oracle",
            "sample": f"{reps} homogenizations ({prob.d * reps} FP64 corrector solves, tol 1e-12, "
                      f"{iters} PCG iterations each) of the same workload, {dt:.2f} s",
            "effective_GBs": round(gbs, 2),
            "value_1_thread": round(1.0 / dt1, 4),
            "sample_1_thread": f"one FP64 corrector solve (j = 1, {it1} PCG iterations), "
                               f"{dt1:.2f} s",
            "host": {"cpu_model": model, "logical_cpus": os.cpu_count()}}


def main():
    args = parse_args()
    if args.copy_probe:
        copy_probe()
        return
    if args.product_probe:
        product_probe()
        return
    if args.batch_breakdown:
        batch_breakdown()
        return
    if args.config_table:
        config_table()
        return
    if args.small_sweep:
        small_sweep()
        return
    if args.gpus != 1:
        print(json.dumps({"error": "the solver runs on one GPU; --gpus must be 1 "
                                   "(independent solves shard by problem; one large solve "
                                   "would shard into slabs along the slowest axis)"}))
        sys.exit(2)
    import numpy as np
    import torch

    from paper_2404_06841_amd import qp
    from paper_2404_06841_amd import workloads as W

    prob = W.eightfold_random(32, 0)
    gold = json.load(open(os.path.join(ROOT, "tests", "golden", "oracle_astar.json")))
    A_ref = np.array(gold["c3_eightfold_random_N32"]["A"])

    # headline: FP32-IR with every full batch of iterations replayed as a HIP graph
    if args.layout:
        pin = [int(v) for v in args.layout.split(",")]
        if len(pin) != 6:
            raise SystemExit("--layout takes six integers: IT,WG,XF,IT64,WG64,XF64")
        gp = qp.Problem(prob, precision="fp32ir")
        gp.set_layout(*pin)
    else:
        gp = qp.Problem(prob, precision="fp32ir", autotune=True)
    for _ in range(args.warmup):
        gp.homogenized(tol=TOL, energy=False)
    dt, lat, r, _ = run_steps(gp, args.steps, torch)
    err_ir = float(np.abs(r.A - A_ref).max() / np.abs(A_ref).max())
    solves = prob.d * args.steps
    value = solves / dt
    if args.headline_only:
        print(json.dumps({"headline_only": round(value, 2), "steps": args.steps,
                          "astar_rel_err": err_ir, "layout": gp.layout()}), flush=True)
        gp.close()
        return
    # latency percentiles over more samples than the timed steps (outside the
    # timed region; each homogenization timed on its own)
    _, lat, _, _ = run_steps(gp, LATENCY_SAMPLES, torch)

    # the same steps with every float stiffness product bracketed by HIP events
    # on the library's stream (profiled batches are launched directly)
    gp.set_options(profile=1)
    gp.homogenized(tol=TOL, energy=False)
    dtp, _, rp, (mv_ms, mv_n, mv_rhs) = run_steps(gp, args.steps, torch)
    gp.set_options(profile=0)

    layout = gp.layout()
    # outside the timed region: the correctors themselves, to compare the two
    # precisions' solutions
    chi32 = [gp.corrector_d(j, tol=TOL)[0] for j in range(prob.d)]
    gp.close()

    # the same steps in plain FP64 (comparison, not the headline), on a problem
    # whose product layout is tuned for the FP64 launch
    gp = qp.Problem(prob, precision="fp64", autotune=True)
    layout64 = gp.layout()
    for _ in range(args.warmup):
        gp.homogenized(tol=TOL, energy=False)
    dt64, _, r64, _ = run_steps(gp, args.steps, torch)
    _, lat64, _, _ = run_steps(gp, LATENCY_SAMPLES, torch)
    err_64 = float(np.abs(r64.A - A_ref).max() / np.abs(A_ref).max())
    chi64 = [gp.corrector_d(j, tol=TOL)[0] for j in range(prob.d)]
    gp.close()
    chi_diff = max(float(torch.linalg.vector_norm(a - b) / torch.linalg.vector_norm(b))
                   for a, b in zip(chi32, chi64))
    del chi32, chi64

    D = prob.D
    # algorithmic bytes of a float product: read x once, write y once (16 B per
    # unknown) for every right-hand side the launch served
    algo_bytes = 16.0 * D * (mv_rhs / mv_n) if mv_n else 16.0 * D
    avg_s = (mv_ms / mv_n) * 1e-3 if mv_n else float("nan")
    achieved = algo_bytes / avg_s / 1e9 if mv_n else None
    float_layout = (layout["item_tiles"], layout["workgroups"], layout["xcd_front"])
    traffic = measured_traffic(layout=float_layout)
    roofline = {"bound": "hbm", "achieved": round(achieved, 1) if achieved else None,
                "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4) if achieved else None,
                "traffic": traffic,
                "kernel": "k_matvec_plane<float> (FP32 stiffness product inside FP32-IR, "
                          "both correctors per launch)",
                "launches": mv_n, "rhs_per_launch": round(mv_rhs / mv_n, 3) if mv_n else None,
                "avg_launch_us": round(avg_s * 1e6, 2) if mv_n else None,
                "algorithmic_bytes_per_launch": round(algo_bytes),
                "timing": "HIP event pair recorded by each launch itself (hipExtLaunchKernelGGL) "
                          "on the library's stream, in a second pass of the same steps "
                          "(profiled batches run without graph replay)",
                "profiled_pass_value": round(solves / dtp, 2),
                "layout": layout}
    lat_sorted = np.sort(np.array(lat))
    # the same roofline for the product at the HBM-sized shape (icosahedral
    # N = 16, FP64, one right-hand side), where the vectors do not fit the
    # caches; traffic from the committed sized-request counter summary
    hbm = hbm_products(torch, qp, W)
    h64 = hbm["fp64"]
    hl = hbm["layout"]
    traffic64 = measured_traffic(TRAFFIC_FILE_HBM, "fp64_bytes_per_launch",
                                 (hl["item_tiles64"], hl["workgroups64"], hl["xcd_front64"]))
    roofline_hbm = {"bound": "hbm", "achieved": h64["achieved_GBs"], "peak": HBM_PEAK_GBS,
                    "unit": "GB/s", "frac": round(h64["achieved_GBs"] / HBM_PEAK_GBS, 4),
                    "traffic": traffic64,
                    "kernel": "k_matvec_plane<double> (FP64 stiffness product, one right-hand side), "
                              "icosahedral d=3 n=6 N=16 (16,777,216 unknowns)",
                    "avg_launch_us": h64["avg_launch_us"],
                    "algorithmic_bytes_per_launch": h64["algorithmic_bytes"],
                    "memory_side_GBs": (round(traffic64 / (h64["avg_launch_us"] * 1e-6) / 1e9, 1)
                                        if traffic64 else None),
                    "copy_GBs": hbm["copy_GBs"], "frac_of_copy": h64["frac_of_copy"],
                    "profile_mean_us": measured_traffic(
                        TRAFFIC_FILE_HBM, "fp64_mean_duration_us",
                        (hl["item_tiles64"], hl["workgroups64"], hl["xcd_front64"])),
                    "timing": "HIP event pair recorded by each launch itself "
                              "(hipExtLaunchKernelGGL) on the library's stream"}
    out = {
        "metric": METRIC,
        "value": round(value, 2),
        "unit": "corrector solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(dt / args.steps * 1e3, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64",
        "data": "synthetic",
        "config": {"workload": "eightfold d=2 n=4 N=32 (1,048,576 unknowns), 8 seeded random "
                               "mode pairs around mean 3; 2 correctors + A* per step",
                   "N": 32, "n": 4, "d": 2, "unknowns": D, "modes": int(prob.g), "tol": TOL,
                   "precision": "fp32-ir", "parallelism": "single GPU"},
        "astar_rel_err": err_ir,
        "latency_ms": {"what": "one homogenization (both corrector solves + A*), "
                               f"{len(lat_sorted)} samples",
                       "p50": round(float(np.percentile(lat_sorted, 50)), 4),
                       "p99": round(float(np.percentile(lat_sorted, 99)), 4)},
        "fp64": {"value": round(solves / dt64, 2), "ms_per_step": round(dt64 / args.steps * 1e3, 4),
                 "astar_rel_err": err_64,
                 "p99_ms": round(float(np.percentile(np.array(lat64), 99)), 4),
                 "iters": [i.iters for i in r64.infos], "layout": layout64},
        "solution": {"what": "corrector solves at tol 1e-12: final relative residual per "
                             "corrector (FP32-IR: the true FP64 residual ||F' - Q chi|| / ||F'||; "
                             "FP64: the PCG residual), and the largest "
                             "||chi_fp32ir - chi_fp64|| / ||chi_fp64|| over the correctors",
                     "rel_resid_fp32ir": [i.rel_resid for i in r.infos],
                     "rel_resid_fp64": [i.rel_resid for i in r64.infos],
                     "corrector_rel_diff": chi_diff},
        "fp32ir_iters": [i.iters for i in r.infos],
        "fp32ir_replacements": [i.outer_iters for i in r.infos],
        "roofline": roofline,
        "diagonal_coefficient": diagonal_workload(torch, np, qp, W, gold,
                                                  max(5, args.steps // 2), args.warmup),
        "hbm_products": hbm,
        "roofline_hbm": roofline_hbm,
        "half_storage": half_storage(torch, np, qp, W, gold),
        "batch_instances": batch_instances(torch, np, qp, W),
        "stored_matrix": stored_matrix(torch, qp, W),
        "sampled_inputs": sampled_inputs(torch, qp),
        "serving": serving(torch, np, qp, W),
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(prob)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
