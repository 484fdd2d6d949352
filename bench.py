"""Benchmark of the implicit viscous PCG solve on one MI355X.

Workload (default): the production-like FP64 solve, a 256 x 320 x 640
spherical-shell grid (52.4M cells), radial stretching 1.01, a smooth random
viscosity field with 100x contrast, diffusion number 1000 and a smoothed
N(0,1) right-hand side, solved to ||b - A x|| <= 1e-10 ||b||.  Inputs are
seeded and synthetic; they are generated on the host and copied to HBM
before the timed region.

One step = build the operator from (nu, dt) + one full FP64 PCG solve to the
tolerance.  `value` is PCG iterations per second of wall time over the K
timed steps.  Alongside, on the same grid and data: the operator build on
its own; the single-precision inner PCG inside double-precision refinement
(both strategies); the adjoint; the paper's second preconditioner
(block-Jacobi ILU(0)) in FP64 and inside refinement; three components under
the same operator; one explicit RKL2 super time-step of the same dt.  Then
the 65,536-cell grid (latency-bound iterations/s), the 96M-cell stress case
(refined forward solves and the adjoint), streaming probes with the kernels'
byte mixes, and the FP64 CPU oracle on the host cores.

The dominant kernel is the fused PCG iteration kernel; its duration is
sampled with HIP events on the solver's stream (inside the library) and
converted to algorithmic HBM bytes per second.

    python bench.py [--steps K] [--warmup W] [--gpus 1] [--workload c1]
                    [--no-cpu-baseline] [--no-refined] [--no-sts] [--no-multi] [--no-pc2]
                    [--no-adjoint] [--no-c0] [--no-c4] [--no-probe]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# Algorithmic bytes of one Jacobi-PCG iteration per cell in its fused
# two-kernel form (SpMV with the p update, then the r update with the Jacobi
# step and the dots; the stored operator streamed once): 14 words.
ALG_BYTES_PER_CELL = {"fp64": 14 * 8, "fp32": 14 * 4}
# What this library's single-kernel iteration has to move per cell: reads r,
# q, p, c_r, c_theta, c_phi and writes r, p, q in every launch; every second
# launch also reads x and the previous p and writes x (it moves x over two
# iterations): 10.5 words on average (12 and 9 in alternate launches).
KERNEL_BYTES_PER_CELL = {"fp64": 21 * 4, "fp32": 21 * 2}
# One RKL2 stage kernel per cell: reads D_{j-1}, nu, D_{j-2}, L_0, writes D_j.
STS_BYTES_PER_CELL = 5 * 8        # one-stage kernel: reads X, nu, Z, L0; writes the stage
STS_PAIR_BYTES_PER_CELL = 6 * 8   # two-stage kernel: reads X, nu, Z, L0; writes both stages
GRAD_BYTES_PER_CELL = 4 * 8       # gradient kernel: reads x, lambda; writes dL/dnu, dL/drhs
CSRC = os.path.join(ROOT, "paper_1811_02605_amd", "csrc")
KERNEL_SRC = os.path.join(CSRC, "kernels.hpp")
STS_KERNEL_SRC = os.path.join(CSRC, "sts_kernels.hpp")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "pcg_iter_fp64_c1_traffic.txt")
STS_TRAFFIC_FILE = os.path.join(ROOT, "profiles", "sts_stage_c1_traffic.txt")
STS_PAIR_TRAFFIC_FILE = os.path.join(ROOT, "profiles", "sts_pair_c1_traffic.txt")
GRAD_TRAFFIC_FILE = os.path.join(ROOT, "profiles", "gradient_c1_kernel_trace.txt")


def kernel_hash(*paths) -> str:
    h = hashlib.sha256()
    for path in paths or (KERNEL_SRC,):
        h.update(open(path, "rb").read())
    return h.hexdigest()[:16]


def read_traffic(path=TRAFFIC_FILE, srcs=(KERNEL_SRC,)):
    """HBM bytes per launch of a kernel from its committed PMC summary, if the
    summary was taken on the current kernel source; else None."""
    if not os.path.exists(path):
        return None
    txt = open(path).read()
    m_hash = re.search(r"kernel_source_sha256_16:\s*([0-9a-f]+)", txt)
    m_bytes = re.search(r"hbm_bytes_per_launch:\s*([0-9.eE+]+)", txt)
    if not m_hash or not m_bytes or m_hash.group(1) != kernel_hash(*srcs):
        return None
    return float(m_bytes.group(1))


def _cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(p, x_gpu=None, budget_iters=400, single_iters=12):
    """The FP64 CPU oracle, as it stands, built -O3 -march=native on this
    host, on the same workload: assemble, then its Jacobi-PCG from x0 = 0 to
    the same 1e-10 tolerance (bounded at budget_iters iterations); PCG
    iterations per second on all the host threads OpenMP uses and on one.
    Also full solves of the 65,536-cell grid and the 9.4M-cell gradient-check
    grid's forward system, and (x_gpu) the oracle's residual of the GPU
    solutions on the benchmark grid."""
    import oracle
    from paper_1811_02605_amd import workloads as W

    oracle.use_native_build()
    threads = oracle.max_threads()
    out = {"unit": "PCG iters/s", "cores": threads, "kind": "oracle",
           "build": "gcc " + " ".join(oracle.NATIVE_FLAGS) + " -fopenmp",
           "cpu_model": _cpu_model(), "nproc": len(os.sched_getaffinity(0)),
           "omp_threads": threads}
    t0 = time.perf_counter()
    ora = oracle.Operator(p.r_faces, p.t_faces, p.cfg.np_, p.nu, p.dt)
    b = ora.rhs_to_b(p.rhs)
    t1 = time.perf_counter()
    _, iters, _, rel_true = ora.pcg(b, tol=p.cfg.rtol, max_iters=budget_iters)
    t2 = time.perf_counter()
    out["value"] = iters / (t2 - t1)
    out["sample"] = (f"{p.cfg.name} grid {p.cfg.nr}x{p.cfg.nt}x{p.cfg.np_}: oracle PCG from x0=0 "
                     f"on {threads} threads, {iters} iterations to rel. residual {rel_true:.2e} "
                     f"in {t2 - t1:.1f} s (time to solution; at most {budget_iters} iterations); "
                     f"assembly {t1 - t0:.1f} s not counted")
    out["time_to_tol_s"] = (t2 - t1) if rel_true <= p.cfg.rtol else None
    if x_gpu:
        out["gpu_solutions_rel_resid_by_oracle"] = {k: ora.rel_residual(b, v) for k, v in x_gpu.items()}
    # one core: a bounded sample of the same solve
    oracle.set_threads(1)
    t3 = time.perf_counter()
    _, it1, _, _ = ora.pcg(b, tol=0.0, max_iters=single_iters)
    t4 = time.perf_counter()
    out["single_core"] = {"value": it1 / (t4 - t3), "unit": "PCG iters/s", "cores": 1,
                          "sample": f"{p.cfg.name}: {it1} oracle PCG iterations on one thread, "
                                    f"{t4 - t3:.1f} s"}
    oracle.set_threads(threads)
    del ora
    # full solves of the two smaller configurations
    for name in ("c0", "c3"):
        q = W.make_problem(W.CONFIGS[name])
        o2 = oracle.Operator(q.r_faces, q.t_faces, q.cfg.np_, q.nu, q.dt)
        b2 = o2.rhs_to_b(q.rhs)
        t5 = time.perf_counter()
        _, it2, _, res2 = o2.pcg(b2, tol=q.cfg.rtol)
        t6 = time.perf_counter()
        out[name] = {"iters": it2, "time_to_tol_s": t6 - t5, "iters_per_s": it2 / (t6 - t5),
                     "rel_resid": res2, "cells": q.cfg.n,
                     "what": f"{name} {q.cfg.nr}x{q.cfg.nt}x{q.cfg.np_} FP64 Jacobi-PCG to "
                             f"{q.cfg.rtol:g} from x0=0 on {threads} threads"}
        del o2
    return out


def bench_build(S, grid, nu, p, reps=5):
    """The operator build on its own (mas_op_build: geometry upload, the
    one-pass build kernel, the validity read-back), host clock around the
    blocking call, after a warm-up; FP64 and with single-precision copies."""
    import numpy as np
    import torch

    res = {"what": "mas_op_build alone (host clock around the blocking call, median of "
                   f"{reps}): w, three scaled couplings and the copy of nu (48 B/cell moved; "
                   "60 B/cell with single-precision copies)"}
    for prec, bpc in (("fp64", 48), ("fp32_refined", 60)):
        S.Operator(grid, nu, p.dt, precision=prec)
        torch.cuda.synchronize()
        ts = []
        for _ in range(reps):
            t0 = time.perf_counter()
            op = S.Operator(grid, nu, p.dt, precision=prec)
            ts.append(time.perf_counter() - t0)
            del op
        ms = 1e3 * float(np.median(ts))
        res[prec] = {"ms": ms, "bytes_per_cell": bpc,
                     "GBs_at_host_time": bpc * grid.n / (ms * 1e-3) / 1e9}
    print(f"[bench] op build: {res['fp64']['ms']:.3f} ms (fp64), {res['fp32_refined']['ms']:.3f} ms "
          "(with fp32 copies)", file=sys.stderr, flush=True)
    return res


def bench_c0(S, W, dev, reps=20):
    """The 65,536-cell grid (32 x 32 x 64): cache-resident and latency-bound,
    iterations per second of full FP64 solves (and through the
    allocation-free entry point)."""
    import numpy as np
    import torch

    q = W.make_problem(W.CONFIGS["c0"])
    g0 = S.Grid.from_problem(q)
    nu0 = torch.from_numpy(q.nu).to(dev)
    rhs0 = torch.from_numpy(q.rhs).to(dev)
    x0 = torch.empty_like(rhs0)
    op = S.Operator(g0, nu0, q.dt)

    def timed(solve, o):
        solve(rhs0, o, out=x0, allow_notconv=False)
        runs = [solve(rhs0, o, out=x0, allow_notconv=False)[1] for _ in range(reps)]
        return float(np.median([r["seconds"] for r in runs])), runs[-1]

    o = S.make_opts(rtol=q.cfg.rtol)
    t, last = timed(op.solve, o)
    t_pi, last_pi = timed(op.solve, S.make_opts(rtol=q.cfg.rtol, launch="per_iteration"))
    t_na, last_na = timed(op.solve_noalloc, o)
    it = last["iters"]
    mode = {1: "per_iteration", 2: "persistent"}.get(last["launch"], "none")
    print(f"[bench] c0: {it} iterations, {1e3 * t:.2f} ms ({it / t:.0f} iters/s, {mode} launch); "
          f"launched per iteration {1e3 * t_pi:.2f} ms; allocation-free {1e3 * t_na:.2f} ms",
          file=sys.stderr, flush=True)
    return {"what": "c0: 32x32x64 (65,536 cells) FP64 Jacobi-PCG to 1e-10, median of "
                    f"{reps} solves (cache-resident, latency-bound: no HBM fraction)",
            "cells": q.cfg.n, "iters": it, "time_to_tol_s": t, "iters_per_s": it / t,
            "launch": mode, "rel_resid_true": last["rel_resid_true"],
            "per_iteration_launch": {"time_to_tol_s": t_pi, "iters_per_s": last_pi["iters"] / t_pi},
            "noalloc": {"time_to_tol_s": t_na, "iters_per_s": last_na["iters"] / t_na}}


def bench_c4(S, W, dev):
    """The 96M-cell stress case (300 x 400 x 800, clustered theta, 1000x
    viscosity contrast, diffusion number 5000): the FP32/FP64-refined forward
    solve with PC1 and with PC2, and the adjoint (refined PC2 solve plus the
    gradient kernel), each after a warm-up."""
    import numpy as np
    import torch

    q = W.make_problem(W.CONFIGS["c4"])
    g4 = S.Grid.from_problem(q)
    nu4 = torch.from_numpy(q.nu).to(dev)
    rhs4 = torch.from_numpy(q.rhs).to(dev)
    x4 = torch.empty_like(rhs4)
    op = S.Operator(g4, nu4, q.dt, precision="fp32_refined")
    res = {"what": "c4: 300x400x800 (96M cells) stress case, FP32 inner / FP64 refinement to 1e-10",
           "cells": q.cfg.n}
    for name, kw in (("refined_pc1", {}), ("refined_pc2", {"precond": "pc2"})):
        o = S.make_opts(rtol=q.cfg.rtol, precision="fp32_refined", **kw)
        op.solve(rhs4, o, out=x4, allow_notconv=False)
        runs = [op.solve(rhs4, o, out=x4, allow_notconv=False)[1] for _ in range(2)]
        res[name] = {"time_to_tol_s": float(np.median([r["seconds"] for r in runs])),
                     "inner_iters": runs[-1]["iters"], "outer_iters": runs[-1]["outer_iters"],
                     "rel_resid_true": runs[-1]["rel_resid_true"]}
    gx = torch.from_numpy(np.random.default_rng(GX_SEED).standard_normal(g4.shape)).to(dev)
    o = S.make_opts(rtol=q.cfg.rtol, precision="fp32_refined", precond="pc2", sample_timing=0)
    op.adjoint(x4, gx, o, allow_notconv=False)
    torch.cuda.synchronize()
    ts = []
    for _ in range(2):
        t0 = time.perf_counter()
        _, _, _, ia = op.adjoint(x4, gx, o, allow_notconv=False)
        torch.cuda.synchronize()
        ts.append(time.perf_counter() - t0)
    res["adjoint_refined_pc2"] = {"time_s": float(np.median(ts)), "inner_iters": ia["iters"],
                                  "outer_iters": ia["outer_iters"],
                                  "rel_resid_true": ia["rel_resid_true"]}
    res["forward_plus_adjoint_s"] = res["refined_pc2"]["time_to_tol_s"] + res["adjoint_refined_pc2"]["time_s"]
    print(f"[bench] c4: refined PC1 {res['refined_pc1']['time_to_tol_s']:.3f} s, refined PC2 "
          f"{res['refined_pc2']['time_to_tol_s']:.3f} s, adjoint {res['adjoint_refined_pc2']['time_s']:.3f} s",
          file=sys.stderr, flush=True)
    return res


# One iteration kernel with m right-hand sides: the couplings (3 words) once,
# 7.5 words per right-hand side on average (6 in every launch, x and the
# previous p read and x written in every second one).
def multi_bytes_per_cell(m, word=8):
    return (3 + 7.5 * m) * word


def bench_multi(S, W, grid, nu, p, t_pcg, k_single_us, m=3):
    """The three components of a vector field under the same operator, solved
    together (one iteration kernel carries all three) to the same tolerance."""
    import numpy as np
    import torch

    op = S.Operator(grid, nu, p.dt, precision="fp64")
    B = torch.from_numpy(W.component_rhs(p.cfg, m)).to(nu.device)
    X = torch.empty_like(B)
    o = S.make_opts(rtol=p.cfg.rtol, sample_timing=1)
    op.solve_multi(B, o, out=X, allow_notconv=False)  # warm-up
    runs = [op.solve_multi(B, o, out=X, allow_notconv=False)[1] for _ in range(2)]
    t = float(np.median([r[0]["seconds"] for r in runs]))
    k_us = runs[-1][0]["iter_kernel_us"] or None
    gbs = multi_bytes_per_cell(m) * grid.n / (k_us * 1e-6) / 1e9 if k_us else None
    print(f"[bench] {m} components: {t:.3f} s, kernel {k_us} us", file=sys.stderr, flush=True)
    # the same components with PC2 (one SpMV launch for all, block solves each)
    o2 = S.make_opts(rtol=p.cfg.rtol, precond="pc2", sample_timing=1)
    op.solve_multi(B, o2, out=X, allow_notconv=False)  # warm-up
    runs2 = [op.solve_multi(B, o2, out=X, allow_notconv=False)[1] for _ in range(2)]
    t2 = float(np.median([r[0]["seconds"] for r in runs2]))
    print(f"[bench] {m} components with PC2: {t2:.3f} s", file=sys.stderr, flush=True)
    # the same components with the single-precision inner PCG inside
    # double-precision refinement, PC2 and PC1 (one operator with FP32 copies)
    del op
    opr = S.Operator(grid, nu, p.dt, precision="fp32_refined")
    ref = {}
    for precond in ("pc2", "pc1"):
        o3 = S.make_opts(rtol=p.cfg.rtol, precision="fp32_refined", precond=precond)
        opr.solve_multi(B, o3, out=X, allow_notconv=False)  # warm-up
        runs3 = [opr.solve_multi(B, o3, out=X, allow_notconv=False)[1] for _ in range(2)]
        single = [opr.solve(B[h].contiguous(), o3, allow_notconv=False)[1]["seconds"] for h in range(m)]
        t3 = float(np.median([r[0]["seconds"] for r in runs3]))
        ref[precond] = {"time_to_tol_s": t3, "inner_iters": [r["iters"] for r in runs3[-1]],
                        "outer_iters": [r["outer_iters"] for r in runs3[-1]],
                        "three_single_refined_solves_s": sum(single),
                        "speedup_vs_single_refined_solves": sum(single) / t3}
        print(f"[bench] {m} components refined {precond}: {t3:.3f} s (three single refined solves "
              f"{sum(single):.3f} s)", file=sys.stderr, flush=True)
    return {
        "what": f"{m} right-hand sides (components) under the same operator, one FP64 solve to "
                "1e-10 each, one iteration kernel carrying all of them",
        "rhs": m, "iters": [r["iters"] for r in runs[-1]],
        "time_to_tol_s": t, "time_per_rhs_s": t / m,
        "speedup_vs_separate_solves": m * t_pcg / t,
        "kernel_us": k_us, "kernel_us_per_rhs": (k_us / m) if k_us else None,
        "kernel_speedup_per_rhs_vs_single": (m * k_single_us / k_us) if k_us else None,
        "bytes_per_cell": multi_bytes_per_cell(m),
        "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
        "frac": (gbs / HBM_PEAK_GBS) if gbs else None,
        "pc2": {"what": "the same components with block-Jacobi ILU(0): per iteration one SpMV "
                        "launch and one block-solve launch carry all of them; factor included",
                "iters": [r["iters"] for r in runs2[-1]], "time_to_tol_s": t2,
                "speedup_vs_pc1_together": t / t2,
                "iteration_us": runs2[-1][0]["iter_kernel_us"] or None},
        "refined": {"what": "the same components with the single-precision inner PCG inside "
                            "double-precision refinement (one launch per step carries all of them)",
                    **ref},
    }


def bench_pc2(S, grid, nu, rhs, p, t_pcg, iters_pc1):
    """The paper's second preconditioner on the same solve: block-Jacobi with
    an ILU(0) factor per 8 x 8 x 64 block (factor included in the time)."""
    import numpy as np

    op = S.Operator(grid, nu, p.dt, precision="fp64")
    o = S.make_opts(rtol=p.cfg.rtol, precond="pc2", sample_timing=1)
    op.solve(rhs, o, allow_notconv=False)  # warm-up
    runs = [op.solve(rhs, o, allow_notconv=False)[1] for _ in range(3)]
    t = float(np.median([r["seconds"] for r in runs]))
    print(f"[bench] PC2: {runs[-1]['iters']} iterations, {t:.3f} s", file=sys.stderr, flush=True)
    x64 = op.solve(rhs, o, allow_notconv=False)[0]
    del op
    # single-precision PC2-PCG inside double-precision refinement
    opr = S.Operator(grid, nu, p.dt, precision="fp32_refined")
    orf = S.make_opts(rtol=p.cfg.rtol, precision="fp32_refined", precond="pc2", sample_timing=1)
    opr.solve(rhs, orf, allow_notconv=False)  # warm-up
    rr = [opr.solve(rhs, orf, allow_notconv=False) for _ in range(3)]
    tr = float(np.median([r[1]["seconds"] for r in rr]))
    xr, ir = rr[-1]
    diff = float((xr - x64).norm() / x64.norm())
    print(f"[bench] PC2 refined: {ir['iters']} inner iterations, {ir['outer_iters']} outer, "
          f"{tr:.3f} s", file=sys.stderr, flush=True)
    return {
        "what": "the same FP64 solve with block-Jacobi ILU(0) (8 x 8 x 64 blocks) in place of "
                "point Jacobi; time includes forming the factor",
        "iters": runs[-1]["iters"], "iters_pc1": iters_pc1,
        "time_to_tol_s": t, "speedup_vs_pc1": t_pcg / t,
        "iteration_us": runs[-1]["iter_kernel_us"] or None,
        "rel_resid_true": runs[-1]["rel_resid_true"],
        "refined": {"what": "single-precision PC2-PCG inside double-precision refinement "
                            "(restarted at each refinement step), factor included",
                    "time_to_tol_s": tr, "speedup_vs_fp64_pc1": t_pcg / tr,
                    "speedup_vs_fp64_pc2": t / tr, "inner_iters": ir["iters"],
                    "outer_iters": ir["outer_iters"], "rel_resid_true": ir["rel_resid_true"],
                    "iteration_us": ir["iter_kernel_us"] or None,
                    "rel_diff_vs_fp64_pc2_solution": diff},
    }


GX_SEED = 600  # dL/dx of the adjoint measurement: N(0,1) per cell


def bench_adjoint(S, grid, nu, x, p, opts, t_pcg):
    """The adjoint of the same solve: for a loss with dL/dx = gx (seeded N(0,1)
    field) at the FP64 solution x, lambda = A^-1 gx by the same PCG, then one
    pass of the gradient kernel (dL/dnu, dL/drhs); timed on the host around
    the blocking call."""
    import numpy as np
    import torch

    op = S.Operator(grid, nu, p.dt, precision="fp64")
    gx = torch.from_numpy(np.random.default_rng(GX_SEED).standard_normal(grid.shape)).to(x.device)
    op.adjoint(x, gx, opts, allow_notconv=False)  # warm-up
    torch.cuda.synchronize()
    ts = []
    for _ in range(3):
        t0 = time.perf_counter()
        _, _, _, info = op.adjoint(x, gx, opts, allow_notconv=False)
        torch.cuda.synchronize()
        ts.append(time.perf_counter() - t0)
    t = float(np.median(ts))
    print(f"[bench] adjoint: {info['iters']} iterations, {t:.3f} s (solve and gradient); "
          f"gradient kernel {info['grad_kernel_us']:.1f} us", file=sys.stderr, flush=True)
    kus = info["grad_kernel_us"]
    achieved = GRAD_BYTES_PER_CELL * grid.n / (kus * 1e-6) / 1e9
    del op
    # the same adjoint with PC2 inside refinement (the fastest solver here)
    opr = S.Operator(grid, nu, p.dt, precision="fp32_refined")
    orf = S.make_opts(rtol=p.cfg.rtol, precision="fp32_refined", precond="pc2")
    opr.adjoint(x, gx, orf, allow_notconv=False)  # warm-up
    torch.cuda.synchronize()
    tr = []
    for _ in range(3):
        t0 = time.perf_counter()
        _, _, _, infr = opr.adjoint(x, gx, orf, allow_notconv=False)
        torch.cuda.synchronize()
        tr.append(time.perf_counter() - t0)
    t_r = float(np.median(tr))
    print(f"[bench] adjoint with refined PC2: {infr['iters']} inner iterations, {t_r:.3f} s",
          file=sys.stderr, flush=True)
    return {"what": "adjoint of the FP64 solve: lambda = A^-1 gx by the same PCG to 1e-10, then "
                    "dL/dnu and dL/drhs in one gradient-kernel pass (4 words/cell)",
            "time_s": t, "iters": info["iters"], "rel_resid_true": info["rel_resid_true"],
            "iteration_kernel_us": info["iter_kernel_us"] if info["iter_kernel_samples"] > 0 else None,
            "forward_plus_adjoint_s": t_pcg + t,
            "gradient_kernel": {"bound": "hbm", "kernel": "k_gradient", "kernel_us": kus,
                                "alg_bytes_per_cell": GRAD_BYTES_PER_CELL, "achieved": achieved,
                                "peak": 8000.0, "unit": "GB/s", "frac": achieved / 8000.0,
                                "traffic": read_traffic(GRAD_TRAFFIC_FILE)},
            "pc2_refined": {"what": "the same adjoint with single-precision PC2-PCG inside "
                                    "double-precision refinement",
                            "time_s": t_r, "inner_iters": infr["iters"],
                            "outer_iters": infr["outer_iters"],
                            "rel_resid_true": infr["rel_resid_true"]}}


def bench_sts(S, grid, nu, rhs, p, t_pcg, steps):
    """The explicit alternative for the same viscous step: one RKL2 super
    time-step of the same dt on the same grid and viscosity (u0 = the smooth
    right-hand-side field), timed with events on the library's stream; stages
    two per kernel (the default) and one per kernel."""
    import torch

    op = S.Operator(grid, nu, p.dt, precision="fp64")

    def run(pairs):
        u = rhs.clone()
        op.sts_step(u, stage_pairs=pairs)  # warm-up (first touch of the stage workspace)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(steps):
            op.sts_step(u, out=u, stage_pairs=pairs)
        e1.record()
        torch.cuda.synchronize()
        # the general kernels' mean, from one more step with the library's events
        _, info = op.sts_step(u, out=u, sample_timing=True, stage_pairs=pairs)
        k_us = info["stage_kernel_us"] if info["stage_kernel_samples"] > 0 else None
        return e0.elapsed_time(e1) * 1e-3 / steps, k_us, info

    step_s, k_us, info = run(True)
    step1_s, k1_us, info1 = run(False)
    paired = info["stages_per_kernel"] == 2
    bpc = STS_PAIR_BYTES_PER_CELL if paired else STS_BYTES_PER_CELL
    gbs = bpc * grid.n / (k_us * 1e-6) / 1e9 if k_us else None
    gbs1 = STS_BYTES_PER_CELL * grid.n / (k1_us * 1e-6) / 1e9 if k1_us else None
    print(f"[bench] RKL2: {info['stages']} stages, {1e3 * step_s:.2f} ms per step (stage kernel "
          f"{k_us} us, {info['stages_per_kernel']} stages each); one stage per kernel "
          f"{1e3 * step1_s:.2f} ms (kernel {k1_us} us)", file=sys.stderr, flush=True)
    return {
        "what": "one RKL2 super time-step of the same dt, nu and grid (explicit alternative to "
                "the implicit solve)",
        "stages": info["stages"], "z_max": info["z_max"],
        "stages_per_kernel": info["stages_per_kernel"],
        "step_ms": 1e3 * step_s,
        "speedup_vs_fp64_pcg_solve": t_pcg / step_s,
        "step_ms_one_stage_per_kernel": 1e3 * step1_s,
        "roofline": {"bound": "hbm",
                     "kernel": ("k_sts_pair (two RKL2 stages per launch)" if paired
                                else "k_sts_stage (one RKL2 stage)"),
                     "alg_bytes_per_cell": bpc, "kernel_us": k_us,
                     "kernel_us_per_stage": (k_us / info["stages_per_kernel"]) if k_us else None,
                     "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": (gbs / HBM_PEAK_GBS) if gbs else None,
                     "samples": info["stage_kernel_samples"],
                     "traffic": read_traffic(STS_PAIR_TRAFFIC_FILE if paired else STS_TRAFFIC_FILE,
                                             (STS_KERNEL_SRC, KERNEL_SRC))},
        "one_stage_kernel": {"kernel": "k_sts_stage", "alg_bytes_per_cell": STS_BYTES_PER_CELL,
                             "kernel_us": k1_us, "achieved": gbs1,
                             "frac": (gbs1 / HBM_PEAK_GBS) if gbs1 else None,
                             "traffic": read_traffic(STS_TRAFFIC_FILE, (STS_KERNEL_SRC, KERNEL_SRC))},
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="c1")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-refined", action="store_true")
    ap.add_argument("--no-sts", action="store_true")
    ap.add_argument("--no-multi", action="store_true")
    ap.add_argument("--no-pc2", action="store_true")
    ap.add_argument("--no-adjoint", action="store_true")
    ap.add_argument("--no-build", action="store_true")
    ap.add_argument("--no-c0", action="store_true")
    ap.add_argument("--no-c4", action="store_true")
    ap.add_argument("--no-probe", action="store_true")
    ap.add_argument("--check-every", type=int, default=8)
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: the library runs on one GPU; --gpus {args.gpus} is not supported "
              "(the multi-GPU r-slab decomposition is a design note, not code).", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_1811_02605_amd import solver as S
    from paper_1811_02605_amd import workloads as W

    dev = "cuda:0"
    cfg = W.CONFIGS[args.workload]
    t_gen = time.perf_counter()
    p = W.make_problem(cfg)
    t_gen = time.perf_counter() - t_gen
    print(f"[bench] inputs {cfg.name} {cfg.shape} generated in {t_gen:.1f} s", file=sys.stderr,
          flush=True)
    grid = S.Grid.from_problem(p)
    nu = torch.from_numpy(p.nu).to(dev)
    rhs = torch.from_numpy(p.rhs).to(dev)
    x = torch.empty_like(rhs)
    torch.cuda.synchronize()

    opts = S.make_opts(rtol=cfg.rtol, precision="fp64", sample_timing=1,
                       check_every=args.check_every)

    def step():
        op = S.Operator(grid, nu, p.dt, precision="fp64")
        _, info = op.solve(rhs, opts, out=x, allow_notconv=False)
        return info

    for w in range(args.warmup):
        info = step()
        print(f"[bench] warmup {w}: {info['iters']} iterations, {info['seconds']:.3f} s",
              file=sys.stderr, flush=True)

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    infos = [step() for _ in range(args.steps)]
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    iters = sum(i["iters"] for i in infos)
    solve_s = [i["seconds"] for i in infos]
    kus = [i["iter_kernel_us"] for i in infos if i["iter_kernel_samples"] > 0]
    kernel_us = float(np.mean(kus)) if kus else None
    print(f"[bench] {args.steps} steps, {iters} iterations in {elapsed:.3f} s; "
          f"iteration kernel {kernel_us} us", file=sys.stderr, flush=True)

    n = cfg.n
    alg_bytes = ALG_BYTES_PER_CELL["fp64"] * n
    achieved = alg_bytes / (kernel_us * 1e-6) / 1e9 if kernel_us else None
    kern_gbs = KERNEL_BYTES_PER_CELL["fp64"] * n / (kernel_us * 1e-6) / 1e9 if kernel_us else None
    traffic = read_traffic()

    out = {
        "metric": "PCG iters/s + HBM GB/s; time-to-1e-10 rel residual, FP64 vs FP32/FP64-refined",
        "value": iters / elapsed,
        "unit": "PCG iters/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1000.0 * elapsed / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic (seeded smooth random viscosity, N(0,1) right-hand side)",
        "config": {"workload": f"{cfg.name}: FP64 Jacobi-PCG to 1e-10, "
                               f"{cfg.nr}x{cfg.nt}x{cfg.np_} spherical shell "
                               f"({n} cells), step = operator build + full solve",
                   "cells": n, "iterations_per_solve": infos[-1]["iters"],
                   "rel_resid_true": infos[-1]["rel_resid_true"],
                   "time_to_tol_s_fp64": float(np.median(solve_s))},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": (achieved / HBM_PEAK_GBS) if achieved else None,
                     "traffic": traffic,
                     "kernel": "k_pcg_iter<double> (one fused PCG iteration)",
                     "alg_bytes_per_cell": ALG_BYTES_PER_CELL["fp64"],
                     "kernel_bytes_per_cell": KERNEL_BYTES_PER_CELL["fp64"],
                     "achieved_at_kernel_bytes": kern_gbs,
                     "frac_at_kernel_bytes": (kern_gbs / HBM_PEAK_GBS) if kern_gbs else None,
                     "kernel_us": kernel_us},
    }

    if not args.no_refined:
        # same grid and data, single-precision inner PCG inside FP64 refinement
        opm = S.Operator(grid, nu, p.dt, precision="fp32_refined")
        mopts = S.make_opts(rtol=cfg.rtol, precision="fp32_refined", sample_timing=1)
        xm = torch.empty_like(rhs)
        ropts = S.make_opts(rtol=cfg.rtol, precision="fp32_refined", refine="restart")
        ri = opm.solve(rhs, ropts, out=xm, allow_notconv=False)[1]
        opm.solve(rhs, mopts, out=xm, allow_notconv=False)  # warm-up
        mi = [opm.solve(rhs, mopts, out=xm, allow_notconv=False)[1] for _ in range(3)]
        t_ref = float(np.median([i["seconds"] for i in mi]))
        kus32 = [i["iter_kernel_us"] for i in mi if i["iter_kernel_samples"] > 0]
        k32 = float(np.mean(kus32)) if kus32 else None
        diff = float(torch.linalg.vector_norm(xm - x) / torch.linalg.vector_norm(x))
        out["refined"] = {
            "time_to_tol_s": t_ref,
            "speedup_vs_fp64": float(np.median(solve_s)) / t_ref,
            "outer_iters": mi[-1]["outer_iters"], "inner_iters": mi[-1]["iters"],
            "rel_resid_true": mi[-1]["rel_resid_true"],
            "rel_diff_vs_fp64_solution": diff,
            "strategy": "residual replacement keeping the search direction",
            "restarted_refinement": {"time_to_tol_s": ri["seconds"], "outer_iters": ri["outer_iters"],
                                     "inner_iters": ri["iters"],
                                     "rel_resid_true": ri["rel_resid_true"]},
            "inner_kernel_us": k32,
            "inner_kernel_GBs": (ALG_BYTES_PER_CELL["fp32"] * n / (k32 * 1e-6) / 1e9) if k32 else None,
            "inner_kernel_GBs_at_kernel_bytes":
                (KERNEL_BYTES_PER_CELL["fp32"] * n / (k32 * 1e-6) / 1e9) if k32 else None,
        }
        print(f"[bench] refined: {t_ref:.3f} s vs fp64 {np.median(solve_s):.3f} s",
              file=sys.stderr, flush=True)

    if not args.no_build:
        out["op_build"] = bench_build(S, grid, nu, p)

    if not args.no_adjoint:
        out["adjoint"] = bench_adjoint(S, grid, nu, x, p, opts, float(np.median(solve_s)))

    if not args.no_pc2:
        out["pc2"] = bench_pc2(S, grid, nu, rhs, p, float(np.median(solve_s)), infos[-1]["iters"])

    if not args.no_multi:
        out["multi"] = bench_multi(S, W, grid, nu, p, float(np.median(solve_s)), kernel_us)
        torch.cuda.empty_cache()

    if not args.no_sts:
        out["sts"] = bench_sts(S, grid, nu, rhs, p, float(np.median(solve_s)), args.steps)

    if not args.no_c0:
        out["c0"] = bench_c0(S, W, dev)

    x_host = {"fp64": x.cpu().numpy()}
    if "refined" in out:
        x_host["refined"] = xm.cpu().numpy()
        del xm, opm
    torch.cuda.empty_cache()

    if not args.no_c4:
        out["c4"] = bench_c4(S, W, dev)
        torch.cuda.empty_cache()

    if not args.no_probe:
        # achievable bandwidth of the byte mixes the kernels stream, at the
        # workload's size (streaming probes of the library), and a plain copy
        # the iteration kernel alternates launches moving 8 read / 4 written
        # words per cell (with the x update) and 6 / 3 (without): its
        # ceiling is the rate of that alternation, each launch at its mix's
        # probe rate
        g84 = S.probe_stream(n, 8, 4, dev)
        g63 = S.probe_stream(n, 6, 3, dev)
        stream_gbs = 2 * KERNEL_BYTES_PER_CELL["fp64"] / (12 * 8 / g84 + 9 * 8 / g63)
        resid_mix_gbs = S.probe_stream(n, 6, 1, dev)
        grad_mix_gbs = S.probe_stream(n, 2, 2, dev)
        copy_gbs = S.probe_stream(n, 1, 1, dev)
        torch.cuda.empty_cache()
        out["roofline"]["stream_8r4w_GBs"] = g84
        out["roofline"]["stream_6r3w_GBs"] = g63
        out["roofline"]["stream_iter_mix_GBs"] = stream_gbs
        out["roofline"]["copy_probe_GBs"] = copy_gbs
        out["roofline"]["kernel_bytes_frac_of_stream"] = (kern_gbs / stream_gbs) if kern_gbs else None
        out["roofline"]["stream_6r1w_GBs"] = resid_mix_gbs
        if "adjoint" in out:
            out["adjoint"]["gradient_kernel"]["stream_2r2w_GBs"] = grad_mix_gbs
        print(f"[bench] stream probes: 8 read / 4 write {g84:.0f} GB/s, 6/3 {g63:.0f} GB/s "
              f"(iteration mix {stream_gbs:.0f} GB/s), 6/1 {resid_mix_gbs:.0f} GB/s, 2/2 "
              f"{grad_mix_gbs:.0f} GB/s, copy {copy_gbs:.0f} GB/s", file=sys.stderr, flush=True)

    if not args.no_cpu_baseline:
        cb = cpu_baseline(p, x_host)
        rr = cb.pop("gpu_solutions_rel_resid_by_oracle", {})
        out["config"]["rel_resid_by_oracle"] = rr.get("fp64")
        if "refined" in out:
            out["refined"]["rel_resid_by_oracle"] = rr.get("refined")
        out["cpu_baseline"] = cb
        print(f"[bench] cpu baseline {out['cpu_baseline']}", file=sys.stderr, flush=True)

    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
