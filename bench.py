"""Benchmark: time to relative residual 1e-10 of adaptive s-step GMRES on
one MI355X, float64 and float32-inner / float64-refinement, on the 3D
Poisson workload (7-point, 128^3 interior grid, n = 2,097,152,
nnz = 14,581,760, b ~ N(0,1) seed 2, x0 = 0, scaled Newton basis,
s_max = 32, restart 128).

One step = one float64 solve plus one float32-IR solve of that system to
||b - A x|| / ||b|| <= 1e-10, with the matrix analysed and every input
already resident in HBM; `value` is the float64 time with the column-wise
Ritz pre-phase and the paper's BCGS2.  The same two solves are timed
with the pre-phase in adaptive monomial-basis blocks
(fp64_monomial_prephase, fp32_ir_monomial_prephase), with the Pythagorean
second BCGS pass (fp64_pyth, fp32_ir_pyth) and with both
(fp64_monomial_pyth, fp32_ir_monomial_pyth), and reported beside it, each
with its speedup over the float64 default.  Prints ONE JSON line (see keys
below).

Roofline: the dominant kernel is the SELL SpMV of the matrix powers kernel
(float64); its rate is also given against a measured triad bandwidth
(torch's a = b + alpha c on three 1 GiB float64 vectors) and, when the
counters are current, on its measured bytes.  Its average launch duration comes from the HIP event pair the
library records around every MPK launch on the solve's stream, during the
timed steps; algorithmic bytes per launch are
nnz (8 + 4) + 4 (n + 1) + 2 * 8 n (values + column indices, row pointers,
x read once, y written once).  `traffic` comes from a committed rocprofv3
FETCH_SIZE / WRITE_SIZE summary under profiles/, when it was taken on the
current SpMV source (matching hash), else null.

CPU baseline: the oracle (numpy/scipy, float64) timed on the host on a
bounded sample -- one full restart cycle (128 iterations) of the same solve
-- and scaled to the float64 solve's iteration count.

--workload selects one of the other synthetic workloads instead (same JSON
line; no CPU baseline, whose bounded sample would not fit in minutes):
  varcd3d_192   3D variable-coefficient convection-diffusion 192^3 (n =
                7.1M) with right Jacobi, s_max 128, restart 256: float64
                and float32-IR to 1e-10, column-wise and monomial pre-phase;
  aniso2d_4096  2D anisotropic diffusion 4096^2 (n = 16.8M), s_max 200,
                restart 400, no preconditioner (condition ~1e7): float64 and
                float32-IR with capped restarts (it does not reach 1e-10 in
                minutes), plus the backward solve for the gradient w.r.t. b;
                --grid N and --max-cycles C run the same family on N^2
                with C cycles;
  banded_1m     random banded nonsymmetric n = 1M, 27 nonzeros per row:
                the differentiable solve to 1e-12, forward and backward
                (adjoint solve + gradient w.r.t. the CSR values);
  laplace2d_400_ilu0
                2D Laplace 400^2 (n = 160,000) with right ILU(0), the
                setting of the paper's test with an ILU preconditioner:
                float64 to 1e-10 with default options and with the paper's
                settings for that test (s0 = 256), and without the
                preconditioner; the factorisation and one M^{-1}
                application timed apart.
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

METRIC = ("time to rel-res 1e-10 (FP64 vs FP32-IR); SpMV/basis HBM GB/s")
HBM_PEAK_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def spmv_source_hash():
    h = hashlib.sha256()
    with open(os.path.join(ROOT, "paper_2303_08953_amd", "csrc",
                           "spmv.hip"), "rb") as f:
        h.update(f.read())
    return h.hexdigest()[:16]


def load_traffic(kernel_hash, name="spmv_poisson3d_128_traffic.json"):
    p = os.path.join(ROOT, "profiles", name)
    if not os.path.exists(p):
        return None
    with open(p) as f:
        d = json.load(f)
    if d.get("spmv_source_sha256_16") != kernel_hash:
        return None
    return d.get("hbm_bytes_per_launch")


def measure_triad(torch, nbytes=1 << 30, reps=10):
    """Achievable HBM bandwidth for a triad a = b + alpha c (torch's own
    elementwise kernel, float64, three 1 GiB vectors, cold in the 256 MB
    Infinity Cache): GB/s counting 2 reads and 1 write per element."""
    n = nbytes // 8
    a = torch.empty(n, dtype=torch.float64, device="cuda")
    b = torch.rand(n, dtype=torch.float64, device="cuda")
    c = torch.rand(n, dtype=torch.float64, device="cuda")
    for _ in range(2):
        torch.add(b, c, alpha=0.5, out=a)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        torch.add(b, c, alpha=0.5, out=a)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del a, b, c
    torch.cuda.empty_cache()
    return 3 * n * 8 / (ms * 1e-3) / 1e9


def stream_probe(torch, nbytes=1 << 30, reps=10):
    """Achievable HBM rates of plain streams with the read/write mixes of
    the solver's kernels, from PyTorch's own elementwise and reduction
    kernels on float64 vectors of nbytes each (cold in the 256 MB Infinity
    Cache): read-only (sum), 1 read : 1 write (copy), 2 : 1 (add), 3 : 1
    (addcmul).  GB/s counting every vector read and written once."""
    n = nbytes // 8
    vs = [torch.rand(n, dtype=torch.float64, device="cuda") for _ in range(4)]
    a, b, c, d = vs
    red = torch.empty((), dtype=torch.float64, device="cuda")
    cases = {
        "read_only": (lambda: torch.sum(a, 0, out=red), 1),
        "read1_write1": (lambda: d.copy_(a), 2),
        "read2_write1": (lambda: torch.add(a, b, alpha=0.5, out=d), 3),
        "read3_write1": (lambda: torch.addcmul(a, b, c, value=0.5, out=d), 4),
    }
    out = {}
    for name, (f, nvec) in cases.items():
        for _ in range(2):
            f()
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            f()
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        out[name] = round(nvec * n * 8 / (ms * 1e-3) / 1e9, 1)
    del vs, a, b, c, d
    torch.cuda.empty_cache()
    return out


def cpu_baseline(A, b, gpu_iters, restart, s_max):
    """The oracle, as it stands, on one restart cycle of the same solve.

    cores is the number of threads the oracle actually kept busy: its
    process CPU time over its wall time, rounded (scipy's sparse products
    and the Python loops run on one thread; only numpy's dense products
    use the BLAS pool, whose size is reported beside it)."""
    import numpy as np
    from oracle import sstep_gmres as o
    try:
        from threadpoolctl import threadpool_info
        pool = max([t.get("num_threads", 1) for t in threadpool_info()] or [1])
    except Exception:
        pool = None
    M = o.csr_matrix(A.n, A.row_ptr, A.col, A.val)
    c0 = time.process_time()
    t0 = time.perf_counter()
    r = o.solve(M, b, opts=o.Options(s_max=s_max, restart=restart,
                                     tol=1e-10, max_restarts=0))
    dt = time.perf_counter() - t0
    cpu = time.process_time() - c0
    its = max(1, r.iters)
    est_ms = dt * 1e3 * gpu_iters / its
    return {"value": round(est_ms, 1), "unit": "ms",
            "cores": max(1, int(round(cpu / dt))),
            "cpu_over_wall": round(cpu / dt, 2),
            "blas_pool_threads": pool, "host_cpus": os.cpu_count(),
            "kind": "oracle",
            "sample": (f"one restart cycle ({its} iterations, {dt:.1f} s "
                       f"wall, {cpu:.1f} s CPU) of the float64 solve on the "
                       f"same system, scaled to the GPU solve's {gpu_iters} "
                       f"iterations")}


def oracle_samples(nx):
    """The oracle's stored float64 solve of the 128^3 system (written by
    tests/golden/make_poisson3d_128_oracle.py): sampled x entries, their
    indices and the oracle's iteration count; None for other sizes."""
    import numpy as np
    p = os.path.join(ROOT, "tests", "golden", "poisson3d_128_oracle.npz")
    if nx != 128 or not os.path.exists(p):
        return None
    with np.load(p, allow_pickle=False) as z:
        return {k: z[k] for k in ("sample_idx", "x_samples", "iters",
                                  "rel_res_true")}


def solve_summary(sgm, rs, ms_list, tol):
    """Per-mode figures of a list of SolveResults and their wall times."""
    import numpy as np
    last = rs[-1]
    i = last.info
    ok = all(r.status == sgm.OK and r.info["rel_res_true"] <= tol for r in rs)
    ph = i["t_phase_ms"]
    return {"ms": round(float(np.mean(ms_list)), 3),
            "ms_min": round(float(np.min(ms_list)), 3),
            "converged": bool(ok), "iters": i["iters"],
            "restarts": i["restarts"], "outer_iters": i["outer_iters"],
            "rel_res_true": i["rel_res_true"], "s0_est": i["s0_est"],
            "s_init": i["s_init"], "blocks": int(len(last.s_hist)),
            "ms_per_iter": round(float(np.mean(ms_list)) / max(1, i["iters"]),
                                 4),
            "s_hist_head": [int(v) for v in last.s_hist[:24]],
            "phase_ms": {"setup": round(ph[0], 3),
                         "prephase_shifts": round(ph[1], 3),
                         "mpk": round(ph[2], 3),
                         "orth_tail": round(ph[3] + ph[4], 3),
                         "cycle_end": round(ph[5], 3),
                         "total": round(ph[7], 3)},
            "spmv_avg_us": round(i["t_spmv_ms"] / max(1, i["n_spmv"]) * 1e3,
                                 2)}


def spmv_roofline(A, G, rs, vb, label):
    """Rate of the matrix powers SpMV over the solves rs: CSR algorithmic
    bytes nnz (vb + 4) + 4 (n + 1) + 2 vb n per launch over the average
    launch time (HIP events around every MPK launch); also the SELL
    format's own minimum, padded entries times (vb + index bytes) plus
    x and y.  None when the solves made no matrix powers launch (they
    converged inside the column-wise Ritz pre-phase)."""
    info = G.info()
    n_spmv = sum(r.info["n_spmv"] for r in rs)
    t_spmv = sum(r.info["t_spmv_ms"] for r in rs)
    if n_spmv == 0 or t_spmv <= 0:
        return None  # converged inside the column-wise pre-phase
    avg_ms = t_spmv / n_spmv
    alg = A.nnz * (vb + 4) + 4 * (A.n + 1) + 2 * vb * A.n
    fmt = info["sell_nnz"] * (vb + info["index_bytes"]) + 2 * vb * A.n
    ach = alg / (avg_ms * 1e-3) / 1e9
    return {"kernel": f"k_spmv<{label}, EPI_MPK, "
                      f"{'int16_t' if info['index_bytes'] == 2 else 'int32_t'}>"
                      " (SELL-C-64 SpMV of the matrix powers kernel; "
                      "achieved is on the CSR bytes)",
            "bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": round(ach / HBM_PEAK_GBS, 4),
            "traffic": None, "algorithmic_bytes_per_launch": int(alg),
            "format_bytes_per_launch": int(fmt),
            "format_gbs": round(fmt / (avg_ms * 1e-3) / 1e9, 1),
            "index_bytes": info["index_bytes"],
            "avg_launch_us": round(avg_ms * 1e3, 2), "launches": int(n_spmv)}


def analyse(torch, sgm, A):
    """Matrix analysis (sgm_matrix_create: SELL-C-64 layout of A and of its
    transpose, float32 values, diagonal) on a CSR already in device memory,
    timed apart from the solves.  A first analysis, discarded, loads the
    kernels; the second is timed.  Returns the handle and milliseconds."""
    rp = torch.as_tensor(A.row_ptr, dtype=torch.int32, device="cuda")
    col = torch.as_tensor(A.col, dtype=torch.int32, device="cuda")
    val = torch.as_tensor(A.val, dtype=torch.float64, device="cuda")
    sgm.Matrix(A.n, rp, col, val)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    G = sgm.Matrix(A.n, rp, col, val)
    torch.cuda.synchronize()
    return G, (time.perf_counter() - t0) * 1e3


def study_ilu(args, np, torch, sgm, W):
    """2D Laplace 400^2 (the matrix of the paper's Test 2) with right ILU(0),
    the setting of its Sec. 4.3 test with an ILU preconditioner, to 1e-10:
    - fp64_ilu0: default options (s_max 256, the library's largest step,
      restart 400, estimator on, pre-phase columns reused);
    - fp64_ilu0_separate_prephase: the paper's settings for that test (a
      separate Ritz pre-phase, no estimator, Omega = 1e7), s0 = 256;
    - fp64_none: the same system without a preconditioner.
    The factorisation (sgm_matrix_ilu0) is matrix analysis and is timed
    apart; one M^{-1} application is timed on its own as well."""
    A = W.laplace_2d(400)
    b_host = W.rhs(A.n, 1)
    G = sgm.Matrix.from_csr(A)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    levels = G.ilu0()
    torch.cuda.synchronize()
    t_fac = (time.perf_counter() - t0) * 1e3
    b = torch.tensor(b_host, device="cuda")
    x = torch.empty_like(b)
    ws = sgm.Workspace()
    base = dict(s_max=256, restart=400, tol=1e-10, max_restarts=100)
    modes = [("fp64_ilu0", dict(base, precond="ilu0")),
             ("fp64_ilu0_separate_prephase",
              dict(base, precond="ilu0", ritz_reuse=False,
                   use_estimator=False, omega=1e7)),
             ("fp64_none", dict(base))]
    for mname, o in modes:
        sgm.solve(G, b, out=x, workspace=ws, **dict(o, max_restarts=0))
        torch.cuda.synchronize()
    per, infos = {}, {}
    t_start = time.perf_counter()
    for k in range(args.steps):
        for mname, o in modes:
            t0 = time.perf_counter()
            r = sgm.solve(G, b, out=x, workspace=ws, **o)
            torch.cuda.synchronize()
            ms = (time.perf_counter() - t0) * 1e3
            per.setdefault(mname, []).append(ms)
            infos.setdefault(mname, []).append(r)
            log(f"[bench] step {k} {mname}: {ms:.1f} ms iters "
                f"{r.info['iters']} rel {r.info['rel_res_true']:.2e}")
    total_ms = (time.perf_counter() - t_start) * 1e3
    # one M^{-1} application, timed alone (HIP events on torch's stream)
    z = torch.empty_like(b)
    for _ in range(3):
        G.ilu0_apply(b, out=z)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(
        enable_timing=True)
    reps = 50
    e0.record()
    for _ in range(reps):
        G.ilu0_apply(b, out=z)
    e1.record()
    torch.cuda.synchronize()
    apply_us = e0.elapsed_time(e1) * 1e3 / reps
    out = {"metric": METRIC, "unit": "ms", "n_gpus": 1,
           "steps": args.steps, "warmup": 1,
           "ms_per_step": round(total_ms / max(1, args.steps), 3),
           "higher_is_better": False, "scaling": "weak",
           "vs_baseline": None, "data": "synthetic",
           "config": {"workload": "laplace2d_400_ilu0",
                      "matrix": "2D Laplace 5-point (4, -1) 400^2, Dirichlet",
                      "precond": "ILU(0), right", "n": A.n, "nnz": A.nnz,
                      "basis": "scaled_newton", "s_max": 256,
                      "restart": 400, "tol": 1e-10, "rhs": "N(0,1) seed 1",
                      "x0": "zero"}}
    for mname, _ in modes:
        out[mname] = solve_summary(sgm, infos[mname], per[mname], 1e-10)
    out["value"] = out["fp64_ilu0"]["ms"]
    out["dtype"] = "f64"
    nl = int(levels[0]) + int(levels[1])
    out["ilu0"] = {"factorisation_ms": round(t_fac, 3),
                   "levels": [int(levels[0]), int(levels[1])],
                   "apply_us": round(apply_us, 2),
                   "apply_ns_per_level": round(apply_us * 1e3 / nl, 1),
                   "bound": "latency: one workgroup walks the levels, "
                            "with LDS reads, its arithmetic and one barrier "
                            "per level"}
    out["roofline"] = None
    out["cpu_baseline"] = None
    return out


def study(args, np, torch, sgm, W):
    """One JSON line for a workload other than the default (see the module
    docstring): every mode is warmed up once with its restarts capped at
    one cycle (kernels loaded, workspace allocated), then timed."""
    name = args.workload
    log(f"[bench] building {name}")
    if name == "banded_1m":
        return study_adjoint(args, np, torch, sgm, W)
    if name == "aniso2d_4096" and args.to_tol:
        return study_to_tol(args, np, torch, sgm, W)
    if name == "laplace2d_400_ilu0":
        return study_ilu(args, np, torch, sgm, W)
    if name == "varcd3d_192":
        A = W.var_conv_diff_3d(192, 3)
        b_host = W.rhs(A.n, 3)
        base = dict(s_max=128, restart=256, tol=1e-10, precond="jacobi",
                    max_restarts=200)
        b32 = dict(base, precision="fp32_ir", inner_tol=1e-6, max_outer=100)
        modes = [("fp64", base), ("fp32_ir", b32),
                 ("fp64_monomial_prephase", dict(base, prephase="monomial")),
                 ("fp32_ir_monomial_prephase",
                  dict(b32, prephase="monomial"))]
        cfg = {"workload": name,
               "matrix": "3D variable-coefficient convection-diffusion "
                         "7-point 192^3, lognormal(0,1) cells, harmonic faces,"
                         " velocity (20,10,5) upwind, Dirichlet",
               "precond": "jacobi (right)", "s_max": 128, "restart": 256,
               "rhs": "N(0,1) seed 3"}
    else:  # aniso2d_4096 (or --grid N: the same matrix family on N^2)
        grid = args.grid or 4096
        cyc = args.max_cycles or 5
        A = W.aniso_diffusion_2d(grid, angle_deg=args.angle)
        b_host = W.rhs(A.n, 5)
        base = dict(s_max=200, restart=400, tol=1e-10, max_restarts=cyc - 1)
        b32 = dict(base, precision="fp32_ir", inner_tol=1e-6, max_outer=cyc,
                   max_restarts=1000)
        modes = [("fp64", base), ("fp32_ir", b32),
                 ("fp64_monomial_prephase", dict(base, prephase="monomial")),
                 ("fp32_ir_monomial_prephase",
                  dict(b32, prephase="monomial")),
                 ("fp32_ir_monomial_no_estimator",
                  dict(b32, prephase="monomial", use_estimator=False))]
        cfg = {"workload": f"aniso2d_{grid}",
               "matrix": f"2D anisotropic diffusion 5-point {grid}^2, "
                         f"K = R({args.angle:g}deg) diag(1, 1e-3) R^T, "
                         f"K_xy dropped (axis ratio Kyy/Kxx = "
                         f"{aniso_axis_ratio(args.angle):.4g})",
               "precond": "none", "s_max": 200, "restart": 400,
               "caps": f"float64: {cyc} restart cycles; float32-IR: {cyc} "
                       "outer steps",
               "rhs": "N(0,1) seed 5"}
    if args.mode == "fp64":
        modes = [m for m in modes if m[0].startswith("fp64")]
    cfg.update({"n": A.n, "nnz": A.nnz, "basis": "scaled_newton",
                "tol": 1e-10, "x0": "zero"})
    G, t_analysis = analyse(torch, sgm, A)
    log(f"[bench] matrix analysis {t_analysis:.1f} ms")
    b = torch.tensor(b_host, device="cuda")
    x = torch.empty_like(b)
    ws = sgm.Workspace()
    for mname, o in modes:
        cap = dict(o, max_restarts=0, max_outer=1)
        t0 = time.perf_counter()
        sgm.solve(G, b, out=x, workspace=ws, mpk_depth=args.mpk_depth, **cap)
        torch.cuda.synchronize()
        log(f"[bench] warmup {mname}: {(time.perf_counter() - t0) * 1e3:.0f}"
            " ms")
    per, infos = {}, {}
    t_start = time.perf_counter()
    for k in range(args.steps):
        for mname, o in modes:
            t0 = time.perf_counter()
            r = sgm.solve(G, b, out=x, workspace=ws,
                          mpk_depth=args.mpk_depth, **o)
            torch.cuda.synchronize()
            ms = (time.perf_counter() - t0) * 1e3
            per.setdefault(mname, []).append(ms)
            infos.setdefault(mname, []).append(r)
            log(f"[bench] step {k} {mname}: {ms:.1f} ms iters "
                f"{r.info['iters']} rel {r.info['rel_res_true']:.2e}")
    total_ms = (time.perf_counter() - t_start) * 1e3
    out = {"metric": METRIC, "unit": "ms", "n_gpus": 1,
           "steps": args.steps, "warmup": 1,
           "ms_per_step": round(total_ms / max(1, args.steps), 3),
           "higher_is_better": False, "scaling": "weak",
           "vs_baseline": None, "data": "synthetic",
           "config": cfg}
    for mname, _ in modes:
        out[mname] = solve_summary(sgm, infos[mname], per[mname], 1e-10)
        if mname != "fp64" and "fp64" in per:
            out[mname]["speedup_vs_fp64"] = round(
                out["fp64"]["ms"] / out[mname]["ms"], 3)
    prim = "fp64" if "fp64" in infos else modes[0][0]
    vb = 8 if prim.startswith("fp64") else 4
    out["value"] = round(float(np.mean(per[prim])), 3)
    out["dtype"] = "f64" if vb == 8 else "f32/f64"
    out["roofline"] = spmv_roofline(A, G, infos[prim], vb,
                                    "double" if vb == 8 else "float")
    if "fp32_ir" in infos:
        out["roofline_fp32"] = spmv_roofline(A, G, infos["fp32_ir"], 4,
                                             "float")
    if name == "aniso2d_4096" and args.mode != "fp64":
        # backward solve for the gradient w.r.t. b (float32-IR, same caps)
        bt = torch.tensor(b_host, device="cuda", requires_grad=True)
        vals = torch.tensor(A.val, device="cuda")
        o = dict(b32, prephase="monomial")
        t0 = time.perf_counter()
        xg = sgm.sstep_solve(vals, bt, G, allow_not_converged=True, **o)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        log(f"[bench] differentiable forward: {(t1 - t0) * 1e3:.0f} ms")
        (0.5 * (xg ** 2).sum()).backward()
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        log(f"[bench] backward: {(t2 - t1) * 1e3:.0f} ms")
        out["fp32_ir_with_backward"] = {
            "forward_ms": round((t1 - t0) * 1e3, 1),
            "backward_ms": round((t2 - t1) * 1e3, 1),
            "grad_b_finite": bool(torch.isfinite(bt.grad).all().item())}
    out["matrix_analysis_ms"] = round(t_analysis, 2)
    out["cpu_baseline"] = None
    return out


def aniso_axis_ratio(angle_deg, ratio=1e-3):
    """K_yy / K_xx of R(angle) diag(1, ratio) R^T: the anisotropy the 5-point
    stencil keeps once K_xy is dropped."""
    import math
    a = math.radians(angle_deg)
    kxx = math.cos(a) ** 2 + ratio * math.sin(a) ** 2
    kyy = math.sin(a) ** 2 + ratio * math.cos(a) ** 2
    return kyy / kxx


def study_to_tol(args, np, torch, sgm, W):
    """aniso2d_4096 solved to ||b - A x|| / ||b|| <= 1e-10.  A single solve
    runs for minutes, so each mode runs as successive solves of
    --chunk-cycles restart cycles (float64) or outer steps (float32-IR),
    each from the previous iterate with its tolerance rescaled to ||b|| (the
    product of the solves' reported residual ratios); each such solve
    computes its own Ritz values and initial step size.  Float32-IR modes
    also run the backward solve for L = 0.5 ||x||^2 (A^T lambda = x, the
    gradient w.r.t. b), chunked the same way.  The final residuals are
    checked on the host (scipy CSR product)."""
    import scipy.sparse as sps
    grid = args.grid or 4096
    A = W.aniso_diffusion_2d(grid, angle_deg=args.angle)
    b_host = W.rhs(A.n, 5)
    M = sps.csr_matrix((A.val, A.col, A.row_ptr), shape=(A.n, A.n))
    G = sgm.Matrix.from_csr(A)
    tol = 1e-10
    base = dict(s_max=200, restart=400)
    b32 = dict(base, precision="fp32_ir", inner_tol=1e-6)
    all_modes = {
        "fp64": base,
        "fp64_monomial_prephase": dict(base, prephase="monomial"),
        "fp32_ir": b32,
        "fp32_ir_monomial_no_estimator": dict(b32, prephase="monomial",
                                              use_estimator=False)}
    names = args.to_tol_modes.split(",")
    C = args.chunk_cycles
    ws = sgm.Workspace()

    def chunked(rhs_host, o, label, transpose=False):
        rhs = torch.tensor(rhs_host, device="cuda")
        xa = torch.zeros_like(rhs)
        xb = torch.empty_like(rhs)
        rho, ms, iters, chunks, s0s = 1.0, 0.0, 0, 0, []
        cap = (dict(max_outer=C) if o.get("precision") == "fp32_ir"
               else dict(max_restarts=C - 1))
        while rho > tol and chunks < args.max_chunks:
            t0 = time.perf_counter()
            r = sgm.solve(G, rhs, x0=xa, out=xb, workspace=ws, tol=tol / rho,
                          transpose=transpose, mpk_depth=args.mpk_depth,
                          **dict(o, **cap))
            torch.cuda.synchronize()
            ms += (time.perf_counter() - t0) * 1e3
            rho *= r.info["rel_res_true"]
            iters += r.info["iters"]
            chunks += 1
            s0s.append(r.info["s0_est"])
            xa, xb = xb, xa
            log(f"[bench] to-tol {label} chunk {chunks}: {ms / 1e3:.1f} s, "
                f"{iters} iterations, rel {rho:.3e}")
        xh = xa.cpu().numpy()
        Mt = M.T.tocsr() if transpose else M
        true = float(np.linalg.norm(rhs_host - Mt @ xh) /
                     np.linalg.norm(rhs_host))
        return xh, {"ms": round(ms, 1), "iters": iters, "chunks": chunks,
                    "converged": bool(true <= tol * 1.0001),
                    "rel_res_true_host": true, "s0_est_per_chunk": s0s}

    out = {"metric": METRIC, "unit": "ms", "n_gpus": 1, "steps": 1,
           "warmup": 0, "higher_is_better": False, "scaling": "weak",
           "vs_baseline": None, "data": "synthetic",
           "config": {"workload": f"aniso2d_{grid}_to_tol",
                      "matrix": f"2D anisotropic diffusion 5-point {grid}^2,"
                                f" K = R({args.angle:g}deg) diag(1, 1e-3) R^T"
                                f" with K_xy dropped (axis ratio Kyy/Kxx = "
                                f"{aniso_axis_ratio(args.angle):.4g})",
                      "n": A.n, "nnz": A.nnz, "s_max": 200, "restart": 400,
                      "tol": tol, "rhs": "N(0,1) seed 5", "x0": "zero",
                      "chunk": f"{C} restart cycles / outer steps per solve"}}
    for mname in names:
        x, summ = chunked(b_host, all_modes[mname], mname)
        out[mname] = summ
        if mname.startswith("fp32_ir") and not args.no_backward:
            _, bw = chunked(x, all_modes[mname], mname + " backward",
                            transpose=True)
            out[mname]["backward"] = bw
    prim = names[0]
    out["value"] = out[prim]["ms"]
    out["ms_per_step"] = out[prim]["ms"]
    out["dtype"] = "f64" if prim.startswith("fp64") else "f32/f64"
    out["roofline"] = None
    out["cpu_baseline"] = None
    return out


def study_adjoint(args, np, torch, sgm, W):
    """banded_1m: the differentiable solve x = A(vals)^{-1} b to 1e-12 and
    the backward pass of L = 0.5 ||x - x*||^2 (adjoint solve on A^T and the
    gradient w.r.t. the CSR values), timed together; the plain forward and
    transposed solves are timed alone for their iteration counts."""
    A, b_host, xs_host = W.banded_problem(1_000_000, seed=4, band=1000)
    G = sgm.Matrix.from_csr(A)
    opts = dict(s_max=8, restart=128, tol=1e-12, max_restarts=200)
    vals = torch.tensor(A.val, device="cuda", requires_grad=True)
    bt = torch.tensor(b_host, device="cuda", requires_grad=True)
    xs = torch.tensor(xs_host, device="cuda")
    ws = sgm.Workspace()

    def diff_step():
        vals.grad = None
        bt.grad = None
        t0 = time.perf_counter()
        x = sgm.sstep_solve(vals, bt, G, **opts)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        (0.5 * ((x - xs) ** 2).sum()).backward()
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        return (t1 - t0) * 1e3, (t2 - t1) * 1e3

    f, bw = diff_step()
    log(f"[bench] warmup: forward {f:.1f} ms backward {bw:.1f} ms")
    fw, bk, tot = [], [], []
    for k in range(args.steps):
        f, bw = diff_step()
        fw.append(f)
        bk.append(bw)
        tot.append(f + bw)
        log(f"[bench] step {k}: forward {f:.1f} ms backward {bw:.1f} ms")
    plain = {}
    for mname, o in (("forward_solve", opts),
                     ("adjoint_solve", dict(opts, transpose=True))):
        t0 = time.perf_counter()
        r = sgm.solve(G, torch.tensor(b_host, device="cuda"), workspace=ws,
                      **o)
        torch.cuda.synchronize()
        plain[mname] = solve_summary(sgm, [r],
                                     [(time.perf_counter() - t0) * 1e3],
                                     1e-12)
        plain[mname]["_r"] = r
    out = {"metric": METRIC, "unit": "ms", "n_gpus": 1,
           "steps": args.steps, "warmup": 1,
           "ms_per_step": round(float(np.mean(tot)), 3),
           "higher_is_better": False, "scaling": "weak", "vs_baseline": None,
           "data": "synthetic", "value": round(float(np.mean(tot)), 3),
           "dtype": "f64",
           "config": {"workload": "banded_1m",
                      "matrix": "random banded nonsymmetric, 26 off-diagonals"
                                " U(-1,1) within |i-j| <= 1000, diagonal "
                                "1.2 x row abs sum",
                      "n": A.n, "nnz": A.nnz, "s_max": 8, "restart": 128,
                      "tol": 1e-12, "loss": "0.5 ||x - x*||^2",
                      "rhs": "N(0,1) seed 1004, x* N(0,1)"},
           "differentiable_step": {"forward_ms": round(float(np.mean(fw)), 3),
                                   "backward_ms": round(float(np.mean(bk)),
                                                        3)}}
    rs = {k: plain[k].pop("_r") for k in plain}
    out.update(plain)
    out["roofline"] = spmv_roofline(A, G, [rs["forward_solve"]], 8, "double")
    out["cpu_baseline"] = None
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--nx", type=int, default=128)
    ap.add_argument("--workload", default="poisson3d_128",
                    choices=["poisson3d_128", "varcd3d_192", "aniso2d_4096",
                             "banded_1m", "laplace2d_400_ilu0"])
    ap.add_argument("--mode", choices=["both", "fp64", "fp32_ir", "all"],
                    default="all")
    ap.add_argument("--grid", type=int, default=0,
                    help="aniso2d_4096 only: grid size N (N^2 unknowns)")
    ap.add_argument("--max-cycles", type=int, default=0,
                    help="aniso2d_4096 only: restart cycles (float64) and "
                         "outer steps (float32-IR), default 5")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--to-tol", action="store_true",
                    help="aniso2d_4096: solve to 1e-10 in chunks of "
                         "--chunk-cycles cycles (see study_to_tol)")
    ap.add_argument("--to-tol-modes", default="fp64",
                    help="comma-separated: fp64, fp64_monomial_prephase, "
                         "fp32_ir, fp32_ir_monomial_no_estimator")
    ap.add_argument("--chunk-cycles", type=int, default=40)
    ap.add_argument("--no-backward", action="store_true",
                    help="--to-tol: skip the float32-IR backward solve")
    ap.add_argument("--angle", type=float, default=30.0,
                    help="aniso2d_4096: rotation of the diffusion tensor in "
                         "degrees (30: axis ratio 0.334 after dropping K_xy;"
                         " 0: the axis-aligned ratio 1e-3)")
    ap.add_argument("--max-chunks", type=int, default=40)
    ap.add_argument("--mpk-depth", type=int, default=1,
                    help="matrix powers steps per pass over the matrix "
                         "(temporal blocking, 1-4) for every mode")
    ap.add_argument("--stream-probe", action="store_true",
                    help="only measure plain HBM stream rates (read-only, "
                         "1:1, 2:1 and 3:1 read/write) and print them")
    ap.add_argument("--calibrate-copy-mb", type=int, default=0,
                    help="run one plain device copy of this size (for the "
                         "rocprof counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: the solver runs on one GPU; --gpus "
              f"{args.gpus} is not supported", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2303_08953_amd as sgm
    import workloads as W

    torch.cuda.set_device(0)
    if args.calibrate_copy_mb > 0:
        nel = args.calibrate_copy_mb * (1 << 20) // 8
        src = torch.ones(nel, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
        torch.cuda.empty_cache()
        log(f"[bench] calibration copy of {args.calibrate_copy_mb} MiB done")
    if args.stream_probe:
        print(json.dumps({"stream_probe_gbs": stream_probe(torch),
                          "vector_bytes": 1 << 30, "dtype": "f64"}),
              flush=True)
        return
    if args.workload != "poisson3d_128":
        print(json.dumps(study(args, np, torch, sgm, W)), flush=True)
        return
    s_max, restart, tol = 32, 128, 1e-10
    log(f"[bench] building poisson3d_{args.nx}")
    A = W.poisson_3d(args.nx)
    b_host = W.rhs(A.n, 2)
    G, t_analysis = analyse(torch, sgm, A)
    log(f"[bench] matrix analysis {t_analysis:.1f} ms")
    b = torch.tensor(b_host, device="cuda")
    x = torch.empty_like(b)
    ws = sgm.Workspace()
    o64 = dict(s_max=s_max, restart=restart, tol=tol, max_restarts=1000)
    o32 = dict(o64, precision="fp32_ir", inner_tol=1e-6, max_outer=500)
    o64m = dict(o64, prephase="monomial", prephase_s=8)
    o32m = dict(o32, prephase="monomial", prephase_s=8)
    o64p = dict(o64, orth="bcgs2_pyth")
    o32p = dict(o32, orth="bcgs2_pyth")
    o64mp = dict(o64m, orth="bcgs2_pyth")
    o32mp = dict(o32m, orth="bcgs2_pyth")
    both = [("fp64", o64), ("fp32_ir", o32)]
    modes = {"both": both,
             "all": both + [("fp64_monomial_prephase", o64m),
                            ("fp32_ir_monomial_prephase", o32m),
                            ("fp64_pyth", o64p), ("fp32_ir_pyth", o32p),
                            ("fp64_monomial_pyth", o64mp),
                            ("fp32_ir_monomial_pyth", o32mp)],
             "fp64": [("fp64", o64)], "fp32_ir": [("fp32_ir", o32)]}[args.mode]


    def run(opts):
        t0 = time.perf_counter()
        r = sgm.solve(G, b, out=x, workspace=ws,
                      **dict(dict(mpk_depth=args.mpk_depth), **opts))
        torch.cuda.synchronize()
        return r, (time.perf_counter() - t0) * 1e3

    for w in range(args.warmup):
        for name, opts in modes:
            r, ms = run(opts)
            log(f"[bench] warmup {w} {name}: {ms:.1f} ms iters "
                f"{r.info['iters']} rel {r.info['rel_res_true']:.2e}")

    torch.cuda.synchronize()
    t_start = time.perf_counter()
    per = {name: [] for name, _ in modes}
    infos = {}
    for k in range(args.steps):
        for name, opts in modes:
            r, ms = run(opts)
            per[name].append(ms)
            infos.setdefault(name, []).append(r)
            log(f"[bench] step {k} {name}: {ms:.1f} ms iters "
                f"{r.info['iters']} rel {r.info['rel_res_true']:.2e}")
    torch.cuda.synchronize()
    total_ms = (time.perf_counter() - t_start) * 1e3

    def summary(name):
        rs = infos[name]
        last = rs[-1]
        i = last.info
        ok = all(rr.status == sgm.OK and rr.info["rel_res_true"] <= tol
                 for rr in rs)
        return {"ms": round(float(np.mean(per[name])), 3),
                "ms_min": round(float(np.min(per[name])), 3),
                "converged": bool(ok), "iters": i["iters"],
                "restarts": i["restarts"], "outer_iters": i["outer_iters"],
                "rel_res_true": i["rel_res_true"], "s0_est": i["s0_est"],
                "s_init": i["s_init"],
                "blocks": int(len(last.s_hist)),
                "s_hist_head": [int(v) for v in last.s_hist[:40]],
                "phase_ms": {"setup": round(i["t_phase_ms"][0], 3),
                             "prephase_shifts": round(i["t_phase_ms"][1], 3),
                             "mpk": round(i["t_phase_ms"][2], 3),
                             "orth_tail": round(i["t_phase_ms"][3]
                                                + i["t_phase_ms"][4], 3),
                             "cycle_end": round(i["t_phase_ms"][5], 3),
                             "total": round(i["t_phase_ms"][7], 3)}}

    out = {"metric": METRIC, "unit": "ms", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup,
           "ms_per_step": round(total_ms / max(1, args.steps), 3),
           "higher_is_better": False, "scaling": "weak",
           "vs_baseline": None, "data": "synthetic"}
    primary = "fp64" if "fp64" in per else "fp32_ir"
    out["value"] = round(float(np.mean(per[primary])), 3)
    out["dtype"] = "f64" if primary == "fp64" else "f32/f64"
    out["matrix_analysis_ms"] = round(t_analysis, 2)
    out["config"] = {"workload": f"poisson3d_{args.nx}",
                     "matrix": f"3D Poisson 7-point {args.nx}^3, Dirichlet",
                     "n": A.n, "nnz": A.nnz, "basis": "scaled_newton",
                     "s_max": s_max, "restart": restart, "tol": tol,
                     "rhs": "N(0,1) seed 2", "x0": "zero"}
    for name in per:
        out[name] = summary(name)
    if "fp64" in per and "fp32_ir" in per:
        out["fp32_ir"]["speedup_vs_fp64"] = round(
            out["fp64"]["ms"] / out["fp32_ir"]["ms"], 3)
    for name in ("fp64_monomial_prephase", "fp32_ir_monomial_prephase",
                 "fp64_pyth", "fp32_ir_pyth", "fp64_monomial_pyth",
                 "fp32_ir_monomial_pyth"):
        if name in per and "fp64" in per:
            out[name]["speedup_vs_fp64"] = round(
                out["fp64"]["ms"] / out[name]["ms"], 3)

    # roofline of the dominant kernel: float64 MPK SpMV
    rs = infos[primary]
    n_spmv = sum(r.info["n_spmv"] for r in rs)
    t_spmv = sum(r.info["t_spmv_ms"] for r in rs)
    avg_ms = t_spmv / max(1, n_spmv)
    vb = 8 if primary == "fp64" else 4
    alg_bytes = A.nnz * (vb + 4) + 4 * (A.n + 1) + 2 * vb * A.n
    achieved = alg_bytes / (avg_ms * 1e-3) / 1e9
    khash = spmv_source_hash()
    traffic = load_traffic(khash)
    triad = measure_triad(torch)
    out["roofline"] = {
        "kernel": f"k_spmv<{'double' if vb == 8 else 'float'}, EPI_MPK, "
                  "int16_t> (SELL-C-64 SpMV of the matrix powers kernel, "
                  "16-bit relative columns; achieved is on the CSR bytes)",
        "bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
        "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
        "traffic": traffic,
        "measured_triad_gbs": round(triad, 1),
        "frac_of_triad": round(achieved / triad, 4),
        "traffic_gbs": (round(traffic / (avg_ms * 1e-3) / 1e9, 1)
                        if traffic else None),
        "algorithmic_bytes_per_launch": int(alg_bytes),
        "avg_launch_us": round(avg_ms * 1e3, 2), "launches": int(n_spmv),
        "spmv_source_sha256_16": khash}
    if primary == "fp64" and "fp32_ir" in infos:
        # the same figure for the float32 inner solves' SpMV
        out["roofline_fp32"] = spmv_roofline(A, G, infos["fp32_ir"], 4,
                                             "float")
        r32 = out["roofline_fp32"]
        if r32 is not None and args.nx == 128:
            t32 = load_traffic(spmv_source_hash(),
                               "spmv_poisson3d_128_fp32_traffic.json")
            r32["traffic"] = t32
            r32["traffic_gbs"] = (round(t32 / (r32["avg_launch_us"] * 1e-6)
                                        / 1e9, 1) if t32 else None)
    gold = oracle_samples(args.nx)
    if gold is not None:
        # error of each mode's solution against the oracle's float64 solve
        # of the same system, on its 8192 stored samples (one more solve
        # per mode, after the timed steps)
        idx = torch.tensor(gold["sample_idx"], device="cuda")
        ref = gold["x_samples"]
        err = {"oracle_iters": int(gold["iters"]),
               "oracle_rel_res_true": float(gold["rel_res_true"]),
               "measure": "||x - x_oracle|| / ||x_oracle|| on 8192 sampled "
                          "entries"}
        for name, opts in modes:
            run(opts)
            xs = x[idx].cpu().numpy()
            err[name] = float(f"{np.linalg.norm(xs - ref) / np.linalg.norm(ref):.3e}")
        out["error_vs_oracle"] = err
    if not args.no_cpu_baseline:
        log("[bench] timing the oracle on one restart cycle (CPU)")
        out["cpu_baseline"] = cpu_baseline(
            A, b_host, out[primary]["iters"], restart, s_max)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
