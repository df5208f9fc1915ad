"""Benchmark: AMG-PCG on one MI355X against the CPU oracle.

A step is one pass of the hot path on one synthetic system held in HBM:
hierarchy set-up (strength, PMIS, direct interpolation, transpose, Galerkin
SpGEMM, smoother weights, last-level Cholesky) followed by the FP64
V-cycle-preconditioned CG solve to rtol 1e-8.  The mixed-precision solve
(FP32 V-cycle inside FP64 PCG) of the same system is timed beside it.

Default workload: 3D 7-point finite-volume diffusion on 128^3 cells with
lognormal(0, 2) face coefficients, b ~ U[-1, 1] (seeds 2021 / 7417).  The
same JSON line carries the other configurations of the metric: the 64x64
Poisson parity case (`c1`), the 64^3-element Q1 elasticity system, FP64
against mixed precision, with its level-0 kernels' roofline (`c3`), 32
right-hand sides on the 160^3 anisotropic problem (`batched`), many small
systems in one launch, and the serving sweep at two request rates
(`serving`).

Prints one JSON line (rank 0).  `value` is the FP64 solve time (ms, lower is
better) of the default workload; `roofline` rates its level-0
post-smoothing kernel against HBM.
"""
from __future__ import annotations

import argparse
import concurrent.futures as cf
import hashlib
import json
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "AMG-PCG solve time & V-cycle HBM GB/s at rtol 1e-8; FP64 vs mixed; p99 latency"
HBM_PEAK_GBS = 8000.0
# every PROFILE_STRIDE-th PCG iteration of a profiled solve is timed; such an
# iteration is launched in three parts (two graphs, and the level-0 kernel
# between events) instead of sharing a two-iteration graph, and each extra
# launch leaves a gap of some 13 us, so one in 16 keeps the timing's cost
# near 0.5 % of the solve while giving several timed launches per solve
PROFILE_STRIDE = 16

WORKLOADS = {
    "lognormal3d_128": "3D 7-point FV diffusion, 128^3 cells, lognormal(0,2) face coefficients, FP64 CSR, "
                       "b~U[-1,1]; theta=0.25, PMIS, direct interpolation, Jacobi 1/1, V-cycle PCG rtol 1e-8",
    "poisson2d_64": "2D 5-point Laplacian, 64x64 interior, FP64; same method",
    "aniso3d_160": "3D anisotropic 7-point, 160^3, eps=1e-3; same method",
    "elasticity_64": "3D Q1 elasticity, 64^3 hex elements, E lognormal(0,1), nu=0.3; same method",
}


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


# ------------------------------------------------------------------ bytes per launch
def vcycle_bytes(info, fp32=False):
    """Algorithmic bytes of one V-cycle: every matrix (A_l twice, P_l, R_l)
    and every vector pass read or written once (int32 indices)."""
    vb = 4 if fp32 else 8
    mb = 4 + vb
    tot = 0
    L = info.levels
    for l in range(L - 1):
        n, nnz, nnzp = info.n[l], info.nnz[l], info.nnz_p[l]
        nc = info.n[l + 1]
        tot += 2 * (mb * nnz + 4 * (n + 1))          # pre and post smoothing sweeps read A_l
        tot += 2 * mb * nnzp + 4 * (n + 1) + 4 * (nc + 1)  # restriction (R) and prolongation (P)
        tot += 11 * vb * n                            # vector passes on level l
        tot += 2 * vb * nc                            # restricted rhs written, correction read
    nL = info.n[L - 1]
    tot += 8 * nL * nL + 2 * vb * nL                  # dense inverse of the last level
    return tot


def post0_bytes(n, nnz, fp32=False, col_bytes=4):
    """Bytes the level-0 post-smoothing kernel must move: A_0 once (row
    pointer, one column word and one value per nonzero), s gathered once,
    y and omega D^{-1} read, z written.  In mixed precision the matrix, s
    and D^{-1} are FP32 while y (the PCG residual) and z stay FP64.
    col_bytes is 4 for int32 column indices, 2 for the 16-bit column words
    the kernels read when compact columns are on."""
    if fp32:
        return 4 * (n + 1) + (4 + col_bytes) * nnz + 4 * n + 4 * n + 8 * n + 8 * n
    return 4 * (n + 1) + (8 + col_bytes) * nnz + 32 * n


def block_post0_bytes(n, nnz, k, fp32):
    """Bytes of the level-0 block post-smoothing kernel on an n-by-k block:
    A_0 once (int32 columns), the block S gathered once, the block Y (the
    FP64 PCG residuals) and omega D^{-1} read, the block Z written (FP32 in
    mixed precision, where A_0, S and D^{-1} are FP32 too)."""
    if fp32:
        return 4 * (n + 1) + 8 * nnz + 4 * n + (4 + 8 + 4) * k * n
    return 4 * (n + 1) + 12 * nnz + 8 * n + (8 + 8 + 8) * k * n


def committed_counters(name):
    """HBM bytes per launch from a committed rocprofv3 counter summary
    (profiles/<name>.md), or None when the kernel sources have changed since
    the counters were taken."""
    path = os.path.join(ROOT, "profiles", name + ".md")
    if not os.path.exists(path):
        return None
    fields = {}
    for line in open(path):
        if ":" in line and not line.startswith(("#", "-", "|", "`")):
            k, v = line.split(":", 1)
            fields[k.strip()] = v.strip()
    try:
        h = hashlib.sha256()
        for s in fields["sources"].split(", "):
            h.update(open(os.path.join(ROOT, s), "rb").read())
        if h.hexdigest() != fields["source_sha256"]:
            return None
        return {k: float(v) for k, v in fields.items() if k.startswith("traffic_bytes")}
    except (KeyError, OSError, ValueError):
        return None


def roofline_of(kernel, bytes_per_launch, ms_per_launch, launches, traffic=None, **extra):
    gbs = bytes_per_launch / (ms_per_launch * 1e-3) / 1e9 if launches else 0.0
    out = {"bound": "hbm", "kernel": kernel, "achieved": round(gbs, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
           "frac": round(gbs / HBM_PEAK_GBS, 4), "traffic": traffic, "alg_bytes_per_launch": int(bytes_per_launch),
           "avg_launch_us": round(ms_per_launch * 1e3, 3), "launches": int(launches)}
    if traffic:
        out["traffic_over_alg"] = round(traffic / bytes_per_launch, 4)
    out.update(extra)
    return out


# ------------------------------------------------------------------ host facts
def host_facts():
    model = ""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    try:
        allowed = len(os.sched_getaffinity(0))
    except AttributeError:
        allowed = None
    return {"cpu_model": model, "nproc": os.cpu_count(), "cpus_allowed": allowed}


class pinned_to_one_core:
    """Pin the calling thread to its first allowed CPU (as `taskset -c`
    would) for the oracle's single-threaded run, and restore afterwards."""

    def __enter__(self):
        self.cpu = None
        try:
            self.saved = os.sched_getaffinity(0)
            self.cpu = min(self.saved)
            os.sched_setaffinity(0, {self.cpu})
        except (AttributeError, OSError):
            self.saved = None
        return self

    def __exit__(self, *exc):
        if self.saved:
            os.sched_setaffinity(0, self.saved)
        return False


# ------------------------------------------------------------------ helpers on the device
def copy_kernel_gbs(dev):
    """Streaming device-to-device copy of 1 GiB (read + write), for the HBM
    calibration beside the 8 TB/s peak."""
    import torch
    src = torch.empty(1 << 27, dtype=torch.float64, device=dev)
    dst = torch.empty_like(src)
    src.fill_(1.0)
    dst.copy_(src)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(10):
        dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    return 10 * 2 * src.numel() * 8 / (e0.elapsed_time(e1) * 1e-3) / 1e9


def solve_once(camg, A, dA, db, dx, stream, precision, max_iter=5000, profile=False, **kw):
    """Set-up then solve of one system (device arrays dA = (rp, ci, val)),
    each timed on the host around a synchronised device; with profile the
    level-0 post-smoothing kernel is timed by HIP events every
    PROFILE_STRIDE iterations."""
    import torch
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s = camg.Solver.from_device(A.n, *dA, stream=stream, precision=precision, max_iter=max_iter, **kw)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    if profile:
        camg.camg_profile(s.h, PROFILE_STRIDE)
    r = s.solve_dev(db, dx, rtol=1e-8, stream=stream)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    prof = camg.camg_profile(s.h, 0) if profile else (0.0, 0)
    info = s.info
    s.close()
    return dict(setup_ms=(t1 - t0) * 1e3, solve_ms=(t2 - t1) * 1e3, iters=r.iters, status=r.status,
                true_relres=r.true_relres, prof=prof, info=info)


def med(rs, key):
    return round(statistics.median(r[key] for r in rs), 4)


# ====================================================================== c2 (headline)
def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="lognormal3d_128", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--no-fsai", action="store_true", help="skip the FSAI-smoother solves")
    ap.add_argument("--no-interp", action="store_true",
                    help="skip the classical / extended+i / hybrid interpolation solves")
    ap.add_argument("--no-c1", action="store_true", help="skip the 64x64 Poisson parity/latency case")
    ap.add_argument("--no-c3", action="store_true", help="skip the 64^3-element elasticity case")
    ap.add_argument("--batched", type=int, default=32,
                    help="right-hand sides of the batched (block) run on aniso3d_160; 0 skips it")
    ap.add_argument("--only-batched", action="store_true", help="print only the batched run")
    ap.add_argument("--only-c3", action="store_true", help="print only the elasticity case")
    ap.add_argument("--c3-runs", type=int, default=2, help="timed solves per precision of the elasticity case")
    ap.add_argument("--small-systems", type=int, default=256,
                    help="independent 100x100 lognormal systems solved in one launch; 0 skips it")
    ap.add_argument("--serve", action="store_true",
                    help="print only the serving sweep (8 resident systems, Poisson arrivals)")
    ap.add_argument("--rates", default="", help="request rates (1/s) of the serving sweep (default: 2 rates)")
    ap.add_argument("--serve-requests", type=int, default=1000, help="requests per rate of the serving sweep")
    ap.add_argument("--no-serve", action="store_true", help="leave the serving sweep out of the default line")
    ap.add_argument("--bamg", type=int, default=0, metavar="NE",
                    help="only run elasticity on NE^3 elements (64: the 811,200-unknown mechanics case) with "
                         "direct interpolation and with BAMG interpolation over the rigid body modes")
    ap.add_argument("--poi65m", type=str, default="", metavar="GRID[,GRID...]",
                    help="only run the context case: 7-point Poisson on GRID^3 (404 is the paper's poi65m size) "
                         "with Jacobi + extended+i, as the paper's Chr-jac set-up, and with direct interpolation")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; multi-GPU sharding is a design note only",
                          "n_gpus": args.gpus}))
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2102_07417_amd import camg, problems

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    camg.load()
    dev = torch.device("cuda:0")
    rates = [float(r) for r in args.rates.split(",")] if args.rates else SERVE_RATES
    if args.only_batched:
        out = {"copy_kernel_gbs": round(copy_kernel_gbs(dev), 1), "batched": batched_run(args.batched or 32, args.steps)}
        if args.small_systems:
            out["small_systems"] = small_systems_run(args.small_systems)
        print(json.dumps(out), flush=True)
        return
    if args.serve:
        print(json.dumps({"serving": serve_run(rates, args.serve_requests)}), flush=True)
        return
    if args.bamg:
        print(json.dumps({"bamg_elasticity": bamg_run(args.bamg)}), flush=True)
        return
    if args.poi65m:
        for grid in [int(g) for g in args.poi65m.split(",")]:
            print(json.dumps({"poisson_context": poisson_context_run(grid)}), flush=True)
        return
    # the elasticity system takes ~20 s to assemble on the host: start it now
    pool = cf.ThreadPoolExecutor(max_workers=1)
    elas = None if (args.no_c3 or args.workload == "elasticity_64") else pool.submit(problems.workload,
                                                                                       "elasticity_64")
    if args.only_c3:
        print(json.dumps({"copy_kernel_gbs": round(copy_kernel_gbs(dev), 1),
                          "c3": c3_run(elas.result() if elas else problems.workload("elasticity_64"),
                                       args.no_cpu_baseline, runs=args.c3_runs)}), flush=True)
        return

    A = problems.workload(args.workload)
    b = problems.rhs(A.n)
    dA = tuple(torch.from_numpy(a).to(dev) for a in (A.row_ptr, A.col_idx, A.val))
    db = torch.from_numpy(b).to(dev)
    dx = torch.zeros_like(db)
    stream = torch.cuda.current_stream()

    def one_step(precision, profile=False, **kw):
        return solve_once(camg, A, dA, db, dx, stream, precision, profile=profile, **kw)

    for _ in range(args.warmup):
        one_step(camg.FP64)
        if not args.no_mixed:
            one_step(camg.MIXED_FP32)
    torch.cuda.synchronize()
    T0 = time.perf_counter()
    fp64 = [one_step(camg.FP64, profile=True) for _ in range(args.steps)]
    torch.cuda.synchronize()
    T1 = time.perf_counter()
    x64 = dx.cpu().numpy().copy()
    mixed = []
    if not args.no_mixed:
        mixed = [one_step(camg.MIXED_FP32, profile=True) for _ in range(args.steps)]
        xm = dx.cpu().numpy().copy()
    log(f"c2: fp64 {med(fp64, 'solve_ms')} ms")
    copy_gbs = copy_kernel_gbs(dev)

    # the FSAI smoother (M^{-1} = G^T G) on the same system, FP64 and mixed
    fsai = {}
    if not args.no_fsai:
        for prec, key in ((camg.FP64, "fp64"), (camg.MIXED_FP32, "mixed")):
            one_step(prec, smoother=camg.SMOOTH_FSAI)
            rs = [one_step(prec, smoother=camg.SMOOTH_FSAI) for _ in range(max(1, min(args.steps, 3)))]
            fsai[key] = {"solve_ms": med(rs, "solve_ms"), "setup_ms": med(rs, "setup_ms"),
                         "iters": rs[-1]["iters"], "true_relres": rs[-1]["true_relres"]}
        # the adaptive factor (the paper's smoother, eq. smo), alone and with
        # extended+i interpolation (the paper's default set-up)
        for interp, akey in ((camg.INTERP_DIRECT, "adaptive"), (camg.INTERP_EXTI, "adaptive_extended_i")):
            fsai[akey] = {}
            for prec, key in ((camg.FP64, "fp64"), (camg.MIXED_FP32, "mixed")):
                one_step(prec, smoother=camg.SMOOTH_AFSAI, interp=interp)
                rs = [one_step(prec, smoother=camg.SMOOTH_AFSAI, interp=interp) for _ in range(max(1, min(args.steps, 2)))]
                fsai[akey][key] = {"solve_ms": med(rs, "solve_ms"), "setup_ms": med(rs, "setup_ms"),
                                   "iters": rs[-1]["iters"], "true_relres": rs[-1]["true_relres"],
                                   "smoother_setup_ms": round(rs[-1]["info"].setup_phase_ms[1], 2)}
        fsai["adaptive"]["params"] = {"afsai_steps": 10, "afsai_step": 2, "afsai_eps": 0.01}

    # the paper's interpolations on the same system (Jacobi, FP64), as in its
    # comparison of prolongations: complexities, iterations, set-up and solve
    interps = {}
    if not args.no_interp:
        for var, key in ((camg.INTERP_CLASSICAL, "classical"), (camg.INTERP_EXTI, "extended_i"),
                         (camg.INTERP_HYBRID, "hybrid")):
            one_step(camg.FP64, interp=var)
            rs = [one_step(camg.FP64, interp=var) for _ in range(max(1, min(args.steps, 3)))]
            inf = rs[-1]["info"]
            interps[key] = {"solve_ms": med(rs, "solve_ms"), "setup_ms": med(rs, "setup_ms"),
                            "iters": rs[-1]["iters"], "true_relres": rs[-1]["true_relres"],
                            "levels": inf.levels, "grid_complexity": round(inf.grid_complexity, 4),
                            "operator_complexity": round(inf.operator_complexity, 4)}

    # host API on the same hierarchy: b copied in and x out over PCIe around the device solve
    sh = camg.Solver.from_device(A.n, *dA, stream=stream, max_iter=5000)
    sh.solve(b)
    th = []
    for _ in range(max(1, min(args.steps, 3))):
        t0 = time.perf_counter()
        sh.solve(b)
        th.append((time.perf_counter() - t0) * 1e3)
    sh.close()
    host_ms = statistics.median(th)

    info = fp64[-1]["info"]
    solve_ms = statistics.median(r["solve_ms"] for r in fp64)
    setup_ms = statistics.median(r["setup_ms"] for r in fp64)
    iters = fp64[-1]["iters"]
    # level-0 post-smoothing kernel, timed with HIP events on the solve stream
    launches = sum(r["prof"][1] for r in fp64)
    k_ms = sum(r["prof"][0] for r in fp64) / max(launches, 1)
    compact = bool(info.compact_cols & 1)
    k_bytes = post0_bytes(A.n, A.nnz, col_bytes=2 if compact else 4)
    k_int32 = post0_bytes(A.n, A.nnz)
    cnt = committed_counters(f"post0_{args.workload}_pmc") or {}
    traffic = cnt.get("traffic_bytes_per_launch")
    per_iter_ms = solve_ms / max(iters, 1)

    out = {
        "metric": METRIC,
        "value": round(solve_ms, 4),
        "unit": "ms",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round((T1 - T0) * 1e3 / args.steps, 4),
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": args.workload, "description": WORKLOADS[args.workload], "n": A.n, "nnz": A.nnz,
                   "rtol": 1e-8, "levels": info.levels, "grid_complexity": round(info.grid_complexity, 4),
                   "operator_complexity": round(info.operator_complexity, 4)},
        "fp64": {"solve_ms": round(solve_ms, 4), "setup_ms": round(setup_ms, 4), "iters": iters,
                 "ms_per_iter": round(per_iter_ms, 5), "true_relres": fp64[-1]["true_relres"],
                 "vcycle_alg_bytes": vcycle_bytes(info), "host_api_solve_ms": round(host_ms, 4),
                 "setup_phase_ms": {k: round(info.setup_phase_ms[i], 2) for i, k in enumerate(camg.SETUP_PHASES)}},
        "roofline": roofline_of(
            "level-0 post-smoothing, FP64 (k_rows<double, EPost, dot>)", k_bytes, k_ms, launches, traffic,
            compact_cols=compact, copy_kernel_gbs=round(copy_gbs, 1), copy_kernel_frac=round(copy_gbs / HBM_PEAK_GBS, 4),
            int32_model_bytes=k_int32,
            int32_model_gbs=round(k_int32 / (k_ms * 1e-3) / 1e9, 2) if launches else 0.0),
    }
    if mixed:
        m_ms = statistics.median(r["solve_ms"] for r in mixed)
        ml = sum(r["prof"][1] for r in mixed)
        mk_ms = sum(r["prof"][0] for r in mixed) / max(ml, 1)
        minfo = mixed[-1]["info"]
        mcomp = bool(minfo.compact_cols & 1)
        mtraffic = (committed_counters(f"post0_{args.workload}_pmc") or {}).get("traffic_bytes_per_launch_fp32")
        out["mixed"] = {"solve_ms": round(m_ms, 4), "setup_ms": med(mixed, "setup_ms"),
                        "iters": mixed[-1]["iters"], "true_relres": mixed[-1]["true_relres"],
                        "speedup_vs_fp64": round(solve_ms / m_ms, 4),
                        "rel_err_vs_fp64_gpu": float(np.linalg.norm(xm - x64) / np.linalg.norm(x64)),
                        "roofline": roofline_of("level-0 post-smoothing, FP32 V-cycle (k_rows<float, EPost, dot>)",
                                                post0_bytes(A.n, A.nnz, fp32=True, col_bytes=2 if mcomp else 4),
                                                mk_ms, ml, mtraffic, compact_cols=mcomp)}
    if fsai:
        out["fsai_smoother"] = fsai
    if interps:
        out["interpolations"] = interps
    if not args.no_c1:
        out["c1"] = c1_run()
        log(f"c1: {out['c1']['solve_ms_median']} ms")
    if elas is not None:
        out["c3"] = c3_run(elas.result(), args.no_cpu_baseline, runs=args.c3_runs)
        log(f"c3: fp64 {out['c3']['fp64']['solve_ms']} ms, mixed {out['c3']['mixed']['solve_ms']} ms")
    pool.shutdown()
    if args.batched:
        out["batched"] = batched_run(args.batched, max(1, min(args.steps, 3)))
        log(f"batched: {out['batched']['block_mixed_autotuned_ms']} ms")
    if args.small_systems:
        out["small_systems"] = small_systems_run(args.small_systems)
    if not args.no_serve:
        out["serving"] = serve_run(rates, args.serve_requests)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(A, b, x64, iters, xm if mixed else None)
        if mixed:
            out["mixed"]["rel_err_vs_oracle"] = out["cpu_baseline"].pop("mixed_vs_oracle_rel_err")
    print(json.dumps(out), flush=True)


# ====================================================================== c1
def c1_run(runs=21):
    """2D 5-point Poisson, 64x64 interior (n = 4096): set-up and FP64 solve
    to rtol 1e-8, median over `runs` timed runs after two warm-ups, with the
    oracle's solve of the same system for the iteration count and error."""
    import numpy as np
    import torch

    import oracle
    from paper_2102_07417_amd import camg, problems

    dev = torch.device("cuda:0")
    A = problems.workload("poisson2d_64")
    b = problems.rhs(A.n)
    dA = tuple(torch.from_numpy(a).to(dev) for a in (A.row_ptr, A.col_idx, A.val))
    db = torch.from_numpy(b).to(dev)
    dx = torch.zeros_like(db)
    stream = torch.cuda.current_stream()
    rs = [solve_once(camg, A, dA, db, dx, stream, camg.FP64) for _ in range(runs + 2)][2:]
    x = dx.cpu().numpy()
    ro = oracle.Hierarchy(A).solve(b, 1e-8)
    # repeated solves on one resident hierarchy (the graphs stay captured)
    s = camg.Solver.from_device(A.n, *dA, stream=stream)
    s.solve_dev(db, dx, stream=stream)
    ts = []
    for _ in range(runs):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s.solve_dev(db, dx, stream=stream)
        torch.cuda.synchronize()
        ts.append((time.perf_counter() - t0) * 1e3)
    levels = s.nlev
    s.close()
    return {"workload": "poisson2d_64", "n": A.n, "nnz": A.nnz, "levels": levels, "runs": runs,
            "setup_ms_median": med(rs, "setup_ms"), "solve_ms_median": med(rs, "solve_ms"),
            "solve_ms_min": round(min(r["solve_ms"] for r in rs), 4),
            "resident_solve_ms_median": round(statistics.median(ts), 4),
            "iters": rs[-1]["iters"], "oracle_iters": ro.iters, "true_relres": rs[-1]["true_relres"],
            "rel_err_vs_oracle": float(np.linalg.norm(x - ro.x) / np.linalg.norm(ro.x))}


# ====================================================================== c3
def c3_run(A, no_oracle_check=False, runs=2):
    """Q1 elasticity on 64^3 elements (n = 811,200, nnz = 63,695,790; the
    paper's mechanical class, ~80 nonzeros per row), direct interpolation:
    set-up and solve to rtol 1e-8 in FP64 and in mixed precision (FP32
    V-cycle), one warm-up then the median of `runs`; the level-0
    post-smoothing kernel of each precision timed by HIP events inside the
    solves.  The FP64 and mixed solutions are compared with the oracle's
    stored natural-stop FP64 solve (4096 sampled unknowns)."""
    import numpy as np
    import torch

    from paper_2102_07417_amd import camg, problems

    dev = torch.device("cuda:0")
    b = problems.rhs(A.n)
    dA = tuple(torch.from_numpy(a).to(dev) for a in (A.row_ptr, A.col_idx, A.val))
    db = torch.from_numpy(b).to(dev)
    dx = torch.zeros_like(db)
    stream = torch.cuda.current_stream()
    gold = None
    if not no_oracle_check:
        sys.path.insert(0, os.path.join(ROOT, "tests", "golden"))
        import make_oracle_solves as G
        gold = G.read("elasticity_64")
    cnt = committed_counters("post0_elasticity_64_pmc") or {}
    out = {"workload": "elasticity_64", "description": WORKLOADS["elasticity_64"], "n": A.n, "nnz": A.nnz}
    for key, prec, fp32 in (("fp64", camg.FP64, False), ("mixed", camg.MIXED_FP32, True)):
        solve_once(camg, A, dA, db, dx, stream, prec)
        rs = [solve_once(camg, A, dA, db, dx, stream, prec, profile=True) for _ in range(runs)]
        x = dx.cpu().numpy()
        inf = rs[-1]["info"]
        launches = sum(r["prof"][1] for r in rs)
        k_ms = sum(r["prof"][0] for r in rs) / max(launches, 1)
        compact = bool(inf.compact_cols & 1)
        kb = post0_bytes(A.n, A.nnz, fp32=fp32, col_bytes=2 if compact else 4)
        d = {"setup_ms": med(rs, "setup_ms"), "solve_ms": med(rs, "solve_ms"), "iters": rs[-1]["iters"],
             "status": rs[-1]["status"], "true_relres": rs[-1]["true_relres"], "levels": inf.levels,
             "operator_complexity": round(inf.operator_complexity, 4),
             "roofline": roofline_of("level-0 post-smoothing, %s" % ("FP32" if fp32 else "FP64"), kb, k_ms,
                                     launches, cnt.get("traffic_bytes_per_launch" + ("_fp32" if fp32 else "")),
                                     compact_cols=compact,
                                     int32_model_bytes=post0_bytes(A.n, A.nnz, fp32=fp32))}
        if gold is not None:
            xs = x[gold["idx"]]
            d["oracle_iters"] = int(gold["iters"])
            d["sampled_rel_err_vs_oracle"] = float(np.linalg.norm(xs - gold["x"]) / np.linalg.norm(gold["x"]))
        out[key] = d
    out["mixed"]["speedup_vs_fp64"] = round(out["fp64"]["solve_ms"] / out["mixed"]["solve_ms"], 4)
    # the paper's smoother for its mechanical problems: adaptive FSAI (one run per precision)
    out["adaptive_fsai"] = {}
    for key, prec in (("fp64", camg.FP64), ("mixed", camg.MIXED_FP32)):
        r = solve_once(camg, A, dA, db, dx, stream, prec, smoother=camg.SMOOTH_AFSAI)
        d = {"setup_ms": round(r["setup_ms"], 2), "solve_ms": round(r["solve_ms"], 2), "iters": r["iters"],
             "status": r["status"], "true_relres": r["true_relres"],
             "smoother_setup_ms": round(r["info"].setup_phase_ms[1], 2)}
        if gold is not None:
            xs = dx.cpu().numpy()[gold["idx"]]
            d["sampled_rel_err_vs_oracle_jacobi_solution"] = float(np.linalg.norm(xs - gold["x"]) / np.linalg.norm(gold["x"]))
        out["adaptive_fsai"][key] = d
    return out


# ====================================================================== c4
def batched_run(k, steps):
    """Block of k right-hand sides on the 160^3 anisotropic problem: one
    FP32-V-cycle / FP64-PCG block solve (all columns to rtol 1e-8) against k
    sequential FP64 single-vector solves on the same GPU code.  Hierarchies
    are set up before the timed regions (both reuse one hierarchy for all
    columns); the block engine is warm (created by an untimed first call).
    The level-0 block post-smoothing kernel of the autotuned mixed solve is
    timed by HIP events inside untimed extra solves."""
    import numpy as np  # noqa: F401
    import torch

    from paper_2102_07417_amd import camg, problems

    dev = torch.device("cuda:0")
    A = problems.workload("aniso3d_160")
    B = problems.rhs_block(A.n, k)
    dA = tuple(torch.from_numpy(a).to(dev) for a in (A.row_ptr, A.col_idx, A.val))
    dB = torch.from_numpy(B).to(dev)
    stream = torch.cuda.current_stream()

    s64 = camg.Solver.from_device(A.n, *dA, stream=stream, max_iter=5000)
    cols = [dB[:, j].contiguous() for j in range(k)]
    X64 = torch.zeros((A.n, k), dtype=torch.float64, device=dev)
    xs = torch.zeros(A.n, dtype=torch.float64, device=dev)
    s64.solve_dev(cols[0], xs, rtol=1e-8, stream=stream)  # warm (graphs)
    seq = []
    seq_iters = []
    for _ in range(steps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for j in range(k):
            r = s64.solve_dev(cols[j], xs, rtol=1e-8, stream=stream)
            X64[:, j].copy_(xs)
            seq_iters.append(r.iters)
        torch.cuda.synchronize()
        seq.append((time.perf_counter() - t0) * 1e3)

    def block(solver):
        dX = torch.zeros_like(dB)
        solver.solve_multi_dev(dB, dX, rtol=1e-8, stream=stream)  # warm: engine + graphs
        ts = []
        for _ in range(steps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            r = solver.solve_multi_dev(dB, dX, rtol=1e-8, stream=stream)
            torch.cuda.synchronize()
            ts.append((time.perf_counter() - t0) * 1e3)
        err = ((dX - X64).norm(dim=0) / X64.norm(dim=0)).max().item()
        return statistics.median(ts), r, err

    def kernel_time(solver):
        dX = torch.zeros_like(dB)
        camg.camg_profile(solver.h, 4)
        solver.solve_multi_dev(dB, dX, rtol=1e-8, stream=stream)
        torch.cuda.synchronize()
        return camg.camg_profile(solver.h, 0)

    b64_ms, r64, e64 = block(s64)
    p64 = kernel_time(s64)
    s64.close()
    smx = camg.Solver.from_device(A.n, *dA, stream=stream, max_iter=5000, precision=camg.MIXED_FP32)
    bmx_ms, rmx, emx = block(smx)
    pmx = kernel_time(smx)  # the rule schedule: the same kernel in every run (the autotuner's pick may vary)
    info = smx.info
    smx.close()
    # the same with autotuned row schedules (tuning happens in the untimed warm call)
    smt = camg.Solver.from_device(A.n, *dA, stream=stream, max_iter=5000, precision=camg.MIXED_FP32)
    smt.set_option(camg.OPT_AUTOTUNE, 1)
    t0 = time.perf_counter()
    bmt_ms, rmt, emt = block(smt)
    tune_s = time.perf_counter() - t0
    smt.close()
    seq_ms = statistics.median(seq)
    kslots = 1 << (k - 1).bit_length()
    cnt = committed_counters("blockpost0_aniso3d_160_rhs32_pmc") or {}
    return {"workload": "aniso3d_160", "n": A.n, "nnz": A.nnz, "rhs": k, "slots": kslots, "levels": info.levels,
            "sequential_fp64_ms": round(seq_ms, 3),
            "sequential_iters": [int(min(seq_iters)), int(max(seq_iters))],
            "block_fp64_ms": round(b64_ms, 3), "block_fp64_speedup": round(seq_ms / b64_ms, 3),
            "block_fp64_iters": [int(r64.iters.min()), int(r64.iters.max())],
            "block_fp64_max_true_relres": float(r64.true_relres.max()),
            "block_fp64_max_rel_err_vs_sequential": e64,
            "block_mixed_ms": round(bmx_ms, 3), "block_mixed_speedup": round(seq_ms / bmx_ms, 3),
            "block_mixed_iters": [int(rmx.iters.min()), int(rmx.iters.max())],
            "block_mixed_max_true_relres": float(rmx.true_relres.max()),
            "block_mixed_max_rel_err_vs_sequential_fp64": emx,
            "block_mixed_autotuned_ms": round(bmt_ms, 3), "block_mixed_autotuned_speedup": round(seq_ms / bmt_ms, 3),
            "block_mixed_autotuned_iters": [int(rmt.iters.min()), int(rmt.iters.max())],
            "block_mixed_autotuned_max_true_relres": float(rmt.true_relres.max()),
            "autotune_and_runs_s": round(tune_s, 2),
            "roofline_mixed": roofline_of(
                "level-0 block post-smoothing, FP32 V-cycle, %d slots, rule schedule (mk_rows<float, MEPost>)" % kslots,
                block_post0_bytes(A.n, A.nnz, kslots, True), pmx[0] / max(pmx[1], 1), pmx[1],
                cnt.get("traffic_bytes_per_launch_fp32")),
            "roofline_fp64": roofline_of(
                "level-0 block post-smoothing, FP64, %d slots (mk_rows<double, MEPost>)" % kslots,
                block_post0_bytes(A.n, A.nnz, kslots, False), p64[0] / max(p64[1], 1), p64[1],
                cnt.get("traffic_bytes_per_launch"))}


def small_systems_run(count, steps=3):
    """count independent 2D lognormal(0, 2) systems on 100x100 cells (each
    its own coefficient seed and right-hand side, n = 10,000), FP64, rtol
    1e-8: one launch with a workgroup per system against solving them one
    after another with the single-system path.  Hierarchies are set up
    before the clock starts."""
    import torch

    from paper_2102_07417_amd import camg, problems

    dev = torch.device("cuda:0")
    solvers, db, dx = [], [], []
    for k in range(count):
        A = problems.lognormal2d(100, 2.0, 5000 + k)
        solvers.append(camg.Solver(A, max_iter=2000))
        db.append(torch.from_numpy(problems.rhs(A.n, 9000 + k)).to(dev))
        dx.append(torch.zeros_like(db[-1]))
    camg.solve_batch_dev(solvers, db, dx)
    tb = []
    for _ in range(steps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        it, rel, st = camg.solve_batch_dev(solvers, db, dx)
        torch.cuda.synchronize()
        tb.append((time.perf_counter() - t0) * 1e3)
    xb = [x.clone() for x in dx]
    for k in range(count):
        solvers[k].solve_dev(db[k], dx[k])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    its = []
    for k in range(count):
        its.append(solvers[k].solve_dev(db[k], dx[k]).iters)
    torch.cuda.synchronize()
    seq_ms = (time.perf_counter() - t0) * 1e3
    err = max(float(((xb[k] - dx[k]).norm() / dx[k].norm()).item()) for k in range(count))
    for s in solvers:
        s.close()
    bms = statistics.median(tb)
    return {"workload": "lognormal2d_100 x %d (independent seeds)" % count, "n_each": 10000, "systems": count,
            "batch_ms": round(bms, 3), "sequential_ms": round(seq_ms, 3), "speedup": round(seq_ms / bms, 3),
            "iters": [int(it.min()), int(it.max())], "sequential_iters": [min(its), max(its)],
            "max_true_relres": float(rel.max()), "not_ok": int((st != camg.OK).sum()),
            "max_rel_diff_vs_sequential": err, "systems_per_s": round(count / (bms * 1e-3), 1)}


# ====================================================================== c5
SERVE_RATES = [60.0, 120.0]


def serve_run(rates, requests=1000, budget_gb=32.0, slots=16, seed=2021, interp=None):
    """Serving sweep: the 8 resident systems (mixed-precision hierarchies,
    one slot engine of `slots` columns and one stream each), `requests`
    Poisson arrivals per rate, system uniform, 1-16 right-hand sides per
    request (uniform), each request's right-hand sides U[-1, 1] drawn on the
    device from a generator seeded with the request id, rtol 1e-8.
    Latency is from the scheduled arrival to the poll that returned the
    completion; a request still unfinished when the drain limit ends the
    rate counts as censored at that time in the percentiles."""
    import numpy as np
    import torch

    from paper_2102_07417_amd import camg, problems

    dev = torch.device("cuda:0")
    interp = camg.INTERP_HYBRID if interp is None else interp
    systems = []
    t0 = time.perf_counter()
    for name, make in problems.SERVING_SYSTEMS:
        A = make()
        s = camg.Solver.from_device(A.n, torch.from_numpy(A.row_ptr).to(dev), torch.from_numpy(A.col_idx).to(dev),
                                    torch.from_numpy(A.val).to(dev), precision=camg.MIXED_FP32, max_iter=2000,
                                    interp=interp)
        systems.append((name, A.n, s))
    setup_s = time.perf_counter() - t0
    budget = int(budget_gb * (1 << 30))
    gen = torch.Generator(device=dev)

    def rhs_of(rid, n, k):
        gen.manual_seed(int(rid))
        return torch.rand((n, k), generator=gen, dtype=torch.float64, device=dev) * 2.0 - 1.0

    out = {"systems": [{"name": nm, "n": n, "iters_alone": None} for nm, n, _ in systems], "slots": slots,
           "budget_bytes": budget, "rtol": 1e-8, "precision": "mixed (FP32 V-cycle, FP64 PCG)",
           "interpolation": {camg.INTERP_DIRECT: "direct", camg.INTERP_HYBRID: "hybrid",
                             camg.INTERP_EXTI: "extended+i"}.get(interp, str(interp)),
           "rhs": "request r: U[-1,1] from torch.Generator(cuda).manual_seed(r)",
           "generation_and_setup_s": round(setup_s, 2), "rates": []}
    # one column alone per system: its iterations and solve time on an idle device
    for si, (nm, n, s) in enumerate(systems):
        B = rhs_of(10 ** 6 + si, n, 1)
        X = torch.zeros_like(B)
        s.solve_multi_dev(B, X)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = s.solve_multi_dev(B, X)
        torch.cuda.synchronize()
        out["systems"][si].update({"iters_alone": int(r.iters.max()),
                                   "one_column_ms": round((time.perf_counter() - t0) * 1e3, 2)})
    for lam in rates:
        srv = camg.Server(budget)
        for _, _, s in systems:
            srv.add(s, slots)
        rng = np.random.default_rng(int(seed + 1000 * lam))
        count = int(requests)
        arr = np.cumsum(rng.exponential(1.0 / lam, count))
        sys_of = rng.integers(0, len(systems), count)
        k_of = rng.integers(1, 17, count)
        # warm every engine (graph capture) before the clock starts
        for si, (_, n, _) in enumerate(systems):
            srv.submit(si, rhs_of(2 * 10 ** 6 + si, n, 1), torch.empty((n, 1), dtype=torch.float64, device=dev),
                       rtol=1e-8, max_iter=2000, tag=-1 - si)
        warm = 0
        while warm < len(systems):
            warm += len(srv.poll())
        torch.cuda.synchronize()
        done_t, res = {}, {}
        nxt = 0
        limit = arr[-1] + 30.0  # drain for at most 30 s after the last arrival
        T0 = time.perf_counter()
        while len(done_t) < count:
            now = time.perf_counter() - T0
            if now > limit:
                break
            while nxt < count and arr[nxt] <= now:
                si, k = int(sys_of[nxt]), int(k_of[nxt])
                n = systems[si][1]
                srv.submit(si, rhs_of(nxt, n, k), torch.empty((n, k), dtype=torch.float64, device=dev),
                           rtol=1e-8, max_iter=2000, tag=nxt)
                nxt += 1
            for c in srv.poll():
                done_t[c["tag"]] = time.perf_counter() - T0
                res[c["tag"]] = c
        T1 = time.perf_counter() - T0
        srv.close()
        # latency of every submitted request; unfinished ones censored at the end
        lat = np.array([(done_t.get(i, T1) - arr[i]) for i in range(nxt)]) * 1e3
        censored = nxt - len(done_t)
        sub_sys, sub_k = sys_of[:nxt], k_of[:nxt]
        fin = np.array(sorted(done_t))
        rhs = int(k_of[fin].sum()) if len(fin) else 0
        worst = max((r["true_relres"] for r in res.values()), default=0.0)
        bad = sum(1 for r in res.values() if r["status"] != camg.OK)
        per_sys = {}
        for si, (nm, _, _) in enumerate(systems):
            m = sub_sys == si
            if m.any():
                per_sys[nm] = {"p50_ms": round(float(np.percentile(lat[m], 50)), 2),
                               "p99_ms": round(float(np.percentile(lat[m], 99)), 2), "requests": int(m.sum()),
                               "rhs": int(sub_k[m].sum())}
        busy_s = max(T1, 1e-9)
        out["rates"].append({"rate_per_s": lam, "requests": count, "submitted": int(nxt),
                             "completed": int(len(done_t)), "censored": int(censored), "rhs_completed": rhs,
                             "p50_ms": round(float(np.percentile(lat, 50)), 2),
                             "p99_ms": round(float(np.percentile(lat, 99)), 2),
                             "max_ms": round(float(lat.max()), 2),
                             "mean_queue_ms": round(float(np.mean([r["queue_ms"] for r in res.values()])), 2),
                             "requests_per_s": round(len(done_t) / busy_s, 2), "solves_per_s": round(rhs / busy_s, 2),
                             "wall_s": round(T1, 3), "max_true_relres": worst, "not_ok": bad,
                             "per_system": per_sys})
        log(f"serve rate {lam}: p50 {out['rates'][-1]['p50_ms']} ms p99 {out['rates'][-1]['p99_ms']} ms "
            f"{out['rates'][-1]['solves_per_s']} solves/s, censored {censored}")
    for _, _, s in systems:
        s.close()
    return out


# ====================================================================== opt-in runs
def bamg_run(ne):
    """Q1 elasticity on ne^3 elements (b ~ U[-1, 1]): set-up and solve to
    rtol 1e-8 with direct interpolation, then with BAMG interpolation over
    the six rigid body modes (FP64 and mixed; mixed with the prolongation
    smoothed and filtered to rho = 0.7; mixed with 3 SRQM steps on the
    modes; direct and BAMG with the FSAI_JACOBI smoother: FSAI on the
    levels whose rows have at most 192 entries on or below the diagonal,
    Jacobi on BAMG's denser coarse levels; direct and BAMG with the
    adaptive FSAI smoother), then from six random vectors
    with and without 10 SRQM steps.  Each configuration runs once untimed,
    then once timed."""
    import numpy as np
    import torch

    from paper_2102_07417_amd import camg, problems

    dev = torch.device("cuda:0")
    A = problems.elasticity3d(ne)
    b = problems.rhs(A.n)
    V = problems.elasticity_rigid_modes(ne)
    rp, ci, va = (torch.from_numpy(a).to(dev) for a in (A.row_ptr, A.col_idx, A.val))
    dV = torch.from_numpy(np.ascontiguousarray(V)).to(dev)
    db = torch.from_numpy(b).to(dev)
    dx = torch.zeros_like(db)
    stream = torch.cuda.current_stream()

    def run(precision, bamg, smoother=0, **extra):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        kw = dict(interp=camg.INTERP_BAMG, V=dV) if bamg else {}
        kw["smoother"] = smoother
        kw.update(extra)
        s = camg.Solver.from_device(A.n, rp, ci, va, stream=stream, precision=precision, max_iter=5000, **kw)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        dx.zero_()
        r = s.solve_dev(db, dx, rtol=1e-8, stream=stream)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        inf = s.info
        s.close()
        return {"setup_ms": round((t1 - t0) * 1e3, 3), "solve_ms": round((t2 - t1) * 1e3, 3), "iters": r.iters,
                "status": r.status, "true_relres": r.true_relres, "levels": inf.levels,
                "grid_complexity": round(inf.grid_complexity, 4),
                "operator_complexity": round(inf.operator_complexity, 4),
                "setup_phase_ms": {k: round(inf.setup_phase_ms[i], 2) for i, k in enumerate(camg.SETUP_PHASES)}}

    out = {"ne": ne, "n": A.n, "nnz": A.nnz, "test_vectors": 6}
    for key, prec, bamg, sm in (("direct_fp64", camg.FP64, False, camg.SMOOTH_JACOBI),
                                ("bamg_fp64", camg.FP64, True, camg.SMOOTH_JACOBI),
                                ("direct_mixed", camg.MIXED_FP32, False, camg.SMOOTH_JACOBI),
                                ("bamg_mixed", camg.MIXED_FP32, True, camg.SMOOTH_JACOBI),
                                ("bamg_psmooth_filter_mixed", camg.MIXED_FP32, True, camg.SMOOTH_JACOBI),
                                ("bamg_srqm3_mixed", camg.MIXED_FP32, True, camg.SMOOTH_JACOBI),
                                ("direct_fsai_jacobi_mixed", camg.MIXED_FP32, False, camg.SMOOTH_FSAI_JACOBI),
                                ("bamg_fsai_jacobi_fp64", camg.FP64, True, camg.SMOOTH_FSAI_JACOBI),
                                ("bamg_fsai_jacobi_mixed", camg.MIXED_FP32, True, camg.SMOOTH_FSAI_JACOBI),
                                ("direct_afsai_mixed", camg.MIXED_FP32, False, camg.SMOOTH_AFSAI),
                                ("bamg_afsai_fp64", camg.FP64, True, camg.SMOOTH_AFSAI),
                                ("bamg_afsai_mixed", camg.MIXED_FP32, True, camg.SMOOTH_AFSAI)):
        extra = {"psmooth": 1, "pfilter": 0.7} if "psmooth" in key else {}
        if "srqm" in key:
            extra["srqm_iters"] = 3
        run(prec, bamg, sm, **extra)
        out[key] = run(prec, bamg, sm, **extra)
        log(f"elasticity {ne}^3 {key}: {out[key]}")
    # without a known near kernel: six seeded N(0, 1) vectors, as given and
    # after 10 SRQM steps
    dV.copy_(torch.from_numpy(np.random.default_rng(0).standard_normal((A.n, 6))).to(dev))
    for key, k in (("bamg_random_mixed", 0), ("bamg_random_srqm10_mixed", 10)):
        run(camg.MIXED_FP32, True, camg.SMOOTH_JACOBI, srqm_iters=k)
        out[key] = run(camg.MIXED_FP32, True, camg.SMOOTH_JACOBI, srqm_iters=k)
        log(f"elasticity {ne}^3 {key}: {out[key]}")
    return out


def poisson_context_run(grid):
    """7-point Poisson on grid^3 (404^3 = the paper's poi65m: n = 65,939,264,
    nnz = 460,595,552), assembled on the GPU, b ~ U[-1, 1] drawn on the
    GPU.  Set-up and FP64 / mixed solve to rtol 1e-8 with Jacobi and
    extended+i interpolation (the paper's Chr-jac configuration), then with
    direct interpolation.  Each configuration runs once untimed, then once
    timed."""
    import torch

    from paper_2102_07417_amd import camg, problems

    dev = torch.device("cuda:0")
    t0 = time.perf_counter()
    n, rp, ci, va = problems.poisson3d_torch(grid, device=dev)
    torch.cuda.synchronize()
    gen_s = time.perf_counter() - t0
    g = torch.Generator(device=dev)
    g.manual_seed(7417)
    db = torch.rand(n, dtype=torch.float64, device=dev, generator=g) * 2.0 - 1.0
    dx = torch.zeros_like(db)
    stream = torch.cuda.current_stream()
    log(f"poisson {grid}^3: n={n} nnz={int(rp[-1])} assembled in {gen_s:.1f} s")

    def run(interp, precision):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s = camg.Solver.from_device(n, rp, ci, va, stream=stream, interp=interp, precision=precision)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        dx.zero_()
        r = s.solve_dev(db, dx, rtol=1e-8, stream=stream)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        inf = s.info
        s.close()
        return {"setup_s": round(t1 - t0, 4), "solve_s": round(t2 - t1, 4), "iters": r.iters, "status": r.status,
                "true_relres": r.true_relres, "ms_per_iter": round((t2 - t1) * 1e3 / max(r.iters, 1), 3),
                "levels": inf.levels, "grid_complexity": round(inf.grid_complexity, 4),
                "operator_complexity": round(inf.operator_complexity, 4),
                "device_gb": round(inf.device_bytes / 1e9, 2),
                "setup_phase_ms": {k: round(inf.setup_phase_ms[i], 2) for i, k in enumerate(camg.SETUP_PHASES)}}

    out = {"grid": grid, "n": n, "nnz": int(rp[-1]), "assembly_s": round(gen_s, 2)}
    for key, interp, prec in (("extended_i_fp64", camg.INTERP_EXTI, camg.FP64),
                              ("extended_i_mixed", camg.INTERP_EXTI, camg.MIXED_FP32),
                              ("direct_fp64", camg.INTERP_DIRECT, camg.FP64)):
        run(interp, prec)
        out[key] = run(interp, prec)
        log(f"poisson {grid}^3 {key}: {out[key]}")
    out["paper_chr_jac_poi65m"] = {"iters": 16, "setup_s": 3.81, "solve_s": 1.65, "cores": 384,
                                   "hardware": "IBM POWER9 (Marconi100)", "grid_complexity": 1.327,
                                   "operator_complexity": 4.036}
    return out


# ====================================================================== CPU baseline
def cpu_baseline(A, b, x_gpu, gpu_iters, x_mixed=None):
    """The CPU oracle (plain single-threaded C, FP64, built with gcc -O2
    -ffp-contract=off) on the same system, pinned to one core: set-up and
    full solve, the solve time being the figure compared."""
    import numpy as np

    import oracle

    with pinned_to_one_core() as pin:
        t0 = time.perf_counter()
        h = oracle.Hierarchy(A, max_iter=5000)
        t1 = time.perf_counter()
        r = h.solve(b, 1e-8, max_iter=5000)
        t2 = time.perf_counter()
    err = float(np.linalg.norm(x_gpu - r.x) / np.linalg.norm(r.x))
    out = {"value": round((t2 - t1) * 1e3, 3), "unit": "ms", "cores": 1, "kind": "oracle",
           "sample": "full set-up and full FP64 PCG solve of the same system (one run, one thread)",
           "pinned_cpu": pin.cpu, "setup_ms": round((t1 - t0) * 1e3, 3), "iters": r.iters, "gpu_iters": gpu_iters,
           "gpu_vs_oracle_rel_err": err}
    out.update(host_facts())
    if x_mixed is not None:
        out["mixed_vs_oracle_rel_err"] = float(np.linalg.norm(x_mixed - r.x) / np.linalg.norm(r.x))
    return out


if __name__ == "__main__":
    main()
