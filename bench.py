"""Time-to-solution of the shrink-and-expand LOBPCG on one MI355X.

Workload (default): 3-D 7-point Dirichlet Laplacian on a 128^3 grid
(n = 2,097,152, 14,581,760 nonzeros, FP64 CSR), the 64 smallest eigenpairs
with 32 extra block columns (block 96, n_es = 69), tol 1e-8, Gaussian starting
block from a fixed seed. One step = one complete solve with the `fix`
shrink-and-expand strategy (inputs resident in HBM before timing). After the
timed solves: one solve with HIP events around every launch (the per-kernel
table and the roofline), the fixed-block solve (no strategy) on the same input
(median of up to three runs), a short serving leg (Poisson arrivals of the
serving stream: p50 / p99 latency and solves/s), and the FP64 oracle on the
host cores for a few iterations (the CPU baseline).

Prints one JSON line (see the contract in the repository's design notes).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "time-to-solution & HBM GB/s, shrink-expand vs fixed block; p50/p99 latency"
MAGNETIC_PHASES = (0.3, 0.7, 1.1)  # phase per grid step of the complex Hermitian workload


# Workloads: matrix family and default sizes (n_ev, n_extra, solver, precision).
WORKLOADS = {
    "laplace3d": dict(grid=128, n_ev=64, n_extra=32, x0_seed=202),
    "laplace2d": dict(grid=32, n_ev=8, n_extra=8, x0_seed=201),
    "magnetic": dict(grid=128, n_ev=64, n_extra=32, x0_seed=207),
    "anderson": dict(grid=100, n_ev=200, n_extra=50, x0_seed=203),
    "chunglu": dict(nodes=500000, n_ev=32, n_extra=16, x0_seed=204),
    "serving": dict(x0_seed=305),
}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="laplace3d", choices=sorted(WORKLOADS))
    ap.add_argument("--grid", type=int, default=None, help="3-D grid side m (n = m^3)")
    ap.add_argument("--nodes", type=int, default=None, help="Chung-Lu graph size")
    ap.add_argument("--n-ev", type=int, default=None)
    ap.add_argument("--n-extra", type=int, default=None)
    ap.add_argument("--solver", default="lobpcg", choices=["lobpcg", "si", "sd", "tracemin"])
    ap.add_argument("--precision", default="fp64", choices=["fp64", "fp32", "bf16"])
    ap.add_argument("--max-iter", type=int, default=None)
    ap.add_argument("--expand-vectors", default="xdrop", choices=["xdrop", "random", "powered"],
                    help="vectors appended at an expansion (powered: subspace iteration only)")
    ap.add_argument("--host-io", action="store_true",
                    help="pass X0, V and lambda as host pointers (PCIe copies inside the timed solves)")
    ap.add_argument("--precond", default="none", choices=["none", "jacobi"],
                    help="LOBPCG / SD preconditioner T of W <- T R")
    ap.add_argument("--filter-degree", type=int, default=0,
                    help="subspace iteration: Chebyshev filter degree (0 = shifted power step)")
    ap.add_argument("--strategy", default="fix")
    ap.add_argument("--no-fixed", action="store_true", help="skip the fixed-block comparison")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-iterations", type=int, default=5,
                    help="oracle iterations timed after its initial Rayleigh-Ritz step")
    ap.add_argument("--cpu-seconds", type=float, default=120.0, help="cap on the oracle sample")
    ap.add_argument("--fixed-runs", type=int, default=3, help="fixed-block solves (median; at most --steps)")
    ap.add_argument("--serve-requests", type=int, default=40,
                    help="serving leg of the default run: measured Poisson requests (0 = none)")
    ap.add_argument("--serve-pilot", type=int, default=8, help="serving leg: closed-loop warm-up requests")
    ap.add_argument("--requests", type=int, default=200, help="serving: measured requests")
    ap.add_argument("--pilot", type=int, default=20, help="serving: warm-up requests (closed loop)")
    ap.add_argument("--load", type=float, default=0.7, help="serving: arrival rate / saturated rate")
    ap.add_argument("--slots", type=int, default=4, help="serving: concurrent solves")
    ap.add_argument("--serve-n", type=float, nargs=2, default=[1e4, 1e6], metavar=("MIN", "MAX"),
                    help="serving: range of the log-uniform matrix order")
    ap.add_argument("--serve-engine", choices=["batched", "slots"], default="slots",
                    help="serving: one lockstep engine for all resident solves (batched) or a stream and "
                         "worker per slot (slots)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="run one plain 1 GiB device copy first (the reference for HBM counters)")
    args = ap.parse_args()
    for key, val in WORKLOADS[args.workload].items():
        if key != "x0_seed" and getattr(args, key, None) is None:
            setattr(args, key, val)
    args.x0_seed = WORKLOADS[args.workload]["x0_seed"]
    return args


def build_matrix(args):
    import workloads as W

    if args.workload == "laplace3d":
        return W.laplacian_3d(args.grid), f"laplace3d_{args.grid}^3"
    if args.workload == "laplace2d":
        return W.laplacian_2d(args.grid), f"laplace2d_{args.grid}^2"
    if args.workload == "magnetic":
        return W.magnetic_laplacian(args.grid, MAGNETIC_PHASES), f"magnetic3d_torus_{args.grid}^3"
    if args.workload == "anderson":
        return W.anderson_3d(args.grid, 4.0, 103), f"anderson3d_{args.grid}^3_w4"
    return W.chung_lu_laplacian(args.nodes, 16.0, 2.5, 104), f"chunglu_n{args.nodes}_d16_b2.5"


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only; --gpus must be 1",
                          "n_gpus": args.gpus}), flush=True)
        sys.exit(2)

    import torch

    import workloads as W
    from paper_2409_05572_amd import api

    def log(msg):
        print(f"[bench] {msg}", file=sys.stderr, flush=True)

    if args.workload == "serving":
        print(json.dumps(serving(args, log)), flush=True)
        return

    t = time.time()
    A, wname = build_matrix(args)
    nb = args.n_ev + args.n_extra
    cplx = A.is_complex
    X0 = (W.gaussian_block_complex if cplx else W.gaussian_block)(A.n, nb, args.x0_seed)
    log(f"inputs n={A.n} nnz={A.nnz} nb={nb} built in {time.time() - t:.1f}s")

    if args.calibrate_copy:
        # one elementwise copy of 2^27 doubles (1 GiB read + 1 GiB written):
        # the known-size reference that scales FETCH_SIZE / WRITE_SIZE
        src = torch.ones(1 << 27, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        torch.mul(src, 1.0, out=dst)
        torch.cuda.synchronize()
        del src, dst
        log("copy calibration: 1 GiB read + 1 GiB written in one elementwise kernel")

    ctx = api.Context(0)
    M = api.Matrix.from_csr(ctx, A)
    # device X0 (n x nb column-major = a contiguous nb x n tensor), or the host
    # array itself with --host-io
    X0d = X0 if args.host_io else torch.from_numpy(np.ascontiguousarray(X0.T)).cuda()
    torch.cuda.synchronize()

    extra = {} if args.max_iter is None else {"max_iter": args.max_iter}
    extra.update(expand_vectors=args.expand_vectors, seed=args.x0_seed, filter_degree=args.filter_degree,
                 precond=args.precond)

    if cplx:  # complex Hermitian: FP64 LOBPCG / SI with X_drop expansions only
        extra = {} if args.max_iter is None else {"max_iter": args.max_iter}

    def run(strategy, profile=0):
        return (api.solve_z if cplx else api.solve)(
            ctx, M, X0d, args.n_ev, args.n_extra, strategy=strategy, tol=1e-8, history_cap=30000,
            profile=profile, solver=args.solver, precision=args.precision, **extra)

    for i in range(args.warmup):
        lam, V, info = run(args.strategy)
        log(f"warmup {i}: {info.time_ms / 1e3:.3f}s iters={info.iterations} conv={info.converged}")
    # timed region: K whole solves, no per-launch events
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    infos = []
    for i in range(args.steps):
        lam, V, info = run(args.strategy)
        infos.append(info)
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) / max(args.steps, 1)
    log(f"timed {args.steps} solve(s): {wall:.3f}s each, iters={infos[-1].iterations}")
    # one more solve with HIP events around every launch: the per-kernel table
    _, _, pinfo = run(args.strategy, profile=1)
    log(f"profiled solve: {pinfo.time_ms / 1e3:.3f}s iters={pinfo.iterations}")

    out = {
        "metric": METRIC,
        "value": round(wall, 4),
        "unit": "s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(wall * 1e3, 2),
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c128" if cplx else {"fp64": "f64", "fp32": "f32+f64", "bf16": "bf16+f64"}[args.precision],
        "data": "synthetic",
        "config": {
            "workload": f"{wname} {args.solver.upper()} n_ev={args.n_ev} n_extra={args.n_extra} "
                        f"strategy={args.strategy} precision={args.precision} tol=1e-8"
                        + ("" if args.expand_vectors == "xdrop" else f" expand={args.expand_vectors}")
                        + (f" filter_degree={args.filter_degree}" if args.filter_degree else "")
                        + (f" precond={args.precond}" if args.precond != "none" else "")
                        + (" host_io" if args.host_io else ""),
            "n": A.n, "nnz": A.nnz, "n_ev": args.n_ev, "block": nb,
        },
        "shrink_expand": {
            "iterations": infos[-1].iterations, "n_shrinks": infos[-1].n_shrinks,
            "n_expands": infos[-1].n_expands, "max_stop_ratio": infos[-1].max_stop_ratio,
            "converged": infos[-1].converged, "low_precision_iterations": infos[-1].lp_iterations,
            "reprojections": infos[-1].n_reprojections,
            "implicit_orthonormalizations": int(((infos[-1].history[:, 7].astype(int) & 8) != 0).sum()),
            "median_solve_s": round(float(np.median([i.time_ms for i in infos])) / 1e3, 4),
        },
    }
    lam_np = lam.cpu().numpy() if hasattr(lam, "cpu") else np.asarray(lam)
    out["parity"] = {"max_stop_ratio": infos[-1].max_stop_ratio}
    if args.workload == "magnetic":
        ex = W.magnetic_spectrum(args.grid, MAGNETIC_PHASES)[: args.n_ev]
        out["parity"]["max_eig_rel_err_vs_closed_form"] = float(np.max(np.abs(lam_np - ex) / ex))
    if args.workload in ("laplace3d", "laplace2d"):
        # Dirichlet Laplacian eigenvalues: sums of 2 - 2 cos(k pi / (m + 1))
        m = args.grid
        one = 2.0 - 2.0 * np.cos(np.arange(1, m + 1) * np.pi / (m + 1))
        if args.workload == "laplace3d":
            ex = (one[:, None, None] + one[None, :, None] + one[None, None, :]).ravel()
        else:
            ex = (one[:, None] + one[None, :]).ravel()
        ex = np.sort(ex)[: args.n_ev]
        out["parity"]["max_eig_rel_err_vs_closed_form"] = float(np.max(np.abs(lam_np - ex) / ex))
    out["lambda_head"] = [float(v) for v in lam_np[:4]]
    out["lambda_tail"] = [float(v) for v in lam_np[-2:]]

    if not args.no_fixed and args.strategy != "none":
        # the fixed block, unprofiled like the timed solves; medians of both
        runs = max(1, min(args.fixed_runs, args.steps))
        finfos = [run("none")[2] for _ in range(runs)]
        fmed = float(np.median([i.time_ms for i in finfos])) / 1e3
        smed = out["shrink_expand"]["median_solve_s"]
        out["fixed_block"] = {"time_s": round(fmed, 4), "runs": runs,
                              "iterations": [i.iterations for i in finfos],
                              "converged": all(i.converged for i in finfos),
                              "low_precision_iterations": finfos[-1].lp_iterations}
        out["speedup_vs_fixed"] = round(fmed / smed, 3)
        log(f"fixed block: median {fmed:.3f}s of {runs} iters={[i.iterations for i in finfos]}")

    tag = {"laplace3d": f"laplace3d_{args.grid}", "laplace2d": f"laplace2d_{args.grid}",
           "magnetic": f"magnetic_{args.grid}",
           "anderson": f"anderson_{args.grid}", "chunglu": f"chunglu_{args.nodes}"}[args.workload]
    out["roofline"], out["kernels"] = roofline([pinfo], f"{tag}_{args.precision}", args.precision)
    # release the solve's device memory before the serving leg and before exit
    del lam, V, X0d
    M.close()
    ctx.close()
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    out["serving"] = None
    if args.serve_requests > 0 and args.workload == "laplace3d":
        sargs = argparse.Namespace(**vars(args))
        sargs.requests, sargs.pilot = args.serve_requests, args.serve_pilot
        leg = serving(sargs, log)
        out["serving"] = dict(leg["serving"], requests=args.serve_requests, pilot=args.serve_pilot,
                              workload=leg["config"]["workload"], slots=args.slots)
        log(f"serving leg ({args.serve_engine}): {out['serving']}")
    out["cpu_baseline"] = None
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(A, X0, args, infos[-1].iterations, log)
    print(json.dumps(out), flush=True)


# Published MI355X peaks: HBM3E 8 TB/s; FP64 vector and matrix 78.6 TFLOP/s.
HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFS = 78.6
FP32_PEAK_TFS = 157.3  # FP32 vector and matrix
# kernel classes whose launches are FP64 MFMA contractions
MFMA_CLASSES = ("gram", "update")
BULK_CLASSES = ("spmm", "gram", "update", "resid", "copy")


def measured_traffic(name, workload):
    """HBM bytes per launch of kernel class `name` on `workload` from the
    committed counter summary, if it was taken on the current kernel source
    (else None)."""
    import hashlib
    import re

    path = os.path.join(ROOT, "profiles", f"{name}_{workload}_hbm_traffic.md")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        text = f.read()
    fields = dict(re.findall(r"^(source|source_sha256|bytes_per_launch): (\S+)$", text, re.M))
    if len(fields) != 3:
        return None
    with open(os.path.join(ROOT, "paper_2409_05572_amd", "csrc", fields["source"]), "rb") as f:
        digest = hashlib.sha256(f.read()).hexdigest()
    if digest != fields["source_sha256"]:
        return None
    return float(fields["bytes_per_launch"])


def roofline(infos, workload=None, precision="fp64"):
    """Per kernel class: device time summed from HIP events around every
    launch in the timed solves, algorithmic bytes and flops. The dominant
    class (largest time) is reported against its roof: FP64 MFMA for FP64
    solves; FP32 MFMA for mixed-precision ones (their classes also hold the
    FP64 refinement launches, so the fraction is approximate there)."""
    from paper_2409_05572_amd._lib import KERNEL_CLASSES

    ms = np.zeros(8)
    by = np.zeros(8)
    fl = np.zeros(8)
    calls = np.zeros(8, dtype=np.int64)
    for info in infos:
        ms += np.array(info.kern_ms)
        by += np.array(info.kern_bytes)
        fl += np.array(info.kern_flops)
        calls += np.array(info.kern_calls)
    table = {}
    for c, name in enumerate(KERNEL_CLASSES):
        if calls[c] == 0:
            continue
        sec = ms[c] / 1e3
        table[name] = {"ms_per_solve": round(ms[c] / len(infos), 2), "calls": int(calls[c]),
                       "avg_us": round(1e3 * ms[c] / calls[c], 1),
                       "GB_s": round(by[c] / sec / 1e9, 1), "TFLOP_s": round(fl[c] / sec / 1e12, 2)}
    # The roofline is taken for the dominant bulk class (products over the n
    # rows); the one-workgroup dense phases (eig, small) are latency-bound and
    # have no roof, so the largest class overall is named beside it.
    bulk = [c for c, nm in enumerate(KERNEL_CLASSES) if nm in BULK_CLASSES and calls[c] > 0]
    dom = max(bulk, key=lambda c: ms[c]) if bulk else int(np.argmax(ms))
    largest = KERNEL_CLASSES[int(np.argmax(ms))]
    sec = ms[dom] / 1e3
    name = KERNEL_CLASSES[dom]
    intensity = fl[dom] / max(by[dom], 1.0)
    peak = FP64_PEAK_TFS if precision == "fp64" else FP32_PEAK_TFS
    if name in ("spmm", "resid", "copy") or intensity < peak * 1e12 / (HBM_PEAK_GBS * 1e9):
        ach = by[dom] / sec / 1e9
        roof = {"bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(ach / HBM_PEAK_GBS, 4)}
    else:
        ach = fl[dom] / sec / 1e12
        roof = {"bound": "mfma" if name in MFMA_CLASSES else "alu", "achieved": round(ach, 2),
                "peak": peak, "unit": "TFLOP/s", "frac": round(ach / peak, 4)}
    traffic = measured_traffic(name, workload) if workload else None
    roof.update({"traffic": None if traffic is None else round(traffic), "kernel": name,
                 "largest_class": largest,
                 "launches": int(calls[dom]), "avg_launch_us": round(1e3 * ms[dom] / calls[dom], 1),
                 "algorithmic_bytes_per_launch": round(by[dom] / calls[dom]),
                 "algorithmic_flops_per_launch": round(fl[dom] / calls[dom])})
    return roof, table


def host_cpu():
    """Host facts for the CPU baseline: logical CPUs, those this process may
    run on, the CPU model, and the thread counts of the BLAS pools."""
    info = {"nproc": os.cpu_count(), "affinity": len(os.sched_getaffinity(0)),
            "omp_num_threads": os.environ.get("OMP_NUM_THREADS")}
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    info["model"] = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        from threadpoolctl import threadpool_info

        info["blas_threads"] = max((d.get("num_threads", 1) for d in threadpool_info()), default=1)
    except Exception:
        info["blas_threads"] = None
    return info


def cpu_baseline(A, X0, args, gpu_iters, log):
    """The FP64 oracle as it stands on the host cores: its initial
    Rayleigh-Ritz step, then --cpu-iterations iterations of the same solve
    timed from the start of the first (from the oracle's per-iteration
    timestamps); time-to-solution extrapolated to the GPU's iteration count."""
    import oracle as O
    import workloads as W

    host = host_cpu()
    t = time.perf_counter()
    solver = {"si": O.subspace_iteration, "sd": O.steepest_descent,
              "tracemin": O.tracemin}.get(args.solver, O.lobpcg)
    nb = args.n_ev + args.n_extra
    draw = lambda e, d: W.seeded_expansion_block(A.n, d, nb, e, args.x0_seed)  # noqa: E731
    res = solver(A.to_scipy(), X0, args.n_ev, A.anorm, tol=1e-8,
                 n_es=args.n_ev + min(5, args.n_extra - 1), se=O.SEParams(args.strategy),
                 max_iter=args.cpu_iterations,
                 time_limit_s=args.cpu_seconds, expand_vectors=args.expand_vectors, random_block=draw,
                 **({"filter_degree": args.filter_degree} if args.solver == "si" else {}),
                 **({"precond": O.jacobi_preconditioner(A.to_scipy())}
                    if args.precond == "jacobi" else {}))
    el = time.perf_counter() - t
    t_first = res.history[0]["t"]  # end of the initial Rayleigh-Ritz step
    done = len(res.history) - (1 if res.converged else 0)  # iterations that took a full step
    per_iter = (el - t_first) / max(done, 1)
    est = per_iter * gpu_iters
    threads = host["blas_threads"] or host["affinity"]
    log(f"cpu oracle: initial RR {t_first:.1f}s, {done} iteration(s) in {el - t_first:.1f}s "
        f"({per_iter:.2f}s each) on {threads} BLAS threads; host {host}")
    return {"value": round(est, 1), "unit": "s", "cores": int(threads), "kind": "oracle",
            "sample": f"{done} FP64 {args.solver.upper()} iteration(s) of the same workload after the "
                      f"initial Rayleigh-Ritz step ({t_first:.1f}s, not counted): {el - t_first:.1f}s, "
                      f"{per_iter:.2f}s/iteration; time-to-solution extrapolated x {gpu_iters} iterations "
                      f"(GPU count). Dense steps use {threads} BLAS threads; the oracle's sparse "
                      "products are single-threaded SciPy",
            "extrapolated": True, "host": host}


def serving(args, log):
    """Continuous-batching service: a stream of 2-D / 3-D Laplacians with a
    random potential (n log-uniform in [1e4, 1e6], n_ev ~ U{4..64}); a
    closed-loop pilot on the warm-up requests measures the saturated rate,
    then the measured requests arrive as a Poisson process at args.load times
    that rate. Latency = arrival to completion."""
    import torch

    import workloads as W
    from paper_2409_05572_amd import api

    total = args.pilot + args.requests
    specs = W.serving_requests(total, seed=305, n_min=args.serve_n[0], n_max=args.serve_n[1])
    t = time.time()
    ctx = api.Context(0)
    mats = []
    for sp in specs:
        A = W.potential_laplacian(sp["m"], sp["dim"], 2.0, sp["pot_seed"])
        mats.append(api.Matrix.from_csr(ctx, A))
    log(f"{total} matrices built and uploaded in {time.time() - t:.1f}s "
        f"(n {min(x['n'] for x in specs)}..{max(x['n'] for x in specs)})")
    free, _ = torch.cuda.mem_get_info()
    budget = int(free * 0.6)
    srv = api.Server(ctx, hbm_budget_bytes=budget, max_slots=args.slots, batched=args.serve_engine == "batched")

    def submit(i):
        sp = specs[i]
        nb = sp["n_ev"] + sp["n_extra"]
        t_arr = time.perf_counter()
        g = torch.Generator(device="cuda").manual_seed(1000 + i)
        x0 = torch.randn((nb, sp["n"]), generator=g, device="cuda", dtype=torch.float64)
        torch.cuda.synchronize()
        tk, lam, V = srv.submit(mats[i], x0, sp["n_ev"], sp["n_extra"], strategy="fix", tol=1e-8)
        return t_arr, time.perf_counter(), tk, x0

    def collect(subs):
        out = []
        for i, (t_arr, t_sub, tk, x0) in subs:
            info, q_ms, run_ms = srv.wait(tk)
            done = t_sub + (q_ms + run_ms) / 1e3
            out.append({"i": i, "arrival": t_arr, "done": done, "lat_ms": (done - t_arr) * 1e3,
                        "converged": info.converged, "stop": info.max_stop_ratio, "iters": info.iterations})
            del x0
        return out

    t0 = time.perf_counter()
    pilot = collect([(i, submit(i)) for i in range(args.pilot)])
    t_pilot = max(r["done"] for r in pilot) - t0
    sat = args.pilot / t_pilot
    rate = args.load * sat
    log(f"pilot: {args.pilot} requests closed-loop in {t_pilot:.2f}s -> {sat:.2f} solves/s; "
        f"arrival rate {rate:.2f}/s")
    gaps = W.poisson_gaps(args.requests, rate, seed=306)
    subs = []
    t_next = time.perf_counter()
    for k in range(args.requests):
        t_next += gaps[k]
        delay = t_next - time.perf_counter()
        if delay > 0:
            time.sleep(delay)
        subs.append((args.pilot + k, submit(args.pilot + k)))
        if (k + 1) % 50 == 0:
            log(f"submitted {k + 1}/{args.requests}")
    res = collect(subs)
    steps = srv.batch_stats() if srv.batched else None
    srv.close()
    for M in mats:
        M.close()
    ctx.close()
    lat = np.array([r["lat_ms"] for r in res])
    span = max(r["done"] for r in res) - min(r["arrival"] for r in res)
    ok = all(r["converged"] and r["stop"] <= 1e-8 for r in res + pilot)
    log(f"measured: p50 {np.percentile(lat, 50):.1f} ms, p99 {np.percentile(lat, 99):.1f} ms, "
        f"{len(res) / span:.2f} solves/s, all converged: {ok}")
    return {
        "metric": METRIC, "value": round(float(np.percentile(lat, 50)), 2), "unit": "ms (p50 latency)",
        "n_gpus": 1, "steps": args.requests, "warmup": args.pilot,
        "ms_per_step": round(span * 1e3 / len(res), 2), "higher_is_better": False, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"serving: {args.requests} Poisson requests at {args.load:g}x saturation, "
                               "2-D/3-D Laplacian + U[-2,2] potential, "
                               f"n log-uniform {args.serve_n[0]:.0e}..{args.serve_n[1]:.0e}, "
                               "n_ev U{4..64}, n_extra n_ev/2, LOBPCG fix, tol 1e-8",
                   "slots": args.slots, "engine": args.serve_engine, "hbm_budget_bytes": budget},
        "serving": {"p50_ms": round(float(np.percentile(lat, 50)), 2),
                    "p99_ms": round(float(np.percentile(lat, 99)), 2),
                    "mean_ms": round(float(lat.mean()), 2), "solves_per_s": round(len(res) / span, 3),
                    "saturated_solves_per_s": round(sat, 3), "arrival_rate_per_s": round(rate, 3),
                    "all_converged": ok, "engine": args.serve_engine,
                    "engine_steps": steps[0] if steps else None,
                    "max_stop_ratio": max(r["stop"] for r in res)},
        "roofline": None, "cpu_baseline": None,
    }


if __name__ == "__main__":
    main()
