"""Benchmark: POD-augmented PCG over a sequence of 3-D diffusion systems on one MI355X.

One step = one whole sequence of config 2 (7-point variable-coefficient
diffusion on a 128^3 grid, n = 2,097,152, 50 implicit time steps, snapshot
memory 20, POD rank 10, relative tolerance 1e-10): for every system,
set_matrix (values only), Stage 1 + augmented PCG, push_snapshot, build_pod.
All 50 matrices are generated on the host and uploaded before timing, so the
timed region starts with every input resident in HBM; the right-hand side
b_j = x_{j-1} / dt + 1 is formed on the device inside the loop.

The same sequence is then solved with plain Jacobi PCG from the library
(warm start x_{j-1} and cold start 0, median of five sequences each) for the
wall-time comparison, and the config-1 sequence (32 x 32, 10 systems) is
timed through the one-workgroup solve and the multi-kernel loop.  The
oracle's baseline covers the whole config-2 sequence.  Last, one short pass
of each other workload (the three-stage method on the same sequence, mixed
precision on the config-3 elasticity sequence, the config-4 batch, the
config-5 adjoint gradient) goes into `other_workloads`; --no-workloads skips
them, and --workload NAME gives each its own full line.

Prints one JSON line.  The value is milliseconds per sequence (lower is
better).  The roofline object covers the loop kernel with the largest share
of time, timed with HIP events on the library stream on every 32nd iteration
of the timed steps; bytes are algorithmic (true nnz, int32 indices, each
vector counted once).
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = ("sequence solve time vs plain GPU PCG at 1e-8 rel residual; SpMV+proj HBM GB/s")
HBM_PEAK_GBPS = 8000.0
TIMING_STRIDE = 32


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_bytes(n: int, nnz: int, y: int, implicit: bool = True) -> dict:
    """Algorithmic bytes of one launch of each loop kernel (FP64 values, int32 columns).
    In the implicit form of the direction (p = pt - W nu) the direction kernel
    reads no basis column."""
    return {
        "spmv": 12 * nnz + 4 * (n + 1) + 16 * n,   # CSR values + int32 columns + row offsets, read p, write q
        "update": (4 + y) * 8 * n,             # read z, q, dinv, A W; write z (r = z / dinv is not stored)
        "dir": (5 + (0 if implicit else y)) * 8 * n,   # read z, p, x (, W); write p, x
    }


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_spmv_gamma2_config2_128_traffic.md")
LOOP_TRAFFIC_FILE = os.path.join(ROOT, "profiles", "loop_update_dir_config2_128_traffic.md")


def _summary_fields(path: str, source: str):
    """Machine-readable lines of a committed traffic summary, or None when the
    kernel source or the device header changed since the counters were taken."""
    import hashlib
    try:
        text = open(path).read()
    except OSError:
        return None
    fields = dict(line.split(": ", 1) for line in text.splitlines() if ": " in line and " " not in line.split(": ", 1)[0])
    csrc = os.path.join(ROOT, "paper_1512_05820_amd", "csrc")
    h1 = hashlib.sha256(open(os.path.join(csrc, source), "rb").read()).hexdigest()[:16]
    h2 = hashlib.sha256(open(os.path.join(csrc, "podcg_device.h"), "rb").read()).hexdigest()[:16]
    if fields.get("kernel_source_sha256_16") != h1 or fields.get("device_header_sha256_16") != h2:
        return None
    return fields


def measured_traffic(kernel: str = "spmv", launches_by_rank: dict | None = None):
    """HBM bytes per launch of a loop kernel from the committed rocprofv3
    FETCH_SIZE/WRITE_SIZE summaries (for the update and direction kernels the
    launch-weighted mean over the basis ranks of the timed launches), or None
    when the kernel sources changed since they were taken."""
    if kernel == "spmv":
        f = _summary_fields(TRAFFIC_FILE, "k_sell.hip")
        return None if f is None else float(f["traffic_bytes_per_launch"])
    f = _summary_fields(LOOP_TRAFFIC_FILE, "k_vec.hip")
    if f is None or not launches_by_rank:
        return None
    tot = cnt = 0.0
    for y, c in launches_by_rank.items():
        key = f"traffic_{kernel}_rank_{y}"
        if key not in f:
            return None
        tot += c * float(f[key])
        cnt += c
    return tot / cnt if cnt else None


def run_sequence(torch, ctx, cfg, vals_dev, method: str, warm: bool = False):
    """Solve the whole sequence on the GPU; returns per-system statistics."""
    n = cfg.n
    src = torch.full((n,), cfg.source, dtype=torch.float64, device="cuda")
    x_prev = torch.zeros(n, dtype=torch.float64, device="cuda")
    ctx.reset_snapshots()
    ctx.set_basis(None)
    out = []
    for j in range(1, cfg.steps + 1):
        ctx.set_matrix(vals_dev[j - 1])
        b = torch.add(src, x_prev, alpha=1.0 / cfg.dt) if j > 1 else src.clone()
        if method == "aug":
            x = torch.zeros(n, dtype=torch.float64, device="cuda")
            st = ctx.solve(b, x, cfg.tol)
            ctx.push_snapshot(x)
            ctx.build_pod(wait=False)
        else:
            x = x_prev.clone() if warm else torch.zeros(n, dtype=torch.float64, device="cuda")
            st = ctx.solve_plain(b, x, cfg.tol)
        if st.status not in (0, 2):
            raise RuntimeError(f"system {j}: status {st.status}")
        out.append(st.as_dict())
        x_prev = x
    return out


def cpu_baseline(cfg, systems: int) -> dict:
    """The oracle as it stands on the first `systems` systems of the sequence
    (all of them by default), on this process's OpenMP threads."""
    import oracle

    def progress(rec):
        log(f"oracle system {rec['j']}: {rec['iters']} iterations, "
            f"{rec['solve_s'] + rec['pod_s']:.2f} s")
    res = oracle.run_sequence(cfg, "aug", steps=systems, on_system=progress)
    t = sum(r["solve_s"] + r["pod_s"] for r in res)
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    sample = (f"the whole sequence ({systems} systems)" if systems == cfg.steps else
              f"first {systems} of {cfg.steps} systems, scaled by {cfg.steps}/{systems}")
    return {"value": round(1e3 * t * cfg.steps / systems, 1), "unit": "ms/sequence", "cores": threads,
            "kind": "oracle",
            "sample": f"{sample}: oracle solve + POD time, generation excluded",
            "iters": [r["iters"] for r in res]}


def cpu_oracle_child(workload: str, threads: int, systems: int) -> dict:
    """cpu_baseline in a child process with OMP_NUM_THREADS = threads (the
    OpenMP runtime reads it once, at start).  The child runs only the oracle."""
    import subprocess
    env = dict(os.environ, OMP_NUM_THREADS=str(threads))
    cmd = [sys.executable, os.path.abspath(__file__), "--cpu-only", "--workload", workload,
           "--systems", str(systems)]
    out = subprocess.run(cmd, env=env, capture_output=True, text=True, check=True)
    return json.loads(out.stdout.strip().splitlines()[-1])


def cpu_only(args):
    """Child mode of cpu_oracle_child: print the oracle's cpu_baseline record."""
    from problems import config1, config2
    cfg = config1() if args.workload == "config1" else config2(N=args.N, steps=args.systems)
    print(json.dumps(cpu_baseline(cfg, cfg.steps)), flush=True)


def median(v):
    v = sorted(v)
    k = len(v)
    return v[k // 2] if k % 2 else 0.5 * (v[k // 2 - 1] + v[k // 2])


def config1_sequences(torch, P, cfg, reps: int) -> dict:
    """Config 1: the 10-system 2-D sequence, whole-sequence wall time (median
    of reps runs after one warm-up) for augmented PCG and plain PCG (warm and
    cold start), through the one-workgroup solve and through the multi-kernel
    loop.  Every input is resident on the GPU before the timed runs."""
    vals = [torch.from_numpy(cfg.matrix_values(j)).cuda() for j in range(1, cfg.steps + 1)]
    rhs = [torch.from_numpy(cfg.rhs(j)).cuda() for j in range(1, cfg.steps + 1)]
    rowptr, colind = torch.from_numpy(cfg.rowptr).cuda(), torch.from_numpy(cfg.colind).cuda()
    res = {}
    for path, lds in (("one_workgroup", True), ("multi_kernel", False)):
        ctx = P.PodCG(cfg.n, omega=cfg.omega, rank_max=cfg.rank, maxit=20000, lds_solve=lds)
        ctx.set_matrix(vals[0], rowptr, colind)
        zeros = torch.zeros(cfg.n, dtype=torch.float64, device="cuda")
        xs = [torch.zeros(cfg.n, dtype=torch.float64, device="cuda") for _ in range(cfg.steps)]
        for method in ("aug", "plain_warm", "plain_cold"):
            def once():
                ctx.reset_snapshots()
                ctx.set_basis(None)
                sts = []
                for j in range(cfg.steps):
                    ctx.set_matrix(vals[j])
                    x = xs[j]
                    if method == "plain_warm" and j > 0:
                        x.copy_(xs[j - 1])
                    else:
                        x.copy_(zeros)
                    if method == "aug":
                        st = ctx.solve(rhs[j], x, cfg.tol)
                        ctx.push_snapshot(x)
                        ctx.build_pod(wait=False)
                    else:
                        st = ctx.solve_plain(rhs[j], x, cfg.tol)
                    if st.status not in (0, 2):
                        raise RuntimeError(f"config1 {path}/{method} system {j + 1}: status {st.status}")
                    sts.append(st.as_dict())
                return sts
            once()
            ms = []
            for _ in range(reps):
                torch.cuda.synchronize()
                t1 = time.perf_counter()
                sts = once()
                torch.cuda.synchronize()
                ms.append(1e3 * (time.perf_counter() - t1))
            iters = sum(s["iters"] for s in sts)
            solve_ms = sum(s["solve_ms"] for s in sts)
            res[f"{path}/{method}"] = {
                "ms": round(median(ms), 3), "ms_runs": [round(v, 3) for v in ms], "iters": iters,
                "path": sorted({s["path"] for s in sts}),
                "solve_gpu_ms": round(solve_ms, 3),
                "us_per_iteration_gpu": round(1e3 * solve_ms / max(iters, 1), 3),
                "max_true_relres": max(s["true_relres"] for s in sts),
                "ranks": [s["rank"] for s in sts]}
            log(f"config1 {path}/{method}: {res[f'{path}/{method}']['ms']:.3f} ms, {iters} iterations")
        ctx.close()
    return res


def bench_config1(args):
    """Config 1 on its own line: 2-D 5-point diffusion, 32 x 32, 10 systems,
    snapshot memory 5, POD rank 4, tolerance 1e-8.  The value is the median
    wall time of one augmented sequence through the one-workgroup solve; plain
    PCG and the multi-kernel loop are timed beside it, and the oracle runs the
    same sequence on one host thread and on all of them."""
    import torch
    import paper_1512_05820_amd as P
    from problems import config1

    torch.cuda.set_device(0)
    cfg = config1()
    reps = max(5, args.steps)
    runs = config1_sequences(torch, P, cfg, reps)
    v = runs["one_workgroup/aug"]["ms"]
    cpu = None
    if not args.no_cpu:
        nproc = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
        cpu = cpu_oracle_child("config1", nproc, cfg.steps)
        cpu["one_thread"] = cpu_oracle_child("config1", 1, cfg.steps)
    out = {"metric": METRIC, "value": v, "unit": "ms/sequence", "n_gpus": 1, "steps": reps,
           "warmup": 1, "ms_per_step": v, "higher_is_better": False, "scaling": "weak",
           "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": {"workload": cfg.name, "N": cfg.N, "n": cfg.n, "nnz": cfg.nnz, "systems": cfg.steps,
                      "omega": cfg.omega, "rank_max": cfg.rank, "rel_tol": cfg.tol,
                      "preconditioner": "jacobi", "value_is": "median of the augmented sequence, one-workgroup solve"},
           "speedup_vs_plain_warm": round(runs["one_workgroup/plain_warm"]["ms"] / v, 3),
           "speedup_vs_multi_kernel_aug": round(runs["multi_kernel/aug"]["ms"] / v, 3),
           "runs": runs,
           "roofline": None,
           "roofline_note": "latency-bound: the one-workgroup solve keeps the system in registers and LDS "
                            "and moves no HBM traffic per iteration; us_per_iteration_gpu is its measure",
           "cpu_baseline": cpu}
    print(json.dumps(out), flush=True)


def run_config3(args, quick=False):
    """Mixed precision at the stated size: Q1 elasticity 64^3 x 3 dof, 30 systems.

    Times whole sequences of augmented PCG (and plain PCG, warm start) in FP64
    and in mixed precision (FP32 inner solve, FP64 refinement), for the stated
    load (scaled, collinear) and for the moving-load variant, and states the
    error of system 1 against the FP64 oracle.  quick: the moving-load
    augmented sequences only, one pass each, no oracle."""
    import torch
    import paper_1512_05820_amd as P
    from problems import config3

    torch.cuda.set_device(0)
    out = {"metric": METRIC, "unit": "ms/sequence", "n_gpus": 1, "higher_is_better": False,
           "data": "synthetic", "dtype": "f32 inner / f64 refinement", "vs_baseline": None}
    results = {}
    for variant in (("moving",) if quick else ("scale", "moving")):
        cfg = config3(variant=variant, steps=args.systems if args.systems != 50 else 30)
        vals = torch.from_numpy(cfg.matrix_values(1)).cuda()
        rowptr, colind = torch.from_numpy(cfg.rowptr).cuda(), torch.from_numpy(cfg.colind).cuda()
        rhs = [torch.from_numpy(cfg.rhs(j)).cuda() for j in range(1, cfg.steps + 1)]
        for precision in ("mixed", "fp64"):
            ctx = P.PodCG(cfg.n, omega=cfg.omega, rank_max=cfg.rank, maxit=20000, precision=precision)
            ctx.set_matrix(vals, rowptr, colind)
            for method in (("aug",) if quick else ("aug", "plain")):
                for rep in range(1 if quick else 1 + args.warmup):
                    ctx.reset_snapshots()
                    ctx.set_basis(None)
                    torch.cuda.synchronize()
                    t1 = time.perf_counter()
                    sts, x_prev, x1 = [], None, None
                    for j in range(cfg.steps):
                        if method == "aug" or x_prev is None:
                            x = torch.zeros(cfg.n, dtype=torch.float64, device="cuda")
                        else:
                            x = x_prev.clone()
                        st = (ctx.solve if method == "aug" else ctx.solve_plain)(rhs[j], x, cfg.tol)
                        if method == "aug":
                            ctx.push_snapshot(x)
                            ctx.build_pod(wait=False)
                        if st.status not in (0, 2):
                            raise RuntimeError(f"{variant}/{precision}/{method} system {j + 1}: {st.status}")
                        sts.append(st.as_dict())
                        x_prev = x
                        if j == 0:
                            x1 = x.clone()
                    torch.cuda.synchronize()
                    ms = 1e3 * (time.perf_counter() - t1)
                key = f"{variant}/{precision}/{method}"
                results[key] = {"ms": round(ms, 2), "iters": sum(s["iters"] for s in sts),
                                "refine_steps": sum(s["refine_steps"] for s in sts),
                                "first_inner_relres_sys1": sts[0]["first_inner_relres"],
                                "max_true_relres": max(s["true_relres"] for s in sts)}
                if variant == "scale" and method == "aug":
                    results[key]["x1"] = x1.cpu().numpy()
                log(key, {k: v for k, v in results[key].items() if k != "x1"})
            ctx.close()
    if quick:
        cfg = config3(variant="moving", steps=args.systems if args.systems != 50 else 30)
        return {"workload": cfg.name + "_moving", "unit": "ms/sequence", "n": cfg.n, "nnz": cfg.nnz,
                "systems": cfg.steps, "omega": cfg.omega, "rank_max": cfg.rank, "rel_tol": cfg.tol,
                "value_is": "moving-load variant, mixed precision, augmented", "value": results["moving/mixed/aug"]["ms"],
                "runs": results}
    import oracle
    # error of system 1 against the FP64 oracle (solved to 1e-12)
    cfg = config3()
    A = oracle.CSR(cfg.rowptr, cfg.colind, cfg.matrix_values(1))
    t1 = time.perf_counter()
    x_ref, so = oracle.plain_pcg(A, cfg.rhs(1), np.zeros(cfg.n), 1e-12, 100000)
    cpu_s = time.perf_counter() - t1
    errs = {}
    for prec in ("mixed", "fp64"):
        x1 = results[f"scale/{prec}/aug"].pop("x1")
        errs[prec] = float(np.linalg.norm(x1 - x_ref) / np.linalg.norm(x_ref))
    for k in results:
        results[k].pop("x1", None)
    out.update({"value": results["moving/mixed/aug"]["ms"], "ms_per_step": results["moving/mixed/aug"]["ms"],
                "steps": 1, "warmup": args.warmup, "scaling": "weak",
                "config": {"workload": cfg.name, "N": cfg.N, "n": cfg.n, "nnz": cfg.nnz,
                           "systems": cfg.steps, "omega": cfg.omega, "rank_max": cfg.rank,
                           "rel_tol": cfg.tol, "value_is": "moving-load variant, mixed precision"},
                "runs": results,
                "rel_error_vs_fp64_oracle_system1": errs,
                "oracle_system1": {"iters": so.iters, "seconds": round(cpu_s, 2),
                                   "threads": int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))}})
    return out


def bench_config3(args):
    print(json.dumps(run_config3(args)), flush=True)


def run_config4(args, quick=False):
    """Batched: 64 independent 2-D diffusion sequences (sides 64..512), 20 systems
    each, advanced together (podcg_batch_set_values, podcg_batch_solve,
    podcg_batch_push_build per system) after the autotuner has picked
    work-item sizes and grid.  Compared with the same
    batch solved by plain Jacobi PCG and with the 64 sequences solved one
    context at a time (single-sequence path).  quick: the batched augmented
    sequences only (one warm-up pass, one timed)."""
    import torch
    import paper_1512_05820_amd as P
    from problems import config4

    torch.cuda.set_device(0)
    steps = args.systems if args.systems != 50 else 20
    t0 = time.perf_counter()
    cfg = config4(steps=steps)
    mem = cfg.members
    vals = [[torch.from_numpy(m.matrix_values(j)).cuda() for j in range(1, steps + 1)] for m in mem]
    rhs = [[torch.from_numpy(m.rhs(j)).cuda() for j in range(1, steps + 1)] for m in mem]
    pats = [(torch.from_numpy(m.rowptr).cuda(), torch.from_numpy(m.colind).cuda()) for m in mem]
    log(f"config4: {len(mem)} sequences, n_total {cfg.n_total}, nnz_total {cfg.nnz_total}, "
        f"inputs {time.perf_counter() - t0:.1f} s")
    ctxs = [P.PodCG(m.n, omega=m.omega, rank_max=m.rank, maxit=20000) for m in mem]
    for k, (rp, ci), v in zip(ctxs, pats, vals):
        k.set_matrix(v[0], rp, ci)
    batch = P.PodCGBatch(ctxs)
    scratch = [torch.zeros(m.n, dtype=torch.float64, device="cuda") for m in mem]
    tuned, tune_ms = batch.tune([r[0] for r in rhs], scratch, iters=32)
    log(f"tuned {tuned}: {tune_ms:.2f} ms per 32 iterations")

    def reset():
        for k in ctxs:
            k.reset_snapshots()
            k.set_basis(None)

    def batched(plain):
        # every step of the sequence batched: values, solve, snapshot push + POD build
        reset()
        sts = []
        for j in range(steps):
            batch.set_values([v[j] for v in vals])
            xs = [torch.zeros(m.n, dtype=torch.float64, device="cuda") for m in mem]
            rc, st = batch.solve([r[j] for r in rhs], xs, [m.tol for m in mem], plain=plain)
            if rc not in (0, 2):
                raise RuntimeError(f"batched system {j + 1}: {rc}")
            if not plain:
                batch.push_build(xs)
            sts.append([s.as_dict() for s in st])
        return sts

    def sequential():
        reset()
        sts = [[None] * len(mem) for _ in range(steps)]
        for i, (k, m) in enumerate(zip(ctxs, mem)):
            for j in range(steps):
                k.set_matrix(vals[i][j])
                x = torch.zeros(m.n, dtype=torch.float64, device="cuda")
                st = k.solve(rhs[i][j], x, m.tol)
                if st.status not in (0, 2):
                    raise RuntimeError(f"member {i} system {j + 1}: {st.status}")
                k.push_snapshot(x)
                k.build_pod(wait=False)
                sts[j][i] = st.as_dict()
        return sts

    def timed(fn, reps):
        ms = []
        for _ in range(reps):
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            sts = fn()
            torch.cuda.synchronize()
            ms.append(1e3 * (time.perf_counter() - t1))
        return min(ms), sts

    for _ in range(1 if quick else args.warmup):
        batched(False)
    aug_ms, aug = timed(lambda: batched(False), 1 if quick else max(1, args.steps))
    log(f"batched augmented: {aug_ms:.1f} ms")
    if quick:
        worst = max(s["true_relres"] for sts in aug for s in sts)
        batch.close()
        for k in ctxs:
            k.close()
        return {"workload": "config4_batched", "unit": "ms per batch of sequences", **cfg.describe(),
                "value": round(aug_ms, 1), "iters_aug": sum(s["iters"] for sts in aug for s in sts),
                "batched_solve_ms": round(sum(sts[0]["solve_ms"] for sts in aug), 1),
                "max_true_relres": worst, "tuned_options": tuned}
    plain_ms, plain = timed(lambda: batched(True), 1)
    log(f"batched plain: {plain_ms:.1f} ms")
    seq_ms, seq = (None, None) if args.no_plain else timed(sequential, 1)
    if seq_ms is not None:
        log(f"one context at a time, augmented: {seq_ms:.1f} ms")

    def iter_bytes(m, y):
        # CSR A, p and q of the SpMV, the vectors of the update and direction
        # kernels, and A W once (the implicit form reads no column of W)
        return 12 * m.nnz + 4 * (m.n + 1) + 16 * m.n + 8 * y * m.n + 88 * m.n

    loop_bytes = sum(iter_bytes(m, s["rank"]) * s["iters"] for sts in aug for m, s in zip(mem, sts))
    solve_ms = sum(sts[0]["solve_ms"] for sts in aug)
    worst = max(s["true_relres"] for sts in aug for s in sts)
    out = {"metric": METRIC, "value": round(aug_ms, 1), "unit": "ms per batch of sequences",
           "n_gpus": 1, "steps": max(1, args.steps), "warmup": args.warmup,
           "ms_per_step": round(aug_ms, 1), "higher_is_better": False, "scaling": "weak",
           "vs_baseline": None, "dtype": "f64", "data": "synthetic", "config": cfg.describe(),
           "batched_plain_ms": round(plain_ms, 1),
           "one_at_a_time_aug_ms": None if seq_ms is None else round(seq_ms, 1),
           "speedup_vs_batched_plain": round(plain_ms / aug_ms, 3),
           "speedup_vs_one_at_a_time": None if seq_ms is None else round(seq_ms / aug_ms, 3),
           "iters_aug": sum(s["iters"] for sts in aug for s in sts),
           "iters_plain": sum(s["iters"] for sts in plain for s in sts),
           "iters_one_at_a_time": None if seq is None else sum(s["iters"] for sts in seq for s in sts),
           "max_true_relres": worst,
           "batched_solve_ms": round(solve_ms, 1),
           "loop_GBps_lower_bound": round(loop_bytes / (solve_ms * 1e-3) / 1e9, 1),
           "tuned_options": tuned, "tune_ms_per_32_iters": round(tune_ms, 3)}
    return out


def bench_config4(args):
    print(json.dumps(run_config4(args)), flush=True)


def run_three_stage(args, quick=False, inputs=None):
    """The paper's full three-stage method (Alg. 3) on the 3-D diffusion
    sequence, next to the POD-of-solutions augmented PCG and plain PCG on the
    same systems.  Variants: ybar 200, POD to 100 vectors, stage-1 basis 5,
    rho 0 (the POD(5,95) family), Stage 3 over [W, X] with the reused
    block-diagonal factor or the computed Gram, and the iterative Stage 3 over
    all of Y (phi = 1, Stage 2 to its tolerance).  quick: the reused factor
    and the iterative Stage 3 only.  inputs: (cfg, matrices on the device,
    rowptr, colind) already resident."""
    import torch
    import paper_1512_05820_amd as P
    from problems import config2

    torch.cuda.set_device(0)
    if inputs is None:
        cfg = config2(N=args.N, steps=args.systems)
        vals_dev = [torch.from_numpy(cfg.matrix_values(j)).cuda() for j in range(1, cfg.steps + 1)]
        rowptr = torch.from_numpy(cfg.rowptr).cuda()
        colind = torch.from_numpy(cfg.colind).cuda()
    else:
        cfg, vals_dev, rowptr, colind = inputs
    ctx = P.PodCG(cfg.n, omega=cfg.omega, rank_max=cfg.rank, maxit=20000)
    ctx.set_matrix(vals_dev[0], rowptr, colind)
    runs = {}

    def timed(fn):
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        out = fn()
        torch.cuda.synchronize()
        return 1e3 * (time.perf_counter() - t1), out

    if not quick:
        ms, st = timed(lambda: run_sequence(torch, ctx, cfg, vals_dev, "aug"))
        runs["pod_of_solutions"] = {"ms": round(ms, 1), "iters": sum(s["iters"] for s in st)}
        log("pod_of_solutions", runs["pod_of_solutions"])
    if not args.no_plain and not quick:
        ms, st = timed(lambda: run_sequence(torch, ctx, cfg, vals_dev, "plain", warm=True))
        runs["plain_warm"] = {"ms": round(ms, 1), "iters": sum(s["iters"] for s in st)}
        log("plain_warm", runs["plain_warm"])

    def three_stage(gram, phi=0):
        ctx.ts_enable(ybar=200, y_trunc=100, w_max=5, w_cap=16, stage2_maxit=512 if phi else 24, rho=0.0,
                      stage2_factor=1e-4, stage3_gram=gram, phi=phi)
        src = torch.full((cfg.n,), cfg.source, dtype=torch.float64, device="cuda")
        x_prev = torch.zeros(cfg.n, dtype=torch.float64, device="cuda")
        sts = []
        for j in range(1, cfg.steps + 1):
            ctx.set_matrix(vals_dev[j - 1])
            b = torch.add(src, x_prev, alpha=1.0 / cfg.dt) if j > 1 else src.clone()
            x = torch.zeros(cfg.n, dtype=torch.float64, device="cuda")
            S = ctx.ts_solve(b, x, cfg.tol)
            if S.status != 0:
                raise RuntimeError(f"three-stage system {j}: status {S.status}")
            sts.append(S.as_dict())
            log(f"three-stage ({gram}, phi {phi}) system {j}: stage-2 steps {S.k2}, stage-3 iterations {S.k3}, "
                f"projection steps {S.k_in}, relres {S.true_relres:.2e}")
            x_prev = x
        return sts

    for gram, phi in ((("blockdiag", 0), ("iterative", 1)) if quick else
                      (("blockdiag", 0), ("exact", 0), ("iterative", 1))):
        ms, sts = timed(lambda: three_stage("blockdiag" if phi else gram, phi))
        runs[f"three_stage_{gram}"] = {
            "ms": round(ms, 1),
            "stage3_iters": sum(s["k3"] for s in sts),
            "stage2_steps": sum(s["k2"] for s in sts),
            "matvecs": sum(s["matvecs"] for s in sts),
            "truncations": sum(s["truncated"] for s in sts),
            "stage12_ms": round(sum(s["stage12_ms"] for s in sts), 1),
            "stage3_ms": round(sum(s["stage3_ms"] for s in sts), 1),
            "accumulate_truncate_ms": round(sum(s["accum_ms"] for s in sts), 1),
            "max_jacobi_sweeps": max(s["jacobi_sweeps"] for s in sts),
            "projection_steps": sum(s["k_in"] for s in sts),
            "max_true_relres": max(s["true_relres"] for s in sts),
            "k3_per_system": [s["k3"] for s in sts],
            "m_per_system": [s["m"] for s in sts],
        }
        log(f"three_stage_{gram}", {k: v for k, v in runs[f"three_stage_{gram}"].items()
                                    if not k.endswith("per_system")})
    ctx.close()
    v = runs["three_stage_blockdiag"]["ms"]
    if quick:
        return {"workload": "three_stage_" + cfg.name, "unit": "ms/sequence", "n": cfg.n, "nnz": cfg.nnz,
                "systems": cfg.steps, "rel_tol": cfg.tol, "ybar": 200, "y_trunc": 100, "w_max": 5,
                "value_is": "Stage 3 with the reused block-diagonal factor", "value": v,
                "runs": {k: {kk: vv for kk, vv in r.items() if not kk.endswith("per_system")}
                         for k, r in runs.items()}}
    out = {"metric": METRIC, "value": v, "unit": "ms/sequence", "n_gpus": 1, "steps": 1, "warmup": 0,
           "ms_per_step": v, "higher_is_better": False, "scaling": "weak", "vs_baseline": None,
           "dtype": "f64", "data": "synthetic",
           "config": {"workload": "three_stage_" + cfg.name, "N": cfg.N, "n": cfg.n, "nnz": cfg.nnz,
                      "systems": cfg.steps, "rel_tol": cfg.tol, "ybar": 200, "y_trunc": 100, "w_max": 5,
                      "rho": 0.0, "stage2_factor": 1e-4},
           "runs": runs}
    return out


def bench_three_stage(args):
    print(json.dumps(run_three_stage(args)), flush=True)


def run_config5(args, quick=False):
    """Differentiation at the stated size: 96^3 diffusion, 200 systems, outputs at
    256 dofs, gradients of J = sum_j w_j . q_j with respect to log kappa and the
    source, adjoint solves reusing the recycled bases, checkpoints every 20.
    quick: one pass, no warm-up."""
    import torch
    import paper_1512_05820_amd as P
    from paper_1512_05820_amd.adjoint import RecycledSequence, SequenceSpec
    from problems import config5
    from problems.fv_torch import FVDiffusionTorch

    torch.cuda.set_device(0)
    steps = args.systems if args.systems != 50 else 200
    cfg = config5(steps=steps)
    fvt = FVDiffusionTorch(cfg.fv, "cuda")
    outs = torch.from_numpy(cfg.outputs).cuda()
    theta = torch.from_numpy(cfg.theta).cuda()

    def assemble(j, params):
        return fvt.values(torch.exp(params[0][cfg.window(j)]), shift=1.0 / cfg.dt)

    def rhs(j, x_prev, params):
        return params[1].clone() if x_prev is None else params[1] + x_prev / cfg.dt

    spec = SequenceSpec(cfg.steps, assemble, rhs, lambda j, x: x[outs], cfg.tol, cfg.checkpoint_every,
                        adjoint_basis=args.adjoint_basis)
    mk = lambda: P.PodCG(cfg.n, omega=cfg.omega, rank_max=cfg.rank, maxit=50000)
    solver, adj = mk(), mk()
    v0 = assemble(1, (theta, None)).contiguous()
    rp, ci = torch.from_numpy(cfg.rowptr).cuda(), torch.from_numpy(cfg.colind).cuda()
    solver.set_matrix(v0, rp, ci)
    adj.set_matrix(v0, rp, ci)
    w = torch.from_numpy(np.random.Generator(np.random.PCG64(7)).standard_normal(
        (cfg.steps, cfg.outputs.size))).cuda()
    rec = {}
    for rep in range(1 if quick else 1 + args.warmup):
        th = theta.clone().requires_grad_(True)
        s = torch.full((cfg.n,), cfg.source, dtype=torch.float64, device="cuda", requires_grad=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        q = RecycledSequence.apply(solver, adj, spec, th, s)
        J = (q * w).sum()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        J.backward()
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        node = q.grad_fn
        rec = {"forward_ms": round(1e3 * (t1 - t0), 1), "backward_ms": round(1e3 * (t2 - t1), 1),
               "J": float(J.detach()), "grad_theta_norm": float(th.grad.norm()),
               "grad_s_norm": float(s.grad.norm())}
        log(f"rep {rep}: {rec}")
    fwd_it = adj_it = None
    try:
        fwd_it = sum(st["iters"] for st in node.forward_stats)
        adj_it = sum(st["iters"] for st in node.adjoint_stats)
    except AttributeError:
        pass
    total = rec["forward_ms"] + rec["backward_ms"]
    out = {"metric": METRIC, "value": round(total, 1), "unit": "ms per forward+backward sequence",
           "n_gpus": 1, "steps": 1, "warmup": args.warmup, "ms_per_step": round(total, 1),
           "higher_is_better": False, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
           "data": "synthetic", "config": {**cfg.describe(), "adjoint_basis": args.adjoint_basis},
           **rec,
           "forward_iters": fwd_it, "adjoint_iters": adj_it}
    solver.close()
    adj.close()
    if quick:
        return {"workload": "config5_adjoint", "unit": "ms per forward+backward sequence",
                **{k: out[k] for k in ("value", "config", "forward_ms", "backward_ms", "forward_iters",
                                       "adjoint_iters", "grad_theta_norm", "grad_s_norm")}}
    return out


def bench_config5(args):
    print(json.dumps(run_config5(args)), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--N", type=int, default=128, help="grid side (128 = the stated workload)")
    ap.add_argument("--systems", type=int, default=50)
    ap.add_argument("--cpu-systems", type=int, default=0, help="oracle systems for cpu_baseline (0 = all)")
    ap.add_argument("--cpu-only", action="store_true", help=argparse.SUPPRESS)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--plain-reps", type=int, default=5, help="plain-PCG sequences timed (median reported)")
    ap.add_argument("--no-config1", action="store_true", help="skip the config-1 sequences of the default run")
    ap.add_argument("--no-workloads", action="store_true",
                    help="skip the short runs of configs 3-5 and the three-stage method in the default run")
    ap.add_argument("--no-other", action="store_true",
                    help="skip the context run of the other direction form")
    ap.add_argument("--projection", default="implicit", choices=["implicit", "explicit"],
                    help="form of the direction recurrence in the augmented loop")
    ap.add_argument("--adjoint-basis", default="forward", choices=["forward", "adjoint", "none"],
                    help="config5: basis of the adjoint solves")
    ap.add_argument("--workload", default="config2",
                    choices=["config1", "config2", "config3", "config4", "config5", "three_stage"],
                    help="config2 (default, the headline), config1 (the 32 x 32 sequence, "
                         "one-workgroup solve), config3 (mixed precision), "
                         "config4 (batched sequences), config5 (adjoint gradients) or three_stage "
                         "(the full method of Alg. 3 on the config-2 sequence)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the library runs one sequence (or one batch) per GPU "
              "and has no multi-GPU path", file=sys.stderr)
        sys.exit(2)
    if args.cpu_only:
        cpu_only(args)
        return
    if args.workload == "config1":
        bench_config1(args)
        return
    if args.workload == "config3":
        bench_config3(args)
        return
    if args.workload == "config4":
        bench_config4(args)
        return
    if args.workload == "config5":
        bench_config5(args)
        return
    if args.workload == "three_stage":
        bench_three_stage(args)
        return

    import torch
    import paper_1512_05820_amd as P
    from problems import config2

    torch.cuda.set_device(0)
    t0 = time.perf_counter()
    cfg = config2(N=args.N, steps=args.systems)
    vals_dev = [torch.from_numpy(cfg.matrix_values(j)).cuda() for j in range(1, cfg.steps + 1)]
    rowptr = torch.from_numpy(cfg.rowptr).cuda()
    colind = torch.from_numpy(cfg.colind).cuda()
    log(f"generated and uploaded {cfg.steps} matrices n={cfg.n} nnz={cfg.nnz} "
        f"in {time.perf_counter() - t0:.1f}s")

    ctx = P.PodCG(cfg.n, omega=cfg.omega, rank_max=cfg.rank, maxit=20000, timing=TIMING_STRIDE,
                  projection=args.projection)
    ctx.set_matrix(vals_dev[0], rowptr, colind)
    fmt = ctx.format_info()
    log(f"matrix storage: {fmt}")

    # achievable bandwidth probe (not part of the method)
    m = 1 << 27
    a = torch.rand(m, dtype=torch.float64, device="cuda")
    bb = torch.rand(m, dtype=torch.float64, device="cuda")
    c = torch.empty_like(a)
    triad_ms = ctx.stream_triad(a, bb, c, 3.0, 20)
    triad_gbps = 3 * 8 * m / (triad_ms * 1e-3) / 1e9
    del a, bb, c
    log(f"stream triad {triad_gbps:.0f} GB/s")

    for w in range(args.warmup):
        st = run_sequence(torch, ctx, cfg, vals_dev, "aug")
        log(f"warmup {w}: iters {[s['iters'] for s in st]}")

    torch.cuda.synchronize()
    t_start = time.perf_counter()
    per_step = []
    for k in range(args.steps):
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        st = run_sequence(torch, ctx, cfg, vals_dev, "aug")
        torch.cuda.synchronize()
        per_step.append((time.perf_counter() - t1, st))
        log(f"step {k}: {1e3 * per_step[-1][0]:.1f} ms, iters {sum(s['iters'] for s in st)}")
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_start
    ms_per_step = 1e3 * elapsed / args.steps
    aug_stats = per_step[-1][1]

    # loop-kernel roofline from the event-timed iterations of all timed steps
    tot = {"spmv": [0.0, 0.0], "update": [0.0, 0.0], "dir": [0.0, 0.0]}
    for _, sts in per_step:
        for s in sts:
            kb = kernel_bytes(cfg.n, cfg.nnz, s["rank"], implicit=args.projection == "implicit")
            for key, ms_key in (("spmv", "spmv_ms"), ("update", "update_ms"), ("dir", "dir_ms")):
                tot[key][0] += s["timed_iters"] * kb[key]
                tot[key][1] += s[ms_key]
    launches = sum(s["timed_iters"] for _, sts in per_step for s in sts)
    by_rank = {}
    for _, sts in per_step:
        for s in sts:
            by_rank[s["rank"]] = by_rank.get(s["rank"], 0) + s["timed_iters"]
    dom = max(tot, key=lambda k: tot[k][1])
    gbps = {k: (v[0] / (v[1] * 1e-3) / 1e9 if v[1] > 0 else 0.0) for k, v in tot.items()}
    loop_bytes = sum(v[0] for v in tot.values())
    loop_ms = sum(v[1] for v in tot.values())
    loop_gbps = loop_bytes / (loop_ms * 1e-3) / 1e9 if loop_ms > 0 else 0.0

    plain = {}
    if not args.no_plain:
        for warm in (True, False):
            ms = []
            for _ in range(args.plain_reps):
                torch.cuda.synchronize()
                t1 = time.perf_counter()
                sts = run_sequence(torch, ctx, cfg, vals_dev, "plain", warm=warm)
                torch.cuda.synchronize()
                ms.append(1e3 * (time.perf_counter() - t1))
            key = "warm" if warm else "cold"
            plain[key] = {"ms": round(median(ms), 3), "ms_runs": [round(v, 1) for v in ms],
                          "iters": sum(s["iters"] for s in sts)}
            log(f"plain {key}: median {plain[key]['ms']:.1f} ms of {ms}, iters {plain[key]['iters']}")

    # the other form of the direction recurrence, once, for context
    other_rec = None
    if not args.no_other:
        other = "explicit" if args.projection == "implicit" else "implicit"
        ctx_o = P.PodCG(cfg.n, omega=cfg.omega, rank_max=cfg.rank, maxit=20000, projection=other)
        ctx_o.set_matrix(vals_dev[0], rowptr, colind)
        run_sequence(torch, ctx_o, cfg, vals_dev, "aug")
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        sts = run_sequence(torch, ctx_o, cfg, vals_dev, "aug")
        torch.cuda.synchronize()
        other_rec = {"projection": other, "ms": round(1e3 * (time.perf_counter() - t1), 3),
                     "iters": sum(s["iters"] for s in sts)}
        log(f"aug {other}: {other_rec['ms']:.1f} ms, iters {other_rec['iters']}")
        del ctx_o

    cpu = None
    if not args.no_cpu:
        t1 = time.perf_counter()
        cpu = cpu_baseline(cfg, min(args.cpu_systems, cfg.steps) if args.cpu_systems > 0 else cfg.steps)
        log(f"cpu baseline {cpu['value']:.0f} ms/sequence ({time.perf_counter() - t1:.1f}s)")

    # config 1 (32 x 32, 10 systems) beside the headline: latency-bound, so
    # whole-sequence wall time, one-workgroup solve against the multi-kernel loop
    c1 = None
    if not args.no_config1:
        from problems import config1
        r1 = config1_sequences(torch, P, config1(), 5)
        c1 = {"unit": "ms/sequence (median of 5)",
              **{k: {"ms": v["ms"], "iters": v["iters"], "us_per_iteration_gpu": v["us_per_iteration_gpu"]}
                 for k, v in r1.items()}}

    # the other workloads, one short pass each, so that the default line
    # records them too (their own lines: --workload config3 / config4 /
    # config5 / three_stage)
    others = None
    if not args.no_workloads and cfg.N == 128 and cfg.steps == 50:
        ctx.close()
        others = {}
        for name, fn in (("three_stage", lambda: run_three_stage(args, quick=True,
                                                                 inputs=(cfg, vals_dev, rowptr, colind))),
                         ("config3", lambda: run_config3(args, quick=True)),
                         ("config4", lambda: run_config4(args, quick=True)),
                         ("config5", lambda: run_config5(args, quick=True))):
            t1 = time.perf_counter()
            others[name] = fn()
            others[name]["wall_s"] = round(time.perf_counter() - t1, 1)
            log(f"{name}: {others[name]['value']} {others[name]['unit']} ({others[name]['wall_s']} s)")
            torch.cuda.empty_cache()

    aug_iters = sum(s["iters"] for s in aug_stats)
    rec = {
        "metric": METRIC,
        "value": round(ms_per_step, 3),
        "unit": "ms/sequence",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": cfg.name, "N": cfg.N, "n": cfg.n, "nnz": cfg.nnz,
                   "systems": cfg.steps, "omega": cfg.omega, "rank_max": cfg.rank,
                   "rel_tol": cfg.tol, "dt": cfg.dt, "preconditioner": "jacobi",
                   "projection": args.projection},
        "aug_iters_total": aug_iters,
        "aug_iters_per_system": [s["iters"] for s in aug_stats],
        "aug_rank_per_system": [s["rank"] for s in aug_stats],
        "max_true_relres": max(s["true_relres"] for s in aug_stats),
        "plain_gpu": plain,
        "aug_other_form": other_rec,
        "speedup_vs_plain_warm": (round(plain["warm"]["ms"] / ms_per_step, 3) if plain else None),
        "iters_saved_vs_plain_warm": (1 - aug_iters / plain["warm"]["iters"]) if plain else None,
        "loop_kernels_GBps": {k: round(v, 1) for k, v in gbps.items()},
        "matrix_storage": fmt,
        "spmv_proj_GBps": round(loop_gbps, 1),
        "stream_triad_GBps": round(triad_gbps, 1),
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": round(gbps[dom], 1),
                     "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                     "frac": round(gbps[dom] / HBM_PEAK_GBPS, 4),
                     "traffic": (measured_traffic(dom, by_rank) if cfg.N == 128 else None),
                     "traffic_unit": "bytes per launch (rocprofv3 FETCH_SIZE x2 + WRITE_SIZE x1, copy-calibrated; "
                                     "update and direction: mean over the timed launches' basis ranks)",
                     "algorithmic_bytes": round(tot[dom][0] / max(launches, 1)),
                     "format_bytes": (8 * fmt["slots"] + fmt["column_bytes"] + 16 * cfg.n + 9 * ((cfg.n + 63) // 64)
                                      if dom == "spmv" else None),
                     "avg_launch_us": round(1e3 * tot[dom][1] / max(launches, 1), 2),
                     "timed_launches": launches},
        "cpu_baseline": cpu,
        "config1_sequence": c1,
        "other_workloads": others,
    }
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
