"""Throughput of the SuperSCS hot path on one MI355X.

A step solves five seeded instances (0..4) of the sparse SOCP workload, each
to pr, dr, gap <= 1e-6 by Algorithm 1: n = 20000, m = 50000, A at density
1e-3 with N(0,1) values, K = zero 1000 + R+ 20000 + second-order cones of
sizes uniform in [3, 50], planted primal-dual optimum, Anderson memory 5,
FP64.  One instance's iteration count moves with the rounding order of its
reductions, so the workload is the family's, over five seeds.  The
instances are resident in HBM before timing; outputs go to device buffers.

Prints one JSON line with the metric (solves per second over the five), the
roofline of the dominant kernel (the persistent solve kernel, averaged over
its launches) and the CPU oracle timed on a bounded sample.  Further fields
measure the other workloads on the same GPU: the SOCP with the
mixed-precision linear step, by plain relaxed DRS, SCS's splitting and
Anderson by QR; the stand-alone SpMV of the CG on the SOCP's matrix and on a
1e8-nonzero matrix past the on-package cache; the LP (single and 1024 seeds
batched); the mixed PSD / exponential-cone instance solved to 1e-6; 4096
batched LASSO instances in one launch; the learned warm start (90000
training / 10000 held-out instances) against the cold-started method and
against a training-mean start; and the oracle timed on the host for every
workload.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "solves/s to 1e-6 residual; CG SpMV HBM GB/s; learned+batched vs plain"

HEADLINE_INSTANCES = 5       # seeded instances of the sparse SOCP family in the headline workload

def spmv_bytes(nnz, rows, cols, bval=8):
    """Algorithmic bytes of one CSR SpMV: values + column indices, row
    pointers, the input vector read once and the output written once."""
    return nnz * (bval + 4) + 4 * (rows + 1) + bval * (cols + rows)


def cg_op_bytes(nnz, m, n, bval=8):
    """One application of I + A^T A: SpMV by A and by A^T plus a fused pass
    over about ten n-vectors."""
    return spmv_bytes(nnz, m, n, bval) + spmv_bytes(nnz, n, m, bval) + 10 * n * bval


def op_units(info):
    """CG-operator equivalents (one product with A and one with A^T) one solve
    launch processes: every CG iteration is one (the last step of a solve is
    applied by its closing pass without products); every linear step adds one
    (the right-hand side's A^T r_y and the closing pass's y-part product A x),
    less a half for each u~ solve prestarted after a K1 step (its right-hand
    side comes by linearity); every termination check adds one (A x and
    A^T y).  The recomputation of r0 from scratch every 64th iteration is not
    counted."""
    iters = info["iters"] + 1
    linear_steps = iters + (info["iters"] - info["k0"])
    return info["cg_iters"] + linear_steps - 0.5 * info["k1"] + iters


def outer_vector_bytes(info, N, mem=5):
    """N-vector passes of the outer iterations beyond the CG operator: the
    projection / residual pass (5 N-vectors), the Anderson update (13 for
    memory 5) at every iteration, and 5 per line-search trial (one trial per
    iteration that is not K0, plus one per backtrack)."""
    iters = info["iters"] + 1
    trials = (info["iters"] - info["k0"]) + info["backtracks"]
    return 8.0 * N * ((5 + 13 * mem / 5) * iters + 5 * trials)


def cpu_baseline(prob, gpu_iters, budget_iters=60):
    """The oracle (FP64 direct factorisation) on a bounded sample: the
    factorisation plus `budget_iters` iterations of Algorithm 1, extrapolated
    to the GPU's iteration count."""
    from oracle import superscs as S
    from oracle.linsys import DirectLinSys
    try:
        import threadpoolctl
        info = threadpoolctl.threadpool_info()
        blas_threads = max([d.get("num_threads", 1) for d in info] or [1])
    except Exception:
        blas_threads = None
    cores = len(os.sched_getaffinity(0))
    t0 = time.perf_counter()
    lin = DirectLinSys(prob.A, prob.b, prob.c)
    t_factor = time.perf_counter() - t0
    t1 = time.perf_counter()
    res = S.solve(prob, S.Settings(direction="aa", mem=5, max_iters=budget_iters), lin=lin, record=False)
    t_iters = time.perf_counter() - t1
    per_iter = t_iters / max(1, res.iters)
    est = t_factor + per_iter * max(1, gpu_iters)
    return {"value": 1.0 / est, "unit": "solves/s", "cores": int(blas_threads or cores), "kind": "oracle",
            "sample": (f"dense Cholesky of I + A^T A ({t_factor:.1f} s) + {res.iters} iterations "
                       f"({per_iter:.3f} s each), extrapolated to {gpu_iters} iterations; "
                       f"{cores} host cores in affinity set")}


def _cpu_env():
    """Host cores in the affinity set, BLAS thread count and CPU model."""
    try:
        import threadpoolctl
        info = threadpoolctl.threadpool_info()
        blas = max([d.get("num_threads", 1) for d in info] or [1])
    except Exception:
        blas = None
    model = ""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return len(os.sched_getaffinity(0)), blas, model


def cpu_config1(prob, budget_s=5.0):
    """The oracle on the LP workload (RB memory 10, direct factorisation),
    whole solves repeated for about budget_s."""
    from oracle import superscs as S
    cores, blas, model = _cpu_env()
    t0 = time.perf_counter()
    k = 0
    while True:
        res = S.solve(prob, S.Settings(direction="rb", mem=10), record=False)
        k += 1
        if time.perf_counter() - t0 > budget_s:
            break
    wall = time.perf_counter() - t0
    return {"value": k / wall, "unit": "solves/s", "cores": int(blas or cores), "kind": "oracle",
            "sample": f"{k} complete solves ({res.iters} iterations, {res.status_name}); {cores} host cores, {model}"}


def cpu_config3(prob, gpu_iters, budget_iters=8):
    """The oracle on the PSD/exp instance: sparse factorisation plus
    budget_iters iterations, extrapolated to the GPU's iteration count."""
    from oracle import superscs as S
    from oracle.linsys import DirectLinSys
    cores, blas, model = _cpu_env()
    t0 = time.perf_counter()
    lin = DirectLinSys(prob.A, prob.b, prob.c)
    t_factor = time.perf_counter() - t0
    t1 = time.perf_counter()
    res = S.solve(prob, S.Settings(direction="aa", mem=5, max_iters=budget_iters), lin=lin, record=False)
    per_iter = (time.perf_counter() - t1) / max(1, res.iters)
    est = t_factor + per_iter * max(1, gpu_iters)
    return {"value": 1.0 / est, "unit": "solves/s", "cores": int(blas or cores), "kind": "oracle",
            "sample": (f"sparse LDL of I + A^T A ({t_factor:.1f} s) + {res.iters} iterations ({per_iter:.2f} s each), "
                       f"extrapolated to {gpu_iters} iterations; {cores} host cores, {model}")}


def _pool_init():
    try:
        import threadpoolctl
        threadpoolctl.threadpool_limits(1)
    except Exception:
        pass


def _oracle_solve_family_instance(arg):
    """Worker: one oracle solve (AA memory 5, eps 1e-6) of instance i of the
    batched LASSO family (kind 4) or of the shared-A family (kind 5)."""
    kind, i = arg
    from paper_1903_06477_amd import generators as G
    from oracle import superscs as S
    if kind == 4:
        p = G.config4_instance(i)
    else:
        p = G.config5_family([i], G.config5_shared_A())[0]
    t0 = time.perf_counter()
    res = S.solve(p, S.Settings(direction="aa", mem=5), record=False)
    return time.perf_counter() - t0, res.status


def cpu_family(kind, indices, total, budget_s=20.0):
    """The oracle on a seeded sample of a batched family, one solve per
    process (1 BLAS thread each, a pool of one process per core, at most 16):
    throughput = completed solves / wall time, for the family of `total`."""
    import multiprocessing as mp
    cores, _, model = _cpu_env()
    workers = max(1, min(16, cores))
    ctx = mp.get_context("spawn")
    done, t0 = 0, time.perf_counter()
    per = []
    with ctx.Pool(workers, initializer=_pool_init) as pool:
        it = iter(indices)
        while time.perf_counter() - t0 < budget_s:
            chunk = [(kind, i) for _, i in zip(range(workers), it)]
            if not chunk:
                break
            for dt, st in pool.map(_oracle_solve_family_instance, chunk):
                per.append(dt)
                done += 1
    wall = time.perf_counter() - t0
    rate = done / wall
    return {"value": rate, "unit": "solves/s", "cores": workers, "kind": "oracle",
            "sample": (f"{done} of the family's {total} instances (seeded order), one process per core with one "
                       f"BLAS thread, {wall:.1f} s wall, {np.mean(per):.2f} s per solve; the rate stands for "
                       f"the whole family ({total / rate:.0f} s extrapolated); {model}")}


def bench_settings(sscs, max_iters):
    """Anderson memory 5 (the workload's direction); relaxation 1.5, K1 factor
    0.9999 and safeguard decay 0.999 (Algorithm 1 inputs lambda, c1, q; the
    paper leaves their values open); inexact CG with tolerance 0.2 ||Ru||/||u||
    clamped to [1e-12, 1e-3]."""
    return sscs.Settings(direction="aa", mem=5, eps=1e-6, lam=1.5, c1=0.9999, q=0.999,
                         cg_tol=1e-12, cg_adapt=0.2, cg_max=500, max_iters=max_iters,
                         data_on_device=True)


def host_io_leg(sscs, prob, stream):
    """The same workload through host buffers: the instance is uploaded and
    set up on the device (transpose, Jacobi diagonal, g and delta), solved,
    and x, y, s are copied back to host memory.  Reports the rate of create +
    solve (a fresh instance per solve) and of solve alone with host outputs;
    `value` is the device-resident rate, these are context."""
    import torch
    st = bench_settings(sscs, 20000)
    st.data_on_device = False
    A = prob.A
    up = A.nnz * 12 + (A.shape[0] + 1) * 4 + 8 * (prob.m + prob.n)
    down = 8 * (prob.n + 2 * prob.m)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sv = sscs.Solver(prob, st, stream=stream.cuda_stream)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    info = sv.solve()[3]
    t2 = time.perf_counter()
    info2 = sv.solve()[3]
    t3 = time.perf_counter()
    sv.close()
    ok = info["status"] == sscs.SOLVED and info2["status"] == sscs.SOLVED
    return {"create_s": t1 - t0, "solve_s": t2 - t1, "second_solve_s": t3 - t2,
            "create_and_solve_per_s": 1.0 / (t2 - t0) if ok else 0.0,
            "solve_host_out_per_s": 1.0 / (t3 - t2) if ok else 0.0,
            "upload_bytes": up, "download_bytes": down, "iters": info2["iters"]}


def batched_leg(sscs, G, count=4096, precision="fp64", probs=None, autotune=True):
    """The batched LASSO family: `count` independent instances (n in 20..400,
    rows in n/2..2n, density 5%) in one persistent launch, AA memory 5,
    eps 1e-6, FP64 or mixed precision (FP32 operator in CG, FP64 refinement).
    Instances are uploaded before timing; outputs stay on the device.  The
    batch is timed with the mean-row-length rule's segment widths (the
    reported figure), then again with the widths sscs_batch_autotune keeps."""
    import torch
    probs = probs or [G.config4_instance(i) for i in range(count)]
    st = bench_settings(sscs, 20000)
    st.precision = precision
    bs = sscs.BatchSolver(probs, st)
    nx, ny = int(bs.ns.sum()), int(bs.ms.sum())
    out = (torch.empty(nx, dtype=torch.float64, device="cuda:0"), torch.empty(ny, dtype=torch.float64, device="cuda:0"),
           torch.empty(ny, dtype=torch.float64, device="cuda:0"))
    bs.solve(out=out)                       # warm-up launch

    def timed():
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, _, _, inf = bs.solve(out=out)
        torch.cuda.synchronize()
        return time.perf_counter() - t0, inf

    wall, infos = timed()
    tuned = None
    if autotune:
        # segment widths tuned per size class (one-off cost per batch handle)
        t0 = time.perf_counter()
        rep = bs.autotune(iters=20)
        tune_s = time.perf_counter() - t0
        wall_t, infos_t = timed()
        ok_t = np.mean([i["status"] == sscs.SOLVED for i in infos_t])
        tuned = {"solves_per_s": count / wall_t if ok_t == 1.0 else 0.0, "wall_s": wall_t,
                 "iters_mean": float(np.mean([i["iters"] for i in infos_t])), "tuning_s": tune_s,
                 "classes": rep, "how": "sscs_batch_autotune, 20 timed iterations per candidate width"}
    bs.close()
    its = np.array([i["iters"] for i in infos])
    ok = np.mean([i["status"] == sscs.SOLVED for i in infos])
    # algorithmic bytes of the launch, with the solve kernel's unit accounting
    # per instance (its CG-operator applications at its own operator's bytes,
    # plus its outer vector passes), over the launch's wall-clock time (one
    # kernel launch between two synchronisations)
    alg = float(sum(op_units(f) * cg_op_bytes(p.A.nnz, p.m, p.n) + outer_vector_bytes(f, p.n + p.m + 1)
                    for p, f in zip(probs, infos)))
    gbs = alg / wall / 1e9
    res = {"workload": f"{count} LASSO-SOCP instances, n in 20..400, m in n/2..2n, density 0.05, one launch",
           "solves_per_s": count / wall if ok == 1.0 else 0.0, "iterations_per_s": float(its.sum()) / wall,
           "wall_s": wall, "solved_frac": float(ok), "iters_mean": float(its.mean()), "iters_max": int(its.max()),
           "cg_per_iter": float(sum(i["cg_iters"] for i in infos)) / max(1, int(its.sum())),
           "segment_widths": "mean-row-length rule",
           "roofline": {"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                        "frac": gbs / HBM_PEAK_GBS, "bytes_per_launch": alg, "timed": "launch wall clock",
                        "note": "one workgroup per instance; bound by memory latency, not bandwidth"},
           "dtype": "f64" if precision == "fp64" else "f32 operator / f64"}
    if tuned is not None:
        res["autotuned_widths"] = tuned
    return res


def learned_leg(ntrain=90000, ntest=10000, epochs=60):
    """Learned warm start vs the plain cold-started method on the shared-A
    LASSO family (A 2000 x 1000 at 2%): batched solves of `ntrain` instances
    (to 1e-4, checked on the host) give the training targets, the network
    (2000-512-512-10005, BF16 matrix cores, minibatches of 1024) is trained on
    them, and `ntest` held-out instances are solved to 1e-6 cold, warm from
    the network, and warm from the training targets' mean; the warm time
    includes inference and cold fallbacks."""
    from paper_1903_06477_amd import warmstart as W
    r = W.experiment(ntrain, ntest, epochs, log=lambda s: print(s, file=sys.stderr, flush=True))
    return {"workload": f"shared-A LASSO family (A 2000 x 1000 at 2%), {ntrain} training / {ntest} test instances; "
                        f"network 2000-512-512-10005, minibatches of 1024",
            "cold_s": r["t_cold"], "warm_total_s": r["t_warm_total"], "inference_s": r["t_inference"],
            "warm_solve_s": r["t_warm_solve"], "fallback_s": r["t_fallback"], "fallbacks": r["n_fallback"],
            "final_solved": r["final_solved"],
            "speedup_vs_cold": r["speedup"], "speedup_vs_mean_start": r["speedup_vs_mean_start"],
            "iters_cold_mean": r["iters_cold_mean"], "iters_warm_mean": r["iters_warm_mean"],
            "cold_solves_per_s": ntest / r["t_cold"], "warm_solves_per_s": ntest / r["t_warm_total"],
            "train_loss": [r["loss_first"], r["loss_last"]], "test_loss": r["test_loss"],
            "training_data": {"seconds": r["t_generate"], "eps": r["train_eps"], "iters_mean": r["iters_train_mean"],
                              "solved": r["train_solved"], "worst_host_residual": r["train_worst_residual"]},
            "training_s": r["t_train"], "family_generation_s": r["t_family"],
            "warm_worst_residual": r["warm_worst_residual"],
            "ablation_training_mean_start": {"solve_s": r["t_mean_start"], "iters_mean": r["iters_mean_start"]}}


def sdp_exp_leg(sscs, G, iters=20000, prob=None):
    """The mixed PSD / exponential-cone instance (64 sparse-PCA blocks of
    order 64 and one of order 256, l1 logistic regression with 5000 samples x
    1000 features; n = 349033, m = 535113) solved to 1e-6 (iteration cap
    `iters`), FP64, AA memory 5; pr, dr, gap recomputed on the host."""
    import torch
    p = prob or G.config3_sdp_exp()
    st = bench_settings(sscs, iters)
    s = sscs.Solver(p, st)
    x = torch.empty(p.n, dtype=torch.float64, device="cuda:0")
    y = torch.empty(p.m, dtype=torch.float64, device="cuda:0")
    sv = torch.empty(p.m, dtype=torch.float64, device="cuda:0")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    info = s.solve(out=(x, y, sv))[3]
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    s.close()
    pr, dr, gap = host_kkt(p, x.cpu().numpy(), y.cpu().numpy(), sv.cpu().numpy())
    solved = info["status"] == sscs.SOLVED and max(pr, dr, gap) <= 1e-6 * 1.0001
    return {"workload": "sparse PCA (64 x order 64 + order 256, lambda 2) + l1 logistic regression "
                        "(5000 x 1000 at 1%), PSD rows 166016, 10000 exp cones, eps 1e-6",
            "n": p.n, "m": p.m, "nnz": int(p.A.nnz), "iters": info["iters"], "wall_s": wall,
            "solves_per_s": 1.0 / wall if solved else 0.0,
            "iterations_per_s": info["iters"] / wall, "cg_iters": info["cg_iters"], "res_fp": info["res_fp"],
            "status": info["status_name"], "pr_host": pr, "dr_host": dr, "gap_host": gap, "dtype": "f64"}


def host_kkt(p, x, y, s):
    """pr, dr, gap of Sec. IV-C recomputed on the host in FP64."""
    nb, nc = np.linalg.norm(p.b), np.linalg.norm(p.c)
    pr = float(np.linalg.norm(p.A @ x + s - p.b) / (1 + nb))
    dr = float(np.linalg.norm(p.A.T @ y + p.c) / (1 + nc))
    cx, by = float(p.c @ x), float(p.b @ y)
    return pr, dr, abs(cx + by) / (1 + abs(cx) + abs(by))


def config1_leg(sscs, G, reps=20, batch=1024):
    """The LP workload (300 x 100, 10% density, planted optimum, RB memory 10,
    eps 1e-6): one instance solved `reps` times on the one-workgroup kernel
    (latency: microseconds per iteration), with the CG and with the direct
    linear step, and `batch` seeded instances of the same family in one
    batched launch (throughput)."""
    import torch
    p = G.config1_lp()
    st = sscs.Settings(direction="rb", mem=10, eps=1e-6, cg_tol=1e-12, cg_adapt=0.2, cg_max=500,
                       max_iters=20000, data_on_device=True)
    dev = torch.device("cuda:0")
    x = torch.empty(p.n, dtype=torch.float64, device=dev)
    y = torch.empty(p.m, dtype=torch.float64, device=dev)
    sv = torch.empty(p.m, dtype=torch.float64, device=dev)
    with sscs.Solver(p, st) as s:
        s.solve(out=(x, y, sv))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            info = s.solve(out=(x, y, sv))[3]
        torch.cuda.synchronize()
        wall = (time.perf_counter() - t0) / reps
    pr, dr, gap = host_kkt(p, x.cpu().numpy(), y.cpu().numpy(), sv.cpu().numpy())
    # the same single solve with the direct linear step
    std = sscs.Settings(direction="rb", mem=10, eps=1e-6, max_iters=20000, data_on_device=True, linsys="direct")
    with sscs.Solver(p, std) as s:
        s.solve(out=(x, y, sv))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            info_d = s.solve(out=(x, y, sv))[3]
        torch.cuda.synchronize()
        wall_d = (time.perf_counter() - t0) / reps
    prd, drd, gapd = host_kkt(p, x.cpu().numpy(), y.cpu().numpy(), sv.cpu().numpy())
    ok_d = info_d["status"] == sscs.SOLVED and max(prd, drd, gapd) <= 1e-6 * 1.0001
    probs = [G.config1_lp(i) for i in range(batch)]
    bs = sscs.BatchSolver(probs, st)
    out = (torch.empty(batch * p.n, dtype=torch.float64, device=dev),
           torch.empty(batch * p.m, dtype=torch.float64, device=dev),
           torch.empty(batch * p.m, dtype=torch.float64, device=dev))
    bs.solve(out=out)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, _, _, infos = bs.solve(out=out)
    torch.cuda.synchronize()
    bwall = time.perf_counter() - t0
    bs.close()
    solved = [i["status"] == sscs.SOLVED for i in infos]
    its = np.array([i["iters"] for i in infos])
    return {"workload": "LP 300 x 100 at 10%, K = R+^300, planted optimum, RB memory 10, eps 1e-6",
            "solves_per_s": 1.0 / wall if info["status"] == sscs.SOLVED else 0.0, "iters": info["iters"],
            "us_per_iteration": wall * 1e6 / max(1, info["iters"]), "pr_host": pr, "dr_host": dr, "gap_host": gap,
            "direct_linear_step": {"solves_per_s": 1.0 / wall_d if ok_d else 0.0, "iters": info_d["iters"],
                                   "us_per_iteration": wall_d * 1e6 / max(1, info_d["iters"]),
                                   "pr_host": prd, "dr_host": drd, "gap_host": gapd},
            "batched": {"instances": batch, "solves_per_s": int(np.sum(solved)) / bwall,
                        "solved_frac": float(np.mean(solved)),
                        "unsolved": [{"instance": k, "status": infos[k]["status_name"], "iters": infos[k]["iters"]}
                                     for k in range(batch) if not solved[k]],
                        "iters_mean": float(its.mean()), "wall_s": bwall,
                        "note": "solves/s counts the instances solved to 1e-6 within the 20000-iteration cap"}}


def direct_leg(sscs, G):
    """The direct linear step (dense Cholesky of I + A^T A factored on the
    device, Sec. IV-A) against the CG on one held-out instance of the
    shared-A LASSO family (conic n 2001, m 4002): create time (which includes
    the factorisation), solve time of a second solve, iterations, host KKT."""
    import torch
    A = G.config5_shared_A()
    p = G.config5_family([90000], A)[0]
    out = {"workload": f"shared-A LASSO instance 90000, conic n {p.n}, m {p.m}, nnz {int(p.A.nnz)}, AA mem 5, eps 1e-6"}
    for ls in ("cg", "direct"):
        st = bench_settings(sscs, 20000)
        st.linsys = ls
        st.data_on_device = False
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s = sscs.Solver(p, st)
        torch.cuda.synchronize()
        t_create = time.perf_counter() - t0
        s.solve()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        x, y, sv, info = s.solve()
        wall = time.perf_counter() - t0
        s.close()
        pr, dr, gap = host_kkt(p, x, y, sv)
        ok = info["status"] == sscs.SOLVED and max(pr, dr, gap) <= 1e-6 * 1.0001
        out[ls] = {"create_s": t_create, "solve_s": wall, "solves_per_s": 1.0 / wall if ok else 0.0,
                   "iters": info["iters"], "cg_iters": info["cg_iters"], "us_per_iteration": wall * 1e6 / max(1, info["iters"]),
                   "pr_host": pr, "dr_host": dr, "gap_host": gap}
    return out


def spmv_large_leg(sscs, G, reps=20):
    """The CG's SpMV on the SOCP workload's matrix shape scaled to 5e6 x 2e4
    with 1e8 nonzeros (1.2 GB of values and indices, past the 256 MB
    on-package cache): A (x of 160 KB, cache-resident) and A^T (gathers from
    a 40 MB vector), FP64, event-timed on device-resident buffers."""
    p = G.spmv_scaled()
    nnz, m, n = int(p.A.nnz), p.m, p.n
    with sscs.Solver(p, sscs.Settings(cg_tol=1e-10, cg_max=50)) as s:
        ms_a = s.spmv_bench(False, reps) / reps
        ms_t = s.spmv_bench(True, reps) / reps
    ba, bt = spmv_bytes(nnz, m, n), spmv_bytes(nnz, n, m)
    del p
    return {"workload": f"{m} x {n}, {nnz} nonzeros (20 per row), N(0,1), FP64 values, int32 indices",
            "device_copy_GBs": copy_bandwidth(),
            "A_ms": ms_a, "A_GBs": ba / (ms_a * 1e-3) / 1e9, "A_frac": ba / (ms_a * 1e-3) / 1e9 / HBM_PEAK_GBS,
            "At_ms": ms_t, "At_GBs": bt / (ms_t * 1e-3) / 1e9, "At_frac": bt / (ms_t * 1e-3) / 1e9 / HBM_PEAK_GBS,
            "bytes_A": ba, "bytes_At": bt}


def source_digest():
    """SHA-256 of the HIP sources the solve kernel is built from."""
    import hashlib
    h = hashlib.sha256()
    d = os.path.join(ROOT, "paper_1903_06477_amd", "csrc")
    for f in sorted(os.listdir(d)):
        with open(os.path.join(d, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic():
    """HBM bytes per solve launch from the committed rocprofv3 counter summary,
    or None when the kernel sources changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", "traffic_k_solve_grid_socp_20000x50000.txt")
    if not os.path.exists(path):
        return None
    kv = {}
    for line in open(path):
        if ":" in line:
            k, v = line.split(":", 1)
            kv[k.strip()] = v.strip()
    if kv.get("source_sha256") != source_digest():
        return None
    try:
        return float(kv["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def performance_ratios(T):
    """Dolan-More ratios r[p, s] = t[p, s] / min_s' t[p, s'] (Sec. V-A,
    equation (performance_ratio)); T is problems x solvers with inf where a
    solver failed, and a row every solver failed stays inf."""
    T = np.asarray(T, dtype=float)
    best = T.min(axis=1, keepdims=True)
    with np.errstate(invalid="ignore", divide="ignore"):
        R = np.where(np.isfinite(T), T / best, np.inf)
    return R


def performance_profile(R, taus):
    """rho_s(tau) = |{p : r[p, s] <= tau}| / |P| for each tau (rows) and
    solver (columns)."""
    R = np.asarray(R, dtype=float)
    return np.array([(R <= tau).mean(axis=0) for tau in taus])


def shifted_geometric_mean(t, sigma):
    """sgm_sigma of Sec. V-A: failures (inf) count as 100 x the largest
    finite time of that solver, and the mean of ln max(1, sigma + t_p) over
    the problems is taken (the printed sum reads as the geometric mean's
    average; with a plain sum the value would grow with |P|)."""
    t = np.asarray(t, dtype=float)
    fin = t[np.isfinite(t)]
    fill = 100.0 * fin.max() if fin.size else np.inf
    tt = np.where(np.isfinite(t), t, fill)
    return float(np.exp(np.mean(np.log(np.maximum(1.0, sigma + tt)))) - sigma)


DM_METHODS = [("SCS (DRS on N_C + Q)", dict(direction="scs")),
              ("relaxed DRS on Q + N_C", dict(direction="zero", c0=0.0)),
              ("RB (mem:10)", dict(direction="rb", mem=10)),
              ("RB (mem:16)", dict(direction="rb", mem=16)),
              ("AA (mem:5)", dict(direction="aa", mem=5)),
              ("AA (mem:10)", dict(direction="aa", mem=10)),
              ("AA-QR (mem:5)", dict(direction="aa_qr", mem=5))]


DM_FAMILIES = {
    "lasso": ("LASSO family of Sec. V-C: n in (631, 1000, 1585, 2512), m = ceil(n/5), kappa_A in (10, 215, 4600, 1e5), "
              "mu in (0.01, 0.1, 1)", "lasso_dm_family"),
    "sdp": ("l1-regularised sparse PCA of Sec. V-B: d in (50, 120, 140, 180), lambda in (0.1, 2, 5)", "sdp_pca_dm_family"),
    "logreg": ("l1-regularised logistic regression of Sec. V-D: p in (80, 100), q in (50, 100, 120), "
               "lambda in (10, 20, 50)", "logreg_dm_family"),
}


def dm_leg(sscs, G, seeds=1, eps=1e-4, max_time=5.0, log=None, family="lasso"):
    """A benchmark family of Sec. V (`seeds` problems per parameter
    combination) solved by each method to eps on the GPU, one problem at a
    time (data on the device, setup not timed), with a time limit per solve
    standing for the paper's failure rule.  Returns per-method success, sgm
    and the Dolan-More profile.  RB memories above 16 are outside the
    engine's limit, so 10 and 16 stand in for the paper's 50 and 100."""
    import torch
    desc, fn = DM_FAMILIES[family]
    probs = getattr(G, fn)(seeds)
    T = np.full((len(probs), len(DM_METHODS)), np.inf)
    iters = np.zeros_like(T)
    for ip, p in enumerate(probs):
        x = torch.empty(p.n, dtype=torch.float64, device="cuda:0")
        y = torch.empty(p.m, dtype=torch.float64, device="cuda:0")
        s = torch.empty(p.m, dtype=torch.float64, device="cuda:0")
        for js, (_, kw) in enumerate(DM_METHODS):
            st = sscs.Settings(eps=eps, lam=1.5, c1=0.9999, q=0.999, cg_tol=1e-12, cg_adapt=0.2, cg_max=500,
                               max_iters=10**7, max_time=max_time, data_on_device=True, **kw)
            with sscs.Solver(p, st) as sv:
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                info = sv.solve(out=(x, y, s))[3]
                torch.cuda.synchronize()
                dt = time.perf_counter() - t0
            iters[ip, js] = info["iters"]
            if info["status"] == sscs.SOLVED:
                T[ip, js] = dt
        if log:
            log(f"dm {ip + 1}/{len(probs)} {p.name}: " + " ".join(f"{v:.3f}" for v in T[ip]))
    R = performance_ratios(T)
    taus = [1.0, 1.25, 1.5, 2.0, 4.0, 10.0, 100.0]
    rho = performance_profile(R, taus)
    out = {"workload": f"{desc}; {len(probs)} problems, eps {eps:g}, time limit {max_time:g} s per solve",
           "family": family, "time_unit": "ms", "sgm_shift_ms": 10.0, "methods": {}}
    for js, (name, _) in enumerate(DM_METHODS):
        out["methods"][name] = {
            "success": float(np.isfinite(T[:, js]).mean()),
            "sgm10_ms": shifted_geometric_mean(T[:, js] * 1e3, 10.0),
            "median_iters": float(np.median(iters[:, js])),
            "rho": {f"{tau:g}": float(rho[i, js]) for i, tau in enumerate(taus)}}
    return out


def copy_bandwidth(nbytes=1 << 30, reps=10):
    """Read + write bandwidth of a plain device copy (torch), event-timed: the
    attainable streaming rate to set the SpMV's fraction of peak against."""
    import torch
    a = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda:0")
    b = torch.empty_like(a)
    b.copy_(a)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del a, b
    return 2 * nbytes / (ms * 1e-3) / 1e9


def copy_calibration():
    """A plain device copy of known size, for scaling the FETCH_SIZE and
    WRITE_SIZE counters (run under rocprofv3 --pmc)."""
    import torch
    nbytes = 1 << 30
    a = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda:0")
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read": nbytes, "copy_bytes_written": nbytes}))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle leg")
    ap.add_argument("--max-iters", type=int, default=20000)
    ap.add_argument("--no-batched", action="store_true", help="skip the batched LASSO leg")
    ap.add_argument("--no-learned", action="store_true", help="skip the learned warm-start leg")
    ap.add_argument("--no-mixed", action="store_true", help="skip the mixed-precision leg")
    ap.add_argument("--no-sdp", action="store_true", help="skip the PSD / exponential-cone leg")
    ap.add_argument("--no-plain", action="store_true", help="skip the plain DRS leg")
    ap.add_argument("--no-host-io", action="store_true", help="skip the host-buffer (PCIe-inclusive) leg")
    ap.add_argument("--sdp-iters", type=int, default=20000,
                    help="iteration cap of the PSD / exponential-cone leg (the default solves it to 1e-6)")
    ap.add_argument("--no-config1", action="store_true", help="skip the LP leg")
    ap.add_argument("--no-spmv-large", action="store_true", help="skip the cache-exceeding SpMV leg")
    ap.add_argument("--no-direct", action="store_true", help="skip the direct-linear-step leg")
    ap.add_argument("--learned-train", type=int, default=90000, help="training instances of the learned leg")
    ap.add_argument("--learned-test", type=int, default=10000, help="held-out instances of the learned leg")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a 1 GiB device copy (counter calibration)")
    ap.add_argument("--dm", type=int, default=0, metavar="SEEDS",
                    help="only run the Dolan-More / sgm comparison on a benchmark family (SEEDS problems per "
                         "parameter combination)")
    ap.add_argument("--dm-family", default="lasso", choices=sorted(DM_FAMILIES),
                    help="the family of the Dolan-More comparison")
    args = ap.parse_args()
    if args.copy_calibration:
        copy_calibration()
        return
    if args.dm > 0:
        from paper_1903_06477_amd import generators as G
        from paper_1903_06477_amd import sscs
        res = dm_leg(sscs, G, seeds=args.dm, log=lambda s: print(s, file=sys.stderr, flush=True),
                     family=args.dm_family)
        print(json.dumps(res))
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported by this build "
              "(the solver has no multi-GPU path)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1903_06477_amd import generators as G
    from paper_1903_06477_amd import sscs

    assert torch.cuda.is_available(), "bench.py needs the GPU"
    dev = torch.device("cuda:0")
    # the workload: HEADLINE_INSTANCES seeded instances of the sparse SOCP
    # family, each solved once per step (one instance's trajectory, and so its
    # iteration count, moves with rounding order; their mean does not)
    probs = [G.config2_socp(i) for i in range(HEADLINE_INSTANCES)]
    prob = probs[0]
    n, m, nnz = prob.n, prob.m, prob.A.nnz
    stream = torch.cuda.current_stream()
    st = bench_settings(sscs, args.max_iters)
    solvers = [sscs.Solver(p, st, stream=stream.cuda_stream) for p in probs]
    outs = [(torch.empty(p.n, dtype=torch.float64, device=dev), torch.empty(p.m, dtype=torch.float64, device=dev),
             torch.empty(p.m, dtype=torch.float64, device=dev)) for p in probs]

    for _ in range(args.warmup):
        for sv_, o in zip(solvers, outs):
            sv_.solve(out=o)
    torch.cuda.synchronize()
    ni = len(probs)
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps * ni + 1)]
    infos = [[] for _ in range(ni)]
    t0 = time.perf_counter()
    evs[0].record(stream)
    for k in range(args.steps):
        for i, (sv_, o) in enumerate(zip(solvers, outs)):
            infos[i].append(sv_.solve(out=o)[3])
            evs[k * ni + i + 1].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    per_ms = np.array([[evs[k * ni + i].elapsed_time(evs[k * ni + i + 1]) for i in range(ni)]
                       for k in range(args.steps)])             # steps x instances, ms per solve

    solved = all(f["status"] == sscs.SOLVED for inf in infos for f in inf)
    ms_per_step = wall * 1e3 / args.steps
    value = args.steps * ni / wall if solved else 0.0
    # roofline of the solve kernel: CG-operator equivalents x bytes per operator,
    # plus the vector passes of the outer iterations, averaged over the launches
    op_b = cg_op_bytes(nnz, m, n)
    launch_bytes = [op_units(f) * op_b + outer_vector_bytes(f, n + m + 1) for inf in infos for f in inf]
    bytes_per_launch = float(np.mean(launch_bytes))
    units = float(np.mean([op_units(f) for inf in infos for f in inf]))
    vec_bytes = float(np.mean([outer_vector_bytes(f, n + m + 1) for inf in infos for f in inf]))
    kernel_ms = float(per_ms.mean())
    achieved = float(np.sum(launch_bytes)) / (per_ms.sum() * 1e-3) / 1e9
    # stand-alone SpMV of the CG (same kernel code), device-resident, event-timed
    reps = 200
    ms_a = solvers[0].spmv_bench(False, reps) / reps
    ms_t = solvers[0].spmv_bench(True, reps) / reps
    gbs_a = spmv_bytes(nnz, m, n) / (ms_a * 1e-3) / 1e9
    gbs_t = spmv_bytes(nnz, n, m) / (ms_t * 1e-3) / 1e9
    # accuracy of every instance's last timed solve, recomputed on the host in FP64
    rows = []
    for i, (p, o) in enumerate(zip(probs, outs)):
        xh, yh, sh = (t.cpu().numpy() for t in o)
        pr, dr, gap = host_kkt(p, xh, yh, sh)
        pstar = float(p.c @ p.x_star)
        f = infos[i][-1]
        rows.append({"instance": i, "iters": f["iters"], "cg_iters": f["cg_iters"], "k0": f["k0"], "k1": f["k1"],
                     "k2": f["k2"], "km": f["km"], "backtracks": f["backtracks"],
                     "solve_ms": float(per_ms[:, i].mean()), "pr_host": pr, "dr_host": dr, "gap_host": gap,
                     "obj_err_vs_planted": abs(float(p.c @ xh) - pstar) / (1 + abs(pstar))})
    iters_mean = float(np.mean([r["iters"] for r in rows]))
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"sparse SOCP n=20000 m=50000 density 1e-3, zero 1000 + R+ 20000 + SOC (sizes 3..50), "
                               f"planted optimum, AA mem 5, eps 1e-6; seeded instances 0..{ni - 1}, each solved "
                               f"once per step",
                   "settings": {"lambda": 1.5, "c1": 0.9999, "q": 0.999, "sigma": 0.01, "c0": 0.99,
                                "cg_adapt": 0.2, "cg_tol": 1e-12},
                   "n": n, "m": m, "nnz": int(nnz), "instances": ni, "parallelism": "single GPU"},
        "iterations_per_s": iters_mean * value,
        "solves": rows,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": measured_traffic(),
                     "kernel": "k_solve_grid", "kernel_ms": kernel_ms,
                     "bytes_per_launch": bytes_per_launch, "cg_op_units": units,
                     "cg_op_bytes": op_b, "outer_vector_bytes": vec_bytes},
        "spmv": {"A_us": ms_a * 1e3, "A_GBs": gbs_a, "At_us": ms_t * 1e3, "At_GBs": gbs_t,
                 "frac_of_hbm": max(gbs_a, gbs_t) / HBM_PEAK_GBS},
    }
    x, y, s = outs[0]
    for sv_ in solvers:
        sv_.close()
    log = lambda msg: print(msg, file=sys.stderr, flush=True)
    if not args.no_host_io:
        out["host_io"] = host_io_leg(sscs, prob, stream)
    if not args.no_mixed:
        # the same workload with the mixed-precision linear step
        stm = bench_settings(sscs, args.max_iters)
        stm.precision = "mixed"
        with sscs.Solver(prob, stm, stream=stream.cuda_stream) as sm:
            sm.solve(out=(x, y, s))
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            im = sm.solve(out=(x, y, s))[3]
            torch.cuda.synchronize()
            wm = time.perf_counter() - t0
        out["mixed"] = {"solves_per_s": 1.0 / wm if im["status"] == sscs.SOLVED else 0.0, "iters": im["iters"],
                        "cg_iters": im["cg_iters"], "pr": im["pr"], "dr": im["dr"], "gap": im["gap"],
                        "dtype": "f32 operator in CG / f64 residuals, refinement, scalars"}
    if not args.no_plain:
        # the same workload by plain relaxed DRS (d = 0, K0 off: u <- u - 1.5 R u)
        stp = bench_settings(sscs, 100000)
        stp.direction, stp.c0 = "zero", 0.0
        with sscs.Solver(prob, stp, stream=stream.cuda_stream) as sp_:
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            ip = sp_.solve(out=(x, y, s))[3]
            torch.cuda.synchronize()
            wp = time.perf_counter() - t0
        out["plain_drs"] = {"solves_per_s": 1.0 / wp if ip["status"] == sscs.SOLVED else 0.0, "iters": ip["iters"],
                            "cg_iters": ip["cg_iters"], "pr": ip["pr"], "dr": ip["dr"], "gap": ip["gap"],
                            "method": "relaxed Douglas-Rachford (lambda 1.5) without SuperMann steps"}
        # the same workload by SCS's splitting (DRS on N_C + Q, lambda 1.5)
        sts = bench_settings(sscs, 100000)
        sts.direction = "scs"
        with sscs.Solver(prob, sts, stream=stream.cuda_stream) as ss_:
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            isc = ss_.solve(out=(x, y, s))[3]
            torch.cuda.synchronize()
            wsc = time.perf_counter() - t0
        # the same workload with Anderson's t from an updated QR factorisation
        stq = bench_settings(sscs, args.max_iters)
        stq.direction = "aa_qr"
        with sscs.Solver(prob, stq, stream=stream.cuda_stream) as sq_:
            sq_.solve(out=(x, y, s))
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            iq = sq_.solve(out=(x, y, s))[3]
            torch.cuda.synchronize()
            wq = time.perf_counter() - t0
        out["aa_qr"] = {"solves_per_s": 1.0 / wq if iq["status"] == sscs.SOLVED else 0.0, "iters": iq["iters"],
                        "cg_iters": iq["cg_iters"], "pr": iq["pr"], "dr": iq["dr"], "gap": iq["gap"],
                        "method": "Anderson memory 5, t from an updated QR factorisation of Xi"}
        out["scs_splitting"] = {"solves_per_s": 1.0 / wsc if isc["status"] == sscs.SOLVED else 0.0,
                                "iters": isc["iters"], "cg_iters": isc["cg_iters"], "pr": isc["pr"], "dr": isc["dr"],
                                "gap": isc["gap"],
                                "method": "SCS's splitting: Douglas-Rachford on N_C + Q (lambda 1.5), no SuperMann steps"}
    del x, y, s
    if not args.no_config1:
        log("bench: LP leg")
        out["config1_lp"] = config1_leg(sscs, G)
    p3 = None
    if not args.no_sdp:
        log("bench: PSD/exp leg")
        p3 = G.config3_sdp_exp()
        out["sdp_exp"] = sdp_exp_leg(sscs, G, args.sdp_iters, prob=p3)
    if not args.no_batched:
        log("bench: batched leg")
        probs4 = [G.config4_instance(i) for i in range(4096)]
        out["batched"] = batched_leg(sscs, G, probs=probs4)
    if not args.no_direct:
        log("bench: direct linear step leg")
        out["direct_linear_step"] = direct_leg(sscs, G)
    if not args.no_spmv_large:
        log("bench: cache-exceeding SpMV leg")
        out["spmv_large"] = spmv_large_leg(sscs, G)
    if not args.no_learned:
        log("bench: learned leg")
        out["learned_vs_plain"] = learned_leg(args.learned_train, args.learned_test)
    if not args.no_cpu:
        log("bench: CPU oracle legs")
        out["cpu_baseline"] = cpu_baseline(prob, iters_mean)
        others = {}
        if not args.no_config1:
            others["config1_lp"] = cpu_config1(G.config1_lp())
        if p3 is not None:
            others["sdp_exp"] = cpu_config3(p3, out["sdp_exp"]["iters"])
        if not args.no_batched:
            others["batched_lasso_4096"] = cpu_family(4, range(4096), 4096)
        if not args.no_learned:
            from paper_1903_06477_amd.warmstart import TEST_OFFSET
            others["learned_family_test_cold"] = cpu_family(5, range(TEST_OFFSET, TEST_OFFSET + args.learned_test),
                                                            args.learned_test)
        out["cpu_baselines_other_workloads"] = others
    print(json.dumps(out))


if __name__ == "__main__":
    main()
