"""Benchmark of the UV-decomposition ADMM sweep on one MI355X.

Workload (default ``lp_large``): random sparse standard-form LP, m = 1e6,
n = 2e6, 10 nonzeros per column at distinct uniform rows, N(0,1) values, rows
scaled to unit 2-norm, b = A x0 and c = A'y0 + s0 from a complementary pair
(seeded synthetic data).  A step is one ADMM iteration (column pass + row
pass, with the FP64 residual check every ``check_every`` iterations).

Printed: one JSON line with iterations/s of the FP64 solver (``value``), the
time to a 1e-4 relative KKT residual, the same for the mixed-precision form,
the roofline of the dominant kernel (algorithmic bytes / measured duration,
timed with HIP events on the solver's stream) and the CPU oracle's rate on a
bounded sample.
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

HBM_PEAK_GBS = 8000.0
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_lp_large_fp64.txt")


SWEEP_SOURCES = ("solver.hip", "common.hpp", "setup.hpp", "spmv.hpp")


def sources_digest() -> str:
    """Digest of the single-problem solver's kernel sources, comments and
    blank space left out; a traffic measurement is only used while the
    kernels are the ones it was taken on."""
    import hashlib
    import re
    h = hashlib.sha256()
    for f in (os.path.join(ROOT, "paper_2203_05027_amd", "csrc", name) for name in SWEEP_SOURCES):
        with open(f, encoding="utf-8") as fh:
            text = fh.read()
        text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)   # block comments
        text = re.sub(r"//[^\n]*", " ", text)                  # line comments
        text = " ".join(text.split())
        h.update(os.path.basename(f).encode())
        h.update(text.encode())
    return h.hexdigest()[:16]


def measured_traffic(pass_name):
    """HBM bytes per launch of a pass from the committed counter summary
    (FETCH_SIZE + WRITE_SIZE, scaled by the copy-kernel calibration), or None
    when there is none or the kernels changed since it was taken."""
    try:
        kv = {}
        with open(TRAFFIC_FILE) as f:
            for line in f:
                if ":" in line and not line.startswith("#"):
                    k, v = line.split(":", 1)
                    kv[k.strip()] = v.strip()
        if kv.get("sources") != sources_digest():
            return None
        return float(kv[f"{pass_name}_bytes_per_launch"])
    except (OSError, KeyError, ValueError):
        return None


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def describe(inst) -> str:
    """Problem class, sizes and cone of a single-instance workload."""
    m, n, nnz = inst["m"], inst["n"], inst["nnz"]
    gen = ""
    if inst.get("bounded") is False:
        gen = (f", the experiments' generator (density {nnz / (m * n):.3%}, b = A proj_K(N(0, I)), "
               f"c ~ N(0, I): not bounded, sweep rate only)")
    soc = inst.get("soc_sizes")
    if soc is not None and len(soc):
        soc = np.asarray(soc)
        return (f"SOCP m={m} n={n} nnz={nnz}, {len(soc)} second-order cones of sizes "
                f"{int(soc.min())}..{int(soc.max())} (sum {int(soc.sum())}), orthant part {inst.get('n_orth', 0)}{gen}")
    rows = ", unit-norm rows" if inst.get("unit_rows") else ""
    return f"LP m={m} n={n} nnz={nnz}{rows}, orthant cone{gen}"


def alg_bytes(m, n, nnz, precision, index_bytes=4):
    """Algorithmic bytes per launch of the row and column passes: every array
    counted once, gathered vectors at their compulsory size, indices of
    `index_bytes` (int32 in the single-problem solver, 16-bit instance-local
    in the batched one)."""
    if precision == "fp64":
        row = (index_bytes + 8) * nnz + 4 * (m + 1) + 8 * n + 8 * m + 8 * m + 16 * m + 8 * m
        col = (index_bytes + 8) * nnz + 4 * (n + 1) + 8 * m + 8 * n + 24 * n + 24 * n
    else:  # FP32 A, x, z, u, b, c, F_U; FP64 lambda, delta
        row = (index_bytes + 4) * nnz + 4 * (m + 1) + 4 * n + 4 * m + 4 * m + 16 * m + 4 * m
        col = (index_bytes + 4) * nnz + 4 * (n + 1) + 4 * m + 4 * n + 4 * n + 8 * n + 4 * n + 4 * n + 4 * n + 8 * n
    return row, col


def measure(inst, precision, steps, warmup, check_every, ttk_cap, mu, ttk=True, history_path=None):
    import torch
    from paper_2203_05027_amd.solver import Solver

    out = {}
    t0 = time.time()
    # every timed step is the whole path: each check evaluates all residuals
    # (with eps = 0 a primal-first check would skip its column half)
    s = Solver.from_instance(inst, mu=mu, precision=precision, eps=0.0,
                             check_every=check_every, full_checks=True)
    out["create_s"] = time.time() - t0
    out.update(s.launch_shape())
    s.iterate(warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s.iterate(steps)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    out["ms_per_step"] = dt * 1e3 / steps
    out["iters_per_s"] = steps / dt
    out["kkt_after"] = s.residuals()["kkt"]
    ms_col, ms_row = s.time_kernels(min(200, max(steps // 5, 20)))
    out["ms_col"], out["ms_row"] = ms_col, ms_row
    s.close()
    if not ttk:
        out.update(ttk_s=None, ttk_iters=None, ttk_status="skipped", ttk_kkt=None, ttk_pobj=None)
        return out

    # time to 1e-4 relative KKT from the zero start: the solver's default
    # checks (primal half first), then every check whole for comparison (the
    # same stopping iteration; a residual history keeps every check whole)
    for full in (False, True):
        cap_checks = ttk_cap // check_every + 1 if history_path and not full else 0
        s = Solver.from_instance(inst, mu=mu, precision=precision, eps=1e-4, check_every=check_every,
                                 max_iter=ttk_cap, history=cap_checks, full_checks=full)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        chunk = 2000
        while not s.iterate(chunk):
            pass
        torch.cuda.synchronize()
        r = s.residuals()
        dt = time.perf_counter() - t0
        if full:
            out["ttk_full_checks_s"] = dt
            out["ttk_full_checks_iters"] = r["iter"]
            s.close()
            continue
        out["ttk_s"] = dt
        out["ttk_iters"] = r["iter"]
        out["ttk_status"] = r["status"]
        out["ttk_kkt"] = r["kkt"]
        out["ttk_pobj"] = r["pobj"]
        if history_path:  # every check of the run, one JSON object a line
            recs = s.history()
            with open(history_path, "a") as f:
                for rec in recs:
                    f.write(json.dumps({"workload": inst.get("name", ""), "precision": precision, **rec}) + "\n")
            out["history_records"] = len(recs)
        s.close()
    return out


def cpu_baseline(inst, mu, seconds):
    import oracle

    orc = oracle.Oracle.from_instance(inst, mu=mu)
    orc.iterate(1)                       # first touch of the o-space arrays
    t0 = time.perf_counter()
    k = 0
    while time.perf_counter() - t0 < seconds:
        orc.iterate(1)
        k += 1
    dt = time.perf_counter() - t0
    return {"value": k / dt, "unit": "iter/s", "cores": oracle.num_threads(),
            "kind": "oracle",
            "sample": f"{k} FP64 iterations of the literal Algorithm 1 oracle on the full "
                      f"workload (timed {dt:.1f} s after one untimed iteration)"}


def small_block(mu, check_every, iters=2000):
    """The small LP (m = 500, n = 1000, 5 per column): `iters` FP64
    iterations from the zero start on the GPU (graph replays, launch-bound)
    and in the CPU oracle (serial at this size), with the KKT residual."""
    import torch
    import oracle
    from paper_2203_05027_amd import instances as I
    from paper_2203_05027_amd.solver import Solver

    inst = I.config_instance("lp_small")
    # every check whole (with eps = 0 a primal-first check skips its column half)
    with Solver.from_instance(inst, mu=mu, eps=0.0, check_every=check_every, full_checks=True) as s:
        s.iterate(iters)                      # warm-up run (graph instantiation, caches)
    with Solver.from_instance(inst, mu=mu, eps=0.0, check_every=check_every, full_checks=True) as s:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s.iterate(iters)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        r = s.residuals()
    # and to a 1e-4 KKT residual with the solver's default checks
    with Solver.from_instance(inst, mu=mu, eps=1e-4, check_every=check_every) as s:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        while not s.iterate(100_000):
            pass
        torch.cuda.synchronize()
        ttk = time.perf_counter() - t0
        rt = s.residuals()
    orc = oracle.Oracle.from_instance(inst, mu=mu)
    t1 = time.perf_counter()
    orc.iterate(iters)
    dto = time.perf_counter() - t1
    ro = orc.residuals()
    return {"workload": f"lp_small: {describe(inst)}, {iters} iterations from the zero start",
            "gpu_iters_per_s": iters / dt, "gpu_kkt": r["kkt"],
            "gpu_time_to_1e-4_s": ttk, "gpu_iters_to_1e-4": rt["iter"], "oracle_iters_per_s": iters / dto,
            "oracle_threads": 1, "oracle_kkt": ro["kkt"]}


def literal_block(inst, iters=20):
    """Ablation: Algorithm 1 as printed (o-space y and gamma stored, FP64,
    plain lane-group kernels) on the same instance: time per iteration and
    its algorithmic bytes (every array once: 56 nnz + 60 n + 36 m) against
    the reduced form's 24 nnz + 68 n + 52 m."""
    from paper_2203_05027_amd.solver import Literal

    m, n, nnz = inst["m"], inst["n"], inst["nnz"]
    with Literal.from_instance(inst) as L:
        L.iterate(2)
        ms_col, ms_row = L.time(iters)
    alg = 56 * nnz + 60 * n + 36 * m
    ms = ms_col + ms_row
    return {"ms_per_iter": ms, "ms_col": ms_col, "ms_row": ms_row, "alg_bytes_per_iter": alg,
            "alg_GBs": alg / (ms * 1e-3) / 1e9,
            "reduced_alg_bytes_per_iter": 24 * nnz + 68 * n + 52 * m}


def gather_floor(m, n, nnz, slabs_row, slabs_col, fp64=True):
    """Duration (ms) of the random-gather probe with each pass's pair count,
    gathered table and slab split: the practical floor of the row pass
    (gathers of x, n entries) and of the column pass (gathers of u, m)."""
    from paper_2203_05027_amd.solver import probe_gather
    return {"row": probe_gather(nnz, n, slabs_row, fp64), "col": probe_gather(nnz, m, slabs_col, fp64)}


def gather_sweep(nnz=20_000_000):
    """The gather probe over table sizes (FP64 and FP32 entries) and slab
    counts, 2e7 pairs each: where the gather rate falls off with the table
    part a workgroup reads (the per-XCD L2 holds 4 MiB)."""
    from paper_2203_05027_amd.solver import probe_gather
    print(f"# random-gather probe: {nnz} (int32 index, value) pairs, one random table read each; ms per launch")
    print(f"# {'table_MiB_f64':>13s} {'slabs':>5s} {'part_MiB':>8s} {'ms_f64':>8s} {'Ggather/s':>9s} {'ms_f32':>8s} {'Ggather/s':>9s}")
    for mib in (2, 4, 8, 16, 32, 128):
        for S in (1, 2, 4, 8):
            tl = mib * (1 << 20) // 8
            a = probe_gather(nnz, tl, S, True)
            b = probe_gather(nnz, tl, S, False)
            print(f"  {mib:13d} {S:5d} {mib / S:8.2f} {a:8.4f} {nnz / a / 1e6:9.1f} {b:8.4f} {nnz / b / 1e6:9.1f}",
                  flush=True)


def standard_block(inst, mu, cg_iters, cg_tol, check_every, cap_s, uv_ttk_s=None):
    """Standard two-block ADMM with a warm-started CG solve of the block
    system (the baseline the decomposition replaces) on the same instance and
    product kernels: wall time, iterations and CG steps to 1e-4 KKT."""
    import torch
    from paper_2203_05027_amd.solver import Standard

    with Standard.from_instance(inst, mu=mu, cg_iters=cg_iters, cg_tol=cg_tol, eps=1e-4,
                                check_every=check_every) as s:
        shape = s.launch_shape()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        done = False
        while not done and time.perf_counter() - t0 < cap_s:
            done = s.iterate(100)
        dt = time.perf_counter() - t0
        r = s.residuals()
    it = max(int(r["iter"]), 1)
    out = {"cg_iters": cg_iters, "cg_tol": cg_tol, "mu": mu, "launch": shape, "status": r["status"],
           "iters": int(r["iter"]), "cg_steps": int(r["cg_steps"]), "seconds": dt, "kkt": r["kkt"],
           "pobj": r["pobj"], "ms_per_iter": dt * 1e3 / it,
           "products_per_iter": 1 + 2 * r["cg_steps"] / it + 2.0 / check_every,
           "cap_s": cap_s}
    if uv_ttk_s and r["status"] == "converged":
        out["time_to_1e-4_over_uv"] = dt / uv_ttk_s   # < 1: the baseline reaches 1e-4 sooner
    return out


def batched_block(steps_sweep=100, ttk_cap=300_000, plain_per_bucket=4, count=4096, log_fn=log, cpu_threads=0,
                  cpu_iters=1000, ttk=True):
    """The batched workload: all instances in one persistent launch (mixed
    precision), sweep throughput, time to 1e-4 for the batch (the time when
    every instance has converged or reached the cap; the instances still
    unconverged at the cap are listed), and the plain single-problem solver
    on a sample stratified by size bucket (plain_per_bucket instances drawn
    from each), scaled bucket by bucket to all instances (ttk=False: the
    sweep alone, its timed launch the last of the block)."""
    from paper_2203_05027_amd import autotune
    from paper_2203_05027_amd import instances as I
    from paper_2203_05027_amd.solver import Batch, Solver

    t0 = time.time()
    insts = [I.batch_lp_instance(i) for i in range(count)]
    M = sum(i["m"] for i in insts)
    N = sum(i["n"] for i in insts)
    NNZ = sum(i["nnz"] for i in insts)
    log_fn(f"batched: {count} LPs, rows {M}, cols {N}, nnz {NNZ}, generated in {time.time() - t0:.1f} s")
    out = {"instances": count, "rows": M, "cols": N, "nnz": NNZ}

    def solve_all(b):
        t0 = time.perf_counter()
        left = count
        while left:
            left = b.iterate(2000)
            if all(b.residuals(i)["status"] != "running" for i in range(count)):
                break
        return time.perf_counter() - t0

    # the sweep is timed with every check whole (each timed step the whole
    # path); the time to 1e-4 both ways, the solver's default (primal half
    # first) reported as the result
    with Batch(insts, precision="mixed", eps=1e-4, max_iter=ttk_cap, full_checks=True) as b:
        rec = autotune.tune(b, iters=20, log=log_fn)
        out["tiles"] = {"threads": rec["threads"], "lanes": rec["lanes"], "cached": rec["cached"]}
        ms = b.time(-1, steps_sweep)
        rb, cb = alg_bytes(M, N, NNZ, "mixed", index_bytes=2)
        out["sweep_ms"] = ms / steps_sweep
        out["instance_iters_per_s"] = count * steps_sweep / (ms * 1e-3)
        out["sweep_GBs"] = (rb + cb) * steps_sweep / (ms * 1e-3) / 1e9
        if not ttk:
            return out
        out["time_to_1e4_full_checks_s"] = solve_all(b)
        its_full = [b.residuals(i)["iter"] for i in range(count)]
    with Batch(insts, precision="mixed", eps=1e-4, max_iter=ttk_cap) as b:
        autotune.tune(b, iters=20, log=log_fn)
        dt = solve_all(b)
        res = [b.residuals(i) for i in range(count)]
        out["same_stopping_iterations"] = [r["iter"] for r in res] == its_full
    its = np.array([r["iter"] for r in res])
    conv = np.array([r["status"] == "converged" for r in res])
    ms_ = np.array([i["m"] for i in insts])
    out.update(time_to_1e4_s=dt, converged=int(conv.sum()), cap=ttk_cap,
               converged_within_60k=int((conv & (its <= 60_000)).sum()),
               iters_median=float(np.median(its[conv])), iters_max_converged=int(its[conv].max()),
               unconverged=[{"instance": int(i), "m": int(ms_[i]), "iter": int(its[i]), "kkt": res[i]["kkt"],
                             "status": res[i]["status"]} for i in np.nonzero(~conv)[0]])
    # plain solver, one instance at a time, on a sample stratified by size bucket
    rng = np.random.default_rng(1)
    edges = [50, 128, 512, 2048, 5001]
    buckets, tp_all, ip_all = [], 0.0, 0
    est = 0.0
    for lo, hi in zip(edges[:-1], edges[1:]):
        members = np.nonzero((ms_ >= lo) & (ms_ < hi))[0]
        if members.size == 0:
            continue
        pick = rng.choice(members, min(plain_per_bucket, members.size), replace=False)
        tp, ip = 0.0, 0
        for i in pick:
            with Solver.from_instance(insts[i], precision="mixed", eps=1e-4, max_iter=ttk_cap) as s:
                t0 = time.perf_counter()
                while not s.iterate(5000):
                    pass
                tp += time.perf_counter() - t0
                ip += s.residuals()["iter"]
        # the bucket's batched iteration count at the plain solver's time per iteration
        b_est = tp / ip * float(its[members].sum())
        est += b_est
        tp_all += tp
        ip_all += ip
        buckets.append({"m_range": [lo, hi - 1], "instances": int(members.size), "sampled": int(pick.size),
                        "seconds": tp, "iters": ip, "us_per_iter": tp / ip * 1e6,
                        "batched_iters_same_sample": int(its[pick].sum()), "est_bucket_s": b_est})
    out["plain_sample"] = {"per_bucket": buckets, "seconds": tp_all, "iters": ip_all,
                           "est_all_instances_s": est,
                           "what": f"{plain_per_bucket} instances drawn per size bucket of m, each solved alone to "
                                   "1e-4; a bucket's estimate is its batched iteration total at the sample's "
                                   "time per iteration"}
    if cpu_threads:
        out["cpu_oracle"] = batched_cpu(insts, sample_size=16 * cpu_threads, iters=cpu_iters, threads=cpu_threads)
    return out


def host_threads() -> int:
    """Threads the CPU legs use: the oracle's OpenMP thread count."""
    import oracle
    return oracle.num_threads()


def batched_cpu(insts, sample_size, iters, threads):
    """The CPU oracle on the batched workload, one instance per host thread
    (ctypes releases the interpreter lock during the oracle's calls; its own
    parallel loops stay serial at these sizes): `iters` FP64 iterations of a
    seeded sample of the instances, as instance-iterations/s."""
    from concurrent.futures import ThreadPoolExecutor
    import oracle

    rng = np.random.default_rng(2)
    pick = rng.choice(len(insts), min(sample_size, len(insts)), replace=False)
    orcs = [oracle.Oracle.from_instance(insts[i]) for i in pick]
    t0 = time.perf_counter()
    with ThreadPoolExecutor(max_workers=threads) as ex:
        list(ex.map(lambda o: o.iterate(iters), orcs))
    dt = time.perf_counter() - t0
    return {"value": len(orcs) * iters / dt, "unit": "instance-iter/s", "threads": threads, "kind": "oracle",
            "sample": f"{len(orcs)} random instances x {iters} FP64 iterations of the literal Algorithm 1 "
                      f"oracle, one instance per thread ({dt:.1f} s)"}


def bench_family_sweep(args, B=256, iters=300):
    """The parametric family's sweep alone: one group of B held-out members
    (one A, B right-hand sides, mixed precision), `iters` iterations with
    the residual check every check_every, as member-iterations/s."""
    import torch
    from paper_2203_05027_amd import instances as I
    from paper_2203_05027_amd.solver import Family

    fam = I.ParametricFamily(m=50_000, n=100_000, k=8, p=64, seed=4)
    th = np.stack([fam.theta(2_000_000 + i) for i in range(B)])
    with Family(fam.m, fam.n, fam.row_ptr, fam.col_idx, fam.val, fam.c, B=B, eps=0.0,
                check_every=args.check_every) as F:
        F.set_rhs(fam.b_many(th))
        F.iterate(20)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        F.iterate(iters)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
    print(json.dumps({"metric": "member-iterations/s of the family sweep (one A, many b)",
                      "value": B * iters / dt, "unit": "member-iter/s", "n_gpus": 1, "higher_is_better": True,
                      "dtype": "f32 sweep / f64 duals", "data": "synthetic",
                      "ms_per_iteration": dt * 1e3 / iters,
                      "config": {"workload": f"lp_family_sweep: m={fam.m} n={fam.n} nnz={fam.row_ptr[-1]}, "
                                             f"B={B} right-hand sides, check_every={args.check_every}"}}),
          flush=True)


BF16_PEAK_TFLOPS = 2500.0  # MI355X dense BF16 matrix-core peak


def mlp_gemm_block(sizes=(8192, 4096), hidden=(512, 512), k=256, p=64, batch=256):
    """The network's matrix-core GEMM (mlp_gemm_bf16) on square problems,
    with B stored k-contiguous and n-contiguous, and the network's own train
    step (BF16 MFMA forward and backward, Adam) at the warm start's shape;
    TFLOP/s against the dense BF16 peak."""
    import torch
    from paper_2203_05027_amd import learn
    out = {"peak_tflops": BF16_PEAK_TFLOPS, "square": []}
    for n in sizes:
        A = torch.randint(-16000, 16000, (n, n), dtype=torch.int16, device="cuda")
        B = torch.randint(-16000, 16000, (n, n), dtype=torch.int16, device="cuda")
        for layout, tb in (("B k-contiguous", True), ("B n-contiguous", False)):
            learn.gemm_bf16(A, B, transB=tb)
            reps = 10
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(reps):
                learn.gemm_bf16(A, B, transB=tb)
            dt = (time.perf_counter() - t0) / reps
            tf = 2.0 * n ** 3 / dt / 1e12
            out["square"].append({"M=N=K": n, "layout": layout, "ms": dt * 1e3, "tflops": tf,
                                  "frac": tf / BF16_PEAK_TFLOPS})
        del A, B
    dims = [p, *hidden, k]
    net = learn.MLP(dims, max_batch=batch, seed=1)
    x = torch.randn(batch, p, device="cuda")
    t = torch.randn(batch, k, device="cuda")
    for _ in range(5):
        net.train_step(x, t, lr=1e-4)
    torch.cuda.synchronize()
    reps = 200
    t0 = time.perf_counter()
    for _ in range(reps):
        net.train_step(x, t, lr=1e-4)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / reps
    fwd = sum(2 * batch * a * b for a, b in zip(dims[:-1], dims[1:]))
    flops = fwd + fwd + (fwd - 2 * batch * dims[0] * dims[1])   # forward, weight gradients, input gradients
    out["train_step"] = {"dims": dims, "batch": batch, "ms": dt * 1e3, "gemm_flops": flops,
                         "tflops": flops / dt / 1e12, "frac": flops / dt / 1e12 / BF16_PEAK_TFLOPS}
    return out


def parametric_block(n_train, n_eval, epochs, train_eps=1e-3, train_cap=20_000, ttk_cap=200_000,
                     parts=("both", "primal", "dual"), projection=True, plain=8, cpu=True):
    """The learned warm start on the parametric family (A 5e4 x 1e5, theta in
    R^64): training solves, PCA, MLP training, then the held-out members
    solved to 1e-4 cold and from the learned starts through the same
    streaming family driver (B = 256 slots, a stopped member's slot takes the
    next one at once)."""
    import torch
    from paper_2203_05027_amd import instances as I
    from paper_2203_05027_amd.solver import Solver
    from paper_2203_05027_amd.warmstart import WarmStart

    t0 = time.time()
    fam = I.ParametricFamily(m=50_000, n=100_000, k=8, p=64, seed=4)
    train = np.stack([fam.theta(1_000_000 + i) for i in range(n_train)])
    held = np.stack([fam.theta(2_000_000 + i) for i in range(n_eval)])
    log(f"parametric family built in {time.time() - t0:.1f} s")
    ws = WarmStart(fam, k=256, hidden=(512, 512), B=256, log=log)
    t0 = time.time()
    Y, st = ws.solve_members(train, eps=train_eps, max_iter=train_cap)
    t_data = time.time() - t0
    Ytrue = Y[: min(512, len(train))].clone()
    t0 = time.time()
    coef = ws.fit_basis(Y)
    t_pca = time.time() - t0
    del Y
    torch.cuda.empty_cache()
    t0 = time.time()
    hist = ws.train(train, coef, epochs=epochs, batch=256, lr=1e-3)
    t_train = time.time() - t0
    fit_err = ws.model_error(ws.predict(train[: len(Ytrue)]), Ytrue)
    cmp = ws.compare_stream(held, eps=1e-4, max_iter=ttk_cap, parts=parts, projection=projection)
    # plain single-problem solver, cold, on a few held-out members
    tp, ip = 0.0, 0
    for th in held[:plain]:
        with Solver.from_instance(fam.instance(th), precision="mixed", eps=1e-4, max_iter=ttk_cap) as s:
            t1 = time.perf_counter()
            while not s.iterate(5000):
                pass
            tp += time.perf_counter() - t1
            ip += s.residuals()["iter"]
    ne = len(held)
    cpu_member = None
    if cpu:
        import oracle
        orc = oracle.Oracle.from_instance(fam.instance(held[0]), mu=1.0)
        orc.iterate(1)
        t1 = time.perf_counter()
        orc.iterate(100)
        rate = 100 / (time.perf_counter() - t1)
        cpu_member = {"value": rate, "unit": "iter/s", "cores": oracle.num_threads(), "kind": "oracle",
                      "est_cold_member_s": float(np.median(cmp["cold"]["iters"])) / rate,
                      "sample": "100 FP64 iterations of the literal Algorithm 1 oracle on the first held-out member"}

    def summary(v):
        d = cmp[v]
        return {"seconds": d["seconds"], "per_member_s": d["seconds"] / ne,
                "iters_median": float(np.median(d["iters"])), "iters_mean": float(np.mean(d["iters"])),
                "iters_total": int(d["iters"].sum()), "converged": int(d["converged"].sum()),
                "iters_p90": float(np.percentile(d["iters"], 90)), "iters_max": int(d["iters"].max()),
                "group_iters": d["group_iters"], "tail_iters": d["tail_iters"], "busy": d["busy"],
                "handed_over": d["handed_over"], "handover_iters": d["handover_iters"],
                "ms_per_group_iter": d["seconds"] * 1e3 / max(d["group_iters"], 1)}

    out = {
        "workload": f"lp_parametric: m={fam.m} n={fam.n} nnz={fam.row_ptr[-1]}, theta in R^64, "
                    f"{len(train)} training members (eps {train_eps}), {ne} held-out, "
                    "MLP 64-512-512-256, PCA k=256, B=256 streaming slots",
        "cold_over_warm_time": cmp["cold"]["seconds"] / cmp["both"]["seconds"],
        "train_data_s": t_data, "train_converged": float(st["converged"].mean()),
        "train_iters_median": float(np.median(st["iters"])), "pca_s": t_pca, "train_s": t_train,
        "train_mse_first_last": [hist[0], hist[-1]], "fit_rel_err_median": fit_err,
        "cold": summary("cold"),
        "warm": dict(summary("both"), predict_s=cmp["predict_seconds"]),
        "plain_gpu_cold": {"members": plain, "seconds": tp, "per_member_s": tp / max(plain, 1), "iters": ip},
        "cpu_baseline": cpu_member,
        "mlp_gemm": mlp_gemm_block(),
    }
    for v, key in (("primal", "warm_primal_only"), ("dual", "warm_dual_only"),
                   ("projection", "basis_projection_of_solution")):
        if v in cmp:
            out[key] = summary(v)
    return out


def bench_parametric(args):
    out = parametric_block(args.train, args.eval, args.epochs, train_eps=args.train_eps,
                           train_cap=args.train_cap, ttk_cap=args.ttk_cap, plain=args.plain, cpu=not args.no_cpu)
    line = {
        "metric": "time to 1e-4 KKT per member, learned warm start vs cold start (parametric LP family)",
        "value": out["cold_over_warm_time"],
        "unit": "x (cold time / warm time, batched family solver)",
        "n_gpus": 1, "higher_is_better": True, "dtype": "f32 sweep / f64 duals / bf16 mlp",
        "data": "synthetic", "config": {"workload": out.pop("workload")}, **out,
    }
    print(json.dumps(line), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--workload", default="lp_large")
    ap.add_argument("--scale", type=float, default=1.0)
    ap.add_argument("--check-every", type=int, default=10)
    ap.add_argument("--mu", type=float, default=1.0)
    ap.add_argument("--ttk-cap", type=int, default=200_000)
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--history", default=None,
                    help="write every residual check of the time-to-1e-4 runs to this JSONL file (a run that "
                         "keeps a history evaluates every check whole, so its time is the whole-check one)")
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--no-ttk", action="store_true",
                    help="skip the time-to-1e-4 runs (with --workload lp_batched: the sweep alone)")
    ap.add_argument("--no-batched", action="store_true", help="skip the batched-workload block")
    ap.add_argument("--no-parametric", action="store_true", help="skip the reduced learned-warm-start block")
    ap.add_argument("--param-train", type=int, default=2048, help="reduced warm-start block: training members")
    ap.add_argument("--param-eval", type=int, default=512, help="reduced warm-start block: held-out members")
    ap.add_argument("--no-standard", action="store_true", help="skip the standard ADMM + CG baseline")
    ap.add_argument("--no-small", action="store_true", help="skip the small-LP block")
    ap.add_argument("--no-literal", action="store_true", help="skip the literal Algorithm 1 ablation")
    ap.add_argument("--no-slab-search", action="store_true", help="skip the slab-count search")
    ap.add_argument("--std-cg-iters", type=int, default=2, help="baseline: CG steps per iteration at most")
    ap.add_argument("--std-cg-tol", type=float, default=0.0, help="baseline: CG stop, ||r|| <= tol (1 + ||b||)")
    ap.add_argument("--std-cap-s", type=float, default=60.0, help="baseline: wall-time cap of its solve")
    ap.add_argument("--train", type=int, default=20_000, help="parametric: training members")
    ap.add_argument("--eval", type=int, default=1000, help="parametric: held-out members")
    ap.add_argument("--epochs", type=int, default=60, help="parametric: training epochs")
    ap.add_argument("--train-eps", type=float, default=1e-3, help="parametric: tolerance of the training solves")
    ap.add_argument("--train-cap", type=int, default=20_000, help="parametric: iteration cap of training solves")
    ap.add_argument("--plain", type=int, default=8, help="members solved by the plain single-problem solver")
    ap.add_argument("--gather-sweep", action="store_true",
                    help="only print the random-gather probe over table sizes and slab counts")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="run a plain device copy of this many MiB first (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: the solver runs on one GPU; sharding a problem over several GPUs is "
              "not implemented, so --gpus must be 1", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2203_05027_amd import instances as I

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if args.calib_copy_mib:
        nel = args.calib_copy_mib * (1 << 20) // 4
        src = torch.ones(nel, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        log(f"calibration copy: 3 x {args.calib_copy_mib} MiB")
        del src, dst
    if args.gather_sweep:
        return gather_sweep()
    if args.workload == "lp_parametric":
        return bench_parametric(args)
    if args.workload == "lp_family_sweep":
        return bench_family_sweep(args)
    if args.workload == "lp_batched":
        out = batched_block(cpu_threads=0 if args.no_cpu else host_threads(), ttk=not args.no_ttk)
        print(json.dumps({"metric": "instance-iterations/s of the batched sweep (4096 LPs, one launch)",
                          "value": out["instance_iters_per_s"], "unit": "instance-iter/s", "n_gpus": 1,
                          "higher_is_better": True, "dtype": "f32 sweep / f64 duals", "data": "synthetic",
                          "config": {"workload": "lp_batched"}, "batched": out}), flush=True)
        return
    t0 = time.time()
    inst = I.config_instance(args.workload, scale=args.scale)
    m, n, nnz = inst["m"], inst["n"], inst["nnz"]
    log(f"workload {args.workload} m={m} n={n} nnz={nnz} generated in {time.time() - t0:.1f} s")

    res = {}
    if args.history:
        open(args.history, "w").close()
    ttk = not args.no_ttk and inst.get("bounded", True)   # no time to a tolerance on unbounded problems
    for prec in (["fp64"] if args.no_mixed else ["fp64", "mixed"]):
        log(f"measuring {prec}")
        res[prec] = measure(inst, prec, args.steps, args.warmup, args.check_every,
                            args.ttk_cap, args.mu, ttk=ttk, history_path=args.history)
        log(f"{prec}: {json.dumps(res[prec])}")

    main_r = res["fp64"]
    slab_search = None
    if args.workload == "lp_large" and not args.no_slab_search:
        from paper_2203_05027_amd import autotune
        rec = autotune.tune_slabs(inst, "fp64", iters=20, cache_path=None, log=log)
        slab_search = {"rule": {"slabs_row": main_r["slabs_row"], "slabs_col": main_r["slabs_col"]},
                       "search": {"slabs_row": rec["slabs_row"], "slabs_col": rec["slabs_col"]},
                       "trials": rec["trials"]}
    floor = gather_floor(m, n, nnz, main_r["slabs_row"], main_r["slabs_col"])
    log(f"gather floor (ms): {floor}")
    row_b, col_b = alg_bytes(m, n, nnz, "fp64")
    kern = {"col": (col_b, main_r["ms_col"]), "row": (row_b, main_r["ms_row"])}
    dom = max(kern, key=lambda k: kern[k][1])
    achieved = kern[dom][0] / (kern[dom][1] * 1e-3) / 1e9
    sweep_gbs = (row_b + col_b) / ((main_r["ms_col"] + main_r["ms_row"]) * 1e-3) / 1e9

    literal = None
    if not args.no_literal and not len(inst.get("soc_sizes", ())) and args.workload == "lp_large":
        log("literal Algorithm 1 ablation")
        literal = literal_block(inst)
        literal["reduced_ms_per_iter"] = main_r["ms_col"] + main_r["ms_row"]
        log(f"literal: {json.dumps(literal)}")

    small = None
    if args.workload == "lp_large" and not args.no_small:
        log("small LP block")
        small = small_block(args.mu, args.check_every)
        log(f"small: {json.dumps(small)}")

    standard = None
    if not args.no_standard and ttk:
        log("standard ADMM + CG baseline")
        standard = standard_block(inst, args.mu, args.std_cg_iters, args.std_cg_tol, args.check_every,
                                  args.std_cap_s, main_r["ttk_s"])
        log(f"standard: {json.dumps(standard)}")

    batched = None
    if not args.no_batched and args.workload == "lp_large":
        log("batched workload")
        batched = batched_block(cpu_threads=0 if args.no_cpu else host_threads())
        log(f"batched: {json.dumps(batched)}")

    parametric = None
    if not args.no_parametric and args.workload == "lp_large":
        log("learned warm start, reduced set (bench.py --workload lp_parametric runs the full one)")
        parametric = parametric_block(args.param_train, args.param_eval, args.epochs, parts=("both",),
                                      projection=False, plain=2, cpu=False)
        log(f"parametric: {json.dumps(parametric)}")

    cpu = None
    if not args.no_cpu:
        log("timing the CPU oracle")
        cpu = cpu_baseline(inst, args.mu, args.cpu_seconds)

    extra = {}
    if "mixed" in res:
        mr = res["mixed"]
        rb, cb = alg_bytes(m, n, nnz, "mixed")
        extra = {
            "iters_per_s": mr["iters_per_s"], "ms_per_step": mr["ms_per_step"],
            "time_to_1e-4_s": mr["ttk_s"], "iters_to_1e-4": mr["ttk_iters"],
            "time_to_1e-4_full_checks_s": mr.get("ttk_full_checks_s"),
            "status": mr["ttk_status"], "pobj": mr["ttk_pobj"],
            "ms_col": mr["ms_col"], "ms_row": mr["ms_row"],
            "sweep_GBs": (rb + cb) / ((mr["ms_col"] + mr["ms_row"]) * 1e-3) / 1e9,
        }
    line = {
        "metric": "iters/s of the FP64 ADMM sweep (time-to-1e-4 KKT and HBM GB/s alongside)",
        "value": main_r["iters_per_s"],
        "unit": "iter/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": main_r["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"{args.workload}: {describe(inst)}, mu={args.mu}, check_every={args.check_every}",
                   "launch": {k: main_r[k] for k in ("lanes_row", "unroll_row", "lanes_col", "slabs_row", "slabs_col",
                                                     "unroll_col")}},
        "time_to_1e-4_s": main_r["ttk_s"],
        "iters_to_1e-4": main_r["ttk_iters"],
        "time_to_1e-4_full_checks_s": main_r.get("ttk_full_checks_s"),
        "iters_to_1e-4_full_checks": main_r.get("ttk_full_checks_iters"),
        "ttk_status": main_r["ttk_status"],
        "ttk_pobj": main_r["ttk_pobj"],
        "p_star": inst.get("p_star"),
        "sweep_GBs": sweep_gbs,
        "kernels_ms": {"col": main_r["ms_col"], "row": main_r["ms_row"]},
        "roofline": {"bound": "hbm", "kernel": f"{dom} pass ({'A^T u, x-step, projection, delta' if dom == 'col' else 'A x, lambda, u'})",
                     "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": measured_traffic(dom),
                     "alg_bytes_per_launch": kern[dom][0], "ms_per_launch": kern[dom][1],
                     "gather_floor": {"ms_per_launch": floor[dom], "frac": floor[dom] / kern[dom][1],
                                      "what": "random-gather probe with the same pairs, table and slabs"}},
        "mixed": extra,
        "batched": batched,
        "learned_warm_start": parametric,
        "standard_admm_cg": standard,
        "small_lp": small,
        "literal_algorithm1": literal,
        "slab_search": slab_search,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
