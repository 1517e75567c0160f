#!/usr/bin/env python3
"""Benchmark: p-BiCGSafe (Algorithm 4) on the 128^3 convection-diffusion system.

One step = one full solve of A x = b to ||r_i|| <= 1e-8 ||r_0|| from x0 = 0
(set-up included), FP64, with the matrix and b already resident on the GPU.

Prints ONE JSON line on stdout:
  value      achieved HBM GB/s of the iteration = algorithmic bytes per
             iteration x iterations / solve time (set-up time counted, its
             bytes not)
  roofline   the dominant kernel: algorithmic bytes per launch / average
             launch time measured with HIP events on its own stream during
             the timed steps, against the 8 TB/s HBM3E peak; `traffic` is the
             counter-measured HBM bytes per launch from the committed
             rocprofv3 summary when it still matches the kernel sources
  cpu_baseline  the FP64 CPU oracle on a bounded sample of the same solve
             (set-up + a fixed number of iterations), on all host threads and
             on one

Everything else (progress, per-variant numbers) goes to stderr or to extra
JSON fields.  Only one GPU is used: --gpus N with N > 1 exits with a message.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "HBM GB/s per pipelined iteration; time-to-1e-8 residual vs plain FP64"
PEAK_GBPS = 8000.0
CLASSES = ["spmv", "dots", "update", "spmv_fused", "other"]
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_cd3d_128.json")


def kernel_name(cls, layout, schedule, streaming=0):
    """The kernel a class means for this layout, schedule and streaming choice (as rocprofv3
    names it, shortened)."""
    k = "k_sell" if layout == "sell" else "k_spmv"
    nt = "true" if streaming else "false"
    if schedule == 1:
        return {"spmv": f"{k}<EpiStore> (A s_i)",
                "update": f"k_passA_pbicgsafe<true, {nt}> (pass A + 5 partial inner products)",
                "spmv_fused": f"{k}<EpiPBiCGSafeBDots<{nt}>> (A w_i + l, g, s + 4 partial inner products)"}[cls]
    if schedule in (2, 3):
        spmv = (f"{k}<EpiStoreFold> (A s_i + the fold and finish of 9 inner products)"
                if schedule == 3 else f"{k}<EpiStore> (A s_i)")
        return {"spmv": spmv, "update": "k_pass_w (w_i)",
                "spmv_fused": f"{k}<EpiPBiCGSafeAll<{nt}>> (A w_i + every other update + 9 partial inner products)"}[cls]
    return {"spmv": f"{k}<EpiStore> (A s_i)", "dots": "k_dots<ProdSafe9<false>> (9 inner products)",
            "update": f"k_passA_pbicgsafe<false, {nt}> (pass A)",
            "spmv_fused": f"{k}<EpiPBiCGSafeB> (A w_i + l, g, s)"}[cls]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def matrix_bytes(n, nnz, info=None):
    """Bytes one sparse product streams from the matrix: CSR int32 column index + FP64
    value per nonzero and an int32 row pointer, or (when the library chose the sliced
    ELLPACK layout) an FP64 value and a 32- or 16-bit column index per stored slot and an
    int32 offset per 64-row slice (ps_info.matrix_bytes)."""
    if info is not None:
        return info["matrix_bytes"]
    return 12 * nnz + 4 * (n + 1)


def bytes_per_iteration(variant, n, nnz, schedule=0, info=None):
    """Algorithmic HBM bytes of one iteration of the implemented schedule (FP64 vectors,
    each vector entry read or written once per kernel that needs it, x-gather once).

    p-BiCGSafe:  A s (M+16n) + 9 dots (40n) + pass A (160n: 12 reads, 8 writes; q_i stays in
                 registers) + A w with q, l, g, s (M+64n)
    ssBiCGSafe2: A r (M+16n) + 9 dots (40n) + p, u (64n) + A u with t, z, y, x, r (M+104n)
    p-BiCGStab:  pass 1 (96n) + A z (M+16n) + 2 dots (16n) + pass 2 (72n) + A w (M+16n)
                 + 5 dots (40n); single-stream schedule (3): the passes also read r0*
                 (104n, 80n) and form the partial sums, no dot passes: 2M + 216n
    (p-BiCGSafe-rr is counted as p-BiCGSafe; its replacement steps add ~1% at m = 100.)
    p-BiCGSafe, fused-dot schedule: A s (M+16n) + pass A with r0* (168n) + A w with q, l, g, s
                 and y, r, r0* (M+88n)
    p-BiCGSafe, fused-epilogue schedule: A s (M+16n) + w pass (40n: As, l, g, w read, w
                 written) + A w with every other update (M+192n: 13 reads, 10 writes, w gather);
                 the same for its single-stream form (schedule 3), whose A s also adds the
                 partial sums (9 triples per product workgroup: 0.2% of the iteration at 128^3,
                 not counted, like every schedule's partial sums)
    """
    M = matrix_bytes(n, nnz, info)
    if variant in ("pbicgsafe", "pbicgsafe_rr") and schedule == 1:
        return 2 * M + 272 * n
    if variant in ("pbicgsafe", "pbicgsafe_rr") and schedule in (2, 3):
        return 2 * M + 248 * n
    if variant == "pbicgstab" and schedule == 3:
        return 2 * M + 216 * n
    return {"pbicgsafe": 2 * M + 280 * n, "pbicgsafe_rr": 2 * M + 280 * n,
            "ssbicgsafe2": 2 * M + 224 * n, "pbicgstab": 2 * M + 256 * n}[variant]


def bytes_per_launch(cls, n, nnz, schedule=0, info=None):
    M = matrix_bytes(n, nnz, info)
    if schedule == 1:
        return {"spmv": M + 16 * n, "update": 168 * n, "spmv_fused": M + 88 * n}[cls]
    if schedule in (2, 3):
        return {"spmv": M + 16 * n, "update": 40 * n, "spmv_fused": M + 192 * n}[cls]
    return {"spmv": M + 16 * n, "dots": 40 * n, "update": 160 * n, "spmv_fused": M + 64 * n}[cls]


SOLVER_SOURCES = ["device_common.hpp", "dots.hpp", "layout.cpp", "layout.hpp", "pipesafe.hip",
                  "solve_one.hpp", "spmv.hpp", "updates.hpp"]


def source_digest():
    """SHA-256 prefix of the solver's sources (kernels and launch code); recorded traffic is
    used only while it matches."""
    h = hashlib.sha256()
    d = os.path.join(ROOT, "paper_2108_10591_amd", "csrc")
    for f in SOLVER_SOURCES:
        h.update(open(os.path.join(d, f), "rb").read())
    return h.hexdigest()[:16]


def load_traffic(cls, workload, schedule):
    """Counter-measured bytes per launch of class `cls`, or None if absent, taken on
    another workload or schedule, or stale (kernel sources changed since)."""
    try:
        t = json.load(open(TRAFFIC_FILE))
    except (OSError, ValueError):
        return None
    if t.get("source_digest") != source_digest() or t.get("workload") != workload \
            or t.get("schedule") != schedule:
        return None
    k = t.get("kernels", {}).get(cls)
    return None if k is None else k.get("bytes_per_launch")


def cpu_model():
    """The host CPU's model name (/proc/cpuinfo), or None."""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def cpu_baseline(A, iters_one, iters_all, variant="pbicgsafe"):
    """The FP64 oracle on the host: the set-up and `iters_one` iterations on one thread,
    then the set-up and `iters_all` iterations on every thread OpenMP gives it (the
    results are bit-identical for any thread count).  Priced with the CSR byte model of
    the iteration (2 M + 288 n, M = 12 nnz + 4 (n + 1): FP64 values, int32 columns and
    row pointers, the storage the oracle streams); the host time includes the set-up."""
    import oracle
    orc = oracle.default()
    bpi = 2 * (12 * A.nnz + 4 * (A.n + 1)) + 288 * A.n
    threads = orc.threads()
    legs = {}
    for name, th, its in (("one_core", 1, iters_one), ("all_cores", threads, iters_all)):
        orc.set_threads(th)
        t0 = time.perf_counter()
        res = orc.solve(A, tol=1e-8, maxit=its, variant=variant)
        dt = time.perf_counter() - t0
        legs[name] = {"threads": th, "iterations": res.iters, "seconds": round(dt, 2),
                      "iters_per_s": round(res.iters / dt, 2),
                      "GBps": round(bpi * res.iters / dt / 1e9, 3)}
    orc.set_threads(threads)
    a = legs["all_cores"]
    return {"value": a["GBps"], "unit": "GB/s", "cores": a["threads"], "kind": "oracle",
            "sample": f"{A.name} {variant}: set-up + {a['iterations']} iterations (maxit = "
                      f"{iters_all}) on {a['threads']} OpenMP threads in {a['seconds']} s, "
                      f"{a['iters_per_s']} iterations/s; FP64 C oracle with exact inner products; "
                      f"priced at {bpi} bytes per iteration (CSR model)",
            "nproc": os.cpu_count(), "cpu_model": cpu_model(),
            "bytes_per_iteration": bpi, "one_core": legs["one_core"], "all_cores": a}


def batch_bytes_per_iteration(info, A, schedule):
    """Bytes one iteration of system A moves in the batch's device layout: its rows padded
    to a multiple of 512, its stored entries at the batch's bytes per slot (FP64 value and
    the stored column index; sliced layout: the batch's padding ratio and one int32 offset
    per 64-row slice, CSR: one int32 row pointer per row)."""
    npad = -(-A.n // 512) * 512
    slot_bytes = 8 + info["index_bits"] // 8 + (2 if info.get("gather_sort") else 0)
    slots = A.nnz * info["slots"] / max(info["nnz"], 1)
    if info["format"] == "sell":
        M = slot_bytes * slots + 4 * (npad / 64 + 1)
    else:
        M = slot_bytes * A.nnz + 4 * (npad + 1)
    # schedules 3 and 4 make schedule 2's passes (4: inside one workgroup per system)
    per_row = {0: 280, 1: 272, 2: 248, 3: 248, 4: 248}[schedule]
    return 2 * M + per_row * npad


def bench_batch(name, reps=3):
    """The batched-systems workload: solves/s of one batched solve of every system, and
    of the same systems solved one after another with single-system handles."""
    import numpy as np
    import torch

    from paper_2108_10591_amd import pipesafe, workloads
    B = workloads.batch(name)
    tol = workloads.BATCHES[name]["tol"]
    C = B.concat()
    log(f"batch {name}: {B.nsys} systems, n = {C.n}, nnz = {C.nnz}")
    b = torch.from_numpy(C.b).cuda()
    x = torch.empty_like(b)
    with pipesafe.BatchMatrix.from_batch(B) as M:
        info = M.info()
        r = M.solve_dev(b, None, x, tol=tol, maxit=10_000, variant="pbicgsafe", hist=False)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            r = M.solve_dev(b, None, x, tol=tol, maxit=10_000, variant="pbicgsafe", hist=False)
        torch.cuda.synchronize()
        t_batch = (time.perf_counter() - t0) / reps
    assert np.all(r.status == pipesafe.CONVERGED), r.status
    # algorithmic bytes: each system's own iterations at the bytes of the layout that ran
    # (its padded rows and stored entries), for the schedule the library chose
    sched = info["auto_schedule"]
    gb = sum(int(r.iters[k]) * batch_bytes_per_iteration(info, A, sched) / 1e9
             for k, A in enumerate(B.systems))
    log(f"  batched: {1e3 * t_batch:.1f} ms, {B.nsys / t_batch:.0f} solves/s, "
        f"iterations {int(r.iters.min())}..{int(r.iters.max())}")
    # one after another (handles created and warmed up outside the timed region)
    mats, bs, xs = [], [], []
    for A in B.systems:
        mats.append(pipesafe.Matrix.from_csr(A))
        bs.append(torch.from_numpy(A.b).cuda())
        xs.append(torch.empty_like(bs[-1]))
    for M1, b1, x1 in zip(mats, bs, xs):
        M1.solve_dev(b1, None, x1, tol=tol, maxit=10_000, variant="pbicgsafe", hist=False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    it_seq = []
    for M1, b1, x1 in zip(mats, bs, xs):
        it_seq.append(M1.solve_dev(b1, None, x1, tol=tol, maxit=10_000, variant="pbicgsafe",
                                   hist=False).iters)
    torch.cuda.synchronize()
    t_seq = time.perf_counter() - t0
    for M1 in mats:
        M1.close()
    assert it_seq == [int(i) for i in r.iters]
    log(f"  one at a time: {1e3 * t_seq:.1f} ms, {B.nsys / t_seq:.0f} solves/s")
    # the autotuner: layout, then options, each by timed iterations
    t0 = time.perf_counter()
    Mt, lrows = pipesafe.BatchMatrix.autotuned(B, reps=10)
    with Mt:
        topts, orows = Mt.tune_options(b, variant="pbicgsafe", iters=30)
        t_tune = time.perf_counter() - t0
        rt = Mt.solve_dev(b, None, x, tol=tol, maxit=10_000, variant="pbicgsafe", hist=False, **topts)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            rt = Mt.solve_dev(b, None, x, tol=tol, maxit=10_000, variant="pbicgsafe", hist=False,
                              **topts)
        torch.cuda.synchronize()
        t_tuned = (time.perf_counter() - t0) / reps
        tinfo = Mt.info()
    assert np.array_equal(rt.iters, r.iters)
    best = next(row for row in lrows if row["best"])
    log(f"  autotuned ({t_tune:.1f} s of tuning): layout {best}, options {topts}: "
        f"{1e3 * t_tuned:.1f} ms, {B.nsys / t_tuned:.0f} solves/s")
    # what the small systems cost the batch: the same solve without them, and theirs alone
    # (a bound on any separate path for them, such as one workgroup per system)
    split = {}
    side = [int(round(np.sqrt(A.n))) for A in B.systems]
    for tag, keep in (("side_gt_64", lambda q: q > 64), ("side_le_64", lambda q: q <= 64)):
        sub = [A for A, q in zip(B.systems, side) if keep(q)]
        Bs = workloads.Batch(sub, f"{name}_{tag}")
        bsub = torch.from_numpy(Bs.concat().b).cuda()
        xsub = torch.empty_like(bsub)
        with pipesafe.BatchMatrix.from_batch(Bs) as Ms:
            Ms.solve_dev(bsub, None, xsub, tol=tol, maxit=10_000, variant="pbicgsafe", hist=False)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(reps):
                rs = Ms.solve_dev(bsub, None, xsub, tol=tol, maxit=10_000, variant="pbicgsafe",
                                  hist=False)
            torch.cuda.synchronize()
            ts = (time.perf_counter() - t0) / reps
        split[tag] = {"systems": len(sub), "time_ms": round(1e3 * ts, 2),
                      "iterations_max": int(np.max(rs.iters))}
    log(f"  split by grid side: {split}")
    # a batch of many small systems (4096 stencils of 8^2..16^2 rows, the same family):
    # the automatic schedule (one workgroup per system) against the shared launches
    Bt = workloads.cd2d_batch(nsys=4096, seed=5, nmin=8, nmax=16)
    bt = torch.from_numpy(Bt.concat().b).cuda()
    xt = torch.empty_like(bt)
    small = {"systems": Bt.nsys, "grid_sides": [8, 16], "tol": tol}
    with pipesafe.BatchMatrix.from_batch(Bt) as Mt2:
        small["auto_schedule"] = Mt2.info()["auto_schedule"]
        for tag, sched in (("automatic", -1), ("schedule_2", 2)):
            Mt2.solve_dev(bt, None, xt, tol=tol, maxit=10_000, variant="pbicgsafe", hist=False,
                          schedule=sched)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(reps):
                rt2 = Mt2.solve_dev(bt, None, xt, tol=tol, maxit=10_000, variant="pbicgsafe",
                                    hist=False, schedule=sched)
            torch.cuda.synchronize()
            ts = (time.perf_counter() - t0) / reps
            small[tag] = {"time_ms": round(1e3 * ts, 3), "solves_per_s": round(Bt.nsys / ts, 1),
                          "iterations_max": int(np.max(rt2.iters))}
    log(f"  small systems: {small}")
    return {"workload": name, "systems": B.nsys, "rows": C.n, "nnz": C.nnz, "tol": tol,
            "variant": "pbicgsafe", "layout": info["format"], "schedule": sched,
            "iterations_min_mean_max": [int(r.iters.min()), round(float(r.iters.mean()), 1),
                                        int(r.iters.max())],
            "time_ms": round(1e3 * t_batch, 2), "solves_per_s": round(B.nsys / t_batch, 1),
            "GBps": round(gb / t_batch, 1),
            "one_at_a_time": {"time_ms": round(1e3 * t_seq, 2),
                              "solves_per_s": round(B.nsys / t_seq, 1)},
            "speedup": round(t_seq / t_batch, 2),
            "autotuned": {"layout": {k: best[k] for k in ("format", "sell_rows_per_lane",
                                                            "spmv_shape", "index_bits")},
                          "options": topts, "tuning_s": round(t_tune, 2),
                          "layouts_timed_us": [round(row["us"], 2) for row in lrows],
                          "time_ms": round(1e3 * t_tuned, 2),
                          "solves_per_s": round(B.nsys / t_tuned, 1),
                          "same_format_as_automatic": tinfo["format"] == info["format"]},
            "split": split, "small_systems": small}


def bench_mixed(name, rr_ms, reps=3):
    """Mixed precision on one system: time to the workload's tolerance from x0 = 0 in FP64
    (p-BiCGSafe, and p-BiCGSafe-rr at each replacement period m), with the matrix values
    rounded to FP32 in every product (p-BiCGSafe), with them rounded in the Krylov
    products only (p-BiCGSafe-rr, FP64 replacement residual), and with p, u, z also held
    in FP32 (p-BiCGSafe-rr).  Each result states its true FP64 residual ||b - A x|| / ||b||
    (FP64 product on the GPU) and its distance from the FP64 p-BiCGSafe solution."""
    import torch

    from paper_2108_10591_amd import pipesafe, workloads
    A = workloads.workload(name)
    tol = workloads.WORKLOADS[name]["tol"]
    log(f"mixed precision {name}: n = {A.n}, nnz = {A.nnz}, tol {tol}")
    b = torch.from_numpy(A.b).cuda()
    x = torch.empty_like(b)
    runs = [("fp64", "pbicgsafe", 0, 100), ("fp32_matrix", "pbicgsafe", 1, 100)]
    for m in rr_ms:
        runs += [(f"fp64_rr_m{m}", "pbicgsafe_rr", 0, m), (f"fp32_krylov_rr_m{m}", "pbicgsafe_rr", 2, m),
                 (f"fp32_vectors_rr_m{m}", "pbicgsafe_rr", 3, m)]
    out = {"workload": name, "n": A.n, "nnz": A.nnz, "tol": tol, "x0": "zero",
           "stop": "||r_i|| <= tol ||r_0|| (recursive residual)"}
    with pipesafe.Matrix.from_csr(A) as M:
        out["layout"] = M.info()["format"]
        nb = float(torch.linalg.vector_norm(b))
        x64 = None
        for label, variant, prec, m in runs:
            kw = dict(tol=tol, maxit=10_000, variant=variant, rr_m=m, precision=prec, hist=False)
            r = M.solve_dev(b, None, x, **kw)
            torch.cuda.synchronize()
            ts = []
            for _ in range(reps):
                t0 = time.perf_counter()
                r = M.solve_dev(b, None, x, **kw)
                torch.cuda.synchronize()
                ts.append(time.perf_counter() - t0)
            t = sorted(ts)[len(ts) // 2]
            res = float(torch.linalg.vector_norm(b - M.spmv_dev(x))) / nb
            if x64 is None:
                x64 = x.clone()
            err = float((x - x64).abs().max() / x64.abs().max())
            out[label] = {"variant": variant, "rr_m": m if variant == "pbicgsafe_rr" else None,
                          "iterations": r.iters, "status": r.status_name,
                          "time_to_tol_ms": round(1e3 * t, 3),
                          "us_per_iter": round(1e6 * t / max(r.iters, 1), 2),
                          "true_residual_fp64": res, "err_vs_fp64_solution": err}
            log(f"  {label}: {out[label]}")
    # a speedup counts only at the same accuracy: the run's true FP64 residual within the
    # tolerance, or within the FP64 p-BiCGSafe run's own true residual (which the recursive
    # residual's drift can put slightly above the tolerance)
    t64 = out["fp64"]["time_to_tol_ms"]
    bar = max(tol, out["fp64"]["true_residual_fp64"])
    for label, *_ in runs[1:]:
        o = out[label]
        if o["status"] == "converged" and o["true_residual_fp64"] <= bar:
            o["speedup_vs_fp64"] = round(t64 / o["time_to_tol_ms"], 3)
        else:
            o["speedup_vs_fp64"] = None
            o["speedup_withheld"] = (f"true FP64 residual {o['true_residual_fp64']:.2e} above "
                                     f"{bar:.2e} (the tolerance or the FP64 run's residual)")
    return out


def bench_small(name, reps=5):
    """A small system (latency-bound): time to the workload's tolerance and microseconds
    per iteration of every method, with the library's automatic choices."""
    import torch

    from paper_2108_10591_amd import pipesafe, workloads
    A = workloads.workload(name)
    tol = workloads.WORKLOADS[name]["tol"]
    b = torch.from_numpy(A.b).cuda()
    x = torch.empty_like(b)
    out = {"workload": name, "n": A.n, "nnz": A.nnz, "tol": tol, "x0": "zero"}
    with pipesafe.Matrix.from_csr(A) as M:
        out["layout"] = M.info()["format"]
        for v in ("pbicgsafe", "ssbicgsafe2", "pbicgsafe_rr", "pbicgstab"):
            r = M.solve_dev(b, None, x, tol=tol, maxit=10_000, variant=v, hist=False)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(reps):
                r = M.solve_dev(b, None, x, tol=tol, maxit=10_000, variant=v, hist=False)
            torch.cuda.synchronize()
            t = (time.perf_counter() - t0) / reps
            out[v] = {"iterations": r.iters, "status": r.status_name,
                      "time_to_tol_ms": round(1e3 * t, 3),
                      "us_per_iter": round(1e6 * t / max(r.iters, 1), 2)}
    # a tiny system (16^2 rows of the same problem family): the automatic choice, the whole
    # solve in one workgroup (schedule 4), against the single-stream launches (3)
    T = workloads.cd2d(16)
    bt = torch.from_numpy(T.b).cuda()
    xt = torch.empty_like(bt)
    tiny = {"workload": "cd2d_16", "n": T.n, "tol": tol}
    with pipesafe.Matrix.from_csr(T) as M:
        tiny["auto_schedule"] = M.info()["auto_schedule"]
        for tag, sched in (("automatic", -1), ("schedule_3", 3)):
            r = M.solve_dev(bt, None, xt, tol=tol, maxit=10_000, variant="pbicgsafe", hist=False,
                            schedule=sched)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(4 * reps):
                r = M.solve_dev(bt, None, xt, tol=tol, maxit=10_000, variant="pbicgsafe",
                                hist=False, schedule=sched)
            torch.cuda.synchronize()
            t = (time.perf_counter() - t0) / (4 * reps)
            tiny[tag] = {"iterations": r.iters, "status": r.status_name,
                         "time_to_tol_ms": round(1e3 * t, 4),
                         "us_per_iter": round(1e6 * t / max(r.iters, 1), 2)}
    out["tiny_system"] = tiny
    log(f"small system {name}: {out}")
    return out


def bench_warmstart(count, epochs):
    """The learned initial guess on 128 x 128 variable-coefficient problems: training data
    solved on the GPU, the network trained on the GPU, then 64 held-out problems solved to
    1e-10 ||b|| by p-BiCGSafe-rr from x0 = 0 and from the prediction."""
    from paper_2108_10591_amd import warmstart
    log(f"warm start: {count} training problems, {epochs} epochs ...")
    m = warmstart.train(N=128, count=count, epochs=epochs, lr=1e-3, seed=1, verbose=log)
    r = warmstart.evaluate(m, N=128, count=64, seed=2)
    log(f"  {r}")
    r.update({"train_problems": count, "train_samples_kept": m.samples, "epochs": epochs,
              "params": m.net.num_params, "train_s": round(m.train_seconds, 2),
              "data": m.data, "loss_first_last": [float(m.loss_hist[0]), float(m.loss_hist[-1])]})
    m.net.close()
    return r


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="cd3d_128")
    ap.add_argument("--variant", default="pbicgsafe")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-variants", action="store_true")
    ap.add_argument("--no-batch", action="store_true", help="skip the batched-systems leg")
    ap.add_argument("--no-warmstart", action="store_true", help="skip the learned-initial-guess leg")
    ap.add_argument("--warmstart-count", type=int, default=20000,
                    help="training problems of the learned-initial-guess leg")
    ap.add_argument("--warmstart-epochs", type=int, default=20)
    ap.add_argument("--no-mixed", action="store_true", help="skip the mixed-precision leg")
    ap.add_argument("--mixed-rr-m", default="100",
                    help="replacement periods of the mixed-precision leg (comma-separated)")
    ap.add_argument("--cpu-iters", type=int, default=30,
                    help="iterations of the one-thread CPU baseline leg")
    ap.add_argument("--cpu-iters-all", type=int, default=150,
                    help="iterations of the all-threads CPU baseline leg")
    ap.add_argument("--overlap", type=int, default=-1, help="1 on, 0 off, -1 automatic")
    ap.add_argument("--schedule", type=int, default=-1,
                    help="p-BiCGSafe: 0 separate inner-product pass, 1 fused partial sums, "
                         "2 fused epilogue, -1 the library's automatic choice")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only run the library's streaming copy on MIB MiB (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py runs on one GPU only: the solver is a single-GPU implementation "
              "(multi-GPU sharding is a design note, not built); use --gpus 1", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2108_10591_amd import pipesafe, workloads

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)

    if args.calibrate_copy:
        nb = args.calibrate_copy * (1 << 20)
        src = torch.ones(nb // 8, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            pipesafe.stream_copy(dst, src)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        reps = 20
        for _ in range(reps):
            pipesafe.stream_copy(dst, src)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / reps
        log(f"copy {args.calibrate_copy} MiB: {2 * nb / dt / 1e9:.1f} GB/s (read + write)")
        print(json.dumps({"copy_bytes_read": nb, "copy_bytes_written": nb,
                          "copy_GBps": round(2 * nb / dt / 1e9, 1)}))
        return

    log(f"building workload {args.workload} ...")
    t0 = time.perf_counter()
    A = workloads.workload(args.workload)
    tol = workloads.WORKLOADS[args.workload]["tol"]
    log(f"  n={A.n} nnz={A.nnz} ({time.perf_counter() - t0:.1f} s)")
    M = pipesafe.Matrix.from_csr(A)
    info = M.info()
    log(f"  device layout: {info}")
    b = torch.from_numpy(A.b).to(dev)
    x = torch.empty(A.n, dtype=torch.float64, device=dev)
    maxit = 10_000
    variant = args.variant

    # one profiled solve to find the dominant kernel class
    if variant in ("pbicgsafe", "pbicgsafe_rr"):
        sched = info["auto_schedule"] if args.schedule < 0 else args.schedule
    elif variant == "pbicgstab":  # the single-stream schedule unless asked for the passes
        sched = 0 if args.schedule == 0 else 3
    else:
        sched = 0
    res = M.solve_dev(b, None, x, tol=tol, maxit=maxit, variant=variant, overlap=args.overlap,
                      schedule=sched, profile=CLASSES[:4], hist=False)
    stats = M.kernel_stats()
    dominant = max([c for c in CLASSES[:4] if sched == 0 or c != "dots"], key=lambda c: stats[c][0])
    log(f"profiled solve: iters={res.iters} status={res.status_name}; per-class ms: "
        + ", ".join(f"{c}={stats[c][0]:.2f}/{stats[c][1]}" for c in CLASSES[:4])
        + f"; dominant: {dominant}")

    opts = dict(overlap=args.overlap, schedule=sched)
    for _ in range(args.warmup):
        M.solve_dev(b, None, x, tol=tol, maxit=maxit, variant=variant, hist=False, **opts)
    # the timed steps: full solves as a caller runs them (no instrumentation)
    torch.cuda.synchronize()
    iters = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        r = M.solve_dev(b, None, x, tol=tol, maxit=maxit, variant=variant, hist=False, **opts)
        iters.append(r.iters)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    assert r.status == pipesafe.CONVERGED, r.status_name
    it = iters[-1]
    assert all(i == it for i in iters), iters
    ms_per_step = 1e3 * elapsed / args.steps
    bpi = bytes_per_iteration(variant, A.n, A.nnz, sched, info)
    value = bpi * it / (ms_per_step * 1e-3) / 1e9
    xh = x.cpu().numpy()
    err1 = float(np.abs(xh - 1.0).max())
    log(f"{variant}: {it} iterations, {ms_per_step:.2f} ms/solve, {1e3 * ms_per_step / it:.1f} us/iter,"
        f" {value:.0f} GB/s, ||x-1||_inf={err1:.2e}")

    # the dominant kernel, timed with HIP events around each of its launches on
    # its own stream over the same number of profiled solves (events disable the
    # graph replay, so they are kept out of the timed steps above)
    kms, kcnt = 0.0, 0
    t1 = time.perf_counter()
    for _ in range(args.steps):
        r = M.solve_dev(b, None, x, tol=tol, maxit=maxit, variant=variant, hist=False,
                        profile=[dominant], **opts)
        st = M.kernel_stats()[dominant]
        kms += st[0]
        kcnt += st[1]
    torch.cuda.synchronize()
    ms_profiled = 1e3 * (time.perf_counter() - t1) / args.steps
    avg_us = 1e3 * kms / max(kcnt, 1)
    bpl = bytes_per_launch(dominant, A.n, A.nnz, sched, info)
    achieved = bpl / (avg_us * 1e-6) / 1e9
    traffic = load_traffic(dominant, args.workload, sched) if variant == "pbicgsafe" else None
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": PEAK_GBPS, "unit": "GB/s",
                "frac": round(achieved / PEAK_GBPS, 4), "traffic": traffic,
                "kernel": kernel_name(dominant, info["format"], sched,
                                      info["streaming"] if variant == "pbicgsafe" else 0), "bytes_per_launch": bpl,
                "avg_launch_us": round(avg_us, 3), "launches": kcnt,
                "measured_over": f"{args.steps} profiled solves ({ms_profiled:.1f} ms each)"}

    out = {"metric": METRIC, "value": round(value, 1), "unit": "GB/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_per_step, 3),
           "higher_is_better": True, "scaling": "strong", "vs_baseline": None, "dtype": "f64",
           "data": "synthetic",
           "config": {"workload": args.workload, "n": A.n, "nnz": A.nnz, "variant": variant,
                      "tol": tol, "x0": "zero", "rhs": "A*ones", "iterations": it,
                      "bytes_per_iteration": bpi, "matrix_layout": info["format"],
                      "matrix_bytes": info["matrix_bytes"], "overlap": args.overlap, "schedule": sched,
                      "graphs": True},
           "time_to_tol_ms": round(ms_per_step, 3), "iters_per_s": round(it / (ms_per_step * 1e-3), 1),
           "us_per_iter": round(1e3 * ms_per_step / it, 2),
           "iteration_hbm_frac": round(value / PEAK_GBPS, 4), "x_minus_1_inf": err1,
           "roofline": roofline}

    if not args.no_variants:
        var = {}
        others = [("ssbicgsafe2", 0), ("pbicgsafe_rr", -1), ("pbicgstab", -1), ("pbicgstab", 0)]
        others += [("pbicgsafe", sc) for sc in (0, 1, 2, 3) if sc != sched]
        for v, sc in others:
            key = {"pbicgsafe": {0: "pbicgsafe_dot_pass", 1: "pbicgsafe_fused_dots",
                                 2: "pbicgsafe_fused_epilogue", 3: "pbicgsafe_single_stream"},
                   "pbicgstab": {-1: "pbicgstab", 0: "pbicgstab_dot_passes"}}.get(v, {}).get(sc, v)
            M.solve_dev(b, None, x, tol=tol, maxit=maxit, variant=v, schedule=sc)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            reps = 3
            for _ in range(reps):
                rv = M.solve_dev(b, None, x, tol=tol, maxit=maxit, variant=v, schedule=sc, hist=False)
            torch.cuda.synchronize()
            ms = 1e3 * (time.perf_counter() - t1) / reps
            sc_run = info["auto_schedule"] if sc < 0 else sc  # what the library chose
            if v == "pbicgstab":  # its own rule: 3 for one system unless asked for 0
                sc_run = 0 if sc == 0 else 3
            gbps = bytes_per_iteration(v, A.n, A.nnz, sc_run, info) * rv.iters / (ms * 1e-3) / 1e9
            v = key
            var[v] = {"iterations": rv.iters, "status": rv.status_name, "time_to_tol_ms": round(ms, 3),
                      "us_per_iter": round(1e3 * ms / max(rv.iters, 1), 2), "GBps": round(gbps, 1)}
            log(f"{v}: {var[v]}")
        out["variants"] = var

    if not args.no_variants:
        out["small_system"] = bench_small("cd2d_64")

    if not args.no_batch:
        out["batched"] = bench_batch("cd2d_batch_512")

    if not args.no_warmstart:
        out["warm_start"] = bench_warmstart(args.warmstart_count, args.warmstart_epochs)
    if not args.no_mixed:
        ms = [int(m) for m in args.mixed_rr_m.split(",")]
        out["mixed_precision"] = bench_mixed("rand_band_1m", ms)
        out["mixed_precision_stencil"] = bench_mixed(args.workload, ms)

    if not args.no_cpu_baseline:
        log(f"cpu baseline: oracle, {args.cpu_iters} iterations on one thread, "
            f"{args.cpu_iters_all} on all ...")
        out["cpu_baseline"] = cpu_baseline(A, args.cpu_iters, args.cpu_iters_all, variant)
        log(f"  {out['cpu_baseline']}")
    M.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
