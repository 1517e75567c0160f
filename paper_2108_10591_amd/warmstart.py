"""Learned initial guess for p-BiCGSafe: data, training and evaluation.

Orchestration only; every numerical step runs in the library's kernels:
  * training data: variable-coefficient problems (workloads.varcoef_problems)
    solved by the batched GPU solver (ps_solve_batch);
  * the network (include/wsnet.h) trained with ws_train on the GPU;
  * evaluation: held-out problems solved from x0 = 0 and from the network's
    prediction, same tolerance and stop-test scale (||b||), same solver.
"""
from __future__ import annotations

import time
from dataclasses import dataclass

import numpy as np

from . import pipesafe, workloads, wsnet


def solve_batch(B, tol, variant="pbicgsafe_rr", x0=None, fallback=0, maxit=20_000, rr_m=50,
                hist0=False):
    """Solve every system of workloads.Batch B on the GPU (norm_ref = ||b||); fallback is
    ps_options.x0_fallback (0 as given, 1 the ||b - A x0|| <= ||b|| rule, 2 the guess scaled
    to its least residual, then the rule).  Returns (x numpy, iters, status, seconds of the
    solve call), and with hist0 also each system's ||r_0|| / ||b|| (its first history entry:
    exactly 1 where the guess was replaced by zero)."""
    import torch
    C = B.concat()
    with pipesafe.BatchMatrix.from_batch(B) as M:
        b = torch.from_numpy(C.b).cuda()
        x0t = None if x0 is None else torch.from_numpy(np.ascontiguousarray(x0, dtype=np.float64)).cuda()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = M.solve_dev(b, x0=x0t, tol=tol, maxit=maxit, variant=variant, norm_ref=1, rr_m=rr_m,
                        x0_fallback=fallback, hist=hist0)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        out = (r.x.cpu().numpy(), r.iters.copy(), r.status.copy(), dt)
        return out + (r.hist[:, 0].copy(),) if hist0 else out


@dataclass
class Trained:
    net: object
    scale: float
    loss_hist: np.ndarray
    train_seconds: float
    data_seconds: float
    samples: int
    data: dict


def make_data(N, count, seed, tol=1e-8, chunk=1024, log=None):
    """Network inputs and GPU-solved targets for `count` problems, generated and
    solved `chunk` at a time; unconverged problems are dropped.
    Returns (inputs float32 [m, N, N, 3], solutions float32 [m, N, N], report)."""
    log = log or (lambda *a: None)
    feats, sols = [], []
    gen_s = solve_s = 0.0
    its, kept = [], 0
    for c0 in range(0, count, chunk):
        m = min(chunk, count - c0)
        t0 = time.perf_counter()
        B, F = workloads.varcoef_problems(m, N, seed=seed * 100_003 + c0)
        gen_s += time.perf_counter() - t0
        x, it, st, dt = solve_batch(B, tol)
        solve_s += dt
        ok = st == pipesafe.CONVERGED
        feats.append(F[ok])
        sols.append(x.reshape(m, N, N)[ok].astype(np.float32))
        its.append(it)
        kept += int(ok.sum())
        log(f"  problems {c0}..{c0 + m - 1}: solved in {dt:.1f} s, iterations {int(it.min())}..{int(it.max())}")
    its = np.concatenate(its)
    report = {"problems": count, "kept": kept, "generate_s": round(gen_s, 1), "solve_s": round(solve_s, 1),
              "iterations_mean": float(its.mean()), "tol": tol}
    return np.concatenate(feats), np.concatenate(sols), report


def train(N=128, count=20_000, epochs=30, batch=32, lr=1e-3, seed=1, data_tol=1e-8, verbose=None):
    """Generate `count` problems, solve them for the targets, train the network."""
    import torch
    log = verbose or (lambda *a: None)
    t0 = time.perf_counter()
    X, T, rep = make_data(N, count, seed, data_tol, log=log)
    scale = float(2.0 * np.abs(T).mean())
    data_seconds = time.perf_counter() - t0
    net = wsnet.WarmStartNet(N, N, 3, 16, seed=seed)
    Xd = torch.from_numpy(X).cuda()
    Td = torch.from_numpy(T / np.float32(scale)).cuda()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    hist = net.train(Xd, Td, batch=batch, epochs=epochs, lr=lr, seed=seed + 7)
    torch.cuda.synchronize()
    train_seconds = time.perf_counter() - t1
    log(f"  trained {epochs} epochs on {len(X)} samples in {train_seconds:.1f} s, "
        f"loss {hist[0]:.3e} -> {hist[-1]:.3e}")
    del Xd, Td
    return Trained(net, scale, hist, train_seconds, data_seconds, len(X), rep)


def predict(model: Trained, F):
    """x0 for problems with network inputs F [count, N, N, 3] (numpy), and the seconds it took."""
    import torch
    Fd = torch.from_numpy(np.ascontiguousarray(F)).cuda()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    y = model.net.forward(Fd, scale=model.scale)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    return y.cpu().numpy().reshape(-1).astype(np.float64), dt


def evaluate(model: Trained, N=128, count=64, seed=2, tol=1e-10, variant="pbicgsafe_rr"):
    """Held-out problems: iterations and time to tol from x0 = 0 and from the
    network's prediction -- as given, with the ||b - A x0|| <= ||b|| rule, and
    scaled on the device to its least residual before the rule (x0_fallback =
    2, the library's own step; its time is inside the solve).  Times include
    the prediction."""
    B, F = workloads.varcoef_problems(count, N, seed=seed)
    x0, t_pred = predict(model, F)
    _, it0, st0, t0 = solve_batch(B, tol, variant)
    _, it1, st1, t1, h1 = solve_batch(B, tol, variant, x0=x0, hist0=True)
    _, it2, st2, t2, h2 = solve_batch(B, tol, variant, x0=x0, fallback=1, hist0=True)
    _, it3, st3, t3, h3 = solve_batch(B, tol, variant, x0=x0, fallback=2, hist0=True)
    return {
        "problems": count, "N": N, "tol": tol, "variant": variant, "norm_ref": "||b||",
        "iters_x0_zero": {"mean": float(it0.mean()), "median": float(np.median(it0))},
        "iters_x0_net": {"mean": float(it1.mean()), "median": float(np.median(it1))},
        "iters_saved_mean": float((it0 - it1).mean()),
        "iters_saved_frac": float((it0 - it1).sum() / it0.sum()),
        "converged": [int((st0 == 0).sum()), int((st1 == 0).sum())],
        "time_x0_zero_ms": round(1e3 * t0, 2),
        "time_x0_net_ms": round(1e3 * (t1 + t_pred), 2),
        "predict_ms": round(1e3 * t_pred, 2),
        "initial_residual_over_b_median": float(np.median(h1)),
        "with_fallback": {"iters_mean": float(it2.mean()), "time_ms": round(1e3 * (t2 + t_pred), 2),
                          "iters_saved_frac": float((it0 - it2).sum() / it0.sum()),
                          "guesses_kept": int((h2 < 1.0).sum()), "converged": int((st2 == 0).sum())},
        "scaled_with_fallback": {"x0_fallback": 2, "iters_mean": float(it3.mean()),
                                 "iters_saved_frac": float((it0 - it3).sum() / it0.sum()),
                                 "time_ms": round(1e3 * (t3 + t_pred), 2),
                                 "initial_residual_over_b_median": float(np.median(h3)),
                                 "guesses_kept": int((h3 < 1.0).sum()),
                                 "converged": int((st3 == 0).sum())},
    }
