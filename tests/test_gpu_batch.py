"""GPU parity of batched solves (ps_create_batch / ps_solve_batch).

A batched solve runs independent systems through shared launches; each system
must come out exactly as the oracle solves it alone: same status, iteration
count, residual history and solution bits.  The batches below mix sizes (not
multiples of the 512-row padding), sparsity patterns and outcomes (converged,
stopped at i = 1, breakdown at i = 0, non-finite inner products, maxit).
"""
import hashlib
import json
import os
import sys

import numpy as np
import pytest

import oracle as O
from paper_2108_10591_amd import pipesafe, workloads as W

pytestmark = pytest.mark.gpu

VARIANTS = ["ssbicgsafe2", "pbicgsafe", "pbicgsafe_rr", "pbicgstab"]
GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "batch_oracle.json")


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need an MI355X"
    torch.cuda.set_device(0)
    pipesafe.library()


def mixed_batch():
    """Systems of assorted sizes and outcomes; b of the NaN system poisoned."""
    systems = [
        W.cd2d(17, 10.0),
        W.small_nonsym(300, 4, density=0.02),
        W.identity(50, seed=1),                                    # stops at i = 1
        W.rand_band(3000, seed=5, band=200),
        W.skew_blocks(64, seed=1),                                 # breakdown at i = 0
        W.cd2d(33, 40.0, kfield=np.exp(0.5 * np.random.default_rng(2).standard_normal((33, 33)))),
        W.small_nonsym(40, 0),                                     # NaN in b
        W.cd3d(9, 20.0, seed=3),
        W.diag_distinct(700, [1.0, 2.0, 5.0], seed=2),             # three eigenvalues
        W.cd2d(5, 10.0),
    ]
    B = W.Batch(systems, "mixed")
    C = B.concat()
    b = C.b.copy()
    p = B.sys_ptr()
    b[p[6] + 7] = np.nan
    return B, C, b


def oracle_each(B, b, tol, maxit, variant, **kw):
    p = B.sys_ptr()
    return [O.solve(A, b=b[p[k]:p[k + 1]], tol=tol, maxit=maxit, variant=variant, **kw)
            for k, A in enumerate(B.systems)]


def check_same(res, refs, B, label):
    p = B.sys_ptr()
    for k, R in enumerate(refs):
        assert res.status[k] == R.status and res.iters[k] == R.iters, \
            (label, k, B.systems[k].name, res.status[k], R.status, res.iters[k], R.iters)
        assert np.array_equal(res.system_hist(k), R.hist, equal_nan=True), (label, k)
        x = res.x[p[k]:p[k + 1]]
        assert np.array_equal(x, R.x, equal_nan=True), (label, k)


@pytest.mark.parametrize("variant", VARIANTS)
def test_batch_equals_each_system_alone(variant):
    B, C, b = mixed_batch()
    for tol, maxit in ((1e-10, 2000), (0.0, 7)):
        refs = oracle_each(B, b, tol, maxit, variant, rr_m=9)
        with pipesafe.BatchMatrix.from_batch(B) as M:
            info = M.info()
            assert info["nsys"] == B.nsys and info["n"] == C.n and info["n_padded"] % 512 == 0
            runs = [dict(overlap=0, graph=0), dict(overlap=1, graph=1, batch_iters=3),
                    dict(graph=1, batch_iters=5)]
            if variant in ("pbicgsafe", "pbicgsafe_rr"):  # the fused-dot schedules
                runs += [dict(schedule=1, graph=0), dict(schedule=1, graph=1, batch_iters=4),
                         dict(schedule=2, overlap=0, graph=0),
                         dict(schedule=2, graph=1, batch_iters=3)]
            for kw in runs:
                say(f"batch {variant} tol={tol} {kw}")
                res = M.solve(b, tol=tol, maxit=maxit, variant=variant, rr_m=9, **kw)
                check_same(res, refs, B, (variant, tol, str(kw)))


@pytest.mark.parametrize("fmt", ["csr", "sell"])
def test_batch_both_layouts_and_device_buffers(fmt):
    import torch
    B, C, b = mixed_batch()
    x0 = np.linspace(0.0, 1.0, C.n)
    # the skew-symmetric system keeps x0 = 0: its (r0*, A r0) is then exactly 0 and the
    # solve stops with a breakdown at i = 0, as in the other batch tests.  With a
    # non-integer x0 that inner product is pure cancellation (condition ~1e17) and
    # alpha = f / g would be ~1e19: a test of overflow, not of the method.
    p = B.sys_ptr()
    x0[p[4]:p[5]] = 0.0
    refs = [O.solve(A, b=b[p0:p1], x0=x0[p0:p1], tol=1e-9, maxit=2000, variant="pbicgsafe",
                    norm_ref=1)
            for A, p0, p1 in zip(B.systems, B.sys_ptr()[:-1], B.sys_ptr()[1:])]
    old = os.environ.get("PIPESAFE_FORMAT")
    os.environ["PIPESAFE_FORMAT"] = {"csr": "0", "sell": "1"}[fmt]
    try:
        M = pipesafe.BatchMatrix.from_batch(B)
    finally:
        if old is None:
            del os.environ["PIPESAFE_FORMAT"]
        else:
            os.environ["PIPESAFE_FORMAT"] = old
    with M:
        assert M.info()["format"] == fmt
        for sched in (0, 1, 2):
            say(f"batch layout {fmt}, device buffers, x0, norm_ref = 1, schedule {sched}")
            res = M.solve_dev(torch.from_numpy(b).cuda(), x0=torch.from_numpy(x0).cuda(),
                              tol=1e-9, maxit=2000, variant="pbicgsafe", norm_ref=1,
                              schedule=sched)
            torch.cuda.synchronize()
            res.x = res.x.cpu().numpy()
            check_same(res, refs, B, (fmt, sched))


def test_batch_rejects_single_system_calls():
    B, C, b = mixed_batch()
    with pipesafe.BatchMatrix.from_batch(B) as M:
        L = pipesafe.library()
        assert L.ps_solve(M._h, None, None, 1e-8, 10, 1, None, None, None, None, None) == -1
        with pytest.raises(pipesafe.PipesafeError):
            M.solve(b, tol=1e-8, maxit=10, variant="pbicgstab", schedule=1)
        with pytest.raises(pipesafe.PipesafeError):  # one stop flag per system: no schedule 3
            M.solve(b, tol=1e-8, maxit=10, variant="pbicgsafe", schedule=3)
        with pytest.raises(pipesafe.PipesafeError):
            M.solve(b, tol=1e-8, maxit=10, variant="pbicgsafe", resume=1)
        # schedule -1 (automatic) means the fused epilogue for batches
        assert M.info()["auto_schedule"] == 2
        res = M.solve(b, tol=1e-10, maxit=50, variant="pbicgsafe", schedule=-1)
        assert res.iters[2] == 1


@pytest.mark.parametrize("schedule", [-1, 1, 2])
def test_full_batch_512_reproduces_oracle(schedule):
    """The 512-system benchmark batch (N ~ U[32, 256], 12.4M rows): every system's
    iteration count, status, history and solution bits against the oracle's
    independent solves, written by tests/golden/make_batch.py, under each
    inner-product schedule."""
    import torch
    g = json.load(open(GOLDEN))
    name = g["workload"]
    Bt = W.batch(name)
    tol = W.BATCHES[name]["tol"]
    C = Bt.concat()
    with pipesafe.BatchMatrix.from_batch(Bt) as M:
        say(f"full batch {name}: {Bt.nsys} systems, n = {C.n}, schedule {schedule}")
        res = M.solve_dev(torch.from_numpy(C.b).cuda(), tol=tol, maxit=10_000, variant="pbicgsafe",
                          schedule=schedule)
        x = res.x.cpu().numpy()
    p = Bt.sys_ptr()
    for k in range(Bt.nsys):
        r = g["runs"][str(k)]
        assert res.status[k] == r["status"] and res.iters[k] == r["iters"], (k, res.iters[k], r)
        h = np.ascontiguousarray(res.system_hist(k))
        assert hashlib.sha256(h.tobytes()).hexdigest() == r["hist_sha256"], k
        xk = np.ascontiguousarray(x[p[k]:p[k + 1]])
        assert hashlib.sha256(xk.tobytes()).hexdigest() == r["x_sha256"], k
