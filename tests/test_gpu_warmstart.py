"""The learned initial guess end to end (small scale): problems solved on the
GPU for training targets, the network trained on the GPU, and held-out
problems solved from x0 = 0 and from the network's prediction with the same
solver, tolerance and stop-test scale (||b||).  Also the x0 fallback rule of
ps_options, exactly: a rejected guess gives the x0 = 0 solve bit for bit."""
import sys

import numpy as np
import pytest

import oracle as O
from paper_2108_10591_amd import pipesafe, warmstart, workloads as W

pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need an MI355X"
    torch.cuda.set_device(0)


def test_trained_guess_saves_iterations():
    model = warmstart.train(N=64, count=1024, epochs=15, lr=1e-3, seed=5, verbose=say)
    assert model.loss_hist[-1] < 0.5 * model.loss_hist[0]
    r = warmstart.evaluate(model, N=64, count=32, seed=6)
    say(str(r))
    assert r["converged"] == [32, 32]
    assert r["iters_saved_mean"] > 0, r
    # with the library's own rule (x0_fallback = 2: least-residual scaling, then the
    # ||b - A x0|| <= ||b|| test) the guesses are kept and still save iterations
    sc = r["scaled_with_fallback"]
    assert sc["converged"] == 32 and sc["guesses_kept"] > 0, sc
    assert sc["iters_saved_frac"] > 0, sc


def test_fallback_rejects_a_bad_guess_exactly():
    """A guess worse than zero is replaced by zero: the same bits as the x0 = 0 solve."""
    import torch
    A = W.workload("cd2d_64")
    bad = 1e3 * np.sin(np.arange(A.n))           # ||b - A x0|| >> ||b||
    ref = O.solve(A, tol=1e-10, maxit=3000, variant="pbicgsafe")
    with pipesafe.Matrix.from_csr(A) as M:
        res = M.solve(A.b, x0=bad, tol=1e-10, maxit=3000, variant="pbicgsafe", x0_fallback=1)
        assert res.iters == ref.iters and np.array_equal(res.x, ref.x) and np.array_equal(res.hist, ref.hist)
        # a good guess is kept, and with the ||b|| stop-test scale it saves iterations
        good = np.ones(A.n) * (1.0 + 1e-6)
        kept = M.solve(A.b, x0=good, tol=1e-10, maxit=3000, variant="pbicgsafe", x0_fallback=1,
                       norm_ref=1)
        plain = M.solve(A.b, x0=good, tol=1e-10, maxit=3000, variant="pbicgsafe", norm_ref=1)
        assert kept.iters == plain.iters and np.array_equal(kept.x, plain.x)
        assert kept.iters < ref.iters


def test_fallback_per_system_in_a_batch():
    import torch
    B = W.Batch([W.workload("cd2d_64"), W.cd2d(20, 5.0), W.small_nonsym(300, 4, density=0.02)], "fb")
    C = B.concat()
    p = B.sys_ptr()
    x0 = np.zeros(C.n)
    x0[p[0]:p[1]] = 1e3 * np.sin(np.arange(p[1] - p[0]))   # rejected
    x0[p[1]:p[2]] = 1.0 + 1e-7                             # kept
    x0[p[2]:p[3]] = 1.0 - 1e-7                             # kept
    with pipesafe.BatchMatrix.from_batch(B) as M:
        res = M.solve(C.b, x0=x0, tol=1e-10, maxit=3000, variant="pbicgsafe", x0_fallback=1)
    for k, A in enumerate(B.systems):
        xk0 = None if k == 0 else x0[p[k]:p[k + 1]]
        R = O.solve(A, x0=xk0, tol=1e-10, maxit=3000, variant="pbicgsafe")
        assert res.iters[k] == R.iters and np.array_equal(res.x[p[k]:p[k + 1]], R.x), k


def _guesses(A):
    """Initial guesses of every kind the scaling meets: close to the solution, a large
    multiple of it, a rough one, exactly zero (no factor) and one with a NaN."""
    g = np.random.default_rng(11)
    xs = np.ones(A.n)
    nan = xs.copy()
    nan[A.n // 3] = np.nan
    return [("near", xs + 1e-3 * g.standard_normal(A.n)), ("multiple", 37.0 * xs),
            ("rough", 50.0 * g.standard_normal(A.n)), ("zero", np.zeros(A.n)), ("nan", nan)]


@pytest.mark.parametrize("precision", [0, 2])
def test_scaled_guess_matches_oracle(precision):
    """x0_fallback = 2: the guess scaled on the device to its least residual, then the
    fallback rule, is the oracle's x0_mode 2 bit for bit (iterations, history, x)."""
    A = W.cd2d(48, 10.0)
    with pipesafe.Matrix.from_csr(A) as M:
        for name, x0 in _guesses(A):
            for v in ("pbicgsafe", "pbicgsafe_rr", "ssbicgsafe2", "pbicgstab"):
                say(f"scaled guess {name} {v} precision {precision}")
                ref = O.solve(A, x0=x0, tol=1e-10, maxit=2000, variant=v, rr_m=20, norm_ref=1,
                              precision=precision, x0_mode=2)
                res = M.solve(A.b, x0=x0, tol=1e-10, maxit=2000, variant=v, rr_m=20, norm_ref=1,
                              precision=precision, x0_fallback=2)
                assert res.status == ref.status and res.iters == ref.iters, (name, v)
                assert np.array_equal(res.hist, ref.hist), (name, v)
                assert np.array_equal(res.x, ref.x), (name, v)


def test_scaled_guess_per_system_in_a_batch():
    B = W.Batch([W.cd2d(40, 10.0), W.cd2d(20, 5.0), W.small_nonsym(300, 4, density=0.02),
                 W.cd2d(33, 30.0)], "scaled")
    C = B.concat()
    p = B.sys_ptr()
    g = np.random.default_rng(5)
    x0 = np.empty(C.n)
    x0[p[0]:p[1]] = 3.0 + 0.01 * g.standard_normal(p[1] - p[0])   # a multiple: scaled back
    x0[p[1]:p[2]] = 0.0                                           # no factor: x0 = 0
    x0[p[2]:p[3]] = 100.0 * g.standard_normal(p[3] - p[2])        # rough
    x0[p[3]:p[4]] = 1.0 - 1e-4                                    # near
    with pipesafe.BatchMatrix.from_batch(B) as M:
        res = M.solve(C.b, x0=x0, tol=1e-10, maxit=3000, variant="pbicgsafe", x0_fallback=2,
                      norm_ref=1)
    for k, A in enumerate(B.systems):
        R = O.solve(A, x0=x0[p[k]:p[k + 1]], tol=1e-10, maxit=3000, variant="pbicgsafe", norm_ref=1,
                    x0_mode=2)
        assert res.iters[k] == R.iters and np.array_equal(res.x[p[k]:p[k + 1]], R.x), k
        assert np.array_equal(res.hist[k, :R.iters + 1], R.hist), k


def test_x0_mode_out_of_range_is_einval():
    A = W.cd2d(8, 1.0)
    with pipesafe.Matrix.from_csr(A) as M:
        with pytest.raises(pipesafe.PipesafeError):
            M.solve(A.b, x0=np.zeros(A.n), tol=1e-8, maxit=10, variant="pbicgsafe", x0_fallback=3)
