"""GPU checks of the explicit layouts and the autotuner (ps_create_ex, ps_autotune_layout,
ps_tune_options).  Every layout, launch shape and schedule computes the same iterates, so
whatever the tuner picks must reproduce the oracle bit for bit."""
import sys

import numpy as np
import pytest
import torch

import oracle as O
from paper_2108_10591_amd import pipesafe, workloads as W

pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    assert torch.cuda.is_available(), "GPU tests need an MI355X"
    torch.cuda.set_device(0)
    pipesafe.library()


def same(res, ref, what):
    assert res.status == ref.status and res.iters == ref.iters, (what, res.iters, ref.iters)
    assert np.array_equal(res.hist, ref.hist) and np.array_equal(res.x, ref.x), what


@pytest.mark.parametrize("lay", [dict(format="sell", sell_rows_per_lane=2, index_bits=32),
                                 dict(format="sell", sell_rows_per_lane=1, index_bits=16),
                                 dict(format="csr", spmv_shape=0), dict(format="csr", spmv_shape=4)])
def test_explicit_layouts_reproduce_oracle(lay):
    A = W.cd3d(16, 20.0, seed=1)
    ref = O.solve(A, tol=1e-10, maxit=2000, variant="pbicgsafe")
    with pipesafe.Matrix.from_csr(A, pipesafe.layout(**lay)) as M:
        info = M.info()
        assert info["format"] == lay["format"]
        if lay["format"] == "sell":
            assert info["index_bits"] == lay["index_bits"]
        else:
            assert info["spmv_shape"] == lay["spmv_shape"]
        same(M.solve(A.b, tol=1e-10, maxit=2000, variant="pbicgsafe"), ref, lay)


@pytest.mark.parametrize("name", ["cd3d_16", "rand_band_20k", "nonsym_ragged_3001"])
def test_autotuned_layout_reproduces_oracle(name):
    A = {"cd3d_16": lambda: W.cd3d(16, 20.0, seed=1),
         "rand_band_20k": lambda: W.rand_band(20_000, seed=3, band=500),
         "nonsym_ragged_3001": lambda: W.small_nonsym(3001, 11, density=0.003)}[name]()
    M, rows = pipesafe.Matrix.autotuned(A, reps=10)
    with M:
        say(f"autotune {name}: " + ", ".join(f"{r.get('format')}/{r.get('sell_rows_per_lane')}/"
                                             f"{r.get('spmv_shape')}/{r.get('index_bits')}:"
                                             f"{r['us']:.1f}" for r in rows))
        assert len(rows) >= 5 and sum(r["best"] for r in rows) == 1
        best = next(r for r in rows if r["best"])
        assert best["us"] == min(r["us"] for r in rows) and best["us"] > 0
        info = M.info()
        assert info["format"] == best["format"]
        if best["format"] == "csr":
            assert info["spmv_shape"] == best["spmv_shape"]
        else:
            assert info["index_bits"] == best["index_bits"]
        for variant in ("pbicgsafe", "pbicgsafe_rr"):
            ref = O.solve(A, tol=1e-10, maxit=2000, variant=variant, rr_m=20)
            same(M.solve(A.b, tol=1e-10, maxit=2000, variant=variant, rr_m=20), ref, (name, variant))


def test_tuned_options_reproduce_oracle():
    A = W.rand_band(20_000, seed=3, band=500)
    b = torch.from_numpy(A.b).cuda()
    with pipesafe.Matrix.from_csr(A) as M:
        # schedules 0-2: overlap x streaming x graph batch; 3: streaming x graph batch
        # (p-BiCGStab: graph batch); 4 is for the sliced layout only
        for variant, ncand in (("pbicgsafe", 3 * 2 * 2 * 3 + 2 * 3), ("ssbicgsafe2", 3),
                               ("pbicgstab", 2 * 3 + 3)):
            opts, rows = M.tune_options(b, variant=variant, iters=20)
            say(f"tune_options {variant}: {opts}")
            assert len(rows) == ncand and sum(r["best"] for r in rows) == 1
            best = next(r for r in rows if r["best"])
            assert best["us"] == min(r["us"] for r in rows)
            assert opts["overlap"] == best["overlap"] and opts["batch_iters"] == best["batch_iters"]
            ref = O.solve(A, tol=1e-10, maxit=2000, variant=variant)
            same(M.solve(A.b, tol=1e-10, maxit=2000, variant=variant, **opts), ref, variant)


def test_autotuned_batch_reproduces_oracle():
    systems = [W.cd2d(20, 4.0), W.cd2d(33, 20.0), W.small_nonsym(900, 2, density=0.01)]
    B = W.Batch(systems, "tune_batch")
    M, rows = pipesafe.BatchMatrix.autotuned(B, reps=5)
    with M:
        assert sum(r["best"] for r in rows) == 1
        b = np.concatenate([S.b for S in systems])
        bd = torch.from_numpy(b).cuda()
        opts, orows = M.tune_options(bd, variant="pbicgsafe", iters=10)
        # schedules 0-2 x overlap x streaming x graph batch, and one run of schedule 4 on
        # the sliced layout with one row per lane (3 is for one system)
        n4 = sum(r["schedule"] == 4 for r in orows)
        assert len(orows) == 3 * 2 * 2 * 3 + n4 and n4 <= 1
        assert n4 == 0 or M.info()["format"] == "sell"
        res = M.solve(b, tol=1e-10, maxit=2000, variant="pbicgsafe", **opts)
    off = 0
    for k, S in enumerate(systems):
        ref = O.solve(S, tol=1e-10, maxit=2000, variant="pbicgsafe")
        assert res.iters[k] == ref.iters and res.status[k] == ref.status, k
        assert np.array_equal(res.x[off:off + S.n], ref.x), k
        off += S.n


def test_tuned_options_on_a_small_sliced_system():
    """A 400-row stencil: the tuner also times the single-stream schedule (3) and the
    one-workgroup solve (4, one run: it has no stream, streaming or graph choice), and
    whatever it picks reproduces the oracle bit for bit."""
    A = W.cd2d(20, 10.0)
    b = torch.from_numpy(A.b).cuda()
    with pipesafe.Matrix.from_csr(A) as M:
        assert M.info()["format"] == "sell"
        opts, rows = M.tune_options(b, variant="pbicgsafe", iters=20)
        say(f"tune_options small sliced: {opts}")
        assert sum(r["schedule"] == 4 for r in rows) == 1
        assert sum(r["schedule"] == 3 for r in rows) == 2 * 3  # streaming x graph batch
        assert len(rows) == 3 * 2 * 2 * 3 + 2 * 3 + 1 and sum(r["best"] for r in rows) == 1
        ref = O.solve(A, tol=1e-10, maxit=2000, variant="pbicgsafe")
        same(M.solve(A.b, tol=1e-10, maxit=2000, variant="pbicgsafe", **opts), ref, "small")
