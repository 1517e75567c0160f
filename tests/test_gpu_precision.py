"""GPU parity of the mixed-precision solves (ps_options.precision).

Mode 1 (fp32_matrix) makes every product read the matrix values rounded to the
nearest FP32 number; mode 2 (fp32_krylov) keeps the FP64 values for the
residual statements (r_0 = b - A x_0 and the replacement residual of
Algorithm 5) and reads the rounded ones in every other product.  Vectors, inner
products and coefficients stay FP64, and a rounded value is widened exactly,
so the GPU computes the same arithmetic as the oracle at the same precision
(oracle.solve(..., precision=...), which rounds the values itself): every
result must be identical bit for bit, as for the FP64 solves.
"""
import contextlib
import os
import sys

import numpy as np
import pytest

import oracle as O
from paper_2108_10591_amd import pipesafe, workloads as W

pytestmark = pytest.mark.gpu

VARIANTS = ["ssbicgsafe2", "pbicgsafe", "pbicgsafe_rr", "pbicgstab"]
PREC = {"fp32_matrix": 1, "fp32_krylov": 2}


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need an MI355X"
    torch.cuda.set_device(0)
    pipesafe.library()


@contextlib.contextmanager
def device_format(fmt):
    old = os.environ.get("PIPESAFE_FORMAT")
    os.environ["PIPESAFE_FORMAT"] = {"csr": "0", "sell": "1"}[fmt]
    try:
        yield
    finally:
        if old is None:
            os.environ.pop("PIPESAFE_FORMAT", None)
        else:
            os.environ["PIPESAFE_FORMAT"] = old


CASES = {
    "cd2d_64": lambda: W.workload("cd2d_64"),
    "nonsym_ragged_3001": lambda: W.small_nonsym(3001, 11, density=0.003),
    "rand_band_20k": lambda: W.rand_band(20_000, seed=3, band=500),
}


def assert_same(res, ref, what):
    assert res.status == ref.status and res.iters == ref.iters, \
        (what, res.status, ref.status, res.iters, ref.iters)
    assert np.array_equal(res.hist, ref.hist, equal_nan=True), what
    assert np.array_equal(res.x, ref.x, equal_nan=True), what


@pytest.mark.parametrize("fmt", ["csr", "sell"])
@pytest.mark.parametrize("case", sorted(CASES))
def test_mixed_precision_solves_bit_identical_to_oracle(case, fmt):
    A = CASES[case]()
    x0 = np.random.default_rng(5).standard_normal(A.n) * 0.1
    with device_format(fmt), pipesafe.Matrix.from_csr(A) as M:
        assert M.info()["format"] == fmt
        for variant in VARIANTS:
            for pname, prec in PREC.items():
                for kw in (dict(), dict(x0=x0, norm_ref=1)):
                    say(f"precision {pname} {case} {fmt} {variant} {sorted(kw)}")
                    ref = O.solve(A, tol=1e-10, maxit=1500, variant=variant, rr_m=10,
                                  precision=prec, **kw)
                    res = M.solve(A.b, tol=1e-10, maxit=1500, variant=variant, rr_m=10,
                                  precision=pname, **kw)
                    assert_same(res, ref, (case, fmt, variant, pname, sorted(kw)))


def test_fused_schedule_graphs_and_streaming_in_mixed_precision():
    """p-BiCGSafe's fused-dot schedule, graph batches and the streaming passes read the same
    FP32 values; switching precision on one handle keeps each solve exact."""
    A = CASES["rand_band_20k"]()
    old = os.environ.get("PIPESAFE_STREAM")
    os.environ["PIPESAFE_STREAM"] = "1"
    try:
        M = pipesafe.Matrix.from_csr(A)
    finally:
        if old is None:
            os.environ.pop("PIPESAFE_STREAM", None)
        else:
            os.environ["PIPESAFE_STREAM"] = old
    with M:
        for prec in (1, 0, 2, 1):
            ref = O.solve(A, tol=1e-10, maxit=1500, variant="pbicgsafe", precision=prec)
            for kw in (dict(schedule=1), dict(schedule=1, graph=1, batch_iters=3),
                       dict(schedule=0, overlap=1), dict(schedule=2)):
                say(f"precision {prec} fused/graphs {kw}")
                res = M.solve(A.b, tol=1e-10, maxit=1500, variant="pbicgsafe", precision=prec,
                              **kw)
                assert_same(res, ref, (prec, kw))


def test_mixed_precision_batch_bit_identical_to_oracle():
    """A batch in mode 2: each system equals the oracle's solve of it alone."""
    systems = [W.cd2d(24, 5.0), W.small_nonsym(700, 3, density=0.01), W.rand_band(3000, seed=9,
                                                                                band=100)]
    with pipesafe.BatchMatrix.from_batch(W.Batch(systems, "mixed_precision")) as M:
        b = np.concatenate([S.b for S in systems])
        res = M.solve(b, tol=1e-10, maxit=1500, variant="pbicgsafe_rr", rr_m=10,
                      precision="fp32_krylov")
    off = 0
    for k, S in enumerate(systems):
        say(f"batch system {k} {S.name}")
        ref = O.solve(S, tol=1e-10, maxit=1500, variant="pbicgsafe_rr", rr_m=10, precision=2)
        assert res.status[k] == ref.status and res.iters[k] == ref.iters, k
        assert np.array_equal(res.hist[k, : ref.iters + 1], ref.hist), k
        assert np.array_equal(res.x[off:off + S.n], ref.x), k
        off += S.n


def test_fp32_subnormal_and_range():
    """Values that round to FP32 subnormals keep them (as the oracle's rounding does); a value
    beyond the FP32 range makes the mixed modes invalid while FP64 still solves."""
    A = W.small_nonsym(300, 4, density=0.05)
    val = A.val.copy()
    off = np.nonzero(A.col != np.repeat(np.arange(A.n), np.diff(A.rowptr)))[0]
    val[off[:40]] = np.linspace(1e-44, 1e-39, 40)  # subnormal in FP32, normal in FP64
    T = W.CSR(A.n, A.rowptr, A.col, val, A.b, name="subnormal_300")
    assert np.any(val[off[:40]].astype(np.float32) != 0)
    with pipesafe.Matrix.from_csr(T) as M:
        for variant in VARIANTS:
            for pname, prec in PREC.items():
                ref = O.solve(T, tol=1e-10, maxit=500, variant=variant, rr_m=7, precision=prec)
                res = M.solve(T.b, tol=1e-10, maxit=500, variant=variant, rr_m=7,
                              precision=pname)
                assert_same(res, ref, ("subnormal", variant, pname))
    val2 = A.val.copy()
    val2[off[0]] = 1e39  # finite in FP64, beyond FP32
    B = W.CSR(A.n, A.rowptr, A.col, val2, A.b, name="f32_overflow_300")
    with pipesafe.Matrix.from_csr(B) as M:
        for pname in list(PREC) + ["fp32_vectors"]:
            with pytest.raises(pipesafe.PipesafeError):
                M.solve(B.b, tol=1e-10, maxit=50, variant="pbicgsafe", precision=pname)
        assert M.solve(B.b, tol=1e-10, maxit=50, variant="pbicgsafe").iters >= 0
    with pipesafe.Matrix.from_csr(A) as M:
        for bad in (4, -1):
            with pytest.raises(pipesafe.PipesafeError):
                M.solve(A.b, tol=1e-10, maxit=50, variant="pbicgsafe", precision=bad)


@pytest.mark.parametrize("gather_sort", [1, 0])
def test_fp32_values_with_the_gather_ordered_csr_layout(gather_sort):
    """FP32 values in the CSR layout whose row blocks store their entries in column order
    (the 1M-row band's layout): a +-5000 band of 100k rows, both layouts forced, every
    precision mode against the oracle bit for bit (FP64 values in the same layout too)."""
    A = W.rand_band(100_000, seed=21, band=5000)
    lay = pipesafe.layout(format="csr", gather_sort=gather_sort, spmv_shape=2)
    with pipesafe.Matrix.from_csr(A, layout=lay) as M:
        info = M.info()
        assert info["format"] == "csr" and info["gather_sort"] == gather_sort
        assert info["index_bits"] == 16
        for variant, prec, m in (("pbicgsafe", 1, 100), ("pbicgsafe_rr", 2, 25), ("pbicgsafe", 0, 100)):
            for sched in (0, 2):
                say(f"gather order {gather_sort}: {variant} precision {prec} schedule {sched}")
                ref = O.solve(A, tol=1e-10, maxit=3000, variant=variant, rr_m=m, precision=prec)
                res = M.solve(A.b, tol=1e-10, maxit=3000, variant=variant, rr_m=m, precision=prec,
                              schedule=sched)
                assert_same(res, ref, (variant, prec, sched))


@pytest.mark.parametrize("fmt", ["csr", "sell"])
@pytest.mark.parametrize("case", sorted(CASES))
def test_fp32_vectors_bit_identical_to_oracle(case, fmt):
    """Precision 3: the Krylov products read FP32 values and p, u, z are held as FP32
    numbers (rounded when formed, widened when read), in every schedule of p-BiCGSafe and
    in p-BiCGSafe-rr's replacement steps; the oracle's precision 3 bit for bit."""
    A = CASES[case]()
    x0 = np.random.default_rng(6).standard_normal(A.n) * 0.1
    with device_format(fmt), pipesafe.Matrix.from_csr(A) as M:
        for variant in ("pbicgsafe", "pbicgsafe_rr"):
            for sched in (0, 1, 2):
                for kw in (dict(), dict(x0=x0, norm_ref=1)):
                    say(f"fp32 vectors {case} {fmt} {variant} schedule {sched} {sorted(kw)}")
                    ref = O.solve(A, tol=1e-10, maxit=1500, variant=variant, rr_m=10, precision=3,
                                  **kw)
                    res = M.solve(A.b, tol=1e-10, maxit=1500, variant=variant, rr_m=10, precision=3,
                                  schedule=sched, **kw)
                    assert_same(res, ref, (case, fmt, variant, sched, sorted(kw)))
        for variant in ("ssbicgsafe2", "pbicgstab"):
            with pytest.raises(pipesafe.PipesafeError):
                M.solve(A.b, tol=1e-10, maxit=10, variant=variant, precision=3)


def test_fp32_vectors_state_round_trip():
    """The state interface is FP64: the oracle's precision-3 state at iteration k, loaded
    into the GPU and advanced one iteration (a replacement step among them), equals the
    oracle's state at k + 1 in every vector; p, u, z read back are FP32 numbers."""
    A = W.cd2d(32, 10.0)
    with pipesafe.Matrix.from_csr(A) as M:
        for k in (3, 4):
            st, _ = O.state_at(A, k, variant="pbicgsafe_rr", rr_m=4, precision=3)
            st1, _ = O.state_at(A, k + 1, variant="pbicgsafe_rr", rr_m=4, precision=3)
            for v in ["x", "r", "rs", "s", "y", "t", "p", "u", "z", "w", "l", "g", "q", "o"]:
                M.set_state(v, st.vec(v))
            M.set_state("b", A.b)
            M.set_scalars({n: st.scal(n) for n in ["alpha", "beta", "zeta", "eta", "f", "rhoref"]})
            res = M.solve(A.b, tol=0.0, maxit=k + 1, variant="pbicgsafe_rr", rr_m=4, precision=3,
                          resume=1, resume_iter=k, schedule=0)
            assert res.status == O.MAXIT and res.iters == k + 1
            for v in ["x", "r", "s", "y", "t", "p", "u", "z", "w", "l", "g"]:
                got = M.get_state(v)
                assert np.array_equal(got, st1.vec(v)), (k, v)
            for v in ("p", "u", "z"):
                got = M.get_state(v)
                assert np.array_equal(got.astype(np.float32).astype(np.float64), got), v
        # a later FP64 solve from the same handle is unaffected by the FP32 storage
        ref = O.solve(A, tol=1e-10, maxit=500, variant="pbicgsafe")
        res = M.solve(A.b, tol=1e-10, maxit=500, variant="pbicgsafe")
        assert_same(res, ref, "fp64 after fp32 vectors")
