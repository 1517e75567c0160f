"""GPU parity of the fused-dot schedules of p-BiCGSafe (option schedule = 1, 2, 3).

A schedule changes where the nine inner products of Algorithm 4 are formed
(per-block partial sums inside pass A and the epilogue of A w_i of the previous
iteration, instead of a pass of their own) and where they are reduced and turned
into the iteration's scalars (a finish kernel of their own, or the prologue of
the A s product and the start of the w pass), not what they are: the partial
sums are triple sums rounded once, as in the separate pass.  So every result
must equal the oracle's p-BiCGSafe bit for bit, like schedule 0.
"""
import os
import sys

import numpy as np
import pytest

import oracle as O
from paper_2108_10591_amd import pipesafe, workloads as W

pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need an MI355X"
    torch.cuda.set_device(0)
    pipesafe.library()


def _long_rows():
    """Rows past a block's LDS budget next to short ones, made diagonally dominant so that
    a few iterations stay finite."""
    rng = np.random.default_rng(3)
    lens = rng.integers(1, 20, 600)
    lens[[5, 100, 101, 599]] = [300, 1500, 9000, 20000]
    S = W.random_csr(600, 3, lengths=lens).to_scipy().tolil()
    S.setdiag(1.5 * np.asarray(abs(S).sum(axis=1)).ravel() + 1.0)
    S = S.tocsr()
    S.sort_indices()
    rowptr = S.indptr.astype(np.int64)
    return W.CSR(n=600, rowptr=rowptr, col=S.indices.astype(np.int32), val=S.data.astype(np.float64),
                 b=W.rhs_ones(rowptr, S.data.astype(np.float64)), name="long_rows_600")


CASES = {
    "cd2d_64": lambda: W.workload("cd2d_64"),
    "rand_band_20k": lambda: W.rand_band(20_000, seed=3, band=500),
    "cd3d_16": lambda: W.cd3d(16, 20.0, seed=1),
    "nonsym_ragged_3001": lambda: W.small_nonsym(3001, 11, density=0.003),
    "long_rows_600": _long_rows,
}


@pytest.mark.parametrize("schedule", [1, 2, 3])
@pytest.mark.parametrize("case", sorted(CASES))
def test_fused_schedule_trajectory_bit_identical_to_oracle(case, schedule):
    """Schedule 1: partial sums in pass A and the A w epilogue; schedule 2: only w_i in a
    pass of its own, every other update and all nine partial sums in the A w epilogue;
    schedule 3: schedule 2 on one stream, the partial sums folded in the A s product's
    prologue and the scalars formed at the start of the w pass."""
    A = CASES[case]()
    for tol, maxit in ((1e-10, 3000), (0.0, 9)):
        say(f"fused schedule {schedule} {case} tol={tol} maxit={maxit}")
        ref = O.solve(A, tol=tol, maxit=maxit, variant="pbicgsafe")
        with pipesafe.Matrix.from_csr(A) as M:
            for overlap in (0, 1):
                res = M.solve(A.b, tol=tol, maxit=maxit, variant="pbicgsafe", schedule=schedule,
                              overlap=overlap)
                assert res.status == ref.status and res.iters == ref.iters, \
                    (case, overlap, res.status, ref.status, res.iters, ref.iters)
                assert np.array_equal(res.hist, ref.hist, equal_nan=True), (case, overlap)
                assert np.array_equal(res.x, ref.x, equal_nan=True), (case, overlap)


def test_fused_schedule_graphs_and_batches_bit_identical():
    """Cached graph replays (several per solve, eager solves in between) and any batch size
    give the same bits as eager one-stream launches; so does schedule 0."""
    for name, A in [("rand_band_100k", W.rand_band(100_000, seed=21, band=3000)),
                    ("cd2d_64", W.workload("cd2d_64"))]:
        say(f"fused dots determinism {name}")
        with pipesafe.Matrix.from_csr(A) as M:
            ref = M.solve(A.b, tol=1e-10, maxit=600, variant="pbicgsafe", graph=0, overlap=0)
            runs = [M.solve(A.b, tol=1e-10, maxit=600, variant="pbicgsafe", schedule=sc, **kw)
                    for sc in (1, 2, 3)
                    for kw in (dict(graph=0, overlap=0), dict(graph=1, batch_iters=4),
                               dict(graph=0, batch_iters=1, overlap=1),
                               dict(graph=1, batch_iters=4), dict(graph=1, batch_iters=7, overlap=0),
                               dict())]
        for k, r in enumerate(runs):
            assert r.iters == ref.iters and r.status == ref.status, (name, k)
            assert np.array_equal(r.x, ref.x) and np.array_equal(r.hist, ref.hist), (name, k)


@pytest.mark.parametrize("case", ["cd2d_64", "nonsym_ragged_3001", "long_rows_600"])
def test_streaming_update_passes_bit_identical_to_oracle(case):
    """PIPESAFE_STREAM=1 forces the streaming (nontemporal) loads and stores of the update
    passes and epilogues (every method), which the library picks by itself only for
    systems far above the last-level cache: a cache hint, so every schedule keeps the
    oracle's bits (odd n: the one-entry tail of each pass)."""
    A = CASES[case]()
    ref = O.solve(A, tol=1e-10, maxit=3000, variant="pbicgsafe")
    old = os.environ.get("PIPESAFE_STREAM")
    os.environ["PIPESAFE_STREAM"] = "1"
    try:
        M = pipesafe.Matrix.from_csr(A)
    finally:
        if old is None:
            del os.environ["PIPESAFE_STREAM"]
        else:
            os.environ["PIPESAFE_STREAM"] = old
    with M:
        assert M.info()["streaming"] == 1
        for kw in (dict(schedule=0), dict(schedule=1), dict(schedule=1, graph=1, batch_iters=4),
                   dict(schedule=0, graph=0, overlap=1), dict(schedule=2),
                   dict(schedule=2, graph=1, batch_iters=3), dict(schedule=3),
                   dict(schedule=3, graph=1, batch_iters=5)):
            say(f"streaming {case} {kw}")
            res = M.solve(A.b, tol=1e-10, maxit=3000, variant="pbicgsafe", **kw)
            assert res.status == ref.status and res.iters == ref.iters, (case, kw)
            assert np.array_equal(res.hist, ref.hist, equal_nan=True), (case, kw)
            assert np.array_equal(res.x, ref.x, equal_nan=True), (case, kw)
        # p-BiCGStab's passes stream p, s, q, y, x and ssBiCGSafe2's epilogue x, z under the
        # same switch
        for v, kws in (("pbicgstab", (dict(schedule=0), dict(schedule=3),
                                      dict(schedule=3, graph=1, batch_iters=3))),
                       ("ssbicgsafe2", (dict(), dict(graph=0)))):
            ref = O.solve(A, tol=1e-10, maxit=3000, variant=v)
            for kw in kws:
                say(f"streaming {case} {v} {kw}")
                res = M.solve(A.b, tol=1e-10, maxit=3000, variant=v, **kw)
                assert res.status == ref.status and res.iters == ref.iters, (case, v, kw)
                assert np.array_equal(res.hist, ref.hist, equal_nan=True), (case, v, kw)
                assert np.array_equal(res.x, ref.x, equal_nan=True), (case, v, kw)
    with pipesafe.Matrix.from_csr(A) as M2:
        assert M2.info()["streaming"] == 0  # small systems: automatic choice is off


@pytest.mark.parametrize("schedule", [1, 2, 3])
@pytest.mark.parametrize("case", ["cd2d_64", "rand_band_20k", "nonsym_ragged_3001"])
def test_fused_schedules_with_residual_replacement(case, schedule):
    """p-BiCGSafe-rr with a fused schedule: a replacement step and the iteration after it
    form their inner products in their own pass, every other iteration from the partial
    sums; every replacement period, graph batch and stream choice gives the oracle's bits."""
    A = CASES[case]()
    with pipesafe.Matrix.from_csr(A) as M:
        for m in (3, 7, 25):
            ref = O.solve(A, tol=1e-10, maxit=3000, variant="pbicgsafe_rr", rr_m=m)
            for kw in (dict(), dict(graph=1, batch_iters=4), dict(graph=0, overlap=1),
                       dict(graph=1, batch_iters=2, overlap=0)):
                say(f"rr fused {case} schedule={schedule} m={m} {kw}")
                res = M.solve(A.b, tol=1e-10, maxit=3000, variant="pbicgsafe_rr", rr_m=m,
                              schedule=schedule, **kw)
                assert res.status == ref.status and res.iters == ref.iters, (m, kw)
                assert np.array_equal(res.hist, ref.hist), (m, kw)
                assert np.array_equal(res.x, ref.x), (m, kw)


def test_fused_schedule_resume_from_oracle_state():
    """The first iteration after a resume forms its inner products in their own pass;
    the following ones take them from the fused partial sums."""
    A = W.workload("cd2d_64")
    k, extra = 6, 4
    st, _ = O.state_at(A, k, variant="pbicgsafe")
    st2, _ = O.state_at(A, k + extra, variant="pbicgsafe")
    with pipesafe.Matrix.from_csr(A) as M:
        for v in ["x", "r", "rs", "s", "y", "t", "p", "u", "z", "w", "l", "g", "q", "o"]:
            M.set_state(v, st.vec(v))
        M.set_state("b", A.b)
        M.set_scalars({k_: st.scal(k_) for k_ in ["alpha", "beta", "zeta", "eta", "f", "rhoref"]})
        for sched in (1, 2, 3):
            for v in ["x", "r", "rs", "s", "y", "t", "p", "u", "z", "w", "l", "g", "q", "o"]:
                M.set_state(v, st.vec(v))
            M.set_scalars({k_: st.scal(k_) for k_ in ["alpha", "beta", "zeta", "eta", "f",
                                                        "rhoref"]})
            res = M.solve(A.b, tol=0.0, maxit=k + extra, variant="pbicgsafe", resume=1,
                          resume_iter=k, schedule=sched, graph=1, batch_iters=2)
            assert res.status == O.MAXIT and res.iters == k + extra
            for v in ["x", "r", "s", "y", "t", "p", "u", "z", "w", "l", "g"]:  # q_i is transient
                assert np.array_equal(M.get_state(v), st2.vec(v)), (sched, v)


@pytest.mark.parametrize("schedule", [1, 2, 3])
def test_fused_schedule_statuses(schedule):
    # A = I converges at i = 1, the first stop test that reads fused partial sums
    for n in (1, 2, 63, 1000):
        E = W.identity(n, seed=n)
        with pipesafe.Matrix.from_csr(E) as M:
            res = M.solve(E.b, tol=1e-12, maxit=50, variant="pbicgsafe", schedule=schedule)
        assert res.status == O.CONVERGED and res.iters == 1 and np.array_equal(res.x, E.b)
    S = W.skew_blocks(64, seed=1)
    with pipesafe.Matrix.from_csr(S) as M:
        res = M.solve(S.b, tol=1e-10, maxit=100, variant="pbicgsafe", schedule=schedule)
    assert res.status == O.BREAKDOWN and res.iters == 0
    B = W.small_nonsym(40, 0)
    b = B.b.copy()
    b[7] = np.nan
    with pipesafe.Matrix.from_csr(B) as M:
        assert M.solve(b, tol=1e-10, maxit=100, variant="pbicgsafe", schedule=schedule).status == \
            O.NONFINITE
        r0 = M.solve(B.b, tol=1e-10, maxit=0, variant="pbicgsafe", schedule=schedule)
        assert r0.status == O.MAXIT and r0.iters == 0
        r3 = M.solve(B.b, tol=1e-30, maxit=3, variant="pbicgsafe", schedule=schedule)
        o3 = O.solve(B, tol=1e-30, maxit=3, variant="pbicgsafe")
        assert r3.iters == 3 and np.array_equal(r3.x, o3.x)
        # the schedules exist for p-BiCGSafe and p-BiCGSafe-rr (and 3 for p-BiCGStab)
        for v in ("ssbicgsafe2", "pbicgstab") if schedule < 3 else ("ssbicgsafe2",):
            with pytest.raises(pipesafe.PipesafeError):
                M.solve(B.b, tol=1e-10, maxit=10, variant=v, schedule=schedule)
        with pytest.raises(pipesafe.PipesafeError):
            M.solve(B.b, tol=1e-10, maxit=10, variant="pbicgsafe", schedule=5)


@pytest.mark.parametrize("case", sorted(CASES))
def test_pbicgstab_single_stream_bit_identical_to_oracle(case):
    """p-BiCGStab, schedule 3: the passes form the partial sums of both reduction phases
    and the products fold and finish them -- the same inner products, so the oracle's
    bits, with graphs or without, and the same bits as the separate passes (0)."""
    A = CASES[case]()
    for tol, maxit in ((1e-10, 3000), (0.0, 9)):
        ref = O.solve(A, tol=tol, maxit=maxit, variant="pbicgstab")
        with pipesafe.Matrix.from_csr(A) as M:
            for kw in (dict(schedule=3), dict(schedule=3, graph=0),
                       dict(schedule=3, graph=1, batch_iters=3), dict(schedule=0, overlap=1)):
                say(f"pbicgstab {case} tol={tol} maxit={maxit} {kw}")
                res = M.solve(A.b, tol=tol, maxit=maxit, variant="pbicgstab", **kw)
                assert res.status == ref.status and res.iters == ref.iters, (case, kw)
                assert np.array_equal(res.hist, ref.hist, equal_nan=True), (case, kw)
                assert np.array_equal(res.x, ref.x, equal_nan=True), (case, kw)


def test_pbicgstab_single_stream_statuses_and_resume():
    # A = I converges at the first stop test (the set-up's); a NaN in b is caught there too
    for n in (1, 63, 1000):
        E = W.identity(n, seed=n)
        with pipesafe.Matrix.from_csr(E) as M:
            res = M.solve(E.b, tol=1e-12, maxit=50, variant="pbicgstab", schedule=3)
            ref = O.solve(E, tol=1e-12, maxit=50, variant="pbicgstab")
        assert res.status == ref.status and res.iters == ref.iters and np.array_equal(res.x, ref.x)
    B = W.small_nonsym(40, 0)
    with pipesafe.Matrix.from_csr(B) as M:
        b = B.b.copy()
        b[7] = np.nan
        assert M.solve(b, tol=1e-10, maxit=100, variant="pbicgstab", schedule=3).status == \
            O.NONFINITE
        for maxit in (0, 1, 3):
            r = M.solve(B.b, tol=1e-30, maxit=maxit, variant="pbicgstab", schedule=3)
            o = O.solve(B, tol=1e-30, maxit=maxit, variant="pbicgstab")
            assert r.status == o.status and r.iters == o.iters and np.array_equal(r.x, o.x)
        for sched in (1, 2):  # p-BiCGStab has the separate passes and schedule 3 only
            with pytest.raises(pipesafe.PipesafeError):
                M.solve(B.b, tol=1e-10, maxit=10, variant="pbicgstab", schedule=sched)
    S = W.skew_blocks(64, seed=1)  # breakdowns: the same status and step as the oracle
    with pipesafe.Matrix.from_csr(S) as M:
        res = M.solve(S.b, tol=1e-10, maxit=100, variant="pbicgstab", schedule=3)
    ref = O.solve(S, tol=1e-10, maxit=100, variant="pbicgstab")
    assert res.status == ref.status and res.iters == ref.iters
    # resume from the oracle's state: every later iteration is the oracle's
    A = W.workload("cd2d_64")
    k, extra = 5, 4
    st, _ = O.state_at(A, k, variant="pbicgstab")
    st2, _ = O.state_at(A, k + extra, variant="pbicgstab")
    names = ["x", "r", "rs", "s", "y", "t", "p", "z", "w", "q", "v"]
    with pipesafe.Matrix.from_csr(A) as M:
        for v in names:
            M.set_state(v, st.vec(v))
        M.set_state("b", A.b)
        M.set_scalars({k_: st.scal(k_) for k_ in ["alpha", "beta", "omega", "f", "rhoref", "rho",
                                                   "gs", "gw", "gz"]}
                      | {"pending": st.scal("pending_breakdown")})
        res = M.solve(A.b, tol=0.0, maxit=k + extra, variant="pbicgstab", resume=1, resume_iter=k,
                      schedule=3, graph=1, batch_iters=2)
        assert res.status == O.MAXIT and res.iters == k + extra
        for v in ["x", "r", "p", "s", "z", "w", "t", "v", "q", "y"]:
            assert np.array_equal(M.get_state(v), st2.vec(v)), v
