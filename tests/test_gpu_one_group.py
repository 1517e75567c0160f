"""GPU parity of schedule 4: the whole p-BiCGSafe solve in one workgroup.

For small systems on the sliced layout, one workgroup runs every iteration of
Algorithm 4 -- the reduction phase from the nine inner products, A s_i, w_i,
A w_i and every other update -- with barriers between the phases that gather.
The row sums are the sliced product's (slots in order, compensated, rounded
once), the updates the separate passes' expressions and the inner products
exact sums rounded once, so every result equals the oracle's p-BiCGSafe bit
for bit, like the multi-kernel schedules.
"""
import sys

import numpy as np
import pytest

import oracle as O
from paper_2108_10591_amd import pipesafe, workloads as W

pytestmark = pytest.mark.gpu

SELL16 = pipesafe.layout("sell", 1, -1, 16)
SELL32 = pipesafe.layout("sell", 1, -1, 32)


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need an MI355X"
    torch.cuda.set_device(0)
    pipesafe.library()


CASES = {
    "cd2d_64": lambda: W.workload("cd2d_64"),
    "cd2d_37": lambda: W.cd2d(37),  # 1369 rows: a ragged last slice
    "cd3d_16": lambda: W.cd3d(16, 20.0, seed=1),
    "nonsym_ragged_3001": lambda: W.small_nonsym(3001, 11, density=0.003),
    "rand_band_20k": lambda: W.rand_band(20_000, seed=3, band=500),
}


@pytest.mark.parametrize("lay", ["sell16", "sell32"])
@pytest.mark.parametrize("case", sorted(CASES))
def test_one_group_trajectory_bit_identical_to_oracle(case, lay):
    A = CASES[case]()
    L = SELL16 if lay == "sell16" else SELL32
    with pipesafe.Matrix.from_csr(A, L) as M:
        if lay == "sell16" and M.info()["index_bits"] != 16:
            pytest.skip("columns too far from the diagonal for 16-bit offsets")
        for tol, maxit in ((1e-10, 3000), (0.0, 9), (0.0, 1)):
            say(f"one group {case} {lay} tol={tol} maxit={maxit}")
            ref = O.solve(A, tol=tol, maxit=maxit, variant="pbicgsafe")
            res = M.solve(A.b, tol=tol, maxit=maxit, variant="pbicgsafe", schedule=4)
            assert res.status == ref.status and res.iters == ref.iters, \
                (case, res.status, ref.status, res.iters, ref.iters)
            assert np.array_equal(res.hist, ref.hist, equal_nan=True), case
            assert np.array_equal(res.x, ref.x, equal_nan=True), case
            # and the same bits as the multi-kernel schedule, twice in a row
            r3 = M.solve(A.b, tol=tol, maxit=maxit, variant="pbicgsafe", schedule=3)
            r4 = M.solve(A.b, tol=tol, maxit=maxit, variant="pbicgsafe", schedule=4)
            assert np.array_equal(r3.x, r4.x) and np.array_equal(r3.hist, r4.hist), case


def test_one_group_statuses_and_options():
    # A = I converges at i = 1
    for n in (1, 2, 63, 1000):
        E = W.identity(n, seed=n)
        with pipesafe.Matrix.from_csr(E, SELL32) as M:
            res = M.solve(E.b, tol=1e-12, maxit=50, variant="pbicgsafe", schedule=4)
        assert res.status == O.CONVERGED and res.iters == 1 and np.array_equal(res.x, E.b)
    S = W.skew_blocks(64, seed=1)
    with pipesafe.Matrix.from_csr(S, SELL32) as M:
        res = M.solve(S.b, tol=1e-10, maxit=100, variant="pbicgsafe", schedule=4)
    ref = O.solve(S, tol=1e-10, maxit=100, variant="pbicgsafe")
    assert res.status == O.BREAKDOWN == ref.status and res.iters == ref.iters == 0
    B = W.small_nonsym(40, 0)
    with pipesafe.Matrix.from_csr(B, SELL32) as M:
        b = B.b.copy()
        b[7] = np.nan
        assert M.solve(b, tol=1e-10, maxit=100, variant="pbicgsafe", schedule=4).status == \
            O.NONFINITE
        r0 = M.solve(B.b, tol=1e-10, maxit=0, variant="pbicgsafe", schedule=4)
        assert r0.status == O.MAXIT and r0.iters == 0
        x1, x2 = np.linspace(-1.0, 1.0, B.n), np.full(B.n, 0.5)
        for kw, okw in ((dict(x0=x1), dict(x0=x1)), (dict(norm_ref=1), dict(norm_ref=1)),
                        (dict(x0=x2, x0_fallback=2), dict(x0=x2, x0_mode=2))):
            ref = O.solve(B, tol=1e-12, maxit=200, variant="pbicgsafe", **okw)
            res = M.solve(B.b, tol=1e-12, maxit=200, variant="pbicgsafe", schedule=4, **kw)
            assert res.status == ref.status and res.iters == ref.iters, kw
            assert np.array_equal(res.x, ref.x) and np.array_equal(res.hist, ref.hist), kw
        # schedule 4 is p-BiCGSafe in FP64 from x_0 only
        for kw in (dict(variant="pbicgsafe_rr"), dict(variant="pbicgstab"),
                   dict(variant="ssbicgsafe2"), dict(variant="pbicgsafe", precision=1),
                   dict(variant="pbicgsafe", schedule=5)):
            kw = dict(dict(schedule=4), **kw)
            with pytest.raises(pipesafe.PipesafeError):
                M.solve(B.b, tol=1e-10, maxit=10, **kw)
    with pipesafe.Matrix.from_csr(B, pipesafe.layout("csr")) as M:  # the sliced layout only
        with pytest.raises(pipesafe.PipesafeError):
            M.solve(B.b, tol=1e-10, maxit=10, variant="pbicgsafe", schedule=4)


def test_one_group_batch_equals_each_system_alone():
    """Batches: one workgroup per system, each over its own padded rows, scalar and
    control blocks and history; systems that stop early (identity, breakdown, NaN) leave
    the others running."""
    import test_gpu_batch as TB
    B, C, b = TB.mixed_batch()
    for tol, maxit in ((1e-10, 2000), (0.0, 7)):
        refs = TB.oracle_each(B, b, tol, maxit, "pbicgsafe")
        for L in (SELL16, SELL32):
            with pipesafe.BatchMatrix.from_batch(B, L) as M:
                say(f"one group batch tol={tol} index_bits={M.info()['index_bits']}")
                for _ in range(2):
                    res = M.solve(b, tol=tol, maxit=maxit, variant="pbicgsafe", schedule=4)
                    TB.check_same(res, refs, B, ("one group", tol))


def test_one_group_automatic_choice():
    """The automatic schedule runs sliced p-BiCGSafe systems of at most 1024 rows in one
    workgroup (ps_info.auto_schedule = 4); p-BiCGSafe-rr and larger systems take 3."""
    for N, want in ((16, 4), (32, 4), (33, 3)):
        A = W.cd2d(N)
        with pipesafe.Matrix.from_csr(A, SELL16) as M:
            assert M.info()["auto_schedule"] == want, N
            for v in ("pbicgsafe", "pbicgsafe_rr"):
                say(f"automatic schedule cd2d_{N} {v}")
                ref = O.solve(A, tol=1e-10, maxit=2000, variant=v, rr_m=13)
                res = M.solve(A.b, tol=1e-10, maxit=2000, variant=v, rr_m=13)
                assert res.status == ref.status and res.iters == ref.iters, (N, v)
                assert np.array_equal(res.x, ref.x) and np.array_equal(res.hist, ref.hist), (N, v)


@pytest.mark.parametrize("case", ["empty_and_single", "long_rows", "one_row", "single_empty_row",
                                  "unsorted_dups"])
def test_one_group_edge_matrices(case):
    """Empty rows, rows of up to 20000 entries beside short ones (a slice as wide as its
    longest row), one-row systems, unsorted and duplicated entries: whatever the oracle
    does in 40 iterations (converge, break down, overflow), the same bits."""
    import test_gpu_parity as TP
    A = TP._spmv_matrix(case)
    ref = O.solve(A, tol=1e-10, maxit=40, variant="pbicgsafe")
    with pipesafe.Matrix.from_csr(A, SELL32) as M:
        assert M.info()["format"] == "sell"
        say(f"one group edge case {case}")
        res = M.solve(A.b, tol=1e-10, maxit=40, variant="pbicgsafe", schedule=4)
    assert res.status == ref.status and res.iters == ref.iters, (case, res.status, ref.status)
    assert np.array_equal(res.hist, ref.hist, equal_nan=True), case
    assert np.array_equal(res.x, ref.x, equal_nan=True), case


def test_one_group_automatic_for_batches_of_small_systems():
    """Batches whose systems have at most 1600 rows (sliced layout) run one workgroup per
    system by default; p-BiCGSafe-rr and larger systems keep the shared launches (2)."""
    small = W.cd2d_batch(nsys=48, seed=7, nmin=6, nmax=40)
    large = W.cd2d_batch(nsys=6, seed=7, nmin=36, nmax=48)
    for B, want in ((small, 4), (large, 2)):
        C = B.concat()
        with pipesafe.BatchMatrix.from_batch(B, SELL16) as M:
            assert M.info()["auto_schedule"] == want, B.name
            for v in ("pbicgsafe", "pbicgsafe_rr"):
                say(f"automatic batch schedule {B.name} max side {max(int(round(A.n ** 0.5)) for A in B.systems)} {v}")
                import test_gpu_batch as TB
                refs = TB.oracle_each(B, C.b, 1e-10, 2000, v, rr_m=11)
                res = M.solve(C.b, tol=1e-10, maxit=2000, variant=v, rr_m=11)
                TB.check_same(res, refs, B, (B.name, v))


def test_one_group_many_tiny_systems():
    """600 systems of 36..144 rows: workgroups of 128 threads (so that more systems are
    resident at once), some threads owning two rows; the oracle's bits for every system,
    and the shared launches' (schedule 2)."""
    import test_gpu_batch as TB
    B = W.cd2d_batch(nsys=600, seed=11, nmin=6, nmax=12)
    C = B.concat()
    refs = TB.oracle_each(B, C.b, 1e-10, 500, "pbicgsafe")
    with pipesafe.BatchMatrix.from_batch(B, SELL16) as M:
        assert M.info()["auto_schedule"] == 4
        say("one group: 600 tiny systems")
        res = M.solve(C.b, tol=1e-10, maxit=500, variant="pbicgsafe")
        TB.check_same(res, refs, B, "600 tiny systems")
        r2 = M.solve(C.b, tol=1e-10, maxit=500, variant="pbicgsafe", schedule=2)
        assert np.array_equal(r2.x, res.x) and np.array_equal(r2.iters, res.iters)


@pytest.mark.parametrize("case", ["cd2d_8", "cd2d_16", "cd2d_22", "cd3d_6", "cd3d_8",
                                  "band_300", "nonsym_500"])
def test_one_group_register_resident(case):
    """Systems of at most 512 rows whose slices hold at most 8 entries per row keep every
    vector entry of their row, and the row's entries, in registers (s and w in LDS): the
    oracle's bits, and schedule 3's, with 16- and 32-bit columns."""
    A = {"cd2d_8": lambda: W.cd2d(8), "cd2d_16": lambda: W.cd2d(16), "cd2d_22": lambda: W.cd2d(22),
         "cd3d_6": lambda: W.cd3d(6, 20.0, seed=2), "cd3d_8": lambda: W.cd3d(8, 20.0, seed=3),
         "band_300": lambda: W.rand_band(300, seed=4, lmin=3, lmax=8, band=40),
         "nonsym_500": lambda: W.random_csr(500, 6, lengths=np.random.default_rng(6).integers(
             1, 8, 500))}[case]()
    if case == "nonsym_500":  # diagonally dominant, so that the solve converges
        S = A.to_scipy().tolil()
        S.setdiag(1.5 * np.asarray(abs(S).sum(axis=1)).ravel() + 1.0)
        S = S.tocsr()
        S.sort_indices()
        rp = S.indptr.astype(np.int64)
        A = W.CSR(n=500, rowptr=rp, col=S.indices.astype(np.int32), val=S.data.astype(np.float64),
                  b=W.rhs_ones(rp, S.data.astype(np.float64)), name="nonsym_500")
    for L in (SELL16, SELL32):
        with pipesafe.Matrix.from_csr(A, L) as M:
            for tol, maxit in ((1e-10, 2000), (0.0, 7)):
                say(f"register-resident {case} tol={tol} index_bits={M.info()['index_bits']}")
                ref = O.solve(A, tol=tol, maxit=maxit, variant="pbicgsafe")
                res = M.solve(A.b, tol=tol, maxit=maxit, variant="pbicgsafe", schedule=4)
                assert res.status == ref.status and res.iters == ref.iters, case
                assert np.array_equal(res.hist, ref.hist) and np.array_equal(res.x, ref.x), case
                r3 = M.solve(A.b, tol=tol, maxit=maxit, variant="pbicgsafe", schedule=3)
                assert np.array_equal(r3.x, res.x), case
            # the state the solve leaves is the multi-kernel solve's too
            M.solve(A.b, tol=0.0, maxit=5, variant="pbicgsafe", schedule=4)
            st4 = {v: M.get_state(v) for v in ("x", "r", "s", "y", "t", "p", "u", "z", "w", "l", "g")}
            M.solve(A.b, tol=0.0, maxit=5, variant="pbicgsafe", schedule=3)
            for v, a in st4.items():
                assert np.array_equal(a, M.get_state(v)), (case, v)


def test_one_group_register_resident_batch():
    """A batch of 200 systems of 36..256 rows (one row per thread in 256-thread
    workgroups), some of them stopping early: each system's bits as the oracle's."""
    import test_gpu_batch as TB
    B = W.cd2d_batch(nsys=200, seed=13, nmin=6, nmax=16)
    C = B.concat()
    b = C.b.copy()
    p = B.sys_ptr()
    b[p[3]:p[4]] = 0.0  # converges at i = 0
    for tol, maxit in ((1e-10, 500), (0.0, 6)):
        refs = TB.oracle_each(B, b, tol, maxit, "pbicgsafe")
        with pipesafe.BatchMatrix.from_batch(B, SELL16) as M:
            say(f"register-resident batch tol={tol}")
            res = M.solve(b, tol=tol, maxit=maxit, variant="pbicgsafe", schedule=4)
            TB.check_same(res, refs, B, ("register-resident batch", tol))


@pytest.mark.parametrize("case", ["cd2d_24", "cd2d_31", "cd3d_10"])
def test_one_group_register_resident_two_rows(case):
    """513..1024 rows: two rows per thread of a 512-thread workgroup, in registers."""
    A = {"cd2d_24": lambda: W.cd2d(24), "cd2d_31": lambda: W.cd2d(31),
         "cd3d_10": lambda: W.cd3d(10, 20.0, seed=4)}[case]()
    for L in (SELL16, SELL32):
        with pipesafe.Matrix.from_csr(A, L) as M:
            for tol, maxit in ((1e-10, 2000), (0.0, 5)):
                say(f"register-resident, two rows per thread: {case} tol={tol}")
                ref = O.solve(A, tol=tol, maxit=maxit, variant="pbicgsafe")
                res = M.solve(A.b, tol=tol, maxit=maxit, variant="pbicgsafe", schedule=4)
                assert res.status == ref.status and res.iters == ref.iters, case
                assert np.array_equal(res.hist, ref.hist) and np.array_equal(res.x, ref.x), case
            st4 = {v: M.get_state(v) for v in ("x", "r", "s", "y", "t", "p", "u", "z", "w", "l", "g")}
            M.solve(A.b, tol=0.0, maxit=5, variant="pbicgsafe", schedule=3)
            for v, a in st4.items():
                assert np.array_equal(a, M.get_state(v)), (case, v)
