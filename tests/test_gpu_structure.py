"""Structure of an iteration on the GPU, from the library's own launch records
(ps_kernel_stats, ps_kernel_streams), against Table 1 and Algorithm 5:

  * p-BiCGSafe: two sparse products and one reduction phase per iteration in
    every schedule, the reduction phase on the second stream when the overlap
    is on (the one-GPU form of hiding the global reduction behind A s_i,
    Section 3) and on the main stream when it is off; schedule 3 puts the
    reduction phase inside the launches around A s_i (the fold in its
    prologue, the finish at the start of the w pass): three launches on one
    stream;
  * p-BiCGSafe-rr: a replacement step (Algorithm 5) forms q, w, r, l, g, s as
    true products -- six launches: the seventh product of the algorithm, A s_i,
    has no use in that step and is skipped -- with its reduction phase on the
    main stream;
  * ssBiCGSafe2: two products and one reduction phase, all on one stream (its
    inner products need s_i = A r_i);
  * p-BiCGStab: two products and two reduction phases, each on the second
    stream beside one product (schedule 0), or inside the product (schedule 3:
    two passes and two products on one stream).
Counts are per iteration: a solve stopped (tol = 0) at k + 1 minus one stopped
at k."""
import sys

import numpy as np
import pytest

from paper_2108_10591_amd import pipesafe, workloads as W

pytestmark = pytest.mark.gpu
ALL = ["spmv", "dots", "update", "spmv_fused", "other", "dots_finish"]


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need an MI355X"
    torch.cuda.set_device(0)


def iteration(M, A, variant, k, **opt):
    """Launches per class, and of those on the second stream, of iteration k alone."""
    rec = []
    for maxit in (k, k + 1):
        r = M.solve(A.b, tol=0.0, maxit=maxit, variant=variant, profile=ALL, **opt)
        assert r.status == pipesafe.MAXIT and r.iters == maxit, (variant, maxit, r.status_name)
        rec.append(({c: n for c, (_, n) in M.kernel_stats().items()}, M.kernel_streams()))
    (s0, a0), (s1, a1) = rec
    launches = {c: s1[c] - s0[c] for c in s1}
    aux = {c: a1[c] - a0[c] for c in a1}
    print(f"{variant} {opt} iteration {k}: {launches}, second stream {aux}", flush=True)
    sys.stdout.flush()
    return launches, aux


@pytest.mark.parametrize("overlap", [0, 1])
@pytest.mark.parametrize("schedule", [0, 1, 2])
def test_pbicgsafe_two_products_one_phase(schedule, overlap):
    A = W.cd2d(48, 10.0)
    with pipesafe.Matrix.from_csr(A) as M:
        for k in (3, 4):
            n, aux = iteration(M, A, "pbicgsafe", k, schedule=schedule, overlap=overlap)
            assert n["spmv"] + n["spmv_fused"] == 2 and n["spmv"] == 1, n
            assert n["dots_finish"] == 1, n
            assert n["other"] == 0, n
            assert n["update"] == 1, n
            # the reduction (its pass or fold, and the finish) runs beside A s_i
            assert aux["spmv"] == 0 and aux["spmv_fused"] == 0 and aux["update"] == 0, aux
            assert aux["dots_finish"] == overlap and aux["dots"] == overlap * n["dots"], aux
            if schedule == 0:
                assert n["dots"] == 1, n  # the separate multi-inner-product pass
            else:
                assert n["dots"] <= 1, n  # a fold of the partial sums, or none


@pytest.mark.parametrize("overlap", [0, 1])
def test_pbicgsafe_single_stream_schedule(overlap):
    A = W.cd2d(48, 10.0)
    with pipesafe.Matrix.from_csr(A) as M:
        for k in (3, 4):
            n, aux = iteration(M, A, "pbicgsafe", k, schedule=3, overlap=overlap)
            # A s_i (folding the partial sums), the w pass (finishing them), A w_i
            assert n == {"spmv": 1, "spmv_fused": 1, "update": 1, "dots": 0, "dots_finish": 0,
                         "other": 0}, n
            assert sum(aux.values()) == 0, aux


def test_replacement_step_products():
    A = W.cd2d(48, 10.0)
    with pipesafe.Matrix.from_csr(A) as M:
        for sched in (0, 2, 3):
            n, aux = iteration(M, A, "pbicgsafe_rr", 4, rr_m=4, schedule=sched, overlap=1)
            # q = A o, w = A u, l = A t, g = A y, s = A r, and r = b - A x
            assert n["spmv"] == 5 and n["spmv_fused"] == 1, n
            assert n["dots"] == 1 and n["dots_finish"] == 1, n  # its own reduction pass
            assert sum(aux.values()) == 0, aux  # a replacement step is one chain
            std, _ = iteration(M, A, "pbicgsafe_rr", 3, rr_m=4, schedule=sched, overlap=1)
            assert std["spmv"] + std["spmv_fused"] == 2, std
            assert std["dots_finish"] == (0 if sched == 3 else 1), std
            # the step after a replacement forms its inner products in their own pass
            nxt, _ = iteration(M, A, "pbicgsafe_rr", 5, rr_m=4, schedule=sched, overlap=1)
            assert nxt["spmv"] + nxt["spmv_fused"] == 2 and nxt["dots_finish"] == 1, nxt


def test_ssbicgsafe2_one_stream():
    A = W.cd2d(48, 10.0)
    with pipesafe.Matrix.from_csr(A) as M:
        n, aux = iteration(M, A, "ssbicgsafe2", 3, overlap=1)
        assert n["spmv"] == 1 and n["spmv_fused"] == 1, n
        assert n["dots"] == 1 and n["dots_finish"] == 1 and n["update"] == 1, n
        assert sum(aux.values()) == 0, aux


@pytest.mark.parametrize("overlap", [0, 1])
def test_pbicgstab_two_products_two_phases(overlap):
    A = W.cd2d(48, 10.0)
    with pipesafe.Matrix.from_csr(A) as M:
        n, aux = iteration(M, A, "pbicgstab", 3, overlap=overlap, schedule=0)
        assert n["spmv"] == 2 and n["spmv_fused"] == 0, n
        assert n["dots"] == 2 and n["dots_finish"] == 2 and n["update"] == 2, n
        assert aux == {"spmv": 0, "dots": 2 * overlap, "update": 0, "spmv_fused": 0, "other": 0,
                       "dots_finish": 2 * overlap}, aux
        # schedule 3: both phases inside the products, one stream
        for k in (0, 3):
            n, aux = iteration(M, A, "pbicgstab", k, overlap=overlap, schedule=3)
            assert n == {"spmv": 2, "spmv_fused": 0, "update": 2, "dots": 0, "dots_finish": 0,
                         "other": 0}, n
            assert sum(aux.values()) == 0, aux
