"""ps_solve_dev_static, the entry point that allocates nothing: through the C ABI,
two calls in a row on one GPU (the second on a smaller system, so the static
workspace holds the first call's contents when it starts) each give exactly
what ps_solve_dev gives -- iterations, status, residual history and solution,
bit for bit -- for every method and schedule; sizes beyond the workspace are
refused with PS_ETOOBIG."""
import sys

import numpy as np
import pytest

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


CASES = [("pbicgsafe", dict(schedule=2)), ("pbicgsafe", dict(schedule=3)), ("pbicgsafe", dict(schedule=0)),
         ("pbicgsafe", dict(schedule=1, overlap=1)), ("pbicgsafe_rr", dict(rr_m=20)),
         ("ssbicgsafe2", {}), ("pbicgstab", dict(overlap=1, schedule=0)),
         ("pbicgstab", dict(schedule=3)), ("pbicgsafe", dict(schedule=4))]


def _same(a, b):
    import torch
    return (a.iters == b.iters and a.status == b.status and np.array_equal(a.hist, b.hist)
            and torch.equal(a.x, b.x))


@pytest.mark.parametrize("variant,opt", CASES, ids=[f"{v}-{o}" for v, o in CASES])
def test_static_equals_allocating_entry_point(variant, opt):
    import torch
    big, small = W.cd3d(40, 20.0, 7), W.cd2d(40, 10.0)
    for A, tol in ((big, 1e-8), (small, 1e-10)):
        say(f"static solve {variant} {opt} n={A.n}")
        b = torch.from_numpy(A.b).cuda()
        x0 = torch.from_numpy(np.full(A.n, 0.5)).cuda()
        with pipesafe.Matrix.from_csr(A) as M:
            for guess in (None, x0):
                ref = M.solve_dev(b, x0=guess, tol=tol, maxit=3000, variant=variant, **opt)
                xs = torch.empty_like(b)
                got = M.solve_dev_static(b, x0=guess, x=xs, tol=tol, maxit=3000, variant=variant, **opt)
                torch.cuda.synchronize()
                assert _same(got, ref), (A.name, variant, opt, got.iters, ref.iters)


def test_static_workspace_limits():
    import torch
    A = W.cd2d(40, 10.0)
    b = torch.from_numpy(A.b).cuda()
    with pipesafe.Matrix.from_csr(A) as M:
        with pytest.raises(pipesafe.PipesafeError) as e:
            M.solve_dev_static(b, tol=1e-8, maxit=1_000_000, variant="pbicgsafe")
        assert e.value.code == -6
        with pytest.raises(pipesafe.PipesafeError) as e:
            M.solve_dev_static(b, tol=1e-8, maxit=100, variant="pbicgsafe", precision=2)
        assert e.value.code == -1  # no FP32 copy of the values yet
        M.solve_dev(b, tol=1e-8, maxit=100, variant="pbicgsafe", precision=2)
        ref = M.solve_dev(b, tol=1e-10, maxit=1000, variant="pbicgsafe_rr", precision=2, rr_m=30)
        got = M.solve_dev_static(b, tol=1e-10, maxit=1000, variant="pbicgsafe_rr", precision=2,
                                 rr_m=30)
        torch.cuda.synchronize()
        assert _same(got, ref)
