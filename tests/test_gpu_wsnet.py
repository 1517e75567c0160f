"""GPU checks of the warm-start network (include/wsnet.h) against its CPU
reference (oracle/wsnet_oracle.py, float64 with the GPU's bfloat16 rounding
points).  Parameters and inputs come from seeded generators, set into both.

Tolerances, elementwise.  Both sides round the same tensors to bfloat16 at the
same points; they differ only in how the products are summed (fp32 on the GPU,
fp64 on the CPU: relative differences of order 2^-24 sqrt(K) before rounding).
A stored activation therefore rounds to the other bfloat16 neighbour only when
its exact value lies that close to a rounding boundary -- a small fraction of
entries, each then off by one bfloat16 step, 2^-7 of its binade.  Such a flip
moves the entries downstream by at most a step of their own scale times the
weights (He-scaled, of norm about 1), and flips in different entries
partly cancel.  So every entry is measured in bfloat16 steps of its size,
floored at the tensor's root mean square (entries near zero have no useful
relative scale):  step(e) = 2^-7 (|ref_e| + rms(ref)).  The bars:
  * forward output: every entry within 2 steps, and at least 99% of the
    entries within half a step (most differ only at the fp32 summation level);
  * every layer's weight and bias gradient, and the head's: every entry within
    1 step (a gradient sums the products of n H W entries, which averages the
    flips: observed at most half a step).
The per-tensor relative 2-norm errors are checked as well.
"""
import sys

import numpy as np
import pytest

from oracle import wsnet_oracle as WO
from paper_2108_10591_amd import wsnet

pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need an MI355X"
    torch.cuda.set_device(0)


def _params(seed, scale=1.0):
    rng = np.random.default_rng(seed)
    p = np.zeros(WO.num_params())
    off = 0
    for i, (ci, co) in enumerate(WO.layer_specs()):
        fan = 9 * (3 if i == 0 else ci)
        w = rng.uniform(-1, 1, (co, 9, ci)) * np.sqrt(6.0 / fan) * scale
        if i == 0:
            w[:, :, 3:] = 0.0
        p[off:off + co * 9 * ci] = w.ravel()
        off += co * 9 * ci
        p[off:off + co] = rng.uniform(-0.1, 0.1, co)
        off += co
    p[off:off + 16] = rng.uniform(-0.5, 0.5, 16)
    p[off + 16] = 0.1
    return p.astype(np.float32)


def _rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30))


def _steps(got, ref):
    """|got - ref| entry by entry, in bfloat16 steps of the entry's size (floored at the
    tensor's root mean square)."""
    ref = np.asarray(ref, dtype=np.float64).ravel()
    got = np.asarray(got, dtype=np.float64).ravel()
    rms = float(np.sqrt(np.mean(ref ** 2)))
    return np.abs(got - ref) / (2.0 ** -7 * (np.abs(ref) + rms))


@pytest.mark.parametrize("H,W,n", [(32, 32, 3), (16, 48, 2), (64, 64, 4)])
def test_forward_matches_reference(H, W, n):
    import torch
    p = _params(1)
    rng = np.random.default_rng(2)
    x = rng.standard_normal((n, H, W, 3)).astype(np.float32)
    with wsnet.WarmStartNet(H, W, 3, 16, seed=0) as net:
        net.set_params(p)
        assert np.array_equal(net.get_params(), p)
        y = net.forward(torch.from_numpy(x).cuda(), scale=2.0).cpu().numpy()
    ref = WO.WsNetOracle().forward(x, p.astype(np.float64))["Y"].numpy()
    err = _rel(y / 2.0, ref)
    st = _steps(y / 2.0, ref)
    say(f"forward {H}x{W} n={n}: relative error {err:.2e}, bfloat16 steps: max {st.max():.3f}, "
        f"99th percentile {np.quantile(st, 0.99):.3f}, within half a step {np.mean(st <= 0.5):.4f}")
    assert st.max() <= 2.0
    assert np.mean(st <= 0.5) >= 0.99
    assert err <= 2e-3


def test_gradients_match_reference():
    import torch
    H = W = 32
    n = 3
    p = _params(4)
    rng = np.random.default_rng(5)
    x = rng.standard_normal((n, H, W, 3)).astype(np.float32)
    t = rng.standard_normal((n, H, W)).astype(np.float32)
    with wsnet.WarmStartNet(H, W, 3, 16, seed=0) as net:
        net.set_params(p)
        loss, g = net.gradients(torch.from_numpy(x).cuda(), torch.from_numpy(t).cuda())
    rloss, rg = WO.WsNetOracle().gradients(x, t, p.astype(np.float64))
    say(f"loss {loss:.6e} vs {rloss:.6e}")
    assert abs(loss - rloss) <= 1e-3 * rloss
    off = 0
    worst = 0.0
    for i, (ci, co) in enumerate(WO.layer_specs()):
        nw = co * 9 * ci
        for name, sl in (("w", slice(off, off + nw)), ("b", slice(off + nw, off + nw + co))):
            e = _rel(g[sl], rg[sl])
            st = _steps(g[sl], rg[sl])
            worst = max(worst, e)
            say(f"layer {i} {name}: relative error {e:.2e}, at most {st.max():.3f} bfloat16 steps")
            assert st.max() <= 1.0, (i, name, float(st.max()))
            assert e <= 1e-2, (i, name, e)
        off += nw + co
    e = _rel(g[off:], rg[off:])
    st = _steps(g[off:], rg[off:])
    say(f"head: relative error {e:.2e}, at most {st.max():.3f} bfloat16 steps")
    assert st.max() <= 1.0
    assert e <= 1e-2
    cos = float(np.dot(g, rg) / (np.linalg.norm(g) * np.linalg.norm(rg)))
    assert cos >= 0.9999, cos


def test_training_lowers_the_loss():
    import torch
    H = W = 32
    rng = np.random.default_rng(7)
    count = 96
    x = rng.standard_normal((count, H, W, 3)).astype(np.float32)
    # a smooth target the network can represent: a blurred, shifted first channel
    t = np.zeros((count, H, W), dtype=np.float32)
    for k in range(count):
        a = x[k, :, :, 0]
        t[k] = 0.25 * (np.roll(a, 1, 0) + np.roll(a, -1, 0) + np.roll(a, 1, 1) + np.roll(a, -1, 1))
    with wsnet.WarmStartNet(H, W, 3, 16, seed=3) as net:
        hist = net.train(torch.from_numpy(x).cuda(), torch.from_numpy(t).cuda(), batch=16, epochs=30,
                         lr=2e-3, seed=1)
    say("loss per epoch: " + " ".join(f"{h:.3e}" for h in hist[::5]))
    assert hist[-1] < 0.3 * hist[0]


def test_invalid_arguments():
    with pytest.raises(wsnet.WsError):
        wsnet.WarmStartNet(30, 32, 3, 16)       # H not a multiple of 8
    with pytest.raises(wsnet.WsError):
        wsnet.WarmStartNet(32, 32, 17, 16)      # too many input channels
