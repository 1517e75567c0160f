"""Pins for the CPU reference of the warm-start network (oracle/wsnet_oracle.py).

The reference's backward pass is written out layer by layer; it is checked
against facts that do not come from it:
  * torch.autograd of the same (unrounded, float64) forward pass;
  * central finite differences of the loss on sampled parameters;
  * a closed form: with every 3x3 weight zero, each layer outputs relu(bias)
    everywhere, so the output is sum_c w_c relu(b9_c) + b_head at every node;
  * the parameter count of the layout documented in include/wsnet.h.
CPU only.
"""
import numpy as np
import torch

from oracle import wsnet_oracle as WO


def _setup(n=2, H=16, W=16, seed=0):
    rng = np.random.default_rng(seed)
    p = rng.standard_normal(WO.num_params()) * 0.1
    # zero weights on the padded input channels (3..15) of the first layer
    ci, co = WO.layer_specs()[0]
    w0 = p[:co * 9 * ci].reshape(co, 9, ci)
    w0[:, :, 3:] = 0.0
    x = rng.standard_normal((n, H, W, 3))
    t = rng.standard_normal((n, H, W))
    return p, x, t


def test_param_count_matches_header_layout():
    c = 16
    expect = (16 * 9 * c + c) + (c * 9 * c + c) + (c * 9 * 2 * c + 2 * c) + (2 * c * 9 * 2 * c + 2 * c) + \
             (2 * c * 9 * 4 * c + 4 * c) + (4 * c * 9 * 4 * c + 4 * c) + (4 * c * 9 * 4 * c + 4 * c) + \
             (8 * c * 9 * 4 * c + 4 * c) + (6 * c * 9 * 2 * c + 2 * c) + (3 * c * 9 * c + c) + c + 1
    assert WO.num_params(c) == expect == 219297


def test_manual_backward_equals_autograd():
    p, x, t = _setup()
    net = WO.WsNetOracle(rounding=False)
    loss, g = net.gradients(x, t, p)
    pt = torch.tensor(p, dtype=torch.float64, requires_grad=True)
    # the forward pass restated here with autograd-tracked parameters
    import torch.nn.functional as F
    off, layers = 0, []
    for ci, co in WO.layer_specs():
        w = pt[off:off + co * 9 * ci].reshape(co, 3, 3, ci).permute(0, 3, 1, 2)
        off += co * 9 * ci
        b = pt[off:off + co]
        off += co
        layers.append((w, b))
    hw, hb = pt[off:off + 16], pt[off + 16]
    X = torch.tensor(x).permute(0, 3, 1, 2)
    X = torch.cat([X, torch.zeros(X.shape[0], 13, X.shape[2], X.shape[3], dtype=torch.float64)], 1)
    conv = lambda z, wb: F.relu(F.conv2d(z, wb[0], wb[1], padding=1))
    up = lambda z: F.interpolate(z, scale_factor=2, mode="nearest")
    A0 = conv(X, layers[0]); S0 = conv(A0, layers[1]); A1 = conv(F.avg_pool2d(S0, 2), layers[2])
    S1 = conv(A1, layers[3]); A2 = conv(F.avg_pool2d(S1, 2), layers[4]); S2 = conv(A2, layers[5])
    BT = conv(F.avg_pool2d(S2, 2), layers[6])
    D2 = conv(torch.cat([up(BT), S2], 1), layers[7])
    D1 = conv(torch.cat([up(D2), S1], 1), layers[8])
    D0 = conv(torch.cat([up(D1), S0], 1), layers[9])
    Y = (D0 * hw.view(1, -1, 1, 1)).sum(1) + hb
    lt = ((Y - torch.tensor(t)) ** 2).mean()
    lt.backward()
    ga = pt.grad.numpy()
    assert abs(float(lt.detach()) - loss) <= 1e-12 * max(1.0, loss)
    assert np.allclose(g, ga, rtol=1e-9, atol=1e-12), float(np.abs(g - ga).max())


def test_finite_differences():
    p, x, t = _setup(n=1, H=8, W=8, seed=3)
    net = WO.WsNetOracle(rounding=False)
    _, g = net.gradients(x, t, p)
    rng = np.random.default_rng(5)
    idx = rng.choice(np.nonzero(np.abs(g) > 1e-6)[0], 12, replace=False)
    for i in idx:
        h = 1e-6 * max(1.0, abs(p[i]))
        pp, pm = p.copy(), p.copy()
        pp[i] += h
        pm[i] -= h
        lp, _ = net.gradients(x, t, pp)
        lm, _ = net.gradients(x, t, pm)
        fd = (lp - lm) / (2 * h)
        assert abs(fd - g[i]) <= 1e-5 * max(1e-3, abs(g[i])), (i, fd, g[i])


def test_zero_weights_closed_form():
    rng = np.random.default_rng(2)
    p = np.zeros(WO.num_params())
    off = 0
    for ci, co in WO.layer_specs():
        off += co * 9 * ci
        p[off:off + co] = rng.uniform(-1.0, 1.0, co)   # biases only
        off += co
    p[off:off + 16] = rng.standard_normal(16)
    p[off + 16] = 0.25
    x = rng.standard_normal((2, 8, 8, 3))
    for rounding in (False, True):
        Y = WO.WsNetOracle(rounding=rounding).forward(x, p)["Y"].numpy()
        b9 = p[off - 16:off]
        act = np.maximum(b9, 0.0)
        if rounding:
            act = torch.tensor(act).to(torch.bfloat16).to(torch.float64).numpy()
        expect = float(np.dot(p[off:off + 16], act) + 0.25)
        assert np.allclose(Y, expect, rtol=1e-15, atol=1e-15)
