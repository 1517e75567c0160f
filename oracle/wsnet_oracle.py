"""CPU reference of the warm-start U-Net (include/wsnet.h), in float64 PyTorch.

TEST INFRASTRUCTURE ONLY: used by the test suite to check the GPU network's
forward pass and gradients; the product path never imports it.  It shares no
code with the GPU library: the layer formulas are written here with torch's
plain CPU convolution, pooling and interpolation routines.

With rounding=True every tensor that the GPU stores in bfloat16 is rounded to
bfloat16 (nearest even) at the same point: the network input, each 3x3
convolution's output (after bias and ReLU), each pooled map, and in the
backward pass the head's input gradient, each convolution's input gradient,
each upsampling gradient and each pooled-gradient sum.  3x3 weights are used
rounded to bfloat16; biases, the head and the loss are unrounded.  With
rounding=False the same network runs in plain float64.

The backward pass is written out layer by layer (torch.nn.grad's convolution
gradients, pooling as 0.25-scaled nearest upsampling and back); its pins are
torch.autograd on the unrounded forward pass and finite differences.
"""
from __future__ import annotations

import numpy as np
import torch
import torch.nn.functional as F

D = torch.float64


def _bf(x, on):
    return x.to(torch.bfloat16).to(D) if on else x


def layer_specs(c: int = 16, cin_pad: int = 16):
    """(Ci, Co) of the ten 3x3 layers, in parameter order."""
    return [(cin_pad, c), (c, c), (c, 2 * c), (2 * c, 2 * c), (2 * c, 4 * c), (4 * c, 4 * c),
            (4 * c, 4 * c), (8 * c, 4 * c), (6 * c, 2 * c), (3 * c, c)]


def num_params(c: int = 16) -> int:
    return sum(co * 9 * ci + co for ci, co in layer_specs(c)) + c + 1


def unpack(params, c: int = 16):
    """Flat fp32 vector -> [(weight [co, ci, 3, 3], bias [co]) x 10], head weights [c], head bias."""
    p = torch.as_tensor(np.asarray(params, dtype=np.float64))
    out, off = [], 0
    for ci, co in layer_specs(c):
        w = p[off:off + co * 9 * ci].reshape(co, 3, 3, ci).permute(0, 3, 1, 2).contiguous()
        off += co * 9 * ci
        b = p[off:off + co]
        off += co
        out.append((w, b))
    hw = p[off:off + c]
    hb = p[off + c]
    return out, hw, hb


def pack_grads(layers, hw, hb) -> np.ndarray:
    parts = []
    for w, b in layers:
        parts.append(w.permute(0, 2, 3, 1).reshape(-1))  # [co][tap][ci]
        parts.append(b.reshape(-1))
    parts += [hw.reshape(-1), hb.reshape(1)]
    return torch.cat(parts).numpy()


class WsNetOracle:
    def __init__(self, cin: int = 3, c: int = 16, rounding: bool = True):
        self.cin, self.c, self.r = cin, c, rounding

    # ---------------------------------------------------------------- pieces
    def _input(self, x_nhwc):
        x = torch.as_tensor(np.asarray(x_nhwc, dtype=np.float64))
        x = x.permute(0, 3, 1, 2)
        pad = torch.zeros((x.shape[0], 16 - x.shape[1], x.shape[2], x.shape[3]), dtype=D)
        return _bf(torch.cat([x, pad], 1), self.r)

    def _conv(self, x, w, b):
        return _bf(F.relu(F.conv2d(x, _bf(w, self.r), b, padding=1)), self.r)

    def _pool(self, x):
        return _bf(F.avg_pool2d(x, 2), self.r)

    @staticmethod
    def _up(x):
        return F.interpolate(x, scale_factor=2, mode="nearest")

    # ---------------------------------------------------------------- forward
    def forward(self, x_nhwc, params):
        L, hw, hb = unpack(params, self.c)
        a = {}
        a["X"] = self._input(x_nhwc)
        a["A0"] = self._conv(a["X"], *L[0])
        a["S0"] = self._conv(a["A0"], *L[1])
        a["P1"] = self._pool(a["S0"])
        a["A1"] = self._conv(a["P1"], *L[2])
        a["S1"] = self._conv(a["A1"], *L[3])
        a["P2"] = self._pool(a["S1"])
        a["A2"] = self._conv(a["P2"], *L[4])
        a["S2"] = self._conv(a["A2"], *L[5])
        a["P3"] = self._pool(a["S2"])
        a["BT"] = self._conv(a["P3"], *L[6])
        a["C2"] = torch.cat([self._up(a["BT"]), a["S2"]], 1)
        a["D2"] = self._conv(a["C2"], *L[7])
        a["C1"] = torch.cat([self._up(a["D2"]), a["S1"]], 1)
        a["D1"] = self._conv(a["C1"], *L[8])
        a["C0"] = torch.cat([self._up(a["D1"]), a["S0"]], 1)
        a["D0"] = self._conv(a["C0"], *L[9])
        a["Y"] = (a["D0"] * hw.view(1, -1, 1, 1)).sum(1) + hb
        return a

    # ---------------------------------------------------------------- backward
    def gradients(self, x_nhwc, t, params):
        """(loss, flat gradient) of the mean squared error of the output against t [n, H, W]."""
        L, hw, hb = unpack(params, self.c)
        a = self.forward(x_nhwc, params)
        t = torch.as_tensor(np.asarray(t, dtype=np.float64))
        e = a["Y"] - t
        loss = float((e * e).mean())
        dy = 2.0 * e / e.numel()
        g_hw = (a["D0"] * dy.unsqueeze(1)).sum((0, 2, 3))
        g_hb = dy.sum()
        r = self.r
        grads = [None] * 10

        def conv_bwd(i, inp, out, g_out, need_input=True):
            w, _ = L[i]
            g = g_out * (out > 0)                                  # ReLU
            gw = torch.nn.grad.conv2d_weight(inp, w.shape, g, padding=1)
            grads[i] = (gw, g.sum((0, 2, 3)))
            if not need_input:
                return None
            return _bf(torch.nn.grad.conv2d_input(inp.shape, _bf(w, r), g, padding=1), r)

        def up_bwd(g):
            return _bf(F.avg_pool2d(g, 2) * 4.0, r)

        def pool_bwd_add(g_coarse, g_fine):
            return _bf(g_fine + 0.25 * self._up(g_coarse), r)

        c = self.c
        dD0 = _bf(hw.view(1, -1, 1, 1) * dy.unsqueeze(1), r)
        dC0 = conv_bwd(9, a["C0"], a["D0"], dD0)
        dD1 = up_bwd(dC0[:, :2 * c])
        dC1 = conv_bwd(8, a["C1"], a["D1"], dD1)
        dD2 = up_bwd(dC1[:, :4 * c])
        dC2 = conv_bwd(7, a["C2"], a["D2"], dD2)
        dBT = up_bwd(dC2[:, :4 * c])
        dP3 = conv_bwd(6, a["P3"], a["BT"], dBT)
        dS2 = pool_bwd_add(dP3, dC2[:, 4 * c:])
        dA2 = conv_bwd(5, a["A2"], a["S2"], dS2)
        dP2 = conv_bwd(4, a["P2"], a["A2"], dA2)
        dS1 = pool_bwd_add(dP2, dC1[:, 4 * c:])
        dA1 = conv_bwd(3, a["A1"], a["S1"], dS1)
        dP1 = conv_bwd(2, a["P1"], a["A1"], dA1)
        dS0 = pool_bwd_add(dP1, dC0[:, 2 * c:])
        dA0 = conv_bwd(1, a["A0"], a["S0"], dS0)
        conv_bwd(0, a["X"], a["A0"], dA0, need_input=False)
        return loss, pack_grads(grads, g_hw, g_hb)
