"""ctypes binding of the warm-start network (include/wsnet.h): argument marshalling only."""
from __future__ import annotations

import ctypes

import numpy as np

from . import pipesafe

_bound = False


def _lib():
    global _bound
    L = pipesafe.library()
    if not _bound:
        P, i32, i64, f32, u64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_float, ctypes.c_uint64
        L.ws_create.argtypes = [ctypes.POINTER(P), i32, i32, i32, i32, u64]
        L.ws_destroy.argtypes = [P]
        L.ws_num_params.argtypes = [P]
        L.ws_num_params.restype = i64
        L.ws_get_params.argtypes = [P, P]
        L.ws_set_params.argtypes = [P, P]
        L.ws_forward.argtypes = [P, P, P, i32, f32, P]
        L.ws_gradients.argtypes = [P, P, P, i32, P, ctypes.POINTER(ctypes.c_double)]
        L.ws_train.argtypes = [P, P, P, i64, i32, i32, f32, u64, P]
        for name in ("ws_create", "ws_destroy", "ws_get_params", "ws_set_params", "ws_forward",
                     "ws_gradients", "ws_train"):
            getattr(L, name).restype = ctypes.c_int
        _bound = True
    return L


class WsError(RuntimeError):
    pass


def _check(rc, what):
    if rc != 0:
        raise WsError(f"{what} failed ({rc})")


def _dev(t):
    return ctypes.c_void_p(t.data_ptr())


class WarmStartNet:
    """The U-Net of include/wsnet.h on the current HIP device."""

    def __init__(self, H: int, W: int, cin: int = 3, c: int = 16, seed: int = 0):
        self.H, self.W, self.cin, self.c = H, W, cin, c
        h = ctypes.c_void_p()
        _check(_lib().ws_create(ctypes.byref(h), H, W, cin, c, seed), "ws_create")
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            _lib().ws_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    @property
    def num_params(self) -> int:
        return int(_lib().ws_num_params(self._h))

    def get_params(self) -> np.ndarray:
        p = np.empty(self.num_params, dtype=np.float32)
        _check(_lib().ws_get_params(self._h, p.ctypes.data_as(ctypes.c_void_p)), "ws_get_params")
        return p

    def set_params(self, p) -> None:
        p = np.ascontiguousarray(p, dtype=np.float32)
        assert p.size == self.num_params
        _check(_lib().ws_set_params(self._h, p.ctypes.data_as(ctypes.c_void_p)), "ws_set_params")

    def forward(self, x, scale: float = 1.0, y=None, stream=None):
        """x: torch float32 CUDA tensor [count, H, W, cin]; returns y [count, H, W] (scaled)."""
        import torch
        x = x.contiguous()
        count = x.shape[0]
        if y is None:
            y = torch.empty((count, self.H, self.W), dtype=torch.float32, device=x.device)
        if stream is None:
            stream = torch.cuda.current_stream(x.device).cuda_stream
        _check(_lib().ws_forward(self._h, _dev(x), _dev(y), count, float(scale), ctypes.c_void_p(stream)),
               "ws_forward")
        return y

    def gradients(self, x, t):
        """Loss and fp32 parameter gradients for one batch (no update)."""
        g = np.empty(self.num_params, dtype=np.float32)
        loss = ctypes.c_double()
        _check(_lib().ws_gradients(self._h, _dev(x.contiguous()), _dev(t.contiguous()), x.shape[0],
                                   g.ctypes.data_as(ctypes.c_void_p), ctypes.byref(loss)),
               "ws_gradients")
        return loss.value, g

    def train(self, x, t, batch=32, epochs=10, lr=1e-3, seed=0) -> np.ndarray:
        """Adam on device tensors x [count, H, W, cin], t [count, H, W]; per-epoch mean losses."""
        hist = np.zeros(max(epochs, 1))
        _check(_lib().ws_train(self._h, _dev(x.contiguous()), _dev(t.contiguous()), x.shape[0], batch,
                               epochs, float(lr), seed, hist.ctypes.data_as(ctypes.c_void_p)),
               "ws_train")
        return hist[:epochs]
