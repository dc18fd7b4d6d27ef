"""Python binding of the surrogate network calls (``include/sclmlp.h``).

Argument marshalling only: the forward pass, the backward pass and Adam run in
the HIP kernels of ``csrc/mlp_kernels.hpp``.  The ``sclmlp_*`` functions mirror
the C calls one to one; :class:`Network` bundles a context with its torch-owned
workspace and stream.
"""
from __future__ import annotations

import ctypes

import numpy as np

from . import SCLBM_OK, SclbmError, _lib

NIN, NHIDDEN, NOUT = 576, 512, 3
NPARAM = 822275
WIDTHS = (NIN, NHIDDEN, NHIDDEN, NHIDDEN, NOUT)


def _check(status: int):
    if status != SCLBM_OK:
        raise SclbmError(status, _lib.sclmlp_last_error().decode())


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _f32(a, n):
    a = np.ascontiguousarray(np.asarray(a, dtype=np.float32).reshape(n))
    return a, a.ctypes.data_as(ctypes.c_void_p)


def sclmlp_workspace_bytes(max_batch: int) -> int:
    b = ctypes.c_size_t()
    _check(_lib.sclmlp_workspace_bytes(int(max_batch), ctypes.byref(b)))
    return b.value


def sclmlp_create(max_batch: int, dev_workspace: int, nbytes: int, stream: int):
    ctx = ctypes.c_void_p()
    _check(_lib.sclmlp_create(int(max_batch), ctypes.c_void_p(dev_workspace), nbytes, ctypes.c_void_p(stream),
                              ctypes.byref(ctx)))
    return ctx


def sclmlp_destroy(ctx):
    _check(_lib.sclmlp_destroy(ctx))


def sclmlp_set_params(ctx, params):
    a, p = _f32(params, NPARAM)
    _check(_lib.sclmlp_set_params(ctx, p))


def sclmlp_get_params(ctx) -> np.ndarray:
    out = np.empty(NPARAM, dtype=np.float32)
    _check(_lib.sclmlp_get_params(ctx, out.ctypes.data_as(ctypes.c_void_p)))
    return out


def sclmlp_get_grads(ctx) -> np.ndarray:
    out = np.empty(NPARAM, dtype=np.float32)
    _check(_lib.sclmlp_get_grads(ctx, out.ctypes.data_as(ctypes.c_void_p)))
    return out


def sclmlp_set_normalization(ctx, in_shift, in_scale, out_shift, out_scale):
    arrs = [_f32(in_shift, NIN), _f32(in_scale, NIN), _f32(out_shift, NOUT), _f32(out_scale, NOUT)]
    _check(_lib.sclmlp_set_normalization(ctx, *[p for _, p in arrs]))


def sclmlp_predict(ctx, windows, n, out):
    _check(_lib.sclmlp_predict(ctx, _ptr(windows), int(n), _ptr(out)))


def sclmlp_gradients(ctx, windows, targets, index, sym, n, ndata, loss=None):
    _check(_lib.sclmlp_gradients(ctx, _ptr(windows), _ptr(targets), _ptr(index), _ptr(sym), int(n), int(ndata),
                                 _ptr(loss)))


def sclmlp_adam(ctx, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    _check(_lib.sclmlp_adam(ctx, float(lr), float(beta1), float(beta2), float(eps)))


def sclmlp_train_step(ctx, windows, targets, index, sym, n, ndata, lr, beta1=0.9, beta2=0.999, eps=1e-8, loss=None):
    _check(_lib.sclmlp_train_step(ctx, _ptr(windows), _ptr(targets), _ptr(index), _ptr(sym), int(n), int(ndata),
                                  float(lr), float(beta1), float(beta2), float(eps), _ptr(loss)))


def sclmlp_get_step(ctx) -> int:
    s = ctypes.c_int64()
    _check(_lib.sclmlp_get_step(ctx, ctypes.byref(s)))
    return s.value


def sclmlp_bad_rows(ctx) -> int:
    s = ctypes.c_int64()
    _check(_lib.sclmlp_bad_rows(ctx, ctypes.byref(s)))
    return s.value


def init_params(seed: int) -> np.ndarray:
    """Weights and biases uniform in +-1/sqrt(fan_in) (float32), drawn on the host
    from a seeded generator.  (A He-normal start, 2.4x wider, fits the training
    windows as well but generalises to unseen trajectories far worse.)"""
    rng = np.random.default_rng(seed)
    parts = []
    for i in range(len(WIDTHS) - 1):
        fan_in, fan_out = WIDTHS[i], WIDTHS[i + 1]
        bound = 1.0 / np.sqrt(fan_in)
        parts.append(rng.uniform(-bound, bound, fan_out * fan_in))
        parts.append(rng.uniform(-bound, bound, fan_out))
    return np.concatenate(parts).astype(np.float32)


class Network:
    """A surrogate context with its workspace and stream.  Device inputs are torch
    tensors (float32 windows [n][576], float32 targets [n][3], int32 indices)."""

    def __init__(self, max_batch: int = 8192, device="cuda:0", stream=None):
        import torch
        self.torch = torch
        self.device = torch.device(device)
        self.max_batch = int(max_batch)
        nbytes = sclmlp_workspace_bytes(self.max_batch)
        with torch.cuda.device(self.device):
            self.stream = stream if stream is not None else torch.cuda.Stream(device=self.device)
            self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
            self.loss_buf = torch.zeros(1, dtype=torch.float64, device=self.device)
        self.ctx = sclmlp_create(self.max_batch, self.workspace.data_ptr(), nbytes, self.stream.cuda_stream)

    def close(self):
        if getattr(self, "ctx", None):
            self.stream.synchronize()
            sclmlp_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _sync_torch(self):
        self.stream.wait_stream(self.torch.cuda.current_stream(self.device))

    def _done(self, *tensors):
        # results are produced on the context's stream; let torch's stream wait for them
        self.torch.cuda.current_stream(self.device).wait_stream(self.stream)
        for t in tensors:
            if t is not None:
                t.record_stream(self.stream)

    def set_params(self, params):
        sclmlp_set_params(self.ctx, params)

    def params(self) -> np.ndarray:
        return sclmlp_get_params(self.ctx)

    def grads(self) -> np.ndarray:
        return sclmlp_get_grads(self.ctx)

    def set_normalization(self, in_shift, in_scale, out_shift, out_scale):
        sclmlp_set_normalization(self.ctx, in_shift, in_scale, out_shift, out_scale)

    @property
    def step_count(self) -> int:
        return sclmlp_get_step(self.ctx)

    def bad_rows(self) -> int:
        return sclmlp_bad_rows(self.ctx)

    def predict(self, windows, out=None):
        """windows: float32 [n][576] device tensor (n may exceed max_batch: chunked)."""
        torch = self.torch
        n = windows.shape[0]
        if out is None:
            out = torch.empty((n, NOUT), dtype=torch.float32, device=self.device)
        self._sync_torch()
        for s in range(0, n, self.max_batch):
            e = min(n, s + self.max_batch)
            sclmlp_predict(self.ctx, windows[s:e], e - s, out[s:e])
        self._done(windows, out)
        return out

    def gradients(self, windows, targets, index=None, sym=None, n=None):
        n = (index.shape[0] if index is not None else windows.shape[0]) if n is None else n
        self._sync_torch()
        sclmlp_gradients(self.ctx, windows, targets, index, sym, n, windows.shape[0], self.loss_buf)
        self._done(windows, targets, index, sym)
        return self.loss_buf

    def adam(self, lr, beta1=0.9, beta2=0.999, eps=1e-8):
        sclmlp_adam(self.ctx, lr, beta1, beta2, eps)

    def train_step(self, windows, targets, index=None, sym=None, n=None, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
        n = (index.shape[0] if index is not None else windows.shape[0]) if n is None else n
        self._sync_torch()
        sclmlp_train_step(self.ctx, windows, targets, index, sym, n, windows.shape[0], lr, beta1, beta2, eps,
                          self.loss_buf)
        self._done(windows, targets, index, sym)
        return self.loss_buf
