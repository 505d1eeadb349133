"""Binding of the convolutional subspace predictor (dd_cnn_* in the C ABI).

Argument marshalling only: the forward pass, backward pass and Adam run in
the library's HIP kernels.
"""
from __future__ import annotations

import ctypes as C

import numpy as np

from . import _lib
from ._lib import check


def _torch():
    import torch
    return torch


def _stream():
    torch = _torch()
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _dev(t, dtype, numel, what):
    torch = _torch()
    if not isinstance(t, torch.Tensor) or not t.is_cuda or not t.is_contiguous():
        raise TypeError(f"{what} must be a contiguous CUDA (HIP) tensor")
    if t.dtype != dtype or t.numel() != numel:
        raise ValueError(f"{what} must be {dtype} with {numel} elements")
    return C.c_void_p(t.data_ptr())


class Cnn:
    """Encoder-decoder CNN mapping permittivity [B, ny, nx] (and, with
    in_channels=3, the effective-index field [B, ny*nx]) to k complex fields."""

    def __init__(self, nx, ny, max_batch, k=10, seed=0, in_channels=1, _handle=None):
        self.nx, self.ny, self.max_batch, self.k = int(nx), int(ny), int(max_batch), int(k)
        self.in_channels = int(in_channels)
        self.D = self.nx * self.ny
        if _handle is not None:
            self._h = _handle
            return
        h = C.c_void_p()
        check(_lib.lib().dd_cnn_create(self.nx, self.ny, self.max_batch, self.k,
                                       self.in_channels, C.c_ulonglong(seed), C.byref(h)),
              "dd_cnn_create")
        self._h = h

    def save(self, path):
        """Parameters and Adam state to a predictor file (dd_cnn_save)."""
        check(_lib.lib().dd_cnn_save(self._h, str(path).encode()), "dd_cnn_save")

    @classmethod
    def load(cls, path, max_batch):
        """A network saved by save(), for batches of up to max_batch images."""
        h = C.c_void_p()
        check(_lib.lib().dd_cnn_load(str(path).encode(), int(max_batch), C.byref(h)), "dd_cnn_load")
        v = [C.c_int() for _ in range(5)]
        check(_lib.lib().dd_cnn_dims(h, *[C.byref(x) for x in v]), "dd_cnn_dims")
        nx, ny, k, cin, mb = (x.value for x in v)
        return cls(nx, ny, mb, k, in_channels=cin, _handle=h)

    def layers(self):
        out = []
        n = _lib.lib().dd_cnn_layer_info(self._h, -1, None, None, None, None, None)
        for l in range(n):
            v = [C.c_int() for _ in range(5)]
            _lib.lib().dd_cnn_layer_info(self._h, l, *[C.byref(x) for x in v])
            out.append(tuple(x.value for x in v))
        return out

    @property
    def num_params(self):
        return _lib.lib().dd_cnn_num_params(self._h)

    def get_params(self):
        out = np.zeros(self.num_params, np.float32)
        check(_lib.lib().dd_cnn_get_params(self._h, out.ctypes.data_as(C.POINTER(C.c_float)),
                                           out.size), "dd_cnn_get_params")
        return out

    def set_params(self, flat):
        flat = np.ascontiguousarray(flat, dtype=np.float32)
        check(_lib.lib().dd_cnn_set_params(self._h, flat.ctypes.data_as(C.POINTER(C.c_float)),
                                           flat.size), "dd_cnn_set_params")

    def _eim(self, eim, B, off=0):
        torch = _torch()
        if self.in_channels == 1:
            if eim is not None:
                raise ValueError("this network takes the permittivity only")
            return None
        if eim is None:
            raise ValueError("this network takes the effective-index field (eim)")
        _dev(eim, torch.complex64, eim.shape[0] * self.D, "eim")
        return C.c_void_p(eim[off:off + B].data_ptr())

    def predict(self, eps, U=None, eim=None):
        """eps: [B, ny, nx] float32 (device); eim: [B, ny*nx] complex64 for a
        three-channel network.  Returns U [B, k, D] complex64.  Batches larger
        than max_batch are run in chunks."""
        torch = _torch()
        B = eps.shape[0]
        if U is None:
            U = torch.empty((B, self.k, self.D), dtype=torch.complex64, device=eps.device)
        _dev(eps, torch.float32, B * self.D, "eps")
        _dev(U, torch.complex64, B * self.k * self.D, "U")
        if eim is not None and eim.shape[0] != B:
            raise ValueError("eim must have one field per image")
        for b0 in range(0, B, self.max_batch):
            nb = min(self.max_batch, B - b0)
            e = eps[b0:b0 + nb]
            u = U[b0:b0 + nb]
            f = self._eim(eim, nb, b0)
            if f is None:
                rc = _lib.lib().dd_cnn_predict(self._h, C.c_void_p(e.data_ptr()), nb,
                                               C.c_void_p(u.data_ptr()), _stream())
            else:
                rc = _lib.lib().dd_cnn_predict_eim(self._h, C.c_void_p(e.data_ptr()), f, nb,
                                                   C.c_void_p(u.data_ptr()), _stream())
            check(rc, "dd_cnn_predict")
        return U

    def train_step(self, eps, target, lr=1e-3, b1=0.9, b2=0.999, eim=None):
        torch = _torch()
        B = eps.shape[0]
        loss = C.c_float()
        check(_lib.lib().dd_cnn_train_step(
            self._h, _dev(eps, torch.float32, B * self.D, "eps"), self._eim(eim, B),
            _dev(target, torch.complex64, B * self.k * self.D, "target"), B, float(lr), float(b1),
            float(b2), C.byref(loss), _stream()), "dd_cnn_train_step")
        return loss.value

    def grad(self, eps, target, eim=None):
        torch = _torch()
        B = eps.shape[0]
        loss = C.c_float()
        g = np.zeros(self.num_params, np.float32)
        check(_lib.lib().dd_cnn_grad(
            self._h, _dev(eps, torch.float32, B * self.D, "eps"), self._eim(eim, B),
            _dev(target, torch.complex64, B * self.k * self.D, "target"), B, C.byref(loss),
            g.ctypes.data_as(C.POINTER(C.c_float)), g.size, _stream()), "dd_cnn_grad")
        return loss.value, g

    def _ops_b(self, ops, b, B):
        torch = _torch()
        if len(ops) != B or len(b) != B:
            raise ValueError("one operator and one right-hand side per image")
        opp = _lib.ptr_array([op._h.value for op in ops])
        bp = _lib.ptr_array([_dev(bb, torch.complex128, self.D, f"b[{p}]").value
                             for p, bb in enumerate(b)])
        return opp, bp

    def train_step_res(self, eps, ops, b, lr=1e-3, b1=0.9, b2=0.999, eim=None):
        """One Adam step on the residual loss (eq:res_loss) of the batch:
        ops / b are the images' operators and right-hand sides."""
        torch = _torch()
        B = eps.shape[0]
        opp, bp = self._ops_b(ops, b, B)
        loss = C.c_float()
        check(_lib.lib().dd_cnn_train_step_res(
            self._h, _dev(eps, torch.float32, B * self.D, "eps"), self._eim(eim, B), opp, bp, B,
            float(lr), float(b1), float(b2), C.byref(loss), _stream()), "dd_cnn_train_step_res")
        return loss.value

    def grad_res(self, eps, ops, b, eim=None):
        torch = _torch()
        B = eps.shape[0]
        opp, bp = self._ops_b(ops, b, B)
        loss = C.c_float()
        g = np.zeros(self.num_params, np.float32)
        check(_lib.lib().dd_cnn_grad_res(
            self._h, _dev(eps, torch.float32, B * self.D, "eps"), self._eim(eim, B), opp, bp, B,
            C.byref(loss), g.ctypes.data_as(C.POINTER(C.c_float)), g.size, _stream()),
            "dd_cnn_grad_res")
        return loss.value, g

    def activation(self, layer, B):
        """Layer output (NHWC, float32) of the last forward pass; layer -1 = input."""
        if layer == -1:
            shape = (B, self.in_channels, self.ny, self.nx)
        else:
            H, W = self.ny, self.nx
            for l, (cin, cout, s, up, relu) in enumerate(self.layers()):
                if up:
                    H, W = 2 * H, 2 * W
                elif s == 2:
                    H, W = H // 2, W // 2
                if l == layer:
                    shape = (B, H, W, cout)
                    break
        out = np.zeros(shape, np.float32)
        check(_lib.lib().dd_cnn_debug_activation(self._h, layer, B,
                                                 out.ctypes.data_as(C.POINTER(C.c_float)),
                                                 out.size), "dd_cnn_debug_activation")
        return out

    def close(self):
        if getattr(self, "_h", None):
            _lib.lib().dd_cnn_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def flat_to_layers(flat, layers):
    """Split the flat parameter vector into [[w (cout, cin, 3, 3), b (cout)], ...]."""
    out, off = [], 0
    for cin, cout, _, _, _ in layers:
        nw = cout * cin * 9
        w = flat[off:off + nw].reshape(cout, cin, 3, 3)
        off += nw
        b = flat[off:off + cout]
        off += cout
        out.append([w, b])
    return out


def layers_to_flat(params):
    return np.concatenate([np.concatenate([w.reshape(-1), b.reshape(-1)]) for w, b in params])
