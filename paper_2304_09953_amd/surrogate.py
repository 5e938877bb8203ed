"""Binding of the pre-filter ABI (``include/ligate_surrogate.h``) and its training driver.

Argument marshalling and the order of calls only; features, the network's forward and backward
passes, Adam and minibatch assembly run in the library's HIP kernels.
"""
from __future__ import annotations

import ctypes

import numpy as np
import torch

from . import dock

FEATURES = 512
SURR_EXPORTS = ("surr_param_count", "surr_features", "surr_feature_stats", "surr_cast", "surr_forward",
                "surr_backward", "surr_adam", "surr_gather", "surr_average")


class SurrModel(ctypes.Structure):
    _fields_ = [("d_in", ctypes.c_int32), ("h1", ctypes.c_int32), ("h2", ctypes.c_int32),
                ("d_master", ctypes.c_void_p), ("d_bf16", ctypes.c_void_p), ("d_grad", ctypes.c_void_p),
                ("d_adam_m", ctypes.c_void_p), ("d_adam_v", ctypes.c_void_p)]


_bound = False


def _lib():
    global _bound
    lib = dock.load()
    if not _bound:
        vp, sz, i32, i64, f32 = ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int32, ctypes.c_int64, ctypes.c_float
        P = ctypes.POINTER
        lib.surr_param_count.argtypes = [i32, i32, i32, P(i64), P(i64)]
        lib.surr_features.argtypes = [vp, vp, vp, vp, i32, i64, i32, vp, vp, vp, vp, vp]
        lib.surr_feature_stats.argtypes = [vp, i64, vp, vp, vp, P(sz), vp]
        lib.surr_cast.argtypes = [P(SurrModel), vp]
        lib.surr_forward.argtypes = [P(SurrModel), vp, i32, vp, vp, P(sz), vp]
        lib.surr_backward.argtypes = [P(SurrModel), vp, vp, i32, vp, vp, P(sz), vp]
        lib.surr_adam.argtypes = [P(SurrModel), f32, f32, f32, f32, i32, vp]
        lib.surr_gather.argtypes = [vp, vp, vp, i64, i32, vp, vp, vp]
        lib.surr_average.argtypes = [vp, i32, i64, vp, vp]
        for n in SURR_EXPORTS:
            getattr(lib, n).restype = ctypes.c_int
        _bound = True
    return lib


_p, _s, _check = dock._ptr, dock._stream, dock._check


def features(lib_dev, mean=None, istd=None, f32: bool = True, bf16: bool = True, stream=None, n_types=None):
    """Features of a DeviceLibrary: (FP32 [n, 512] or None, BF16 bits as int16 [n, 512] or None).
    n_types: the type count stated to the call (default: the library's)."""
    n = lib_dev.n_lig
    dev = lib_dev.pack.device
    F = torch.empty((n, FEATURES), dtype=torch.float32, device=dev) if f32 else None
    Fb = torch.empty((n, FEATURES), dtype=torch.int16, device=dev) if bf16 else None
    _check(_lib().surr_features(_p(lib_dev.atom_off), _p(lib_dev.xyz), _p(lib_dev.types), _p(lib_dev.pack), n,
                                lib_dev.n_atoms, lib_dev.n_types if n_types is None else n_types, _p(mean), _p(istd),
                                _p(F), _p(Fb), _s(stream)),
           "surr_features")
    return F, Fb


def feature_stats(F: torch.Tensor, stream=None):
    n = F.shape[0]
    sz = ctypes.c_size_t()
    lib = _lib()
    _check(lib.surr_feature_stats(None, n, None, None, None, ctypes.byref(sz), None), "surr_feature_stats(size)")
    ws = torch.empty(sz.value, dtype=torch.uint8, device=F.device)
    mean = torch.empty(FEATURES, dtype=torch.float32, device=F.device)
    istd = torch.empty(FEATURES, dtype=torch.float32, device=F.device)
    _check(lib.surr_feature_stats(_p(F), n, _p(mean), _p(istd), _p(ws), ctypes.byref(sz), _s(stream)),
           "surr_feature_stats")
    return mean, istd


def gather(x_bf16, t, idx, x_out, t_out, stream=None):
    _check(_lib().surr_gather(_p(x_bf16), _p(t), _p(idx), idx.numel(), x_bf16.shape[1] if x_bf16 is not None else 1,
                              _p(x_out), _p(t_out), _s(stream)), "surr_gather")


class Model:
    """A pre-filter network with its FP32 master weights, BF16 copies, gradient and Adam state."""

    def __init__(self, init: np.ndarray, d_in: int = 512, h1: int = 1024, h2: int = 1024, device="cuda"):
        lib = _lib()
        nm, nb = ctypes.c_int64(), ctypes.c_int64()
        _check(lib.surr_param_count(d_in, h1, h2, ctypes.byref(nm), ctypes.byref(nb)), "surr_param_count")
        assert init.size == nm.value, (init.size, nm.value)
        self.d_in, self.h1, self.h2 = d_in, h1, h2
        self.master = torch.as_tensor(np.ascontiguousarray(init, dtype=np.float32)).to(device)
        self.bf16 = torch.empty(nb.value, dtype=torch.int16, device=device)
        self.grad = torch.zeros(nm.value, dtype=torch.float32, device=device)
        self.m = torch.zeros(nm.value, dtype=torch.float32, device=device)
        self.v = torch.zeros(nm.value, dtype=torch.float32, device=device)
        self.step = 0
        self.c = SurrModel(d_in, h1, h2, self.master.data_ptr(), self.bf16.data_ptr(), self.grad.data_ptr(),
                           self.m.data_ptr(), self.v.data_ptr())
        self._ws = {}
        self.cast()

    def cast(self, stream=None):
        _check(_lib().surr_cast(ctypes.byref(self.c), _s(stream)), "surr_cast")

    def _workspace(self, kind: str, batch: int):
        key = (kind, batch)
        if key not in self._ws:
            sz = ctypes.c_size_t()
            lib = _lib()
            if kind == "fwd":
                _check(lib.surr_forward(ctypes.byref(self.c), None, batch, None, None, ctypes.byref(sz), None), "size")
            else:
                _check(lib.surr_backward(ctypes.byref(self.c), None, None, batch, None, None, ctypes.byref(sz), None),
                       "size")
            self._ws[key] = torch.empty(sz.value, dtype=torch.uint8, device=self.master.device)
        return self._ws[key]

    def forward(self, x_bf16: torch.Tensor, out: torch.Tensor | None = None, stream=None) -> torch.Tensor:
        batch = x_bf16.shape[0]
        y = out if out is not None else torch.empty(batch, dtype=torch.float32, device=x_bf16.device)
        ws = self._workspace("fwd", batch)
        sz = ctypes.c_size_t(ws.numel())
        _check(_lib().surr_forward(ctypes.byref(self.c), _p(x_bf16), batch, _p(y), _p(ws), ctypes.byref(sz),
                                   _s(stream)), "surr_forward")
        return y

    def backward(self, x_bf16: torch.Tensor, t: torch.Tensor, loss: torch.Tensor, stream=None):
        batch = x_bf16.shape[0]
        ws = self._workspace("bwd", batch)
        sz = ctypes.c_size_t(ws.numel())
        _check(_lib().surr_backward(ctypes.byref(self.c), _p(x_bf16), _p(t), batch, _p(loss), _p(ws),
                                    ctypes.byref(sz), _s(stream)), "surr_backward")

    def adam(self, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8, stream=None):
        self.step += 1
        _check(_lib().surr_adam(ctypes.byref(self.c), lr, b1, b2, eps, self.step, _s(stream)), "surr_adam")

    def state(self) -> dict:
        """Training state: FP32 master weights, Adam moments and step count.  The BF16 copies follow
        from the master weights and the gradient buffer is overwritten by every step, so restoring
        these continues training exactly."""
        return {"master": self.master.cpu().numpy().copy(), "m": self.m.cpu().numpy().copy(),
                "v": self.v.cpu().numpy().copy(), "step": np.array(self.step)}

    def load_state(self, st: dict) -> None:
        for name in ("master", "m", "v"):
            t = getattr(self, name)
            t.copy_(torch.as_tensor(np.asarray(st[name], dtype=np.float32)).to(t.device))
        self.step = int(st["step"])
        self.cast()

    def predict(self, x_bf16: torch.Tensor, chunk: int = 65536) -> torch.Tensor:
        out = torch.empty(x_bf16.shape[0], dtype=torch.float32, device=x_bf16.device)
        for s in range(0, x_bf16.shape[0], chunk):
            self.forward(x_bf16[s:s + chunk], out[s:s + chunk])
        return out


def train(model: Model, X_bf16: torch.Tensor, t: torch.Tensor, epochs: int = 30, batch: int = 1024,
          lr: float = 1e-3, seed: int = 0, log=None) -> list:
    """Minibatch Adam on the mean squared error; the sample order is reshuffled each epoch with a
    seeded permutation and the incomplete last batch of an epoch is dropped.  Returns epoch losses."""
    n = X_bf16.shape[0]
    dev = X_bf16.device
    xb = torch.empty((batch, X_bf16.shape[1]), dtype=torch.int16, device=dev)
    tb = torch.empty(batch, dtype=torch.float32, device=dev)
    nb = n // batch
    losses = torch.empty(max(nb, 1), dtype=torch.float32, device=dev)  # one slot per step of an epoch
    rng = np.random.default_rng(seed)
    hist = []
    for ep in range(epochs):
        perm = torch.as_tensor(rng.permutation(n).astype(np.int32)).to(dev)
        for b in range(nb):
            gather(X_bf16, t, perm[b * batch:(b + 1) * batch], xb, tb)
            model.backward(xb, tb, losses[b:b + 1])
            model.adam(lr)
        hist.append(float(losses[:nb].cpu().numpy().astype(np.float64).mean()) if nb else float("nan"))
        if log:
            log(f"epoch {ep + 1}/{epochs}: loss {hist[-1]:.4f}")
    return hist


def average(ys: torch.Tensor, stream=None) -> torch.Tensor:
    """Members' mean of predictions ys [n_members, n] (surr_average): [n] FP32."""
    ys = ys.contiguous()
    out = torch.empty(ys.shape[1], dtype=torch.float32, device=ys.device)
    _check(_lib().surr_average(_p(ys), ys.shape[0], ys.shape[1], _p(out), _s(stream)), "surr_average")
    return out
