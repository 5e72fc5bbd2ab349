"""Binding of the learned coupling-flow transform of ``libqmcamp.so`` (argument
marshalling only; every step runs in the library's kernels).  See the flow section of
``include/qmcamp.h`` for the transform, its parameter layout and the training rule."""
from __future__ import annotations

import contextlib
import ctypes

import numpy as np

from ._abi import QmcError, lib

FLOW_LAYERS = 4
FLOW_HIDDEN = 64
SAMPLE, DENSITY = 0, 1

_dp = ctypes.c_void_p


def _check(rc, what):
    if rc != 0:
        raise QmcError(rc, f"{what}: {lib().qmc_last_error().decode(errors='replace')}")


def _torch():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("the flow transform needs a HIP device; the library has no CPU path")
    return torch


@contextlib.contextmanager
def _ordered(stream=None):
    """The stream to launch on, ordered after the current stream's work (where the inputs
    were prepared) and before its later work (where the outputs are read and the
    temporaries freed)."""
    torch = _torch()
    cur = torch.cuda.current_stream()
    if stream is None or stream == cur:
        yield ctypes.c_void_p(cur.cuda_stream)
        return
    stream.wait_stream(cur)
    try:
        yield ctypes.c_void_p(stream.cuda_stream)
    finally:
        cur.wait_stream(stream)


def param_count(d: int, n_cond: int = 0) -> int:
    return int(lib().qmc_flow_param_count(d, n_cond))


def glorot_params(d: int, seed: int = 0, zero_last: bool = True, scale: float = 1.0,
                  n_cond: int = 0):
    """Initial parameters in the library layout: Glorot-uniform W1 [64, d + n_cond], W2
    (and W3 unless zero_last), zero biases; with zero_last the flow starts as the
    identity."""
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([seed, 17])))
    parts = []
    for _ in range(FLOW_LAYERS):
        def glorot(o, i):
            lim = scale * np.sqrt(6.0 / (i + o))
            return rng.uniform(-lim, lim, size=(o, i))
        W3 = np.zeros((2 * d, FLOW_HIDDEN)) if zero_last else glorot(2 * d, FLOW_HIDDEN)
        parts += [glorot(FLOW_HIDDEN, d + n_cond), np.zeros(FLOW_HIDDEN),
                  glorot(FLOW_HIDDEN, FLOW_HIDDEN),
                  np.zeros(FLOW_HIDDEN), W3, np.zeros(2 * d)]
    return np.concatenate([p.reshape(-1) for p in parts]).astype(np.float32)


class Flow:
    """Device state of one flow of dimension d (parameters, Adam moments, gradient and
    the packed matrix-core operands) in a torch-allocated buffer.  n_cond > 0: a
    conditional flow whose networks also see n_cond conditioning features per point."""

    def __init__(self, d: int, params=None, seed: int = 0, device=None, n_cond: int = 0):
        torch = _torch()
        self.d = int(d)
        self.n_cond = int(n_cond)
        nbytes = int(lib().qmc_flow_bytes(self.d, self.n_cond))
        if nbytes == 0:
            raise QmcError(-1, f"flow shape d = {d}, n_cond = {n_cond} out of range")
        self.device = torch.device("cuda", torch.cuda.current_device()) if device is None else device
        self.buf = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        off = (-self.buf.data_ptr()) % 256
        self.ptr = self.buf.data_ptr() + off
        self.load(glorot_params(self.d, seed, n_cond=self.n_cond) if params is None else params)

    def load(self, params, stream=None):
        v = np.ascontiguousarray(params, dtype=np.float32).reshape(-1)
        P = param_count(self.d, self.n_cond)
        if v.size != P:
            raise ValueError(f"expected {P} parameters, got {v.size}")
        with _ordered(stream) as sp:
            _check(lib().qmc_flow_load(_dp(self.ptr), self.d, self.n_cond,
                                       v.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), sp),
                   "qmc_flow_load")

    def read(self, stream=None):
        """(parameters, last gradient) as float32 host arrays."""
        P = param_count(self.d, self.n_cond)
        prm = np.empty(P, dtype=np.float32)
        grd = np.empty(P, dtype=np.float32)
        fp = ctypes.POINTER(ctypes.c_float)
        with _ordered(stream) as sp:
            _check(lib().qmc_flow_read(_dp(self.ptr), self.d, self.n_cond, prm.ctypes.data_as(fp),
                                       grd.ctypes.data_as(fp), sp), "qmc_flow_read")
        return prm, grd

    def _cond(self, cond, n):
        """Conditioning features as a device [n, n_cond] float64 tensor (None: no features;
        a single row is repeated for every point)."""
        torch = _torch()
        if self.n_cond == 0:
            return None
        if cond is None:
            raise ValueError("a conditional flow needs conditioning features")
        c = torch.as_tensor(cond, dtype=torch.float64, device=self.device)
        if c.ndim == 1:
            c = c.reshape(1, -1).expand(n, -1)
        if tuple(c.shape) != (n, self.n_cond):
            raise ValueError(f"conditioning features of shape {tuple(c.shape)}, "
                             f"expected ({n}, {self.n_cond})")
        return c.contiguous()

    def transform(self, pts, direction: int = SAMPLE, stream=None, cond=None):
        """(out, logdet) for points [count, d] (device float64 tensor or array-like) and,
        for a conditional flow, conditioning features cond [count, n_cond] or [n_cond]."""
        torch = _torch()
        t = torch.as_tensor(pts, dtype=torch.float64, device=self.device).contiguous()
        n = t.shape[0]
        c = self._cond(cond, n)
        out = torch.empty_like(t)
        ld = torch.empty(n, dtype=torch.float64, device=self.device)
        with _ordered(stream) as sp:
            _check(lib().qmc_flow_transform(_dp(self.ptr), self.d, self.n_cond, direction,
                                            _dp(t.data_ptr()),
                                            _dp(None if c is None else c.data_ptr()), n, sp,
                                            _dp(out.data_ptr()), _dp(ld.data_ptr())),
                   "qmc_flow_transform")
        return out, ld

    def _scratch(self, count):
        torch = _torch()
        nb = int(lib().qmc_flow_scratch_bytes(self.d, self.n_cond, count))
        return torch.empty(nb, dtype=torch.uint8, device=self.device), nb

    def gradient(self, x, w, w_sum=None, stream=None, cond=None) -> float:
        """Gradient of -(1/w_sum) sum w log q(x | cond) into the flow's gradient buffer;
        returns the loss (synchronises)."""
        torch = _torch()
        xt = torch.as_tensor(x, dtype=torch.float64, device=self.device).contiguous()
        wt = torch.as_tensor(w, dtype=torch.float64, device=self.device).contiguous()
        c = self._cond(cond, xt.shape[0])
        ws = 0.0 if w_sum is None else float(w_sum)   # 0: the library sums w on the device
        sc, nb = self._scratch(xt.shape[0])
        loss = torch.zeros(1, dtype=torch.float64, device=self.device)
        with _ordered(stream) as sp:
            _check(lib().qmc_flow_gradient(_dp(self.ptr), self.d, self.n_cond,
                                           _dp(xt.data_ptr()), _dp(wt.data_ptr()),
                                           _dp(None if c is None else c.data_ptr()), xt.shape[0],
                                           ctypes.c_double(ws), _dp(sc.data_ptr()),
                                           ctypes.c_size_t(nb), sp, _dp(loss.data_ptr())),
                   "qmc_flow_gradient")
        return float(loss.item())

    def adam_step(self, step: int, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8, stream=None):
        opt = _adam(lr, beta1, beta2, eps, step)
        with _ordered(stream) as sp:
            _check(lib().qmc_flow_adam_step(_dp(self.ptr), self.d, self.n_cond,
                                            ctypes.byref(opt), sp), "qmc_flow_adam_step")

    def train(self, x, w, batches: int, epochs: int, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8,
              step0: int = 1, stream=None, cond=None):
        """Minibatch Adam over the samples (with per-sample conditioning features cond
        for a conditional flow); returns the per-step losses (host array)."""
        torch = _torch()
        xt = torch.as_tensor(x, dtype=torch.float64, device=self.device).contiguous()
        wt = torch.as_tensor(w, dtype=torch.float64, device=self.device).contiguous()
        c = self._cond(cond, xt.shape[0])
        ws = 0.0   # the library sums the weights on the device
        sc, nb = self._scratch(xt.shape[0] // batches)
        hist = torch.zeros(batches * epochs, dtype=torch.float64, device=self.device)
        opt = _adam(lr, beta1, beta2, eps, step0)
        with _ordered(stream) as sp:
            _check(lib().qmc_flow_train(_dp(self.ptr), self.d, self.n_cond, _dp(xt.data_ptr()),
                                        _dp(wt.data_ptr()),
                                        _dp(None if c is None else c.data_ptr()), xt.shape[0],
                                        ctypes.c_double(ws), ctypes.byref(opt), batches, epochs,
                                        _dp(sc.data_ptr()), ctypes.c_size_t(nb), sp,
                                        _dp(hist.data_ptr())), "qmc_flow_train")
        return hist.cpu().numpy()


class _Adam(ctypes.Structure):
    _fields_ = [("lr", ctypes.c_float), ("beta1", ctypes.c_float), ("beta2", ctypes.c_float),
                ("eps", ctypes.c_float), ("step", ctypes.c_int32), ("reserved0", ctypes.c_int32)]


def _adam(lr, beta1, beta2, eps, step):
    a = _Adam()
    a.lr, a.beta1, a.beta2, a.eps, a.step = lr, beta1, beta2, eps, int(step)
    return a


def bind(L):
    """ctypes signatures of the flow entry points (called by the library loader)."""
    vp, i64, i32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32
    L.qmc_flow_param_count.argtypes = [i32, i32]
    L.qmc_flow_param_count.restype = i64
    L.qmc_flow_bytes.argtypes = [i32, i32]
    L.qmc_flow_bytes.restype = ctypes.c_size_t
    L.qmc_flow_load.argtypes = [vp, i32, i32, ctypes.POINTER(ctypes.c_float), vp]
    L.qmc_flow_read.argtypes = [vp, i32, i32, ctypes.POINTER(ctypes.c_float),
                                ctypes.POINTER(ctypes.c_float), vp]
    L.qmc_flow_transform.argtypes = [vp, i32, i32, i32, vp, vp, i64, vp, vp, vp]
    L.qmc_flow_scratch_bytes.argtypes = [i32, i32, i64]
    L.qmc_flow_scratch_bytes.restype = ctypes.c_size_t
    L.qmc_flow_gradient.argtypes = [vp, i32, i32, vp, vp, vp, i64, ctypes.c_double, vp,
                                    ctypes.c_size_t, vp, vp]
    L.qmc_flow_adam_step.argtypes = [vp, i32, i32, ctypes.POINTER(_Adam), vp]
    L.qmc_flow_train.argtypes = [vp, i32, i32, vp, vp, vp, i64, ctypes.c_double,
                                 ctypes.POINTER(_Adam), i32, i32, vp, ctypes.c_size_t, vp, vp]
    L.qmc_flow_samples.argtypes = [vp, i32, ctypes.c_uint64, ctypes.c_uint64, i32, vp, vp, vp]
    L.qmc_flow_attach.argtypes = [vp, i32, vp, i32, ctypes.POINTER(ctypes.c_double), vp]
    for f in ("qmc_flow_load", "qmc_flow_read", "qmc_flow_transform", "qmc_flow_gradient",
              "qmc_flow_adam_step", "qmc_flow_train", "qmc_flow_samples", "qmc_flow_attach"):
        getattr(L, f).restype = ctypes.c_int
