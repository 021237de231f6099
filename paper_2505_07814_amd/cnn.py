"""Python front end of the learned initial guess (include/ptyr_cnn.h).

A 5-layer 3x3 convolutional net, run and trained by the library's BF16
matrix-core kernels, maps the diffraction patterns of a 3 x 3 neighbourhood of
scan positions to the projected phase of the 32 x 32 patch centred on the
middle position; stitched patches give an initial object phase for the
multislice reconstruction, whose plain initial object remains the fallback.

Tensors: patterns float32 (n_pat, 64, 64) with zero frequency at (32, 32);
neighbourhood tables int32 (B, 9); outputs and targets float32 (B, 32, 32);
parameters one float32 vector of `param_count()` entries (layout in
include/ptyr_cnn.h).  This module marshals arguments only.
"""
from __future__ import annotations

import ctypes as C

import numpy as np
import torch

from . import _lib as L
from .ptyr import _need, _ptr

CHANNELS = (9, 32, 32, 32, 32, 1)
CIN_P = (16, 32, 32, 32, 32)
COUT_P = (32, 32, 32, 32, 16)
NLAYER = 5


def _kp(l):
    return (9 * CIN_P[l] + 31) // 32 * 32


def param_count() -> int:
    return int(L.lib().ptyr_cnn_param_count())


def pack_params(layers) -> np.ndarray:
    """[(W (Cout, Cin, 3, 3), b (Cout,)), ...] -> the packed float32 vector:
    per layer W_p[o][(3u + v) Cin_p + c] = W[o, c, u, v] (zero padded), then
    bias (Cout_p)."""
    out = []
    for l, (W, b) in enumerate(layers):
        W = np.asarray(W, np.float64)
        co, ci = W.shape[:2]
        Wp = np.zeros((COUT_P[l], _kp(l)))
        taps = W.transpose(0, 2, 3, 1)                      # (o, u, v, c)
        for t in range(9):
            Wp[:co, t * CIN_P[l]:t * CIN_P[l] + ci] = taps[:, t // 3, t % 3, :]
        bp = np.zeros(COUT_P[l])
        bp[:co] = b
        out += [Wp.ravel(), bp]
    return np.concatenate(out).astype(np.float32)


def unpack_params(vec) -> list:
    """Inverse of pack_params (drops the padding)."""
    v = np.asarray(vec, np.float64)
    layers, off = [], 0
    for l in range(NLAYER):
        ci, co = CHANNELS[l], CHANNELS[l + 1]
        n = COUT_P[l] * _kp(l)
        Wp = v[off:off + n].reshape(COUT_P[l], _kp(l))
        off += n
        b = v[off:off + co].copy()
        off += COUT_P[l]
        W = np.zeros((co, ci, 3, 3))
        for t in range(9):
            W[:, :, t // 3, t % 3] = Wp[:co, t * CIN_P[l]:t * CIN_P[l] + ci]
        layers.append((W, b))
    return layers


def init_params(seed: int) -> np.ndarray:
    """Seeded initial weights and biases, each uniform in +-1/sqrt(fan_in)
    with fan_in = 9 Cin (the default of common deep-learning libraries for
    a convolution; it keeps the first outputs small for log-count inputs of
    a few units), packed."""
    rng = np.random.default_rng(seed)
    layers = []
    for l in range(NLAYER):
        ci, co = CHANNELS[l], CHANNELS[l + 1]
        bound = 1.0 / np.sqrt(9 * ci)
        layers.append((rng.uniform(-bound, bound, (co, ci, 3, 3)), rng.uniform(-bound, bound, co)))
    return pack_params(layers)


class ConvInit:
    """One ptyr_cnn context: workspace for batches of up to B_max
    neighbourhoods and the stream its calls are queued on."""

    def __init__(self, B_max: int, device=None, stream=None):
        self.lib = L.lib()
        self.B_max = int(B_max)
        self.device = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        nbytes = self.lib.ptyr_cnn_workspace_bytes(self.B_max)
        if nbytes == 0:
            raise L.PtyrError(L.PTYR_E_ARG, "ptyr_cnn_workspace_bytes")
        self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        ptr = (self.workspace.data_ptr() + 255) // 256 * 256
        ctx = C.c_void_p()
        L.check(self.lib.ptyr_cnn_create(self.B_max, C.c_void_p(ptr), nbytes, C.c_void_p(self.stream.cuda_stream),
                                         C.byref(ctx)), "ptyr_cnn_create")
        self._ctx = ctx
        self.n_param = param_count()

    def __del__(self):
        ctx = getattr(self, "_ctx", None)
        if ctx is not None and ctx.value:
            try:
                self.lib.ptyr_cnn_destroy(ctx)
            except Exception:
                pass

    def sync(self):
        L.check(self.lib.ptyr_cnn_sync(self._ctx), "ptyr_cnn_sync")

    def _batch(self, params, patterns, nbr):
        _need(params, "params", torch.float32, (self.n_param,), self.device)
        _need(patterns, "patterns", torch.float32, None, self.device)
        if patterns.dim() != 3 or tuple(patterns.shape[1:]) != (64, 64):
            raise ValueError("patterns must be (n_pat, 64, 64)")
        _need(nbr, "nbr", torch.int32, None, self.device)
        if nbr.dim() != 2 or nbr.shape[1] != 9:
            raise ValueError("nbr must be (B, 9)")
        return nbr.shape[0]

    def forward(self, params, patterns, nbr, out=None):
        """Network output (B, 32, 32) for the neighbourhoods nbr."""
        B = self._batch(params, patterns, nbr)
        if out is None:
            out = torch.empty((B, 32, 32), dtype=torch.float32, device=self.device)
        _need(out, "out", torch.float32, (B, 32, 32), self.device)
        L.check(self.lib.ptyr_cnn_forward(self._ctx, _ptr(params), _ptr(patterns), patterns.shape[0], _ptr(nbr), B,
                                          _ptr(out)), "ptyr_cnn_forward")
        return out

    def gradient(self, params, patterns, nbr, target, grad, loss=None):
        """grad += dL/dparams of the mean-squared error against target
        (B, 32, 32); loss (float64 (1,) tensor, optional) receives L."""
        B = self._batch(params, patterns, nbr)
        _need(target, "target", torch.float32, (B, 32, 32), self.device)
        _need(grad, "grad", torch.float32, (self.n_param,), self.device)
        if loss is not None:
            _need(loss, "loss", torch.float64, (1,), self.device)
        L.check(self.lib.ptyr_cnn_gradient(self._ctx, _ptr(params), _ptr(patterns), patterns.shape[0], _ptr(nbr),
                                           _ptr(target), B, _ptr(grad), _ptr(loss)), "ptyr_cnn_gradient")

    def adam(self, params, grad, m, v, step, lr, beta1=0.9, beta2=0.999, eps=1e-8):
        for t, n in ((params, "params"), (grad, "grad"), (m, "m"), (v, "v")):
            _need(t, n, torch.float32, (self.n_param,), self.device)
        L.check(self.lib.ptyr_cnn_adam(self._ctx, _ptr(params), _ptr(grad), _ptr(m), _ptr(v), int(step), float(lr),
                                       float(beta1), float(beta2), float(eps)), "ptyr_cnn_adam")

    def stitch(self, patches, centres, img):
        """img (H, W) <- mean of the covering patches (P, 32, 32) centred at
        round(centres) (P, 2); uncovered pixels keep their value."""
        _need(img, "img", torch.float32, None, self.device)
        P = patches.shape[0]
        _need(patches, "patches", torch.float32, (P, 32, 32), self.device)
        _need(centres, "centres", torch.float32, (P, 2), self.device)
        H, W = img.shape
        L.check(self.lib.ptyr_cnn_stitch(self._ctx, _ptr(patches), _ptr(centres), P, H, W, _ptr(img)),
                "ptyr_cnn_stitch")
        return img
