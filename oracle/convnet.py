"""FP64 reference of the learned initial-guess network (test infrastructure only).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import or call this
module; only tests, the smoke check and the benchmark's CPU-baseline leg do.
It shares no code with the HIP path.

The paper itself uses a plain initial object (unit amplitude, near-zero random
phase; Sec. "Preprocessing and initialization") and its introduction mentions
machine-learned direct solvers only as related work.  The
network here is an addition on top of the method, specified as:

    a_0 = log(1 + I)                      I: 9 x 64 x 64 (3 x 3 neighbourhood
                                          of diffraction patterns, row-major)
    z_l = conv3x3(a_l, W_l, b_l, stride_l)   l = 0..4, zero padding 1
    a_{l+1} = max(z_l, 0)                 l = 0..3
    out = z_4                             1 x 32 x 32 projected phase
    L = mean over batch and pixels of (out - target)^2

with channels 9 -> 32 -> 32 -> 32 -> 32 -> 1 and strides 1, 2, 1, 1, 1.
conv3x3 is the cross-correlation
    z[b, o, i, j] = bias[o] + sum_{c, u, v} W[o, c, u, v] * a_pad[b, c, s i + u, s j + v]
(u, v = 0, 1, 2; a_pad has one ring of zeros).  Its adjoints follow from the
same index map: the input gradient scatters W[o, c, u, v] g[b, o, i, j] back to
a_pad[b, c, s i + u, s j + v]; the weight gradient is the sum over b, i, j of
g[b, o, i, j] a_pad[b, c, s i + u, s j + v]; the bias gradient sums g.

`bf16=True` evaluates the same net with the rounding points of a BF16
matrix-core implementation: the input, the weights, every stored hidden
activation and every stored back-propagated gradient are rounded to bfloat16
(round to nearest, ties to even); sums stay in float64.  The network output and
the parameter gradients are not rounded.
"""
from __future__ import annotations

import numpy as np

CHANNELS = (9, 32, 32, 32, 32, 1)
STRIDES = (1, 2, 1, 1, 1)
NLAYER = 5


def round_bf16(x):
    """Round to the nearest bfloat16 (8 significant bits, float32 exponent
    range), ties to even, returned as float64.  Works on the float32 bit
    pattern: add 0x7fff plus the lowest kept bit, then clear the 16 low bits.
    Values are first rounded to float32 (the format bfloat16 truncates)."""
    x32 = np.asarray(x, dtype=np.float32)
    u = x32.view(np.uint32).astype(np.uint64)
    keep_lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + keep_lsb) & 0xFFFF0000).astype(np.uint32)
    return r.view(np.float32).astype(np.float64)


def conv3x3(a, W, b, stride):
    """z = bias + cross-correlation of a (B, C, H, H) with W (O, C, 3, 3),
    zero padding 1, given stride.  Output (B, O, Ho, Ho), Ho = (H - 1)//s + 1."""
    B, C, H, _ = a.shape
    Ho = (H - 1) // stride + 1
    ap = np.pad(a, ((0, 0), (0, 0), (1, 1), (1, 1)))
    z = np.broadcast_to(b[None, :, None, None], (B, W.shape[0], Ho, Ho)).copy()
    for u in range(3):
        for v in range(3):
            win = ap[:, :, u:u + stride * (Ho - 1) + 1:stride, v:v + stride * (Ho - 1) + 1:stride]
            z += np.einsum("oc,bchw->bohw", W[:, :, u, v], win)
    return z


def conv3x3_backward(a, W, g, stride):
    """Adjoint of conv3x3 at input a for output gradient g (B, O, Ho, Ho):
    returns (da, dW, db)."""
    B, C, H, _ = a.shape
    Ho = g.shape[2]
    ap = np.pad(a, ((0, 0), (0, 0), (1, 1), (1, 1)))
    dap = np.zeros_like(ap)
    dW = np.zeros_like(W)
    for u in range(3):
        for v in range(3):
            sl = (slice(None), slice(None), slice(u, u + stride * (Ho - 1) + 1, stride),
                  slice(v, v + stride * (Ho - 1) + 1, stride))
            dap[sl] += np.einsum("oc,bohw->bchw", W[:, :, u, v], g)
            dW[:, :, u, v] = np.einsum("bohw,bchw->oc", g, ap[sl])
    return dap[:, :, 1:H + 1, 1:H + 1], dW, g.sum(axis=(0, 2, 3))


def forward(params, I, bf16=False, return_acts=False):
    """Network output (B, 32, 32) for raw neighbourhood intensities I
    (B, 9, 64, 64).  params: list of (W_l, b_l) in float64."""
    rnd = round_bf16 if bf16 else (lambda x: x)
    a = rnd(np.log1p(np.asarray(I, np.float64)))
    acts = [a]
    z = None
    for l, (W, b) in enumerate(params):
        z = conv3x3(a, rnd(W), np.asarray(b, np.float64), STRIDES[l])
        if l < NLAYER - 1:
            a = rnd(np.maximum(z, 0.0))
            acts.append(a)
    out = z[:, 0]
    return (out, acts) if return_acts else out


def loss(out, target):
    """Mean squared error over every output pixel of the batch."""
    return float(np.mean((out - np.asarray(target, np.float64)) ** 2))


def gradients(params, I, target, bf16=False):
    """(loss, [(dW_l, db_l)]) of the mean-squared error with respect to the
    FP64 master parameters (with bf16=True: through the BF16-rounded copies,
    as a matrix-core implementation computes it)."""
    rnd = round_bf16 if bf16 else (lambda x: x)
    out, acts = forward(params, I, bf16, return_acts=True)
    t = np.asarray(target, np.float64)
    n = out.size
    g = rnd(2.0 * (out - t) / n)[:, None]
    grads = [None] * NLAYER
    for l in range(NLAYER - 1, -1, -1):
        W, _ = params[l]
        da, dW, db = conv3x3_backward(acts[l], rnd(W), g, STRIDES[l])
        grads[l] = (dW, db)
        if l > 0:
            g = rnd(np.where(acts[l] > 0, da, 0.0))
    return loss(out, t), grads


def init_params(seed):
    """He-normal weights (std sqrt(2 / (9 Cin))) and zero biases, seeded."""
    rng = np.random.default_rng(seed)
    ps = []
    for l in range(NLAYER):
        ci, co = CHANNELS[l], CHANNELS[l + 1]
        ps.append((rng.standard_normal((co, ci, 3, 3)) * np.sqrt(2.0 / (9 * ci)), np.zeros(co)))
    return ps


def stitch(patches, centres, base):
    """Average of overlapping 32 x 32 patches placed with their centre at
    round_half_even(centre) (rows [cy - 16, cy + 16)); the parts of a patch
    outside the image are dropped; pixels no patch covers keep the value of
    `base`."""
    img = np.array(base, np.float64)
    H, W = img.shape
    acc = np.zeros_like(img)
    cnt = np.zeros_like(img)
    for p, (cy, cx) in zip(patches, centres):
        y0, x0 = int(np.rint(cy)) - 16, int(np.rint(cx)) - 16
        for i in range(32):
            for j in range(32):
                y, x = y0 + i, x0 + j
                if 0 <= y < H and 0 <= x < W:
                    acc[y, x] += p[i, j]
                    cnt[y, x] += 1
    m = cnt > 0
    img[m] = acc[m] / cnt[m]
    return img
