"""Discrete Fourier transforms for the FP64 oracle, written out by hand.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The transforms follow the definition
    X[k] = sum_n x[n] exp(sign * 2 pi i n k / n_len)
and evaluate it in complex128 along one axis at a time:

* the iterative radix-2 Cooley-Tukey algorithm (decimation in time): the
  input is put in bit-reversed order, then log2(n) butterfly stages combine
  pairs of half-length transforms, X[k] = E[k] + w^k O[k],
  X[k + h] = E[k] - w^k O[k] with w = exp(sign i pi / h);
* a length with an odd factor r > 1 (the depth and lateral sizes of the k_z
  filter, e.g. 12 = 4 * 3 and 640 = 128 * 5) stops the halving at r-point
  subsequences, which are transformed by the definition itself: a product
  with the r x r DFT matrix, whose entries are formed from (n k mod r) so that
  the angle stays exact.

The paper fixes neither the normalisation nor the sign of its transforms; the
multislice oracle uses the orthonormal pair with exp(-2 pi i ...) forward
(`fft2`, `ifft2`), the k_z filter the unnormalised forward / 1/n inverse pair
(`fftn`, `ifftn`, whose product is the identity either way).
"""
from __future__ import annotations

import functools

import numpy as np


@functools.lru_cache(maxsize=None)
def _bit_reverse(n: int) -> np.ndarray:
    bits = n.bit_length() - 1
    idx = np.arange(n)
    rev = np.zeros(n, dtype=np.int64)
    for b in range(bits):
        rev |= ((idx >> b) & 1) << (bits - 1 - b)
    return rev


@functools.lru_cache(maxsize=None)
def _twiddles(h: int, sign: int) -> np.ndarray:
    """w^k = exp(sign i pi k / h), k = 0..h-1: the butterfly factors that
    combine two h-point transforms into one of 2h points."""
    return np.exp(sign * 1j * np.pi * np.arange(h) / h)


def _fft_mid(x: np.ndarray, sign: int) -> np.ndarray:
    """Unnormalised DFT along the middle axis of a (pre, n, post) array by
    iterative radix-2 decimation in time.  For n = 2^a * r with r odd the
    leaves of the recursion are the r-point subsequences x[j + 2^a t]
    (t = 0..r-1), transformed by the definition; a power of two has r = 1 and
    the leaves are the samples themselves.  The post axis (many independent
    lines) stays innermost, so every butterfly stage is a few whole-array
    operations."""
    pre, n, post = x.shape
    p = n & -n                                   # largest power of two dividing n
    r = n // p
    leaves = np.asarray(x, np.complex128).reshape(pre, r, p, post)      # [t, j]
    a = np.swapaxes(leaves, 1, 2)[:, _bit_reverse(p)]                   # [bitrev j, t]
    if r > 1:
        k = np.arange(r)
        F = np.exp(sign * 2j * np.pi * (np.outer(k, k) % r) / r)
        a = np.einsum("kt,pjtq->pjkq", F, a)
    a = np.array(a, dtype=np.complex128, order="C").reshape(pre, n, post)
    h = r                                        # length of the transforms being combined
    while h < n:
        # groups of 2h: the first h entries hold the transform E of the
        # even-index half of the group's samples, the next h the transform O
        # of the odd-index half; X[k] = E[k] + w^k O[k], X[k + h] = E[k] - w^k O[k]
        g = a.reshape(pre, n // (2 * h), 2, h, post)
        e = g[:, :, 0]
        wo = g[:, :, 1] * _twiddles(h, sign)[:, None]
        np.subtract(e, wo, out=g[:, :, 1])
        e += wo
        h *= 2
    return a


def dft(x, axis: int = -1, sign: int = -1) -> np.ndarray:
    """Unnormalised DFT of sign `sign` (-1 forward, +1 inverse) along `axis`."""
    x = np.asarray(x, np.complex128)
    axis = axis % x.ndim
    shape = x.shape
    pre = int(np.prod(shape[:axis], dtype=np.int64))
    post = int(np.prod(shape[axis + 1:], dtype=np.int64))
    if axis == x.ndim - 1 and x.ndim > 1:
        # a last-axis transform: put the lines of the axis before it innermost
        y = dft(np.swapaxes(x, -1, -2), -2, sign)
        return np.swapaxes(y, -1, -2)
    return _fft_mid(x.reshape(pre, shape[axis], post), sign).reshape(shape)


def _dft2(x, sign: int) -> np.ndarray:
    """Unnormalised 2-D DFT over the last two axes: along y, then along x."""
    return dft(dft(x, -2, sign), -1, sign)


def fft2(x) -> np.ndarray:
    """Orthonormal forward 2-D DFT over the last two axes (sign -1)."""
    x = np.asarray(x, np.complex128)
    ny, nx = x.shape[-2:]
    return _dft2(x, -1) / np.sqrt(ny * nx)


def ifft2(x) -> np.ndarray:
    """Orthonormal inverse 2-D DFT over the last two axes (sign +1)."""
    x = np.asarray(x, np.complex128)
    ny, nx = x.shape[-2:]
    return _dft2(x, +1) / np.sqrt(ny * nx)


def fftn(x) -> np.ndarray:
    """Unnormalised forward DFT over every axis."""
    y = np.asarray(x, np.complex128)
    for ax in range(y.ndim):
        y = dft(y, ax, -1)
    return y


def ifftn(x) -> np.ndarray:
    """Inverse DFT over every axis, scaled by 1 / (number of elements)."""
    y = np.asarray(x, np.complex128)
    for ax in range(y.ndim):
        y = dft(y, ax, +1)
    return y / y.size


def fftfreq(n: int, d: float = 1.0) -> np.ndarray:
    """Sample frequencies of an n-point DFT, in cycles per unit of d: index k
    maps to k / (n d) for k < ceil(n / 2) and to (k - n) / (n d) above, so the
    Nyquist entry of an even n is negative."""
    k = np.arange(n)
    return np.where(k < (n + 1) // 2, k, k - n) * (1.0 / (n * d))


def fftshift2(x) -> np.ndarray:
    """Move index 0 of the last two axes to the centre (n // 2)."""
    x = np.asarray(x)
    return np.roll(x, (x.shape[-2] // 2, x.shape[-1] // 2), axis=(-2, -1))


def ifftshift2(x) -> np.ndarray:
    """Inverse of fftshift2 (the same roll for even sizes)."""
    x = np.asarray(x)
    return np.roll(x, (-(x.shape[-2] // 2), -(x.shape[-1] // 2)), axis=(-2, -1))
