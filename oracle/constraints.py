"""FP64 per-iteration constraints on the object and probe (oracle).

TEST INFRASTRUCTURE ONLY: imported by tests, the smoke check and the
benchmark's CPU baseline, never by the product path.

After each gradient step the paper applies physical constraints to the
probe and object (Sec. "Physical constraints"); three of them are written
out here, in the order the library applies them:

* r_z filter (Sec. "Real-space depth regularization", the equation that
  convolves O with G_sigma_z along depth): a 1-D Gaussian blur of the object
  along the slice axis.  Readings (not fixed by the paper): the object is
  held as amplitude and phase, and each is blurred; the Gaussian is
  exp(-k^2 / 2 sigma^2) for integer slice offsets k, truncated at
  |k| <= ceil(4 sigma) and normalised to sum 1; beyond the first and last
  slice the stack is mirrored about the outer slice faces (..., s1, s0 | s0,
  s1, ...), so no slice mixes with the far end of the stack.
* positivity (Sec. "Positivity and sparsity"): negative object phase is
  clipped to zero.
* k_z filter (Sec. "Fourier-space depth regularization"): the object is
  multiplied in 3-D Fourier space by W_a(k) = W(k) exp(-alpha (k_x^2 +
  k_y^2)) with W = 1 - (2/pi) arctan(beta^2 k_z^2 / (k_x^2 + k_y^2 + eps)),
  eps = 1e-3; k in 1/angstrom from the pixel size dx and the slice spacing dz
  (fftfreq grids, periodic).  Reading: applied to the amplitude and to the
  phase, each a real field (W_a is real and even, so they stay real).
* probe-mode orthogonalisation (Sec. "Physical constraints", after
  Thibault & Menzel 2013): the mixed-state modes are replaced by the
  eigenvectors of their overlap matrix, ordered by decreasing power.
"""
from __future__ import annotations

import math

import numpy as np

from . import dft


def gaussian_taps(sigma: float, truncate: float = 4.0) -> np.ndarray:
    """Normalised taps w[k + R], k = -R..R, R = ceil(truncate * sigma)."""
    if sigma <= 0:
        return np.ones(1)
    R = int(math.ceil(truncate * sigma))
    k = np.arange(-R, R + 1, dtype=np.float64)
    w = np.exp(-k * k / (2.0 * sigma * sigma))
    return w / w.sum()


def mirror_index(i: int, S: int) -> int:
    """Index i of the stack extended by mirroring about its outer faces."""
    if S == 1:
        return 0
    period = 2 * S
    i %= period
    return i if i < S else period - 1 - i


def rz_filter(vol, sigma: float, truncate: float = 4.0) -> np.ndarray:
    """Blur an S x H x W stack along axis 0 (one slice = one sample)."""
    vol = np.asarray(vol, np.float64)
    S = vol.shape[0]
    w = gaussian_taps(sigma, truncate)
    R = (len(w) - 1) // 2
    out = np.zeros_like(vol)
    for s in range(S):
        for k in range(-R, R + 1):
            out[s] += w[k + R] * vol[mirror_index(s + k, S)]
    return out


def kz_weight(S, H, W, beta, alpha, dx, dz, eps=1e-3) -> np.ndarray:
    """W_a on the S x H x W fftfreq grid (zero frequency at index 0)."""
    kz = dft.fftfreq(S, d=dz)[:, None, None]
    ky = dft.fftfreq(H, d=dx)[None, :, None]
    kx = dft.fftfreq(W, d=dx)[None, None, :]
    kr2 = kx ** 2 + ky ** 2
    Wk = 1.0 - (2.0 / np.pi) * np.arctan(beta ** 2 * kz ** 2 / (kr2 + eps))
    return Wk * np.exp(-alpha * kr2)


def kz_filter(vol, beta, alpha, dx, dz) -> np.ndarray:
    """F3^-1[W_a F3[vol]] of a real S x H x W field (real part of the result)."""
    vol = np.asarray(vol, np.float64)
    Wa = kz_weight(*vol.shape, beta, alpha, dx, dz)
    return np.real(dft.ifftn(Wa * dft.fftn(vol)))


def positivity(phase) -> np.ndarray:
    return np.maximum(np.asarray(phase, np.float64), 0.0)


def probe_overlap(probe) -> np.ndarray:
    """A[m, n] = sum_r conj(P_m(r)) P_n(r)  (Hermitian, M x M)."""
    P = np.asarray(probe, np.complex128).reshape(probe.shape[0], -1)
    return np.conj(P) @ P.T


def probe_orthogonalize(probe):
    """Modes Q_k = sum_m V[m, k] P_m with A V = V diag(lam), lam decreasing.
    Returns (Q (M x N x N), lam).  The incoherent sum sum_k |Q_k|^2 equals
    sum_m |P_m|^2 pixel by pixel (V is unitary), so the model intensities do
    not change; each Q_k is fixed up to a unit phase factor (and within a
    set of equal powers, up to a unitary mixing)."""
    M = probe.shape[0]
    A = probe_overlap(probe)
    lam, V = np.linalg.eigh(A)              # ascending
    order = np.argsort(lam)[::-1]
    lam, V = lam[order], V[:, order]
    P = np.asarray(probe, np.complex128).reshape(M, -1)
    Q = (V.T @ P).reshape(probe.shape)      # Q_k = sum_m V[m, k] P_m
    return Q, lam


def apply(amp, phase, probe, rz_sigma=0.0, phase_positive=False, probe_orthogonal=False, kz_beta=0.0,
          kz_alpha=0.0, dx=1.0, dz=1.0):
    """The constraints in the library's order: k_z filter, r_z filter (each on
    amplitude and phase), positivity, probe orthogonalisation."""
    amp = np.asarray(amp, np.float64)
    phase = np.asarray(phase, np.float64)
    probe = None if probe is None else np.asarray(probe, np.complex128)
    if kz_beta > 0 or kz_alpha > 0:
        amp = kz_filter(amp, kz_beta, kz_alpha, dx, dz)
        phase = kz_filter(phase, kz_beta, kz_alpha, dx, dz)
    if rz_sigma > 0:
        amp = rz_filter(amp, rz_sigma)
        phase = rz_filter(phase, rz_sigma)
    if phase_positive:
        phase = positivity(phase)
    if probe_orthogonal:
        probe, _ = probe_orthogonalize(probe)
    return amp, phase, probe
