"""FP64 CPU oracle for the multislice forward model, its loss and its gradient.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import or call this
module; only tests, the smoke check and the benchmark's CPU-baseline leg do.
It shares no code with the HIP path (the two only share the seeded input
generator, which holds none of this arithmetic).

Everything is plain NumPy in float64 / complex128, with a loop over scan
positions and arrays over probe modes, written in the order of the paper's
equations:

* forward model, Eq. (1)-(4) of Sec. "Physical model": sub-pixel Fourier shift
  of each probe mode, integer crop of the object patch, transmission through
  every slice with the tilted Fresnel propagator of Eq. (4) between slices,
  far-field intensity summed incoherently over modes (Eq. 2);
* the Gaussian and Poisson losses of Eq. (5)-(6), Sec. "Optimizers and loss
  functions";
* the gradient of the loss with respect to the six optimisable parameters of
  Sec. "AD-optimizable parameters" (object amplitude, object phase, probe,
  position, local tilt, slice spacing), obtained by the chain rule through the
  same steps in reverse.  Complex gradients follow the convention
  dL/dRe + i dL/dIm.

Conventions (readings where the paper is silent):
* F is the orthonormal 2-D DFT with the e^{-2 pi i} sign; F^-1 uses e^{+2 pi i};
  both are the oracle's own radix-2 FFT (`oracle/dft.py`).
* q = fftfreq(N) in cycles/pixel, k = q/dx in 1/angstrom; axis 0 is y, axis 1
  is x; positions and tilts are given as (y, x) pairs.
* the patch for position rho has top-left corner round_half_even(rho) - N/2;
  the probe is shifted by dr = rho - round(rho) with the ramp
  exp(-2 pi i (q_y dr_y + q_x dr_x)).
* S slices use S-1 propagations; the far field is F of the last transmitted
  wave; intensities are returned fftshifted (zero frequency at (N/2, N/2)).
* loss averages run over all B*N*N values of the batch; singular points
  (I = 0 with p < 1, zero Gaussian residual) give a zero gradient.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from . import dft

POISSON_EPS = 1e-6   # epsilon inside the Poisson log, Eq. (6)


# ---------------------------------------------------------------- transforms
def fft2(x):
    """Orthonormal forward 2-D DFT over the last two axes (own radix-2 FFT)."""
    return dft.fft2(x)


def ifft2(x):
    """Orthonormal inverse 2-D DFT over the last two axes (own radix-2 FFT)."""
    return dft.ifft2(x)


def kgrid(N, dx):
    """Spatial frequencies (k_y column, k_x row) in 1/angstrom."""
    k = dft.fftfreq(N) / dx
    return k[:, None], k[None, :]


# ---------------------------------------------------------------- pieces
def split_position(rho, N):
    """Integer crop corner and sub-pixel remainder for one (y, x) position
    (Sec. "Physical model": dr = rho - round(rho), the patch centred on rho)."""
    r = np.round(np.asarray(rho, np.float64))      # round half to even
    dr = np.asarray(rho, np.float64) - r
    t = r.astype(np.int64) - N // 2
    return t, dr


def shift_ramp(dr, N):
    """Fourier shift ramp R(u,v) = exp(-2 pi i (q_u dr_y + q_v dr_x)); applying
    F^-1[R F[P]] moves the probe by +dr pixels."""
    q = dft.fftfreq(N)
    return np.exp(-2j * np.pi * (q[:, None] * dr[0] + q[None, :] * dr[1]))


def propagator_phase(N, dx, lam, dz, tilt):
    """Phase of the adaptive propagator, Eq. (4):
    -pi lam |k|^2 dz + 2 pi dz (k_x tan theta_x + k_y tan theta_y)."""
    dx, lam, dz, tilt = float(dx), float(lam), float(dz), np.asarray(tilt, np.float64)
    ky, kx = kgrid(N, dx)
    return (-np.pi * lam * dz * (kx ** 2 + ky ** 2)
            + 2 * np.pi * dz * (kx * np.tan(tilt[1]) + ky * np.tan(tilt[0])))


def propagator(N, dx, lam, dz, tilt):
    """Adaptive Fresnel propagator with local tilt, Eq. (4)."""
    return np.exp(1j * propagator_phase(N, dx, lam, dz, tilt))


def transmission(amp, phase):
    """Complex object from the two real arrays: O = a exp(i phi)."""
    return amp * np.exp(1j * phase)


def crop(arr, t, N):
    return arr[..., t[0]:t[0] + N, t[1]:t[1] + N]


def check_bounds(pos, N, H, W):
    for rho in np.asarray(pos):
        t, _ = split_position(rho, N)
        if t[0] < 0 or t[1] < 0 or t[0] + N > H or t[1] + N > W:
            raise ValueError(f"patch for position {rho} leaves the {H}x{W} object")


# ---------------------------------------------------------------- forward
@dataclass
class ForwardTrace:
    """Per-position intermediates kept for the gradient."""
    t: np.ndarray          # (2,) int crop corner
    dr: np.ndarray         # (2,) sub-pixel shift
    R: np.ndarray          # (N,N) shift ramp
    H: np.ndarray          # (N,N) propagator
    phi: list              # S arrays (M,N,N): wave incident on slice s
    chi: list              # S arrays (M,N,N): wave leaving slice s
    Psi: np.ndarray        # (M,N,N) far-field waves


def forward_batch(O, Phat, pos, tilt, dz, dx, lam):
    """Multislice exit waves and far-field intensities for a batch of scan
    positions, Eq. (2)-(4), each position on its own (the arrays run over
    positions and modes: (B, M, N, N)).  O: (S,H,W) complex object; Phat:
    (M,N,N) probe spectra; pos, tilt: (B,2).  Returns the (B,N,N) intensities
    (zero frequency at (0, 0)) and one ForwardTrace per position."""
    S = O.shape[0]
    N = Phat.shape[-1]
    dz, dx, lam = float(dz), float(dx), float(lam)
    pos = np.asarray(pos, np.float64).reshape(-1, 2)
    tilt = np.asarray(tilt, np.float64).reshape(-1, 2)
    B = len(pos)
    split = [split_position(rho, N) for rho in pos]
    R = np.stack([shift_ramp(dr, N) for _, dr in split])                     # (B,N,N)
    Hp = np.stack([propagator(N, dx, lam, dz, tilt[j]) for j in range(B)])    # (B,N,N)
    phi = ifft2(Phat[None] * R[:, None])       # shifted probe modes P_j^(m), (B,M,N,N)
    phis, chis = [], []
    for s in range(S):
        phis.append(phi)
        patch = np.stack([crop(O[s], t, N) for t, _ in split])                # (B,N,N)
        chi = patch[:, None] * phi             # transmit through slice s
        chis.append(chi)
        if s < S - 1:
            phi = ifft2(Hp[:, None] * fft2(chi))   # propagate to slice s+1
    Psi = fft2(chis[-1])
    I = np.sum(np.abs(Psi) ** 2, axis=1)       # incoherent sum over modes
    traces = [ForwardTrace(split[j][0], split[j][1], R[j], Hp[j], [p_[j] for p_ in phis],
                           [c_[j] for c_ in chis], Psi[j]) for j in range(B)]
    return I, traces


def forward_one(O, Phat, rho, tilt, dz, dx, lam):
    """Multislice exit wave and far-field intensity for one scan position,
    Eq. (2)-(4).  O: (S,H,W) complex object; Phat: (M,N,N) probe spectra."""
    I, traces = forward_batch(O, Phat, [rho], [tilt], dz, dx, lam)
    return I[0], traces[0]


def forward(amp, phase, probe, pos, tilt, dz, dx, lam, return_trace=False):
    """Model intensities for a batch of positions, fftshifted, (B,N,N) float64.

    amp, phase: (S,H,W), or (n_obj,S,H,W) for mixed object modes (Eq. 2: the
    intensity sums incoherently over probe and object modes); probe: (M,N,N)
    complex; pos, tilt: (B,2) (y,x); dz, dx in angstrom; lam in angstrom.
    With object modes the traces are per mode: traces[o][j]."""
    amp = np.asarray(amp, np.float64)
    phase = np.asarray(phase, np.float64)
    if amp.ndim == 4:
        outs = [forward(amp[o], phase[o], probe, pos, tilt, dz, dx, lam, True) for o in range(amp.shape[0])]
        total = np.sum([o_[0] for o_ in outs], axis=0)
        return (total, [o_[1] for o_ in outs]) if return_trace else total
    probe = np.asarray(probe, np.complex128)
    pos = np.asarray(pos, np.float64)
    tilt = np.asarray(tilt, np.float64)
    N = probe.shape[-1]
    check_bounds(pos, N, amp.shape[1], amp.shape[2])
    O = transmission(amp, phase)
    Phat = fft2(probe)
    I, traces = forward_batch(O, Phat, pos, tilt, dz, dx, lam)
    out = dft.fftshift2(I)
    return (out, traces) if return_trace else out


def exit_waves(amp, phase, probe, rho, tilt, dz, dx, lam):
    """Exit waves chi_{S-1} (M,N,N) for one position (used by invariance tests)."""
    O = transmission(np.asarray(amp, np.float64), np.asarray(phase, np.float64))
    _, tr = forward_one(O, fft2(np.asarray(probe, np.complex128)), rho, tilt, dz, dx, lam)
    return tr.chi[-1]


# ---------------------------------------------------------------- loss
def pacbed_loss(I_model, I_meas, p):
    """The PACBED loss (Sec. "Optimizers and loss functions"): the RMS over
    the detector of the difference between the p-th powers of the batch-mean
    model and measured patterns, over the batch mean of the measured patterns
    to the power p (the data term's normaliser).  Returns (L, dL/dI_model);
    batch rows along axis 0."""
    I = np.asarray(I_model, np.float64)
    Im = np.asarray(I_meas, np.float64)
    B = I.shape[0]
    Abar = I.mean(axis=0)                      # <I_model>_B
    Ebar = Im.mean(axis=0)                     # <I_meas>_B
    R = Abar ** p - Ebar ** p
    D = np.mean(R ** 2)                        # <.>_D
    Z = np.mean(Im ** p)                       # <I_meas^p>_{D,B}
    L = np.sqrt(D) / Z
    if D == 0:
        return float(L), np.zeros_like(I)
    npix = R.size
    with np.errstate(divide="ignore", invalid="ignore"):
        dAbar = np.where(Abar > 0, R * p * Abar ** (p - 1.0), 0.0) / (npix * np.sqrt(D) * Z)
    return float(L), np.broadcast_to(dAbar / B, I.shape).copy()


def data_term(I_model, I_meas, kind, p, eps=POISSON_EPS):
    """One data term: Eq. (5) (kind='gaussian') or Eq. (6) (kind='poisson')
    with power p, averaged over detector and batch.  Returns (L, dL/dI)."""
    I = np.asarray(I_model, np.float64)
    Im = np.asarray(I_meas, np.float64)
    K = I.size
    A = I ** p
    E = Im ** p
    Z = E.mean()
    if Z <= 0:
        raise ValueError("mean of the measured patterns is zero")
    if kind == "gaussian":
        D = np.mean((A - E) ** 2)
        L = np.sqrt(D) / Z
        dA = (A - E) / (K * np.sqrt(D) * Z) if D > 0 else np.zeros_like(A)
    elif kind == "poisson":
        L = -np.mean(E * np.log(A + eps) - A) / Z
        dA = -(E / (A + eps) - 1.0) / (K * Z)
    else:
        raise ValueError(kind)
    if p == 1.0:
        dI = dA
    else:
        with np.errstate(divide="ignore", invalid="ignore"):
            dI = np.where(I > 0, dA * p * I ** (p - 1.0), 0.0)
    return float(L), dI


def loss(I_model, I_meas, kind="gaussian", p=None, eps=POISSON_EPS, pacbed_w=0.0, terms=None):
    """Loss of Eq. (5) (kind='gaussian', default p=0.5) or Eq. (6)
    (kind='poisson', default p=1), averaged over detector and batch; or, with
    terms = [(kind, w, p), ...], the weighted sum of data terms of Eq. (9)
    (w_1 L_Gaussian + w_2 L_Poisson, each term with its own power and its own
    batch normaliser).  pacbed_w > 0 adds pacbed_w times the PACBED loss, with
    the power of the (first) data term.  Returns (L, dL/dI_model) with the
    gradient in the layout of I_model."""
    if terms is None:
        if p is None:
            p = 0.5 if kind == "gaussian" else 1.0
        terms = [(kind, 1.0, p)]
    L, dI = 0.0, 0.0
    for k, w, pt in terms:
        Lt, dIt = data_term(I_model, I_meas, k, pt, eps)
        L = L + w * Lt
        dI = dI + w * dIt
    if pacbed_w:
        Lp, dIp = pacbed_loss(I_model, I_meas, terms[0][2])
        L = L + pacbed_w * Lp
        dI = dI + pacbed_w * dIp
    return float(L), dI


# ---------------------------------------------------------------- gradient
@dataclass
class Gradients:
    amp: np.ndarray      # (S,H,W)
    phase: np.ndarray    # (S,H,W)
    probe: np.ndarray    # (M,N,N) complex, dL/dRe + i dL/dIm
    pos: np.ndarray      # (B,2)  dL/d(rho_y, rho_x)
    tilt: np.ndarray     # (B,2)  dL/d(theta_y, theta_x)
    dz: float
    loss: float


def sparse_term(phase, pos, N):
    """The sparsity regulariser with p = 1 (Sec. "Optimizers and loss
    functions"): the mean of |phase| over the object patches of the batch
    (each position's N x N integer crop, every slice), and its gradient with
    respect to the phase: sign(phase) / (B S N^2) per covering patch, with
    sign(0) = 0."""
    phase = np.asarray(phase, np.float64)
    S = phase.shape[0]
    total = 0.0
    g = np.zeros_like(phase)
    for rho in np.asarray(pos, np.float64):
        t, _ = split_position(rho, N)
        patch = crop(phase, t, N)
        total += np.sum(np.abs(patch))
        crop(g, t, N)[...] += np.sign(patch)
    norm = len(pos) * S * N * N
    return total / norm, g / norm


def gradients(amp, phase, probe, pos, tilt, dz, dx, lam, I_meas, kind="gaussian",
              p=None, sparse_w=0.0, pacbed_w=0.0, terms=None):
    """Loss and its gradient w.r.t. all six parameters for one batch.
    sparse_w > 0 adds sparse_w times the sparsity term, pacbed_w > 0 adds
    pacbed_w times the PACBED loss, terms (see `loss`) weights the data terms
    (the weighted total loss of Eq. 9; by default one data term at weight 1).

    The chain rule is taken through the forward steps in reverse:
    far field -> last slice -> (slice s: object, then propagator) -> shift ->
    probe spectrum.  With L real and y = A x linear, dL/dx = A^H dL/dy; with
    y = c * x elementwise, dL/dx = conj(c) dL/dy and dL/dc = conj(x) dL/dy."""
    amp = np.asarray(amp, np.float64)
    phase = np.asarray(phase, np.float64)
    probe = np.asarray(probe, np.complex128)
    pos = np.asarray(pos, np.float64)
    tilt = np.asarray(tilt, np.float64)
    dz, dx, lam = float(dz), float(dx), float(lam)   # every scalar in float64
    I_model, traces = forward(amp, phase, probe, pos, tilt, dz, dx, lam, return_trace=True)
    L, dI = loss(I_model, I_meas, kind, p, pacbed_w=pacbed_w, terms=terms)
    if amp.ndim == 4:
        # I = sum over object modes: each mode's adjoint takes the same dL/dI;
        # the probe, position, tilt and dz gradients add over the modes
        parts = [_adjoint(amp[o], phase[o], probe, pos, tilt, dz, dx, lam, dI, traces[o])
                 for o in range(amp.shape[0])]
        g_amp = np.stack([q[0] for q in parts])
        g_phase = np.stack([q[1] for q in parts])
        G_probe, g_pos, g_tilt = (sum(q[k] for q in parts) for k in (2, 3, 4))
        g_dz = sum(q[5] for q in parts)
    else:
        g_amp, g_phase, G_probe, g_pos, g_tilt, g_dz = _adjoint(amp, phase, probe, pos, tilt, dz, dx, lam, dI,
                                                                traces)
    if sparse_w:
        S_all = phase.reshape(-1, *phase.shape[-2:])
        Ls, gs = sparse_term(S_all, pos, probe.shape[-1])
        L = L + sparse_w * Ls
        g_phase = g_phase + sparse_w * gs.reshape(phase.shape)
    return Gradients(g_amp, g_phase, G_probe, g_pos, g_tilt, float(g_dz), L)


def _adjoint(amp, phase, probe, pos, tilt, dz, dx, lam, dI, traces):
    """Gradients of one object mode (S,H,W) given dL/dI (fftshifted) and the
    forward traces: (g_amp, g_phase, G_probe, g_pos, g_tilt, g_dz)."""
    S, Hh, Ww = amp.shape
    M, N, _ = probe.shape
    O = transmission(amp, phase)
    Phat = fft2(probe)
    ky, kx = kgrid(N, dx)
    q = dft.fftfreq(N)
    G_O = np.zeros_like(O)
    G_Phat = np.zeros_like(Phat)
    g_pos = np.zeros((len(pos), 2))
    g_tilt = np.zeros((len(pos), 2))
    g_dz = 0.0
    for j, tr in enumerate(traces):
        gI = dft.ifftshift2(dI[j])                       # back to DC-at-0 layout
        G_Psi = 2.0 * gI * tr.Psi                           # I = sum_m |Psi_m|^2
        G_chi = ifft2(G_Psi)                                # Psi = F chi_{S-1}
        G_H = np.zeros((N, N), np.complex128)
        for s in range(S - 1, -1, -1):
            Oj = crop(O[s], tr.t, N)
            crop(G_O[s], tr.t, N)[...] += np.sum(np.conj(tr.phi[s]) * G_chi, axis=0)
            G_phi = np.conj(Oj) * G_chi                     # chi_s = O_s phi_s
            if s > 0:                                        # phi_s = F^-1 H F chi_{s-1}
                X = fft2(tr.chi[s - 1])
                G_hat = fft2(G_phi)
                G_H += np.sum(np.conj(X) * G_hat, axis=0)
                G_chi = ifft2(np.conj(tr.H) * G_hat)
        # shift: phi_0 = F^-1 [Phat R]
        G_hat0 = fft2(G_phi)
        G_Phat += np.conj(tr.R)[None] * G_hat0
        G_R = np.sum(np.conj(Phat) * G_hat0, axis=0)
        dR_dy = -2j * np.pi * q[:, None] * tr.R
        dR_dx = -2j * np.pi * q[None, :] * tr.R
        g_pos[j, 0] = np.sum(np.real(np.conj(G_R) * dR_dy))
        g_pos[j, 1] = np.sum(np.real(np.conj(G_R) * dR_dx))
        # propagator H = exp(i Phi(dz, theta)): dH/dt = i dPhi/dt H
        ty, tx = np.tan(tilt[j][0]), np.tan(tilt[j][1])
        dPhi_ddz = -np.pi * lam * (kx ** 2 + ky ** 2) + 2 * np.pi * (kx * tx + ky * ty)
        dPhi_dty = 2 * np.pi * dz * ky / np.cos(tilt[j][0]) ** 2
        dPhi_dtx = 2 * np.pi * dz * kx / np.cos(tilt[j][1]) ** 2
        w = np.conj(G_H) * 1j * tr.H
        g_dz += np.sum(np.real(w * dPhi_ddz))
        g_tilt[j, 0] = np.sum(np.real(w * dPhi_dty))
        g_tilt[j, 1] = np.sum(np.real(w * dPhi_dtx))
    G_probe = ifft2(G_Phat)                                 # Phat = F P
    g_amp = np.real(np.conj(G_O) * np.exp(1j * phase))      # O = a e^{i phi}
    g_phase = np.imag(G_O * np.conj(O))
    return g_amp, g_phase, G_probe, g_pos, g_tilt, float(g_dz)


def loss_of(amp, phase, probe, pos, tilt, dz, dx, lam, I_meas, kind="gaussian", p=None, sparse_w=0.0,
            pacbed_w=0.0, terms=None):
    """Scalar loss of the forward model (for finite differences)."""
    I = forward(amp, phase, probe, pos, tilt, dz, dx, lam)
    L = loss(I, I_meas, kind, p, pacbed_w=pacbed_w, terms=terms)[0]
    if sparse_w:
        ph = np.asarray(phase, np.float64)
        L += sparse_w * sparse_term(ph.reshape(-1, *ph.shape[-2:]), pos, probe.shape[-1])[0]
    return L


def scatter_patches(patches, ts, S, H, W):
    """Sum of (B,S,N,N) complex patches into an (S,H,W) array at crop corners
    ts (B,2): the adjoint of cropping."""
    out = np.zeros((S, H, W), np.complex128)
    N = patches.shape[-1]
    for b in range(len(ts)):
        out[:, ts[b][0]:ts[b][0] + N, ts[b][1]:ts[b][1] + N] += patches[b]
    return out


def count_parameters(S, H, W, M, N, n_pos, n_obj_modes=1, tilt="none"):
    """Number of real optimisable values: object amplitude + phase per slice,
    complex probe modes, (y, x) per position, and tilts (Sec. "AD-optimizable
    parameters")."""
    obj = 2 * n_obj_modes * S * H * W
    prb = 2 * M * N * N
    ps = 2 * n_pos
    tl = {"none": 0, "global": 2, "local": 2 * n_pos}[tilt]
    return obj, prb, ps, tl
