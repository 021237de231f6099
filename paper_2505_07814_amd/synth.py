"""Seeded synthetic inputs shaped like the PtyRAD paper's workloads.

This module builds *inputs only*: electron wavelength, mixed-state probes,
Gaussian-atom objects, scan positions, tilts, the plain initial object and
Poisson sampling of a given intensity.  It contains none of the multislice
forward model, loss or gradient arithmetic; both the FP64 oracle tests and the
GPU path draw their inputs from here so that the two never share method code.

Random numbers come from NumPy's PCG64 (`numpy.random.default_rng(seed)`).
Every workload uses seeds ``100*c + k`` with k = 1 object, 2 positions/jitter,
3 mode weights / tilts, 4 Poisson, 5 initial phase.

Stand-ins: the paper reconstructs experimental MOSS-6 / ZSM-5 / tBL-WSe2 /
PrScO3 data and an abTEM-simulated tBL-WSe2 set (Sec. "Benchmarking on
published datasets", Sec. "Computation speed and convergence").  None of those
datasets is reproduced; the generators below make seeded objects of the same
kind (crystalline Gaussian-atom lattices, a twisted bilayer pair) at the
detector size, slice count, mode count, scan size and dose of those runs.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Optional

import numpy as np


# --------------------------------------------------------------------------
# optics
# --------------------------------------------------------------------------
def wavelength_A(kv: float) -> float:
    """Relativistic electron wavelength in angstrom for an accelerating
    voltage in kV: lambda = h / sqrt(2 m e V (1 + e V / 2 m c^2))."""
    v = kv * 1e3
    return 12.2643 / np.sqrt(v * (1.0 + 0.97845e-6 * v))


def _kgrid(N: int, dx: float):
    k = np.fft.fftfreq(N) / dx
    return k[:, None], k[None, :]


def probe_single(N: int, dx: float, kv: float, alpha_mrad: float,
                 defocus_A: float) -> np.ndarray:
    """Aberration-limited STEM probe: hard aperture of semi-angle alpha and a
    defocus phase chi(k) = pi*lambda*df*|k|^2, transformed to real space and
    centred at pixel (N/2, N/2).  Unit norm (sum |P|^2 = 1)."""
    lam = wavelength_A(kv)
    ky, kx = _kgrid(N, dx)
    k2 = ky ** 2 + kx ** 2
    kmax = alpha_mrad * 1e-3 / lam
    aperture = (np.sqrt(k2) <= kmax).astype(np.float64)
    spec = aperture * np.exp(-1j * np.pi * lam * defocus_A * k2)
    p = np.fft.fftshift(np.fft.ifft2(spec))
    return p / np.sqrt(np.sum(np.abs(p) ** 2))


def hermite_modes(p0: np.ndarray, orders, seed: int, w0: float = 0.6,
                  dose: float = 1.0) -> np.ndarray:
    """Mixed-state probe: p0 times Hermite-Gaussian perturbations
    H_a(x/w) H_b(y/w) (w = RMS radius of |p0|^2), orthonormalised with
    modified Gram-Schmidt in the given order, then weighted: the first mode
    carries w0 of the power, the rest a sorted seeded Dirichlet share of
    1 - w0.  Total power sum_m ||P_m||^2 = dose."""
    from numpy.polynomial.hermite import hermval
    N = p0.shape[0]
    yy, xx = np.mgrid[0:N, 0:N].astype(np.float64) - N / 2
    inten = np.abs(p0) ** 2
    w = np.sqrt(np.sum((yy ** 2 + xx ** 2) * inten) / np.sum(inten))
    modes = []
    for (a, b) in orders:
        ca = np.zeros(a + 1); ca[a] = 1.0
        cb = np.zeros(b + 1); cb[b] = 1.0
        m = p0 * hermval(xx / w, ca) * hermval(yy / w, cb)
        for q in modes:  # modified Gram-Schmidt
            m = m - np.vdot(q, m) * q
        m = m / np.sqrt(np.vdot(m, m).real)
        modes.append(m)
    M = len(modes)
    rng = np.random.default_rng(seed)
    if M == 1:
        weights = np.array([1.0])
    else:
        rest = np.sort(rng.dirichlet(np.ones(M - 1)))[::-1] * (1.0 - w0)
        weights = np.concatenate([[w0], rest])
    return np.stack([np.sqrt(wt * dose) * m for wt, m in zip(weights, modes)])


HG_ORDERS_6 = [(0, 0), (1, 0), (0, 1), (2, 0), (1, 1), (0, 2)]
HG_ORDERS_8 = HG_ORDERS_6 + [(3, 0), (0, 3)]


# --------------------------------------------------------------------------
# objects
# --------------------------------------------------------------------------
def render_atoms(shape, centers_px: np.ndarray, sigma_px: float,
                 peak: float) -> np.ndarray:
    """Sum of isotropic Gaussians exp(-r^2/2 sigma^2) * peak at sub-pixel
    centres (y, x), each rendered in a +-5 sigma window."""
    H, W = shape
    out = np.zeros(shape, np.float64)
    r = int(np.ceil(5 * sigma_px))
    for cy, cx in centers_px:
        y0, y1 = max(int(np.floor(cy)) - r, 0), min(int(np.floor(cy)) + r + 2, H)
        x0, x1 = max(int(np.floor(cx)) - r, 0), min(int(np.floor(cx)) + r + 2, W)
        if y0 >= y1 or x0 >= x1:
            continue
        yy = np.arange(y0, y1)[:, None] - cy
        xx = np.arange(x0, x1)[None, :] - cx
        out[y0:y1, x0:x1] += peak * np.exp(-(yy ** 2 + xx ** 2) / (2 * sigma_px ** 2))
    return out


def random_atom_object(H: int, W: int, S: int, n_atoms: int, sigma_px: float,
                       peak: float, seed: int, amp_k: float = 0.05):
    """n_atoms Gaussian atoms at uniform random positions, each assigned to a
    uniformly random slice.  Returns (amp, phase), each (S, H, W) float64,
    amp = exp(-amp_k * phase)."""
    rng = np.random.default_rng(seed)
    cy = rng.uniform(0, H, n_atoms)
    cx = rng.uniform(0, W, n_atoms)
    sl = rng.integers(0, S, n_atoms) if S > 1 else np.zeros(n_atoms, int)
    phase = np.zeros((S, H, W))
    for s in range(S):
        sel = sl == s
        phase[s] = render_atoms((H, W), np.stack([cy[sel], cx[sel]], 1), sigma_px, peak)
    return np.exp(-amp_k * phase), phase


def lattice_object(H: int, W: int, S: int, dx: float, a_A: float, sigma_A: float,
                   peak: float, seed: int, kind: str = "square",
                   vacancy: float = 0.0, twist_deg: float = 0.0,
                   twist_from: Optional[int] = None, amp_k: float = 0.05):
    """Crystalline Gaussian-atom object.  kind 'square' or 'hex' lattice of
    constant a_A; columns aligned across slices; each site of each slice is
    independently vacant with probability `vacancy`.  With twist_from=s0,
    slices s >= s0 use the lattice rotated by twist_deg (twisted bilayer)."""
    rng = np.random.default_rng(seed)
    a = a_A / dx
    sig = sigma_A / dx
    if kind == "square":
        b1, b2 = np.array([a, 0.0]), np.array([0.0, a])
    elif kind == "hex":
        b1, b2 = np.array([a, 0.0]), np.array([a / 2, a * np.sqrt(3) / 2])
    else:
        raise ValueError(kind)
    R = int(np.ceil(1.5 * max(H, W) / a)) + 2
    ii, jj = np.meshgrid(np.arange(-R, R + 1), np.arange(-R, R + 1), indexing="ij")
    base = ii.reshape(-1, 1) * b1 + jj.reshape(-1, 1) * b2  # (n, 2) as (y, x)
    ctr = np.array([H / 2, W / 2])

    def sites(theta):
        c, s_ = np.cos(theta), np.sin(theta)
        rot = base @ np.array([[c, -s_], [s_, c]]).T
        pts = rot + ctr
        keep = (pts[:, 0] > -3 * sig) & (pts[:, 0] < H + 3 * sig) & \
               (pts[:, 1] > -3 * sig) & (pts[:, 1] < W + 3 * sig)
        return pts[keep]

    s0 = sites(0.0)
    s1 = sites(np.deg2rad(twist_deg)) if twist_from is not None else s0
    phase = np.zeros((S, H, W))
    cache = {}
    for s in range(S):
        pts = s1 if (twist_from is not None and s >= twist_from) else s0
        keep = rng.random(len(pts)) >= vacancy
        if vacancy == 0.0:
            key = id(pts)
            if key not in cache:
                cache[key] = render_atoms((H, W), pts, sig, peak)
            phase[s] = cache[key]
        else:
            phase[s] = render_atoms((H, W), pts[keep], sig, peak)
    return np.exp(-amp_k * phase), phase


def plain_init(S: int, H: int, W: int, seed: int):
    """Plain initial object: unit amplitude, phase ~ U[0, 1e-8]."""
    rng = np.random.default_rng(seed)
    return np.ones((S, H, W)), rng.uniform(0.0, 1e-8, (S, H, W))


# --------------------------------------------------------------------------
# scan
# --------------------------------------------------------------------------
def raster_positions(ny: int, nx: int, step: float, origin: float, jitter: float,
                     seed: int) -> np.ndarray:
    """Row-major raster of (y, x) probe positions in object pixels with
    uniform seeded jitter in [-jitter, +jitter] per coordinate."""
    rng = np.random.default_rng(seed)
    gy, gx = np.meshgrid(origin + step * np.arange(ny), origin + step * np.arange(nx),
                         indexing="ij")
    pos = np.stack([gy.ravel(), gx.ravel()], 1).astype(np.float64)
    if jitter > 0:
        pos = pos + rng.uniform(-jitter, jitter, pos.shape)
    return pos


def poisson(intensity: np.ndarray, seed: int) -> np.ndarray:
    """Poisson counts of a non-negative expected intensity, as float32."""
    rng = np.random.default_rng(seed)
    return rng.poisson(np.maximum(intensity, 0.0)).astype(np.float32)


# --------------------------------------------------------------------------
# workloads
# --------------------------------------------------------------------------
@dataclass
class Workload:
    name: str
    N: int
    S: int
    M: int
    B: int
    H: int
    W: int
    dx: float
    kv: float
    dz: float
    amp: np.ndarray
    phase: np.ndarray
    probe: np.ndarray            # (M, N, N) complex128
    pos: np.ndarray              # (Ntot, 2) float64, (y, x)
    tilt: np.ndarray             # (Ntot, 2) float64, (theta_y, theta_x) rad
    dose: float
    seed_base: int
    extra: dict = field(default_factory=dict)

    @property
    def lam(self) -> float:
        return wavelength_A(self.kv)


def workload(name: str, scan: Optional[int] = None) -> Workload:
    """The seeded workloads.  `scan` optionally truncates the raster to its
    first `scan` positions (row-major)."""
    if name == "single_slice_64":         # N=64, 1 slice, 1 mode
        c = 1
        N, S, M, B, H, W, dx, kv, dz = 64, 1, 1, 16, 128, 128, 0.2, 300.0, 10.0
        amp, phase = random_atom_object(H, W, S, 40, 0.3 / dx, 0.5, 100 * c + 1)
        probe = probe_single(N, dx, kv, 20.0, 100.0)[None] * np.sqrt(1e5)
        pos = raster_positions(4, 4, 8, 52, 0.3, 100 * c + 2)
        tilt = np.zeros_like(pos)
        dose = 1e5
    elif name == "multislice_128":        # N=128, 12 slices, 6 modes, B=64
        c = 2
        N, S, M, B, H, W, dx, kv, dz = 128, 12, 6, 64, 640, 640, 0.15, 300.0, 20.0
        amp, phase = lattice_object(H, W, S, dx, 3.9, 0.3, 0.1, 100 * c + 1,
                                    kind="square", vacancy=0.05)
        p0 = probe_single(N, dx, kv, 20.0, 100.0)
        probe = hermite_modes(p0, HG_ORDERS_6, 100 * c + 3, dose=1e6)
        pos = raster_positions(128, 128, 4, 66, 0.5, 100 * c + 2)
        tilt = np.zeros_like(pos)
        dose = 1e6
    elif name == "diffcheck_64":          # N=64, 24 slices, local tilts
        c = 3
        N, S, M, B, H, W, dx, kv, dz = 64, 24, 1, 16, 128, 128, 0.2, 300.0, 10.0
        amp, phase = random_atom_object(H, W, S, 40, 0.3 / dx, 0.5, 100 * c + 1)
        probe = probe_single(N, dx, kv, 20.0, 100.0)[None] * np.sqrt(1e5)
        pos = raster_positions(4, 4, 8, 52, 0.3, 100 * c + 2)
        tilt = np.random.default_rng(100 * c + 3).uniform(-2e-3, 2e-3, pos.shape)
        dose = 1e5
    elif name == "large_256":             # N=256, 30 slices, 8 modes, B=16
        c = 4
        N, S, M, B, H, W, dx, kv, dz = 256, 30, 8, 16, 1024, 1024, 0.15, 300.0, 10.0
        amp, phase = lattice_object(H, W, S, dx, 3.3, 0.3, 0.1, 100 * c + 1,
                                    kind="hex", twist_deg=1.1, twist_from=15)
        p0 = probe_single(N, dx, kv, 20.0, 100.0)
        probe = hermite_modes(p0, HG_ORDERS_8, 100 * c + 3, dose=1e6)
        pos = raster_positions(192, 192, 4, 130, 0.5, 100 * c + 2)
        tilt = np.zeros_like(pos)
        dose = 1e6
    else:
        raise KeyError(name)
    if scan is not None:
        pos = pos[:scan]
        tilt = tilt[:scan]
    return Workload(name, N, S, M, B, H, W, dx, kv, dz, amp, phase, probe, pos, tilt,
                    dose, 100 * c)


def small_case(N: int = 16, S: int = 3, M: int = 2, B: int = 3, H: int = 40,
               W: int = 44, seed: int = 7, tilt_scale: float = 2e-3,
               jitter: float = 0.3) -> Workload:
    """A tiny random case for exhaustive checks: smooth random object, random
    mixed probe confined to the window, positions kept |dr| <= jitter off the
    rounding edge, random local tilts."""
    rng = np.random.default_rng(seed)
    dx, kv, dz = 0.25, 300.0, 7.0
    phase = 0.3 * rng.standard_normal((S, H, W))
    amp = 1.0 + 0.1 * rng.standard_normal((S, H, W))
    yy, xx = np.mgrid[0:N, 0:N] - N / 2
    env = np.exp(-(yy ** 2 + xx ** 2) / (2 * (N / 5) ** 2))
    probe = env * (rng.standard_normal((M, N, N)) + 1j * rng.standard_normal((M, N, N)))
    lo_y, hi_y = N / 2 + 1, H - N / 2 - 1
    lo_x, hi_x = N / 2 + 1, W - N / 2 - 1
    base = np.stack([rng.integers(int(lo_y), int(hi_y), B),
                     rng.integers(int(lo_x), int(hi_x), B)], 1).astype(np.float64)
    pos = base + rng.uniform(-jitter, jitter, (B, 2))
    tilt = rng.uniform(-tilt_scale, tilt_scale, (B, 2))
    return Workload("small", N, S, M, B, H, W, dx, kv, dz, amp, phase, probe, pos, tilt,
                    float(np.sum(np.abs(probe) ** 2)), seed)


# --------------------------------------------------------------------------
# learned initial guess: neighbourhood scans of random single-slice objects
# --------------------------------------------------------------------------
LI_N, LI_DX, LI_KV, LI_DZ, LI_DOSE = 64, 0.2, 300.0, 10.0, 1e5
LI_H = 144                     # object side: a 10 x 10 raster of step 8 with a 64-px window fits
LI_SCAN = (10, 10, 8, 36, 0.3)  # ny, nx, step, origin (centre of the first window), jitter
LI_ATOMS = 51                  # the atom density of the 40-atom 128 x 128 single-slice object
LI_OBJECT_SEED0 = 10 ** 6      # training object i uses seed 10^6 + i
LI_EVAL_SEED = 999             # held-out evaluation object


def li_probe() -> np.ndarray:
    """The single-slice optics: 64 x 64 at 0.2 A/px, 300 kV, 20 mrad, 100 A
    defocus, 1e5 electrons per pattern; shape (1, 64, 64)."""
    return probe_single(LI_N, LI_DX, LI_KV, 20.0, 100.0)[None] * np.sqrt(LI_DOSE)


def li_object(seed: int):
    """One random single-slice object for the learned initial guess and its
    scan: (amp, phase) each (1, 144, 144) and positions (100, 2).  The scan
    jitter uses seed + 500000 so objects and jitters never share a stream."""
    amp, phase = random_atom_object(LI_H, LI_H, 1, LI_ATOMS, 0.3 / LI_DX, 0.5, seed)
    ny, nx, step, origin, jitter = LI_SCAN
    pos = raster_positions(ny, nx, step, origin, jitter, seed + 500000)
    return amp, phase, pos


def li_neighbourhoods(ny: int = 10, nx: int = 10):
    """3 x 3 neighbourhoods of a row-major ny x nx raster: (nbr, centre) with
    nbr (K, 9) raster indices in row-major (dy, dx) order and centre (K,) the
    middle index, for the (ny-2)(nx-2) interior positions."""
    nbr, ctr = [], []
    for iy in range(1, ny - 1):
        for ix in range(1, nx - 1):
            nbr.append([(iy + a) * nx + ix + b for a in (-1, 0, 1) for b in (-1, 0, 1)])
            ctr.append(iy * nx + ix)
    return np.array(nbr, np.int32), np.array(ctr, np.int64)


def li_targets(phase2d: np.ndarray, centres: np.ndarray) -> np.ndarray:
    """True-phase crops (K, 32, 32) with rows round(cy) - 16 .. round(cy) + 15
    (round half to even) and columns likewise."""
    out = np.empty((len(centres), 32, 32), np.float32)
    for q, (cy, cx) in enumerate(centres):
        y0, x0 = int(np.rint(cy)) - 16, int(np.rint(cx)) - 16
        out[q] = phase2d[y0:y0 + 32, x0:x0 + 32]
    return out
