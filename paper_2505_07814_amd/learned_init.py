"""Learned initial guess for the multislice reconstruction.

Training pairs come from the library's own forward model (ptyr_forward) on
random single-slice Gaussian-atom objects, with Poisson counting noise: the
diffraction patterns of each 3 x 3 neighbourhood of a 10 x 10 raster (step 8
px) and the true phase of the 32 x 32 patch centred on the middle position.
The conv net (include/ptyr_cnn.h) is trained with the library's BF16
matrix-core gradient kernels and Adam; at inference its patches are stitched
into an initial phase, and the multislice reconstruction (ptyr_step) starts
from that instead of the plain initial object of the paper (unit amplitude,
near-zero random phase; Sec. "Preprocessing and initialization").

Everything on the device runs in libptyr; PyTorch provides memory, streams,
Poisson sampling of the synthetic data and the batch gathers of the training
loop.
"""
from __future__ import annotations

import math
import time
from dataclasses import dataclass, field

import numpy as np
import torch

from . import synth
from .cnn import ConvInit, init_params
from .ptyr import AdamState, Engine


@dataclass
class Dataset:
    patterns: torch.Tensor       # (n_obj * 100, 64, 64) float32, Poisson counts
    nbr: torch.Tensor            # (n_obj * 64, 9) int32, rows of `patterns`
    target: torch.Tensor         # (n_obj * 64, 32, 32) float32 true phase
    seconds: float = 0.0


def make_dataset(n_obj: int, device, seed0: int = synth.LI_OBJECT_SEED0, poisson_seed: int = 7) -> Dataset:
    """Simulate n_obj random objects (seeds seed0 + i) through the library's
    forward model and sample Poisson counts."""
    t0 = time.perf_counter()
    lam = synth.wavelength_A(synth.LI_KV)
    probe = torch.from_numpy(synth.li_probe().astype(np.complex64)).to(device)
    H = synth.LI_H
    n_scan = synth.LI_SCAN[0] * synth.LI_SCAN[1]
    eng = Engine(synth.LI_N, 1, 1, H, H, n_scan, synth.LI_DX, lam, device=device)
    nb, ctr = synth.li_neighbourhoods(synth.LI_SCAN[0], synth.LI_SCAN[1])
    K = len(nb)
    patterns = torch.empty((n_obj * n_scan, 64, 64), dtype=torch.float32, device=device)
    target = np.empty((n_obj * K, 32, 32), np.float32)
    nbr = np.empty((n_obj * K, 9), np.int32)
    gen = torch.Generator(device=device)
    gen.manual_seed(poisson_seed)
    tilt = torch.zeros((n_scan, 2), dtype=torch.float32, device=device)
    dz = torch.tensor([synth.LI_DZ], dtype=torch.float32, device=device)
    for i in range(n_obj):
        amp, phase, pos = synth.li_object(seed0 + i)
        I = eng.forward(torch.from_numpy(amp.astype(np.float32)).to(device),
                        torch.from_numpy(phase.astype(np.float32)).to(device), probe,
                        torch.from_numpy(pos.astype(np.float32)).to(device), tilt, dz)
        patterns[i * n_scan:(i + 1) * n_scan] = torch.poisson(I, generator=gen)
        target[i * K:(i + 1) * K] = synth.li_targets(phase[0], pos[ctr])
        nbr[i * K:(i + 1) * K] = nb + i * n_scan
    eng.sync()
    return Dataset(patterns, torch.from_numpy(nbr).to(device), torch.from_numpy(target).to(device),
                   time.perf_counter() - t0)


@dataclass
class TrainResult:
    params: torch.Tensor
    losses: list = field(default_factory=list)     # mean training loss per epoch
    seconds: float = 0.0
    steps: int = 0


def train(data: Dataset, epochs: int, batch: int = 256, lr: float = 1e-3, seed: int = 0,
          net: ConvInit | None = None, log=None) -> TrainResult:
    """Adam on the mean-squared phase error, cosine-decayed learning rate,
    seeded shuffles; the last partial batch of an epoch is dropped."""
    dev = data.patterns.device
    net = net or ConvInit(batch, device=dev)
    params = torch.from_numpy(init_params(seed)).to(dev)
    grad = torch.zeros_like(params)
    m = torch.zeros_like(params)
    v = torch.zeros_like(params)
    loss = torch.zeros(1, dtype=torch.float64, device=dev)
    n = data.nbr.shape[0]
    nb = n // batch
    total = epochs * nb
    rng = np.random.default_rng(seed + 1)
    res = TrainResult(params)
    torch.cuda.synchronize(dev)
    t0 = time.perf_counter()
    step = 0
    for ep in range(epochs):
        perm = torch.from_numpy(rng.permutation(n)).to(dev)
        acc = torch.zeros(1, dtype=torch.float64, device=dev)
        for b in range(nb):
            sel = perm[b * batch:(b + 1) * batch]
            grad.zero_()
            net.gradient(params, data.patterns, data.nbr[sel].contiguous(), data.target[sel].contiguous(), grad, loss)
            step += 1
            lr_t = lr * 0.5 * (1.0 + math.cos(math.pi * (step - 1) / total))
            net.adam(params, grad, m, v, step, lr_t)
            acc += loss
        net.sync()
        res.losses.append(float(acc.item()) / nb)
        if log:
            log(f"epoch {ep + 1}/{epochs}: mean loss {res.losses[-1]:.3e} ({time.perf_counter() - t0:.1f} s)")
    torch.cuda.synchronize(dev)
    res.seconds = time.perf_counter() - t0
    res.steps = step
    return res


def roi_mask(probe: np.ndarray, pos: np.ndarray, H: int, W: int) -> np.ndarray:
    """Illuminated region: pixels where the probe intensity summed over all
    scan positions reaches half its maximum."""
    N = probe.shape[-1]
    ill = np.zeros((H, W))
    pint = np.sum(np.abs(probe) ** 2, axis=0)
    for p in pos:
        y0, x0 = np.rint(p).astype(int) - N // 2
        ill[y0:y0 + N, x0:x0 + N] += pint
    return ill >= 0.5 * ill.max()


def rms_phase_error(phase: np.ndarray, truth: np.ndarray, roi: np.ndarray) -> float:
    """RMS of the phase difference over the ROI after removing its mean (the
    reconstruction fixes the phase only up to a constant)."""
    d = (np.asarray(phase, np.float64) - truth)[roi]
    d = d - d.mean()
    return float(np.sqrt(np.mean(d * d)))


def rms_phase_error_dev(phase: torch.Tensor, truth: torch.Tensor, roi: torch.Tensor) -> float:
    """rms_phase_error on device tensors (truth float64, roi bool): the same
    float64 arithmetic, only the scalar is read back."""
    d = (phase.double() - truth)[roi]
    d = d - d.mean()
    return float(torch.sqrt(torch.mean(d * d)))


@dataclass
class EvalCase:
    amp: np.ndarray
    phase: np.ndarray
    pos: np.ndarray
    probe: np.ndarray
    patterns: torch.Tensor       # (100, 64, 64) measured counts on the device
    roi: np.ndarray


def eval_case(device, seed: int = synth.LI_EVAL_SEED, poisson_seed: int = 11) -> EvalCase:
    amp, phase, pos = synth.li_object(seed)
    probe = synth.li_probe()
    lam = synth.wavelength_A(synth.LI_KV)
    n = pos.shape[0]
    eng = Engine(synth.LI_N, 1, 1, synth.LI_H, synth.LI_H, n, synth.LI_DX, lam, device=device)
    T = lambda a, dt: torch.from_numpy(np.ascontiguousarray(a).astype(dt)).to(device)
    I = eng.forward(T(amp, np.float32), T(phase, np.float32), T(probe, np.complex64), T(pos, np.float32),
                    torch.zeros((n, 2), dtype=torch.float32, device=device),
                    torch.tensor([synth.LI_DZ], dtype=torch.float32, device=device))
    gen = torch.Generator(device=device)
    gen.manual_seed(poisson_seed)
    meas = torch.poisson(I, generator=gen)
    eng.sync()
    return EvalCase(amp, phase, pos, probe, meas, roi_mask(probe, pos, synth.LI_H, synth.LI_H))


def learned_phase(net: ConvInit, params: torch.Tensor, case: EvalCase, plain: torch.Tensor) -> torch.Tensor:
    """Network patches for the interior neighbourhoods of the scan, stitched
    over the plain initial phase (which stays where no patch reaches)."""
    dev = plain.device
    nb, ctr = synth.li_neighbourhoods(synth.LI_SCAN[0], synth.LI_SCAN[1])
    patches = net.forward(params, case.patterns, torch.from_numpy(nb).to(dev))
    centres = torch.from_numpy(case.pos[ctr].astype(np.float32)).to(dev)
    img = plain.clone()
    net.stitch(patches, centres, img)
    return img


@dataclass
class ReconResult:
    errors: list                 # RMS phase error after each iteration (errors[0]: initial)
    seconds: list                # wall time after each iteration (seconds[0]: initial guess cost)
    iterations_to_target: int | None
    seconds_to_target: float | None


def reconstruct(case: EvalCase, phase0: torch.Tensor, iterations: int, target: float = 0.02, lr: float = 1e-2,
                batch: int = 20, seed: int = 6, setup_seconds: float = 0.0) -> ReconResult:
    """Gradient reconstruction of object amplitude and phase (known probe and
    positions) with ptyr_step: Gaussian amplitude loss, Adam, `batch`
    positions per step in a seeded random order, one iteration = one pass over
    the scan.  The error is measured after every iteration (on the device, one
    scalar read back); the clock includes setup_seconds (the cost of computing
    phase0), the upload of each iteration's order and the error read-back."""
    dev = phase0.device
    lam = synth.wavelength_A(synth.LI_KV)
    n = case.pos.shape[0]
    H = synth.LI_H
    eng = Engine(synth.LI_N, 1, 1, H, H, batch, synth.LI_DX, lam, n_scan=n, device=dev)
    T = lambda a, dt: torch.from_numpy(np.ascontiguousarray(a).astype(dt)).to(dev)
    st = AdamState(torch.ones((1, H, H), dtype=torch.float32, device=dev), phase0.reshape(1, H, H).clone(),
                   T(case.probe, np.complex64), T(case.pos, np.float32),
                   torch.zeros((n, 2), dtype=torch.float32, device=dev),
                   torch.tensor([synth.LI_DZ], dtype=torch.float32, device=dev))
    rates = dict(amp=lr, phase=lr, probe=0.0, pos=0.0, tilt=0.0, dz=0.0)
    rng = np.random.default_rng(seed)
    truth = torch.from_numpy(np.ascontiguousarray(case.phase[0], np.float64)).to(dev)
    roi = torch.from_numpy(np.ascontiguousarray(case.roi)).to(dev)
    step = eng.bind_step(st, case.patterns, rates)
    errors = [rms_phase_error_dev(st.phase[0], truth, roi)]
    seconds = [setup_seconds]
    hit_it, hit_s = (0, setup_seconds) if errors[0] <= target else (None, None)
    torch.cuda.synchronize(dev)
    t0 = time.perf_counter() - setup_seconds
    for it in range(iterations):
        # one upload of the iteration's order; the batches are views of it
        perm = torch.from_numpy(rng.permutation(n).astype(np.int32)).to(dev)
        for b in range(0, n - batch + 1, batch):
            step(perm[b:b + batch])
        e = rms_phase_error_dev(st.phase[0], truth, roi)                       # synchronises
        errors.append(e)
        seconds.append(time.perf_counter() - t0)
        if hit_it is None and e <= target:
            hit_it, hit_s = it + 1, seconds[-1]
    eng.sync()
    return ReconResult(errors, seconds, hit_it, hit_s)
