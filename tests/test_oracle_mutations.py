"""Planted mistakes in the oracle must trip its pins.

Each case patches one piece of the FP64 oracle with a plausible error (a
dropped term, a flipped sign, a missing conjugate, a transposed operand) and
checks that at least one of the pins in test_oracle_pins fails.  Mistakes are
planted only in the CPU oracle, never in GPU code.
"""
import numpy as np
import pytest

from oracle import multislice as ms
from paper_2505_07814_amd import synth
import tests.test_oracle_pins as pins


def _fd_small():
    pins._fd_check(synth.small_case(N=16, S=3, M=2, B=3, seed=16), "gaussian", 0.5, 2, 17)


def _tilt_pin():
    pins.test_tilt_in_vacuum_is_translation(3, 2)


def _propagator_pins():
    pins.test_vacuum_propagator_composition()
    _tilt_pin()


MUTANTS = {
    "tilt sign flipped": (
        "propagator_phase",
        lambda N, dx, lam, dz, tilt: (
            -np.pi * lam * dz * (ms.kgrid(N, dx)[1] ** 2 + ms.kgrid(N, dx)[0] ** 2)
            - 2 * np.pi * dz * (ms.kgrid(N, dx)[1] * np.tan(tilt[1]) + ms.kgrid(N, dx)[0] * np.tan(tilt[0]))),
        _tilt_pin),
    "tilt axes swapped": (
        "propagator_phase",
        lambda N, dx, lam, dz, tilt: (
            -np.pi * lam * dz * (ms.kgrid(N, dx)[1] ** 2 + ms.kgrid(N, dx)[0] ** 2)
            + 2 * np.pi * dz * (ms.kgrid(N, dx)[1] * np.tan(tilt[0]) + ms.kgrid(N, dx)[0] * np.tan(tilt[1]))),
        _tilt_pin),
    "Fresnel sign flipped": (
        "propagator_phase",
        lambda N, dx, lam, dz, tilt: (
            +np.pi * lam * dz * (ms.kgrid(N, dx)[1] ** 2 + ms.kgrid(N, dx)[0] ** 2)
            + 2 * np.pi * dz * (ms.kgrid(N, dx)[1] * np.tan(tilt[1]) + ms.kgrid(N, dx)[0] * np.tan(tilt[0]))),
        pins.test_vacuum_fresnel_gaussian_closed_form),
    "Fresnel k_y term dropped": (
        "propagator_phase",
        lambda N, dx, lam, dz, tilt: (
            -np.pi * lam * dz * (ms.kgrid(N, dx)[1] ** 2 + 0 * ms.kgrid(N, dx)[0])
            + 2 * np.pi * dz * (ms.kgrid(N, dx)[1] * np.tan(tilt[1]) + ms.kgrid(N, dx)[0] * np.tan(tilt[0]))),
        pins.test_vacuum_fresnel_gaussian_closed_form),
    "conjugated transmission": (
        "transmission", lambda a, p: a * np.exp(-1j * p), _fd_small),
    "shift ramp sign flipped": (
        "shift_ramp",
        lambda dr, N: np.exp(+2j * np.pi * (np.fft.fftfreq(N)[:, None] * dr[0]
                                            + np.fft.fftfreq(N)[None, :] * dr[1])),
        pins.test_integer_shift_is_roll_and_sign),
    "non-orthonormal forward FFT": (
        "fft2", lambda x: np.fft.fft2(x), lambda: pins.test_fft_is_orthonormal_dft(8)),
}


def _fft_pins():
    pins.test_fft_is_orthonormal_dft(8)
    pins.test_fft_is_orthonormal_dft(64)


FFT_MUTANTS = {   # wrong butterfly twiddle angles, as functions of (sign, h)
    # the twiddle with the wrong sign
    "conjugated butterfly twiddle": lambda s, h: -s * np.pi * np.arange(h) / h,
    # w = exp(sign 2 pi i / h) instead of exp(sign pi i / h)
    "twiddle angle doubled": lambda s, h: s * 2 * np.pi * np.arange(h) / h,
    # a twiddle index off by one
    "twiddle index shifted": lambda s, h: s * np.pi * (np.arange(h) + 1) / h,
}


@pytest.mark.parametrize("name", list(FFT_MUTANTS) + ["bit reversal skipped", "plain reversal instead of bit reversal"])
def test_planted_fft_mistake_is_caught(name, monkeypatch):
    """Mistakes planted inside the oracle's own radix-2 FFT trip the
    brute-force DFT pins."""
    from oracle import dft
    if name in FFT_MUTANTS:
        tw = FFT_MUTANTS[name]
        monkeypatch.setattr(dft, "_twiddles", lambda h, sign: np.exp(1j * tw(sign, h)))
    elif name == "bit reversal skipped":
        monkeypatch.setattr(dft, "_bit_reverse", lambda n: np.arange(n))
    else:
        monkeypatch.setattr(dft, "_bit_reverse", lambda n: np.arange(n)[::-1].copy())
    with pytest.raises(AssertionError):
        _fft_pins()


@pytest.mark.parametrize("name", list(MUTANTS))
def test_planted_mistake_is_caught(name, monkeypatch):
    attr, bad, pin = MUTANTS[name]
    monkeypatch.setattr(ms, attr, bad)
    with pytest.raises(AssertionError):
        pin()


def test_gradient_mistakes_are_caught(monkeypatch):
    """A gradient written with a missing conjugate fails the difference check."""
    real_grad = ms.gradients

    def bad_gradients(*a, **k):
        g = real_grad(*a, **k)
        g.probe = np.conj(g.probe)          # wrong complex convention
        return g

    monkeypatch.setattr(ms, "gradients", bad_gradients)
    with pytest.raises(AssertionError):
        _fd_small()


# ---------------------------------------------------------------- conv-net oracle
from oracle import convnet as cn              # noqa: E402
import tests.test_oracle_convnet as cpins      # noqa: E402

_conv = cn.conv3x3
_conv_bwd = cn.conv3x3_backward
_round = cn.round_bf16

CONV_MUTANTS = {
    "convolution instead of correlation (flipped kernel)": (
        "conv3x3", lambda a, W, b, s: _conv(a, W[:, :, ::-1, ::-1], b, s),
        lambda: cpins.test_conv_matches_library(1, 9, 3, 5)),
    "stride grid starts at pixel 1": (
        "conv3x3", lambda a, W, b, s: _conv(np.pad(a, ((0, 0), (0, 0), (0, 1), (0, 1)))[:, :, 1:, 1:], W, b, s),
        lambda: cpins.test_conv_matches_library(2, 10, 4, 2)),
    "input gradient with transposed taps": (
        "conv3x3_backward",
        lambda a, W, g, s: (_conv_bwd(a, W[:, :, ::-1, ::-1], g, s)[0],) + _conv_bwd(a, W, g, s)[1:],
        lambda: cpins.test_conv_backward_is_adjoint(1, 8)),
    "weight gradient with swapped tap axes": (
        "conv3x3_backward",
        lambda a, W, g, s: (_conv_bwd(a, W, g, s)[0], _conv_bwd(a, W, g, s)[1].transpose(0, 1, 3, 2),
                            _conv_bwd(a, W, g, s)[2]),
        lambda: cpins.test_conv_backward_is_adjoint(2, 9)),
    "bf16 rounding truncates": (
        "round_bf16",
        lambda x: (np.asarray(x, np.float32).view(np.uint32) & np.uint32(0xFFFF0000)).view(np.float32).astype(np.float64),
        cpins.test_round_bf16_matches_library_and_ties),
}


@pytest.mark.parametrize("name", list(CONV_MUTANTS))
def test_planted_conv_mistake_is_caught(name, monkeypatch):
    attr, bad, pin = CONV_MUTANTS[name]
    monkeypatch.setattr(cn, attr, bad)
    with pytest.raises(AssertionError):
        pin()


def test_missing_relu_mask_is_caught(monkeypatch):
    """Back-propagating through the ReLU without its mask fails autograd parity."""
    monkeypatch.setattr(cn.np, "where", lambda c, x, y: x)
    with pytest.raises(AssertionError):
        cpins.test_net_gradient_matches_autograd()
