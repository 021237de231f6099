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
