"""Pins of the FP64 oracle with mixed object modes (amplitude / phase of
shape n_obj x S x H x W; the intensity sums over probe and object modes):
reduction to the single-mode path, a closed form for repeated modes, and
central differences of the loss for every parameter block."""
import numpy as np
import pytest

from oracle import multislice as ms
from paper_2505_07814_amd import synth


def _case(seed=81):
    c = synth.small_case(N=16, S=2, M=2, B=3, H=16 + 11, W=16 + 13, seed=seed)
    rng = np.random.default_rng(seed + 1)
    amp2 = np.stack([c.amp, c.amp * rng.uniform(0.8, 1.0, c.amp.shape)])
    ph2 = np.stack([c.phase, 0.7 * c.phase + 0.1 * rng.standard_normal(c.phase.shape)])
    return c, amp2, ph2


def test_one_object_mode_is_the_plain_path():
    c, _, _ = _case()
    lam = synth.wavelength_A(c.kv)
    I3 = ms.forward(c.amp, c.phase, c.probe, c.pos, c.tilt, c.dz, c.dx, lam)
    I4 = ms.forward(c.amp[None], c.phase[None], c.probe, c.pos, c.tilt, c.dz, c.dx, lam)
    assert np.array_equal(I3, I4)


def test_repeated_object_mode_doubles_the_intensity():
    c, _, _ = _case()
    lam = synth.wavelength_A(c.kv)
    I1 = ms.forward(c.amp, c.phase, c.probe, c.pos, c.tilt, c.dz, c.dx, lam)
    I2 = ms.forward(np.stack([c.amp, c.amp]), np.stack([c.phase, c.phase]), c.probe, c.pos, c.tilt, c.dz, c.dx, lam)
    assert np.allclose(I2, 2 * I1, rtol=1e-14, atol=0)


def _fd(c, amp2, ph2, names=("amp", "phase", "probe", "pos", "tilt", "dz")):
    lam = synth.wavelength_A(c.kv)
    rng = np.random.default_rng(83)
    I_true = ms.forward(amp2, ph2, c.probe, c.pos, c.tilt, c.dz, c.dx, lam)
    probe = c.probe * np.sqrt(50.0 / I_true.max())
    I_meas = rng.poisson(I_true * 50.0 / I_true.max() + 0.01).astype(np.float64) + 0.5
    g = ms.gradients(amp2, ph2, probe, c.pos, c.tilt, c.dz, c.dx, lam, I_meas)
    base = dict(amp=amp2, phase=ph2, probe=probe, pos=c.pos, tilt=c.tilt, dz=c.dz)

    def L(**over):
        a = dict(base, **over)
        return ms.loss_of(a["amp"], a["phase"], a["probe"], a["pos"], a["tilt"], a["dz"], c.dx, lam, I_meas)
    grads = dict(amp=g.amp, phase=g.phase, probe=g.probe, pos=g.pos, tilt=g.tilt, dz=g.dz)
    for name in names:
        x = base[name]
        if name == "probe":
            d = rng.standard_normal(x.shape) + 1j * rng.standard_normal(x.shape)
            an = np.sum(np.real(np.conj(grads[name]) * d))
        elif name == "dz":
            d, an = 1.0, grads[name]
        else:
            d = rng.standard_normal(np.shape(x))
            an = np.sum(grads[name] * d)
        h = 1e-7 if name == "tilt" else 1e-6
        fd = (8 * (L(**{name: x + h * d}) - L(**{name: x - h * d}))
              - (L(**{name: x + 2 * h * d}) - L(**{name: x - 2 * h * d}))) / (12 * h)
        assert abs(fd - an) <= 1e-5 * abs(an) + 1e-9, (name, fd, an)


def test_two_object_modes_match_central_differences():
    c, amp2, ph2 = _case()
    _fd(c, amp2, ph2)


def test_probe_gradient_of_one_mode_only_is_caught(monkeypatch):
    """Taking the probe gradient from the first object mode alone fails."""
    real = ms._adjoint
    calls = {"n": 0}

    def first_only(*args):
        out = list(real(*args))
        calls["n"] += 1
        if calls["n"] > 1:
            out[2] = np.zeros_like(out[2])
        return tuple(out)
    monkeypatch.setattr(ms, "_adjoint", first_only)
    c, amp2, ph2 = _case()
    with pytest.raises(AssertionError):
        _fd(c, amp2, ph2, names=("probe",))
