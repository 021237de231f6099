"""Pins of the oracle's weighted total loss (Sec. "Optimizers and loss
functions", Eq. 9: w_1 L_Gaussian + w_2 L_Poisson, each data term with its own
power p and its own batch normaliser <I_meas^p>_{D,B}).

Closed forms on constant patterns, difference quotients of dL/dI, central
differences of the total loss through the forward model, and planted mistakes
(a term taking the other term's power, a normaliser shared between the terms).
"""
import numpy as np
import pytest

from oracle import multislice as ms
from paper_2505_07814_amd import synth

EPS = ms.POISSON_EPS


def closed_gauss(c1, c2, p):
    """Eq. 5 on constant arrays: sqrt(<(c1^p - c2^p)^2>) / <c2^p>."""
    return abs(c1 ** p - c2 ** p) / c2 ** p


def closed_poisson(c1, c2, p):
    """Eq. 6 on constant arrays: -(c2^p log(c1^p + eps) - c1^p) / c2^p."""
    return -(c2 ** p * np.log(c1 ** p + EPS) - c1 ** p) / c2 ** p


@pytest.mark.parametrize("w1,w2,pg,pp", [(0.7, 0.3, 0.5, 1.0), (1.0, 2.0, 1.0, 0.5), (0.0, 1.0, 0.5, 1.0)])
def test_weighted_total_on_constant_patterns(w1, w2, pg, pp):
    c1, c2 = 37.0, 52.0
    I = np.full((3, 8, 8), c1)
    Ie = np.full((3, 8, 8), c2)
    terms = [t for t in (("gaussian", w1, pg), ("poisson", w2, pp)) if t[1] > 0]
    L, _ = ms.loss(I, Ie, terms=terms)
    ref = w1 * closed_gauss(c1, c2, pg) + w2 * closed_poisson(c1, c2, pp)
    assert abs(L - ref) < 1e-13 * abs(ref)


def test_weighted_total_gradient_by_differences():
    rng = np.random.default_rng(3)
    I = rng.gamma(2.0, 10.0, (2, 8, 8))
    Ie = rng.poisson(I + 1.0).astype(np.float64) + 0.5
    terms = [("gaussian", 0.6, 0.5), ("poisson", 0.4, 1.0)]
    L, dI = ms.loss(I, Ie, terms=terms)
    h = 1e-5
    for _ in range(6):
        k = tuple(rng.integers(0, s) for s in I.shape)
        Ip, Imn = I.copy(), I.copy()
        Ip[k] += h
        Imn[k] -= h
        fd = (ms.loss(Ip, Ie, terms=terms)[0] - ms.loss(Imn, Ie, terms=terms)[0]) / (2 * h)
        assert abs(fd - dI[k]) <= 1e-6 * abs(dI).max(), (k, fd, dI[k])


def test_weighted_total_through_the_model():
    """Central differences of w_1 L_Gaussian(p=0.5) + w_2 L_Poisson(p=1) (plus
    the PACBED term with the first term's power) along phase, probe, position
    and dz directions against the oracle's gradient."""
    c = synth.small_case(N=16, S=3, M=2, B=3, seed=41)
    lam = synth.wavelength_A(c.kv)
    rng = np.random.default_rng(42)
    I_true = ms.forward(c.amp, c.phase, c.probe, c.pos, c.tilt, c.dz, c.dx, lam)
    probe = c.probe * np.sqrt(50.0 / I_true.max())
    I_meas = rng.poisson(I_true * 50.0 / I_true.max() + 0.5).astype(np.float64) + 0.5
    terms = [("gaussian", 0.8, 0.5), ("poisson", 0.5, 1.0)]
    g = ms.gradients(c.amp, c.phase, probe, c.pos, c.tilt, c.dz, c.dx, lam, I_meas, terms=terms, pacbed_w=0.3)
    base = dict(amp=c.amp, phase=c.phase, probe=probe, pos=c.pos, tilt=c.tilt, dz=c.dz)

    def L(**over):
        a = dict(base, **over)
        return ms.loss_of(a["amp"], a["phase"], a["probe"], a["pos"], a["tilt"], a["dz"], c.dx, lam, I_meas,
                          terms=terms, pacbed_w=0.3)

    assert abs(L() - g.loss) < 1e-13 * abs(g.loss)
    h = 1e-6
    for name, grad in [("phase", g.phase), ("amp", g.amp), ("probe", g.probe), ("pos", g.pos), ("dz", g.dz)]:
        x = base[name]
        if name == "probe":
            d = rng.standard_normal(x.shape) + 1j * rng.standard_normal(x.shape)
            an = np.sum(np.real(np.conj(grad) * d))
        elif name == "dz":
            d, an = 1.0, grad
        else:
            d = rng.standard_normal(np.shape(x))
            an = np.sum(grad * d)
        fd = (8 * (L(**{name: x + h * d}) - L(**{name: x - h * d}))
              - (L(**{name: x + 2 * h * d}) - L(**{name: x - 2 * h * d}))) / (12 * h)
        assert abs(fd - an) <= 2e-7 * abs(fd) + 1e-11, (name, fd, an)
    # each term contributes measurably
    g1 = ms.gradients(c.amp, c.phase, probe, c.pos, c.tilt, c.dz, c.dx, lam, I_meas, terms=terms[:1], pacbed_w=0.3)
    assert np.linalg.norm(g.phase - g1.phase) > 1e-3 * np.linalg.norm(g.phase)


def _closed_pins():
    test_weighted_total_on_constant_patterns(0.7, 0.3, 0.5, 1.0)
    test_weighted_total_on_constant_patterns(1.0, 2.0, 1.0, 0.5)


def test_planted_loss_term_mistakes_are_caught(monkeypatch):
    real = ms.data_term

    # the second term evaluated with the first term's power
    def same_power(I, Im, kind, p, eps=EPS):
        return real(I, Im, kind, 0.5 if kind == "poisson" else p, eps)
    monkeypatch.setattr(ms, "data_term", same_power)
    with pytest.raises(AssertionError):
        _closed_pins()
    monkeypatch.setattr(ms, "data_term", real)

    # one normaliser <I_meas^0.5> shared by both terms
    def shared_norm(I, Im, kind, p, eps=EPS):
        L, dI = real(I, Im, kind, p, eps)
        f = np.mean(np.asarray(Im, np.float64) ** p) / np.mean(np.asarray(Im, np.float64) ** 0.5)
        return L * f, dI * f
    monkeypatch.setattr(ms, "data_term", shared_norm)
    with pytest.raises(AssertionError):
        _closed_pins()
