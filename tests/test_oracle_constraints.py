"""Pins of the FP64 constraints oracle (r_z filter, positivity, probe-mode
orthogonalisation) against a library routine, closed forms and invariants,
and planted mistakes in it that those pins must catch."""
import math

import numpy as np
import pytest
from scipy.ndimage import gaussian_filter1d

from oracle import constraints as oc


def _vol(S=12, H=5, W=6, seed=0):
    return np.random.default_rng(seed).standard_normal((S, H, W))


# ------------------------------------------------------------ r_z filter
@pytest.mark.parametrize("S,sigma", [(12, 0.6), (12, 1.0), (12, 1.3), (30, 2.5), (12, 7.0), (2, 1.0), (1, 1.5)])
def test_rz_matches_library_gaussian_filter(S, sigma):
    """scipy's gaussian_filter1d with mode='reflect' (mirror about the outer
    sample faces) and the same radius is the same convolution, including
    kernels wider than the stack (repeated mirroring)."""
    v = _vol(S)
    R = int(math.ceil(4 * sigma))
    ref = gaussian_filter1d(v, sigma, axis=0, mode="reflect", radius=R)
    assert np.max(np.abs(oc.rz_filter(v, sigma) - ref)) < 1e-13


def test_rz_impulse_response_is_the_normalised_gaussian():
    S, sigma = 41, 1.7
    v = np.zeros((S, 1, 1))
    v[20] = 1.0
    out = oc.rz_filter(v, sigma)[:, 0, 0]
    R = int(math.ceil(4 * sigma))
    k = np.arange(-R, R + 1)
    g = np.exp(-k ** 2 / (2 * sigma ** 2))
    assert np.allclose(out[20 - R:20 + R + 1], g / g.sum(), atol=1e-15)
    assert np.all(out[:20 - R] == 0) and np.all(out[20 + R + 1:] == 0)


def test_rz_keeps_constants_and_mean_and_is_linear():
    v, u = _vol(9, seed=1), _vol(9, seed=2)
    assert np.allclose(oc.rz_filter(np.full((9, 2, 3), 2.5), 1.2), 2.5, atol=1e-14)
    assert np.allclose(oc.rz_filter(2 * v - u, 0.9), 2 * oc.rz_filter(v, 0.9) - oc.rz_filter(u, 0.9), atol=1e-13)
    # mirrored ends: the filter is doubly stochastic, so the depth mean is kept
    assert np.allclose(oc.rz_filter(v, 1.1).mean(0), v.mean(0), atol=1e-13)


def test_rz_does_not_mix_top_and_bottom():
    """Unlike a periodic (Fourier) depth filter, a feature in the first slice
    never reaches the last one when the stack is deeper than the kernel."""
    v = np.zeros((20, 1, 1))
    v[0] = 1.0
    out = oc.rz_filter(v, 1.0)[:, 0, 0]
    assert out[-1] == 0.0 and out[0] > 0.3
    # and the first slice's weight comes back from the mirror: sum is kept
    assert abs(out.sum() - 1.0) < 1e-14


def test_rz_zero_sigma_is_identity():
    v = _vol(5)
    assert np.array_equal(oc.rz_filter(v, 0.0), v)


def test_positivity_clips_only_negatives():
    p = np.array([-1.0, -0.0, 0.0, 1e-9, 0.3])
    assert np.array_equal(oc.positivity(p), [0.0, 0.0, 0.0, 1e-9, 0.3])


# ------------------------------------------------------------ probe orthogonalisation
def _probe(M=3, N=8, seed=3):
    rng = np.random.default_rng(seed)
    return rng.standard_normal((M, N, N)) + 1j * rng.standard_normal((M, N, N))


def test_orthogonalised_modes_are_orthogonal_power_ordered_and_keep_the_incoherent_sum():
    P = _probe(4)
    Q, lam = oc.probe_orthogonalize(P)
    G = oc.probe_overlap(Q)
    assert np.max(np.abs(G - np.diag(np.diag(G)))) < 1e-10 * np.max(np.abs(G))
    assert np.allclose(np.diag(G).real, lam) and np.all(np.diff(lam) <= 0)
    assert np.allclose((np.abs(Q) ** 2).sum(0), (np.abs(P) ** 2).sum(0), rtol=1e-12)
    # the mutual intensity rho(r, r') = sum_k Q_k(r) conj(Q_k(r')) is the same
    Pf, Qf = P.reshape(4, -1), Q.reshape(4, -1)
    assert np.allclose(Qf.T @ np.conj(Qf), Pf.T @ np.conj(Pf), atol=1e-10)


def test_two_mode_powers_match_the_closed_form():
    """Eigenvalues of [[a, b], [conj b, d]]: (a+d)/2 +- sqrt(((a-d)/2)^2 + |b|^2)."""
    P = _probe(2, seed=5)
    a = np.vdot(P[0], P[0]).real
    d = np.vdot(P[1], P[1]).real
    b = np.vdot(P[0], P[1])
    r = math.sqrt(((a - d) / 2) ** 2 + abs(b) ** 2)
    _, lam = oc.probe_orthogonalize(P)
    assert np.allclose(lam, [(a + d) / 2 + r, (a + d) / 2 - r], rtol=1e-12)


def test_orthogonal_input_is_only_reordered():
    """Modes that are already orthogonal with distinct powers come back
    sorted by power, each up to a unit phase factor."""
    N = 8
    y, x = np.mgrid[0:N, 0:N] - (N - 1) / 2            # symmetric grid
    g = np.exp(-(x ** 2 + y ** 2) / 8.0)
    P = np.stack([0.5 * g, 2.0 * x * g, 1.0 * y * g]).astype(np.complex128)     # distinct parities
    Q, lam = oc.probe_orthogonalize(P)
    for k, m in enumerate([1, 2, 0]):                  # powers: x g (4x), y g, 0.5 g
        c = np.vdot(P[m], Q[k]) / np.vdot(P[m], P[m])
        assert abs(abs(c) - 1) < 1e-12
        assert np.allclose(Q[k], c * P[m], atol=1e-12)


def test_apply_order_blur_then_clip():
    amp, ph = _vol(6, seed=7), _vol(6, seed=8)
    P = _probe(2)
    a2, p2, P2 = oc.apply(amp, ph, P, rz_sigma=1.0, phase_positive=True, probe_orthogonal=False)
    assert np.array_equal(p2, np.maximum(oc.rz_filter(ph, 1.0), 0))
    assert np.array_equal(a2, oc.rz_filter(amp, 1.0)) and np.array_equal(P2, P)


# ------------------------------------------------------------ planted mistakes
def _rz_pins():
    for S, sigma in [(12, 1.0), (12, 7.0), (2, 1.0)]:
        test_rz_matches_library_gaussian_filter(S, sigma)
    test_rz_does_not_mix_top_and_bottom()
    test_rz_keeps_constants_and_mean_and_is_linear()


def _orth_pins():
    test_orthogonalised_modes_are_orthogonal_power_ordered_and_keep_the_incoherent_sum()
    test_two_mode_powers_match_the_closed_form()
    test_orthogonal_input_is_only_reordered()


MUTANTS = {
    "periodic depth boundary": ("mirror_index", lambda i, S: i % S, _rz_pins),
    "mirror about the outer sample instead of its face": (
        "mirror_index", lambda i, S: 0 if S == 1 else (lambda j: j if j < S else 2 * S - 2 - j)(i % (2 * S - 2)),
        _rz_pins),
    "taps not normalised": (
        "gaussian_taps",
        lambda sigma, truncate=4.0: np.exp(-np.arange(-math.ceil(truncate * sigma), math.ceil(truncate * sigma) + 1)
                                           ** 2 / (2.0 * sigma * sigma)) if sigma > 0 else np.ones(1),
        _rz_pins),
    "sigma used as variance": (
        "gaussian_taps",
        lambda sigma, truncate=4.0: (lambda w: w / w.sum())(
            np.exp(-np.arange(-math.ceil(truncate * sigma), math.ceil(truncate * sigma) + 1) ** 2 / (2.0 * sigma)))
        if sigma > 0 else np.ones(1),
        _rz_pins),
    "overlap not conjugated": (
        "probe_overlap", lambda probe: (lambda P: P @ P.T)(np.asarray(probe).reshape(probe.shape[0], -1)), _orth_pins),
}


@pytest.mark.parametrize("name", list(MUTANTS))
def test_planted_constraint_mistake_is_caught(name, monkeypatch):
    attr, bad, pin = MUTANTS[name]
    monkeypatch.setattr(oc, attr, bad)
    with pytest.raises(AssertionError):
        pin()


def test_mixing_with_the_wrong_side_of_the_eigenvectors_is_caught(monkeypatch):
    """Q = V^H P instead of V^T P (the conjugate mixing)."""
    def bad(probe):
        A = oc.probe_overlap(probe)
        lam, V = np.linalg.eigh(A)
        order = np.argsort(lam)[::-1]
        lam, V = lam[order], V[:, order]
        P = np.asarray(probe, np.complex128).reshape(probe.shape[0], -1)
        return (np.conj(V).T @ P).reshape(probe.shape), lam
    monkeypatch.setattr(oc, "probe_orthogonalize", bad)
    with pytest.raises(AssertionError):
        _orth_pins()


# ------------------------------------------------------------ sparsity term of the loss
from oracle import multislice as ms                       # noqa: E402
from paper_2505_07814_amd import synth                    # noqa: E402


def test_sparse_term_constant_phase_closed_form():
    """A constant phase c gives L = |c|; each pixel's gradient is
    sign(c) * (patches covering it) / (B S N^2)."""
    S, H, W, N = 3, 40, 44, 16
    pos = np.array([[12.0, 12.0], [20.3, 25.6], [27.0, 30.0]])
    for c in (0.7, -0.4):
        L, g = ms.sparse_term(np.full((S, H, W), c), pos, N)
        assert abs(L - abs(c)) < 1e-15
        cover = np.zeros((H, W))
        for rho in pos:
            t = np.round(rho).astype(int) - N // 2
            cover[t[0]:t[0] + N, t[1]:t[1] + N] += 1
        assert np.allclose(g, np.sign(c) * cover[None] / (len(pos) * S * N * N), atol=1e-18)
    L0, g0 = ms.sparse_term(np.zeros((S, H, W)), pos, N)
    assert L0 == 0.0 and not np.any(g0)                  # sign(0) = 0


def test_total_loss_with_sparsity_matches_central_differences():
    """The data term plus 0.1 x the sparsity term: the phase gradient against
    fourth-order central differences along random directions (phase kept
    away from 0, where |phase| has its kink)."""
    c = synth.small_case(N=16, S=2, M=2, B=3, H=16 + 11, W=16 + 13, seed=61)
    lam = synth.wavelength_A(c.kv)
    rng = np.random.default_rng(62)
    phase = np.abs(c.phase) + 0.3
    phase[:, ::3, ::2] *= -1                              # both signs present
    I_true = ms.forward(c.amp, phase, c.probe, c.pos, c.tilt, c.dz, c.dx, lam)
    probe = c.probe * np.sqrt(50.0 / I_true.max())
    I_meas = rng.poisson(I_true * 50.0 / I_true.max() + 0.01).astype(np.float64) + 0.5
    args = (c.amp, phase, probe, c.pos, c.tilt, c.dz, c.dx, lam, I_meas)
    g = ms.gradients(*args, sparse_w=0.1)
    g0 = ms.gradients(*args)
    Ls, gs = ms.sparse_term(phase, c.pos, 16)
    assert abs(g.loss - (g0.loss + 0.1 * Ls)) < 1e-15
    h = 1e-6
    for _ in range(4):
        d = rng.standard_normal(phase.shape)
        f = lambda x: ms.loss_of(c.amp, x, probe, c.pos, c.tilt, c.dz, c.dx, lam, I_meas, sparse_w=0.1)
        fd = (8 * (f(phase + h * d) - f(phase - h * d)) - (f(phase + 2 * h * d) - f(phase - 2 * h * d))) / (12 * h)
        an = np.sum(g.phase * d)
        assert abs(fd - an) <= 1e-6 * abs(an) + 1e-9, (fd, an)
    # and the sparsity part alone is what it adds
    assert np.allclose(g.phase - g0.phase, 0.1 * gs, atol=1e-18)


def test_sparse_term_mistakes_are_caught(monkeypatch):
    """Dropping the slice count from the normaliser, or the sign, trips the pins."""
    real = ms.sparse_term

    def no_slices(phase, pos, N):
        L, g = real(phase, pos, N)
        S = np.asarray(phase).shape[0]
        return L * S, g * S
    monkeypatch.setattr(ms, "sparse_term", no_slices)
    with pytest.raises(AssertionError):
        test_sparse_term_constant_phase_closed_form()

    def unsigned(phase, pos, N):
        L, g = real(phase, pos, N)
        return L, np.abs(g)
    monkeypatch.setattr(ms, "sparse_term", unsigned)
    with pytest.raises(AssertionError):
        test_sparse_term_constant_phase_closed_form()


# ------------------------------------------------------------ k_z filter
def _plane(S, H, W, f, dx, dz):
    z, y, x = np.meshgrid(np.arange(S), np.arange(H), np.arange(W), indexing="ij")
    kz, ky, kx = f[0] / (S * dz), f[1] / (H * dx), f[2] / (W * dx)
    return np.cos(2 * np.pi * (kz * z * dz + ky * y * dx + kx * x * dx)), (kz, ky, kx)


@pytest.mark.parametrize("f", [(1, 2, 3), (5, 0, 1), (0, 4, 4), (2, 7, -9)])
def test_kz_plane_waves_are_eigenfunctions(f):
    """A real plane wave on the grid comes back multiplied by the closed-form
    W_a at its wave vector (W_a is even, so the cosine stays a cosine)."""
    S, H, W, dx, dz, beta, alpha = 12, 20, 18, 0.3, 7.0, 0.7, 0.2
    v, (kz, ky, kx) = _plane(S, H, W, f, dx, dz)
    kr2 = kx ** 2 + ky ** 2
    w = (1 - 2 / np.pi * math.atan(beta ** 2 * kz ** 2 / (kr2 + 1e-3))) * math.exp(-alpha * kr2)
    assert np.allclose(oc.kz_filter(v, beta, alpha, dx, dz), w * v, atol=1e-12)


def test_kz_identity_and_depth_constant_fields():
    v = _vol(6, 10, 12)
    assert np.allclose(oc.kz_filter(v, 0.0, 0.0, 0.2, 5.0), v, atol=1e-13)
    # k_z = 0 everywhere for a depth-constant field: W = 1, any beta
    d = np.repeat(_vol(1, 10, 12, seed=4), 6, axis=0)
    assert np.allclose(oc.kz_filter(d, 3.0, 0.0, 0.2, 5.0), d, atol=1e-13)


def test_kz_filter_mistakes_are_caught(monkeypatch):
    real = oc.kz_weight
    monkeypatch.setattr(oc, "kz_weight", lambda S, H, W, beta, alpha, dx, dz, eps=1e-3:
                        real(S, H, W, beta, alpha, dx, 1.0, eps))                       # dz units dropped
    with pytest.raises(AssertionError):
        test_kz_plane_waves_are_eigenfunctions((1, 2, 3))
    monkeypatch.setattr(oc, "kz_weight", lambda S, H, W, beta, alpha, dx, dz, eps=1e-3:
                        real(S, H, W, beta, 0.0, dx, dz, eps))                          # lateral blur dropped
    with pytest.raises(AssertionError):
        test_kz_plane_waves_are_eigenfunctions((1, 2, 3))
