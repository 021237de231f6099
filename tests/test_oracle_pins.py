"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Each test checks the oracle against something other than itself: a brute-force
DFT, an exact invariant of the forward model (unitarity, composition of
propagators, tilt = translation, unit-object limit), a closed-form loss value,
central finite differences of the oracle's own loss, or a library routine that
a special case reduces to.
"""
import json
import os

import numpy as np
import pytest

from oracle import multislice as ms
from oracle.adam import adam_step
from paper_2505_07814_amd import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ------------------------------------------------------------------ FFT
def brute_dft2(f, sign):
    N = f.shape[-1]
    n = np.arange(N)
    W = np.exp(sign * 2j * np.pi * np.outer(n, n) / N) / np.sqrt(N)
    return W @ f @ W.T


@pytest.mark.parametrize("N", [4, 8, 16, 64, 128, 256])
def test_fft_is_orthonormal_dft(N):
    """The oracle's radix-2 FFT equals the DFT written out as a matrix product
    (the definition, O(N^3) for a 2-D field) at every size the path uses."""
    rng = np.random.default_rng(N)
    f = rng.standard_normal((N, N)) + 1j * rng.standard_normal((N, N))
    tol = 1e-13 * max(1.0, np.sqrt(N) / 4)
    assert np.max(np.abs(ms.fft2(f) - brute_dft2(f, -1))) < tol
    assert np.max(np.abs(ms.ifft2(f) - brute_dft2(f, +1))) < tol
    assert np.max(np.abs(ms.ifft2(ms.fft2(f)) - f)) < tol


@pytest.mark.parametrize("N", [64, 128, 256])
def test_fft_matches_library_fft(N):
    """Test-time library pin: numpy's pocketfft, orthonormal, on a stack of
    fields (the oracle itself never calls it)."""
    rng = np.random.default_rng(100 + N)
    f = rng.standard_normal((3, N, N)) + 1j * rng.standard_normal((3, N, N))
    assert np.max(np.abs(ms.fft2(f) - np.fft.fft2(f, norm="ortho"))) < 1e-13
    assert np.max(np.abs(ms.ifft2(f) - np.fft.ifft2(f, norm="ortho"))) < 1e-13


@pytest.mark.parametrize("n", [1, 2, 3, 5, 6, 12, 20, 40, 640])
def test_dft_any_length_is_definition(n):
    """Lengths with an odd factor (the k_z filter's 12 and 640) against the
    definition summed term by term, and numpy as a library pin; the 3-D
    transforms against numpy's fftn / ifftn."""
    from oracle import dft
    rng = np.random.default_rng(n)
    x = rng.standard_normal((2, n)) + 1j * rng.standard_normal((2, n))
    k = np.arange(n)
    for sign in (-1, 1):
        ref = np.array([[np.sum(row * np.exp(sign * 2j * np.pi * k * kk / n)) for kk in range(n)] for row in x])
        got = dft.dft(x, -1, sign)
        assert np.max(np.abs(got - ref)) < 1e-12 * n
    assert np.max(np.abs(dft.dft(x, -1, -1) - np.fft.fft(x))) < 1e-12 * n
    v = rng.standard_normal((6, 10, n))
    assert np.max(np.abs(dft.fftn(v) - np.fft.fftn(v))) < 1e-12 * v.size
    assert np.max(np.abs(dft.ifftn(v) - np.fft.ifftn(v))) < 1e-14 * n
    assert np.max(np.abs(dft.fftfreq(n, 0.3) - np.fft.fftfreq(n, 0.3))) == 0.0


def test_fftshift_is_library_shift():
    from oracle import dft
    for shape in [(4, 4), (2, 8, 6), (64, 64)]:
        x = np.arange(np.prod(shape)).reshape(shape)
        assert np.array_equal(dft.fftshift2(x), np.fft.fftshift(x, axes=(-2, -1)))
        assert np.array_equal(dft.ifftshift2(dft.fftshift2(x)), x)


# ------------------------------------------------------------------ shift
def test_integer_shift_is_roll_and_sign():
    rng = np.random.default_rng(1)
    N = 16
    P = rng.standard_normal((N, N)) + 1j * rng.standard_normal((N, N))
    for d in [(2, -3), (-5, 1), (8, 8)]:
        got = ms.ifft2(ms.fft2(P) * ms.shift_ramp(np.array(d, float), N))
        assert np.max(np.abs(got - np.roll(P, d, axis=(0, 1)))) < 1e-12


def test_subpixel_shift_keeps_spectrum_modulus_and_composes():
    rng = np.random.default_rng(2)
    N = 16
    P = rng.standard_normal((N, N)) + 1j * rng.standard_normal((N, N))
    a, b = np.array([0.3, -0.2]), np.array([-0.45, 0.35])
    Sa = ms.ifft2(ms.fft2(P) * ms.shift_ramp(a, N))
    assert np.allclose(np.abs(ms.fft2(Sa)), np.abs(ms.fft2(P)), atol=1e-12)
    SbSa = ms.ifft2(ms.fft2(Sa) * ms.shift_ramp(b, N))
    Sab = ms.ifft2(ms.fft2(P) * ms.shift_ramp(a + b, N))
    assert np.max(np.abs(SbSa - Sab)) < 1e-12


def test_position_rounding_is_half_even_and_centred():
    t, dr = ms.split_position([10.5, 11.5], 8)
    assert list(t) == [10 - 4, 12 - 4] and np.allclose(dr, [0.5, -0.5])
    t, dr = ms.split_position([20.3, 19.7], 16)
    assert list(t) == [20 - 8, 20 - 8] and np.allclose(dr, [0.3, -0.3])


def test_translation_covariance_of_forward():
    """Moving the position by one pixel equals moving the object the other way."""
    c = synth.small_case(N=16, S=3, M=2, B=2, seed=11)
    lam = synth.wavelength_A(c.kv)
    I0 = ms.forward(c.amp, c.phase, c.probe, c.pos + [1.0, -2.0], c.tilt, c.dz, c.dx, lam)
    amp_r = np.roll(c.amp, (-1, 2), axis=(1, 2))
    ph_r = np.roll(c.phase, (-1, 2), axis=(1, 2))
    I1 = ms.forward(amp_r, ph_r, c.probe, c.pos, c.tilt, c.dz, c.dx, lam)
    assert np.max(np.abs(I0 - I1)) <= 1e-12 * np.max(I0)


# ------------------------------------------------------------------ propagator
def _vacuum(S, H=40, W=44):
    return np.ones((S, H, W)), np.zeros((S, H, W))


def test_vacuum_propagator_composition():
    """Unit object: S=3 with spacing a equals S=2 with spacing 2a (H(a)H(a)=H(2a)),
    including the tilt term."""
    c = synth.small_case(N=16, S=3, M=2, B=1, seed=3)
    lam = synth.wavelength_A(c.kv)
    a3, p3 = _vacuum(3)
    a2, p2 = _vacuum(2)
    e3 = ms.exit_waves(a3, p3, c.probe, c.pos[0], c.tilt[0], 13.0, c.dx, lam)
    e2 = ms.exit_waves(a2, p2, c.probe, c.pos[0], c.tilt[0], 26.0, c.dx, lam)
    assert np.max(np.abs(e3 - e2)) < 1e-12 * np.max(np.abs(e2))
    # and two different gaps compose through explicit propagators
    Ha = ms.propagator(16, c.dx, lam, 5.0, c.tilt[0])
    Hb = ms.propagator(16, c.dx, lam, 8.0, c.tilt[0])
    Hab = ms.propagator(16, c.dx, lam, 13.0, c.tilt[0])
    assert np.max(np.abs(Ha * Hb - Hab)) < 1e-12


def test_vacuum_fresnel_gaussian_closed_form():
    """A Gaussian packet exp(-r^2/2s^2) propagated a distance z by the Fresnel
    kernel exp(-i pi lam z |k|^2) is (s^2/s_z^2) exp(-r^2/2 s_z^2) with
    s_z^2 = s^2 + i lam z / (2 pi) (the paraxial free-space solution)."""
    N, dx, lam, z, sig = 128, 0.2, synth.wavelength_A(300.0), 150.0, 1.2
    yy, xx = (np.mgrid[0:N, 0:N] - N // 2) * dx
    r2 = yy ** 2 + xx ** 2
    packet = np.exp(-r2 / (2 * sig ** 2))[None].astype(np.complex128)
    a, p = _vacuum(2, 2 * N, 2 * N)
    e = ms.exit_waves(a, p, packet, np.array([N, N], float), np.zeros(2), z, dx, lam)[0]
    sz2 = sig ** 2 + 1j * lam * z / (2 * np.pi)
    ref = (sig ** 2 / sz2) * np.exp(-r2 / (2 * sz2))
    assert np.max(np.abs(e - ref)) < 1e-12


def test_zero_spacing_is_projection_approximation():
    c = synth.small_case(N=16, S=4, M=2, B=1, seed=4)
    lam = synth.wavelength_A(c.kv)
    e = ms.exit_waves(c.amp, c.phase, c.probe, c.pos[0], c.tilt[0], 0.0, c.dx, lam)
    t, dr = ms.split_position(c.pos[0], 16)
    Pj = ms.ifft2(ms.fft2(c.probe) * ms.shift_ramp(dr, 16))
    Oprod = np.prod(ms.crop(c.amp * np.exp(1j * c.phase), t, 16), axis=0)
    assert np.max(np.abs(e - Oprod * Pj)) < 1e-12 * np.max(np.abs(e))


@pytest.mark.parametrize("n,S", [(3, 2), (-2, 3), (1, 4)])
def test_tilt_in_vacuum_is_translation(n, S):
    """dz*tan(theta_x)/dx = n: each gap translates the wave by n pixels, so the
    vacuum exit wave is the untilted one rolled by -(S-1)*n along x (and y)."""
    c = synth.small_case(N=16, S=S, M=1, B=1, seed=5)
    lam = synth.wavelength_A(c.kv)
    dz = 30.0
    th = np.arctan(n * c.dx / dz)
    a, p = _vacuum(S)
    e0 = ms.exit_waves(a, p, c.probe, c.pos[0], np.array([0.0, 0.0]), dz, c.dx, lam)
    ex = ms.exit_waves(a, p, c.probe, c.pos[0], np.array([0.0, th]), dz, c.dx, lam)
    ey = ms.exit_waves(a, p, c.probe, c.pos[0], np.array([th, 0.0]), dz, c.dx, lam)
    sh = -(S - 1) * n
    assert np.max(np.abs(ex - np.roll(e0, sh, axis=2))) < 1e-11
    assert np.max(np.abs(ey - np.roll(e0, sh, axis=1))) < 1e-11


# ------------------------------------------------------------------ intensities
def test_unitarity_for_pure_phase_object():
    c = synth.small_case(N=16, S=4, M=3, B=3, seed=6)
    lam = synth.wavelength_A(c.kv)
    I = ms.forward(np.ones_like(c.amp), c.phase, c.probe, c.pos, c.tilt, c.dz, c.dx, lam)
    total = np.sum(np.abs(c.probe) ** 2)
    assert np.allclose(I.sum(axis=(1, 2)), total, rtol=1e-12)


@pytest.mark.parametrize("S", [1, 3])
def test_unit_object_limit_is_probe_spectrum(S):
    c = synth.small_case(N=16, S=S, M=2, B=3, seed=8)
    lam = synth.wavelength_A(c.kv)
    a, p = _vacuum(S)
    I = ms.forward(a, p, c.probe, c.pos, c.tilt, c.dz, c.dx, lam)
    ref = np.fft.fftshift(np.sum(np.abs(brute_dft2(c.probe, -1)) ** 2, axis=0))
    for j in range(len(I)):
        assert np.max(np.abs(I[j] - ref)) < 1e-12 * ref.max()


def test_single_slice_is_fft_of_product():
    """S=1, integer position: I = |F[O_patch * P]|^2 written with a brute DFT."""
    c = synth.small_case(N=8, S=1, M=1, B=1, seed=9, jitter=0.0)
    lam = synth.wavelength_A(c.kv)
    rho = np.round(c.pos[0])
    I = ms.forward(c.amp, c.phase, c.probe, rho[None], c.tilt[:1], c.dz, c.dx, lam)[0]
    t = rho.astype(int) - 4
    Op = c.amp[0, t[0]:t[0] + 8, t[1]:t[1] + 8] * np.exp(1j * c.phase[0, t[0]:t[0] + 8, t[1]:t[1] + 8])
    ref = np.fft.fftshift(np.abs(brute_dft2(Op * c.probe[0], -1)) ** 2)
    assert np.max(np.abs(I - ref)) < 1e-12 * ref.max()


def test_out_of_bounds_patch_raises():
    c = synth.small_case(N=16, S=1, M=1, B=1, seed=10)
    lam = synth.wavelength_A(c.kv)
    with pytest.raises(ValueError):
        ms.forward(c.amp, c.phase, c.probe, np.array([[7.0, 20.0]]), c.tilt[:1], c.dz, c.dx, lam)


# ------------------------------------------------------------------ loss
def test_gaussian_loss_closed_forms():
    rng = np.random.default_rng(12)
    I = rng.uniform(0.5, 3, (2, 8, 8))
    assert ms.loss(I, I, "gaussian")[0] == 0.0
    c1, c2 = 2.25, 4.0
    L, _ = ms.loss(np.full((3, 4, 4), c1), np.full((3, 4, 4), c2), "gaussian")
    assert abs(L - abs(np.sqrt(c1) - np.sqrt(c2)) / np.sqrt(c2)) < 1e-15
    L, _ = ms.loss(np.full((3, 4, 4), c1), np.full((3, 4, 4), c2), "gaussian", p=1.0)
    assert abs(L - abs(c1 - c2) / c2) < 1e-15


def test_poisson_loss_closed_forms():
    c1, c2 = 3.0, 5.0
    L, dI = ms.loss(np.full((2, 4, 4), c1), np.full((2, 4, 4), c2), "poisson")
    assert abs(L - (-(c2 * np.log(c1 + ms.POISSON_EPS) - c1) / c2)) < 1e-14
    # at I_model = I_meas the gradient is only the epsilon remainder
    I = np.full((2, 4, 4), 7.0)
    _, dI = ms.loss(I, I, "poisson")
    assert np.max(np.abs(dI)) < 1e-6 / (7.0 * I.size)


@pytest.mark.parametrize("kind,p", [("gaussian", 0.5), ("poisson", 1.0), ("gaussian", 1.0),
                                    ("poisson", 0.5)])
def test_loss_gradient_finite_difference(kind, p):
    rng = np.random.default_rng(13)
    I = rng.uniform(0.2, 4, (2, 6, 6))
    E = rng.uniform(0.2, 4, (2, 6, 6))
    _, g = ms.loss(I, E, kind, p)
    d = rng.standard_normal(I.shape)
    h = 1e-6
    fd = (ms.loss(I + h * d, E, kind, p)[0] - ms.loss(I - h * d, E, kind, p)[0]) / (2 * h)
    assert abs(fd - np.sum(g * d)) < 1e-7 * abs(fd) + 1e-12


def test_zero_measurement_rejected():
    with pytest.raises(ValueError):
        ms.loss(np.ones((1, 4, 4)), np.zeros((1, 4, 4)))


# ------------------------------------------------------------------ adjoint
def test_linear_stage_dot_products():
    """<A x, y> = <x, A^H y> for the linear stages the gradient transposes."""
    rng = np.random.default_rng(14)
    N = 16
    cplx = lambda *s: rng.standard_normal(s) + 1j * rng.standard_normal(s)
    x, y = cplx(N, N), cplx(N, N)
    # F and its adjoint F^-1
    assert abs(np.vdot(ms.fft2(x), y) - np.vdot(x, ms.ifft2(y))) < 1e-12
    # propagator step F^-1 H F and its adjoint F^-1 conj(H) F
    H = ms.propagator(N, 0.2, 0.0197, 17.0, [1e-3, -2e-3])
    A = lambda z: ms.ifft2(H * ms.fft2(z))
    AH = lambda z: ms.ifft2(np.conj(H) * ms.fft2(z))
    assert abs(np.vdot(A(x), y) - np.vdot(x, AH(y))) < 1e-12
    # crop and its adjoint, the scatter
    big = cplx(2, 30, 31)
    t = np.array([5, 9])
    patch = cplx(1, 2, N, N)
    lhs = np.vdot(ms.crop(big, t, N), patch[0])
    rhs = np.vdot(big, ms.scatter_patches(patch, [t], 2, 30, 31))
    assert abs(lhs - rhs) < 1e-12


def test_scatter_sum_and_placement():
    rng = np.random.default_rng(15)
    p = rng.standard_normal((3, 2, 4, 4)) + 0j
    ts = [np.array([0, 0]), np.array([3, 5]), np.array([6, 6])]
    out = ms.scatter_patches(p, ts, 2, 10, 12)
    assert abs(out.sum() - p.sum()) < 1e-12
    one = ms.scatter_patches(p[1:2], ts[1:2], 2, 10, 12)
    assert np.array_equal(one[:, 3:7, 5:9], p[1]) and abs(one.sum() - p[1].sum()) < 1e-12


_FD = {}   # state of the running difference check, inherited by forked workers


def _fd_quotient(i):
    """Fourth-order central difference of the loss along task i's direction."""
    st = _FD
    name, d, hb = st["tasks"][i]
    x = st["base"][name]

    def L(v):
        a = dict(st["base"], **{name: v})
        return ms.loss_of(a["amp"], a["phase"], a["probe"], a["pos"], a["tilt"], a["dz"],
                          st["dx"], st["lam"], st["I_meas"], st["kind"], st["p"])
    return (8 * (L(x + hb * d) - L(x - hb * d)) - (L(x + 2 * hb * d) - L(x - 2 * hb * d))) / (12 * hb)


def _fd_check(c, kind, p, n_dir, seed, tol=2e-7):
    lam = synth.wavelength_A(c.kv)
    rng = np.random.default_rng(seed)
    I_true = ms.forward(c.amp, c.phase, c.probe, c.pos, c.tilt, c.dz, c.dx, lam)
    I_meas = rng.poisson(I_true * 50.0 / I_true.max() + 0.01).astype(np.float64) + 0.5
    # scale the probe so that the model and the data are comparable
    probe = c.probe * np.sqrt(50.0 / I_true.max())
    g = ms.gradients(c.amp, c.phase, probe, c.pos, c.tilt, c.dz, c.dx, lam, I_meas, kind, p)
    base = dict(amp=c.amp, phase=c.phase, probe=probe, pos=c.pos, tilt=c.tilt, dz=c.dz)

    h = 1e-6
    # rounding floor of the difference quotient: the loss carries a relative
    # rounding error of about (number of FFT stages) * eps after 2S transforms
    # of log2(N^2) stages each, divided by the step h
    n_stage = 2 * c.S * int(np.log2(c.N * c.N))
    atol = n_stage * np.finfo(np.float64).eps * abs(g.loss) / h
    tasks, analytic = [], []
    for k in range(n_dir):
        for name, grad in [("amp", g.amp), ("phase", g.phase), ("probe", g.probe),
                           ("pos", g.pos), ("tilt", g.tilt), ("dz", g.dz)]:
            x = base[name]
            if name == "probe":
                d = rng.standard_normal(x.shape) + 1j * rng.standard_normal(x.shape)
                an = np.sum(np.real(np.conj(grad) * d))
            elif name == "dz":
                if k > 0:
                    continue        # one direction only: every repeat is the same quotient
                d = 1.0
                an = grad
            else:
                d = rng.standard_normal(np.shape(x))
                an = np.sum(grad * d)
            # fourth-order central difference (steps hb and 2hb).  The loss
            # bends on a scale of ~1e-4 rad in the tilt (a 1e-4 rad tilt shifts
            # the exit wave by ~(S-1) dz 1e-4 / dx pixels), so the tilt block
            # takes a step ten times smaller than the others.
            hb = h / 10 if name == "tilt" else h
            tasks.append((name, d, hb))
            analytic.append(an)
    _FD.clear()
    _FD.update(tasks=tasks, base=base, dx=c.dx, lam=lam, I_meas=I_meas, kind=kind, p=p)
    workers = min(8, os.cpu_count() or 1, len(tasks))
    if workers > 1 and len(tasks) > 12:
        import multiprocessing
        with multiprocessing.get_context("fork").Pool(workers) as pool:
            fds = pool.map(_fd_quotient, range(len(tasks)))
    else:
        fds = [_fd_quotient(i) for i in range(len(tasks))]
    worst = 0.0
    for (name, _, hb), an, fd in zip(tasks, analytic, fds):
        err = abs(fd - an) / max(abs(fd), 1e-300)
        worst = max(worst, err)
        assert err < tol or abs(fd - an) < atol * h / hb, (name, fd, an, err)
    return worst


@pytest.mark.parametrize("kind,p", [("gaussian", 0.5), ("poisson", 1.0)])
def test_gradient_central_differences_small(kind, p):
    c = synth.small_case(N=16, S=3, M=2, B=3, seed=16)
    _fd_check(c, kind, p, n_dir=4, seed=17)


@pytest.mark.slow
@pytest.mark.parametrize("kind,p", [("poisson", 1.0), ("gaussian", 1.0)])
def test_gradient_central_differences_24_slices(kind, p):
    """The 24-slice, local-tilt workload (N=64, one mode, 16 positions), 32
    random directions per parameter block, step 1e-6.  Its far field reaches
    intensities of 1e-12, where the p=0.5 loss (sqrt I) is too curved for a
    difference quotient, so the smooth p=1 forms are used here; p=0.5 is
    checked on the small case above."""
    c = synth.workload("diffcheck_64")
    _fd_check(c, kind, p, n_dir=32 if kind == "poisson" else 6, seed=18, tol=1e-5)


# ------------------------------------------------------------------ Adam
def test_adam_matches_torch_adam():
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(19)
    x0 = rng.standard_normal(20)
    z0 = rng.standard_normal(6) + 1j * rng.standard_normal(6)
    tx = torch.tensor(x0, requires_grad=True)
    tz = torch.tensor(z0, requires_grad=True)
    opt = torch.optim.Adam([tx, tz], lr=0.01)
    x, z = x0.copy(), z0.copy()
    mx = vx = np.zeros_like(x)
    mz = vz = np.zeros_like(z)
    for step in range(5):
        gx = rng.standard_normal(20)
        gz = rng.standard_normal(6) + 1j * rng.standard_normal(6)
        tx.grad = torch.tensor(gx)
        tz.grad = torch.tensor(gz)
        opt.step()
        x, mx, vx = adam_step(x, gx, mx, vx, step, 0.01)
        z, mz, vz = adam_step(z, gz, mz, vz, step, 0.01)
    assert np.max(np.abs(x - tx.detach().numpy())) < 1e-14
    assert np.max(np.abs(z - tz.detach().numpy())) < 1e-14


# ------------------------------------------------------------------ printed counts
def test_parameter_counts_match_paper():
    with open(os.path.join(GOLDEN, "param_counts.json")) as f:
        gold = json.load(f)
    s = gold["shapes"]
    obj, prb, ps, tl = ms.count_parameters(s["slices"], s["obj_px"], s["obj_px"], s["probe_modes"],
                                           s["N"], s["positions"])
    assert obj == gold["object"] and prb == gold["probe"] and ps == gold["positions"]
    assert obj + prb + ps + tl == gold["total"]
    assert s["N"] ** 4 == gold["measured_values"]


def test_wavelength_300kv():
    assert abs(synth.wavelength_A(300.0) - 0.0196875) < 2e-7


def test_position_pool_equals_batch_gradient():
    """The per-position worker pool used for the N = 256 launch batch gives the
    oracle's batch gradient (object gradient on the patches' window)."""
    from tests import oracle_pool
    c = synth.small_case(N=16, S=3, M=2, B=4, seed=43)
    lam = synth.wavelength_A(c.kv)
    rng = np.random.default_rng(44)
    I = ms.forward(c.amp, c.phase, c.probe, c.pos, c.tilt, c.dz, c.dx, lam)
    meas = rng.poisson(I * 50.0 / I.max() + 0.5).astype(np.float64)
    ref = ms.gradients(c.amp, c.phase, c.probe, c.pos, c.tilt, c.dz, c.dx, lam, meas)
    got = oracle_pool.gradients(c.amp, c.phase, c.probe, c.pos, c.tilt, c.dz, c.dx, lam, meas, workers=2)
    (y0, y1), (x0, x1) = got["window"]
    assert abs(got["loss"] - ref.loss) <= 1e-14 * abs(ref.loss)
    for k in ("probe", "pos", "tilt"):
        assert np.allclose(got[k], getattr(ref, k), rtol=1e-12, atol=1e-14 * np.abs(getattr(ref, k)).max())
    assert abs(got["dz"] - ref.dz) <= 1e-12 * abs(ref.dz)
    for k in ("amp", "phase"):
        full = getattr(ref, k)
        assert np.allclose(got[k], full[:, y0:y1, x0:x1], rtol=1e-12, atol=1e-14 * np.abs(full).max())
        outside = full.copy()
        outside[:, y0:y1, x0:x1] = 0
        assert not outside.any()
