"""Parity of ptyr_constrain (r_z depth filter, phase positivity, probe-mode
orthogonalisation) with the FP64 constraints oracle.

Bars (derived from the arithmetic): the depth filter is a convex combination
of the column's values with float weights (each the float sum of at most
2R+1 taps rounded to 2^-24 relative) summed in float over at most S or 2R+1
terms, so each output is within (S + 2R + 2) 2^-24 max|v| of the exact value;
clipping is exact.  The orthogonalised modes are sums of M float products of
a double-precision eigenvector with the float input (relative error ~M 2^-24)
and the eigenvectors of well-separated powers are stable, so each mode must
match the oracle's to relative L2 <= 1e-5 up to its (arbitrary) unit phase.
"""
import math

import numpy as np
import pytest
import torch

from oracle import constraints as oc
from paper_2505_07814_amd import _lib as L
from paper_2505_07814_amd.ptyr import Engine

pytestmark = pytest.mark.gpu

DEV = torch.device("cuda:0")


def T(a, dt=None):
    a = np.ascontiguousarray(a if dt is None else np.asarray(a).astype(dt))
    return torch.from_numpy(a).to(DEV)


def engine(S, H, W, N=64, M=1):
    return Engine(N, M, S, H, W, 1, 0.2, 0.02, device=DEV)


def rz_bound(sigma, v):
    R = int(math.ceil(4 * sigma))
    return (v.shape[0] + 2 * R + 2) * 2.0 ** -24 * float(np.max(np.abs(v)))


@pytest.mark.parametrize("S,sigma", [(12, 0.6), (12, 1.0), (30, 2.5), (12, 7.0), (2, 1.0), (1, 1.5), (32, 1.0),
                                     (33, 1.0), (70, 3.0), (140, 16.0)])
def test_rz_filter_matches_oracle(S, sigma):
    print(f"rz filter S={S} sigma={sigma}", flush=True)
    H, W = 70, 67                                   # HW not a multiple of the 64-pixel workgroup
    rng = np.random.default_rng(S * 100 + int(10 * sigma))
    amp = rng.uniform(0.5, 1.5, (S, H, W)).astype(np.float32)
    ph = rng.uniform(-0.5, 1.0, (S, H, W)).astype(np.float32)
    eng = engine(S, H, W)
    a, p = T(amp), T(ph)
    eng.constrain(a, p, rz_sigma=sigma, phase_positive=True)
    eng.sync()
    ra, rp, _ = oc.apply(amp, ph, None, rz_sigma=sigma, phase_positive=True)
    ea = np.max(np.abs(a.cpu().numpy() - ra))
    ep = np.max(np.abs(p.cpu().numpy() - rp))
    print(f"max |err| amp {ea:.2e} phase {ep:.2e} (bound {rz_bound(sigma, amp):.2e})", flush=True)
    assert ea <= rz_bound(sigma, amp) and ep <= rz_bound(sigma, ph)
    got = p.cpu().numpy()
    assert np.all(got >= 0)
    # clipping decides exactly where the filtered value is clearly negative
    assert np.all(got[rp == 0] <= rz_bound(sigma, ph))


def test_clip_alone_is_exact():
    rng = np.random.default_rng(3)
    ph = rng.standard_normal((3, 70, 75)).astype(np.float32)
    eng = engine(3, 70, 75)
    p = T(ph)
    eng.constrain(phase=p, phase_positive=True)
    eng.sync()
    assert np.array_equal(p.cpu().numpy(), np.maximum(ph, 0))


def test_rz_filter_full_object_sampled():
    """The 12 x 640 x 640 object of the N=128 workload: 4000 sampled pixel
    columns against the oracle, and the depth mean of every column kept (the
    mirrored filter is doubly stochastic)."""
    S, H = 12, 640
    rng = np.random.default_rng(11)
    ph = rng.uniform(-0.2, 1.0, (S, H, H)).astype(np.float32)
    eng = engine(S, H, H, N=128, M=1)
    p = T(ph)
    eng.constrain(phase=p, amp=T(np.ones((S, H, H), np.float32)), rz_sigma=1.0)
    eng.sync()
    got = p.cpu().numpy()
    idx = rng.integers(0, H * H, 4000)
    cols = ph.reshape(S, -1)[:, idx]
    ref = oc.rz_filter(cols[:, :, None], 1.0)[:, :, 0]
    assert np.max(np.abs(got.reshape(S, -1)[:, idx] - ref)) <= rz_bound(1.0, ph)
    assert np.max(np.abs(got.mean(0) - ph.mean(0))) < 1e-6


def _modes(M, N, seed, powers):
    rng = np.random.default_rng(seed)
    P = rng.standard_normal((M, N, N)) + 1j * rng.standard_normal((M, N, N))
    P *= np.sqrt(np.asarray(powers))[:, None, None] / np.sqrt(N * N * 2)
    return P.astype(np.complex64)


@pytest.mark.parametrize("M,N", [(2, 64), (6, 128), (12, 64), (24, 64)])
def test_probe_orthogonalisation_matches_oracle(M, N):
    print(f"probe orthogonalisation M={M} N={N}", flush=True)
    powers = 1.0 + 0.3 * np.arange(M)[::-1]          # well separated (overlaps mix them a little)
    P = _modes(M, N, 20 + M, powers)
    eng = Engine(N, M, 1, N, N, 1, 0.2, 0.02, device=DEV)
    pr = T(P)
    eng.constrain(probe=pr, probe_orthogonal=True)
    eng.sync()
    Q = pr.cpu().numpy().astype(np.complex128)
    Qr, lam = oc.probe_orthogonalize(P.astype(np.complex128))
    for k in range(M):
        c = np.vdot(Qr[k], Q[k]) / np.vdot(Qr[k], Qr[k])
        err = np.linalg.norm(Q[k] - c * Qr[k]) / np.linalg.norm(Qr[k])
        assert abs(abs(c) - 1) < 1e-5 and err < 1e-5, (k, abs(c), err)
    G = oc.probe_overlap(Q)
    assert np.max(np.abs(G - np.diag(np.diag(G)))) < 1e-5 * lam[0]
    assert np.allclose(np.diag(G).real, lam, rtol=1e-5)
    inc0 = (np.abs(P.astype(np.complex128)) ** 2).sum(0)
    assert np.linalg.norm((np.abs(Q) ** 2).sum(0) - inc0) < 1e-5 * np.linalg.norm(inc0)


def test_orthogonalisation_keeps_model_intensities():
    """The incoherent mode sum is invariant, so the forward model gives the
    same patterns with the orthogonalised probe."""
    from paper_2505_07814_amd import synth
    w = synth.small_case(N=64, S=2, M=3, B=3, H=64 + 30, W=64 + 30, seed=41)
    eng = Engine(64, 3, 2, w.H, w.W, 3, w.dx, synth.wavelength_A(w.kv), device=DEV)
    args = [T(w.amp, np.float32), T(w.phase, np.float32), T(w.probe, np.complex64), T(w.pos, np.float32),
            T(w.tilt, np.float32), T(np.array([w.dz], np.float32))]
    I0 = eng.forward(*args).clone()
    eng.constrain(probe=args[2], probe_orthogonal=True)
    I1 = eng.forward(*args)
    eng.sync()
    a, b = I1.cpu().numpy(), I0.cpu().numpy()
    assert np.linalg.norm(a - b) / np.linalg.norm(b) < 1e-5


def test_single_mode_and_degenerate_modes():
    eng = Engine(64, 1, 1, 64, 64, 1, 0.2, 0.02, device=DEV)
    P = _modes(1, 64, 5, [1.0])
    pr = T(P)
    eng.constrain(probe=pr, probe_orthogonal=True)          # one mode: nothing to do
    eng.sync()
    assert np.array_equal(pr.cpu().numpy(), P)
    # two orthogonal modes of equal power: any unitary mix is a valid answer;
    # what is unique (orthogonality, powers, incoherent sum) must hold
    N = 64
    y, x = np.mgrid[0:N, 0:N] - (N - 1) / 2
    g = np.exp(-(x ** 2 + y ** 2) / 50.0)
    a, b = x * g, y * g
    P2 = np.stack([a / np.linalg.norm(a), b / np.linalg.norm(b)]).astype(np.complex64)
    eng2 = Engine(64, 2, 1, 64, 64, 1, 0.2, 0.02, device=DEV)
    pr2 = T(P2)
    eng2.constrain(probe=pr2, probe_orthogonal=True)
    eng2.sync()
    Q = pr2.cpu().numpy().astype(np.complex128)
    G = oc.probe_overlap(Q)
    assert abs(G[0, 1]) < 1e-6 and np.allclose(np.diag(G).real, [1, 1], atol=1e-6)
    assert np.allclose((np.abs(Q) ** 2).sum(0), (np.abs(P2.astype(np.complex128)) ** 2).sum(0), atol=1e-7)


def test_bad_arguments_are_rejected():
    eng = engine(3, 70, 70)
    a = torch.ones((3, 70, 70), device=DEV)
    for kw in (dict(rz_sigma=-1.0), dict(rz_sigma=17.0)):
        with pytest.raises(L.PtyrError) as e:
            eng.constrain(a, a.clone(), **kw)
        assert e.value.status == L.PTYR_E_ARG
    with pytest.raises(L.PtyrError):
        eng.constrain(phase=a, rz_sigma=1.0)             # amplitude missing
    big = Engine(64, 25, 1, 64, 64, 1, 0.2, 0.02, device=DEV)
    with pytest.raises(L.PtyrError):
        big.constrain(probe=torch.zeros((25, 64, 64), dtype=torch.complex64, device=DEV), probe_orthogonal=True)


def rel(a, b):
    a, b = np.ravel(np.asarray(a, np.float64)), np.ravel(np.asarray(b, np.float64))
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


@pytest.mark.parametrize("S,H,W", [(12, 80, 75), (1, 64, 90), (30, 72, 72), (6, 64, 64), (45, 64, 72),
                                   (2, 2048, 64), (2, 4096, 64)])
def test_kz_filter_matches_oracle(S, H, W):
    """Mixed-radix 3-D transform, weight, inverse: relative L2 <= 1e-5 of the
    oracle for each field (float transforms of ~log2(SHW) stages each way).
    The shapes give short last tiles of rows, columns and depth columns,
    three radices along depth and along x (45 = 5 x 3 x 3, 72 = 3 x 3 x 8),
    and columns of 2048 and 4096 (the longest line: one column per tile,
    filling the 64 KiB of LDS)."""
    print(f"kz filter {S}x{H}x{W}", flush=True)
    rng = np.random.default_rng(S + H + W)
    amp = rng.uniform(0.5, 1.5, (S, H, W)).astype(np.float32)
    ph = rng.uniform(-0.5, 1.0, (S, H, W)).astype(np.float32)
    eng = Engine(64, 1, S, H, W, 1, 0.2, 0.02, device=DEV)
    a, p = T(amp), T(ph)
    eng.constrain(a, p, kz_beta=0.8, kz_alpha=0.5, kz_dz=5.0)
    eng.sync()
    ra = oc.kz_filter(amp, 0.8, 0.5, 0.2, 5.0)
    rp = oc.kz_filter(ph, 0.8, 0.5, 0.2, 5.0)
    ea, ep = rel(a.cpu().numpy(), ra), rel(p.cpu().numpy(), rp)
    print(f"rel-L2 amp {ea:.2e} phase {ep:.2e}", flush=True)
    assert ea <= 1e-5 and ep <= 1e-5


def test_kz_filter_full_object():
    """The 12 x 640 x 640 object of the N=128 workload (640 = 5 x 2^7)."""
    S, H = 12, 640
    rng = np.random.default_rng(21)
    ph = rng.uniform(-0.2, 1.0, (S, H, H)).astype(np.float32)
    amp = np.ones((S, H, H), np.float32)
    eng = Engine(128, 1, S, H, H, 1, 0.15, 0.02, device=DEV)
    a, p = T(amp), T(ph)
    eng.constrain(a, p, kz_beta=0.1, kz_alpha=1.0, kz_dz=20.0)
    eng.sync()
    assert rel(p.cpu().numpy(), oc.kz_filter(ph, 0.1, 1.0, 0.15, 20.0)) <= 1e-5
    assert np.allclose(a.cpu().numpy(), 1.0, atol=1e-5)        # a constant is kept (W_a(0) = 1)


def test_all_constraints_in_order():
    S, H, W = 12, 64, 80
    rng = np.random.default_rng(23)
    amp = rng.uniform(0.5, 1.5, (S, H, W)).astype(np.float32)
    ph = rng.uniform(-0.5, 1.0, (S, H, W)).astype(np.float32)
    P = _modes(3, 64, 24, [1.0, 1.5, 2.0])
    eng = Engine(64, 3, S, H, W, 1, 0.2, 0.02, device=DEV)
    a, p, pr = T(amp), T(ph), T(P)
    cfg = dict(rz_sigma=1.0, phase_positive=True, probe_orthogonal=True, kz_beta=0.5, kz_alpha=0.2)
    eng.constrain(a, p, pr, kz_dz=4.0, **cfg)
    eng.sync()
    ra, rp, _ = oc.apply(amp, ph, None, dx=0.2, dz=4.0, **dict(cfg, probe_orthogonal=False))
    assert rel(a.cpu().numpy(), ra) <= 1e-5 and rel(p.cpu().numpy(), rp) <= 1e-5
    assert np.all(p.cpu().numpy() >= 0)


def test_kz_bad_arguments():
    eng = Engine(64, 1, 3, 70, 64, 1, 0.2, 0.02, device=DEV)          # 70 = 2 x 5 x 7
    a = torch.ones((3, 70, 64), device=DEV)
    with pytest.raises(L.PtyrError):
        eng.constrain(a, a.clone(), kz_beta=1.0, kz_dz=5.0)
    eng3 = Engine(64, 1, 1, 64, 4320, 1, 0.2, 0.02, device=DEV)      # 4320 = 2^5 3^3 5 > 4096
    c = torch.ones((1, 64, 4320), device=DEV)
    with pytest.raises(L.PtyrError):
        eng3.constrain(c, c.clone(), kz_beta=1.0, kz_dz=5.0)
    eng2 = engine(3, 64, 64)
    b = torch.ones((3, 64, 64), device=DEV)
    for kw in (dict(kz_beta=1.0, kz_dz=0.0), dict(kz_beta=-1.0, kz_dz=1.0), dict(kz_alpha=1.0, kz_dz=-2.0)):
        with pytest.raises(L.PtyrError):
            eng2.constrain(b, b.clone(), **kw)
