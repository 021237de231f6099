"""GPU parity with mixed object modes (amplitude / phase of n_obj x S x H x W;
the model intensity sums over every probe mode with every object mode):
forward, loss and gradients through the C-ABI against the FP64 oracle, on one
stream and on the two-stream schedule, the fused Adam step, and the
constraints applied to each object mode."""
import numpy as np
import pytest
import torch

from oracle import constraints as oc
from oracle import multislice as ms
from oracle.adam import adam_step
from paper_2505_07814_amd import synth

pytestmark = pytest.mark.gpu

DEV = torch.device("cuda:0")


def rel(a, b):
    a, b = np.ravel(np.asarray(a)), np.ravel(np.asarray(b))
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def T(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


class ModeCase:
    """Two object modes (the second a weaker, partly different copy of the
    first), float32-rounded inputs shared by the oracle and the GPU, and
    Poisson patterns of the true objects; gradients are taken away from them."""

    def __init__(self, N, S, M, B, seed, H=None, W=None, n_obj=2):
        w = synth.small_case(N=N, S=S, M=M, B=B, H=H or N + 37, W=W or N + 45, seed=seed)
        rng = np.random.default_rng(seed + 7)
        self.w, self.n_obj = w, n_obj
        self.lam = synth.wavelength_A(w.kv)
        amps = [w.amp] + [w.amp * rng.uniform(0.85, 1.0, w.amp.shape) for _ in range(n_obj - 1)]
        phs = [w.phase] + [0.6 * w.phase + 0.05 * rng.standard_normal(w.phase.shape) for _ in range(n_obj - 1)]
        self.amp_true = np.stack(amps).astype(np.float32)
        self.phase_true = np.stack(phs).astype(np.float32)
        self.probe = w.probe.astype(np.complex64)
        self.pos = w.pos.astype(np.float32)
        self.tilt = w.tilt.astype(np.float32)
        self.dz = np.float32(w.dz)
        self.I_true = ms.forward(self.amp_true, self.phase_true, self.probe, self.pos, self.tilt, self.dz, w.dx,
                                 self.lam)
        self.meas = rng.poisson(self.I_true).astype(np.float32)
        self.amp = (1.0 + 0.9 * (self.amp_true - 1.0)).astype(np.float32)
        self.phase = (0.8 * self.phase_true + 0.02 * rng.standard_normal(self.phase_true.shape)).astype(np.float32)
        self.B = B

    def engine(self, **kw):
        from paper_2505_07814_amd.ptyr import Engine
        w = self.w
        return Engine(w.N, w.M, w.S, w.H, w.W, self.B, w.dx, self.lam, n_obj=self.n_obj, device=DEV, **kw)

    def gpu_args(self):
        return (T(self.amp), T(self.phase), T(self.probe), T(self.pos), T(self.tilt),
                T(np.array([self.dz], np.float32)))


@pytest.mark.parametrize("N,S,M,B", [(64, 3, 2, 5), (128, 2, 2, 3), (256, 2, 1, 2)])
def test_forward_parity(N, S, M, B):
    print(f"object modes forward N={N} S={S} M={M} B={B}", flush=True)
    c = ModeCase(N, S, M, B, seed=40 + N % 7)
    eng = c.engine()
    I = eng.forward(*c.gpu_args())
    eng.sync()
    ref = ms.forward(c.amp, c.phase, c.probe, c.pos, c.tilt, c.dz, c.w.dx, c.lam)
    e = rel(I.cpu().numpy(), ref)
    print(f"rel-L2 {e:.2e}", flush=True)
    assert e < 2e-5


def test_repeated_mode_doubles_the_intensity():
    """Two equal object modes with one probe mode: exactly twice the
    single-object intensity (the same kernels on the same data give the same
    bits for both modes, and their sum doubles them exactly)."""
    from paper_2505_07814_amd.ptyr import Engine
    c = ModeCase(64, 2, 1, 4, seed=44)
    a1, p1 = c.amp[0], c.phase[0]
    w = c.w
    e1 = Engine(w.N, w.M, w.S, w.H, w.W, 4, w.dx, c.lam, device=DEV)
    e2 = Engine(w.N, w.M, w.S, w.H, w.W, 4, w.dx, c.lam, n_obj=2, device=DEV)
    rest = c.gpu_args()[2:]
    I1 = e1.forward(T(a1), T(p1), *rest)
    I2 = e2.forward(T(np.stack([a1, a1])), T(np.stack([p1, p1])), *rest)
    e1.sync()
    e2.sync()
    assert torch.equal(I2, 2 * I1)


def _grad_errors(c, eng, sparse_w=0.0):
    loss, g = eng.adjoint(*c.gpu_args(), T(c.meas))
    eng.sync()
    ref = ms.gradients(c.amp, c.phase, c.probe, c.pos, c.tilt, c.dz, c.w.dx, c.lam, c.meas, sparse_w=sparse_w)
    errs = {"loss": abs(float(loss.cpu()[0]) - ref.loss) / abs(ref.loss),
            "amp": rel(g["amp"].cpu().numpy(), ref.amp), "phase": rel(g["phase"].cpu().numpy(), ref.phase),
            "probe": rel(g["probe"].cpu().numpy(), ref.probe), "pos": rel(g["pos"].cpu().numpy(), ref.pos),
            "tilt": rel(g["tilt"].cpu().numpy(), ref.tilt), "dz": rel(g["dz"].cpu().numpy(), [ref.dz])}
    # each object mode's gradient on its own (a mode left out would show here)
    for o in range(c.n_obj):
        errs[f"phase[{o}]"] = rel(g["phase"][o].cpu().numpy(), ref.phase[o])
    print({k: f"{v:.2e}" for k, v in errs.items()}, flush=True)
    return errs


@pytest.mark.parametrize("N,S,M,B", [(64, 3, 2, 5), (128, 2, 2, 3), (256, 2, 1, 2)])
def test_gradient_parity(N, S, M, B):
    print(f"object modes gradients N={N} S={S} M={M} B={B}", flush=True)
    c = ModeCase(N, S, M, B, seed=50 + N % 7)
    errs = _grad_errors(c, c.engine())
    for k, v in errs.items():
        assert v < (1e-6 if k == "loss" else 1e-4), (k, v)


@pytest.mark.parametrize("sparse_w", [0.0, 0.1])
def test_gradient_parity_two_streams(sparse_w):
    """B = 60 rows x 3 probe modes x 2 object modes = 360 chains: the
    two-stream schedule, with the sparsity term over both modes' slices."""
    print(f"object modes, two streams, sparse_w={sparse_w}", flush=True)
    c = ModeCase(64, 3, 3, 60, seed=61, H=64 + 60, W=64 + 70)
    errs = _grad_errors(c, c.engine(sparse_w=sparse_w), sparse_w)
    for k, v in errs.items():
        assert v < (1e-6 if k == "loss" else 1e-4), (k, v)


def test_step_matches_adjoint_then_adam():
    """ptyr_step (object Adam fused into the last scatter, over both modes)
    against ptyr_adjoint's gradients followed by Adam in float64."""
    from paper_2505_07814_amd.ptyr import AdamState
    c = ModeCase(64, 3, 3, 60, seed=62, H=64 + 60, W=64 + 70)
    lr = dict(amp=1e-3, phase=2e-3, probe=1e-2, pos=1e-2, tilt=1e-4, dz=1e-1)
    eng = c.engine(n_scan=60)
    ref_eng = c.engine()
    st = AdamState(*[t.clone() for t in c.gpu_args()])
    meas = T(c.meas)
    b1, b2, eps = float(np.float32(0.9)), float(np.float32(0.999)), float(np.float32(1e-8))
    for t, order in enumerate([np.arange(60), np.arange(60)[::-1].copy()]):
        idx = torch.tensor(order, dtype=torch.int32, device=DEV)
        before = {k: getattr(st, k).clone() for k in st.NAMES}
        m0 = {k: st.m[k].clone() for k in st.NAMES}
        v0 = {k: st.v[k].clone() for k in st.NAMES}
        eng.step(st, idx, meas, lr)
        _, g = ref_eng.adjoint(*[before[k] for k in st.NAMES], meas, idx=idx)
        eng.sync()
        ref_eng.sync()
        for k in ("amp", "phase"):
            p0 = before[k].cpu().numpy().astype(np.float64)
            got = getattr(st, k).cpu().numpy()
            rp, _, _ = adam_step(p0, g[k].cpu().numpy().astype(np.float64), m0[k].cpu().numpy().astype(np.float64),
                                 v0[k].cpu().numpy().astype(np.float64), t, lr[k], beta1=b1, beta2=b2, eps=eps)
            d = np.abs(got.astype(np.float64) - rp)
            tol = 2 * np.spacing(np.abs(rp).astype(np.float32)) + 1e-5 * np.abs(rp - p0)
            print(f"step {t + 1} {k}: max |P - P_ref| / tol {np.max(d / tol):.2f}", flush=True)
            assert np.all(d <= tol), (t, k, float(np.max(d / tol)))
            # the second object mode moved too
            assert np.any(got[1] != before[k][1].cpu().numpy())


def test_constraints_per_mode():
    """k_z and r_z filters and positivity on each object mode's stack."""
    c = ModeCase(64, 6, 1, 2, seed=63, H=64 + 26, W=64 + 36)   # 90 x 100: factors 2, 3, 5
    eng = c.engine()
    amp, phase = T(c.amp), T(c.phase - np.float32(0.01))
    eng.constrain(amp, phase, rz_sigma=1.3, phase_positive=True, kz_beta=0.8, kz_alpha=0.5, kz_dz=2.0)
    eng.sync()
    for o in range(2):
        ra, rp, _ = oc.apply(c.amp[o], c.phase[o] - np.float32(0.01), None, rz_sigma=1.3, phase_positive=True,
                             kz_beta=0.8, kz_alpha=0.5, dx=c.w.dx, dz=2.0)
        ea, ep = rel(amp[o].cpu().numpy(), ra), rel(phase[o].cpu().numpy(), rp)
        print(f"mode {o}: amp {ea:.2e} phase {ep:.2e}", flush=True)
        assert ea < 1e-5 and ep < 1e-5


@pytest.mark.parametrize("budget", [0, 3])
def test_recompute_equals_stored_waves(budget):
    """Per-slice recomputation from checkpoints (budget 0: from the probe;
    3: every few slices) gives the stored-wave gradients of both object modes
    up to float32 rounding."""
    c = ModeCase(64, 5, 2, 4, seed=64)
    g_store = c.engine().adjoint(*c.gpu_args(), T(c.meas))[1]
    eng = c.engine(wave_budget=budget * c.B * 4 * 64 * 64 * 8)       # 4 chain modes per row
    g_rec = eng.adjoint(*c.gpu_args(), T(c.meas))[1]
    eng.sync()
    print(f"budget {budget}: checkpoint stride {eng.checkpoint_stride}", flush=True)
    for k in g_store:
        a, b = g_rec[k].cpu().numpy(), g_store[k].cpu().numpy()
        assert rel(a, b) <= 1e-7, (k, rel(a, b))


def test_pacbed_with_object_modes():
    """The PACBED term on the pattern summed over all probe and object modes."""
    c = ModeCase(64, 3, 2, 5, seed=65)
    loss, g = c.engine(pacbed_w=0.5).adjoint(*c.gpu_args(), T(c.meas))
    ref = ms.gradients(c.amp, c.phase, c.probe, c.pos, c.tilt, c.dz, c.w.dx, c.lam, c.meas, pacbed_w=0.5)
    el = abs(float(loss.cpu()[0]) - ref.loss) / abs(ref.loss)
    ep, eb = rel(g["phase"].cpu().numpy(), ref.phase), rel(g["probe"].cpu().numpy(), ref.probe)
    print(f"loss {el:.2e} phase {ep:.2e} probe {eb:.2e}", flush=True)
    assert el < 1e-6 and ep < 1e-4 and eb < 1e-4
