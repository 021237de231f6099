"""Parity of the HIP path (through the C ABI) with the FP64 oracle.

Both sides get the same float32-rounded inputs from the seeded generator; the
measured patterns are Poisson samples of the oracle's own forward model.
Bars: intensities relative L2 <= 1e-5, loss relative <= 1e-6 on identical
inputs, every gradient block relative L2 <= 1e-4.
"""
import numpy as np
import pytest
import torch

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


class Case:
    """float32-rounded inputs shared by the oracle and the GPU."""

    def __init__(self, w, B=None, start=0, perturb=True, seed=0):
        rng = np.random.default_rng(1000 + seed)
        B = w.pos.shape[0] if B is None else B
        self.w = w
        self.lam = synth.wavelength_A(w.kv)
        self.amp_true = w.amp.astype(np.float32)
        self.phase_true = w.phase.astype(np.float32)
        self.probe = w.probe.astype(np.complex64)
        self.pos = w.pos[start:start + B].astype(np.float32)
        self.tilt = w.tilt[start:start + B].astype(np.float32)
        self.dz = np.float32(w.dz)
        I = ms.forward(self.amp_true, self.phase_true, self.probe, self.pos, self.tilt, self.dz, w.dx, self.lam)
        self.I_true = I
        self.meas = rng.poisson(I).astype(np.float32)
        if perturb:  # evaluate gradients away from the truth
            self.amp = (1.0 + 0.9 * (self.amp_true - 1.0)).astype(np.float32)
            self.phase = (0.8 * self.phase_true + 0.02 * rng.standard_normal(self.phase_true.shape)).astype(np.float32)
        else:
            self.amp, self.phase = self.amp_true, self.phase_true
        self.B = B

    def engine(self, loss="gaussian", p=None, **kw):
        from paper_2505_07814_amd.ptyr import Engine
        w = self.w
        return Engine(w.N, w.M, w.S, w.H, w.W, self.B, w.dx, self.lam, loss=loss, p=p, device=DEV, **kw)

    def gpu_args(self, amp=None, phase=None):
        amp = self.amp if amp is None else amp
        phase = self.phase if phase is None else phase
        return (T(amp), T(phase), T(self.probe), T(self.pos), T(self.tilt), T(np.array([self.dz], np.float32)))

    def oracle_grad(self, kind="gaussian", p=None):
        return ms.gradients(self.amp, self.phase, self.probe, self.pos, self.tilt, self.dz, self.w.dx, self.lam,
                            self.meas, kind, p)


def small(N, S, M, B, seed, H=None, W=None, tilt=2e-3):
    H = H or N + 37
    W = W or N + 41
    return synth.small_case(N=N, S=S, M=M, B=B, H=H, W=W, seed=seed, tilt_scale=tilt)


SMALL = [(64, 1, 1, 1, 1), (64, 3, 2, 5, 2), (64, 4, 3, 7, 3), (128, 2, 2, 3, 4), (128, 3, 1, 2, 5)]


@pytest.mark.parametrize("N,S,M,B,seed", SMALL)
def test_forward_parity_small(N, S, M, B, seed):
    print(f"forward small N={N} S={S} M={M} B={B}", flush=True)
    c = Case(small(N, S, M, B, seed), perturb=False)
    eng = c.engine()
    I = eng.forward(*c.gpu_args())
    eng.sync()
    e = rel(I.cpu().numpy(), c.I_true)
    print(f"forward rel-L2 {e:.2e}", flush=True)
    assert e < 1e-5


def test_forward_unaligned_object_matches_aligned():
    """The transmission pass takes 16-byte aligned parameters four pixels at a
    time and others pixel by pixel: an object passed as views 4 bytes into
    larger buffers (and a pixel count that is not a multiple of 4) gives
    bitwise the patterns of the aligned call."""
    print("forward unaligned object N=64 S=3", flush=True)
    c = Case(small(64, 3, 2, 5, 2), perturb=False)
    assert c.amp.size % 4 != 0
    eng = c.engine()
    args = c.gpu_args()
    I0 = eng.forward(*args).clone()
    views = []
    for a in args[:2]:
        buf = torch.zeros(a.numel() + 1, dtype=a.dtype, device=DEV)
        v = buf[1:].view(a.shape)
        v.copy_(a)
        assert v.data_ptr() % 16 != 0
        views.append(v)
    I1 = eng.forward(*views, *args[2:])
    eng.sync()
    assert torch.equal(I0, I1)
    assert rel(I1.cpu().numpy(), c.I_true) < 1e-5


def test_forward_parity_single_slice_64():
    print("forward single_slice_64", flush=True)
    c = Case(synth.workload("single_slice_64"), perturb=False)
    eng = c.engine()
    I = eng.forward(*c.gpu_args())
    eng.sync()
    e = rel(I.cpu().numpy(), c.I_true)
    print(f"forward rel-L2 {e:.2e}", flush=True)
    assert e < 1e-5


def test_forward_parity_multislice_128_batch():
    """The benchmark's launch: N=128, 12 slices, 6 modes, one batch of 64."""
    print("forward multislice_128 B=64", flush=True)
    c = Case(synth.workload("multislice_128", scan=64), perturb=False)
    eng = c.engine()
    I = eng.forward(*c.gpu_args())
    eng.sync()
    e = rel(I.cpu().numpy(), c.I_true)
    print(f"forward rel-L2 {e:.2e}", flush=True)
    assert e < 1e-5


@pytest.mark.parametrize("kind,p", [("gaussian", 0.5), ("poisson", 1.0), ("gaussian", 1.0), ("poisson", 0.5)])
def test_loss_parity(kind, p):
    rng = np.random.default_rng(7)
    Im = rng.gamma(2.0, 20.0, (5, 64, 64)).astype(np.float32)
    Im[:, :3, :3] = 0.0                                  # exact zeros in the model
    Ie = rng.poisson(Im + 0.5).astype(np.float32)
    from paper_2505_07814_amd.ptyr import Engine
    eng = Engine(64, 1, 1, 64, 64, 5, 0.2, 0.02, loss=kind, p=p, device=DEV)
    L, g = eng.loss(T(Im), T(Ie), want_grad=True)
    eng.sync()
    L0, g0 = ms.loss(Im, Ie, kind, p)
    assert abs(float(L.cpu()[0]) - L0) <= 1e-6 * abs(L0)
    assert rel(g.cpu().numpy(), g0) < 1e-6


GRAD_SMALL = [(64, 1, 1, 3, 11), (64, 3, 2, 5, 12), (128, 3, 2, 3, 13), (64, 5, 3, 6, 14)]


def _check_grads(c, eng, kind="gaussian", p=None, tol=1e-4, **kw):
    loss, g = eng.adjoint(*c.gpu_args(), T(c.meas), **kw)
    eng.sync()
    ref = c.oracle_grad(kind, p)
    errs = {
        "loss": abs(float(loss.cpu()[0]) - ref.loss) / abs(ref.loss),
        "amp": rel(g["amp"].cpu().numpy(), ref.amp),
        "phase": rel(g["phase"].cpu().numpy(), ref.phase),
        "probe": rel(g["probe"].cpu().numpy(), ref.probe),
        "pos": rel(g["pos"].cpu().numpy(), ref.pos),
        "dz": rel(g["dz"].cpu().numpy(), [ref.dz]),
    }
    if c.w.S > 1:
        errs["tilt"] = rel(g["tilt"].cpu().numpy(), ref.tilt)
    print({k: f"{v:.2e}" for k, v in errs.items()}, flush=True)
    for k, v in errs.items():
        assert v < (1e-6 if k == "loss" else tol), (k, v)
    return g


@pytest.mark.parametrize("N,S,M,B,seed", GRAD_SMALL)
@pytest.mark.parametrize("kind", ["gaussian", "poisson"])
def test_gradient_parity_small(N, S, M, B, seed, kind):
    print(f"gradient small N={N} S={S} M={M} B={B} {kind}", flush=True)
    c = Case(small(N, S, M, B, seed))
    _check_grads(c, c.engine(kind), kind)


def test_gradient_parity_diffcheck_64():
    """24 slices, local tilts (the differentiation-check workload)."""
    print("gradient diffcheck_64", flush=True)
    c = Case(synth.workload("diffcheck_64"))
    _check_grads(c, c.engine())


def test_gradient_parity_multislice_128():
    print("gradient multislice_128 B=8", flush=True)
    c = Case(synth.workload("multislice_128", scan=8))
    _check_grads(c, c.engine())


def test_gradient_parity_multislice_128_full_batch():
    """The benchmark batch (64 rows x 6 modes = 384 chains, more than the 256
    compute units): the step runs as two chain ranges on two streams, with the
    loss batch factor applied at the reductions."""
    print("gradient multislice_128 B=64 (two chain ranges)", flush=True)
    c = Case(synth.workload("multislice_128", scan=64))
    _check_grads(c, c.engine())


def test_gradient_parity_uneven_chain_split():
    """270 chains: a first range of 256, then 14 more chains of which the
    first 4 belong to the last row of the first range's forward."""
    print("gradient N=64 S=3 M=3 B=90 (uneven split)", flush=True)
    w = synth.small_case(N=64, S=3, M=3, B=90, H=64 + 60, W=64 + 70, seed=31)
    c = Case(w)
    g1 = _check_grads(c, c.engine())
    eng = c.engine()
    g2 = eng.adjoint(*c.gpu_args(), T(c.meas))[1]
    eng.sync()
    for k in g1:
        assert torch.equal(g1[k], g2[k]), k        # the two-stream schedule is deterministic


def test_recompute_equals_stored_waves():
    print("recompute vs store", flush=True)
    c = Case(synth.workload("diffcheck_64"))
    g_store = c.engine().adjoint(*c.gpu_args(), T(c.meas))[1]
    for budget in (0, 3 * 16 * 64 * 64 * 8, 7 * 16 * 64 * 64 * 8):
        eng = c.engine(wave_budget=budget)
        g_rec = eng.adjoint(*c.gpu_args(), T(c.meas))[1]
        eng.sync()
        for k in g_store:
            a, b = g_rec[k].cpu().numpy(), g_store[k].cpu().numpy()
            assert rel(a, b) <= 1e-7, (budget, eng.checkpoint_stride, k, rel(a, b))


def test_deterministic():
    c = Case(small(64, 3, 2, 6, 21))
    eng = c.engine()
    g1 = eng.adjoint(*c.gpu_args(), T(c.meas))[1]
    g2 = eng.adjoint(*c.gpu_args(), T(c.meas))[1]
    eng.sync()
    for k in g1:
        assert torch.equal(g1[k], g2[k]), k


def test_reuse_forward_matches_recompute():
    c = Case(small(64, 3, 2, 4, 22))
    eng = c.engine()
    eng.forward(*c.gpu_args())
    g1 = eng.adjoint(*c.gpu_args(), T(c.meas), reuse=True)[1]
    g2 = eng.adjoint(*c.gpu_args(), T(c.meas), reuse=False)[1]
    eng.sync()
    for k in g1:
        assert torch.equal(g1[k], g2[k]), k


def test_accumulation_over_sub_batches():
    """Two calls on the halves of a batch add their gradients (+=)."""
    c = Case(small(64, 2, 1, 6, 23))
    from paper_2505_07814_amd.ptyr import Engine
    eng = Engine(64, 1, 2, c.w.H, c.w.W, 3, c.w.dx, c.lam, device=DEV)
    args = c.gpu_args()
    grads = None
    for h in (0, 1):
        idx = torch.arange(3 * h, 3 * h + 3, dtype=torch.int32, device=DEV)
        _, grads = eng.adjoint(*args, T(c.meas), idx=idx, grads=grads)
    eng.sync()
    ref = {k: np.zeros_like(v) for k, v in [("amp", c.amp), ("phase", c.phase)]}
    for h in (0, 1):
        sl = slice(3 * h, 3 * h + 3)
        r = ms.gradients(c.amp, c.phase, c.probe, c.pos[sl], c.tilt[sl], c.dz, c.w.dx, c.lam, c.meas[sl])
        ref["amp"] += r.amp
        ref["phase"] += r.phase
    assert rel(grads["amp"].cpu().numpy(), ref["amp"]) < 1e-4
    assert rel(grads["phase"].cpu().numpy(), ref["phase"]) < 1e-4


def test_out_of_bounds_position_is_reported_and_skipped():
    c = Case(small(64, 2, 1, 3, 24), perturb=False)
    pos = c.pos.copy()
    pos[1] = [5.0, 50.0]                                 # patch leaves the object
    from paper_2505_07814_amd import _lib as L
    eng = c.engine()
    args = list(c.gpu_args())
    args[3] = T(pos)
    I = eng.forward(*args)
    with pytest.raises(L.PtyrError) as e:
        eng.sync()
    assert e.value.status == L.PTYR_E_BOUNDS
    I = I.cpu().numpy()
    assert np.all(I[1] == 0.0)
    assert rel(I[[0, 2]], c.I_true[[0, 2]]) < 1e-5
    eng.sync()                                            # flag was cleared


def test_bad_row_index_is_reported():
    c = Case(small(64, 2, 1, 3, 25), perturb=False)
    from paper_2505_07814_amd import _lib as L
    eng = c.engine()
    idx = torch.tensor([0, 7, 2], dtype=torch.int32, device=DEV)
    eng.forward(*c.gpu_args(), idx=idx)
    with pytest.raises(L.PtyrError) as e:
        eng.sync()
    assert e.value.status == L.PTYR_E_ARG


def test_adam_step_parity():
    """Two mini-batch steps: GPU ptyr_step vs oracle gradient + oracle Adam."""
    from paper_2505_07814_amd.ptyr import AdamState, Engine
    w = small(64, 3, 2, 8, 26)
    c = Case(w)
    eng = Engine(64, 2, 3, w.H, w.W, 4, w.dx, c.lam, device=DEV, n_scan=8)
    st = AdamState(*[t.clone() for t in c.gpu_args()])
    lr = dict(amp=1e-3, phase=2e-3, probe=1e-2, pos=1e-2, tilt=1e-4, dz=1e-1)
    ref = dict(amp=c.amp.astype(np.float64), phase=c.phase.astype(np.float64), probe=c.probe.astype(np.complex128),
               pos=c.pos.astype(np.float64), tilt=c.tilt.astype(np.float64), dz=np.array([float(c.dz)]))
    mom = {k: (np.zeros_like(v), np.zeros_like(v)) for k, v in ref.items()}
    batches = [np.array([0, 2, 4, 6]), np.array([7, 5, 3, 1])]
    meas = T(c.meas)
    for t, b in enumerate(batches):
        eng.step(st, torch.tensor(b, dtype=torch.int32, device=DEV), meas, lr)
        gr = ms.gradients(ref["amp"], ref["phase"], ref["probe"], ref["pos"][b], ref["tilt"][b], ref["dz"][0],
                          w.dx, c.lam, c.meas[b])
        dense = dict(amp=gr.amp, phase=gr.phase, probe=gr.probe, dz=np.array([gr.dz]))
        dense["pos"] = np.zeros_like(ref["pos"]); dense["pos"][b] = gr.pos
        dense["tilt"] = np.zeros_like(ref["tilt"]); dense["tilt"][b] = gr.tilt
        for k in ref:
            ref[k], m, v = adam_step(ref[k], dense[k], mom[k][0], mom[k][1], t, lr[k])
            mom[k] = (m, v)
    eng.sync()
    assert st.step == 2
    for k in ref:
        init = np.ravel(np.asarray(getattr(c, k) if k != "dz" else [c.dz])).astype(ref[k].dtype)
        d_got = np.ravel(getattr(st, k).cpu().numpy()).astype(ref[k].dtype) - init
        d_ref = np.ravel(ref[k]) - init
        err = rel(d_got, d_ref)
        print(k, f"update rel-L2 {err:.2e}", flush=True)
        # Adam divides by sqrt(v): entries whose gradient nearly cancels keep an
        # O(1) relative difference, so the bar is on the whole update
        assert err < 1e-3, (k, err)


def test_launch_timing_counts_every_fused_launch():
    """With timing on, every fused forward / gradient dispatch is timed by
    start / stop events bound to the dispatch: two steps of a batch that
    splits over two streams (more chains than compute units) give each
    kernel's launches, all with positive durations, and results bitwise
    those of the same steps untimed."""
    import torch as _t
    from paper_2505_07814_amd.ptyr import AdamState, Engine
    print("launch timing N=64 S=3 M=3 B=90", flush=True)
    w = synth.small_case(N=64, S=3, M=3, B=90, H=64 + 60, W=64 + 70, seed=31)
    c = Case(w)
    lr = dict(amp=1e-3, phase=2e-3, probe=1e-2, pos=1e-2, tilt=1e-4, dz=1e-1)
    meas = T(c.meas)
    states = []
    for timed in (True, False):
        eng = Engine(64, 3, 3, w.H, w.W, 90, w.dx, c.lam, device=DEV, n_scan=90)
        st = AdamState(*[t.clone() for t in c.gpu_args()])
        eng.timing(timed)
        for order in (np.arange(90), np.arange(90)[::-1].copy()):
            eng.step(st, _t.tensor(order, dtype=_t.int32, device=DEV), meas, lr)
        eng.sync()
        if timed:
            kt = eng.timing_read()
            eng.timing(False)
            print(kt, flush=True)
            split = 270 > _t.cuda.get_device_properties(DEV).multi_processor_count
            for k in ("forward", "gradient"):
                ms, n = kt[k]
                assert n >= 2 and ms > 0.0, (k, kt[k])
                if split:
                    assert n >= 4, (k, kt[k])
        states.append(st)
    for k in states[0].NAMES:
        assert _t.equal(getattr(states[0], k), getattr(states[1], k)), k


def test_bound_step_matches_step():
    """Engine.bind_step (parameters and rates marshalled once) gives bitwise
    the parameters, moments, step counter and losses of Engine.step over
    three batches, the last given as a view into a larger index tensor, and
    refuses a batch larger than the engine's."""
    from paper_2505_07814_amd.ptyr import AdamState, Engine
    print("bound step N=64 S=3 M=2 B=4", flush=True)
    w = small(64, 3, 2, 8, 26)
    c = Case(w)
    lr = dict(amp=1e-3, phase=2e-3, probe=1e-2, pos=1e-2, tilt=1e-4, dz=1e-1)
    meas = T(c.meas)
    eng_a = Engine(64, 2, 3, w.H, w.W, 4, w.dx, c.lam, device=DEV, n_scan=8)
    eng_b = Engine(64, 2, 3, w.H, w.W, 4, w.dx, c.lam, device=DEV, n_scan=8)
    sa = AdamState(*[t.clone() for t in c.gpu_args()])
    sb = AdamState(*[t.clone() for t in c.gpu_args()])
    step_b = eng_b.bind_step(sb, meas, lr)
    order = torch.tensor([0, 2, 4, 6, 7, 5, 3, 1, 6, 1, 4, 3], dtype=torch.int32, device=DEV)
    for k in range(3):
        idx = order[4 * k:4 * k + 4]
        la = eng_a.step(sa, idx.clone(), meas, lr)
        lb = step_b(idx)
        eng_a.sync()
        eng_b.sync()
        assert torch.equal(la, lb), k
    assert sa.step == sb.step == 3
    for k in sa.NAMES:
        assert torch.equal(getattr(sa, k), getattr(sb, k)), k
        assert torch.equal(sa.m[k], sb.m[k]) and torch.equal(sa.v[k], sb.v[k]), k
    with pytest.raises(ValueError):
        step_b(order[:5])


@pytest.mark.parametrize("which", ["all", "phase_only", "sparse", "pacbed", "terms"])
def test_step_split_batch_matches_adjoint_then_adam(which):
    """ptyr_step on a batch of more chains than compute units (two-stream
    schedule, the object's Adam fused into the batch's last scatter) equals
    ptyr_adjoint's gradients of the same batch followed by Adam in float64,
    over two steps (the second also shows that no gradient sums of the first
    leak into it).  The gradients are the same kernels' in the same order,
    so the parameters differ only by the float32 Adam arithmetic and the
    rounding of the updated parameter."""
    from paper_2505_07814_amd.ptyr import AdamState, Engine
    print(f"step N=64 S=3 M=3 B=90 ({which})", flush=True)
    w = synth.small_case(N=64, S=3, M=3, B=90, H=64 + 60, W=64 + 70, seed=31)
    c = Case(w)
    lr = dict(amp=1e-3, phase=2e-3, probe=1e-2, pos=1e-2, tilt=1e-4, dz=1e-1)
    if which == "phase_only":
        lr = dict(amp=0.0, phase=2e-3, probe=0.0, pos=0.0, tilt=0.0, dz=0.0)
    sw = 0.1 if which == "sparse" else 0.0
    pw = 0.5 if which == "pacbed" else 0.0              # one stream: the batch means couple the rows
    kw = _mix_engine_kw() if which == "terms" else {}     # one stream: the weights need both batch factors
    eng = Engine(64, 3, 3, w.H, w.W, 90, w.dx, c.lam, device=DEV, n_scan=90, sparse_w=sw, pacbed_w=pw, **kw)
    ref_eng = c.engine(sparse_w=sw, pacbed_w=pw, **kw)
    st = AdamState(*[t.clone() for t in c.gpu_args()])
    meas = T(c.meas)
    b1, b2, eps = float(np.float32(0.9)), float(np.float32(0.999)), float(np.float32(1e-8))
    for t, order in enumerate([np.arange(90), np.arange(90)[::-1].copy()]):
        idx = torch.tensor(order, dtype=torch.int32, device=DEV)
        before = {k: getattr(st, k).clone() for k in st.NAMES}
        m0 = {k: st.m[k].clone() for k in st.NAMES}
        v0 = {k: st.v[k].clone() for k in st.NAMES}
        eng.step(st, idx, meas, lr)
        _, g = ref_eng.adjoint(*[before[k] for k in st.NAMES], meas, idx=idx)
        eng.sync()
        ref_eng.sync()
        for k in st.NAMES:
            p0 = before[k].cpu().numpy()
            got = getattr(st, k).cpu().numpy()
            if lr[k] == 0:
                assert np.array_equal(got, p0), k
                continue
            f64 = lambda x: np.asarray(x, np.complex128 if np.iscomplexobj(x) else np.float64)
            rp, _, _ = adam_step(f64(p0), f64(g[k].cpu().numpy()), f64(m0[k].cpu().numpy()),
                                 f64(v0[k].cpu().numpy()), t, lr[k], beta1=b1, beta2=b2, eps=eps)
            # the float32 parameter is the reference update rounded, to 2 ulp
            # (an update of 1e-3 on a parameter near 1 is itself only held to
            # ~6e-5 relative by float32)
            got_r = got.view(np.float32) if np.iscomplexobj(got) else got
            p0_r = p0.view(np.float32) if np.iscomplexobj(p0) else p0
            rp_r = np.stack([rp.real, rp.imag], -1).ravel() if np.iscomplexobj(rp) else np.ravel(rp)
            d = np.abs(np.ravel(got_r).astype(np.float64) - rp_r)
            tol = 2 * np.spacing(np.abs(rp_r).astype(np.float32)) + 1e-5 * np.abs(rp_r - np.ravel(p0_r))
            print(f"step {t + 1} {k}: max |P - P_ref| / tol {np.max(d / tol):.2f}", flush=True)
            assert np.all(d <= tol), (t, k, float(np.max(d / tol)))


def test_step_full_workload_matches_adjoint_then_adam():
    """The benchmark's own launch (multislice_128: N=128, 12 slices of
    640 x 640, 6 modes, 64 positions per step, two-stream schedule, object
    Adam fused into the last scatter): ptyr_step equals ptyr_adjoint's
    gradients of the same batch (which the oracle checks at this size)
    followed by Adam in float64, within the rounding of a float32 Adam update
    (bound below)."""
    from paper_2505_07814_amd.ptyr import AdamState, Engine
    print("step multislice_128 B=64", flush=True)
    w = synth.workload("multislice_128", scan=128)
    c = Case(w, B=128)
    lr = dict(amp=5e-4, phase=5e-4, probe=1e-4, pos=1e-3, tilt=1e-5, dz=1e-2)
    eng = Engine(w.N, w.M, w.S, w.H, w.W, 64, w.dx, c.lam, device=DEV, n_scan=128)
    ref_eng = Engine(w.N, w.M, w.S, w.H, w.W, 64, w.dx, c.lam, device=DEV)
    st = AdamState(*[t.clone() for t in c.gpu_args()])
    meas = T(c.meas)
    b1, b2, eps = float(np.float32(0.9)), float(np.float32(0.999)), float(np.float32(1e-8))
    order = np.random.default_rng(5).permutation(128)
    for t, idx_np in enumerate([order[:64], order[64:]]):
        idx = torch.tensor(idx_np, dtype=torch.int32, device=DEV)
        before = {k: getattr(st, k).clone() for k in st.NAMES}
        m0 = {k: st.m[k].clone() for k in st.NAMES}
        v0 = {k: st.v[k].clone() for k in st.NAMES}
        eng.step(st, idx, meas, lr)
        _, g = ref_eng.adjoint(*[before[k] for k in st.NAMES], meas, idx=idx)
        eng.sync()
        ref_eng.sync()
        for k in st.NAMES:
            f64 = lambda x: np.asarray(x, np.complex128 if np.iscomplexobj(x) else np.float64)
            p0 = before[k].cpu().numpy()
            got = getattr(st, k).cpu().numpy()
            rp, _, _ = adam_step(f64(p0), f64(g[k].cpu().numpy()), f64(m0[k].cpu().numpy()),
                                 f64(v0[k].cpu().numpy()), t, lr[k], beta1=b1, beta2=b2, eps=eps)
            flat = lambda x: np.ravel(np.asarray(x).view(np.float32) if np.iscomplexobj(x) else x).astype(np.float64)
            got_r, gr, mr, vr = flat(got), flat(g[k].cpu().numpy()), flat(m0[k].cpu().numpy()), flat(v0[k].cpu().numpy())
            rp_r = np.stack([rp.real, rp.imag], -1).ravel() if np.iscomplexobj(rp) else np.ravel(rp)
            # float32 Adam: the update u = a m' / D (a = lr / bc1, D = sqrt(v') / bc2s + eps)
            # carries a few roundings relative to itself, plus the absolute error
            # of m' = b1 m + (1 - b1) g, which can cancel: ~u32 (|b1 m| + |(1 - b1) g|);
            # the parameter adds half an ulp of its own
            u32 = 2.0 ** -24
            a = lr[k] / (1.0 - b1 ** (t + 1))
            D = np.sqrt(b2 * vr + (1 - b2) * gr * gr) / np.sqrt(1.0 - b2 ** (t + 1)) + eps
            mm = np.abs(b1 * mr) + np.abs((1 - b1) * gr)
            u = np.abs(a * (b1 * mr + (1 - b1) * gr) / D)
            tol = 2 * np.spacing(np.abs(rp_r).astype(np.float32)) + 8 * u32 * u + 2 * u32 * a * mm / D
            d = np.abs(got_r - rp_r)
            print(f"step {t + 1} {k}: max |P - P_ref| / tol {np.max(d / tol):.2f}", flush=True)
            assert np.all(d <= tol), (t, k, float(np.max(d / tol)))


@pytest.mark.parametrize("split", [False, True])
def test_sparsity_term_parity(split):
    """Loss and gradients with 0.1 x the L1 sparsity term of the phase, on one
    stream (B = 5) and on the two-stream schedule (B = 90, 270 chains)."""
    print(f"sparsity term (split={split})", flush=True)
    if split:
        w = synth.small_case(N=64, S=3, M=3, B=90, H=64 + 60, W=64 + 70, seed=31)
    else:
        w = small(64, 3, 2, 5, 12)
    c = Case(w)
    phase = (c.phase + np.float32(0.2)) * np.where(np.arange(c.phase.size).reshape(c.phase.shape) % 3 == 0,
                                                   -1, 1).astype(np.float32)
    eng = c.engine(sparse_w=0.1)
    loss, g = eng.adjoint(*c.gpu_args(phase=phase), T(c.meas))
    eng.sync()
    ref = ms.gradients(c.amp, phase, c.probe, c.pos, c.tilt, c.dz, w.dx, c.lam, c.meas, sparse_w=0.1)
    el = abs(float(loss.cpu()[0]) - ref.loss) / abs(ref.loss)
    ep = rel(g["phase"].cpu().numpy(), ref.phase)
    ea = rel(g["amp"].cpu().numpy(), ref.amp)
    print(f"loss {el:.2e} phase {ep:.2e} amp {ea:.2e}", flush=True)
    assert el < 1e-6 and ep < 1e-4 and ea < 1e-4
    # the sparsity part of the loss and of the phase gradient are really there
    Ls, gs = ms.sparse_term(phase, c.pos, 64)
    assert 0.1 * Ls > 1e-3 * abs(ref.loss) and np.linalg.norm(0.1 * gs) > 1e-3 * np.linalg.norm(ref.phase)


def test_pacbed_loss_parity():
    """ptyr_loss with 0.5 x the PACBED term: loss and dL/dI against the oracle."""
    rng = np.random.default_rng(17)
    Im = rng.gamma(2.0, 20.0, (6, 64, 64)).astype(np.float32)
    Ie = rng.poisson(Im + 0.5).astype(np.float32)
    from paper_2505_07814_amd.ptyr import Engine
    for kind in ("gaussian", "poisson"):
        eng = Engine(64, 1, 1, 64, 64, 6, 0.2, 0.02, loss=kind, pacbed_w=0.5, device=DEV)
        L, g = eng.loss(T(Im), T(Ie), want_grad=True)
        eng.sync()
        p = 0.5 if kind == "gaussian" else 1.0
        L0, g0 = ms.loss(Im, Ie, kind, p, pacbed_w=0.5)
        print(kind, abs(float(L.cpu()[0]) - L0) / abs(L0), rel(g.cpu().numpy(), g0), flush=True)
        assert abs(float(L.cpu()[0]) - L0) <= 1e-6 * abs(L0)
        assert rel(g.cpu().numpy(), g0) < 1e-6


@pytest.mark.parametrize("B", [5, 90])
def test_pacbed_gradient_parity(B):
    """Loss and gradients with 0.5 x the PACBED term; B = 90 (270 chains) would
    take the two-stream schedule without it."""
    print(f"pacbed gradients B={B}", flush=True)
    if B == 90:
        w = synth.small_case(N=64, S=3, M=3, B=90, H=64 + 60, W=64 + 70, seed=31)
    else:
        w = small(64, 3, 2, 5, 12)
    c = Case(w)
    eng = c.engine(pacbed_w=0.5)
    loss, g = eng.adjoint(*c.gpu_args(), T(c.meas))
    eng.sync()
    ref = ms.gradients(c.amp, c.phase, c.probe, c.pos, c.tilt, c.dz, w.dx, c.lam, c.meas, pacbed_w=0.5)
    errs = {"loss": abs(float(loss.cpu()[0]) - ref.loss) / abs(ref.loss),
            "amp": rel(g["amp"].cpu().numpy(), ref.amp), "phase": rel(g["phase"].cpu().numpy(), ref.phase),
            "probe": rel(g["probe"].cpu().numpy(), ref.probe), "pos": rel(g["pos"].cpu().numpy(), ref.pos),
            "tilt": rel(g["tilt"].cpu().numpy(), ref.tilt), "dz": rel(g["dz"].cpu().numpy(), [ref.dz])}
    print({k: f"{v:.2e}" for k, v in errs.items()}, flush=True)
    for k, v in errs.items():
        assert v < (1e-6 if k == "loss" else 1e-4), (k, v)
    # the term changes the gradient measurably
    ref0 = ms.gradients(c.amp, c.phase, c.probe, c.pos, c.tilt, c.dz, w.dx, c.lam, c.meas)
    assert rel(ref.phase, ref0.phase) > 1e-3


def test_autograd_function_matches_adjoint():
    from paper_2505_07814_amd.ptyr import multislice_loss
    c = Case(small(64, 3, 2, 4, 27))
    eng = c.engine()
    args = [t.clone().requires_grad_(True) for t in c.gpu_args()]
    loss = multislice_loss(eng, *args, T(c.meas))
    (2.0 * loss).backward()
    ref = c.oracle_grad()
    assert abs(float(loss.detach().cpu()) - ref.loss) < 1e-6 * abs(ref.loss)
    assert rel(args[1].grad.cpu().numpy(), 2 * ref.phase) < 1e-4
    assert rel(args[2].grad.cpu().numpy(), 2 * ref.probe) < 1e-4
    assert rel(args[3].grad.cpu().numpy(), 2 * ref.pos) < 1e-4


def test_autograd_function_with_sparsity_matches_oracle():
    """With the sparsity term the autograd node's value and gradient are those
    of the same loss (data term + 0.1 x L1 of the phase over the batch's
    patches): both against the oracle's gradients(..., sparse_w=0.1)."""
    from paper_2505_07814_amd.ptyr import multislice_loss
    c = Case(small(64, 3, 2, 4, 28))
    eng = c.engine(sparse_w=0.1)
    args = [t.clone().requires_grad_(True) for t in c.gpu_args()]
    loss = multislice_loss(eng, *args, T(c.meas))
    (3.0 * loss).backward()
    ref = ms.gradients(c.amp, c.phase, c.probe, c.pos, c.tilt, c.dz, c.w.dx, c.lam, c.meas, sparse_w=0.1)
    el = abs(float(loss.detach().cpu()) - ref.loss) / abs(ref.loss)
    errs = {k: rel(a.grad.cpu().numpy(), 3 * getattr(ref, k)) for k, a in
            zip(("amp", "phase", "probe", "pos", "tilt"), args[:5])}
    print(f"loss {el:.2e}", {k: f"{v:.2e}" for k, v in errs.items()}, flush=True)
    assert el < 1e-6
    for k, v in errs.items():
        assert v < 1e-4, (k, v)
    Ls, _ = ms.sparse_term(c.phase, c.pos, 64)
    assert 0.1 * Ls > 1e-3 * abs(ref.loss)            # the term is really in the value


# ---------------------------------------------------------------- N = 256 (line passes through HBM)
@pytest.mark.parametrize("S,M,B,seed", [(1, 1, 2, 31), (3, 2, 3, 32)])
def test_forward_parity_small_256(S, M, B, seed):
    print(f"forward small N=256 S={S} M={M} B={B}", flush=True)
    c = Case(small(256, S, M, B, seed), perturb=False)
    eng = c.engine()
    I = eng.forward(*c.gpu_args())
    eng.sync()
    e = rel(I.cpu().numpy(), c.I_true)
    print(f"forward rel-L2 {e:.2e}", flush=True)
    assert e < 1e-5


@pytest.mark.parametrize("kind", ["gaussian", "poisson"])
def test_gradient_parity_small_256(kind):
    print(f"gradient small N=256 {kind}", flush=True)
    c = Case(small(256, 3, 2, 3, 33))
    _check_grads(c, c.engine(kind), kind)


def test_forward_parity_large_256_batch():
    """The N=256 / 30-slice / 8-mode workload at its launch batch of 16."""
    print("forward large_256 B=16", flush=True)
    c = Case(synth.workload("large_256", scan=16), perturb=False)
    eng = c.engine()
    I = eng.forward(*c.gpu_args())
    eng.sync()
    e = rel(I.cpu().numpy(), c.I_true)
    print(f"forward rel-L2 {e:.2e}", flush=True)
    assert e < 1e-5


def test_gradient_parity_large_256():
    print("gradient large_256 B=2", flush=True)
    c = Case(synth.workload("large_256", scan=2))
    _check_grads(c, c.engine())


def test_gradient_parity_large_256_launch_batch():
    """The N=256 / 30-slice / 8-mode workload at its launch batch of 16 (the
    configuration the benchmark times): loss and all six gradients against the
    oracle, which runs one position per worker process.  The object gradient
    is compared on the window the batch's patches cover and must be exactly
    zero outside it."""
    from tests import oracle_pool
    print("gradient large_256 B=16", flush=True)
    w = synth.workload("large_256", scan=16)
    lam = synth.wavelength_A(w.kv)
    rng = np.random.default_rng(1000)
    amp_t, ph_t = w.amp.astype(np.float32), w.phase.astype(np.float32)
    probe, pos, tilt, dz = w.probe.astype(np.complex64), w.pos.astype(np.float32), w.tilt.astype(np.float32), \
        np.float32(w.dz)
    I_true = oracle_pool.intensities(amp_t, ph_t, probe, pos, tilt, dz, w.dx, lam)
    print("oracle intensities done", flush=True)
    meas = rng.poisson(I_true).astype(np.float32)
    amp = (1.0 + 0.9 * (amp_t - 1.0)).astype(np.float32)
    phase = (0.8 * ph_t + 0.02 * rng.standard_normal(ph_t.shape)).astype(np.float32)
    ref = oracle_pool.gradients(amp, phase, probe, pos, tilt, dz, w.dx, lam, meas)
    print("oracle gradients done", flush=True)
    from paper_2505_07814_amd.ptyr import Engine
    eng = Engine(w.N, w.M, w.S, w.H, w.W, 16, w.dx, lam, device=DEV)
    args = (T(amp), T(phase), T(probe), T(pos), T(tilt), T(np.array([dz], np.float32)))
    loss, g = eng.adjoint(*args, T(meas))
    eng.sync()
    (y0, y1), (x0, x1) = ref["window"]
    errs = {"loss": abs(float(loss.cpu()[0]) - ref["loss"]) / abs(ref["loss"])}
    for k in ("amp", "phase"):
        full = g[k].cpu().numpy()
        errs[k] = rel(full[:, y0:y1, x0:x1], ref[k])
        full[:, y0:y1, x0:x1] = 0
        assert not full.any(), k
    for k in ("probe", "pos", "tilt"):
        errs[k] = rel(g[k].cpu().numpy(), ref[k])
    errs["dz"] = rel(g["dz"].cpu().numpy(), [ref["dz"]])
    print({k: f"{v:.2e}" for k, v in errs.items()}, flush=True)
    for k, v in errs.items():
        assert v < (1e-6 if k == "loss" else 1e-4), (k, v)


# ---------------------------------------------------------------- global tilt, error paths
@pytest.mark.parametrize("N,S,M,B,seed", [(64, 4, 2, 5, 51), (128, 3, 2, 3, 52)])
def test_global_tilt_parity(N, S, M, B, seed):
    """PTYR_GLOBAL_TILT: one (th_y, th_x) pair for every position.  The forward
    equals the oracle's with that pair repeated for each position; the tilt
    gradient is the sum of the oracle's per-position tilt gradients; the other
    five gradients match as usual."""
    print(f"global tilt N={N} S={S} M={M} B={B}", flush=True)
    c = Case(small(N, S, M, B, seed))
    th = np.array([1.5e-3, -2.5e-3], np.float32)
    tilt_rows = np.tile(th, (B, 1))
    I_ref = ms.forward(c.amp, c.phase, c.probe, c.pos, tilt_rows, c.dz, c.w.dx, c.lam)
    ref = ms.gradients(c.amp, c.phase, c.probe, c.pos, tilt_rows, c.dz, c.w.dx, c.lam, c.meas)
    eng = c.engine(global_tilt=True)
    args = list(c.gpu_args())
    args[4] = T(th)
    I = eng.forward(*args)
    loss, g = eng.adjoint(*args, T(c.meas))
    eng.sync()
    errs = {"I": rel(I.cpu().numpy(), I_ref),
            "loss": abs(float(loss.cpu()[0]) - ref.loss) / abs(ref.loss),
            "amp": rel(g["amp"].cpu().numpy(), ref.amp), "phase": rel(g["phase"].cpu().numpy(), ref.phase),
            "probe": rel(g["probe"].cpu().numpy(), ref.probe), "pos": rel(g["pos"].cpu().numpy(), ref.pos),
            "tilt": rel(g["tilt"].cpu().numpy(), ref.tilt.sum(axis=0)),
            "dz": rel(g["dz"].cpu().numpy(), [ref.dz])}
    print({k: f"{v:.2e}" for k, v in errs.items()}, flush=True)
    assert tuple(g["tilt"].shape) == (2,)
    for k, v in errs.items():
        assert v < {"I": 1e-5, "loss": 1e-6}.get(k, 1e-4), (k, v)


def test_global_tilt_step_parity():
    """ptyr_step with a global tilt: the tilt's Adam sees the summed gradient."""
    from paper_2505_07814_amd.ptyr import AdamState, Engine
    w = small(64, 3, 2, 6, 53)
    c = Case(w)
    th = np.array([1e-3, 2e-3], np.float32)
    eng = Engine(64, 2, 3, w.H, w.W, 6, w.dx, c.lam, device=DEV, n_scan=6, global_tilt=True)
    args = list(c.gpu_args())
    args[4] = T(th)
    st = AdamState(*[t.clone() for t in args])
    lr = dict(tilt=1e-4)
    idx = torch.arange(6, dtype=torch.int32, device=DEV)
    eng.step(st, idx, T(c.meas), lr)
    eng.sync()
    ref = ms.gradients(c.amp, c.phase, c.probe, c.pos, np.tile(th, (6, 1)), c.dz, w.dx, c.lam, c.meas)
    rp, _, _ = adam_step(th.astype(np.float64), ref.tilt.sum(axis=0), np.zeros(2), np.zeros(2), 0, 1e-4)
    got = st.tilt.cpu().numpy().astype(np.float64)
    # the first Adam step moves each entry by lr * sign(g) (to eps): the sign is what matters
    assert np.allclose(got, rp, rtol=0, atol=1e-8), (got, rp)
    for k in ("amp", "phase", "probe", "pos", "dz"):
        assert torch.equal(getattr(st, k), args[("amp", "phase", "probe", "pos", "tilt", "dz").index(k)]), k


def test_nonfinite_pattern_is_reported():
    """PTYR_CHECK_FINITE: a NaN in the measured batch is reported by ptyr_sync
    as PTYR_E_NONFINITE (the same batch without the flag is not checked)."""
    from paper_2505_07814_amd import _lib as L
    c = Case(small(64, 2, 1, 3, 54))
    meas = c.meas.copy()
    meas[1, 5, 7] = np.nan
    eng = c.engine(check_finite=True)
    eng.adjoint(*c.gpu_args(), T(meas))
    with pytest.raises(L.PtyrError) as e:
        eng.sync()
    assert e.value.status == L.PTYR_E_NONFINITE
    eng.adjoint(*c.gpu_args(), T(c.meas))
    eng.sync()                                             # flag cleared, finite data pass
    I = T(np.abs(c.I_true).astype(np.float32))
    eng.loss(I, T(meas))
    with pytest.raises(L.PtyrError) as e:
        eng.sync()
    assert e.value.status == L.PTYR_E_NONFINITE


def test_zero_measured_batch_is_reported():
    """A measured batch that is zero everywhere has no loss normaliser (Eq. 5-6
    divide by its mean): ptyr_sync reports PTYR_E_ARG, and the loss and the
    gradients stay zero instead of NaN."""
    from paper_2505_07814_amd import _lib as L
    c = Case(small(64, 2, 1, 3, 55))
    eng = c.engine()
    zero = np.zeros_like(c.meas)
    loss, g = eng.adjoint(*c.gpu_args(), T(zero))
    with pytest.raises(L.PtyrError) as e:
        eng.sync()
    assert e.value.status == L.PTYR_E_ARG
    assert float(loss.cpu()[0]) == 0.0
    for k, v in g.items():
        assert torch.isfinite(v).all() and not v.any(), k
    L0, _ = eng.loss(T(c.I_true.astype(np.float32)), T(zero))
    with pytest.raises(L.PtyrError) as e:
        eng.sync()
    assert e.value.status == L.PTYR_E_ARG


@pytest.mark.parametrize("reuse", [False, True])
def test_repeated_row_is_reported(reuse):
    """A gradient batch must hold distinct rows: a row met again is skipped and
    reported by ptyr_sync as PTYR_E_ARG; the gradient is that of the batch
    without the repeat."""
    from paper_2505_07814_amd import _lib as L
    c = Case(small(64, 2, 1, 4, 56))
    eng = c.engine()
    idx = torch.tensor([0, 2, 2, 3], dtype=torch.int32, device=DEV)
    if reuse:
        eng.forward(*c.gpu_args(), idx=idx)
        eng.sync()                                       # the forward allows repeats
    loss, g = eng.adjoint(*c.gpu_args(), T(c.meas), idx=idx, reuse=reuse)
    with pytest.raises(L.PtyrError) as e:
        eng.sync()
    assert e.value.status == L.PTYR_E_ARG
    rows = [0, 2, 3]
    ref = ms.gradients(c.amp, c.phase, c.probe, c.pos[rows], c.tilt[rows], c.dz, c.w.dx, c.lam, c.meas[rows])
    # the skipped row's detector values are left out of the gradient and of the
    # loss sums but still count in the batch size of the means: compare what
    # does not depend on that normalisation, the direction of the phase gradient
    gp = g["phase"].cpu().numpy()
    cos = float(np.vdot(gp, ref.phase) / (np.linalg.norm(gp) * np.linalg.norm(ref.phase)))
    assert cos > 1 - 1e-6, cos
    gpos = g["pos"].cpu().numpy()
    assert not gpos[1].any()                              # row 1 never used
    eng.adjoint(*c.gpu_args(), T(c.meas), idx=torch.tensor([0, 1, 2, 3], dtype=torch.int32, device=DEV))
    eng.sync()


# ---------------------------------------------------------------- weighted data terms (Eq. 9)
TERMS = [("gaussian", 0.7, 0.5), ("poisson", 0.4, 1.0)]


def _mix_engine_kw():
    return dict(w_gaussian=0.7, w_poisson=0.4, p_gaussian=0.5, p_poisson=1.0)


def test_loss_terms_parity():
    """ptyr_loss with w_1 L_Gaussian(p=0.5) + w_2 L_Poisson(p=1), alone and with
    the PACBED term: loss and dL/dI against the oracle."""
    rng = np.random.default_rng(57)
    Im = rng.gamma(2.0, 20.0, (5, 64, 64)).astype(np.float32)
    Im[:, :3, :3] = 0.0
    Ie = rng.poisson(Im + 0.5).astype(np.float32)
    from paper_2505_07814_amd.ptyr import Engine
    for pw in (0.0, 0.5):
        eng = Engine(64, 1, 1, 64, 64, 5, 0.2, 0.02, pacbed_w=pw, device=DEV, **_mix_engine_kw())
        L, g = eng.loss(T(Im), T(Ie), want_grad=True)
        eng.sync()
        L0, g0 = ms.loss(Im, Ie, terms=TERMS, pacbed_w=pw)
        el, eg = abs(float(L.cpu()[0]) - L0) / abs(L0), rel(g.cpu().numpy(), g0)
        print(f"pacbed_w={pw}: loss {el:.2e} dL/dI {eg:.2e}", flush=True)
        assert el <= 1e-6 and eg < 1e-6


@pytest.mark.parametrize("B", [5, 90])
def test_loss_terms_gradient_parity(B):
    """Loss and all six gradients with both data terms weighted (one stream:
    the weights need both batch factors); B = 90 would otherwise take the
    two-stream schedule."""
    print(f"weighted data terms B={B}", flush=True)
    if B == 90:
        w = synth.small_case(N=64, S=3, M=3, B=90, H=64 + 60, W=64 + 70, seed=31)
    else:
        w = small(64, 3, 2, 5, 12)
    c = Case(w)
    eng = c.engine(**_mix_engine_kw())
    loss, g = eng.adjoint(*c.gpu_args(), T(c.meas))
    eng.sync()
    ref = ms.gradients(c.amp, c.phase, c.probe, c.pos, c.tilt, c.dz, w.dx, c.lam, c.meas, terms=TERMS)
    errs = {"loss": abs(float(loss.cpu()[0]) - ref.loss) / abs(ref.loss)}
    for k in ("amp", "phase", "probe", "pos", "tilt"):
        errs[k] = rel(g[k].cpu().numpy(), getattr(ref, k))
    errs["dz"] = rel(g["dz"].cpu().numpy(), [ref.dz])
    print({k: f"{v:.2e}" for k, v in errs.items()}, flush=True)
    for k, v in errs.items():
        assert v < (1e-6 if k == "loss" else 1e-4), (k, v)
    ref1 = ms.gradients(c.amp, c.phase, c.probe, c.pos, c.tilt, c.dz, w.dx, c.lam, c.meas, terms=TERMS[:1])
    assert rel(ref.phase, ref1.phase) > 1e-3            # the second term is really there
