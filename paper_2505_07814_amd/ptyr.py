"""Python front end of libptyr: device memory and streams come from PyTorch,
every step of the computation runs in the library's HIP kernels.

Conventions (see include/ptyr.h): object amplitude / phase are float32
(S, H, W); the probe is complex64 (M, N, N); positions and tilts are float32
(rows, 2) in (y, x) order, positions in object pixels, tilts in radians (or a
single (2,) pair with global_tilt); dz is a float32 (1,) tensor in angstrom;
batch index arrays are int32.  Measured and model intensities are float32
(B, N, N) with zero frequency at (N/2, N/2).
"""
from __future__ import annotations

import ctypes as C
from typing import Optional

import torch

from . import _lib as L


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else C.c_void_p(t.data_ptr())


def _need(t, name, dtype, shape=None, device=None):
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch.Tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_cuda:
        raise ValueError(f"{name} must be a device tensor")
    if device is not None and t.device != device:
        raise ValueError(f"{name} is on {t.device}, the engine on {device}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")


class Engine:
    """One libptyr context: geometry, workspace and stream.

    loss: 'gaussian' (Eq. 5, default p=0.5) or 'poisson' (Eq. 6, default p=1);
    w_gaussian, w_poisson: weights w_1, w_2 of Eq. 9's two data terms (both 0 =
    the `loss` term alone at weight 1), with powers p_gaussian, p_poisson
    (None = 0.5 and 1);
    sparse_w: weight of the L1 sparsity term of the object phase (0 = off);
    pacbed_w: weight of the PACBED term of the batch-mean patterns (0 = off).
    wave_budget: bytes the forward may keep for the gradient (None = all
    waves, B_max*M*2S*N*N*8); below that the gradient recomputes waves per
    slice from checkpoints.  n_scan: positions addressable by step()."""

    def __init__(self, N, M, S, H, W, B_max, dx, lam, loss="gaussian", p=None, wave_budget=None,
                 global_tilt=False, check_finite=False, n_scan=0, sparse_w=0.0, pacbed_w=0.0, n_obj=1,
                 w_gaussian=0.0, w_poisson=0.0, p_gaussian=None, p_poisson=None, device=None, stream=None):
        self.lib = L.lib()
        kind = {"gaussian": L.PTYR_LOSS_GAUSSIAN, "poisson": L.PTYR_LOSS_POISSON}[loss]
        if p is None:
            p = 0.5 if kind == L.PTYR_LOSS_GAUSSIAN else 1.0
        if wave_budget is None:
            wave_budget = B_max * M * n_obj * 2 * S * N * N * 8     # keep every slice's waves
        flags = (L.PTYR_GLOBAL_TILT if global_tilt else 0) | (L.PTYR_CHECK_FINITE if check_finite else 0)
        self.geom = L.Geom(N, M, S, H, W, B_max, float(dx), float(lam), kind, float(p),
                           int(wave_budget), flags, int(n_scan), float(sparse_w),
                           float(pacbed_w), int(n_obj), float(w_gaussian), float(w_poisson),
                           float(p_gaussian or 0.0), float(p_poisson or 0.0))
        L.check(self.lib.ptyr_check_geom(C.byref(self.geom)), "geometry")
        self.N, self.M, self.S, self.H, self.W, self.B_max = N, M, S, H, W, B_max
        self.n_obj = int(n_obj)
        # object arrays: (S, H, W) for one object mode, (n_obj, S, H, W) for several
        self.obj_shape = (S, H, W) if self.n_obj == 1 else (self.n_obj, S, H, W)
        self.global_tilt = global_tilt
        self.device = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        nbytes = self.lib.ptyr_workspace_bytes(C.byref(self.geom))
        self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        base = self.workspace.data_ptr()
        self._ws_ptr = (base + 255) // 256 * 256
        self._ws_bytes = nbytes
        ctx = C.c_void_p()
        L.check(self.lib.ptyr_create(C.byref(self.geom), C.c_void_p(self._ws_ptr), nbytes,
                                     C.c_void_p(self.stream.cuda_stream), C.byref(ctx)), "ptyr_create")
        self._ctx = ctx
        self.forward_epoch = 0

    def __del__(self):
        ctx = getattr(self, "_ctx", None)
        if ctx is not None and ctx.value:
            try:
                self.lib.ptyr_destroy(ctx)
            except Exception:
                pass
            self._ctx = None

    # -------------------------------------------------------------- helpers
    @property
    def checkpoint_stride(self) -> int:
        k = C.c_int()
        L.check(self.lib.ptyr_checkpoint_plan(C.byref(self.geom), C.byref(k)), "checkpoint plan")
        return k.value

    def _check_params(self, amp, phase, probe, pos, tilt, dz, idx, B):
        M, N = self.M, self.N
        d = self.device
        _need(amp, "amp", torch.float32, self.obj_shape, d)
        _need(phase, "phase", torch.float32, self.obj_shape, d)
        _need(probe, "probe", torch.complex64, (M, N, N), d)
        _need(pos, "pos", torch.float32, None, d)
        if pos.dim() != 2 or pos.shape[1] != 2:
            raise ValueError("pos must be (rows, 2)")
        _need(tilt, "tilt", torch.float32, None, d)
        if self.global_tilt:
            if tilt.numel() != 2:
                raise ValueError("tilt must hold one (th_y, th_x) pair with global_tilt")
        elif tuple(tilt.shape) != tuple(pos.shape):
            raise ValueError("tilt must have the shape of pos")
        _need(dz, "dz", torch.float32, (1,), d)
        rows = pos.shape[0]
        if idx is not None:
            _need(idx, "idx", torch.int32, (B,), d)
        elif rows < B:
            raise ValueError("fewer positions than the batch")
        return rows

    def timing(self, on: bool = True):
        """Bracket the fused kernels with HIP events on the engine's stream."""
        L.check(self.lib.ptyr_timing_enable(self._ctx, 1 if on else 0), "ptyr_timing_enable")

    def timing_read(self):
        """{'forward': (total_ms, launches), 'gradient': (...), 'rz': (...)} for
        the kernels launched since timing was enabled; clears the record (it
        is read once, so all kernels are read together)."""
        out = {}
        for name, k in (("forward", L.PTYR_K_FORWARD), ("gradient", L.PTYR_K_GRADIENT), ("rz", L.PTYR_K_RZ)):
            ms, n = C.c_double(), C.c_int()
            L.check(self.lib.ptyr_timing_read(self._ctx, k, C.byref(ms), C.byref(n)), "ptyr_timing_read")
            if n.value:
                out[name] = (ms.value, n.value)
        L.check(self.lib.ptyr_timing_enable(self._ctx, 1), "ptyr_timing_enable")
        return out

    def sync(self):
        """Wait for the stream; raise on asynchronous errors (bounds, indices, non-finite)."""
        L.check(self.lib.ptyr_sync(self._ctx), "ptyr_sync")

    # -------------------------------------------------------------- entry points
    def forward(self, amp, phase, probe, pos, tilt, dz, idx=None, B=None, out=None):
        """Model intensities (B, N, N), fftshifted."""
        B = (idx.numel() if idx is not None else pos.shape[0]) if B is None else B
        rows = self._check_params(amp, phase, probe, pos, tilt, dz, idx, B)
        if out is None:
            out = torch.empty((B, self.N, self.N), dtype=torch.float32, device=self.device)
        _need(out, "out", torch.float32, (B, self.N, self.N), self.device)
        L.check(self.lib.ptyr_forward(self._ctx, _ptr(amp), _ptr(phase), _ptr(probe), _ptr(pos), _ptr(tilt),
                                      _ptr(dz), _ptr(idx), rows, B, _ptr(out)), "ptyr_forward")
        self.forward_epoch += 1
        return out

    def loss(self, I_model, I_meas, meas_idx=None, want_grad=False):
        """(loss as a (1,) float64 device tensor, dL/dI or None)."""
        B = I_model.shape[0]
        _need(I_model, "I_model", torch.float32, (B, self.N, self.N), self.device)
        _need(I_meas, "I_meas", torch.float32, None, self.device)
        if meas_idx is not None:
            _need(meas_idx, "meas_idx", torch.int32, (B,), self.device)
        elif I_meas.shape[0] < B:
            raise ValueError("fewer measured patterns than the batch")
        out = torch.empty(1, dtype=torch.float64, device=self.device)
        g = torch.empty_like(I_model) if want_grad else None
        L.check(self.lib.ptyr_loss(self._ctx, _ptr(I_model), _ptr(I_meas), _ptr(meas_idx), I_meas.shape[0], B,
                                   _ptr(out), _ptr(g)), "ptyr_loss")
        return out, g

    def adjoint(self, amp, phase, probe, pos, tilt, dz, I_meas, idx=None, B=None, grads=None, reuse=False,
                want=("amp", "phase", "probe", "pos", "tilt", "dz")):
        """Loss and accumulated gradients.  grads: dict of existing gradient
        tensors to accumulate into (created zero otherwise)."""
        B = (idx.numel() if idx is not None else pos.shape[0]) if B is None else B
        rows = self._check_params(amp, phase, probe, pos, tilt, dz, idx, B)
        _need(I_meas, "I_meas", torch.float32, None, self.device)
        if I_meas.shape[0] < (rows if idx is not None else B):
            raise ValueError("fewer measured patterns than rows")
        like = dict(amp=amp, phase=phase, probe=probe, pos=pos, tilt=tilt, dz=dz)
        grads = dict(grads or {})
        for k in want:
            if k not in grads:
                grads[k] = torch.zeros_like(like[k])
            else:
                _need(grads[k], "grad " + k, like[k].dtype, like[k].shape, self.device)
        loss = torch.empty(1, dtype=torch.float64, device=self.device)
        flags = L.PTYR_REUSE_FORWARD if reuse else 0
        L.check(self.lib.ptyr_adjoint(self._ctx, _ptr(amp), _ptr(phase), _ptr(probe), _ptr(pos), _ptr(tilt),
                                      _ptr(dz), _ptr(idx), rows, B, _ptr(I_meas),
                                      _ptr(grads.get("amp")), _ptr(grads.get("phase")), _ptr(grads.get("probe")),
                                      _ptr(grads.get("pos")), _ptr(grads.get("tilt")), _ptr(grads.get("dz")),
                                      _ptr(loss), flags), "ptyr_adjoint")
        return loss, grads

    def step(self, state: "AdamState", idx, I_meas_all, lr: dict, betas=(0.9, 0.999), eps=1e-8):
        """One mini-batch Adam update of `state` in place; returns the batch loss (device)."""
        B = idx.numel()
        _need(idx, "idx", torch.int32, (B,), self.device)
        _need(I_meas_all, "I_meas_all", torch.float32, (state.pos.shape[0], self.N, self.N), self.device)
        self._check_params(state.amp, state.phase, state.probe, state.pos, state.tilt, state.dz, idx, B)
        rates = L.LR(*(float(lr.get(k, 0.0)) for k in ("amp", "phase", "probe", "pos", "tilt", "dz")),
                     float(betas[0]), float(betas[1]), float(eps))
        prm = state.as_struct()
        loss = torch.empty(1, dtype=torch.float64, device=self.device)
        L.check(self.lib.ptyr_step(self._ctx, C.byref(prm), _ptr(idx), B, _ptr(I_meas_all), C.byref(rates),
                                   _ptr(loss)), "ptyr_step")
        state.step = prm.step
        self.forward_epoch += 1
        return loss


    def bind_step(self, state: "AdamState", I_meas_all, lr: dict, betas=(0.9, 0.999), eps=1e-8):
        """`step` for a loop of updates of one state with fixed rates: the
        parameters, moments, measured data and rates are checked and marshalled
        once, and the returned function(idx) checks only idx before calling
        ptyr_step (the host work per call of `step` is then left out; at small
        batches it is comparable to the device work).  The function keeps the
        tensors the state held when it was bound and writes each batch's loss
        into one device buffer, which it returns."""
        B_max = self.B_max
        _need(I_meas_all, "I_meas_all", torch.float32, (state.pos.shape[0], self.N, self.N), self.device)
        self._check_params(state.amp, state.phase, state.probe, state.pos, state.tilt, state.dz, None, 1)
        rates = L.LR(*(float(lr.get(k, 0.0)) for k in ("amp", "phase", "probe", "pos", "tilt", "dz")),
                     float(betas[0]), float(betas[1]), float(eps))
        prm = state.as_struct()
        loss = torch.empty(1, dtype=torch.float64, device=self.device)
        fn, ctx, meas, lptr = self.lib.ptyr_step, self._ctx, _ptr(I_meas_all), _ptr(loss)
        dev = self.device

        def run(idx):
            B = idx.numel()
            if idx.dtype != torch.int32 or idx.device != dev or not idx.is_contiguous() or not 0 < B <= B_max:
                _need(idx, "idx", torch.int32, (B,), dev)
                raise ValueError(f"batch of {B} rows, engine B_max {B_max}")
            prm.step = state.step
            L.check(fn(ctx, C.byref(prm), C.c_void_p(idx.data_ptr()), B, meas, C.byref(rates), lptr), "ptyr_step")
            state.step = prm.step
            self.forward_epoch += 1
            return loss
        return run

    def constrain(self, amp=None, phase=None, probe=None, rz_sigma=0.0, phase_positive=False,
                  probe_orthogonal=False, kz_beta=0.0, kz_alpha=0.0, kz_dz=0.0):
        """Per-iteration constraints in place (include/ptyr.h, ptyr_constrain):
        k_z filter (kz_beta, kz_alpha in angstrom^2, slice spacing kz_dz) and
        r_z depth filter (rz_sigma slices) of amplitude and phase, clipping of
        negative phase, orthogonalisation of the probe modes."""
        for t, n, dt in ((amp, "amp", torch.float32), (phase, "phase", torch.float32)):
            if t is not None:
                _need(t, n, dt, self.obj_shape, self.device)
        if probe is not None:
            _need(probe, "probe", torch.complex64, (self.M, self.N, self.N), self.device)
        cfg = L.Constraints(float(rz_sigma), int(bool(phase_positive)), int(bool(probe_orthogonal)),
                            float(kz_beta), float(kz_alpha), float(kz_dz))
        L.check(self.lib.ptyr_constrain(self._ctx, _ptr(amp), _ptr(phase), _ptr(probe), C.byref(cfg)),
                "ptyr_constrain")


class AdamState:
    """Parameters of one reconstruction with their Adam moments (device tensors)."""

    NAMES = ("amp", "phase", "probe", "pos", "tilt", "dz")

    def __init__(self, amp, phase, probe, pos, tilt, dz):
        self.amp, self.phase, self.probe, self.pos, self.tilt, self.dz = amp, phase, probe, pos, tilt, dz
        self.m = {k: torch.zeros_like(getattr(self, k)) for k in self.NAMES}
        self.v = {k: torch.zeros_like(getattr(self, k)) for k in self.NAMES}
        self.step = 0

    def as_struct(self):
        p = L.Params()
        for k in self.NAMES:
            setattr(p, k, getattr(self, k).data_ptr())
            setattr(p, "m_" + k, self.m[k].data_ptr())
            setattr(p, "v_" + k, self.v[k].data_ptr())
        p.n_pos = self.pos.shape[0]
        p.step = self.step
        return p


class MultisliceLoss(torch.autograd.Function):
    """Loss of the multislice model as an autograd node whose backward is the
    library's hand-derived gradient (no autograd graph through the model).
    The backward reuses the waves the forward kept (or recomputes them per
    slice from checkpoints when the engine's wave budget is smaller).

    The value is the engine's whole loss: with a sparsity term (sparse_w > 0),
    which needs the batch's object patches rather than the intensities, the
    forward runs ptyr_adjoint at once (value and gradient of the same
    function) and the backward scales the gradients it kept."""

    @staticmethod
    def forward(ctx, amp, phase, probe, pos, tilt, dz, I_meas, engine, idx):
        ctx.engine = engine
        ctx.idx = idx
        ctx.grads = None
        if engine.geom.sparse_w > 0.0:
            loss, ctx.grads = engine.adjoint(amp, phase, probe, pos, tilt, dz, I_meas, idx=idx)
            return loss[0]
        I = engine.forward(amp, phase, probe, pos, tilt, dz, idx=idx)
        loss, _ = engine.loss(I, I_meas, meas_idx=idx)
        ctx.epoch = engine.forward_epoch
        ctx.save_for_backward(amp, phase, probe, pos, tilt, dz, I_meas)
        return loss[0]

    @staticmethod
    def backward(ctx, grad_loss):
        g = ctx.grads
        if g is None:
            amp, phase, probe, pos, tilt, dz, I_meas = ctx.saved_tensors
            eng = ctx.engine
            reuse = eng.forward_epoch == ctx.epoch
            _, g = eng.adjoint(amp, phase, probe, pos, tilt, dz, I_meas, idx=ctx.idx, reuse=reuse)
        gl = grad_loss.to(torch.float32)
        out = []
        for k, need in zip(("amp", "phase", "probe", "pos", "tilt", "dz"), ctx.needs_input_grad[:6]):
            out.append(g[k] * gl if need else None)
        return (*out, None, None, None)


def multislice_loss(engine, amp, phase, probe, pos, tilt, dz, I_meas, idx=None):
    return MultisliceLoss.apply(amp, phase, probe, pos, tilt, dz, I_meas, engine, idx)
