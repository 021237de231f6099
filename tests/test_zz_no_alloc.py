"""ptyr_loss_noalloc (the allocation-free loss: its scratch is a static device
array of the library instead of a context's workspace) against ptyr_loss on
the same inputs, through the C ABI.  The two run the same kernels with the
same launch shapes, so loss and dL/dI must agree bit for bit: on two calls in
a row, the second with a smaller batch (the scratch keeps the first call's
contents), with the PACBED term and Eq. 9's two weighted data terms, and with
the error flag for a bad measured-row index."""
import ctypes as C

import numpy as np
import pytest
import torch

from paper_2505_07814_amd import _lib as L
from paper_2505_07814_amd.ptyr import Engine

pytestmark = pytest.mark.gpu

DEV = torch.device("cuda:0")


def T(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def noalloc(eng, I, Ie, midx=None, want_grad=True):
    lib = L.lib()
    B = I.shape[0]
    loss = torch.full((1,), float("nan"), dtype=torch.float64, device=DEV)
    g = torch.full_like(I, float("nan")) if want_grad else None
    err = torch.zeros(1, dtype=torch.int32, device=DEV)
    p = lambda t: None if t is None else C.c_void_p(t.data_ptr())
    st = lib.ptyr_loss_noalloc(C.byref(eng.geom), p(I), p(Ie), p(midx), Ie.shape[0], B, p(loss), p(g), p(err),
                               C.c_void_p(eng.stream.cuda_stream))
    assert st == L.PTYR_OK, st
    torch.cuda.synchronize()
    return loss, g, int(err.cpu()[0])


def patterns(B, N, seed):
    rng = np.random.default_rng(seed)
    Im = rng.gamma(2.0, 20.0, (B, N, N)).astype(np.float32)
    Im[:, :2, :2] = 0.0
    Ie = rng.poisson(Im + 0.5).astype(np.float32)
    return T(Im), T(Ie)


@pytest.mark.parametrize("kw", [dict(), dict(pacbed_w=0.5), dict(w_gaussian=0.7, w_poisson=0.4),
                                dict(loss="poisson", pacbed_w=0.25)])
def test_noalloc_loss_matches_context_loss(kw):
    N = 128
    eng = Engine(N, 1, 1, N, N, 12, 0.15, 0.02, device=DEV, **kw)
    for B, seed in ((12, 1), (5, 2)):                 # second call: smaller batch
        I, Ie = patterns(B, N, seed)
        L0, g0 = eng.loss(I, Ie, want_grad=True)
        eng.sync()
        L1, g1, err = noalloc(eng, I, Ie)
        print(kw, B, float(L0.cpu()[0]), float(L1.cpu()[0]), flush=True)
        assert err == 0
        assert torch.equal(L0, L1), (float(L0.cpu()[0]), float(L1.cpu()[0]))
        assert torch.equal(g0, g1)
        # loss only (dL/dI NULL)
        L2, _, err = noalloc(eng, I, Ie, want_grad=False)
        assert err == 0 and torch.equal(L0, L2)


def test_noalloc_rows_and_errors():
    """Measured rows through an index; a row index outside [0, n_meas) sets the
    index bit of err_dev (and a later good call is clean)."""
    N = 64
    eng = Engine(N, 1, 1, N, N, 6, 0.2, 0.02, device=DEV)
    I, _ = patterns(4, N, 3)
    _, Ie = patterns(9, N, 4)
    midx = torch.tensor([8, 0, 3, 5], dtype=torch.int32, device=DEV)
    L0, g0 = eng.loss(I, Ie, meas_idx=midx, want_grad=True)
    eng.sync()
    L1, g1, err = noalloc(eng, I, Ie, midx)
    assert err == 0 and torch.equal(L0, L1) and torch.equal(g0, g1)
    bad = torch.tensor([8, 0, 9, 5], dtype=torch.int32, device=DEV)
    _, _, err = noalloc(eng, I, Ie, bad)
    assert err & L.PTYR_ERRBIT_INDEX
    _, _, err = noalloc(eng, I, Ie, midx)
    assert err == 0


def test_noalloc_rejects_bad_arguments():
    eng = Engine(64, 1, 1, 64, 64, 4, 0.2, 0.02, device=DEV)
    lib = L.lib()
    I, Ie = patterns(2, 64, 5)
    out = torch.empty(1, dtype=torch.float64, device=DEV)
    p = lambda t: C.c_void_p(t.data_ptr())
    assert lib.ptyr_loss_noalloc(C.byref(eng.geom), p(I), p(Ie), None, 0, 2, p(out), None, None, None) == L.PTYR_E_ARG
    err = torch.zeros(1, dtype=torch.int32, device=DEV)
    assert lib.ptyr_loss_noalloc(C.byref(eng.geom), p(I), p(Ie), None, 0, 0, p(out), None, p(err),
                                 None) == L.PTYR_E_ARG
    g = L.Geom.from_buffer_copy(eng.geom)
    g.N = 96
    assert lib.ptyr_loss_noalloc(C.byref(g), p(I), p(Ie), None, 0, 2, p(out), None, p(err), None) == L.PTYR_E_ARG
