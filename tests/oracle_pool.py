"""The oracle's gradient of a large batch, one scan position per worker process.

Test infrastructure: the FP64 oracle at the N = 256, 30-slice, 8-mode launch
batch takes about 15 s per position, so the positions run in parallel worker
processes.  The workers are started with the "spawn" method (fresh
interpreters that import only NumPy and `oracle/`, never the GPU runtime of
the parent) and read the object from .npy files memory-mapped from a
temporary directory.

The result is exactly the oracle's `gradients`: the batch loss and dL/dI come
from `ms.loss` over all positions' intensities (the batch normaliser couples
the rows), and the per-position adjoints `ms._adjoint` add up, as inside
`ms.gradients`.  The object gradient is returned on the bounding window of the
batch's patches (it is zero outside).
"""
from __future__ import annotations

import multiprocessing as mp
import os
import tempfile

import numpy as np

_W = {}


def _init(d):
    _W["amp"] = np.load(os.path.join(d, "amp.npy"), mmap_mode="r")
    _W["phase"] = np.load(os.path.join(d, "phase.npy"), mmap_mode="r")
    for k in ("probe", "pos", "tilt", "scal"):
        _W[k] = np.load(os.path.join(d, k + ".npy"))


def _intensity(j):
    from oracle import multislice as ms
    dz, dx, lam = _W["scal"]
    return ms.forward(_W["amp"], _W["phase"], _W["probe"], _W["pos"][j:j + 1], _W["tilt"][j:j + 1], dz, dx, lam)[0]


def _gradient(args):
    j, dI, win = args
    from oracle import multislice as ms
    dz, dx, lam = _W["scal"]
    amp = np.asarray(_W["amp"], np.float64)
    phase = np.asarray(_W["phase"], np.float64)
    probe = np.asarray(_W["probe"], np.complex128)
    pos, tilt = _W["pos"][j:j + 1], _W["tilt"][j:j + 1]
    _, traces = ms.forward(amp, phase, probe, pos, tilt, dz, dx, lam, return_trace=True)
    g_amp, g_phase, G_probe, g_pos, g_tilt, g_dz = ms._adjoint(amp, phase, probe, pos, tilt, dz, dx, lam,
                                                              dI[None], traces)
    (y0, y1), (x0, x1) = win
    return g_amp[:, y0:y1, x0:x1], g_phase[:, y0:y1, x0:x1], G_probe, g_pos[0], g_tilt[0], g_dz


def batch_window(pos, N):
    """Bounding window ((y0, y1), (x0, x1)) of the N x N patches of a batch."""
    from oracle import multislice as ms
    ts = np.array([ms.split_position(r, N)[0] for r in np.asarray(pos, np.float64)])
    return (int(ts[:, 0].min()), int(ts[:, 0].max()) + N), (int(ts[:, 1].min()), int(ts[:, 1].max()) + N)


class _Pool:
    """Worker processes holding the inputs of one batch."""

    def __init__(self, amp, phase, probe, pos, tilt, dz, dx, lam, workers):
        self._dir = tempfile.TemporaryDirectory()
        d = self._dir.name
        np.save(os.path.join(d, "amp.npy"), np.asarray(amp))
        np.save(os.path.join(d, "phase.npy"), np.asarray(phase))
        np.save(os.path.join(d, "probe.npy"), np.asarray(probe))
        np.save(os.path.join(d, "pos.npy"), np.asarray(pos))
        np.save(os.path.join(d, "tilt.npy"), np.asarray(tilt))
        np.save(os.path.join(d, "scal.npy"), np.array([float(dz), float(dx), float(lam)]))
        self.pool = mp.get_context("spawn").Pool(min(workers, len(pos)), initializer=_init, initargs=(d,))

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.pool.terminate()
        self.pool.join()
        self._dir.cleanup()


def intensities(amp, phase, probe, pos, tilt, dz, dx, lam, workers=16):
    """The oracle's fftshifted model intensities (B, N, N) of the batch."""
    with _Pool(amp, phase, probe, pos, tilt, dz, dx, lam, workers) as P:
        return np.stack(P.pool.map(_intensity, range(len(pos))))


def gradients(amp, phase, probe, pos, tilt, dz, dx, lam, meas, kind="gaussian", p=None, workers=16):
    """Loss and gradients of the batch (one object mode) as a dict; 'amp' and
    'phase' cover batch_window(pos, N)."""
    from oracle import multislice as ms
    N = probe.shape[-1]
    B = len(pos)
    win = batch_window(pos, N)
    with _Pool(amp, phase, probe, pos, tilt, dz, dx, lam, workers) as P:
        I = np.stack(P.pool.map(_intensity, range(B)))
        L, dI = ms.loss(I, meas, kind, p)
        parts = P.pool.map(_gradient, [(j, dI[j], win) for j in range(B)])
    out = dict(loss=L, window=win)
    out["amp"] = sum(q[0] for q in parts)
    out["phase"] = sum(q[1] for q in parts)
    out["probe"] = sum(q[2] for q in parts)
    out["pos"] = np.stack([q[3] for q in parts])
    out["tilt"] = np.stack([q[4] for q in parts])
    out["dz"] = float(sum(q[5] for q in parts))
    return out
