"""FP64 Adam step (oracle).

TEST INFRASTRUCTURE ONLY: imported by tests, the smoke check and the
benchmark's CPU baseline, never by the product path.

The paper optimises its parameters with PyTorch's Adam by default (Sec.
"Optimizers and loss functions"); the update below is Kingma & Ba's Adam with
bias correction, in the form PyTorch documents, applied elementwise (complex
parameters are updated on their real and imaginary parts separately).
"""
from __future__ import annotations

import numpy as np


def adam_step(param, grad, m, v, step, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update.  `step` is the number of updates already taken;
    returns (param, m, v) after update number step+1."""
    cplx = np.iscomplexobj(param)
    as_real = (lambda a: np.stack([a.real, a.imag], -1)) if cplx else (lambda a: np.asarray(a, np.float64))
    p, g = as_real(param), as_real(grad)
    mm, vv = as_real(m), as_real(v)
    t = step + 1
    mm = beta1 * mm + (1 - beta1) * g
    vv = beta2 * vv + (1 - beta2) * g * g
    mhat = mm / (1 - beta1 ** t)
    vhat = vv / (1 - beta2 ** t)
    p = p - lr * mhat / (np.sqrt(vhat) + eps)
    if cplx:
        back = lambda a: a[..., 0] + 1j * a[..., 1]
        return back(p), back(mm), back(vv)
    return p, mm, vv
