"""The learned initial guess, end to end on the GPU: training pairs from the
library's forward model, training with the BF16 matrix-core kernels, and the
gain over the plain initial object in the multislice reconstruction.

The network is trained here on 300 objects (19,200 neighbourhoods, a tenth
of the full set) for 12 epochs so that the test stays short; the full training
run is `bench.py --learned-init`.  The gain measured is that of this smaller
net, on the held-out object (seed 999).
"""
import numpy as np
import pytest
import torch

from paper_2505_07814_amd import learned_init as li
from paper_2505_07814_amd import synth
from paper_2505_07814_amd.cnn import ConvInit

pytestmark = pytest.mark.gpu

DEV = torch.device("cuda:0")


@pytest.fixture(scope="module")
def trained():
    data = li.make_dataset(300, DEV)
    assert data.patterns.shape == (30000, 64, 64) and data.nbr.shape == (19200, 9)
    net = ConvInit(256, device=DEV)
    res = li.train(data, epochs=12, batch=256, lr=1e-3, net=net, log=print)
    return net, res


def test_training_reduces_loss(trained):
    _, res = trained
    print("epoch losses", res.losses)
    assert all(np.isfinite(res.losses))
    assert res.losses[-1] < 0.9 * res.losses[0]


def test_learned_init_reaches_target_sooner(trained):
    net, res = trained
    case = li.eval_case(DEV)
    plain = torch.from_numpy(synth.plain_init(1, synth.LI_H, synth.LI_H, 5)[1][0].astype(np.float32)).to(DEV)
    li.learned_phase(net, res.params, case, plain)          # warm-up of the inference launches
    li.reconstruct(case, plain, 2)                           # and of the reconstruction launches
    torch.cuda.synchronize()
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    t0.record()
    init = li.learned_phase(net, res.params, case, plain)
    t1.record()
    torch.cuda.synchronize()
    setup = t0.elapsed_time(t1) / 1e3
    r_plain = li.reconstruct(case, plain, 40)
    r_learn = li.reconstruct(case, init, 40, setup_seconds=setup)
    print("plain  ", np.round(r_plain.errors, 4).tolist(), r_plain.iterations_to_target)
    print("learned", np.round(r_learn.errors, 4).tolist(), r_learn.iterations_to_target)
    assert r_learn.errors[0] < 0.9 * r_plain.errors[0]
    assert r_plain.iterations_to_target is not None and r_learn.iterations_to_target is not None
    assert r_learn.iterations_to_target < r_plain.iterations_to_target
    # metric 2 is wall time: the learned start, inference and stitching
    # included, reaches the target in less time on the same GPU
    print(f"seconds to target: learned {r_learn.seconds_to_target:.4f} (inference {setup:.4f}), "
          f"plain {r_plain.seconds_to_target:.4f}")
    assert r_learn.seconds_to_target < r_plain.seconds_to_target
