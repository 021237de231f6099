"""Pins of the FP64 conv-net oracle (learned initial guess).

The network is not in the paper, so its pins come from mathematics and from
independent library routines: PyTorch's float64 conv2d and autograd for the
cross-correlation and its adjoint, central finite differences for the whole
gradient, dot-product (adjoint) identities, and the bfloat16 rounding of
PyTorch for the rounding helper, plus hand-worked ties.
"""
import numpy as np
import pytest
import torch

from oracle import convnet as cn


def _torch_conv(a, W, b, s):
    return torch.nn.functional.conv2d(torch.from_numpy(a), torch.from_numpy(W), torch.from_numpy(b),
                                      stride=s, padding=1).numpy()


@pytest.mark.parametrize("stride,H,C,O", [(1, 9, 3, 5), (2, 10, 4, 2), (2, 7, 2, 3), (1, 1, 2, 2)])
def test_conv_matches_library(stride, H, C, O):
    rng = np.random.default_rng(H * 10 + stride)
    a = rng.standard_normal((2, C, H, H))
    W = rng.standard_normal((O, C, 3, 3))
    b = rng.standard_normal(O)
    z = cn.conv3x3(a, W, b, stride)
    ref = _torch_conv(a, W, b, stride)
    assert z.shape == ref.shape
    np.testing.assert_allclose(z, ref, rtol=1e-12, atol=1e-12)


def test_conv_single_tap_is_shift():
    """A kernel with one non-zero tap (u, v) shifts the image by (u-1, v-1)."""
    rng = np.random.default_rng(3)
    a = rng.standard_normal((1, 1, 6, 6))
    W = np.zeros((1, 1, 3, 3)); W[0, 0, 2, 0] = 1.0
    z = cn.conv3x3(a, W, np.zeros(1), 1)[0, 0]
    exp = np.zeros((6, 6)); exp[:5, 1:] = a[0, 0, 1:, :5]
    np.testing.assert_array_equal(z, exp)


@pytest.mark.parametrize("stride,H", [(1, 8), (2, 8), (2, 9)])
def test_conv_backward_is_adjoint(stride, H):
    """<conv(a) - b, g> = <a, da> and = <W, dW> (bilinearity), db = sum g."""
    rng = np.random.default_rng(stride * 100 + H)
    a = rng.standard_normal((2, 3, H, H))
    W = rng.standard_normal((4, 3, 3, 3))
    b = rng.standard_normal(4)
    z = cn.conv3x3(a, W, b, stride) - b[None, :, None, None]
    g = rng.standard_normal(z.shape)
    da, dW, db = cn.conv3x3_backward(a, W, g, stride)
    lhs = np.sum(z * g)
    assert abs(lhs - np.sum(a * da)) < 1e-11 * max(1.0, abs(lhs))
    assert abs(lhs - np.sum(W * dW)) < 1e-11 * max(1.0, abs(lhs))
    np.testing.assert_allclose(db, g.sum(axis=(0, 2, 3)), rtol=1e-13)


def _small_net(seed):
    """The real channel/stride layout on a small 9 x 12 x 12 input with
    positive and negative pre-activations, scaled so ReLUs are mixed."""
    ps = cn.init_params(seed)
    rng = np.random.default_rng(seed + 1)
    ps = [(W, 0.1 * rng.standard_normal(b.shape)) for W, b in ps]
    I = rng.exponential(20.0, (2, 9, 12, 12))
    t = rng.standard_normal((2, 6, 6))
    return ps, I, t


def test_net_shapes_and_library_forward():
    ps, I, t = _small_net(5)
    out = cn.forward(ps, I)
    assert out.shape == (2, 6, 6)
    x = torch.from_numpy(np.log1p(I))
    for l, (W, b) in enumerate(ps):
        x = torch.nn.functional.conv2d(x, torch.from_numpy(W), torch.from_numpy(b), stride=cn.STRIDES[l], padding=1)
        if l < 4:
            x = torch.relu(x)
    np.testing.assert_allclose(out, x[:, 0].numpy(), rtol=1e-12, atol=1e-12)


def test_net_gradient_matches_autograd():
    ps, I, t = _small_net(6)
    L, grads = cn.gradients(ps, I, t)
    tw = [(torch.from_numpy(W).requires_grad_(), torch.from_numpy(b).requires_grad_()) for W, b in ps]
    x = torch.from_numpy(np.log1p(I))
    for l, (W, b) in enumerate(tw):
        x = torch.nn.functional.conv2d(x, W, b, stride=cn.STRIDES[l], padding=1)
        if l < 4:
            x = torch.relu(x)
    Lt = ((x[:, 0] - torch.from_numpy(t)) ** 2).mean()
    Lt.backward()
    assert abs(L - Lt.item()) < 1e-12 * abs(L)
    for (dW, db), (W, b) in zip(grads, tw):
        np.testing.assert_allclose(dW, W.grad.numpy(), rtol=1e-10, atol=1e-14)
        np.testing.assert_allclose(db, b.grad.numpy(), rtol=1e-10, atol=1e-14)


def _relu_pattern(ps, I):
    _, acts = cn.forward(ps, I, return_acts=True)
    return [a > 0 for a in acts[1:]]


def test_net_gradient_finite_differences():
    """Central differences along 8 random directions over all parameters.
    A direction whose +-h steps flip any ReLU is replaced by a new one (the
    loss is then not smooth along it), so the check sees no kinks."""
    ps, I, t = _small_net(7)
    L, grads = cn.gradients(ps, I, t)
    rng = np.random.default_rng(8)
    h = 1e-6
    done = 0
    for _ in range(40):
        dirs = [(rng.standard_normal(W.shape), rng.standard_normal(b.shape)) for W, b in ps]
        plus = [(W + h * dW, b + h * db) for (W, b), (dW, db) in zip(ps, dirs)]
        minus = [(W - h * dW, b - h * db) for (W, b), (dW, db) in zip(ps, dirs)]
        if any(np.any(p != m) for p, m in zip(_relu_pattern(plus, I), _relu_pattern(minus, I))):
            continue
        fd = (cn.loss(cn.forward(plus, I), t) - cn.loss(cn.forward(minus, I), t)) / (2 * h)
        an = sum(np.sum(gW * dW) + np.sum(gb * db) for (gW, gb), (dW, db) in zip(grads, dirs))
        assert abs(fd - an) <= 1e-7 * max(abs(an), 1e-3), (fd, an)
        done += 1
        if done == 8:
            break
    assert done == 8


def test_round_bf16_matches_library_and_ties():
    rng = np.random.default_rng(9)
    x = np.concatenate([rng.standard_normal(5000) * 10.0 ** rng.integers(-6, 6, 5000),
                        [0.0, -0.0, 1.0, -2.5, 3.0e38, 1e-39]])
    ref = torch.from_numpy(x.astype(np.float32)).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(cn.round_bf16(x), ref)
    # ties go to the even significand: 1 + 2^-8 -> 1, 1 + 3*2^-8 -> 1 + 2^-6
    assert cn.round_bf16(1.0 + 2.0 ** -8) == 1.0
    assert cn.round_bf16(1.0 + 3 * 2.0 ** -8) == 1.0 + 2.0 ** -6
    assert cn.round_bf16(1.0 + 2.0 ** -8 + 2.0 ** -20) == 1.0 + 2.0 ** -7


def test_bf16_mode_matches_library_rounding():
    """bf16=True rounds the input, the weights, each hidden activation and each
    back-propagated gradient (and nothing else): the same net in PyTorch
    float64 with those values passed through torch.bfloat16 gives the same
    output and gradients."""
    ps, I, t = _small_net(10)
    rb = lambda x: x.to(torch.bfloat16).to(torch.float64)
    tw = [(torch.from_numpy(W).requires_grad_(), torch.from_numpy(b).requires_grad_()) for W, b in ps]

    class Rnd(torch.autograd.Function):          # round forward, round the incoming gradient
        @staticmethod
        def forward(ctx, x):
            return rb(x)

        @staticmethod
        def backward(ctx, g):
            return rb(g)

    x = rb(torch.log1p(torch.from_numpy(I)))
    for l, (W, b) in enumerate(tw):
        Wr = W + (rb(W) - W).detach()             # rounded value, identity gradient
        x = torch.nn.functional.conv2d(x, Wr, b, stride=cn.STRIDES[l], padding=1)
        if l < 4:
            x = Rnd.apply(torch.relu(x))
    out = x[:, 0]
    d = (out - torch.from_numpy(t))
    n = d.numel()

    class RndLoss(torch.autograd.Function):       # the output gradient 2 d / n is stored rounded
        @staticmethod
        def forward(ctx, o):
            return o

        @staticmethod
        def backward(ctx, g):
            return rb(g)

    Lt = ((RndLoss.apply(out) - torch.from_numpy(t)) ** 2).sum() / n
    Lt.backward()
    L, grads = cn.gradients(ps, I, t, bf16=True)
    np.testing.assert_allclose(cn.forward(ps, I, bf16=True), out.detach().numpy(), rtol=1e-12, atol=1e-13)
    assert abs(L - Lt.item()) < 1e-12 * abs(L)
    for (dW, db), (W, b) in zip(grads, tw):
        np.testing.assert_allclose(dW, W.grad.numpy(), rtol=1e-9, atol=1e-13)
        np.testing.assert_allclose(db, b.grad.numpy(), rtol=1e-9, atol=1e-13)
    # and bf16 rounding moves the result by about the format's precision, no more
    rel = np.linalg.norm(cn.forward(ps, I) - out.detach().numpy()) / np.linalg.norm(out.detach().numpy())
    assert 1e-5 < rel < 2e-2


def test_stitch():
    base = np.full((80, 90), -1.0)
    p = np.arange(1024, dtype=float).reshape(32, 32)
    one = cn.stitch([p], [(40.4, 50.5)], base)     # rint: 40, 50 (half to even)
    np.testing.assert_array_equal(one[24:56, 34:66], p)
    assert np.all(one[:24] == -1.0) and np.all(one[:, :34] == -1.0)
    two = cn.stitch([np.ones((32, 32)), 3 * np.ones((32, 32))], [(40, 40), (40, 48)], base)
    assert two[40, 30] == 1.0 and two[40, 60] == 3.0 and two[40, 40] == 2.0
    assert two[10, 40] == -1.0
    edge = cn.stitch([p], [(5, 85)], base)         # rows -11..20, cols 69..100: clipped
    np.testing.assert_array_equal(edge[0:21, 69:90], p[11:32, 0:21])
    assert edge[21, 70] == -1.0 and edge[5, 68] == -1.0
