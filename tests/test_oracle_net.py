"""Pins of the FP64 reference network (oracle/net.py), CPU only.

* The 3x3 convolution equals scipy's 2-D cross-correlation summed over input
  channels (a library routine with the same definition).
* Pooling and upsampling on hand-checked arrays.
* Every gradient of the full encoder-decoder equals a central finite difference of the
  loss (h = 1e-6, FP64: agreement to 1e-6 relative is far above the truncation and
  rounding errors of the difference quotient).
"""
import numpy as np
import pytest
from scipy.signal import correlate2d

from oracle import net


def test_conv_matches_cross_correlation():
    rng = np.random.default_rng(0)
    x = rng.normal(size=(3, 7, 9))
    w = rng.normal(size=(4, 3, 3, 3))
    b = rng.normal(size=4)
    y = net.conv3x3(x, w, b)
    for co in range(4):
        want = sum(correlate2d(x[ci], w[co, ci], mode="same") for ci in range(3)) + b[co]
        np.testing.assert_allclose(y[co], want, atol=1e-12)


def test_pool_and_upsample():
    x = np.arange(16.0).reshape(1, 4, 4)
    np.testing.assert_array_equal(net.avgpool2(x)[0], [[2.5, 4.5], [10.5, 12.5]])
    u = net.upsample2(np.array([[[1.0, 2.0], [3.0, 4.0]]]))
    np.testing.assert_array_equal(u[0], [[1, 1, 2, 2], [1, 1, 2, 2], [3, 3, 4, 4], [3, 3, 4, 4]])
    np.testing.assert_array_equal(net.upsample2_backward(np.ones((1, 4, 4)))[0], 4 * np.ones((2, 2)))
    np.testing.assert_array_equal(net.avgpool2_backward(np.ones((1, 2, 2)))[0], 0.25 * np.ones((4, 4)))


def test_gradients_match_finite_differences():
    rng = np.random.default_rng(1)
    cin, cout, widths, H = 3, 2, (2, 3, 4, 5), 8
    params = net.init_params(cin, cout, widths, seed=2)
    params = [(w, rng.normal(scale=0.1, size=b.shape)) for w, b in params]
    xs = rng.normal(size=(2, cin, H, H))
    ts = rng.normal(size=(2, cout, H, H))
    loss, grads = net.loss_and_grads(params, xs, ts)
    h = 1e-6
    checked = 0
    for k in range(len(params)):
        w, b = params[k]
        for which, arr in ((0, w), (1, b)):
            flat = arr.reshape(-1)
            for idx in rng.choice(flat.size, size=min(3, flat.size), replace=False):
                old = flat[idx]
                flat[idx] = old + h
                lp, _ = net.loss_and_grads(params, xs, ts)
                flat[idx] = old - h
                lm, _ = net.loss_and_grads(params, xs, ts)
                flat[idx] = old
                fd = (lp - lm) / (2 * h)
                g = grads[k][which].reshape(-1)[idx]
                assert g == pytest.approx(fd, rel=1e-6, abs=1e-9), (k, which, idx)
                checked += 1
    assert checked >= 60


def test_bf16_round_matches_torch():
    """The BF16 rounding of the reference's quantized mode is round-to-nearest-even, as
    torch's float -> bfloat16 conversion (a library routine) defines it: random values
    over many magnitudes and both signs, and exact ties."""
    import torch
    rng = np.random.default_rng(7)
    x = rng.normal(size=4000) * 10.0 ** rng.integers(-30, 30, 4000)
    ties = np.array([1 + 2.0 ** -8, 1 + 3 * 2.0 ** -8, -(1 + 2.0 ** -8), 3 * 2.0 ** -9 + 2.0 ** -1,
                     255.5, 256.5, 257.0, 2.0 ** -126 * (1 + 2.0 ** -8)])
    for v in (x, ties):
        want = torch.from_numpy(v.astype(np.float32)).to(torch.bfloat16).to(torch.float64).numpy()
        np.testing.assert_array_equal(net.bf16_round(v), want)


def test_quantized_network_stays_within_bf16_error():
    """quant=True rounds operands to BF16 (8 significant bits, 2^-9 relative) at every
    storage point: outputs and gradients move from the exact network's (pinned by finite
    differences above) by more than round-off, but by a few units of 2^-8 of each tensor's
    largest element at most (gradients up to about ten: a ReLU whose input lies within the
    rounding of zero passes or stops a whole gradient element)."""
    rng = np.random.default_rng(3)
    cin, cout, widths, H = 4, 3, (8, 16, 16, 32), 32
    params = net.init_params(cin, cout, widths, seed=4)
    params = [(w, rng.normal(scale=0.05, size=b.shape)) for w, b in params]
    xs = rng.normal(size=(2, cin, H, H))
    ts = rng.normal(scale=0.5, size=(2, cout, H, H))
    y0, yq = net.forward(params, xs[0]), net.forward(params, xs[0], quant=True)
    assert 1e-6 * np.abs(y0).max() < np.abs(yq - y0).max() <= 8 * 2.0 ** -8 * np.abs(y0).max()
    l0, g0 = net.loss_and_grads(params, xs, ts)
    lq, gq = net.loss_and_grads(params, xs, ts, quant=True)
    assert lq == pytest.approx(l0, rel=1e-2)
    for (w0, b0), (wq, bq) in zip(g0, gq):
        for a, b in ((wq, w0), (bq, b0)):
            assert np.abs(a - b).max() <= 16 * 2.0 ** -8 * np.abs(b).max()
