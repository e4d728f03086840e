"""Pins of the network oracle (oracle/net.py) against facts fixed outside it:
a library cross-correlation, the adjoint identity, central finite
differences, positive homogeneity of a bias-free ReLU network, torch's own
BF16 rounding, and the features against scipy's sparse product."""
import numpy as np
import pytest
import scipy.signal
import torch

import oracle
from oracle import net as ON
from paper_1410_4054_amd import problems as P


def _weights(layers, seed, scale=1.0):
    return P.net_init(layers, seed).astype(np.float64) * scale


def test_conv_matches_scipy_correlate():
    rng = np.random.default_rng(1)
    x = rng.standard_normal((3, 7, 9))
    W = rng.standard_normal((5, 3, 3, 3))  # the convolution itself, any channel counts
    out = ON.conv(x, W)
    for co in range(5):
        ref = sum(scipy.signal.correlate2d(x[ci], W[co, ci], mode="same", boundary="fill")
                  for ci in range(3))
        np.testing.assert_allclose(out[co], ref, rtol=1e-13, atol=1e-13)


def test_conv_adjoint_identity():
    rng = np.random.default_rng(2)
    x = rng.standard_normal((4, 6, 5))
    g = rng.standard_normal((3, 6, 5))
    W = rng.standard_normal((3, 4, 3, 3))
    lhs = np.sum(ON.conv(x, W) * g)
    rhs = np.sum(x * ON.conv_adjoint(g, W))
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)
    # weight gradient: <conv(x, W), g> is linear in W
    dw = ON.conv_weight_grad(g, x)
    assert abs(np.sum(dw * W) - lhs) <= 1e-12 * abs(lhs)


@pytest.mark.parametrize("linear", [False, True], ids=["relu", "linear"])
def test_gradient_finite_differences(linear):
    """FP64 analytic gradient of the loss against central differences."""
    layers, nx, ny = 3, 6, 5
    rng = np.random.default_rng(3)
    planes = rng.standard_normal((1, ny, nx))
    target = rng.standard_normal((ny, nx))
    w = _weights(layers, 4)
    loss, grad = ON.loss_and_gradient(w, planes, target, layers, bf=False, linear=linear)
    h = 1e-5
    idx = rng.choice(w.size, 40, replace=False)
    for i in idx:
        wp, wm = w.copy(), w.copy()
        wp[i] += h
        wm[i] -= h
        lp, _ = ON.loss_and_gradient(wp, planes, target, layers, bf=False, linear=linear)
        lm, _ = ON.loss_and_gradient(wm, planes, target, layers, bf=False, linear=linear)
        fd = (lp - lm) / (2 * h)
        assert abs(fd - grad[i]) <= 1e-8 * max(1.0, abs(grad).max()), (i, fd, grad[i])


def test_positive_homogeneity():
    layers = 4
    rng = np.random.default_rng(5)
    planes = rng.standard_normal((1, 8, 8))
    w = _weights(layers, 6)
    y1, _ = ON.forward(w, planes, layers, bf=False)
    y2, _ = ON.forward(w, 3.7 * planes, layers, bf=False)
    np.testing.assert_allclose(y2, 3.7 * y1, rtol=1e-12, atol=1e-14)
    # powers of two commute with BF16 rounding: exact with rounding on
    y3, _ = ON.forward(w, planes, layers, bf=True)
    y4, _ = ON.forward(w, 0.25 * planes, layers, bf=True)
    np.testing.assert_array_equal(y4, 0.25 * y3)


def test_linear_network_is_linear():
    """With the identity between layers N is linear: additive and odd, and
    equal to the single convolution with the composed filter."""
    layers = 3
    rng = np.random.default_rng(13)
    w = _weights(layers, 14)
    p1, p2 = rng.standard_normal((2, 1, 9, 7))
    f = lambda p: ON.forward(w, p, layers, bf=False, linear=True)[0]
    np.testing.assert_allclose(f(p1 + p2), f(p1) + f(p2), rtol=1e-11, atol=1e-12)
    np.testing.assert_allclose(f(-p1), -f(p1), rtol=1e-12, atol=1e-13)
    # the response to a unit impulse is the composed 7x7 filter; convolving
    # with it (away from the boundary) reproduces N
    imp = np.zeros((1, 21, 21))
    imp[0, 10, 10] = 1.0
    h = f(imp)[7:14, 7:14]  # support of three stacked 3x3 filters
    big = rng.standard_normal((1, 30, 30))
    ref = scipy.signal.convolve2d(big[0], h, mode="same")
    np.testing.assert_allclose(f(big)[5:-5, 5:-5], ref[5:-5, 5:-5], rtol=1e-10, atol=1e-10)


def test_bf16_rounding_matches_torch():
    rng = np.random.default_rng(7)
    x = np.concatenate([rng.standard_normal(10000) * 10.0 ** rng.uniform(-20, 20, 10000),
                        [1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, -1.0 - 2 ** -8, 0.0, 65504.0]])
    ref = torch.tensor(x.astype(np.float32)).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(ON.bf16(x), ref)


def test_features_match_scipy():
    A = P.heat2d(9)
    rng = np.random.default_rng(8)
    um, um1, b, un = (rng.standard_normal(81) for _ in range(4))
    plane, g, target, s = ON.features(A, 9, 9, b, um, um1, unext=un, normalize=True, bf=False)
    r = b - A.to_scipy() @ (2 * um - um1)
    assert s == np.max(np.abs(r))
    np.testing.assert_allclose(plane[0].ravel(), r / s, rtol=1e-13, atol=1e-15)
    np.testing.assert_allclose(target.ravel(), (un - g) / s, rtol=1e-7)
    assert np.array_equal(g, 2 * um - um1)
    # the CSR product used is the oracle's (rows left to right)
    assert np.array_equal(plane[0].ravel(), (b - oracle.spmv(A, g)) / s)


def test_passes_follow_the_definition():
    """Two passes: the second corrects the first with N of its residual;
    with an exact inverse in place of N one pass would solve the system, so
    a pass is x + N(b - A x) and nothing else."""
    layers = 3
    w = _weights(layers, 11)
    A = P.heat2d(7)
    rng = np.random.default_rng(12)
    b, um, um1 = (rng.standard_normal(49) for _ in range(3))
    x1 = ON.guess(w, A, 7, 7, b, um, um1, layers, passes=1, bf=False)
    x2 = ON.guess(w, A, 7, 7, b, um, um1, layers, passes=2, bf=False)
    r1 = (b - A.to_scipy() @ x1).reshape(1, 7, 7)
    y, _ = ON.forward(w, r1, layers, bf=False)
    np.testing.assert_allclose(x2, x1 + y.ravel(), rtol=1e-12, atol=1e-14)


def test_zero_last_layer_gives_extrapolation():
    """With the last layer zero, N = 0 and x0 = 2 u_m - u_{m-1} exactly."""
    layers = 3
    w = _weights(layers, 9)
    w[-16 * 9:] = 0.0
    A = P.heat2d(6)
    rng = np.random.default_rng(10)
    b, um, um1 = (rng.standard_normal(36) for _ in range(3))
    np.testing.assert_array_equal(ON.guess(w, A, 6, 6, b, um, um1, layers), 2 * um - um1)


@pytest.mark.parametrize("layers", [2, 4])
def test_num_weights(layers):
    assert ON.num_weights(layers) == P.net_init(layers, 0).size == \
        16 * 9 + (layers - 2) * 16 * 16 * 9 + 16 * 9
