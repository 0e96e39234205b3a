"""Pins of the corrector network's FP64 reference (oracle/cnn_oracle.py):
the convolution against an FFT circular correlation and explicit shifts, the
adjoint and weight-gradient identities, the full gradient against central
finite differences, bfloat16 rounding against torch's CPU cast and hand
cases, and Adam against its closed form."""
import numpy as np
import pytest
import torch

from oracle import cnn_oracle as C


def test_bf16_round_matches_torch_and_hand_cases():
    rng = np.random.default_rng(0)
    x = np.concatenate([rng.standard_normal(5000) * 10.0 ** rng.integers(-8, 8, 5000),
                        [0.0, -0.0, 1.0, -3.5, 1e-30, 3e38]])
    want = torch.from_numpy(x.astype(np.float32)).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(C.bf16_round(x), want)
    # ties to even at 1: ulp = 2^-7
    assert C.bf16_round(1.0 + 2.0 ** -8) == 1.0
    assert C.bf16_round(1.0 + 3 * 2.0 ** -8) == 1.0 + 2.0 ** -6
    assert C.bf16_round(1.0 + 2.0 ** -8 + 2.0 ** -20) == 1.0 + 2.0 ** -7


def _rand_layer(rng, O, Ci):
    return rng.standard_normal((O, Ci, 3, 3)), rng.standard_normal(O)


def test_conv_equals_fft_circular_correlation():
    rng = np.random.default_rng(1)
    Ci, O, H, W = 3, 4, 7, 9
    x = rng.standard_normal((Ci, H, W))
    w, b = _rand_layer(rng, O, Ci)
    got = C.conv3x3(x, w, b)
    want = np.zeros((O, H, W))
    X = np.fft.fft2(x)
    for o in range(O):
        acc = np.zeros((H, W), dtype=complex)
        for c in range(Ci):
            K = np.zeros((H, W))
            for dy in (-1, 0, 1):
                for dx in (-1, 0, 1):
                    K[(-dy) % H, (-dx) % W] += w[o, c, dy + 1, dx + 1]
            acc += X[c] * np.fft.fft2(K)
        want[o] = np.fft.ifft2(acc).real + b[o]
    assert np.max(np.abs(got - want)) < 1e-12


def test_single_tap_is_an_explicit_shift():
    rng = np.random.default_rng(2)
    x = rng.standard_normal((2, 5, 6))
    w = np.zeros((2, 2, 3, 3))
    w[0, 0, 1, 2] = 1.0   # (dy, dx) = (0, +1)
    w[1, 1, 0, 1] = 1.0   # (dy, dx) = (-1, 0)
    y = C.conv3x3(x, w, np.zeros(2))
    for yy in range(5):
        for xx in range(6):
            assert y[0, yy, xx] == x[0, yy, (xx + 1) % 6]
            assert y[1, yy, xx] == x[1, (yy - 1) % 5, xx]


def test_transpose_and_weight_gradient_identities():
    rng = np.random.default_rng(3)
    x = rng.standard_normal((3, 6, 5))
    g = rng.standard_normal((4, 6, 5))
    w, _ = _rand_layer(rng, 4, 3)
    z = np.zeros(4)
    lhs = np.sum(C.conv3x3(x, w, z) * g)
    assert abs(lhs - np.sum(x * C.conv3x3_transpose(g, w))) < 1e-10 * abs(lhs)
    dw = rng.standard_normal(w.shape)
    assert abs(np.sum(C.conv3x3_wgrad(g, x) * dw) - np.sum(C.conv3x3(x, dw, z) * g)) < 1e-10 * abs(lhs)


def test_gradient_matches_central_differences():
    rng = np.random.default_rng(4)
    N, H, W = 4, 5, 6
    p = C.init_params(N, seed=5)
    # a nonzero last layer so every weight matters
    p[2 * C.NL:] = 0.05 * rng.standard_normal(C.NL)
    p[2 * C.NL:2 * C.NL + C.NW].reshape(C.CP, C.CP, 3, 3)[N:] = 0.0
    p[2 * C.NL + C.NW + N:] = 0.0
    xs = [rng.standard_normal((N, H, W)) for _ in range(2)]
    ts = [x + 0.1 * rng.standard_normal(x.shape) for x in xs]
    loss, g = C.loss_and_grads(xs, ts, p)
    idx = np.concatenate([rng.choice(np.arange(l * C.NL, (l + 1) * C.NL), 25, replace=False) for l in range(3)])
    h = 1e-6
    for i in idx:
        pp, pm = p.copy(), p.copy()
        pp[i] += h
        pm[i] -= h
        fd = (C.loss_and_grads(xs, ts, pp)[0] - C.loss_and_grads(xs, ts, pm)[0]) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, np.abs(g).max()), (i, fd, g[i])


def test_padded_parameters_get_no_gradient_and_change_nothing():
    rng = np.random.default_rng(6)
    N = 6
    p = C.init_params(N, seed=7)
    p[2 * C.NL:2 * C.NL + C.NW] = 0.01 * rng.standard_normal(C.NW)
    p[2 * C.NL:2 * C.NL + C.NW].reshape(C.CP, C.CP, 3, 3)[N:] = 0.0
    x = rng.standard_normal((N, 4, 4))
    _, g = C.loss_and_grads([x], [x + 1.0], p)
    L = C.unpack(g)
    assert np.all(L[0][0][:, N:] == 0.0)      # layer 1 reads only N channels
    assert np.all(L[2][0][N:] == 0.0) and np.all(L[2][1][N:] == 0.0)  # layer 3 writes N channels
    out = C.forward(x, p)["out"]
    q = p.copy()
    q[2 * C.NL:2 * C.NL + C.NW].reshape(C.CP, C.CP, 3, 3)[N:] = 1.0   # unused output channels
    assert np.array_equal(C.forward(x, q)["out"], out)


def test_zero_last_layer_is_the_identity():
    rng = np.random.default_rng(8)
    x = rng.standard_normal((5, 6, 6))
    p = C.init_params(5, seed=9)
    assert np.array_equal(C.forward(x, p)["out"], x)


def test_adam_closed_forms():
    rng = np.random.default_rng(10)
    p = rng.standard_normal(50)
    g = rng.standard_normal(50)
    lr, eps = 1e-3, 1e-8
    p1, m1, v1 = C.adam(p, g, np.zeros(50), np.zeros(50), 1, lr, eps=eps)
    # first step: bias-corrected moments are g and g^2
    assert np.allclose(p1, p - lr * g / (np.abs(g) + eps), rtol=0, atol=1e-15)
    g2 = rng.standard_normal(50)
    p2, _, _ = C.adam(p1, g2, m1, v1, 2, lr, eps=eps)
    m = 0.9 * 0.1 * g + 0.1 * g2
    v = 0.999 * 0.001 * g * g + 0.001 * g2 * g2
    want = p1 - lr * (m / (1 - 0.81)) / (np.sqrt(v / (1 - 0.999 ** 2)) + eps)
    assert np.allclose(p2, want, rtol=0, atol=1e-14)


def test_scale_invariance():
    """The network works in units of the input's RMS: scaling the input scales
    the output (biases included), and the loss is unchanged."""
    rng = np.random.default_rng(11)
    N = 4
    p = C.init_params(N, seed=12)
    p[2 * C.NL:] = 0.05 * rng.standard_normal(C.NL)
    p[2 * C.NL:2 * C.NL + C.NW].reshape(C.CP, C.CP, 3, 3)[N:] = 0.0
    p[2 * C.NL + C.NW + N:] = 0.0
    x = rng.standard_normal((N, 5, 5))
    t = x + 0.1 * rng.standard_normal(x.shape)
    out1 = C.forward(x, p)["out"]
    out2 = C.forward(1e-3 * x, p)["out"]
    assert np.max(np.abs(out2 - 1e-3 * out1)) < 1e-15
    l1, g1 = C.loss_and_grads([x], [t], p)
    l2, g2 = C.loss_and_grads([1e-3 * x], [1e-3 * t], p)
    assert abs(l1 - l2) < 1e-12 * l1 and np.max(np.abs(g1 - g2)) < 1e-10 * np.max(np.abs(g1))
    assert C.rms(np.zeros((2, 3, 3))) == 1.0
