"""Pins of the FP64 oracle of the learned propagator (oracle/conv_ref.py):
the convolution against its definition on a delta input, the backward pass
against central finite differences, and bfloat16 rounding against values
fixed by the format."""
import math

import numpy as np
import pytest

from oracle import conv_ref as cr


def test_conv_delta_response_reproduces_the_taps():
    rng = np.random.default_rng(0)
    w = rng.standard_normal((5, 3, 2))
    x = np.zeros((1, 11, 2))
    x[0, 5, 1] = 1.0
    y = cr.conv(x, w)
    # y[w] = sum_k W[k] x[w + k - 2]: the delta at 5 shows W[k] at w = 7 - k
    for k in range(5):
        np.testing.assert_array_equal(y[0, 7 - k], w[k][:, 1])
    assert np.count_nonzero(y[0, :3]) == 0 and np.count_nonzero(y[0, 8:]) == 0


@pytest.mark.parametrize("d", [2, 5])
def test_dilated_conv_delta_response(d):
    rng = np.random.default_rng(d)
    w = rng.standard_normal((5, 3, 2))
    x = np.zeros((1, 41, 2))
    x[0, 20, 0] = 1.0
    y = cr.conv(x, w, d)
    # y[p] = sum_k W[k] x[p + (k - 2) d]: the delta at 20 shows W[k] at p = 20 - (k - 2) d
    for k in range(5):
        np.testing.assert_array_equal(y[0, 20 - (k - 2) * d], w[k][:, 0])
    assert np.count_nonzero(np.abs(y[0]).sum(axis=1)) == 5


def test_conv_zero_padding_at_rod_ends():
    w = np.ones((5, 1, 1))
    x = np.ones((1, 6, 1))
    np.testing.assert_array_equal(cr.conv(x, w)[0, :, 0], [3, 4, 5, 5, 4, 3])


@pytest.mark.parametrize("d", [1, 3])
def test_input_and_weight_gradients_are_adjoint(d):
    """<conv(x, w), g> = <x, conv_input_grad(g, w)> = <w, conv_weight_grad(x, g)>."""
    rng = np.random.default_rng(1)
    x = rng.standard_normal((2, 13, 4))
    w = rng.standard_normal((5, 3, 4))
    g = rng.standard_normal((2, 13, 3))
    lhs = np.sum(cr.conv(x, w, d) * g)
    assert lhs == pytest.approx(np.sum(x * cr.conv_input_grad(g, w, d)), rel=1e-12)
    assert lhs == pytest.approx(np.sum(w * cr.conv_weight_grad(x, g, d)), rel=1e-12)


def test_gelu_values():
    """The tanh form against z Phi(z) with Phi from the error function: the
    form's known largest gap, about 4.7e-4 near |z| = 2.7 (a dropped cubic
    term gives 2e-2, a wrong scale more), odd-symmetric gaps, the limits, and
    the derivative against central differences."""
    z = np.linspace(-10.0, 10.0, 200001)
    exact = 0.5 * z * (1.0 + np.vectorize(math.erf)(z / math.sqrt(2.0)))
    gap = np.abs(cr.gelu(z) - exact)
    assert 4.6e-4 < gap.max() < 4.8e-4
    assert 2.6 < abs(z[np.argmax(gap)]) < 2.8
    # gelu(z) - gelu(-z) = z for both (Phi(z) + Phi(-z) = 1)
    np.testing.assert_allclose(cr.gelu(z) - cr.gelu(-z), z, atol=1e-14)
    assert cr.gelu(np.array([0.0]))[0] == 0.0
    np.testing.assert_allclose(cr.gelu(np.array([-40.0, 40.0])), [0.0, 40.0], atol=1e-300)
    zs = np.array([-2.0, -0.3, 0.0, 1.0, 2.7])
    eps = 1e-6
    fd = (cr.gelu(zs + eps) - cr.gelu(zs - eps)) / (2 * eps)
    np.testing.assert_allclose(cr.gelu_grad(zs), fd, rtol=1e-8, atol=1e-10)


def _small_params(seed):
    rng = np.random.default_rng(seed)
    layers = [(2, 4), (4, 4), (4, 4), (4, 4), (4, 4), (4, 1)]
    return [(rng.standard_normal((5, co, ci)) * 0.5, rng.standard_normal(co) * 0.1)
            for ci, co in layers]


def test_backward_matches_central_differences():
    rng = np.random.default_rng(2)
    params = _small_params(3)
    x = rng.standard_normal((2, 37, 2))
    t = rng.standard_normal((2, 37))
    loss, grads = cr.loss_and_grads(params, x, t)
    eps = 1e-5   # central-difference truncation ~eps^2, roundoff ~1e-16/eps
    for li in range(len(params)):
        w, b = params[li]
        for _ in range(4):
            idx = tuple(rng.integers(0, s) for s in w.shape)
            wp = w.copy(); wp[idx] += eps
            wm = w.copy(); wm[idx] -= eps
            lp = cr.loss_and_grads(params[:li] + [(wp, b)] + params[li + 1:], x, t)[0]
            lm = cr.loss_and_grads(params[:li] + [(wm, b)] + params[li + 1:], x, t)[0]
            fd = (lp - lm) / (2 * eps)
            assert grads[li][0][idx] == pytest.approx(fd, rel=1e-6, abs=1e-10), (li, idx)
        j = rng.integers(0, b.size)
        bp = b.copy(); bp[j] += eps
        bm = b.copy(); bm[j] -= eps
        fd = (cr.loss_and_grads(params[:li] + [(w, bp)] + params[li + 1:], x, t)[0] -
              cr.loss_and_grads(params[:li] + [(w, bm)] + params[li + 1:], x, t)[0]) / (2 * eps)
        assert grads[li][1][j] == pytest.approx(fd, rel=1e-6, abs=1e-10), (li, "bias")


def test_bf16_rounding_values():
    # 1 + 2^-8 is a tie between 1 and 1 + 2^-7: ties go to the even 1.0;
    # 1 + 3*2^-8 rounds up to 1 + 2^-6
    v = np.array([1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, -2.5, 3.1415926, 1e-40])
    out = cr.bf16(v)
    assert out[0] == 1.0
    assert out[1] == 1.0
    assert out[2] == 1.0 + 2 ** -6
    assert out[3] == -2.5
    assert out[4] == 3.140625
    assert out[5] == np.float64(np.float32(1e-40)).item() or abs(out[5]) < 1e-38


def test_receptive_field_is_64_points():
    """A change of the input at one point reaches the output exactly
    2 (1 + 2 + 4 + 8 + 16 + 1) = 64 points away and no farther (all weights
    nonzero, so no tap is hidden)."""
    params = [(np.ones((5, co, ci)) * 0.1, np.zeros(co)) for ci, co in cr.LAYERS]
    x = np.zeros((1, 201, 2))
    base, _ = cr.forward(params, x)
    x[0, 100, 0] = 1.0
    out, _ = cr.forward(params, x)
    reach = np.nonzero(np.abs(out - base)[0] > 0)[0]
    assert reach.min() == 100 - 64 and reach.max() == 100 + 64


def test_parameter_count():
    params = cr.init_params(0)
    n = sum(w.size + b.size for w, b in params)
    assert n == 83201


def test_features_of_a_sine_mode_in_closed_form():
    """D of sin(k pi x_i) is -4 sin^2(k pi h / 2) sin(k pi x_i), and the sum of
    sin^2(k pi x_i) over the N interior points is (N + 1) / 2, so the scaled
    feature is -sin(k pi x_i) / sqrt((N + 1) / (2 N))."""
    n, k = 127, 5
    x = np.arange(1, n + 1) / (n + 1)
    u = np.sin(k * np.pi * x)[None, :] * 3.0
    feat, s = cr.features(u, np.array([2.0]))
    np.testing.assert_allclose(feat[0, :, 0], -np.sin(k * np.pi * x) / np.sqrt((n + 1) / (2 * n)),
                               atol=1e-12)
    h = 1.0 / (n + 1)
    assert s[0] == pytest.approx(3.0 * 4 * np.sin(k * np.pi * h / 2) ** 2 *
                                 np.sqrt((n + 1) / (2 * n)), rel=1e-12)
    np.testing.assert_array_equal(feat[0, :, 1], (2.0 - 1.25) / 0.75)


def test_jump_inverts_target():
    rng = np.random.default_rng(5)
    u = rng.standard_normal((2, 16))
    u64 = u + 1e-3 * rng.standard_normal((2, 16))
    r = np.array([0.7, 1.9])
    _, s = cr.features(u, r)
    np.testing.assert_allclose(cr.jump(u, cr.target(u, u64, r, s), r, s), u64, rtol=0, atol=1e-15)


def test_bf16_forward_rounds_where_the_device_stores_bf16():
    """forward(bf=True) rounds to bfloat16 exactly where the GPU network
    keeps bfloat16 tensors -- the input features, each layer's weights, the
    stored pre-activations and activations -- while the sums, the bias, the
    GELU argument and the output stay unrounded: checked against the layer
    sequence written out step by step, and the rounding points shown to
    matter (moving one changes the result)."""
    rng = np.random.default_rng(5)
    params = [(w, 0.05 * rng.standard_normal(b.size)) for w, b in cr.init_params(5)]
    u = rng.standard_normal((2, 128)).cumsum(axis=1)
    x, _ = cr.features(u, np.array([0.7, 1.6]))
    out, cache = cr.forward(params, x, bf=True)
    h = cr.bf16(x)
    for li, (w, b) in enumerate(params):
        np.testing.assert_array_equal(cache["inputs"][li], h)
        z = cr.conv(h, cr.bf16(w), cr.DILATIONS[li]) + b
        if li == len(params) - 1:
            np.testing.assert_array_equal(out, z[:, :, 0])
            break
        np.testing.assert_array_equal(cache["pre"][li], cr.bf16(z))
        a = cr.gelu(z)
        h = cr.bf16(h + a if li > 0 else a)
    for t in cache["inputs"] + cache["pre"][:5]:
        np.testing.assert_array_equal(t, cr.bf16(t))
    # GELU of the rounded pre-activation would be another function
    h0 = cr.bf16(x)
    z0 = cr.conv(h0, cr.bf16(params[0][0]), 1) + params[0][1]
    assert not np.array_equal(cr.bf16(cr.gelu(z0)), cr.bf16(cr.gelu(cr.bf16(z0))))
    # and the rounded forward differs from the FP64 one
    out64, _ = cr.forward(params, x, bf=False)
    assert 1e-6 < np.linalg.norm(out - out64) / np.linalg.norm(out64) < 0.1
