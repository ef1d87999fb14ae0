"""Pins of the FP64 network oracle (oracle/cnn.py) against references other
than itself: scipy's 2-D correlation, shifted identities, central finite
differences, Adam's closed-form first step and known binary16 values."""
import numpy as np
import pytest
from scipy.signal import correlate2d

from oracle import cnn


def rnd(shape, seed, lo=-1.0, hi=1.0):
    return np.random.Generator(np.random.PCG64(seed)).uniform(lo, hi, size=shape)


def test_f16_rounding_known_values():
    one = 1.0
    ulp = 2.0 ** -10
    assert cnn.f16(one + ulp / 2) == one                  # tie -> even
    assert cnn.f16(one + 3 * ulp / 2) == one + 2 * ulp     # tie -> even (up)
    assert cnn.f16(one + 0.51 * ulp) == one + ulp
    assert cnn.f16(65504.0) == 65504.0
    assert cnn.f16(2.0 ** -24) == 2.0 ** -24               # smallest subnormal
    assert cnn.f16(2.0 ** -26) == 0.0
    assert cnn.f16(0.1) == 0.0999755859375


def test_conv_matches_scipy_correlate():
    x = rnd((2, 7, 9, 3), 1)
    w = rnd((9, 3, 4), 2)
    b = rnd(4, 3)
    y = cnn.conv3x3(x, w, b, half=False)
    for n in range(2):
        for o in range(4):
            ref = np.full((7, 9), b[o])
            for i in range(3):
                k = w[:, i, o].reshape(3, 3)       # k[dh, dw]
                ref += correlate2d(x[n, :, :, i], k, mode="same", boundary="fill")
            np.testing.assert_allclose(y[n, :, :, o], ref, rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("tap", range(9))
def test_single_tap_identity_is_a_shift(tap):
    x = rnd((1, 6, 5, 2), 4)
    w = np.zeros((9, 2, 2))
    w[tap] = np.eye(2)
    y = cnn.conv3x3(x, w, half=False)
    dh, dw = cnn.TAPS[tap]
    ref = np.zeros_like(x)
    for h in range(6):
        for c in range(5):
            hh, cc = h + dh - 1, c + dw - 1
            if 0 <= hh < 6 and 0 <= cc < 5:
                ref[0, h, c] = x[0, hh, cc]
    np.testing.assert_array_equal(y, ref)


def test_relu_and_half_rounding_points():
    x = rnd((1, 4, 4, 2), 5)
    w = rnd((9, 2, 3), 6)
    y16 = cnn.conv3x3(x, w, relu=True, half=True)
    y = cnn.conv3x3(cnn.f16(x), cnn.f16(w), relu=True, half=False)
    np.testing.assert_array_equal(y16, y)
    assert np.all(y16 >= 0) and np.any(y16 == 0)


def tiny_net(seed=7, ch=(3, 4, 4, 3)):
    rng = np.random.Generator(np.random.PCG64(seed))
    return [{"w": rng.normal(0, 0.5, (9, ch[k], ch[k + 1])), "b": rng.normal(0, 0.2, ch[k + 1])}
            for k in range(len(ch) - 1)]


def test_backward_matches_finite_differences():
    params = tiny_net()
    x = rnd((2, 5, 6, 3), 8, 0.0, 1.0)
    t = rnd((2, 5, 6, 3), 9, 0.0, 2.0)
    acts = cnn.forward(params, x, half=False)
    L, grads = cnn.backward(params, acts, t, half=False)
    assert L == pytest.approx(cnn.loss(params, x, t, half=False), rel=1e-14)
    rng = np.random.Generator(np.random.PCG64(10))
    h = 1e-6
    for k, lay in enumerate(params):
        for name in ("w", "b"):
            arr = lay[name]
            for flat in rng.choice(arr.size, size=min(12, arr.size), replace=False):
                idx = np.unravel_index(flat, arr.shape)
                old = arr[idx]
                arr[idx] = old + h
                lp = cnn.loss(params, x, t, half=False)
                arr[idx] = old - h
                lm = cnn.loss(params, x, t, half=False)
                arr[idx] = old
                fd = (lp - lm) / (2 * h)
                an = grads[k][name][idx]
                assert abs(fd - an) <= 1e-6 * max(1.0, abs(fd)), (k, name, idx, fd, an)


def test_backward_data_is_adjoint_of_forward():
    """<conv(x), dy> = <x, conv^T(dy)> for the bias-free convolution."""
    x = rnd((2, 6, 7, 3), 11)
    w = rnd((9, 3, 5), 12)
    dy = rnd((2, 6, 7, 5), 13)
    lhs = np.sum(cnn.conv3x3(x, w, half=False) * dy)
    rhs = np.sum(x * cnn.conv3x3_backward_data(dy, w, half=False))
    assert lhs == pytest.approx(rhs, rel=1e-12)


def test_head_gradient():
    o = np.array([-3.0, 0.0, 2.5])
    t = np.array([0.1, 0.2, 0.3])
    L, d = cnn.head(o, t, 2)
    assert L == pytest.approx((3.1 ** 2 + 0.2 ** 2 + 2.2 ** 2) / 2, rel=1e-15)
    h = 1e-6
    for k in range(3):
        e = np.zeros(3)
        e[k] = h
        fd = (cnn.head(o + e, t, 2)[0] - cnn.head(o - e, t, 2)[0]) / (2 * h)
        assert d[k] == pytest.approx(fd, rel=1e-7)


def test_last_layer_adds_the_input():
    """With zero weights and biases the network is the identity map."""
    p = [{"w": np.zeros((9, c0, c1)), "b": np.zeros(c1)} for c0, c1 in [(3, 4), (4, 4), (4, 3)]]
    x = rnd((1, 4, 5, 3), 14)
    np.testing.assert_array_equal(cnn.forward(p, x, half=False)[-1], x)


def test_adam_first_step_closed_form():
    g = np.array([3.0, -0.5, 1e-3, 0.0])
    w = np.array([1.0, 2.0, 3.0, 4.0])
    w1, m, v = cnn.adam(w, np.zeros(4), np.zeros(4), g, 1, lr=0.01, eps=1e-8)
    np.testing.assert_allclose(w1, w - 0.01 * g / (np.abs(g) + 1e-8), rtol=1e-13)
    np.testing.assert_allclose(m, 0.1 * g)
    np.testing.assert_allclose(v, 0.001 * g * g)


def test_adam_minimises_a_quadratic():
    w = np.array([0.0, 10.0])
    m = v = np.zeros(2)
    for k in range(1, 3001):
        w, m, v = cnn.adam(w, m, v, 2 * (w - np.array([3.0, -1.0])), k, lr=0.05)
    np.testing.assert_allclose(w, [3.0, -1.0], atol=1e-3)


def test_warm_input_is_the_first_em_factor(oracle_mod):
    """u x is the first iterate of the unpenalised EM update from the uniform
    start (beta = 0 in Alg. 5 reduces the update to f b2 / b1), and x = 1
    wherever b1 > 0 when y is exactly the mean of a uniform image."""
    from paper_1603_06400_amd import inputs
    g = inputs.standard_geometry(8, 6, ndet=10)
    o = oracle_mod.Oracle(g)
    y = inputs.poisson_counts(o.forward(inputs.phantom(g, 3, 2)) * 50.0, 4)
    b1 = o.sensitivity()
    u = cnn.uniform_value(y, b1)
    f1, _ = o.recon_step(y, None, np.full(b1.shape, u), 0.0)
    x = cnn.warm_input(o, y)
    seen = b1 > 0
    np.testing.assert_allclose((u * x)[seen], f1[seen], rtol=1e-12)
    y_flat = o.forward(np.full(b1.shape, 2.5))
    x_flat = cnn.warm_input(o, y_flat)
    np.testing.assert_allclose(x_flat[seen], 1.0, rtol=1e-12)
    assert np.all(x_flat[~seen] == 0.0)


def test_feature_target_output_maps():
    d = 0.05
    f0 = cnn.warm_output(np.array([-50.0, 0.0, 1.0, 500.0]), 2.0, d)
    assert np.all(f0 > 0) and np.all(np.isfinite(f0))
    assert f0[0] == pytest.approx(2.0 * 0.01 * d, rel=1e-15)
    assert f0[1] == pytest.approx(2.0 * (1.0 - d), rel=1e-15)
    assert f0[3] == pytest.approx(2.0 * (np.exp(30.0) - d), rel=1e-15)
    # the output map inverts the target map above the floor
    f = np.array([0.001, 0.5, 7.0])
    np.testing.assert_allclose(cnn.warm_output(cnn.target(f, 2.0, d), 2.0, d), f, rtol=1e-12)
    assert cnn.features(np.array([0.0]), d)[0] == pytest.approx(np.log(d))


def test_mass_normalise_matches_the_em_invariant(oracle_mod):
    """One unpenalised EM step (Alg. 5, beta = 0, no background) from any
    positive image lands on sum(b1 f) = sum(y); the normalised start carries
    the same total."""
    from paper_1603_06400_amd import inputs
    g = inputs.standard_geometry(8, 6, ndet=10)
    o = oracle_mod.Oracle(g)
    y = inputs.poisson_counts(o.forward(inputs.phantom(g, 5, 2)) * 80.0, 6)
    b1 = o.sensitivity()
    f = inputs.random_image(g, 7, 0.1, 3.0)
    f1, _ = o.recon_step(y, None, f, 0.0)
    fn = cnn.mass_normalise(f, y, b1)
    assert np.sum(b1 * fn) == pytest.approx(np.sum(b1 * f1), rel=1e-12)
    assert np.sum(b1 * fn) == pytest.approx(np.sum(y), rel=1e-12)
    np.testing.assert_allclose(fn / f, fn.flat[0] / f.flat[0], rtol=1e-13)
