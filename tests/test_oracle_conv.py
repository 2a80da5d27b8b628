"""Pins of the reference network of the learned stage (oracle/conv.py)."""
import numpy as np
import scipy.signal

from oracle import conv


def rand(shape, seed):
    return np.random.default_rng(seed).standard_normal(shape)


def test_conv_matches_library_correlation():
    x = rand((5, 6, 7, 3), 1)
    w = rand((4, 3, 3, 3, 3), 2)
    b = rand(4, 3)
    y = conv.conv3d(x, w, b)
    for co in range(4):
        ref = np.full(x.shape[:3], b[co])
        for ci in range(3):
            ref += scipy.signal.correlate(x[..., ci], w[co, ci], mode="same", method="direct")
        assert np.allclose(y[..., co], ref, rtol=0, atol=1e-12)


def test_identity_kernel_and_bias():
    x = rand((4, 5, 6, 2), 3)
    w = np.zeros((2, 2, 3, 3, 3))
    w[0, 0, 1, 1, 1] = 1.0
    w[1, 1, 1, 1, 1] = 1.0
    b = np.array([0.5, -2.0])
    assert np.allclose(conv.conv3d(x, w, b), x + b, atol=0)
    # a pure shift: the tap at dx = 2 reads x + 1, zero past the last column
    w = np.zeros((1, 1, 3, 3, 3))
    w[0, 0, 1, 1, 2] = 1.0
    y = conv.conv3d(x[..., :1], w, np.zeros(1))
    assert np.array_equal(y[:, :, :-1, 0], x[:, :, 1:, 0]) and np.all(y[:, :, -1, 0] == 0)


def test_data_gradient_is_the_adjoint():
    x = rand((4, 5, 6, 3), 4)
    w = rand((5, 3, 3, 3, 3), 5)
    g = rand((4, 5, 6, 5), 6)
    gx, _, _ = conv.conv3d_backward(x, w, g)
    lhs = np.sum(conv.conv3d(x, w, np.zeros(5)) * g)
    assert abs(lhs - np.sum(x * gx)) <= 1e-11 * abs(lhs)


def test_network_gradients_match_central_differences():
    channels = (3, 4, 4, 2)
    params = conv.init_params(7, channels)
    for p in params:
        p["b"] = rand(p["b"].shape, 8) * 0.1
    x = rand((3, 4, 5, 3), 9)
    target = rand((3, 4, 5, 2), 10)
    _, grads = conv.mse_loss_and_grad(params, x, target)
    rng = np.random.default_rng(11)
    h = 1e-6
    for l, p in enumerate(params):
        for key in ("w", "b"):
            flat = p[key].reshape(-1)
            for idx in rng.choice(flat.size, size=min(6, flat.size), replace=False):
                old = flat[idx]
                flat[idx] = old + h
                lp, _ = conv.mse_loss_and_grad(params, x, target)
                flat[idx] = old - h
                lm, _ = conv.mse_loss_and_grad(params, x, target)
                flat[idx] = old
                fd = (lp - lm) / (2 * h)
                an = grads[l][key].reshape(-1)[idx]
                assert abs(fd - an) <= 1e-6 * max(1.0, abs(an)), (l, key, idx)


def test_adam_first_step_is_signed_learning_rate():
    params = [{"w": np.array([1.0, -2.0, 3.0]), "b": np.array([0.0])}]
    grads = [{"w": np.array([0.5, -4.0, 1e-3]), "b": np.array([2.0])}]
    state = {}
    conv.adam_step(params, grads, state, lr=0.01, eps=0.0)
    assert np.allclose(params[0]["w"], [1.0 - 0.01, -2.0 + 0.01, 3.0 - 0.01], rtol=0, atol=1e-15)
    assert np.allclose(params[0]["b"], [-0.01], rtol=0, atol=1e-15)


def test_adam_constant_gradient_steps_the_signed_learning_rate_every_time():
    """With a constant gradient g the bias-corrected moments are exactly g and
    g^2 at every step t (m_t = (1 - b1^t) g, v_t = (1 - b2^t) g^2), so each step
    moves a parameter by lr sign(g): after T steps, by T lr.  A missing or
    wrong bias correction (e.g. 1 - b instead of 1 - b^t) fails at t >= 2."""
    params = [{"w": np.array([0.5, -1.0, 2.0])}]
    g = np.array([3.0, -0.25, 1e-2])
    state = {}
    for t in range(1, 8):
        conv.adam_step(params, [{"w": g.copy()}], state, lr=0.01, eps=0.0)
        assert np.allclose(params[0]["w"], [0.5 - 0.01 * t, -1.0 + 0.01 * t, 2.0 - 0.01 * t], rtol=0, atol=1e-13), t


def test_adam_second_step_closed_form():
    """Two steps with gradients a then b.  Dividing out (1 - beta) from the
    moment recurrences gives, at t = 2, m_hat = (b1 a + b) / (1 + b1) and
    v_hat = (b2 a^2 + b^2) / (1 + b2).  For a = 1, b = -1 the second step is
    -lr (1 - b1) / (1 + b1) = -lr / 19 (v_hat = 1), and for a = 2, b = -1 it is
    lr (0.8 / 1.9) / sqrt(4.996 / 1.999)."""
    for a, b, step2 in ((1.0, -1.0, -0.01 / 19.0),
                        (2.0, -1.0, 0.01 * (0.8 / 1.9) / np.sqrt(4.996 / 1.999))):
        params = [{"w": np.array([0.0])}]
        state = {}
        conv.adam_step(params, [{"w": np.array([a])}], state, lr=0.01, eps=0.0)
        p1 = params[0]["w"][0]
        assert abs(p1 - (-0.01 * np.sign(a))) <= 1e-15
        conv.adam_step(params, [{"w": np.array([b])}], state, lr=0.01, eps=0.0)
        assert abs((p1 - params[0]["w"][0]) - step2) <= 1e-15, (a, b)


def test_bf16_rounding():
    assert conv.to_bf16(np.array([1.0]))[0] == 1.0
    # 1 + 2^-8 is exactly halfway between 1 and 1 + 2^-7: ties to even gives 1
    assert conv.to_bf16(np.array([1.0 + 2.0 ** -8]))[0] == 1.0
    assert conv.to_bf16(np.array([1.0 + 3 * 2.0 ** -8]))[0] == 1.0 + 2.0 ** -6
    a = conv.to_bf16(rand(1000, 12))
    assert np.array_equal(conv.to_bf16(a), a)
    assert np.max(np.abs(a - rand(1000, 12)) / np.abs(rand(1000, 12))) <= 2.0 ** -8
