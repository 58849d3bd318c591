"""Pins of the corrector network's FP64 oracle (conv, backprop, Adam)."""
import numpy as np

from oracle import corrector_oracle as co


def test_parameter_count():
    assert co.NPARAMS == 19970


def test_conv_matches_direct_loops():
    rng = np.random.default_rng(0)
    x = rng.standard_normal((2, 5, 7, 3))
    w = rng.standard_normal((9, 4, 3))
    b = rng.standard_normal(4)
    assert np.max(np.abs(co.conv(x, w, b) - co.conv_direct(x, w, b))) < 1e-12


def test_conv_tap_convention_and_periodic_wrap():
    # a single unit weight on tap (dy, dx) = (0, 2), i.e. offset (-1, +1):
    # out[y, x] = in[y-1, x+1] with wrap-around
    x = np.arange(4 * 5, dtype=float).reshape(1, 4, 5, 1)
    w = np.zeros((9, 1, 1))
    w[2, 0, 0] = 1.0
    out = co.conv(x, w, np.zeros(1))[0, :, :, 0]
    for y in range(4):
        for xx in range(5):
            assert out[y, xx] == x[0, (y - 1) % 4, (xx + 1) % 5, 0]


def test_gradients_match_central_finite_differences():
    rng = np.random.default_rng(1)
    x = rng.standard_normal((2, 6, 6, 3))
    target = rng.standard_normal((2, 6, 6, 2))
    theta = co.init_params(3)
    loss, g = co.backward(x, theta, target)
    assert loss == co.mse(co.forward(x, theta)[0], target)
    idx = rng.choice(co.NPARAMS, size=60, replace=False)
    # include every bias of the last layer and some first-layer weights
    idx = np.concatenate([idx, np.arange(co.NPARAMS - 2, co.NPARAMS), np.arange(0, 5)])
    h = 1e-6
    for i in idx:
        tp, tm = theta.copy(), theta.copy()
        tp[i] += h
        tm[i] -= h
        fd = (co.mse(co.forward(x, tp)[0], target) - co.mse(co.forward(x, tm)[0], target)) / (2 * h)
        assert abs(fd - g[i]) < 1e-6 * max(1.0, abs(fd)), (i, fd, g[i])


def test_adam_first_step_is_sign_times_lr():
    # with m = v = 0 and t = 1, mhat = g and vhat = g^2, so the step is lr*g/(|g|+eps)
    g = np.array([0.3, -2.0, 1e-3])
    th, m, v = co.adam(np.zeros(3), g, np.zeros(3), np.zeros(3), 1, 0.01)
    assert np.allclose(th, -0.01 * g / (np.abs(g) + 1e-8), rtol=1e-12)
    assert np.allclose(m, 0.1 * g) and np.allclose(v, 0.001 * g * g)


def test_adam_bias_correction_after_the_first_step():
    """Closed forms of the bias-corrected moments: a constant gradient g gives
    mhat = g and vhat = g^2 at every t, so every step is -lr g/(|g| + eps);
    gradients g then -g give at t = 2 mhat = -(1-b1)/(1+b1) g and vhat = g^2."""
    lr, b1 = 0.01, 0.9
    g = np.array([0.3, -2.0, 1.5e-2])
    th, m, v = np.zeros(3), np.zeros(3), np.zeros(3)
    for t in (1, 2, 3):
        prev = th
        th, m, v = co.adam(th, g, m, v, t, lr)
        assert np.allclose(th - prev, -lr * g / (np.abs(g) + 1e-8), rtol=1e-12, atol=1e-15), t
    th, m, v = co.adam(np.zeros(3), g, np.zeros(3), np.zeros(3), 1, lr)
    th2, _, _ = co.adam(th, -g, m, v, 2, lr)
    step = lr * (1 - b1) / (1 + b1) * g / (np.abs(g) + 1e-8)
    assert np.allclose(th2 - th, step, rtol=1e-9, atol=1e-15)


def test_bf16_rounding():
    vals = np.array([1.0, 1.00390625, 1.005859375, -3.14159, 0.0, 65504.0])
    r = co.bf16_round(vals)
    assert r[0] == 1.0 and r[1] == 1.0          # halfway, ties to even
    assert r[2] == 1.0078125                    # above halfway rounds up
    assert abs(r[3] + 3.140625) < 1e-12
    assert r[4] == 0.0
