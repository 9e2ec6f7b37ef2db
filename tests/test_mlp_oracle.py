"""Pins of the warm-start network's reference (oracle/mlp.py) against what
the mathematics fixes: finite differences, closed-form properties of Adam,
and the bfloat16 format's definition."""
import numpy as np
import pytest

from oracle import mlp

WIDTHS = [6, 9, 7, 5, 4]


def _net(seed=3, scale=0.6):
    rng = np.random.default_rng(seed)
    w = rng.normal(0.0, scale, mlp.n_params(WIDTHS))
    X = rng.normal(0.0, 1.0, (23, WIDTHS[0]))
    T = rng.normal(0.0, 1.0, (23, WIDTHS[-1]))
    return w, X, T


def test_parameter_count_of_the_warm_start_network():
    # 6 -> 4 x 128 (tanh) -> 4
    assert mlp.n_params([6, 128, 128, 128, 128, 4]) == 50948


def test_gradient_matches_central_differences():
    w, X, T = _net()
    _, g = mlp.loss_grad(w, WIDTHS, X, T)
    h = 1e-6
    fd = np.empty_like(w)
    for i in range(w.size):
        e = np.zeros_like(w)
        e[i] = h
        fd[i] = (mlp.loss_grad(w + e, WIDTHS, X, T)[0] - mlp.loss_grad(w - e, WIDTHS, X, T)[0]) / (2 * h)
    assert np.max(np.abs(g - fd)) <= 1e-8 * max(1.0, np.max(np.abs(fd)))


def test_flat_layout_round_trip_and_order():
    w = np.arange(mlp.n_params(WIDTHS), dtype=np.float64)
    layers = mlp.unflatten(w, WIDTHS)
    # W_1 row-major first, then b_1, then W_2 ...
    assert layers[0][0][0, 1] == 1.0 and layers[0][0][1, 0] == WIDTHS[1]
    assert layers[0][1][0] == WIDTHS[0] * WIDTHS[1]
    assert layers[1][0][0, 0] == WIDTHS[0] * WIDTHS[1] + WIDTHS[1]
    np.testing.assert_array_equal(mlp.flatten(layers), w)


def test_zero_weights_output_is_the_last_bias():
    w = np.zeros(mlp.n_params(WIDTHS))
    layers = mlp.unflatten(w, WIDTHS)
    layers[-1][1][:] = [1.0, -2.0, 3.0, 0.5]
    _, y = mlp.forward(w, WIDTHS, np.ones((3, WIDTHS[0])))
    np.testing.assert_array_equal(y, np.tile([1.0, -2.0, 3.0, 0.5], (3, 1)))


def test_adam_constant_gradient_steps_are_lr_sign():
    # with a constant gradient the bias-corrected moments equal g and g^2
    # exactly in exact arithmetic, so every step moves lr g / (|g| + eps)
    g = np.array([3.0, -0.25, 1e-3, -7.0])
    w = np.zeros(4)
    m = np.zeros(4)
    v = np.zeros(4)
    lr = 1e-2
    for t in range(1, 40):
        w_new, m, v = mlp.adam(w, g, m, v, t, lr)
        step = w_new - w
        np.testing.assert_allclose(step, -lr * g / (np.abs(g) + 1e-8), rtol=1e-12, atol=0)
        w = w_new


def test_adam_first_step_ignores_gradient_scale():
    w = np.ones(3)
    for s in (1e-3, 1.0, 1e3):
        g = s * np.array([1.0, -2.0, 0.5])
        w1, _, _ = mlp.adam(w, g, np.zeros(3), np.zeros(3), 1, 0.1, eps=0.0)
        np.testing.assert_allclose(w1 - w, -0.1 * np.sign(g), rtol=1e-15)


@pytest.mark.parametrize("x, want", [
    (1.0, 1.0),
    (1.0 + 2.0 ** -8, 1.0),                  # halfway, ties to the even 1.0
    (1.0 + 3 * 2.0 ** -8, 1.0 + 2.0 ** -6),  # halfway, ties to the even 1+2^-6
    (1.0 + 2.0 ** -8 + 2.0 ** -20, 1.0 + 2.0 ** -7),  # above halfway
    (-3.0 - 2.0 ** -7, -3.0),                # spacing 2^-6 at 2..4
    (2.0 ** -130, 2.0 ** -130),              # subnormal, exactly representable
    (3.3895313892515355e38, 3.3895313892515355e38),  # the largest bf16
    (3.4028234663852886e38, np.inf),         # FP32 max rounds past it
])
def test_bf16_rounding_follows_the_format(x, want):
    got = mlp.bf16(np.float32(x)).item()
    assert got == want


def test_bf16_keeps_nan_and_is_idempotent():
    rng = np.random.default_rng(1)
    x = rng.normal(0, 10, 1000).astype(np.float32)
    r = mlp.bf16(x)
    np.testing.assert_array_equal(mlp.bf16(r), r)
    assert np.all(np.abs(r - x) <= np.abs(x) * 2.0 ** -8)
    assert np.isnan(mlp.bf16(np.float32(np.nan)))


def test_bf16_forward_stays_within_the_format_error():
    w, X, _ = _net(scale=0.3)
    _, y = mlp.forward(w, WIDTHS, X)
    yb = mlp.forward_bf16(w, WIDTHS, X)
    # each layer loses ~2^-8 relative in its operands
    assert np.max(np.abs(yb - y)) <= 0.05 * np.max(np.abs(y))
    assert np.max(np.abs(yb - y)) > 0  # the emulation really rounds


def test_training_reduces_the_loss():
    rng = np.random.default_rng(5)
    widths = [2, 16, 16, 1]
    X = rng.uniform(-1, 1, (256, 2))
    T = (np.sin(2 * X[:, :1]) * np.cos(X[:, 1:]))
    w = rng.normal(0, 0.5, mlp.n_params(widths))
    m = np.zeros_like(w)
    v = np.zeros_like(w)
    l0, _ = mlp.loss_grad(w, widths, X, T)
    for t in range(1, 400):
        _, g = mlp.loss_grad(w, widths, X, T)
        w, m, v = mlp.adam(w, g, m, v, t, 1e-2)
    l1, _ = mlp.loss_grad(w, widths, X, T)
    assert l1 < 0.05 * l0


def test_bf16_gradient_is_exact_where_bf16_is_exact():
    # one linear layer, small integers, n * w_out a power of two: every
    # rounding in the emulated arithmetic is exact, so it equals FP64
    rng = np.random.default_rng(9)
    widths = [5, 4]
    w = rng.integers(-8, 9, mlp.n_params(widths)).astype(np.float64)
    X = rng.integers(-8, 9, (32, 5)).astype(np.float64)
    _, y = mlp.forward(w, widths, X)
    T = y - rng.integers(-4, 5, y.shape)
    l, g = mlp.loss_grad(w, widths, X, T)
    lb, gb = mlp.loss_grad_bf16(w, widths, X, T)
    assert lb == l
    np.testing.assert_array_equal(gb, g)


def test_bf16_gradient_close_to_fp64():
    w, X, T = _net(scale=0.4)
    _, g = mlp.loss_grad(w, WIDTHS, X, T)
    _, gb = mlp.loss_grad_bf16(w, WIDTHS, X, T)
    assert np.max(np.abs(gb - g)) <= 0.03 * np.max(np.abs(g))
