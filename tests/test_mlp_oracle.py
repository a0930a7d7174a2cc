"""CPU pins of the surrogate-network oracle: the analytic gradient of the
loss against central finite differences (FP64), and the BF16 rounding helper
against exactly representable values and ties."""
import numpy as np

from oracle import mlp_ref


def _frozen_loss(theta0, x, y, dims):
    """The loss as a function the finite differences can see: the residual
    inside exp(-s) is frozen at theta0 (sg), and the log variances s take the
    hidden layers frozen at theta0 and only the output layer from theta."""
    F = dims[3] // 2
    n_out_w = dims[3] * dims[1]
    out0, (acts0, _, _) = mlp_ref.forward(theta0, x, dims)
    r0 = (y - out0[:, :F]) ** 2
    h0 = acts0[-1]

    def L(th):
        out, _ = mlp_ref.forward(th, x, dims)
        W = th[-(n_out_w + dims[3]):-dims[3]].reshape(dims[3], dims[1])
        b = th[-dims[3]:]
        s = (h0 @ W.T + b)[:, F:]
        res = y - out[:, :F]
        return np.sum(res * res + r0 * np.exp(-s) + s) / x.shape[0]

    return L


def test_analytic_gradient_matches_finite_differences():
    rng = np.random.default_rng(0)
    dims = (16, 12, 3, 4)
    theta = mlp_ref.init(16, 12, 3, seed=1)
    theta[-4:] = rng.normal(0, 0.1, 4)           # non-zero output bias
    x = rng.normal(0, 1, (9, 16))
    y = rng.normal(0, 1, (9, 2))
    loss, g = mlp_ref.loss_and_grad(theta, x, y, dims)
    L = _frozen_loss(theta, x, y, dims)
    idx = np.concatenate([rng.choice(theta.size - 52, 40, replace=False),
                          np.arange(theta.size - 52, theta.size)])   # all of the output layer
    h = 1e-6
    for i in idx:
        tp, tm = theta.copy(), theta.copy()
        tp[i] += h
        tm[i] -= h
        fd = (L(tp) - L(tm)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-7 * max(1.0, abs(fd)), (i, fd, g[i])
    assert abs(L(theta) - loss) < 1e-12


def test_variance_outputs_do_not_train_hidden_layers():
    """With targets equal to the predicted means (r = 0) only the variance
    term is left; its gradient must vanish outside the output layer."""
    rng = np.random.default_rng(3)
    dims = (6, 5, 2, 4)
    theta = mlp_ref.init(6, 5, 2, seed=4)
    x = rng.normal(0, 1, (4, 6))
    out, _ = mlp_ref.forward(theta, x, dims)
    _, g = mlp_ref.loss_and_grad(theta, x, out[:, :2].copy(), dims)
    n_out_params = 4 * 5 + 4
    assert np.all(g[:-n_out_params] == 0.0)
    assert np.any(g[-n_out_params:] != 0.0)


def test_gradient_with_four_targets():
    """n_out = 8: four means then four log variances."""
    rng = np.random.default_rng(1)
    dims = (8, 10, 2, 8)
    theta = mlp_ref.init(8, 10, 2, seed=2, n_out=8)
    x = rng.normal(0, 1, (7, 8))
    y = rng.normal(0, 1, (7, 4))
    loss, g = mlp_ref.loss_and_grad(theta, x, y, dims)
    L = _frozen_loss(theta, x, y, dims)
    for i in rng.choice(theta.size, 60, replace=False):
        tp, tm = theta.copy(), theta.copy()
        tp[i] += 1e-6
        tm[i] -= 1e-6
        fd = (L(tp) - L(tm)) / 2e-6
        assert abs(fd - g[i]) <= 1e-7 * max(1.0, abs(fd)), (i, fd, g[i])
    assert abs(L(theta) - loss) < 1e-12


def test_bf16_rounding():
    # BF16 keeps 7 fraction bits: steps of 2^-7 just above 1
    v = np.array([1.0 + 2 ** -7, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, 1.0 + 2 ** -9,
                  1.0 + 3 * 2 ** -9, -2.5, 3e38, 0.0])
    out = mlp_ref.bf16(v)
    assert out[0] == 1.0 + 2 ** -7            # representable
    assert out[1] == 1.0                      # tie -> even fraction (0)
    assert out[2] == 1.0 + 2 ** -6            # tie -> even fraction (2)
    assert out[3] == 1.0                      # below half a step
    assert out[4] == 1.0 + 2 ** -7            # above half a step
    assert out[5] == -2.5 and out[7] == 0.0
    assert np.isfinite(out[6])


# GELU(z) = z Phi(z) with the standard normal CDF Phi, and its derivative
# Phi(z) + z phi(z): Phi(1) = 0.8413447460685429, phi(1) = 0.24197072451914337
# (textbook values of the normal distribution).
GELU_POINTS = [(1.0, 0.8413447460685429, 0.8413447460685429 + 0.24197072451914337),
               (-1.0, -0.15865525393145707, 0.15865525393145707 - 0.24197072451914337),
               (0.0, 0.0, 0.5),
               (2.0, 2.0 * 0.9772498680518208, 0.9772498680518208 + 2.0 * 0.05399096651318806)]


def _gelu_pins(gelu, gelu_d):
    for z, g, d in GELU_POINTS:
        assert abs(float(gelu(np.float64(z))) - g) <= 1e-15 * max(1.0, abs(g)), (z, gelu(z), g)
        assert abs(float(gelu_d(np.float64(z))) - d) <= 1e-15 * max(1.0, abs(d)), (z, gelu_d(z), d)


def test_gelu_at_literal_points():
    """The erf-form GELU and its derivative at points where the normal CDF
    and density are known."""
    _gelu_pins(mlp_ref.gelu, mlp_ref.gelu_d)


def test_tanh_form_gelu_fails_the_pins():
    """A planted mistake: the tanh approximation of GELU (off by 1.5e-4 at
    z = 1) must fail the literal pins."""
    import math

    import pytest

    def tanh_gelu(z):
        return 0.5 * z * (1 + np.tanh(math.sqrt(2 / math.pi) * (z + 0.044715 * z ** 3)))

    with pytest.raises(AssertionError):
        _gelu_pins(tanh_gelu, mlp_ref.gelu_d)
