"""Pins of the network oracle (oracle/mlp.py) against facts fixed independently of its code:
central finite differences, Adam's closed form under a constant gradient, silu values and
bfloat16 rounding of values with known neighbours and ties."""
import numpy as np
import pytest

import synth
from oracle import mlp


def _small():
    dims = [3, 5, 4, 2]
    flat = synth.mlp_init(dims, tag=901).astype(np.float64)
    x = synth.mlp_batch(3, 4, tag=902).astype(np.float64)
    t = synth.mlp_batch(2, 4, tag=903).astype(np.float64) * 0.7 + 0.2
    mean, std = np.array([0.1, -0.3]), np.array([0.9, 1.7])
    return dims, flat, x, t, mean, std


def test_gradients_match_central_differences():
    dims, flat, x, t, mean, std = _small()
    params = mlp.unflatten(flat, dims)
    _, grads = mlp.loss_and_grads(params, x, t, mean, std, rounding=False)
    g = mlp.flat_grads(grads)
    h = 1e-6
    fd = np.empty_like(flat)
    for i in range(flat.size):
        e = np.zeros_like(flat)
        e[i] = h
        lp, _ = mlp.loss_and_grads(mlp.unflatten(flat + e, dims), x, t, mean, std, rounding=False)
        lm, _ = mlp.loss_and_grads(mlp.unflatten(flat - e, dims), x, t, mean, std, rounding=False)
        fd[i] = (lp - lm) / (2 * h)
    assert np.abs(g - fd).max() <= 1e-8 * max(1.0, np.abs(fd).max())
    # every parameter (weights of each layer, biases) carries gradient
    assert np.count_nonzero(np.abs(fd) > 1e-12) == flat.size


def test_rounded_gradients_are_gradients_at_the_rounded_weights():
    dims, flat, x, t, mean, std = _small()
    params = mlp.unflatten(flat, dims)
    _, g_round = mlp.loss_and_grads(params, x, t, mean, std, rounding=True)
    rounded = [(mlp.bf16_round(W), b) for W, b in params]
    _, g_exact = mlp.loss_and_grads(rounded, x, t, mean, std, rounding=False)
    assert np.array_equal(mlp.flat_grads(g_round), mlp.flat_grads(g_exact))


def test_adam_constant_gradient_closed_form():
    # with a constant gradient the bias-corrected moments are g and g^2 at every step,
    # so each update is lr * g / (|g| + eps)
    g = np.array([0.3, -2.0, 1e-3, 0.0, 5.0])
    th = np.array([1.0, 2.0, 3.0, 4.0, 5.0])
    opt = mlp.Adam(g.size)
    lr = 1e-2
    for k in range(1, 6):
        th = opt.step(th, g, lr)
        want = np.array([1.0, 2.0, 3.0, 4.0, 5.0]) - k * lr * g / (np.abs(g) + mlp.ADAM_EPS)
        assert np.allclose(th, want, rtol=0, atol=1e-12)


def test_silu_values():
    assert mlp.silu(np.array(0.0)) == 0.0
    assert mlp.silu_grad(np.array(0.0)) == 0.5
    z = np.array(40.0)
    assert abs(mlp.silu(z) - 40.0) < 1e-12 and abs(mlp.silu_grad(z) - 1.0) < 1e-12
    assert abs(mlp.silu(np.array(-40.0))) < 1e-12
    # silu(1) = 1 / (1 + e^-1)
    assert abs(mlp.silu(np.array(1.0)) - 1.0 / (1.0 + np.exp(-1.0))) < 1e-15


@pytest.mark.parametrize("x,want", [
    (1.0, 1.0),
    (1.0 + 2.0 ** -8, 1.0),                   # tie -> even mantissa (0)
    (1.0 + 3 * 2.0 ** -8, 1.0 + 2.0 ** -6),   # tie -> even mantissa (2)
    (1.0 + 2.0 ** -8 + 2.0 ** -20, 1.0 + 2.0 ** -7),  # above the tie -> up
    (-3.0, -3.0),
    (0.1, 0.10009765625),                     # 0x3DCCCCCD -> 0x3DCD
    (65504.0, 65536.0),
])
def test_bf16_rounding(x, want):
    assert mlp.bf16_round(np.array([x], np.float32))[0] == want


def test_normalisation_of_constant_column_is_floored():
    t = np.array([[1.0, 2.0], [1.0, 4.0], [1.0, 6.0]])
    mean, std = mlp.normalisation(t)
    assert mean.tolist() == [1.0, 4.0]
    assert std[0] == mlp.STD_FLOOR and abs(std[1] - np.sqrt(8.0 / 3.0)) < 1e-15


def test_relative_std_floor():
    t = np.array([[0.0, 0.0, 1.0, 0.0], [0.0, 2e-3, -1.0, 2e-4], [0.0, -2e-3, 1.0, -2e-4], [0.0, 0.0, -1.0, 0.0]])
    _, std = mlp.normalisation(t, rel_floor=1e-3)
    # floor = 1e-3 * 1: column 0 (constant) and column 3 (std 1.4e-4) are lifted to it
    assert np.allclose(std, [1e-3, np.sqrt(2e-6), 1.0, 1e-3], rtol=1e-15, atol=0)
