"""Pins of the FP64 learned-width oracle (oracle/mlp.py): gradients against
central finite differences, a hand-evaluated forward pass, Adam's closed form
under a constant gradient, features of a constructed spectrum, and the width
and fallback rules on their boundary cases."""
import math

import numpy as np
import pytest

from oracle import mlp


def _rand_theta(seed, scale=1.0):
    g = np.random.default_rng(seed)
    theta = mlp.init_params(g) * scale
    theta += 0.05 * g.standard_normal(theta.shape)  # nonzero biases too
    return theta


def test_param_count_and_flatten_roundtrip():
    assert mlp.N_PARAMS == 128 * 32 + 128 + 128 * 128 + 128 + 128 + 1
    theta = _rand_theta(0)
    assert np.array_equal(mlp.flatten(mlp.unflatten(theta)), theta)


def test_forward_by_hand():
    p = {k: np.zeros(mlp.SHAPES[k]) for k in mlp.ORDER}
    p["W1"][0, 0], p["b1"][0] = 2.0, -1.0
    p["W2"][0, 0], p["W3"][0, 0], p["b3"][0] = 3.0, 0.5, 0.25
    theta = mlp.flatten(p)
    X = np.zeros((3, 32))
    X[0, 0], X[1, 0], X[2, 0] = 2.0, 0.25, 0.5
    z, _ = mlp.forward(theta, X)
    # z = 0.5 * 3 * relu(2 x0 - 1) + 0.25
    assert np.allclose(z, [0.5 * 3 * 3.0 + 0.25, 0.25, 0.25], rtol=0, atol=1e-15)


@pytest.mark.parametrize("seed", [1, 2])
def test_backward_matches_central_differences(seed):
    g = np.random.default_rng(100 + seed)
    theta = _rand_theta(seed)
    X = g.standard_normal((6, 32))
    y = g.standard_normal(6)
    _, grad = mlp.backward(theta, X, y)
    # every block, random entries; ReLU kinks are avoided by the random inputs
    idx = np.concatenate([g.choice(mlp.N_PARAMS, 300, replace=False),
                          np.arange(mlp.N_PARAMS - 129, mlp.N_PARAMS)])
    h = 1e-6
    for i in idx:
        tp, tm = theta.copy(), theta.copy()
        tp[i] += h
        tm[i] -= h
        fd = (mlp.loss(tp, X, y) - mlp.loss(tm, X, y)) / (2 * h)
        assert abs(fd - grad[i]) <= 1e-6 * max(1.0, abs(fd)), f"param {i}: fd {fd} vs {grad[i]}"


def test_backward_loss_value():
    theta = _rand_theta(3)
    X = np.random.default_rng(4).standard_normal((5, 32))
    y = np.arange(5.0)
    L, _ = mlp.backward(theta, X, y)
    z, _ = mlp.forward(theta, X)
    assert L == pytest.approx(float(np.mean((z - y) ** 2)), rel=1e-15)


def test_adam_constant_gradient_moves_by_lr_sign():
    # with a constant gradient the bias-corrected moments are g and g^2, so
    # every step moves each parameter by lr * g / (|g| + eps)
    theta = np.array([1.0, -2.0, 0.5])
    grad = np.array([0.3, -4.0, 1e-3])
    m = np.zeros(3)
    v = np.zeros(3)
    lr, eps = 0.01, 1e-8
    for step in range(1, 4):
        new, m, v = mlp.adam_step(theta, m, v, grad, step, lr, eps=eps)
        assert np.allclose(new - theta, -lr * grad / (np.abs(grad) + eps), rtol=1e-12, atol=0)
        theta = new


def test_training_reduces_loss_on_a_learnable_target():
    g = np.random.default_rng(7)
    X = g.standard_normal((256, 32))
    y = 0.5 * X[:, 0] - 0.25 * X[:, 3] + 1.0
    theta = mlp.init_params(g) * 0.5
    m = np.zeros_like(theta)
    v = np.zeros_like(theta)
    l0 = mlp.loss(theta, X, y)
    for step in range(1, 301):
        _, grad = mlp.backward(theta, X, y)
        theta, m, v = mlp.adam_step(theta, m, v, grad, step, 1e-3)
    assert mlp.loss(theta, X, y) < 0.05 * l0


def test_features_of_a_constructed_spectrum():
    sigma = np.array([8.0, 4.0, 2.0, 1.0, 0, 0, 0, 0, 0, 0])
    f = mlp.features(sigma, kept_prev=3, l_prev=10, anorm2=100.0, tau=1.5, iteration=10, n1=128, n2=128)
    assert np.allclose(f[:4], [1.0, 0.5, 0.25, 0.125]) and np.all(f[4:16] == 0.0)
    assert f[16] == pytest.approx(0.2)
    assert f[17] == pytest.approx((100.0 - 85.0) / 100.0)  # ||B||^2 = 64 + 16 + 4 + 1
    assert f[18] == pytest.approx(1.5 / 8.0)
    assert f[19] == pytest.approx(0.3) and f[20] == pytest.approx(0.3)  # 8, 4, 2 above tau
    assert f[21] == pytest.approx(math.log(2.0))  # sigma_2 / sigma_3
    assert f[22] == 10.0  # sigma_4 = 1 > sigma_5 = 0
    assert f[23] == 0.0 and f[24] == 0.0  # both zero; k = 16 >= l_prev
    assert f[25] == pytest.approx(math.log10(1 / 1.5) / 10)
    assert f[26] == pytest.approx(0.1) and f[27] == 0.0 and f[28] == pytest.approx(0.7)
    assert f[29] == pytest.approx(10 / 64) and f[30] == pytest.approx(3 / 64) and f[31] == 0.0


def test_features_degenerate_slice():
    f = mlp.features(np.zeros(5), kept_prev=0, l_prev=5, anorm2=0.0, tau=0.0, iteration=500, n1=64, n2=256)
    assert np.all(f[:16] == 0.0) and f[17] == 0.0 and f[18] == 10.0 and f[25] == 1.0
    assert f[26] == 2.0 and f[27] == pytest.approx(math.log(0.25))


def test_width_rule_clamps():
    p, l_fix, k_fix = 10, 74, 64
    assert mlp.width_from_prediction(math.log(1 + 5.0), p, l_fix, k_fix) == (15, 15)
    assert mlp.width_from_prediction(math.log(1 + 5.2), p, l_fix, k_fix) == (16, 16)  # ceil
    assert mlp.width_from_prediction(-50.0, p, l_fix, k_fix) == (11, 11)  # at least p + 1
    assert mlp.width_from_prediction(math.log(1 + 59.5), p, l_fix, k_fix) == (70, 64)  # k = min(k_fix, l)
    assert mlp.width_from_prediction(50.0, p, l_fix, k_fix) == (74, 64)  # at most the fixed width
    assert mlp.width_from_prediction(1e4, p, l_fix, k_fix) == (74, 64)  # overflow to inf


def test_fallback_rule():
    sig = np.array([5.0, 3.0, 0.5, 0.1])
    # all kept survived -> redo
    assert mlp.needs_fallback(4, 3, 3, 40.0, sig, 0.2, 74, 6)
    # two of three survive; residual energy 40 - 34.26 = 5.74 over 6 - 4 = 2
    # remaining values: mean square 2.87 > tau^2 = 2.25 -> one is above tau -> redo
    assert mlp.needs_fallback(4, 3, 2, 40.0, sig, 1.5, 74, 6)
    # tau = 2: mean square 2.87 < 4, no value is certainly above tau -> keep
    assert not mlp.needs_fallback(4, 3, 2, 40.0, sig, 2.0, 74, 6)
    # at the fixed width there is nothing to redo
    assert not mlp.needs_fallback(74, 64, 64, 40.0, sig, 0.0, 74, 128)


def test_fallback_energy_test_is_certain():
    """When the energy test fires, the residual has a singular value above tau
    (checked on explicit residual spectra)."""
    g = np.random.default_rng(11)
    for _ in range(200):
        rho = np.sort(g.exponential(1.0, size=g.integers(1, 20)))[::-1]
        tau = g.uniform(0.1, 2.0)
        fires = float(np.sum(rho ** 2)) > len(rho) * tau * tau
        if fires:
            assert rho[0] > tau


def test_fallback_uses_the_zero_threshold_of_the_penalty():
    """MCP with gamma <= tau hard-thresholds at sqrt(gamma tau) < tau: values in
    (sqrt(gamma tau), tau] survive, so the certain-miss test must use that
    threshold.  Residual energy 5.74 over 2 residual values: certainly one above
    sqrt(2.5) = 1.58 but not certainly one above tau = 2."""
    sig = np.array([5.0, 3.0, 0.5, 0.1])
    assert not mlp.needs_fallback(4, 3, 2, 40.0, sig, 2.0, 74, 6, ("l1", ()))
    assert mlp.needs_fallback(4, 3, 2, 40.0, sig, 2.0, 74, 6, ("mcp", (1.25,)))
    # gamma above tau: the firm regime keeps tau as the threshold
    assert not mlp.needs_fallback(4, 3, 2, 40.0, sig, 2.0, 74, 6, ("mcp", (5.0,)))


def test_fallback_energy_test_is_certain_for_every_penalty():
    """When the energy test fires, the residual holds a value the prox keeps
    (explicit residual spectra, every penalty)."""
    from oracle import prox
    g = np.random.default_rng(12)
    pens = [("l1", ()), ("mcp", (0.5,)), ("mcp", (4.0,)), ("scad", (3.7, 0.4)), ("log", (0.5,)),
            ("capped_l1", (0.3,)), ("firm", (2.0,))]
    fired = 0
    for _ in range(300):
        kind, params = pens[g.integers(len(pens))]
        rho = np.sort(g.exponential(1.0, size=g.integers(1, 12)))[::-1]
        tau = g.uniform(0.1, 2.0)
        sig = np.array([10.0, 8.0])  # the sketched values; two kept, one survived
        an = float(np.sum(sig ** 2) + np.sum(rho ** 2))
        if mlp.needs_fallback(2, 2, 1, an, sig, tau, 74, 2 + len(rho), (kind, params)):
            fired += 1
            assert prox.prox_scalar(kind, rho[0], tau, params) > 0.0
    assert fired > 20
