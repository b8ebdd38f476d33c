"""Pins of the MLP oracle (oracle/mlp.py): finite-difference gradients, the
closed form of an Adam step, He-init moments, properties of the pilot
features on matrices with known spectra, and learning a known relation."""

import math

import numpy as np
import pytest

import synth
from oracle import mlp


def test_parameter_count():
    # 16*64+64 + 64*64+64 + 64*3+3
    assert mlp.N_PARAMS == 5443


def _data(B, seed):
    rng = np.random.default_rng(seed)
    X = rng.uniform(-4.0, 0.0, size=(B, mlp.N_IN))
    T = rng.standard_normal((B, mlp.N_OUT))
    return X, T


def test_gradient_matches_central_differences():
    theta = mlp.he_init(7)
    X, T = _data(40, 1)
    L, g = mlp.grad(theta, X, T)
    assert L == pytest.approx(mlp.loss(theta, X, T), rel=1e-15)
    rng = np.random.default_rng(2)
    idx = rng.choice(mlp.N_PARAMS, size=300, replace=False)
    # fourth-order central differences: truncation ~h^4, rounding ~u/h
    h = 1e-4
    worst = 0.0
    for i in idx:
        e = np.zeros_like(theta)
        e[i] = h
        f = lambda s: mlp.loss(theta + s * e, X, T)  # noqa: E731
        fd = (-f(2) + 8 * f(1) - 8 * f(-1) + f(-2)) / (12 * h)
        worst = max(worst, abs(fd - g[i]) / max(abs(g[i]), 1e-3 * np.abs(g).max()))
    assert worst <= 1e-7


def test_adam_first_steps_closed_form():
    theta = np.array([1.0, -2.0, 0.5])
    g = np.array([0.3, -0.01, 0.0])
    m = np.zeros(3)
    v = np.zeros(3)
    th1, m1, v1 = mlp.adam_step(theta, m, v, g, 1, lr=0.1)
    # t = 1: mhat = g, vhat = g^2, so the step is lr g / (|g| + eps)
    assert np.allclose(th1, theta - 0.1 * g / (np.abs(g) + 1e-8), rtol=0, atol=1e-15)
    assert np.allclose(m1, 0.1 * g) and np.allclose(v1, 0.001 * g * g)
    # t = 2 with the same gradient: still mhat = g, vhat = g^2
    th2, _, _ = mlp.adam_step(th1, m1, v1, g, 2, lr=0.1)
    assert np.allclose(th2, th1 - 0.1 * g / (np.abs(g) + 1e-8), rtol=1e-12, atol=1e-15)


def test_he_init_moments_and_determinism():
    theta = mlp.he_init(11)
    p = mlp.unpack(theta)
    for name, fan_in in (("W1", 16), ("W2", 64), ("W3", 64)):
        w = p[name]
        assert abs(w.mean()) < 4 * math.sqrt(2.0 / fan_in) / math.sqrt(w.size)
        assert w.var() == pytest.approx(2.0 / fan_in, rel=0.35 if w.size < 500 else 0.1)
    assert np.all(p["b1"] == 0) and np.all(p["b2"] == 0) and np.all(p["b3"] == 0)
    assert np.array_equal(theta, mlp.he_init(11))
    assert not np.array_equal(theta, mlp.he_init(12))


def test_pilot_features_properties():
    n = 300
    sigma = 10.0 ** (-np.arange(n) / 4.0)
    A = synth.general(350, n, sigma, tag=700)
    f = mlp.pilot_features(A, seed=3)
    assert f[0] == 0.0
    assert np.all(np.diff(f) <= 0)
    # power-of-two scaling leaves every rounded operand's ratios unchanged
    assert np.array_equal(f, mlp.pilot_features(8.0 * A, seed=3))
    # the sketch tracks the spectrum's slope (-1/4 decade per index) within
    # Gaussian factors: a wrong log base or squared values would fail this
    slope = np.polyfit(np.arange(12), f[:12], 1)[0]
    assert -0.3 < slope < -0.2
    assert np.all(np.abs(f[:12] - np.log10(sigma[:12])) <= 1.5)


def test_pilot_features_floor_on_rank_one():
    A, _ = synth.rank_r(200, 150, 1, tag=701)
    f = mlp.pilot_features(A, seed=4)
    # beyond rank 1 only FP32 rounding remains (~1e-7 relative)
    assert f[0] == 0.0 and np.all(f[1:] <= -6.0) and np.all(f >= mlp.FEATURE_FLOOR)


def test_training_learns_a_linear_relation():
    rng = np.random.default_rng(5)
    X = rng.uniform(-3.0, 0.0, size=(512, mlp.N_IN))
    Wt = rng.standard_normal((mlp.N_OUT, mlp.N_IN)) / 4
    T = X @ Wt.T
    theta = mlp.he_init(9)
    L0 = mlp.loss(theta, X, T)
    theta, hist = mlp.train(theta, X, T, epochs=60, batch=128, lr=3e-3)
    assert mlp.loss(theta, X, T) < 0.02 * L0


def _hand_params():
    """A sparse parameter vector set through the documented flat layout
    (W1 at 0, b1 at 1024, W2 at 1088, b2 at 5184, W3 at 5248, b3 at 5440)."""
    t = np.zeros(5443)
    w1 = lambda i, j: i * 16 + j          # noqa: E731
    w2 = lambda i, j: 1088 + i * 64 + j   # noqa: E731
    w3 = lambda i, j: 5248 + i * 64 + j   # noqa: E731
    t[w1(0, 0)], t[w1(1, 1)], t[w1(2, 0)], t[w1(2, 1)] = 1.0, -2.0, 0.5, 0.5
    t[1024 + 0], t[1024 + 1], t[1024 + 2] = 0.25, 1.0, -0.5
    t[w2(0, 0)], t[w2(0, 1)], t[w2(1, 2)], t[w2(1, 0)] = 2.0, 1.0, -1.0, 1.0
    t[5184 + 1] = 3.0
    t[w3(0, 0)], t[w3(1, 1)], t[w3(2, 0)], t[w3(2, 1)] = 1.0, 0.5, -1.0, 1.0
    t[5440:5443] = [0.1, -0.2, 0.3]
    return t


# worked by hand: sample 1 x = (1, -1, 0, ...): z1 = (1.25, 3, -0.5) -> h1 = (1.25, 3, 0);
# z2 = (2*1.25 + 3, 1.25 - 0 + 3) = (5.5, 4.25); y = (5.5 + 0.1, 0.5*4.25 - 0.2, -5.5 + 4.25 + 0.3).
# sample 2 x = (-2, 0.5, 0, ...): z1 = (-1.75, 0, -1.25) -> h1 = 0; h2 = (0, 3); y = (0.1, 1.3, 3.3)
HAND_X = np.zeros((2, 16))
HAND_X[0, :2] = [1.0, -1.0]
HAND_X[1, :2] = [-2.0, 0.5]
HAND_Y = np.array([[5.6, 1.925, -0.95], [0.1, 1.3, 3.3]])


def test_forward_hand_computed_two_samples():
    # pins the architecture independently of backprop: layer order, the
    # orientation of each weight matrix, the biases and where ReLU applies
    y, _ = mlp.forward(_hand_params(), HAND_X)
    assert np.allclose(y, HAND_Y, rtol=0, atol=1e-14)


# ---- sizing rules: standardization, decoding, labels ------------------------

def test_targets_standardize_by_hand():
    labels = [(10, 16, 1), (100, 32, 1), (1000, 64, 1)]
    T, mean, sd = mlp.targets(labels)
    # log10 k = 1, 2, 3: mean 2, population sd sqrt(2/3)
    assert mean[0] == pytest.approx(2.0) and sd[0] == pytest.approx(math.sqrt(2 / 3))
    assert np.allclose(T[:, 0], np.array([-1.0, 0.0, 1.0]) / math.sqrt(2 / 3))
    assert mean[1] == pytest.approx(112 / 3)
    # q constant: zero deviation counts as 1, targets 0
    assert sd[2] == 1.0 and np.all(T[:, 2] == 0.0)


def test_decode_by_hand():
    # raw = (2.5, 20, 1.2): k = ceil(1.05 * 316.23) = 333, p -> 32, q -> 1 (nearest)
    assert mlp.decode([0, 0, 0], [2.5, 20, 1.2], [1, 1, 1], 10**6) == (333, 32, 1)
    assert mlp.decode([0, 0, 0], [2.5, 20, 1.7], [1, 1, 1], 10**6) == (333, 32, 2)
    # on the grid, beyond the grid, negative q, capped k
    assert mlp.decode([0, 0, 0], [2.5, 200, -0.5], [1, 1, 1], 100) == (100, 256, 0)
    assert mlp.decode([0, 0, 0], [2.5, 500, -0.5], [1, 1, 1], 100) == (100, 512, 0)
    assert mlp.decode([0, 0, 0], [2.5, 600, -0.5], [1, 1, 1], 100) == (100, 512, 0)
    # de-standardization: raw = (1 + 1, 20 - 12, 1 + 6) = (2, 8, 7): p exactly on the grid
    k, p, q = mlp.decode([1, -1, 2], [1, 20, 1], [1, 12, 3], 10**6)
    assert k in (105, 106) and p == 8 and q == 4


def test_size_label_by_hand():
    # s_i = 10^(-i/9): (s_{k+p-1}/s_{k-1})^(4q+2) = 10^(-p (4q+2) / 9) <= 1e-8
    # needs p (4q+2) >= 72: q=0 p=48 (l=98), q=1 p=16 (l=66), q=2 p=8 (l=58).
    # cost (2q+2) (2 n^2 l / 60e12 + 0.44e-3 w) + 3.2e-3 w, w = (l/272)^1.6;
    # n = 10000: 1.45e-3, 1.40e-3, 1.65e-3 -> q = 1, p = 16
    s = 10.0 ** (-np.arange(400) / 9.0)
    assert mlp.size_label(s, 50, 10000) == (50, 16, 1)
    # n = 60: p = 16 reaches n (exact, l = 60, q = 0: 3.6e-4) and beats the
    # converged q = 2, p = 8 (l = 58: 4.9e-4)
    assert mlp.size_label(s, 50, 60) == (50, 16, 0)
    # a spectrum reaching only k + 10: q = 1 cannot be shown converged (its
    # last value gives 10^(-6.7)); q = 2 with p = 8 is (10^(-8.9))
    assert mlp.size_label(s[:60], 50, 10000) == (50, 8, 2)
    # coverage: the labelling run needed l >= 140 -> p >= 90 -> 96, q = 0
    # converges (96 * 2 / 9 >= 8) and is the cheapest
    assert mlp.size_label(s, 50, 10000, l_min=140) == (50, 96, 0)
    # nothing converges and nothing reaches n
    assert mlp.size_label(np.ones(100), 50, 10000) == (50, -1, -1)
