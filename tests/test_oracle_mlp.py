"""Pins for the FP64 perceptron reference (no GPU): backpropagated gradients
against central finite differences, Adam against its closed-form first step,
and the feature map against hand-checkable populations."""
import numpy as np

from oracle import mlp


def test_gradient_matches_central_differences():
    rng = np.random.default_rng(0)
    p = mlp.init_params(1) + rng.normal(0, 0.05, mlp.N_PARAMS)
    X = rng.normal(0, 1, (12, mlp.N_IN))
    T = rng.normal(0, 1, 12)
    L0, g = mlp.loss_and_grad(p, X, T)
    assert abs(L0 - mlp.loss(p, X, T)) < 1e-15
    idx = np.concatenate([rng.choice(mlp.N_PARAMS, 120, replace=False),
                          [0, 64 * 35, 64 * 35 + 64, mlp.N_PARAMS - 65, mlp.N_PARAMS - 1]])
    h = 1e-6
    for k in idx:
        e = np.zeros(mlp.N_PARAMS)
        e[k] = h
        fd = (mlp.loss(p + e, X, T) - mlp.loss(p - e, X, T)) / (2 * h)
        assert abs(fd - g[k]) <= 1e-7 + 1e-5 * abs(g[k]), (k, fd, g[k])


def test_adam_first_step_moves_each_parameter_by_lr():
    # at t = 1 the bias-corrected update is lr * g / (|g| + eps) = lr * sign(g)
    g = np.array([0.5, -2.0, 1e-3])
    p, m, v = mlp.adam_step(np.zeros(3), np.zeros(3), np.zeros(3), g, 0.01, 1)
    assert np.allclose(p, -0.01 * np.sign(g), atol=1e-7)


def test_network_output_for_zero_weights_is_the_output_bias():
    p = np.zeros(mlp.N_PARAMS)
    p[-1] = 0.7
    y, h1, h2 = mlp.forward(p, np.ones((3, mlp.N_IN)))
    assert np.allclose(y, 0.7) and np.allclose(h1, 0) and np.allclose(h2, 0)


def test_features_of_simple_populations():
    # two equally populated energies: z = -1 and +1 exactly -> bins 12 and 20
    f = mlp.features([-8, -8, 0, 0], 0.3, 16)
    assert f[12] == 0.5 and f[20] == 0.5 and f[:32].sum() == 1.0
    assert f[32] == 0.3 and f[33] == -4 / 16 and f[34] == 16 / 16
    # a single energy: sigma = 0, all mass in the central bin
    f = mlp.features([4] * 10, 0.1, 16)
    assert f[16] == 1.0 and f[34] == 0.0
