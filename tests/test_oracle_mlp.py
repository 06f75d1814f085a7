"""Pins of the oracle's network forward and gradient (CPU): a reduced network
whose output and gradient follow from the chain rule by hand, and central
finite differences of the loss for every parameter group."""
import math

import numpy as np

W1, B1, W2, B2, W3, B3 = 0, 160, 192, 1216, 1248, 1280


def rand_params(seed=0, scale=0.5):
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.normal(scale=scale, size=1281)


def test_reduced_network_closed_form(orc):
    """Only W1[0][2], b1[0], W2[0][0], b2[0], w3[0], b3 nonzero:
    y = w3 tanh(W2 tanh(a x_2 + b1) + b2) + b3, and the gradient of
    L = (y - t)^2 by hand."""
    p = np.zeros(1281)
    a, c1, w2, c2, w3, c3 = 0.7, -0.2, 1.3, 0.1, -0.9, 0.05
    p[W1 + 0 * 5 + 2], p[B1], p[W2], p[B2], p[W3], p[B3] = a, c1, w2, c2, w3, c3
    x = np.array([[0.3, -1.0, 0.8, 2.0, 0.5]])
    t = np.array([0.4])
    h1 = math.tanh(a * 0.8 + c1)
    h2 = math.tanh(w2 * h1 + c2)
    y = w3 * h2 + c3
    assert abs(orc.mlp_forward(p, x)[0] - y) <= 1e-15
    g, L = orc.mlp_grad(p, x, t)
    dy = 2 * (y - 0.4)
    assert abs(L - (y - 0.4) ** 2) <= 1e-15
    np.testing.assert_allclose(g[B3], dy, rtol=1e-14)
    np.testing.assert_allclose(g[W3], dy * h2, rtol=1e-14)
    dz2 = dy * w3 * (1 - h2 * h2)
    np.testing.assert_allclose(g[B2], dz2, rtol=1e-14)
    np.testing.assert_allclose(g[W2], dz2 * h1, rtol=1e-14)
    dz1 = dz2 * w2 * (1 - h1 * h1)
    np.testing.assert_allclose(g[B1], dz1, rtol=1e-14)
    np.testing.assert_allclose(g[W1 + 2], dz1 * 0.8, rtol=1e-14)
    # every other hidden unit is tanh(0) = 0 with zero outgoing weight: their
    # input weights get no gradient
    assert np.all(g[W1 + 5:B1] == 0.0)


def test_gradient_matches_finite_differences(orc):
    p = rand_params(3)
    rng = np.random.Generator(np.random.PCG64(4))
    X = rng.normal(size=(17, 5))
    T = rng.normal(size=17)
    g, L0 = orc.mlp_grad(p, X, T)

    def loss(q):
        return float(np.mean((orc.mlp_forward(q, X) - T) ** 2))

    assert abs(loss(p) - L0) <= 1e-14 * max(1.0, L0)
    idx = list(range(0, 160, 23)) + [160, 175, 192, 500, 1215, 1216, 1240, 1248, 1270, 1280]
    h = 1e-6
    for q in idx:
        e = np.zeros_like(p)
        e[q] = h
        fd = (loss(p + e) - loss(p - e)) / (2 * h)
        assert abs(fd - g[q]) <= 1e-7 * max(1.0, abs(g[q])), q


def test_adam_first_steps_closed_form(orc):
    """With m = v = 0 and a constant gradient g, bias correction makes the
    moment estimates exactly g and g^2 at every step, so each update moves a
    parameter by lr g / (|g| + eps); a zero gradient moves nothing."""
    rng = np.random.Generator(np.random.PCG64(7))
    p0 = rng.normal(size=1281)
    g = rng.normal(size=1281) * 10.0 ** rng.uniform(-6, 2, size=1281)
    g[::97] = 0.0
    p, m, v = p0.copy(), np.zeros(1281), np.zeros(1281)
    lr = 1e-3
    for step in (1, 2, 3):
        orc.mlp_adam(p, g, m, v, step, lr)
        expect = p0 - step * lr * g / (np.abs(g) + 1e-8)
        np.testing.assert_allclose(p, expect, rtol=0, atol=1e-15 * step + 1e-12 * lr)
    assert np.all(p[::97] == p0[::97])


def test_prepare_fit_standardizes(orc):
    """After fitting, every normalized input column and the target have mean 0
    and (population) standard deviation 1; a raw value equal to its column's
    scale maps to (asinh(1) - mean) / std; the target inverts to the given
    q = (gamma - 1) / dt^2."""
    rng = np.random.Generator(np.random.PCG64(8))
    B = 257
    raw = np.stack([rng.normal(scale=1e-5, size=B), rng.normal(scale=3e-6, size=B),
                    rng.uniform(1e-3, 2e-3, size=B), rng.uniform(1.0, 2.0, size=B),
                    -rng.exponential(1e-7, size=B)], axis=1)
    q = rng.normal(loc=-0.3, scale=0.05, size=B)
    gamma = 1.0 + raw[:, 2] ** 2 * q
    model0 = np.zeros(orc.MLP_MODEL)
    model, xn, tn = orc.mlp_prepare(model0, raw, gamma, fit=True)
    np.testing.assert_allclose(xn.mean(axis=0), 0.0, atol=1e-12)
    np.testing.assert_allclose(xn.std(axis=0), 1.0, rtol=1e-12)
    np.testing.assert_allclose(tn.mean(), 0.0, atol=1e-9)
    np.testing.assert_allclose(tn.std(), 1.0, rtol=1e-9)
    scale = model[1281:1286]
    np.testing.assert_allclose(scale, np.abs(raw).mean(axis=0), rtol=1e-14)
    _, x1, _ = orc.mlp_prepare(model, scale[None, :], None, fit=False)
    np.testing.assert_allclose(x1[0], (math.asinh(1.0) - model[1286:1291]) / model[1291:1296],
                               rtol=1e-14)
    # (gamma - 1)/dt^2 loses digits to the subtraction: compare at that accuracy
    np.testing.assert_allclose(tn * model[1297] + model[1296], q, atol=1e-9)
    # refitting on the same samples reproduces the model
    model2, _, _ = orc.mlp_prepare(model, raw, gamma, fit=True)
    np.testing.assert_allclose(model2, model, rtol=1e-14)
