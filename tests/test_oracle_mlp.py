"""Pins of the float64 surrogate MLP: GELU against the normal CDF (library),
backward against central finite differences, Adam's first step against its
closed form, and the protocol encoding on a hand-written example."""
import numpy as np
from scipy.stats import norm

from oracle import mlp


def _params(rng, scale=0.05):
    return [rng.normal(0, scale, size=s) for s in mlp.SHAPES]


def test_gelu_is_x_times_normal_cdf(rng):
    x = rng.normal(0, 3, size=200)
    np.testing.assert_allclose(mlp.gelu(x), x * norm.cdf(x), rtol=1e-12, atol=1e-14)
    h = 1e-6
    fd = (mlp.gelu(x + h) - mlp.gelu(x - h)) / (2 * h)
    np.testing.assert_allclose(mlp.gelu_grad(x), fd, rtol=1e-6, atol=1e-8)


def test_backward_matches_finite_differences(rng):
    params = _params(rng, 0.08)
    X = rng.normal(0, 1, size=(5, mlp.N_IN))
    t = rng.normal(0, 1, size=5)
    _, grads = mlp.loss_and_grads(params, X, t)
    h = 1e-6
    for i, p in enumerate(params):
        flat = p.reshape(-1)
        for idx in rng.choice(flat.size, size=min(12, flat.size), replace=False):
            old = flat[idx]
            flat[idx] = old + h
            lp = mlp.loss_and_grads(params, X, t)[0]
            flat[idx] = old - h
            lm = mlp.loss_and_grads(params, X, t)[0]
            flat[idx] = old
            fd = (lp - lm) / (2 * h)
            g = grads[i].reshape(-1)[idx]
            assert abs(fd - g) <= 1e-6 * max(1.0, abs(fd)) + 1e-9, (i, idx, fd, g)


def test_adam_first_step_closed_form(rng):
    p = [rng.normal(size=(3, 4))]
    g = [rng.normal(size=(3, 4))]
    z = [np.zeros((3, 4))]
    newp, m, v = mlp.adam_step(p, g, z, z, step=1, lr=0.01)
    np.testing.assert_allclose(newp[0], p[0] - 0.01 * g[0] / (np.abs(g[0]) + 1e-8), rtol=1e-12)
    np.testing.assert_allclose(m[0], 0.1 * g[0]) and np.testing.assert_allclose(v[0], 0.001 * g[0] ** 2)


def test_encoding_example():
    X = mlp.encode(np.array([[2.0, 1.0, 0.0]], np.float32), np.array([[0, 30, 12]]), [2])
    assert X.shape == (1, 128)
    np.testing.assert_allclose(X[0, :9], [0.4, 0.0, 1.0, 0.2, 0.5, 1.0, 0, 0, 0])
    assert np.all(X[0, 9:] == 0)


def test_training_reduces_loss(rng):
    params = _params(rng, 0.05)
    m = [np.zeros_like(p) for p in params]
    v = [np.zeros_like(p) for p in params]
    X = rng.normal(0, 1, size=(64, mlp.N_IN))
    t = np.tanh(X[:, 0] - X[:, 3])
    first = None
    for step in range(1, 31):
        loss, grads = mlp.loss_and_grads(params, X, t)
        first = first if first is not None else loss
        params, m, v = mlp.adam_step(params, grads, m, v, step, 1e-3)
    assert loss < 0.5 * first
