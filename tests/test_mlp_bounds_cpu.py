"""The pass-by-pass MLP checker (mlp_bounds.check_passes) on the CPU: it
accepts a float32 emulation of the kernels' arithmetic (bf16 stores at the
same points, GELU from the same rational erf, Abramowitz & Stegun 7.1.26) and
rejects planted mistakes in one block of a gradient or one stored element."""
import numpy as np
import pytest
import torch

from oracle import mlp as omlp
import mlp_bounds as mb

f32 = np.float32


def _bf(x):
    return torch.as_tensor(np.asarray(x, f32)).to(torch.bfloat16).to(torch.float32).numpy()


def _phi(x):
    a = np.abs(x) * f32(0.70710678118654752)
    t = f32(1) / (f32(0.3275911) * a + f32(1))
    p = t * (t * (t * (t * (t * f32(1.061405429) - f32(1.453152027)) + f32(1.421413741)) - f32(0.284496736)) +
             f32(0.254829592))
    e = np.exp(-(x * x) / f32(2)).astype(f32)
    return (f32(0.5) + np.copysign(f32(0.5) * (f32(1) - p * e), x)).astype(f32), e


def _gelu(x):
    return (x * _phi(x.astype(f32))[0]).astype(f32)


def _gelu_grad(x):
    p, e = _phi(x.astype(f32))
    return (x * f32(0.39894228040143268) * e + p).astype(f32)


def _mm(a, b):
    return (torch.from_numpy(np.ascontiguousarray(a, f32)) @ torch.from_numpy(np.ascontiguousarray(b, f32))).numpy()


def _emulate(B, seed):
    rng = np.random.default_rng(seed)
    params = []
    for s in omlp.SHAPES:
        params.append(rng.uniform(-1, 1, size=s) / np.sqrt(s[0] if len(s) == 2 else 512))
    for i in (0, 2, 4):
        params[i] = _bf(params[i]).astype(np.float64)
    dose = rng.choice([0.5, 1.0, 1.5, 2.0, 2.5], size=(B, 10))
    gap = rng.choice(np.arange(6, 61, 6), size=(B, 10))
    X = _bf(omlp.encode(dose, gap, rng.integers(1, 11, B)))
    t = rng.normal(size=B)
    W1, b1, W2, b2, W3, b3, w4, b4 = [p.astype(f32) for p in params]
    Z1 = _mm(X, W1) + b1
    H1 = _bf(_gelu(Z1))
    Z2 = _mm(H1, W2) + b2
    H2 = _bf(_gelu(Z2))
    Z3 = _mm(H2, W3) + b3
    H3 = _bf(_gelu(Z3))
    y = _mm(H3, w4[:, None])[:, 0] + b4[0]
    dy = (f32(2) * (y - t.astype(f32)) / f32(B)).astype(f32)
    dZ3 = _bf(dy[:, None] * w4[None, :] * _gelu_grad(Z3))
    dZ2 = _bf(_mm(dZ3, W3.T) * _gelu_grad(Z2))
    dZ1 = _bf(_mm(dZ2, W2.T) * _gelu_grad(Z1))
    grads = [_mm(X.T, dZ1), dZ1.sum(0), _mm(H1.T, dZ2), dZ2.sum(0), _mm(H2.T, dZ3), dZ3.sum(0),
             _mm(H3.T, dy[:, None])[:, 0], np.array([dy.sum()])]
    v = dict(X=X, Z1=Z1, Z2=Z2, Z3=Z3, H1=H1, H2=H2, H3=H3, y=y, dy=dy, dZa=dZ1, dZb=dZ2)
    v = {k: np.asarray(x, np.float64) for k, x in v.items()}
    loss = float(np.mean((y - t.astype(f32)) ** 2))
    return v, [np.asarray(g, np.float64) for g in grads], params, t, loss


@pytest.fixture(scope="module")
def case():
    return _emulate(192, 3)


@pytest.mark.parametrize("z3_kept", [True, False])
def test_checker_accepts_the_kernels_arithmetic(case, z3_kept):
    v, grads, params, t, loss = case
    shares = mb.check_passes(v, grads, params, t, loss, z3_kept)
    assert shares["H1"] < 0.01 and shares["dZ1"] > 0.0


@pytest.mark.parametrize("which,rows,cols,factor", [(0, slice(3, 19), slice(8, 24), 1.01),   # dW1 block
                                                    (4, slice(100, 116), slice(0, 16), 0.99),  # dW3 block
                                                    (5, slice(40, 56), None, 1.02)])           # db3 entries
def test_checker_rejects_a_wrong_gradient_block(case, which, rows, cols, factor):
    v, grads, params, t, loss = case
    bad = [g.copy() for g in grads]
    if cols is None:
        bad[which][rows] *= factor
    else:
        bad[which][rows, cols] *= factor
    with pytest.raises(AssertionError):
        mb.check_passes(v, bad, params, t, loss, True)


def test_checker_rejects_a_wrong_stored_activation(case):
    v, grads, params, t, loss = case
    bad = dict(v)
    H2 = v["H2"].copy()
    i = np.argmax(np.abs(H2))
    H2.flat[i] = _bf(H2.flat[i] * 1.05)[()]          # one element, a few bf16 steps off
    bad["H2"] = H2
    with pytest.raises(AssertionError):
        mb.check_passes(bad, grads, params, t, loss, True)
