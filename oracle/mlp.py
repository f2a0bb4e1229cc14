"""Float64 reference of the protocol-to-fitness surrogate MLP.

Test infrastructure: part of the CPU oracle (see oracle/__init__.py).

The surrogate maps an encoded protocol to its predicted (normalised) fitness;
it only pre-screens GA offspring, the full simulation keeps the final word.  It is
not in the paper; its shape is fixed here: input 128 features (40 fractions x
(dose / 5 Gy, delay / 60 h, present), zero-padded from 120), three hidden
layers of 512 with GELU(x) = x * Phi(x) (Phi the standard normal CDF), one
linear output.  Loss: mean squared error.  Optimiser: Adam (Kingma and Ba,
2015) with bias correction.

Parameters are held as float64 arrays in the order W1 (128x512), b1, W2
(512x512), b2, W3 (512x512), b3, w4 (512), b4 (1).
"""
import math

import numpy as np

N_IN, N_HID, N_FRAC = 128, 512, 40
DOSE_SCALE, GAP_SCALE = 5.0, 60.0
SHAPES = [(N_IN, N_HID), (N_HID,), (N_HID, N_HID), (N_HID,), (N_HID, N_HID), (N_HID,), (N_HID,), (1,)]


def encode(dose, gap, nfrac):
    """Features [B, 128]: for fraction j < 40, (dose/5, gap/60, 1) if j < nfrac else 0."""
    dose = np.asarray(dose, np.float64)
    gap = np.asarray(gap, np.float64)
    nfrac = np.asarray(nfrac).reshape(-1)
    B, K = dose.shape
    X = np.zeros((B, N_IN))
    for j in range(min(K, N_FRAC)):
        on = (j < nfrac).astype(np.float64)
        X[:, 3 * j] = dose[:, j] / DOSE_SCALE * on
        X[:, 3 * j + 1] = gap[:, j] / GAP_SCALE * on
        X[:, 3 * j + 2] = on
    return X


def gelu(x):
    return 0.5 * x * (1.0 + _erf(x / math.sqrt(2.0)))


def gelu_grad(x):
    return 0.5 * (1.0 + _erf(x / math.sqrt(2.0))) + x * np.exp(-0.5 * x * x) / math.sqrt(2.0 * math.pi)


def _erf(x):
    return np.vectorize(math.erf, otypes=[np.float64])(x)


def forward(params, X):
    """Returns (y [B], cache) with cache = (X, Z1, H1, Z2, H2, Z3, H3)."""
    W1, b1, W2, b2, W3, b3, w4, b4 = params
    Z1 = X @ W1 + b1
    H1 = gelu(Z1)
    Z2 = H1 @ W2 + b2
    H2 = gelu(Z2)
    Z3 = H2 @ W3 + b3
    H3 = gelu(Z3)
    y = H3 @ w4 + b4[0]
    return y, (X, Z1, H1, Z2, H2, Z3, H3)


def loss_and_grads(params, X, t):
    """MSE loss mean((y - t)^2) and its gradients, in parameter order."""
    W1, b1, W2, b2, W3, b3, w4, b4 = params
    y, (X, Z1, H1, Z2, H2, Z3, H3) = forward(params, X)
    B = len(t)
    loss = float(np.mean((y - t) ** 2))
    dy = 2.0 * (y - t) / B
    dw4 = H3.T @ dy
    db4 = np.array([dy.sum()])
    dZ3 = np.outer(dy, w4) * gelu_grad(Z3)
    dW3 = H2.T @ dZ3
    db3 = dZ3.sum(0)
    dZ2 = (dZ3 @ W3.T) * gelu_grad(Z2)
    dW2 = H1.T @ dZ2
    db2 = dZ2.sum(0)
    dZ1 = (dZ2 @ W2.T) * gelu_grad(Z1)
    dW1 = X.T @ dZ1
    db1 = dZ1.sum(0)
    return loss, [dW1, db1, dW2, db2, dW3, db3, dw4, db4]


def adam_step(params, grads, m, v, step, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (step counts from 1); returns new (params, m, v)."""
    out_p, out_m, out_v = [], [], []
    for p, g, mm, vv in zip(params, grads, m, v):
        mm = beta1 * mm + (1 - beta1) * g
        vv = beta2 * vv + (1 - beta2) * g * g
        mhat = mm / (1 - beta1 ** step)
        vhat = vv / (1 - beta2 ** step)
        out_p.append(p - lr * mhat / (np.sqrt(vhat) + eps))
        out_m.append(mm)
        out_v.append(vv)
    return out_p, out_m, out_v
