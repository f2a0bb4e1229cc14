"""Element-wise checks of the surrogate MLP kernels against the float64 oracle
(oracle/mlp.py), one pass at a time.

Where the kernels round: every hidden activation H_l and every backward
activation gradient dZ_l is stored as bf16; products of bf16 values are exact
in fp32 and every sum accumulates in fp32; GELU and GELU' take Phi from a
rational erf with |error| <= 1.5e-7.  Inputs and the three MFMA layers'
weights are bf16 on both sides (the oracle is given the same rounded values).

Each pass is checked from the kernels' own stored inputs of that pass, as the
simulation's single steps start from identical state: the oracle's float64
arithmetic on those inputs, against
  * an fp32 accumulation bound for every sum (acc), and
  * for every bf16 store, equality wherever no rounding boundary lies within
    the bound d of the value before rounding.  R (float64 -> float32 -> bf16,
    nearest even at each step) is monotone and leaves the kernels' float32
    values unchanged in its first step, so a kernel value v_k within d of the
    reference v is stored as R(v_k) in [R(v - d), R(v + d)]: equal to R(v)
    where those ends agree, and within R(v + d) - R(v - d) elsewhere (the
    decision is "open" there).
Perturbations pass through GELU with a factor max |GELU'| <= 1.13 and through
GELU' with max |GELU''| = 2 phi(0) <= 0.8.

(A worst-case bound carried through all three layers at once, end to end, is
vacuous for these networks: the bf16 roundings of one layer, summed with
absolute values over 512 products, exceed the next layer's values, so it
grows past the gradients themselves.)
"""
import numpy as np
import torch

from oracle import mlp as omlp

DPHI = 4e-7              # |GELU_kernel(z) - GELU(z)| <= DPHI |z| (erf error 1.5e-7 plus fp32 roundings)
DGP = 1e-6               # |GELU'_kernel(z) - GELU'(z)|, absolute
GELU1 = 1.13             # max |GELU'|
GELU2 = 0.8              # max |GELU''|
EPS32 = 2.0 ** -24       # fp32 unit roundoff


def bf16(x):
    """R: float64 -> float32 -> bf16 (nearest even), returned as float64."""
    t = torch.as_tensor(np.asarray(x, np.float64).astype(np.float32))
    return t.to(torch.bfloat16).to(torch.float32).numpy().astype(np.float64)


def acc(n):
    """Relative bound of an fp32 sum of n terms against their absolute sum:
    the MFMA adds 32 products per instruction, and every accumulator chain
    (including a split over workgroups added in order, and the column sums'
    chunked order) is at most n / 32 + 64 additions long; each rounds by at
    most EPS32, doubled for safety."""
    return (n / 32.0 + 64.0) * 2.0 * EPS32


def stored(v, d):
    """(R(v), bound of |R(v_k) - R(v)| over |v_k - v| <= d, share of elements
    whose rounding decision is open)."""
    lo, hi = bf16(v - d), bf16(v + d)
    open_ = lo != hi
    return bf16(v), np.where(open_, hi - lo, 0.0), float(open_.mean())


def _check(name, got, ref, bound):
    err = np.abs(np.asarray(got, np.float64) - ref)
    bad = err > bound
    assert not bad.any(), (name, int(bad.sum()), float(err[bad].max()), float(bound[bad].min()))


def check_passes(v, grads, params, t, loss, z3_kept):
    """Check a gradient call pass by pass.

    v: the work buffer after the call, float64 arrays X, Z1, Z2, Z3, H1, H2,
    H3, y, dy, dZa (= dZ1), dZb (= dZ2); grads: the eight gradient tensors in
    parameter order; params: the oracle's parameters with W1, W2, W3
    bf16-valued; t: the normalised targets; loss: the kernel's loss; z3_kept:
    whether Z3 is still in the buffer.  Asserts every element, and that the
    checks are tight (open decisions bounded, gradient bounds far below the
    gradients).  Returns the open shares per stored tensor."""
    W1, b1, W2, b2, W3, b3, w4, b4 = params
    a = np.abs
    B = len(t)
    shares = {}

    def check_store(name, got, val, d):
        ref, spread, shares[name] = stored(val, d)
        _check(name, got, ref, spread)

    # forward: Z_l from the stored H_{l-1}, H_l = bf16(GELU(Z_l)) from the stored Z_l
    hin = v["X"]
    for l, (W, b) in enumerate(((W1, b1), (W2, b2), (W3, b3))):
        z = hin @ W + b
        ez = acc(W.shape[0]) * (a(hin) @ a(W) + a(b))
        if l < 2 or z3_kept:
            _check("Z%d" % (l + 1), v["Z%d" % (l + 1)], z, ez)
            z, ez = v["Z%d" % (l + 1)], 0.0
        check_store("H%d" % (l + 1), v["H%d" % (l + 1)], omlp.gelu(z), DPHI * a(z) + GELU1 * ez)
        if l == 2:
            Z3, eZ3 = z, ez
        hin = v["H%d" % (l + 1)]
    X, H1, H2, H3 = v["X"], v["H1"], v["H2"], v["H3"]
    _check("y", v["y"], H3 @ w4 + b4[0], acc(512) * (a(H3) @ a(w4) + a(b4[0])))
    y, dy = v["y"], v["dy"]
    _check("dy", dy, 2.0 * (y - t) / B, 4.0 * EPS32 * (a(dy) + 2.0 * a(t) / B))
    mse = np.mean((y - t) ** 2)
    assert abs(loss - mse) <= acc(B) * mse + 1e-7, (loss, mse)
    ref, bound = [None] * 8, [None] * 8
    # dw4 = H3^T dy, db4 = sum dy
    ref[6], bound[6] = H3.T @ dy, acc(B) * (a(H3).T @ a(dy))
    ref[7], bound[7] = np.array([dy.sum()]), np.array([acc(B) * a(dy).sum()])
    # dZ3 = bf16(dy w4 GELU'(Z3)) (overwritten by dZ1 afterwards): reference and bound
    val = np.outer(dy, w4) * omlp.gelu_grad(Z3)
    d = np.outer(a(dy), a(w4)) * (DGP + GELU2 * eZ3) + 3.0 * EPS32 * a(val)
    dZ3, e3, shares["dZ3"] = stored(val, d)
    ref[4], bound[4] = H2.T @ dZ3, a(H2).T @ e3 + acc(B) * (a(H2).T @ a(dZ3))
    ref[5], bound[5] = dZ3.sum(0), e3.sum(0) + acc(B) * a(dZ3).sum(0)
    # dZ2 = bf16((dZ3 W3^T) GELU'(Z2)) from the reference dZ3 and the stored Z2
    S = dZ3 @ W3.T
    gp = omlp.gelu_grad(v["Z2"])
    d = (e3 @ a(W3).T + acc(512) * (a(dZ3) @ a(W3).T)) * a(gp) + DGP * a(S) + 2.0 * EPS32 * a(S * gp)
    check_store("dZ2", v["dZb"], S * gp, d)
    dZ2 = v["dZb"]
    ref[2], bound[2] = H1.T @ dZ2, acc(B) * (a(H1).T @ a(dZ2))
    ref[3], bound[3] = dZ2.sum(0), acc(B) * a(dZ2).sum(0)
    # dZ1 = bf16((dZ2 W2^T) GELU'(Z1)) from the stored dZ2 and Z1
    S = dZ2 @ W2.T
    gp = omlp.gelu_grad(v["Z1"])
    d = acc(512) * (a(dZ2) @ a(W2).T) * a(gp) + DGP * a(S) + 2.0 * EPS32 * a(S * gp)
    check_store("dZ1", v["dZa"], S * gp, d)
    dZ1 = v["dZa"]
    ref[0], bound[0] = X.T @ dZ1, acc(B) * (a(X).T @ a(dZ1))
    ref[1], bound[1] = dZ1.sum(0), acc(B) * a(dZ1).sum(0)
    names = ("dW1", "db1", "dW2", "db2", "dW3", "db3", "dw4", "db4")
    for name, g, r, bd in zip(names, grads, ref, bound):
        _check(name, g, r, bd)
        # tight: the worst-case fp32 bound grows with the batch (acc(16,600) is
        # 7e-5 of the absolute sum, and the weight gradients' sums cancel about
        # a hundredfold), reaching about 1 % of the largest gradient at
        # B = 16,600; it stays 20x below it
        assert bd.max() < 0.05 * np.abs(r).max(), (name, bd.max(), np.abs(r).max())
    # open decisions: rare where the value before rounding comes from a stored
    # input (GELU of a stored Z); where it is a 512-term sum with cancelling
    # signs (the data gradients dZ2 and dZ1, and H3 from a recomputed Z3) the
    # accumulation allowance is a few 1e-4 of the value, and up to about a
    # third of the bf16 roundings stay open
    summed = ("dZ2", "dZ1") if z3_kept else ("dZ2", "dZ1", "H3")
    assert max(s for k, s in shares.items() if k not in summed) < 0.01, shares
    assert max(shares[k] for k in summed) < 0.4, shares
    return shares
