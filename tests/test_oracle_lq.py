"""Pins of the irradiation step against the linear-quadratic closed form."""
import decimal
import math

import numpy as np

from oracle import sim
from oracle.model import DEAD, PROLIF, QUIESC
from oracle.philox import site_words
from oracle.protocol import lq_survival, lq_threshold
from oracle.sim import pack, unpack


def _exact_threshold(d, m, alpha, beta):
    """floor(exp(-a x - b x^2) * 2^32) with 50-digit decimal arithmetic."""
    decimal.getcontext().prec = 50
    D = decimal.Decimal
    x = D(float(m)) * D(float(d))
    s = (-(D(alpha) * x) - D(beta) * x * x).exp()
    return min(int((s * D(2) ** 32).to_integral_value(rounding=decimal.ROUND_FLOOR)), 2**32 - 1)


def test_threshold_is_floor_of_scaled_survival(params):
    for d in (0.25, 0.5, 1.0, 1.25, 1.5, 2.0, 2.5, 3.0, 4.5, 5.0, 10.0, 20.0):
        for m in params.m + (1.0,):
            t = lq_threshold(d, m, params.alpha, params.beta)
            assert abs(t - _exact_threshold(d, m, params.alpha, params.beta)) <= 1
    assert lq_threshold(0.0, 1.0, 0.3, 0.03) == 2**32 - 1


def _lattice(L, state, age):
    return pack(np.full((L, L), state), np.full((L, L), age))


def test_survivors_follow_lq_closed_form(params):
    """Freeze-all: N live cells, one fraction -> survivors ~ Binomial(N, S(m d))."""
    L = 300
    for state, age, cls in ((PROLIF, 2, 0), (PROLIF, 8, 1), (PROLIF, 40, 2), (QUIESC, 40, 3)):
        cells = _lattice(L, state, age)
        for d in (0.5, 2.0, 5.0):
            thr = [lq_threshold(d, params.m[c], params.alpha, params.beta) for c in range(4)]
            out = sim.irradiate(cells, thr, lambda s: site_words(s, 7, 1, 2, 11), params)
            surv = np.count_nonzero(unpack(out)[0] == state)
            S = math.exp(-params.alpha * params.m[cls] * d - params.beta * (params.m[cls] * d) ** 2)
            N = L * L
            assert abs(surv - N * S) < 5 * math.sqrt(N * S * (1 - S)), (state, d)
            killed = unpack(out)[0] == DEAD
            assert np.all(unpack(out)[1][killed] == 0)


def test_fractions_multiply_without_repopulation(params):
    """Two fractions at different steps: surviving fraction = S(d1) S(d2)."""
    L = 300
    cells = _lattice(L, PROLIF, 40)
    d1, d2 = 1.5, 2.5
    t1 = [lq_threshold(d1, params.m[c], params.alpha, params.beta) for c in range(4)]
    t2 = [lq_threshold(d2, params.m[c], params.alpha, params.beta) for c in range(4)]
    c1 = sim.irradiate(cells, t1, lambda s: site_words(s, 10, 0, 0, 5), params)
    c2 = sim.irradiate(c1, t2, lambda s: site_words(s, 34, 0, 0, 5), params)
    S = lq_survival(d1, params.m[2], params.alpha, params.beta) * lq_survival(d2, params.m[2], params.alpha, params.beta)
    surv = np.count_nonzero(unpack(c2)[0] == PROLIF)
    N = L * L
    assert abs(surv - N * S) < 5 * math.sqrt(N * S * (1 - S))


def test_pathwise_dose_monotonicity(params, rng):
    """Same words: survivors at the larger dose are a subset of those at the smaller."""
    L = 64
    cells = pack(rng.choice([PROLIF, QUIESC], size=(L, L)), rng.integers(0, 30, size=(L, L)))
    draw = lambda s: site_words(s, 3, 2, 9, 1)
    prev = None
    for d in (0.25, 0.5, 1.0, 2.0, 3.5, 5.0):
        thr = [lq_threshold(d, params.m[c], params.alpha, params.beta) for c in range(4)]
        alive = unpack(sim.irradiate(cells, thr, draw, params))[0] != DEAD
        if prev is not None:
            assert np.all(prev | ~alive)
        prev = alive


def test_class_assignment(params):
    st = np.array([[PROLIF, PROLIF, PROLIF, PROLIF, QUIESC]])
    ag = np.array([[0, 5, 6, 12, 3]])
    np.testing.assert_array_equal(sim.sensitivity_class(st, ag, params), [[0, 0, 1, 2, 3]])
