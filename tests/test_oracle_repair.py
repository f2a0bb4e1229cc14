"""Pins of the incomplete-repair form of the linear-quadratic law in the
oracle (the paper's model includes DNA damage and repair without stating a
law; the mono-exponential incomplete-repair form is the textbook one).
Checked against the protocol's total survival written as a sum over pairs of
fractions, the plain law when repair is complete, dose additivity when no
repair happens, exact values at one and two half-times, monotonicity in the
gap, and the binomial law of survivors through the simulation step."""
import copy
import math

import numpy as np

from oracle import sim
from oracle.model import DEAD, PROLIF, Params
from oracle.protocol import events, lq_survival, lq_threshold, prior_damage
from oracle.sim import pack, unpack


def _survival_from_threshold_inputs(d, m, alpha, beta, prior):
    x, y = m * d, m * prior
    return math.exp(-alpha * x - beta * x * (x + 2.0 * y))


def test_complete_repair_is_the_plain_law(params):
    dose = np.float32([2.0, 1.5, 2.5])
    gap = np.int32([0, 6, 18])
    assert params.repair_half_time == 0.0
    for j in range(3):
        assert prior_damage(dose, gap, j, 0.0) == 0.0
    ev = events(dose, gap, 3, 100, params)
    for (t, thr), d in zip(ev, dose):
        assert thr == [lq_threshold(float(d), m, params.alpha, params.beta) for m in params.m]
        assert thr[0] == min(int(math.floor(lq_survival(float(d), params.m[0], params.alpha, params.beta) * 2.0**32)),
                             2**32 - 1)


def test_total_survival_is_the_pairwise_closed_form(params):
    """prod_j S_j = exp(-alpha sum x - beta sum x^2 - 2 beta sum_{i<j} x_i x_j 2^(-(t_j - t_i)/T))."""
    rng = np.random.default_rng(4)
    a, b = params.alpha, params.beta
    for _ in range(50):
        k = int(rng.integers(1, 8))
        dose = rng.choice(np.float32([0.0, 0.5, 1.0, 2.0, 3.0]), k).astype(np.float32)
        gap = rng.integers(1, 20, k).astype(np.int32)
        T = float(rng.choice([0.5, 1.0, 2.5, 6.0]))
        m = float(rng.choice(params.m))
        logs = sum(math.log(_survival_from_threshold_inputs(float(dose[j]), m, a, b,
                                                            prior_damage(dose, gap, j, T))) for j in range(k))
        t = np.cumsum(gap)
        x = [m * float(v) for v in dose]
        total = a * sum(x) + b * sum(v * v for v in x)
        for j in range(k):
            for i in range(j):
                total += 2 * b * x[i] * x[j] * 2.0 ** (-(t[j] - t[i]) / T)
        assert math.isclose(-logs, total, rel_tol=1e-12, abs_tol=1e-15)


def test_no_repair_adds_the_doses(params):
    """With a half-time far beyond the gaps, the fractions kill like one
    fraction of their summed dose (the LQ law is additive only then)."""
    dose = np.float32([1.0, 2.0, 1.5])
    gap = np.int32([0, 1, 1])
    m = params.m[2]
    p = 1.0
    for j in range(3):
        p *= _survival_from_threshold_inputs(float(dose[j]), m, params.alpha, params.beta,
                                             prior_damage(dose, gap, j, 1e12))
    assert math.isclose(p, lq_survival(4.5, m, params.alpha, params.beta), rel_tol=1e-9)


def test_prior_damage_at_whole_half_times():
    dose = np.float32([2.0, 3.0, 1.0])
    gap = np.int32([5, 4, 8])                      # times 5, 9, 17
    assert prior_damage(dose, gap, 1, 4.0) == 1.0  # 2 Gy one half-time earlier
    assert prior_damage(dose, gap, 2, 4.0) == 2.0 * 2.0**-3 + 3.0 * 2.0**-2
    assert prior_damage(dose, gap, 2, 8.0, unit=0.5) == 2.0 * 2.0**-0.75 + 3.0 * 2.0**-0.5
    assert prior_damage(dose, gap, 0, 4.0) == 0.0


def test_survival_rises_with_the_gap(params):
    d = np.float32([2.0, 2.0])
    prev = 0.0
    for g in range(1, 30):
        s = _survival_from_threshold_inputs(2.0, 1.0, params.alpha, params.beta,
                                            prior_damage(d, np.int32([0, g]), 1, 3.0))
        assert s > prev
        prev = s
    assert prev < lq_survival(2.0, 1.0, params.alpha, params.beta)


def test_survivors_of_two_fractions_with_incomplete_repair(model_dict):
    """A full lattice of young proliferating cells takes 2 Gy at step 0 and
    3 Gy at step 1 with a 1-hour half-time: survivors ~ Binomial(N, S1 S2),
    S2 with half of the first dose unrepaired."""
    md = copy.deepcopy(model_dict)
    md["repair_half_time"] = 1.0
    prm = Params.from_dict(md)
    L = 120
    cells = pack(np.full((L, L), PROLIF), np.full((L, L), 1))
    fields = np.empty((3, L, L))
    for f in range(3):
        fields[f] = prm.init[f]
    ev = events(np.float32([2.0, 3.0]), np.int32([0, 1]), 2, 2, prm)
    m = prm.m[0]
    x1, x2 = 2.0 * m, 3.0 * m                       # pairwise form, gap = one half-time
    s = math.exp(-prm.alpha * (x1 + x2) - prm.beta * (x1 * x1 + x2 * x2) - 2 * prm.beta * x1 * x2 * 0.5)
    plain = lq_survival(2.0, m, prm.alpha, prm.beta) * lq_survival(3.0, m, prm.alpha, prm.beta)
    N = L * L
    for seed in (1, 2):
        _, out, _ = sim.run_instance(prm, L, 2, 2, ev, 0, 0, seed, state=(fields, cells))
        surv = int(np.count_nonzero(unpack(out)[0] != DEAD))
        sd = math.sqrt(N * s * (1 - s))
        assert abs(surv - N * s) < 4.5 * sd, (surv, N * s)
        assert abs(surv - N * plain) > 4.5 * sd      # the unrepaired damage is visible
