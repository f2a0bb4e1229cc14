"""Pins of the oracle's 30-minute fraction timing (protocols timed in
half-hours: a fraction at an odd half-hour falls in the middle of its step,
after half of the hour's diffusion sub-steps).  Checked against what must
hold whatever the arithmetic: even half-hour times reproduce the hourly
protocol exactly; the comparison principle orders the fields by when a lethal
fraction strikes; two fractions in one hour kill independently, so the
survivors follow the binomial law of the product of the two surviving
fractions; the event list keeps the half-hour times and the horizon."""
import numpy as np

from oracle import sim
from oracle.model import DEAD, PROLIF
from oracle.protocol import events, lq_survival, lq_threshold
from oracle.sim import pack, unpack


def grown_state(params, L, p, r, seed, steps):
    fields, cells, _ = sim.run_instance(params, L, steps, 10, [], p, r, seed)
    return fields, cells


def test_even_half_hours_reproduce_the_hourly_protocol(params):
    dose = np.float32([2.0, 1.5, 2.5, 1.0])
    gap = np.int32([3, 6, 5, 7])
    L, H, seed = 32, 30, 11
    ev_h = events(dose, gap, 4, H, params)
    ev_half = events(dose, 2 * gap, 4, H, params, half_hour=True)
    assert [t for t, _ in ev_half] == [2 * t for t, _ in ev_h]
    for r in range(2):
        a = sim.run_instance(params, L, H, 10, ev_h, 0, r, seed)
        b = sim.run_instance(params, L, H, 10, ev_half, 0, r, seed, half_hour=True)
        assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1]) and np.array_equal(a[2], b[2])


def test_half_hour_events_and_horizon(params):
    dose = np.float32([1.0, 0.0, 2.0, 3.0])
    gap = np.int32([1, 2, 2, 4])                     # half-hours 1, 3 (zero dose), 5, 9
    ev = events(dose, gap, 4, 5, params, half_hour=True)
    assert [t for t, _ in ev] == [1, 5, 9]           # 9 < 2 * 5: inside a 5-hour horizon
    assert [t for t, _ in events(dose, gap, 4, 4, params, half_hour=True)] == [1, 5]
    assert ev[0][1] == [lq_threshold(1.0, m, params.alpha, params.beta) for m in params.m]


def test_lethal_fraction_timing_orders_the_fields(params):
    """A fraction that kills every cell at the start of the hour, at its
    middle, or not at all: the cells after the step agree for the two lethal
    timings, and oxygen and glucose are pointwise highest when the consumers
    die first and lowest when they survive (acid the reverse), strictly
    somewhere: the FTCS map with lambda <= 1/4 and the clamp is monotone."""
    L, seed = 32, 5
    f0, c0 = grown_state(params, L, 0, 0, seed, 40)
    n = 40
    lethal = [0, 0, 0, 0]
    fa, ca = sim.step(f0, c0, n, lethal, 0, 0, seed, params, 10)
    fb, cb = sim.step(f0, c0, n, None, 0, 0, seed, params, 10, thresholds_mid=lethal)
    fc, cc = sim.step(f0, c0, n, None, 0, 0, seed, params, 10)
    assert np.array_equal(ca, cb)
    assert np.all(unpack(ca)[0][unpack(c0)[0] != 0] != PROLIF)
    for f in (0, 1):
        assert np.all(fa[f] >= fb[f]) and np.all(fb[f] >= fc[f])
        assert np.any(fa[f] > fb[f]) and np.any(fb[f] > fc[f])
    assert np.all(fa[2] <= fb[2]) and np.all(fb[2] <= fc[2])
    assert np.any(fa[2] < fb[2]) and np.any(fb[2] < fc[2])


def test_two_fractions_in_one_hour_kill_independently(params):
    """A full lattice of young proliferating cells (no free site, fields at
    their initial values) takes fractions at the start and the middle of one
    hour: survivors ~ Binomial(N, S1 S2).  Reusing the start's word for the
    middle fraction would give min(S1, S2) instead."""
    L = 120
    cells = pack(np.full((L, L), PROLIF), np.full((L, L), 1))
    fields = np.empty((3, L, L))
    for f in range(3):
        fields[f] = params.init[f]
    d1, d2 = 2.0, 3.0
    m = params.m[0]
    thr1 = [lq_threshold(d1, mc, params.alpha, params.beta) for mc in params.m]
    thr2 = [lq_threshold(d2, mc, params.alpha, params.beta) for mc in params.m]
    s = lq_survival(d1, m, params.alpha, params.beta) * lq_survival(d2, m, params.alpha, params.beta)
    N = L * L
    for seed in (1, 2, 3):
        _, out = sim.step(fields, cells, 7, thr1, 0, 0, seed, params, 2, thresholds_mid=thr2)
        st = unpack(out)[0]
        surv = int(np.count_nonzero(st != DEAD))
        assert abs(surv - N * s) < 4.5 * np.sqrt(N * s * (1 - s)), (seed, surv, N * s)
