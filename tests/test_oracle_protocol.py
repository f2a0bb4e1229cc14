"""Pins of protocol handling: the paper's benchmark protocols and counts of
feasible protocols, the validator's rules, and the population sampler."""
import math

import numpy as np
import pytest

from oracle import protocol as pr


def test_benchmark_protocol_fraction_times(golden, params):
    """BMI: 1.25 Gy at 0, 6, 24, 30, 48, 54, 72, 78 h; BMII: 2 Gy every 24 h."""
    for name, times in (("BMI", [0, 6, 24, 30, 48, 54, 72, 78]), ("BMII", [0, 24, 48, 72, 96])):
        g = golden[name]
        ev = pr.events(np.array(g["dose"], np.float32), np.array(g["delay_h"]), len(g["dose"]), 240, params)
        assert [t for t, _ in ev] == times
        assert math.isclose(sum(g["dose"]), 10.0)


def test_paper_counts_of_feasible_protocols(golden):
    """The paper's counts (3.0e11 for BMI, 4.1e6 for BMII, at least 1.39e15 for
    the phase-2 space) follow from a plain count under the stated rules."""
    half_hours = lambda lo, hi: list(range(int(2 * lo), int(2 * hi) + 1))
    bmi = pr.count_sequences(half_hours(4, 26), 7, 240)
    bmii = pr.count_sequences(half_hours(10, 32), 4, 240)
    assert f"{bmi:.1e}" == f"{golden['count_BMI_approx']:.1e}"
    assert f"{bmii:.1e}" == f"{golden['count_BMII_approx']:.1e}"
    ph2 = pr.count_sequences(list(range(0, 21)), 20, 40, exact=True)
    assert ph2 >= golden["count_phase2_lower_bound"]
    assert pr.count_sequences(list(range(0, 41)), 20, 40, exact=True) == math.comb(59, 19)
    assert pr.count_sequences(list(range(50)), 10, 490) == 50 ** 10   # (10 x 5)^10


def test_count_matches_enumeration():
    vals = [1, 2, 4]
    for length in range(0, 5):
        for budget in range(0, 12):
            brute = sum(1 for seq in np.ndindex(*([len(vals)] * length))
                        if sum(vals[i] for i in seq) <= budget)
            assert pr.count_sequences(vals, length, budget) == brute


def test_validator_rules():
    K = 3
    dose = np.array([[1, 1, 1], [1, -1, 1], [5, 5, 5], [1, 1, 1], [1, 1, 1], [1, 1, 0], [np.nan, 1, 1]], np.float32)
    gap = np.array([[0, 1, 1], [0, 1, 1], [0, 1, 1], [-1, 1, 1], [0, 0, 1], [0, 3, 0], [0, 1, 1]])
    nfrac = np.array([3, 3, 3, 3, 3, 2, 3])
    st = pr.validate(dose, gap, nfrac, K, cap=12.0)
    assert list(st) == [pr.OK, pr.E_DOSE, pr.E_CAP, pr.E_GAP, pr.E_GAP, pr.OK, pr.E_DOSE]
    assert list(pr.validate(dose[:1], gap[:1], [4], K, 12.0)) == [pr.E_NFRAC]
    assert list(pr.validate(dose[:1], gap[:1], [-1], K, 12.0)) == [pr.E_NFRAC]
    assert list(pr.validate(np.array([[4, 4, 4.0000005]], np.float32), gap[:1], [3], K, 12.0)) == [pr.OK]


def test_events_drop_late_and_zero_dose_fractions(params):
    ev = pr.events(np.array([1.0, 0.0, 2.0, 1.0], np.float32), np.array([5, 5, 5, 100]), 4, 50, params)
    assert [t for t, _ in ev] == [5, 15]


SMALL = dict(dose_quantum=0.5, dose_q=[1, 2, 3], gaps=[6, 12], kmin=3, kmax=3, cap=3.0)


def test_sampler_is_uniform_over_feasible_set():
    """Dose sequences of 3 fractions from {0.5, 1, 1.5} Gy with total <= 3 Gy:
    every one of the 17 feasible sequences is equally likely (chi-square)."""
    from scipy.stats import chisquare
    feas = [s for s in np.ndindex(3, 3, 3) if sum(v + 1 for v in s) <= 6]
    assert len(feas) == pr.count_sequences([1, 2, 3], 3, 6) == 17
    dose, gap, nfrac = pr.sample_population(SMALL, 6000, 4, seed=21)
    assert np.all(nfrac == 3) and np.all(dose[:, 3] == 0) and np.all(gap[:, 3] == 0)
    assert np.all(dose.sum(1) <= 3.0)
    idx = {s: i for i, s in enumerate(feas)}
    counts = np.zeros(len(feas))
    for row in dose:
        counts[idx[tuple(int(round(v / 0.5)) - 1 for v in row[:3])]] += 1
    assert chisquare(counts).pvalue > 1e-3
    assert set(np.unique(gap[:, :3])) == {6, 12}


def test_sampler_config2_alphabet_matches_rejection_statistics():
    """Config-2 alphabet (10 fractions, doses 0.5..2.5 Gy, cap 20 Gy): the mean
    dose per fraction equals that of rejection sampling (exact enumeration by
    the counting programme)."""
    a = dict(dose_quantum=0.5, dose_q=[1, 2, 3, 4, 5], gaps=list(range(6, 61, 6)), kmin=10, kmax=10, cap=20.0)
    dose, gap, nfrac = pr.sample_population(a, 3000, 10, seed=3)
    assert np.all(dose.sum(1) <= 20.0 + 1e-6)
    # exact mean of the first dose under the uniform law on the feasible set
    C = pr.completion_table([1, 2, 3, 4, 5], 10, 40)
    w = np.array([C[9, 40 - v] for v in (1, 2, 3, 4, 5)])
    mean_q = (w * np.arange(1, 6)).sum() / w.sum()
    sd = math.sqrt(((w * np.arange(1, 6) ** 2).sum() / w.sum() - mean_q ** 2) / len(dose))
    assert abs(dose[:, 0].mean() / 0.5 - mean_q) < 5 * sd
    assert abs(gap[:, :].mean() - 33.0) < 0.5


def test_sampler_fraction_count_range():
    a = dict(dose_quantum=0.5, dose_q=list(range(1, 11)), gaps=[6, 12, 24], kmin=3, kmax=40, cap=30.0)
    dose, gap, nfrac = pr.sample_population(a, 400, 40, seed=8)
    assert nfrac.min() >= 3 and nfrac.max() <= 40 and len(np.unique(nfrac)) > 20
    assert np.all(dose.sum(1) <= 30.0 + 1e-6)
    for p in range(len(nfrac)):
        assert np.all(dose[p, :nfrac[p]] >= 0.5) and np.all(dose[p, nfrac[p]:] == 0)
    assert np.all(pr.validate(dose, gap, nfrac, 40, 30.0) == 0)


def test_sampler_rejects_infeasible_alphabet():
    with pytest.raises(ValueError):
        pr.sample_population(dict(dose_quantum=1.0, dose_q=[2], gaps=[6], kmin=4, kmax=4, cap=7.0), 1, 4, 0)
