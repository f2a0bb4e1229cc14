"""Protocols: validation, event decoding, LQ survival thresholds, counting, sampling.

Test infrastructure: part of the CPU oracle (see oracle/__init__.py).

A protocol is a sequence of k (dose, delay) pairs; the delay of the first pair
counts from the start of the simulation and every later delay is the wait after
the previous fraction (Results, "Defining the search problem").  The total dose
is capped (same section, the constraint under the max-f problem).  Time is
counted in whole model hours here: fraction j is given at the start of step
t_j = sum_{i<=j} delay_i.
"""
import math

import numpy as np

from .philox import philox4x32_10

# Per-protocol status codes (shared meaning with the library's validator).
OK, E_NFRAC, E_DOSE, E_CAP, E_GAP = 0, 1, 2, 3, 4
CAP_SLACK = 1e-6


def validate(dose, gap, nfrac, K, cap):
    """Status of each protocol: OK, or the first rule it breaks.

    Rules, checked in this order: 0 <= nfrac <= K; every used dose finite and
    >= 0; delay_1 >= 0 and delay_j >= 1 (hours) for j >= 2, so no two fractions
    share a step; total dose <= cap (+1e-6 slack), summed in float64 in index
    order.
    """
    dose = np.asarray(dose, dtype=np.float32).reshape(-1, K)
    gap = np.asarray(gap, dtype=np.int64).reshape(-1, K)
    nfrac = np.asarray(nfrac, dtype=np.int64).reshape(-1)
    out = np.zeros(len(nfrac), dtype=np.int32)
    for p in range(len(nfrac)):
        k = int(nfrac[p])
        if k < 0 or k > K:
            out[p] = E_NFRAC
            continue
        status, total = OK, 0.0
        for j in range(k):
            d = float(dose[p, j])
            if not math.isfinite(d) or d < 0.0:
                status = E_DOSE
                break
            if gap[p, j] < (0 if j == 0 else 1):
                status = E_GAP
                break
            total += d
        if status == OK and total > cap + CAP_SLACK:
            status = E_CAP
        out[p] = status
    return out


def lq_survival(d, m, alpha, beta):
    """Linear-quadratic surviving fraction exp(-alpha x - beta x^2), x = m d."""
    x = float(m) * float(d)
    return math.exp(-alpha * x - beta * x * x)


def lq_threshold(d, m, alpha, beta, prior=0.0):
    """32-bit survival threshold: a cell survives iff its word w1 < threshold.

    threshold = min(floor(S * 2**32), 2**32 - 1), S the LQ surviving fraction,
    evaluated in float64 (the multiplication by 2**32 is exact).  With
    unrepaired damage from earlier fractions (`prior`, in Gy, see
    prior_damage), S = exp(-alpha x - beta x (x + 2 y)), x = m d, y = m prior:
    the incomplete-repair form of the linear-quadratic law, in which the
    quadratic term couples each fraction with the unrepaired part of every
    earlier one; prior = 0 is the plain law.
    """
    x = float(m) * float(d)
    y = float(m) * float(prior)
    s = math.exp(-alpha * x - beta * x * (x + 2.0 * y))
    return min(int(math.floor(s * 4294967296.0)), 0xFFFFFFFF)


def prior_damage(dose_row, gap_row, j, half_time, unit=1.0):
    """Unrepaired dose before fraction j: sum over earlier fractions i of
    d_i 2^(-(t_j - t_i) / half_time) (mono-exponential repair with the given
    half-time in hours; times in units of `unit` hours), summed in index
    order; 0 when half_time is 0 (complete repair between fractions)."""
    if half_time <= 0.0:
        return 0.0
    t = [0]
    for i in range(j + 1):
        t.append(t[-1] + int(gap_row[i]))
    tj = t[j + 1]
    acc = 0.0
    for i in range(j):
        di = float(np.float32(dose_row[i]))
        if di > 0.0:
            acc += di * 2.0 ** (-(float(tj - t[i + 1]) * unit / half_time))
    return acc


def events(dose_row, gap_row, nfrac, horizon, params, half_hour=False):
    """Irradiation events of one protocol inside [0, horizon) steps.

    Returns a list of (time, thresholds[4]) in time order; thresholds are per
    sensitivity class (young, mid and old proliferating, quiescent).  Fractions
    with zero dose, or falling at or after the horizon, give no event.  Times
    are steps (hours), or with half_hour=True half-hours: the delays are then
    counted in 30-minute units (the paper's slot length, Materials and
    Methods, "GA Resolution, constraints") and an event at half-hour tau falls
    in step tau // 2, at its start (tau even) or its middle (tau odd).
    """
    out, t = [], 0
    end = 2 * horizon if half_hour else horizon
    for j in range(int(nfrac)):
        t += int(gap_row[j])
        d = float(np.float32(dose_row[j]))
        if d <= 0.0 or t >= end:
            continue
        prior = prior_damage(dose_row, gap_row, j, params.repair_half_time, 0.5 if half_hour else 1.0)
        if params.oxygen_effect:
            thr = oxygen_thresholds(d, prior, params)
        else:
            thr = [lq_threshold(d, params.m[c], params.alpha, params.beta, prior) for c in range(4)]
        out.append((t, thr))
    return out


def oxygen_modification(b, params):
    """Dose-modifying factor of oxygen bin b: the oxygen enhancement ratio law
    OMF(O) = (oer_max O + K) / (oer_max (O + K)) (1 when well oxygenated,
    1 / oer_max without oxygen) at the bin's midpoint O = (b + 1/2) O_ref / B,
    O_ref the boundary oxygen value, B = OER_BINS."""
    from .model import OER_BINS
    o = (b + 0.5) * float(params.ghost[0]) / OER_BINS
    return (params.oer_max * o + params.oer_k) / (params.oer_max * (o + params.oer_k))


def oxygen_thresholds(d, prior, params):
    """Thresholds [class][oxygen bin] of a fraction of d Gy (unrepaired dose
    `prior`): the dose and the unrepaired dose are both scaled by the bin's
    oxygen modification factor."""
    from .model import OER_BINS
    out = []
    for c in range(4):
        row = []
        for b in range(OER_BINS):
            f = oxygen_modification(b, params)
            row.append(lq_threshold(f * d, params.m[c], params.alpha, params.beta, f * prior))
        out.append(row)
    return out


def oxygen_bin(o, params):
    """Bin of oxygen level o: floor(B o / O_ref) clamped to 0 .. B - 1."""
    from .model import OER_BINS
    q = float(o) / float(params.ghost[0])
    return min(OER_BINS - 1, max(0, int(math.floor(q * OER_BINS))))


def count_sequences(values, length, budget, exact=False):
    """Number of sequences of `length` items from `values` (non-negative ints)
    whose sum is <= budget (or == budget with exact=True).

    Plain dynamic programme over (items placed, running sum); Python ints, so
    exact at any size.  Used to count the paper's feasible protocol sets
    (Results, "Defining the search problem") and by the population sampler.
    """
    ways = [0] * (budget + 1)
    ways[0] = 1
    for _ in range(length):
        nxt = [0] * (budget + 1)
        for s, w in enumerate(ways):
            if w:
                for v in values:
                    if s + v <= budget:
                        nxt[s + v] += w
        ways = nxt
    return ways[budget] if exact else sum(ways)


def completion_table(dose_q, kmax, cap_q):
    """C[j][s] = number of length-j dose sequences (values dose_q) with sum <= s.

    Returned as float64 (every entry used by the configured alphabets is below
    2**53 and therefore exact).
    """
    C = np.zeros((kmax + 1, cap_q + 1), dtype=np.float64)
    C[0, :] = 1.0
    for j in range(1, kmax + 1):
        for s in range(cap_q + 1):
            C[j, s] = sum(C[j - 1, s - v] for v in dose_q if v <= s)
    return C


POP_TAG = 0x504F5055  # counter word 2 of the population generator's blocks
KPOS = 0xFFFFFFFF     # counter word 1 used for the fraction-count draw


def sample_population(alphabet, P, K, seed):
    """Random protocols, uniform over the feasible set of each fraction count.

    alphabet: dict with dose_quantum (Gy), dose_q (allowed doses in quanta,
    increasing), gaps (allowed delays, hours), kmin, kmax (kmax <= K), cap (Gy).
    For protocol p: k = kmin + floor(w0 * (kmax - kmin + 1) / 2**32) from block
    (p, KPOS, POP_TAG, 0); then for position i, block (p, i, POP_TAG, 0) gives
    U = ((w0 >> 5) * 2**26 + (w1 >> 6)) / 2**53, the dose is the first value v
    whose cumulative completion count exceeds U * C[k-i][budget] (sequential
    conditional sampling, which is uniform over all length-k sequences under the
    cap), and the delay is gaps[floor(w2 * len(gaps) / 2**32)].
    Entries past k are zero.
    """
    q = float(np.float32(alphabet["dose_quantum"]))   # single-precision inputs
    dose_q = [int(v) for v in alphabet["dose_q"]]
    gaps = [int(v) for v in alphabet["gaps"]]
    kmin, kmax = int(alphabet["kmin"]), int(alphabet["kmax"])
    cap_q = int(math.floor(float(np.float32(alphabet["cap"])) / q + 1e-9))
    C = completion_table(dose_q, kmax, cap_q)
    if C[kmax, cap_q] == 0.0:
        raise ValueError("alphabet admits no protocol with kmax fractions under the cap")
    k0, k1 = seed & 0xFFFFFFFF, (seed >> 32) & 0xFFFFFFFF
    dose = np.zeros((P, K), dtype=np.float32)
    gap = np.zeros((P, K), dtype=np.int32)
    nfrac = np.zeros(P, dtype=np.int32)
    for p in range(P):
        wk = philox4x32_10(p, KPOS, POP_TAG, 0, k0, k1)
        k = kmin + (int(wk[0]) * (kmax - kmin + 1) >> 32)
        nfrac[p] = k
        budget = cap_q
        for i in range(k):
            w = [int(x) for x in philox4x32_10(p, i, POP_TAG, 0, k0, k1)]
            u = ((w[0] >> 5) * 67108864.0 + (w[1] >> 6)) * (1.0 / 9007199254740992.0)
            x = u * C[k - i, budget]
            acc, pick = 0.0, None
            for v in dose_q:
                if v > budget or C[k - i - 1, budget - v] == 0.0:
                    break
                acc += C[k - i - 1, budget - v]
                pick = v
                if x < acc:
                    break
            budget -= pick
            dose[p, i] = np.float32(pick * q)
            gap[p, i] = gaps[(w[2] * len(gaps)) >> 32]
    return dose, gap, nfrac
