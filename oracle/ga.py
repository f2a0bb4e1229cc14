"""Genetic-algorithm operators over fixed-length protocols.

Test infrastructure: part of the CPU oracle (see oracle/__init__.py).

The paper's GA (Materials and Methods, "The Main GA Loop"; appendix "GA
Operators: additional details") keeps the best protocols unchanged (elitism),
selects parents, recombines them by crossover, mutates the children and repairs
them with guard algorithms, among them one that lowers the largest dose while
the total dose exceeds the cap.  This module fixes the variant used by the
device GA: a genome is K genes (dose_j, delay_j); lower fitness is better.

One generation, from population (dose, gap) with fitness f:
  1. rank: order by (f, index), NaN last; position[i] = rank of protocol i;
  2. the n_elite best protocols are copied to slots 0 .. n_elite-1;
  3. child pair c fills slots n_elite + 2c and n_elite + 2c + 1:
     parents a, b by tournament: k uniform picks idx = floor(w * N / 2^32),
       the pick with the smallest rank position wins;
     with probability p_cross (w < floor(p_cross * 2^32)) one-point crossover
       at cut = 1 + floor(w' * (K - 1) / 2^32): child 1 = a[:cut] + b[cut:],
       child 2 = b[:cut] + a[cut:]; otherwise the children copy a and b;
     per-gene mutation: the dose of gene j is redrawn from the dose alphabet
       iff w0 < floor(p_mut * 2^32) (value index floor(w1 n_dose / 2^32)), the
       delay likewise with w2, w3;
     guard: while the total exceeds the cap, the largest dose (first one among
       equals) moves down to the next smaller alphabet value (if none is
       smaller, the next largest dose moves instead).
Random words: Philox4x32-10 blocks, counter (c, generation, 0x47414741, sub),
key (seed lo, seed hi): sub 0 .. nb-1 tournament a, nb .. 2nb-1 tournament b
(nb = ceil(k / 4), words used in order), sub 2nb crossover (w0, w1), sub
2nb + 1 + child * K + j mutation of gene j of child 0 / 1.

Variants closer to the paper's appendix (selected by keyword; the defaults
above are selection "tournament", crossover "one_point", mutation ("gene",)):
  selection "rank": k uniform picks sorted by rank; the j-th best is taken
    with probability q (1 - q)^j for j < k - 1 (word k + j < floor(q 2^32)),
    else the last: the paper's rank-based tournament;
  selection "roulette": score_i = max(base - f_i, 0) (the paper's
    fitness-proportional rule on its score base - live count; NaN scores 0),
    summed in index order in float64; u = w0 * total / 2^32; the first i whose
    running sum exceeds u (uniform pick if the total is 0);
  selection "truncation": uniform over the best M = max(1, floor(frac N))
    (the paper's "simple" selection of the top 40 %);
  the selection words per parent are k (tournament), 2k - 1 (rank) or 1, and
  nb = ceil(words / 4);
  crossover "middle": one cut uniform on [max(1, K // 4), min(K - 1, 3K // 4)]
    (the paper draws it between 25 % and 75 % of the length);
  crossover "two_point": cuts c1 uniform on [K // 4, K // 2] (w1) and c2 on
    [K // 2, 3K // 4] (w2); genes c1 .. c2 - 1 are exchanged;
  crossover "uniform": gene j comes from the other parent iff bit j of
    w1 + 2^32 w2 is set (complementary children);
  mutation "swap" (sub 2nb + 1 + 2K + 2 child): with probability p_mut the
    doses at positions i = floor(w1 K / 2^32) and j (floor(w2 (K - 1) / 2^32),
    shifted past i) are exchanged;
  mutation "raise" (sub 2nb + 2 + 2K + 2 child): with probability p_mut, if
    the total is below the cap, the dose at floor(w1 K / 2^32) is replaced by
    a larger alphabet dose chosen uniformly (w2), then the guard applies;
  mutations run in the order gene, swap, raise, then the guard.
"""
import math

import numpy as np

from .philox import philox4x32_10

GA_TAG = 0x47414741


def rank_order(fitness):
    """(order, position): order[r] = index of rank r; position[i] = rank of i."""
    f = np.asarray(fitness, dtype=np.float64)
    key = np.where(np.isnan(f), np.inf, f)
    order = np.array(sorted(range(len(f)), key=lambda i: (key[i], i)), dtype=np.int64)
    position = np.empty(len(f), dtype=np.int64)
    position[order] = np.arange(len(f))
    return order, position


def _words(c, generation, sub, seed):
    w = philox4x32_10(c, generation, GA_TAG, sub, seed & 0xFFFFFFFF, (seed >> 32) & 0xFFFFFFFF)
    return [int(x) for x in w]


def _threshold(p):
    return min(int(math.floor(p * 4294967296.0)), 0xFFFFFFFF)


def guard(q, dose_q, cap_q):
    """Lower the largest dose (in quanta) one alphabet step until sum <= cap_q."""
    q = list(q)
    steps = sorted(dose_q)
    while sum(q) > cap_q:
        order = sorted(range(len(q)), key=lambda j: (-q[j], j))
        for j in order:
            lower = [v for v in steps if v < q[j]]
            if lower:
                q[j] = lower[-1]
                break
        else:
            raise ValueError("guard cannot meet the cap with this alphabet")
    return q


def _select(words, k, N, position, order, fitness, selection, q, trunc_frac, roulette_base):
    if selection == "tournament":
        picks = [(words[i] * N) >> 32 for i in range(k)]
        return min(picks, key=lambda i: position[i])
    if selection == "rank":
        picks = sorted(((words[i] * N) >> 32 for i in range(k)), key=lambda i: position[i])
        t_q = _threshold(q)
        for j in range(k - 1):
            if words[k + j] < t_q:
                return picks[j]
        return picks[k - 1]
    if selection == "roulette":
        score = [0.0 if math.isnan(f) else max(roulette_base - float(f), 0.0) for f in fitness]
        total = 0.0
        for v in score:
            total += v
        if total <= 0.0:
            return (words[0] * N) >> 32
        u = words[0] * total / 4294967296.0
        run, last = 0.0, 0
        for i, v in enumerate(score):
            run += v
            if v > 0.0:
                last = i
            if run > u:
                return i
        return last
    if selection == "truncation":
        m = max(1, min(N, int(math.floor(trunc_frac * N))))
        return int(order[(words[0] * m) >> 32])
    raise ValueError(selection)


def _selection_words(selection, k):
    return {"tournament": k, "rank": 2 * k - 1, "roulette": 1, "truncation": 1}[selection]


def _crossover(ga, gb, w, crossover, t_cross):
    K = len(ga)
    if not (w[0] < t_cross and K > 1):
        return [list(ga), list(gb)]
    if crossover in ("one_point", "middle"):
        lo, hi = (1, K - 1) if crossover == "one_point" else (max(1, K // 4), max(max(1, K // 4), min(K - 1, 3 * K // 4)))
        cut = lo + ((w[1] * (hi - lo + 1)) >> 32)
        return [ga[:cut] + gb[cut:], gb[:cut] + ga[cut:]]
    if crossover == "two_point":
        c1 = K // 4 + ((w[1] * (K // 2 - K // 4 + 1)) >> 32)
        c2 = K // 2 + ((w[2] * (3 * K // 4 - K // 2 + 1)) >> 32)
        if c1 >= c2:
            return [list(ga), list(gb)]
        return [ga[:c1] + gb[c1:c2] + ga[c2:], gb[:c1] + ga[c1:c2] + gb[c2:]]
    if crossover == "uniform":
        bits = w[1] | (w[2] << 32)
        return [[gb[j] if (bits >> j) & 1 else ga[j] for j in range(K)],
                [ga[j] if (bits >> j) & 1 else gb[j] for j in range(K)]]
    raise ValueError(crossover)


def next_generation(dose, gap, fitness, generation, seed, alphabet, n_elite, k, p_cross, p_mut, n_out=None,
                    selection="tournament", crossover="one_point", mutation=("gene",), q=0.9, trunc_frac=0.4,
                    roulette_base=0.0):
    """Return (next_dose, next_gap) with n_out rows (default: as many as the
    population); slots n_elite .. n_out-1 hold children."""
    dose = np.asarray(dose, np.float32)
    gap = np.asarray(gap, np.int32)
    N, K = dose.shape
    n_out = N if n_out is None else int(n_out)
    quantum = float(np.float32(alphabet["dose_quantum"]))
    dose_q = [int(v) for v in alphabet["dose_q"]]
    gaps = [int(v) for v in alphabet["gaps"]]
    cap_q = int(math.floor(float(np.float32(alphabet["cap"])) / quantum + 1e-9))
    order, position = rank_order(fitness)
    out_d = np.zeros((n_out, K), np.float32)
    out_g = np.zeros((n_out, K), np.int32)
    out_d[:n_elite] = dose[order[:n_elite]]
    out_g[:n_elite] = gap[order[:n_elite]]
    nb = (_selection_words(selection, k) + 3) // 4
    t_cross, t_mut = _threshold(p_cross), _threshold(p_mut)
    n_pairs = (n_out - n_elite + 1) // 2
    fit = np.asarray(fitness, np.float32)
    for c in range(n_pairs):
        parents = []
        for t in range(2):
            words = []
            for b in range(nb):
                words += _words(c, generation, t * nb + b, seed)
            parents.append(_select(words, k, N, position, order, fit, selection, q, trunc_frac, roulette_base))
        a, b = parents
        wc = _words(c, generation, 2 * nb, seed)
        ga = [(int(round(float(dose[a, j]) / quantum)), int(gap[a, j])) for j in range(K)]
        gb = [(int(round(float(dose[b, j]) / quantum)), int(gap[b, j])) for j in range(K)]
        kids = _crossover(ga, gb, wc, crossover, t_cross)
        for ch in range(2):
            slot = n_elite + 2 * c + ch
            if slot >= n_out:
                break
            genes = kids[ch]
            if "gene" in mutation:
                for j in range(K):
                    w = _words(c, generation, 2 * nb + 1 + ch * K + j, seed)
                    qd, gg = genes[j]
                    if w[0] < t_mut:
                        qd = dose_q[(w[1] * len(dose_q)) >> 32]
                    if w[2] < t_mut:
                        gg = gaps[(w[3] * len(gaps)) >> 32]
                    genes[j] = (qd, gg)
            qs = [g[0] for g in genes]
            if "swap" in mutation and K > 1:
                w = _words(c, generation, 2 * nb + 1 + 2 * K + 2 * ch, seed)
                if w[0] < t_mut:
                    i = (w[1] * K) >> 32
                    j = (w[2] * (K - 1)) >> 32
                    j += j >= i
                    qs[i], qs[j] = qs[j], qs[i]
            if "raise" in mutation:
                w = _words(c, generation, 2 * nb + 2 + 2 * K + 2 * ch, seed)
                if w[0] < t_mut and sum(qs) < cap_q:
                    i = (w[1] * K) >> 32
                    larger = [v for v in dose_q if v > qs[i]]
                    if larger:
                        qs[i] = larger[(w[2] * len(larger)) >> 32]
            qs = guard(qs, dose_q, cap_q)
            out_d[slot] = np.array([qq * quantum for qq in qs], np.float64).astype(np.float32)
            out_g[slot] = [g[1] for g in genes]
    return out_d, out_g
