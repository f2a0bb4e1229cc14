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


def next_generation(dose, gap, fitness, generation, seed, alphabet, n_elite, k, p_cross, p_mut, n_out=None):
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
    nb = (k + 3) // 4
    t_cross, t_mut = _threshold(p_cross), _threshold(p_mut)
    n_pairs = (n_out - n_elite + 1) // 2
    for c in range(n_pairs):
        parents = []
        for t in range(2):
            words = []
            for b in range(nb):
                words += _words(c, generation, t * nb + b, seed)
            picks = [(words[i] * N) >> 32 for i in range(k)]
            parents.append(min(picks, key=lambda i: position[i]))
        a, b = parents
        wc = _words(c, generation, 2 * nb, seed)
        ga = [(int(round(float(dose[a, j]) / quantum)), int(gap[a, j])) for j in range(K)]
        gb = [(int(round(float(dose[b, j]) / quantum)), int(gap[b, j])) for j in range(K)]
        if wc[0] < t_cross and K > 1:
            cut = 1 + ((wc[1] * (K - 1)) >> 32)
            kids = [ga[:cut] + gb[cut:], gb[:cut] + ga[cut:]]
        else:
            kids = [list(ga), list(gb)]
        for ch in range(2):
            slot = n_elite + 2 * c + ch
            if slot >= n_out:
                break
            genes = kids[ch]
            for j in range(K):
                w = _words(c, generation, 2 * nb + 1 + ch * K + j, seed)
                qd, gg = genes[j]
                if w[0] < t_mut:
                    qd = dose_q[(w[1] * len(dose_q)) >> 32]
                if w[2] < t_mut:
                    gg = gaps[(w[3] * len(gaps)) >> 32]
                genes[j] = (qd, gg)
            q = guard([g[0] for g in genes], dose_q, cap_q)
            out_d[slot] = np.array([qq * quantum for qq in q], np.float64).astype(np.float32)
            out_g[slot] = [g[1] for g in genes]
    return out_d, out_g
