"""GA over the paper's sparse time-slot genome.

Test infrastructure: part of the CPU oracle (see oracle/__init__.py).

The paper's GA (Materials and Methods, "GA Resolution, constraints" and
"Protocol Representation"; appendix "GA Operators: additional details")
holds a protocol as a vector of doses, one per time slot of the treatment
window and mostly zero, under a cap on the total dose, a maximal single dose
and a minimal interval between doses.  Crossover acts on slots; mutations
swap, split, move (dose time) and enlarge (dose value) doses; guard
algorithms restore the interval and the total.

Genome: S slots of one model hour (the paper's slots are 30 minutes of its
finer model clock; this model steps in hours), each a dose in quanta (0: no
dose; at most dmax).  pick(w, n) = floor(w n / 2^32).  "The i-th dose" counts
the nonzero slots in slot order from 0.

Child pair c of generation g.  Parents as in oracle.ga (same words and rules,
blocks sub 0 .. 2nb - 1).  Then, with the GA's Philox blocks
(c, g, 0x47414741, sub):
  crossover (block 2nb, taken iff w0 < t_cross): one_point (cut
    1 + pick(w1, S - 1)); middle (cut uniform on max(1, S // 4) ..
    min(S - 1, 3 S // 4): the paper's single point between 25 % and 75 %);
    two_point (c1 = S // 4 + pick(w1, S // 2 - S // 4 + 1), c2 = S // 2 +
    pick(w2, 3 S // 4 - S // 2 + 1), slots [c1, c2) exchanged); uniform (slot
    j exchanged iff bit j % 32 of word (j // 32) % 4 of block
    2nb + 1 + j // 128); slots at or after the cut are exchanged;
  mutations of child ch (ch = 0, 1), block m of the child is sub
    B + 8 ch + m with B = 2nb + 1 + ceil(S / 128); each enabled operator runs
    once, in the order below, iff w0 of its block is below t_mut:
    swap (m = 0): the pick(w1, n)-th of the n doses (slot i) and slot
      j = pick(w2, S - 1), shifted past i, exchange their contents;
    split (m = 1, 2): the pick(w1, n)-th of the n doses of at least 2 quanta
      (slot s, v quanta) is removed and split into a = 1 + pick(w2, v - 1) and
      v - a; part a goes to slot pick(w3, S), then part v - a to slot
      pick(w0 of block m = 2, S); a part whose slot would exceed dmax goes to
      the next slot, cyclically, where it fits (the emptied slot s always
      does);
    dose time (m = 3): the pick(w1, n)-th dose (slot s) moves to slot
      t = pick(w2, S): min(v_s, dmax - v_t) quanta pass from s to t, the rest
      stays at s;
    dose value (m = 4): when the total is below the cap, the pick(w1, n)-th
      dose v becomes v + 1 + pick(w2, h - v), h = min(dmax, v + cap - total)
      (nothing when h = v);
  then the guards.
Guards, in order:
  clamp: every slot above dmax is set to dmax;
  interval: slots are scanned in time order; a dose less than g_min after the
    last kept dose is removed and placed at the first later slot t with no
    dose in t - g_min + 1 .. t + g_min - 1; if there is none it is dropped
    (the paper skips the allocation when the doses leave no room);
  total: while the total exceeds the cap, the largest dose (first among
    equals) loses one quantum.
Decode: the doses in slot order; delay_1 = slot of the first dose, delay_j =
  slot difference to the previous dose (the simulation's protocol format); at
  most K doses, the first ones (a guarded genome holds at most ceil(S / g_min)).
Encode: fraction j (j < nfrac, nfrac clipped to 0 .. K) lands on slot
  t_j = delay_1 + .. + delay_j, adding round(dose_j / quantum) quanta
  (float32 quotient, ties to even; 0 unless the quotient is positive; a slot
  saturates at 255); the walk stops at the first t_j outside 0 .. S - 1; the
  guards then run.
"""
import math

import numpy as np

from . import ga as fixed

SLOT_MUTATIONS = ("swap", "split", "time", "value")
MUT_BLOCKS = 8


def pick(w, n):
    return (int(w) * int(n)) >> 32


def clamp_guard(v, dmax):
    return [min(int(x), dmax) for x in v]


def interval_guard(v, g_min):
    v = list(v)
    S = len(v)
    last = None
    for s in range(S):
        if v[s] == 0:
            continue
        if last is None or s - last >= g_min:
            last = s
            continue
        d, v[s] = v[s], 0
        for t in range(s + 1, S):
            lo, hi = max(0, t - g_min + 1), min(S, t + g_min)
            if all(v[u] == 0 for u in range(lo, hi)):
                v[t] = d
                break
    return v


def total_guard(v, cap_q):
    v = list(v)
    while sum(v) > cap_q:
        j = max(range(len(v)), key=lambda i: (v[i], -i))
        v[j] -= 1
    return v


def guards(v, g_min, dmax, cap_q):
    return total_guard(interval_guard(clamp_guard(v, dmax), g_min), cap_q)


def crossover(a, b, wc, mask_bit, kind, t_cross):
    """Children of parents a, b: wc the crossover block, mask_bit(j) the
    uniform mask bit of slot j."""
    S = len(a)
    if not (wc[0] < t_cross and S > 1):
        return list(a), list(b)
    if kind in ("one_point", "middle"):
        lo, hi = (1, S - 1) if kind == "one_point" else (max(1, S // 4), max(max(1, S // 4), min(S - 1, 3 * S // 4)))
        cut = lo + pick(wc[1], hi - lo + 1)
        swap = [j >= cut for j in range(S)]
    elif kind == "two_point":
        c1 = S // 4 + pick(wc[1], S // 2 - S // 4 + 1)
        c2 = S // 2 + pick(wc[2], 3 * S // 4 - S // 2 + 1)
        swap = [c1 <= j < c2 for j in range(S)]
    elif kind == "uniform":
        swap = [bool(mask_bit(j)) for j in range(S)]
    else:
        raise ValueError(kind)
    return ([b[j] if swap[j] else a[j] for j in range(S)],
            [a[j] if swap[j] else b[j] for j in range(S)])


def _nth(v, i, least):
    """Slot of the i-th entry (slot order, from 0) holding at least `least`."""
    seen = 0
    for s, x in enumerate(v):
        if x >= least:
            if seen == i:
                return s
            seen += 1
    raise AssertionError("index past the end")


def mutate_swap(v, w):
    v = list(v)
    S = len(v)
    n = sum(1 for x in v if x > 0)
    if n == 0 or S < 2:
        return v
    i = _nth(v, pick(w[1], n), 1)
    j = pick(w[2], S - 1)
    j += j >= i
    v[i], v[j] = v[j], v[i]
    return v


def mutate_split(v, w, w_second, dmax):
    v = list(v)
    S = len(v)
    n = sum(1 for x in v if x >= 2)
    if n == 0:
        return v
    s = _nth(v, pick(w[1], n), 2)
    total, v[s] = v[s], 0
    a = 1 + pick(w[2], total - 1)
    for part, r in ((a, pick(w[3], S)), (total - a, pick(w_second, S))):
        t = r
        for step in range(S):
            t = (r + step) % S
            if v[t] + part <= dmax:
                break
        else:
            t = s
        v[t] += part
    return v


def mutate_time(v, w, dmax):
    v = list(v)
    S = len(v)
    n = sum(1 for x in v if x > 0)
    if n == 0:
        return v
    s = _nth(v, pick(w[1], n), 1)
    t = pick(w[2], S)
    if t != s:
        m = max(0, min(v[s], dmax - v[t]))
        v[t] += m
        v[s] -= m
    return v


def mutate_value(v, w, dmax, cap_q):
    v = list(v)
    n = sum(1 for x in v if x > 0)
    total = sum(v)
    if n == 0 or total >= cap_q:
        return v
    s = _nth(v, pick(w[1], n), 1)
    h = min(dmax, v[s] + cap_q - total)
    if h > v[s]:
        v[s] = v[s] + 1 + pick(w[2], h - v[s])
    return v


def mutate(v, block, t_mut, mutations, dmax, cap_q):
    """All enabled mutations of one child; block(m) gives its m-th block."""
    if "swap" in mutations:
        w = block(0)
        if w[0] < t_mut:
            v = mutate_swap(v, w)
    if "split" in mutations:
        w = block(1)
        if w[0] < t_mut:
            v = mutate_split(v, w, block(2)[0], dmax)
    if "time" in mutations:
        w = block(3)
        if w[0] < t_mut:
            v = mutate_time(v, w, dmax)
    if "value" in mutations:
        w = block(4)
        if w[0] < t_mut:
            v = mutate_value(v, w, dmax, cap_q)
    return v


def next_generation_slots(pop, fitness, generation, seed, g_min, dmax, cap_q, n_elite, k, p_cross, p_mut,
                          selection="tournament", crossover_kind="one_point", mutations=SLOT_MUTATIONS, q=0.9,
                          trunc_frac=0.4, roulette_base=0.0, n_out=None, rows=None):
    """Next population [n_out][S] (uint8) of population pop [N][S]; rows
    n_elite .. n_out - 1 hold children.  With `rows` (an iterable of row
    indices) only those rows are computed; the others stay 0."""
    pop = np.asarray(pop, np.int64)
    N, S = pop.shape
    n_out = N if n_out is None else int(n_out)
    order, position = fixed.rank_order(fitness)
    out = np.zeros((n_out, S), np.uint8)
    out[:n_elite] = pop[order[:n_elite]]
    nb = (fixed._selection_words(selection, k) + 3) // 4
    t_cross, t_mut = fixed._threshold(p_cross), fixed._threshold(p_mut)
    fit = np.asarray(fitness, np.float32)
    n_mask = (S + 127) // 128
    base = 2 * nb + 1 + n_mask
    want = None if rows is None else set(int(r) for r in rows)
    for c in range((n_out - n_elite + 1) // 2):
        if want is not None and not ({n_elite + 2 * c, n_elite + 2 * c + 1} & want):
            continue
        parents = []
        for t in range(2):
            words = []
            for b in range(nb):
                words += fixed._words(c, generation, t * nb + b, seed)
            parents.append(fixed._select(words, k, N, position, order, fit, selection, q, trunc_frac,
                                         roulette_base))
        wc = fixed._words(c, generation, 2 * nb, seed)
        mask = [fixed._words(c, generation, 2 * nb + 1 + m, seed) for m in range(n_mask)]
        kids = crossover(pop[parents[0]].tolist(), pop[parents[1]].tolist(), wc,
                         lambda j: (mask[j // 128][(j // 32) % 4] >> (j % 32)) & 1, crossover_kind, t_cross)
        for ch in range(2):
            row = n_elite + 2 * c + ch
            if row >= n_out:
                break
            if want is not None and row not in want:
                continue
            sub0 = base + MUT_BLOCKS * ch
            v = mutate(kids[ch], lambda m: fixed._words(c, generation, sub0 + m, seed), t_mut, mutations,
                       dmax, cap_q)
            out[row] = guards(v, g_min, dmax, cap_q)
    return out


def decode(v, quantum, K):
    """(dose[K] in Gy, delay[K] in hours, nfrac) of one genome; a genome with
    more than K doses gives its first K."""
    slots = [s for s, x in enumerate(v) if x > 0][:K]
    dose = np.zeros(K, np.float32)
    gap = np.zeros(K, np.int32)
    prev = 0
    qf = np.float32(quantum)
    for j, s in enumerate(slots):
        dose[j] = np.float32(v[s]) * qf
        gap[j] = s - prev
        prev = s
    return dose, gap, len(slots)


def encode(dose, gap, nfrac, S, quantum, g_min, dmax, cap_q):
    """Guarded slot genome (list of S quanta) of one (dose, delay) protocol."""
    v = [0] * S
    t = 0
    qf = np.float32(quantum)
    for j in range(min(max(int(nfrac), 0), len(gap))):
        t += int(gap[j])
        if t < 0 or t >= S:
            break
        x = np.float32(dose[j]) / qf
        qd = int(min(np.rint(x), np.float32(255))) if x > 0 else 0
        v[t] = min(255, v[t] + qd)
    return guards(v, g_min, dmax, cap_q)


def max_doses(S, g_min):
    """Most doses a genome of S slots can hold at interval g_min."""
    return (S + g_min - 1) // g_min
