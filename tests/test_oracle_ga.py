"""Pins of the GA operators: ranking against a library sort, tournament
selection against its exact order-statistic law, crossover and mutation
statistics, the dose guard, and elitism."""
import math

import numpy as np
import pytest
from scipy.stats import chisquare

from oracle import ga

ALPHA = dict(dose_quantum=0.5, dose_q=[1, 2, 3, 4, 5], gaps=list(range(6, 61, 6)), cap=20.0)


def _pop(N, K, seed):
    rng = np.random.default_rng(seed)
    dose = rng.choice([0.5, 1.0, 1.5, 2.0], size=(N, K)).astype(np.float32)
    gap = rng.choice(ALPHA["gaps"], size=(N, K)).astype(np.int32)
    return dose, gap


def test_rank_matches_stable_library_sort(rng):
    f = rng.integers(0, 20, size=300).astype(np.float64)
    f[rng.uniform(size=300) < 0.05] = np.nan
    order, pos = ga.rank_order(f)
    key = np.where(np.isnan(f), np.inf, f)
    assert np.array_equal(order, np.argsort(key, kind="stable"))
    assert np.array_equal(pos[order], np.arange(300))


def test_tournament_follows_order_statistic_law():
    """k picks with replacement, the best rank wins:
    P(rank r) = ((N - r)^k - (N - r - 1)^k) / N^k."""
    N, K, k = 40, 4, 4
    dose, gap = _pop(N, K, 0)
    fitness = np.arange(N, dtype=np.float64)[::-1].copy()   # protocol N-1 is best
    order, pos = ga.rank_order(fitness)
    counts = np.zeros(N)
    nb = 1
    for c in range(6000):
        words = ga._words(c, 3, 0, 99)
        picks = [(w * N) >> 32 for w in words[:k]]
        counts[pos[min(picks, key=lambda i: pos[i])]] += 1
    expect = np.array([((N - r) ** k - (N - r - 1) ** k) / N ** k for r in range(N)]) * counts.sum()
    keep = expect > 5
    obs = np.append(counts[keep], counts[~keep].sum())
    exp = np.append(expect[keep], expect[~keep].sum())
    assert chisquare(obs, exp).pvalue > 1e-3


def test_crossover_exchanges_tails_at_uniform_cut():
    N, K = 64, 10
    dose, gap = _pop(N, K, 1)
    fitness = np.arange(N, dtype=np.float64)
    big = dict(ALPHA, cap=1e6)
    nd, ng = ga.next_generation(dose, gap, fitness, 0, 5, big, n_elite=0, k=1, p_cross=1.0, p_mut=0.0)
    cuts = []
    for c in range(N // 2):
        words = ga._words(c, 0, 0, 5)
        a = (words[0] * N) >> 32
        b = (ga._words(c, 0, 1, 5)[0] * N) >> 32
        wc = ga._words(c, 0, 2, 5)
        cut = 1 + ((wc[1] * (K - 1)) >> 32)
        cuts.append(cut)
        c1, c2 = 2 * c, 2 * c + 1
        assert np.array_equal(nd[c1], np.concatenate([dose[a, :cut], dose[b, cut:]]))
        assert np.array_equal(nd[c2], np.concatenate([dose[b, :cut], dose[a, cut:]]))
        assert np.array_equal(ng[c1], np.concatenate([gap[a, :cut], gap[b, cut:]]))
    assert min(cuts) >= 1 and max(cuts) <= K - 1


def test_mutation_rate():
    N, K, p = 400, 10, 0.05
    dose, gap = _pop(N, K, 2)
    fitness = np.zeros(N)
    big = dict(ALPHA, cap=1e6)
    nd, ng = ga.next_generation(dose, gap, fitness, 1, 7, big, n_elite=0, k=1, p_cross=0.0, p_mut=p)
    # with k = 1 and no crossover each child copies its single pick
    changed_d = changed_g = total = 0
    for c in range(N // 2):
        for t, ch in ((0, 2 * c), (1, 2 * c + 1)):
            src = (ga._words(c, 1, t, 7)[0] * N) >> 32
            changed_d += np.sum(nd[ch] != dose[src])
            changed_g += np.sum(ng[ch] != gap[src])
            total += K
    for changed, n_alpha in ((changed_d, 5), (changed_g, 10)):
        rate = p * (1 - 1.0 / n_alpha) if n_alpha == 10 else None
        if rate is None:   # parent doses are in {0.5..2.0}: redraw hits the old value 1 time in 5
            rate = p * (1 - 1.0 / 5)
        assert abs(changed / total - rate) < 5 * math.sqrt(rate * (1 - rate) / total)


def test_guard_lowers_largest_dose_first():
    assert ga.guard([5, 5, 3], [1, 2, 3, 4, 5], 12) == [4, 5, 3]
    assert ga.guard([5, 5, 3], [1, 2, 3, 4, 5], 11) == [4, 4, 3]
    assert ga.guard([5, 4, 3], [1, 3, 5], 9) == [3, 3, 3]
    assert ga.guard([5, 1, 1], [1, 2, 3, 4, 5], 5) == [3, 1, 1]
    assert ga.guard([2, 2], [1, 2, 3], 10) == [2, 2]
    with pytest.raises(ValueError):
        ga.guard([3, 3], [3], 5)


def test_children_respect_cap_and_elites_are_kept():
    N, K = 64, 10
    rng = np.random.default_rng(3)
    dose = rng.choice([2.0, 2.5], size=(N, K)).astype(np.float32)   # totals 20..25 Gy
    gap = rng.choice(ALPHA["gaps"], size=(N, K)).astype(np.int32)
    fitness = rng.uniform(size=N)
    nd, ng = ga.next_generation(dose, gap, fitness, 4, 11, ALPHA, n_elite=4, k=4, p_cross=0.8, p_mut=0.05)
    order, _ = ga.rank_order(fitness)
    assert np.array_equal(nd[:4], dose[order[:4]]) and np.array_equal(ng[:4], gap[order[:4]])
    assert np.all(nd[4:].astype(np.float64).sum(1) <= 20.0 + 1e-6)
    assert set(np.unique(nd[4:])) <= {0.5, 1.0, 1.5, 2.0, 2.5}


def test_elitism_keeps_best_fitness_monotone():
    """With a deterministic fitness of the protocol, the best never worsens."""
    N, K = 40, 10
    dose, gap = _pop(N, K, 4)
    w = np.linspace(1, 2, K)
    best = []
    for g in range(15):
        f = (dose.astype(np.float64) * w).sum(1) - 0.01 * gap.sum(1)
        best.append(f.min())
        dose, gap = ga.next_generation(dose, gap, f, g, 13, ALPHA, n_elite=2, k=4, p_cross=0.8, p_mut=0.05)
    assert all(b2 <= b1 + 1e-12 for b1, b2 in zip(best, best[1:]))
    assert best[-1] < best[0]


def test_random_screen_generation_invariants(params):
    """The screened generation keeps N rows sorted by fitness, each row either
    an old member with its old fitness or one of the S candidates picked by
    the smallest random keys."""
    from oracle import sga
    rng = np.random.default_rng(5)
    N, K, C, S = 6, 4, 12, 3
    alphabet = dict(dose_quantum=0.5, dose_q=[1, 2, 3, 4], gaps=[6, 12, 24], kmin=K, kmax=K, cap=8.0)
    dose = rng.choice([0.5, 1.0, 1.5], size=(N, K)).astype(np.float32)
    gap = rng.choice([6, 12, 24], size=(N, K)).astype(np.int32)
    fit = sga.simulate_fitness(params, 16, 12, 2, 1, 3, dose, gap)
    d, g, f = sga.generation_random_screen(params, 16, 12, 2, 1, 3, dose, gap, fit, 0, 9, alphabet,
                                           2, 0.8, 0.2, C, S)
    assert d.shape == (N, K) and np.all(np.diff(f) >= 0)
    cd, cg = ga.next_generation(dose, gap, fit, 0, 9, alphabet, 0, 2, 0.8, 0.2, n_out=C)
    keys = sga.random_keys(C, 0, 9)
    assert len(np.unique(keys)) == C and np.all(keys < 2 ** 24)
    picked = np.argsort(keys, kind="stable")[:S]
    new_f = sga.simulate_fitness(params, 16, 12, 2, 1, 3 + sga.W64, cd[picked], cg[picked])
    pool = [(dose[i], gap[i], fit[i]) for i in range(N)] + [(cd[j], cg[j], new_f[n]) for n, j in enumerate(picked)]
    expect = sorted(range(N + S), key=lambda i: (pool[i][2], i))[:N]
    for row, i in enumerate(expect):
        assert np.array_equal(d[row], pool[i][0]) and np.array_equal(g[row], pool[i][1]) and f[row] == pool[i][2]


def _draw_parents(N, K, seed, n_out, **kw):
    """Children of a population whose rows are all distinct, with crossover and
    mutation off, so each child names its parent."""
    rng = np.random.default_rng(seed)
    dose = np.full((N, K), 0.5, np.float32)
    gap = np.zeros((N, K), np.int32)
    for i in range(N):                          # row i spells i in base 10 over the delays
        gap[i] = [ALPHA["gaps"][(i // 10 ** j) % 10] for j in range(K)]
    fitness = rng.permutation(N).astype(np.float64)
    nd, ng = ga.next_generation(dose, gap, fitness, 2, 21, dict(ALPHA, cap=1e6), n_elite=0, p_cross=0.0,
                                p_mut=0.0, n_out=n_out, **kw)
    index = {tuple(r): i for i, r in enumerate(gap.tolist())}
    parents = np.array([index[tuple(r)] for r in ng.tolist()])
    _, pos = ga.rank_order(fitness)
    return parents, pos, fitness


def _chi2_ok(counts, expect):
    keep = expect > 5
    obs, exp = counts[keep], expect[keep]
    if (~keep).any():
        obs, exp = np.append(obs, counts[~keep].sum()), np.append(exp, expect[~keep].sum())
    exp = exp * obs.sum() / exp.sum()
    return chisquare(obs, exp).pvalue > 1e-3


def test_rank_selection_follows_truncated_geometric_over_order_statistics():
    """The j-th best of k uniform picks is taken with probability q (1-q)^j
    (the last with the rest): P(rank r) = sum_j P(take j) P(X_(j) = r), with
    P(X_(j) <= r) = sum_{m > j} C(k, m) p^m (1-p)^(k-m), p = (r + 1) / N."""
    N, K, k, q = 40, 3, 4, 0.6
    parents, pos, _ = _draw_parents(N, K, 0, 8000, k=k, selection="rank", q=q)
    counts = np.bincount(pos[parents], minlength=N).astype(float)
    take = [q * (1 - q) ** j for j in range(k - 1)] + [(1 - q) ** (k - 1)]

    def cdf(j, r):
        p = (r + 1) / N
        return sum(math.comb(k, m) * p ** m * (1 - p) ** (k - m) for m in range(j + 1, k + 1))
    law = np.array([sum(take[j] * (cdf(j, r) - (cdf(j, r - 1) if r else 0.0)) for j in range(k)) for r in range(N)])
    assert abs(law.sum() - 1) < 1e-12
    assert _chi2_ok(counts, law * counts.sum())


def test_roulette_selection_is_proportional_to_score():
    N, K = 30, 3
    parents, _, fitness = _draw_parents(N, K, 1, 8000, k=1, selection="roulette", roulette_base=25.0)
    score = np.maximum(25.0 - fitness, 0.0)
    counts = np.bincount(parents, minlength=N).astype(float)
    assert counts[score == 0].sum() == 0                  # scores at or below zero are never drawn
    assert _chi2_ok(counts[score > 0], score[score > 0] / score.sum() * counts.sum())


def test_truncation_selection_is_uniform_over_the_best():
    N, K = 50, 3
    parents, pos, _ = _draw_parents(N, K, 2, 6000, k=1, selection="truncation", trunc_frac=0.4)
    counts = np.bincount(pos[parents], minlength=N).astype(float)
    assert counts[20:].sum() == 0
    assert _chi2_ok(counts[:20], np.full(20, counts.sum() / 20))


@pytest.mark.parametrize("kind", ["middle", "two_point", "uniform"])
def test_crossover_variants_exchange_genes_between_the_two_parents(kind):
    N, K = 64, 12
    dose, gap = _pop(N, K, 5)
    gap = (np.arange(N * K).reshape(N, K) % 997 + 1).astype(np.int32)      # every gene distinct
    fitness = np.arange(N, dtype=np.float64)
    nd, ng = ga.next_generation(dose, gap, fitness, 0, 8, dict(ALPHA, cap=1e6), n_elite=0, k=1, p_cross=1.0,
                                p_mut=0.0, crossover=kind)
    where = {v: divmod(i, K) for i, v in enumerate(gap.ravel().tolist())}
    cuts, exchanged = [], []
    for c in range(N // 2):
        src = [[where[v] for v in ng[2 * c + h]] for h in (0, 1)]
        assert all(j == jj for h in (0, 1) for jj, (_, j) in enumerate(src[h]))   # genes keep their position
        a = src[0][0][0] if kind != "uniform" else None
        rows0 = [p for p, _ in src[0]]
        rows1 = [p for p, _ in src[1]]
        pa, pb = sorted(set(rows0 + rows1))[0], sorted(set(rows0 + rows1))[-1]
        assert set(rows0 + rows1) <= {pa, pb}
        assert all({x, y} == {pa, pb} or pa == pb for x, y in zip(rows0, rows1))   # complementary children
        if kind == "middle" and pa != pb:
            cut = next(j for j in range(1, K) if rows0[j] != rows0[0])
            assert all(r == rows0[0] for r in rows0[:cut]) and all(r != rows0[0] for r in rows0[cut:])
            cuts.append(cut)
        if kind == "two_point" and pa != pb:
            inside = [j for j in range(K) if rows0[j] != a]
            if inside:
                c1, c2 = inside[0], inside[-1] + 1
                assert inside == list(range(c1, c2)) and K // 4 <= c1 <= K // 2 and K // 2 <= c2 <= 3 * K // 4
        if kind == "uniform" and pa != pb:
            exchanged.append(np.mean([r != rows0[0] for r in rows0]))
    if kind == "middle":
        assert min(cuts) >= K // 4 and max(cuts) <= 3 * K // 4 and len(set(cuts)) == 3 * K // 4 - K // 4 + 1
    if kind == "uniform":
        assert abs(np.mean(exchanged) - 0.5) < 0.1


def test_swap_mutation_exchanges_two_doses():
    N, K = 60, 8
    rng = np.random.default_rng(6)
    dose = rng.choice([0.5, 1.0, 1.5, 2.0, 2.5], size=(N, K)).astype(np.float32)
    gap = np.tile((np.arange(N)[:, None] % 10 + 1) * 6, (1, K)).astype(np.int32)  # delays name the parent
    nd, ng = ga.next_generation(dose, gap, np.zeros(N), 1, 4, dict(ALPHA, cap=1e6), n_elite=0, k=1, p_cross=0.0,
                                p_mut=1.0, mutation=("swap",))
    swapped = 0
    for c in range(N // 2):
        for t, ch in ((0, 2 * c), (1, 2 * c + 1)):
            src = (ga._words(c, 1, t, 4)[0] * N) >> 32
            assert np.array_equal(ng[ch], gap[src])
            diff = np.nonzero(nd[ch] != dose[src])[0]
            assert len(diff) in (0, 2) and sorted(nd[ch]) == sorted(dose[src])
            swapped += len(diff) == 2
    assert swapped > N // 2


def test_raise_mutation_lifts_one_dose_then_the_guard_holds_the_cap():
    N, K = 60, 8
    dose = np.full((N, K), 1.0, np.float32)
    gap = np.full((N, K), 12, np.int32)
    nd, _ = ga.next_generation(dose, gap, np.zeros(N), 3, 9, dict(ALPHA, cap=1e6), n_elite=0, k=1, p_cross=0.0,
                               p_mut=1.0, mutation=("raise",))
    for row in nd:
        up = np.nonzero(row != 1.0)[0]
        assert len(up) == 1 and row[up[0]] in (1.5, 2.0, 2.5)
    tight = dict(ALPHA, cap=8.5)
    nd, _ = ga.next_generation(dose, gap, np.zeros(N), 3, 9, tight, n_elite=0, k=1, p_cross=0.0, p_mut=1.0,
                               mutation=("raise",))
    assert np.all(nd.astype(np.float64).sum(1) <= 8.5 + 1e-9) and np.any(nd > 1.0)
