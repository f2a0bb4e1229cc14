"""One generation of the surrogate-screened GA, with the screen replaced by
random keys (the variant the oracle can reproduce; the surrogate's own
arithmetic is checked against oracle/mlp.py separately).

Test infrastructure: part of the CPU oracle (see oracle/__init__.py).

Generation g from a population (dose, gap) of N protocols with simulated
fitness f: breed C candidates (GA operators, no elites); key candidate i by
Philox block (i, g, 0x53435245, 0) word w0 >> 8 (as a float); keep the S
smallest keys (ties by index); simulate those S as members of population g + 1
(run seed seed + (g + 1) * 0x9E3779B97F4A7C15 mod 2^64, the key the plain GA
gives population g + 1; the initial population is population 0), protocol
index = their rank 0..S-1;
keep the N best of the N + S protocols by (fitness, index), index running over
the population first.
"""
import numpy as np

from . import ga
from .philox import philox4x32_10
from .protocol import events
from .sim import run_instance

SCREEN_TAG = 0x53435245
W64 = 0x9E3779B97F4A7C15


def random_keys(C, generation, seed):
    w0 = philox4x32_10(np.arange(C), generation, SCREEN_TAG, 0, seed & 0xFFFFFFFF, (seed >> 32) & 0xFFFFFFFF)[0]
    return (w0 >> np.uint32(8)).astype(np.float32)


def simulate_fitness(params, L, horizon, substeps, R, seed, dose, gap):
    """Mean final live count over R replicas of each row (all fractions used)."""
    P, K = dose.shape
    fit = np.zeros(P, np.float32)
    for p in range(P):
        ev = events(dose[p], gap[p], K, horizon, params)
        fit[p] = np.float32(np.mean([run_instance(params, L, horizon, substeps, ev, p, r, seed)[2][-1]
                                     for r in range(R)]))
    return fit


def generation_random_screen(params, L, horizon, substeps, R, run_seed, dose, gap, fitness, g, ga_seed,
                             alphabet, k, p_cross, p_mut, C, S):
    """Returns the kept (dose, gap, fitness), N rows sorted by (fitness, index)."""
    N, K = dose.shape
    cd, cg = ga.next_generation(dose, gap, fitness, g, ga_seed, alphabet, 0, k, p_cross, p_mut, n_out=C)
    keys = random_keys(C, g, ga_seed)
    pick, _ = ga.rank_order(keys)
    nd, ng = cd[pick[:S]], cg[pick[:S]]
    nf = simulate_fitness(params, L, horizon, substeps, R, (run_seed + (g + 1) * W64) % 2**64, nd, ng)
    all_d = np.concatenate([dose, nd])
    all_g = np.concatenate([gap, ng])
    all_f = np.concatenate([np.asarray(fitness, np.float32), nf])
    order, _ = ga.rank_order(all_f)
    keep = order[:N]
    return all_d[keep], all_g[keep], all_f[keep]
