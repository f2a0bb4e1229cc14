"""Pins of the oracle's mitotic (delayed) death (mitotic_death = 1): a
lethally hit cell is marked and lives on until it next becomes ready to
divide, and then dies instead.  Checked against what the rule fixes: nothing
dies at the fraction; marked cells past T_min die at the per-step readiness
rate P_div (binomial), never divide, and stay alive while quiescent; and with
T_min = 0 and P_div = 1 delayed death removes the same cells within the step
as immediate death."""
import copy
import math

import numpy as np

from oracle import sim
from oracle.model import DEAD, DOOM, EMPTY, PROLIF, QUIESC, Params
from oracle.philox import site_words
from oracle.sim import doomed, pack, unpack


def delayed(md, **kw):
    d = copy.deepcopy(md)
    d["mitotic_death"] = 1
    d.update(kw)
    return Params.from_dict(d)


def good_fields(p, L):
    f = np.empty((3, L, L))
    for k in range(3):
        f[k] = p.init[k]
    return f


LETHAL = [0, 0, 0, 0]


def test_nothing_dies_at_the_fraction(model_dict):
    p = delayed(model_dict)
    L = 40
    rng = np.random.default_rng(1)
    cells = pack(rng.choice([PROLIF, QUIESC], (L, L)), rng.integers(0, 40, (L, L)))
    out = sim.irradiate(cells, LETHAL, lambda s: site_words(s, 3, 0, 0, 9), p)
    assert np.array_equal(out & ~DOOM, cells) and np.all(doomed(out) == 1)
    # without the option the same fraction kills every cell at once
    plain = sim.irradiate(cells, LETHAL, lambda s: site_words(s, 3, 0, 0, 9), Params.from_dict(model_dict))
    assert np.all(unpack(plain)[0] == DEAD)


def test_marked_cells_die_at_the_readiness_rate(model_dict):
    """Marked proliferating cells past T_min on a full lattice (no free
    neighbour): each dies in a step with probability P_div."""
    p = delayed(model_dict)
    L = 120
    cells = pack(np.full((L, L), PROLIF), np.full((L, L), p.T_min + 3), np.ones((L, L), np.int64))
    N, q = L * L, p.P_div
    for seed in (1, 2):
        _, out = sim.step(good_fields(p, L), cells, 5, None, 0, 0, seed, p, 2)
        dead = int(np.count_nonzero(unpack(out)[0] == DEAD))
        assert abs(dead - N * q) < 4.5 * math.sqrt(N * q * (1 - q)), (dead, N * q)
        survivors = unpack(out)[0] == PROLIF
        assert np.all(doomed(out)[survivors] == 1) and np.all(doomed(out)[~survivors] == 0)


def test_marked_cells_never_divide(model_dict):
    """A sparse lattice of ready-aged marked cells with free neighbours all
    around: no daughter appears over several steps."""
    p = delayed(model_dict)
    L = 60
    state = np.zeros((L, L), np.int64)
    state[::3, ::3] = PROLIF
    cells = pack(state, np.where(state == PROLIF, p.T_min + 1, 0), (state == PROLIF).astype(np.int64))
    f = good_fields(p, L)
    n0 = int(np.count_nonzero(state == PROLIF))
    for n in range(6):
        f, cells = sim.step(f, cells, n, None, 0, 0, 4, p, 2)
        st = unpack(cells)[0]
        assert np.all(st[state == EMPTY] == EMPTY)          # no daughter anywhere
        assert int(np.count_nonzero(st == PROLIF)) <= n0
    # the unmarked lattice does divide
    plain = Params.from_dict(model_dict)
    f2, c2 = good_fields(p, L), pack(state, np.where(state == PROLIF, p.T_min + 1, 0))
    for n in range(6):
        f2, c2 = sim.step(f2, c2, n, None, 0, 0, 4, plain, 2)
    assert np.count_nonzero(unpack(c2)[0] == PROLIF) > n0


def test_instant_readiness_matches_immediate_death(model_dict):
    """With T_min = 0 and P_div = 1 every marked proliferating cell dies in the
    cell update of the step it was hit: the same live count as immediate death."""
    md = dict(model_dict, T_min=0, P_div=1.0)
    p_late, p_now = delayed(md), Params.from_dict(md)
    L = 80
    rng = np.random.default_rng(3)
    cells = pack(np.full((L, L), PROLIF), rng.integers(0, 10, (L, L)))
    f = good_fields(p_now, L)
    thr = [2**31, 2**31, 2**31, 2**31]               # half the cells are hit
    _, a = sim.step(f, cells, 0, thr, 0, 0, 6, p_late, 2)
    _, b = sim.step(f, cells, 0, thr, 0, 0, 6, p_now, 2)
    assert sim.live_count(a) == sim.live_count(b)
    assert np.array_equal(unpack(a)[0] == DEAD, unpack(b)[0] == DEAD)


def test_quiescent_marked_cells_persist(model_dict):
    """Marked cells held quiescent by low oxygen never reach mitosis: they
    stay alive (and marked) step after step."""
    p = delayed(model_dict)
    L = 30
    cells = pack(np.full((L, L), QUIESC), np.full((L, L), 20), np.ones((L, L), np.int64))
    f = good_fields(p, L)
    f[0][:] = 0.5 * (p.th_Oq + p.th_Od)              # between the quiescence and death thresholds
    c = cells
    for n in range(5):                                 # the cell update alone, at fixed fields
        c = sim.cell_update(c, f, lambda s: site_words(s, n, 0, 0, 2), p)
    assert np.all(unpack(c)[0] == QUIESC) and np.all(doomed(c) == 1)
    # let the oxygen return: they turn proliferative and die at the rate P_div
    f[0][:] = p.init[0]
    c = sim.cell_update(c, f, lambda s: site_words(s, 9, 0, 0, 2), p)
    st = unpack(c)[0]
    assert np.all((st == PROLIF) | (st == DEAD)) and 0 < np.count_nonzero(st == DEAD) < L * L

