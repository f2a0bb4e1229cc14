"""Pins of the oracle's quasi-3D variant (several cells per site).

Checked against what does not depend on the variant's own code: with one slot
per site it is the 2D model (whole trajectories with every radiobiology option
equal the pinned 2D oracle's); a per-cell loop over the rules on tiny lattices
equals the vectorised update; daughters are as many as winning parents and go
only into free slots; a column of identical cells acts like one 2D cell; and a
lone ready cell places its daughter in its own site with probability
(C - 1) / (5 C - 1), the share of its free places that are there.
"""
import copy
import math

import numpy as np
import pytest

from oracle import protocol, quasi3d, sim
from oracle.model import AGE_MAX, DEAD, EMPTY, PROLIF, QUIESC, Params


def variant_params(md, **kw):
    d = copy.deepcopy(md)
    d.update(kw)
    return Params.from_dict(d)


OPTIONS = [
    ({}, False),
    ({"repair_half_time": 2.0}, True),
    ({"oer_max": 3.0, "oer_k": 0.1, "kappa": [4.0e-3, 2.0e-3, 2.0e-3]}, False),
    ({"mitotic_death": 1}, True),
]


@pytest.mark.parametrize("opts,half", OPTIONS)
def test_one_slot_is_the_2d_model(model_dict, opts, half):
    prm = variant_params(model_dict, **opts)
    L, H, seed = 24, 70, 5
    dose = np.array([2.0, 3.0, 1.5, 2.5], np.float32)
    gap = np.array([20, 9, 13, 7], np.int64) if not half else np.array([41, 17, 25, 15], np.int64)
    ev = protocol.events(dose, gap, 4, H, prm, half_hour=half)
    for p, r in ((0, 0), (3, 1)):
        f2, c2, t2 = sim.run_instance(prm, L, H, 10, ev, p, r, seed, half_hour=half)
        f3, c3, t3 = quasi3d.run_instance(prm, L, 1, H, 10, ev, p, r, seed, half_hour=half)
        assert np.array_equal(t2, t3)
        assert np.array_equal(c2, c3[0])
        assert np.array_equal(f2, f3)
    assert t2.max() > 40 and len(set(t2.tolist())) > 10      # a growing, irradiated tumour


def loop_update(cells, fields, draw, prm):
    """The cell-update rules, one cell at a time."""
    C, L, _ = cells.shape
    snap = [[[int(cells[z, y, x]) for x in range(L)] for y in range(L)] for z in range(C)]
    out = [[[0] * L for _ in range(L)] for _ in range(C)]
    free = lambda y, x: [z for z in range(C) if 0 <= y < L and 0 <= x < L and snap[z][y][x] & 3 == EMPTY]
    proposals = {}
    for z in range(C):
        for y in range(L):
            for x in range(L):
                w = snap[z][y][x]
                st, age, doom = w & 3, (w >> 2) & 255, (w >> 14) & 1
                older = min(age + 1, AGE_MAX)
                if st == EMPTY:
                    continue
                if st == DEAD:
                    out[z][y][x] = 0 if older >= prm.T_lys else DEAD | (older << 2)
                    continue
                O, G, Hf = (float(fields[f][y, x]) for f in range(3))
                if G < prm.th_Gd or O < prm.th_Od or Hf > prm.th_Hd:
                    out[z][y][x] = DEAD
                    continue
                if O < prm.th_Oq or G < prm.th_Gq:
                    out[z][y][x] = QUIESC | (age << 2) | (doom << 14)
                    continue
                out[z][y][x] = PROLIF | (older << 2) | (doom << 14)
                if age < prm.T_min:
                    continue
                idx = (z * L + y) * L + x
                if doom:
                    if prm.mitotic_death and int(draw(np.array([idx]))[3][0]) < prm.T_div:
                        out[z][y][x] = DEAD
                    continue
                places = [(zz, y, x, 4) for zz in free(y, x)]
                for dy, dx, code in ((-1, 0, 2), (0, 1, 3), (1, 0, 0), (0, -1, 1)):
                    places += [(zz, y + dy, x + dx, code) for zz in free(y + dy, x + dx)]
                if not places:
                    continue
                wd = [int(v[0]) for v in draw(np.array([idx]))]
                if wd[3] >= prm.T_div:
                    continue
                k = (wd[0] * len(places)) >> 32
                tz, ty, tx, code = places[k]
                key = ((wd[2] >> 3) << 8) | (code << 5) | z
                proposals.setdefault((tz, ty, tx), []).append((key, (z, y, x)))
    for (tz, ty, tx), lst in proposals.items():
        key, (z, y, x) = min(lst)
        out[tz][ty][tx] = PROLIF
        out[z][y][x] = PROLIF | ((out[z][y][x] >> 14) << 14)
    return np.array(out, np.int64)


@pytest.mark.parametrize("C,seed", [(1, 1), (2, 2), (3, 3), (5, 4)])
def test_vectorised_update_equals_a_per_cell_loop(model_dict, C, seed):
    rng = np.random.default_rng(seed)
    for mitotic in (0, 1):
        prm = variant_params(model_dict, mitotic_death=mitotic, T_min=2, P_div=0.7)
        L = 6
        st = rng.choice([EMPTY, PROLIF, PROLIF, QUIESC, DEAD], (C, L, L))
        cells = sim.pack(st, rng.integers(0, 12, (C, L, L)), (rng.random((C, L, L)) < 0.3) * (st != EMPTY) * mitotic)
        cells[st == EMPTY] = 0
        fields = np.empty((3, L, L))
        fields[0] = rng.uniform(0.5 * prm.th_Od, 2 * prm.th_Oq + 0.1, (L, L))
        fields[1] = rng.uniform(0.5 * prm.th_Gd, 2 * prm.th_Gq + 0.1, (L, L))
        fields[2] = rng.uniform(0, 1.2 * prm.th_Hd, (L, L))
        for n in range(3):
            draw = quasi3d.slot_draw(n, 1, 2, seed, L)
            got = quasi3d.cell_update(cells, fields, draw, prm)
            assert np.array_equal(got, loop_update(cells, fields, draw, prm)), (C, mitotic, n)


def test_daughters_match_winning_parents(model_dict):
    """Over a grown run with 4 slots: every PROLIF cell of age 0 after a step
    either sits in a slot that was EMPTY (a daughter) or was a ready PROLIF
    cell (its parent), as many of each; no slot is ever over-filled."""
    prm = Params.from_dict(model_dict)
    L, C, seed = 20, 4, 7
    fields, cells = quasi3d.init_state(prm, L, C, 0, 0, seed)
    total_births = 0
    for n in range(80):
        f2, c2 = quasi3d.step(fields, cells, n, None, 0, 0, seed, prm, 10)
        st0, st1, age1 = cells & 3, c2 & 3, (c2 >> 2) & 255
        newborn = (st1 == PROLIF) & (age1 == 0)
        daughters = newborn & (st0 == EMPTY)
        parents = newborn & (st0 == PROLIF)
        assert not (newborn & ~daughters & ~parents).any()
        assert int(daughters.sum()) == int(parents.sum())
        total_births += int(daughters.sum())
        fields, cells = f2, c2
    assert total_births > 100
    # the own column fills: some site holds more than one live cell
    live = ((cells & 3) == PROLIF) | ((cells & 3) == QUIESC)
    assert live.sum(axis=0).max() == C


def test_a_column_of_identical_cells_acts_like_one_2d_cell(model_dict):
    prm = Params.from_dict(model_dict)
    L, C = 16, 3
    rng = np.random.default_rng(9)
    plane = sim.pack(rng.choice([EMPTY, PROLIF, QUIESC, DEAD], (L, L)), 0)
    cells = np.stack([plane] * C)
    a3, a2 = quasi3d.activity(cells, prm), sim.activity(plane, prm)
    assert np.allclose(a3, a2, rtol=1e-15, atol=0)
    f = sim.init_state(prm, L, 0, 0, 1)[0]
    f2 = f3 = f
    for _ in range(20):
        f2, f3 = sim.diffuse_substep(f2, a2, prm), sim.diffuse_substep(f3, a3, prm)
    assert np.allclose(f2, f3, rtol=1e-13, atol=1e-15)
    # half the slots EMPTY (activity 0 unless EMPTY sites consume) halves the uptake
    half = np.stack([plane, np.zeros_like(plane)])
    assert np.allclose(quasi3d.activity(half, prm), 0.5 * (a2 + prm.act[EMPTY]), rtol=1e-15)


@pytest.mark.parametrize("C", [2, 4])
def test_daughter_placement_odds(model_dict, C):
    """A lone ready cell (P_div = 1) in slot 0 of the centre site: its free
    places are C - 1 own slots and 4 C in the neighbours, so the daughter lands
    in its own site with probability (C - 1) / (5 C - 1)."""
    prm = variant_params(model_dict, P_div=1.0, T_min=0)
    L = 5
    cells = np.zeros((C, L, L), np.int64)
    cells[0, 2, 2] = sim.pack(PROLIF, 3)
    fields = sim.init_state(prm, L, 0, 0, 1)[0]
    n_trials, own = 4000, 0
    for t in range(n_trials):
        out = quasi3d.cell_update(cells, fields, quasi3d.slot_draw(t, 0, 0, 77, L), prm)
        born = ((out & 3) == PROLIF) & (((out >> 2) & 255) == 0)
        born[0, 2, 2] = False
        assert born.sum() == 1
        own += int(born[:, 2, 2].any())
    q = (C - 1) / (5 * C - 1)
    assert abs(own - n_trials * q) < 4.5 * math.sqrt(n_trials * q * (1 - q)), (own, n_trials * q)


def test_full_neighbourhood_blocks_division(model_dict):
    prm = variant_params(model_dict, P_div=1.0, T_min=0)
    L, C = 3, 2
    cells = sim.pack(np.full((C, L, L), PROLIF), 5)
    fields = sim.init_state(prm, L, 0, 0, 1)[0]
    out = quasi3d.cell_update(cells, fields, quasi3d.slot_draw(0, 0, 0, 3, L), prm)
    assert np.all(out == sim.pack(PROLIF, 6))


def test_invalid_protocols_and_zero_horizon(model_dict):
    prm = Params.from_dict(model_dict)
    dose = np.array([[2.0, 2.0], [30.0, 0.0]], np.float32)
    gap = np.array([[0, 24], [0, 0]])
    live, fit = quasi3d.simulate(prm, 16, 2, 0, 10, 2, 1, dose, gap, [2, 1], 2, 20.0)
    assert live[1].tolist() == [-1, -1] and math.isnan(fit[1])
    disc = sim.live_count(sim.init_state(prm, 16, 0, 0, 1)[1])
    assert live[0].tolist() == [disc, disc]
