"""Pins of the oracle's synchronous cell update: a rule table for single sites,
exhaustive brute force on tiny lattices against a scalar pull-style reference
written from the rules, and per-step count balance."""
import itertools

import numpy as np
import pytest

from oracle import sim
from oracle.model import AGE_MAX, DEAD, EMPTY, PROLIF, QUIESC
from oracle.sim import cell_update, pack, unpack

NB = ((-1, 0), (0, 1), (1, 0), (0, -1))  # N, E, S, W as (dy, dx)


def scalar_reference(cells, fields, words, params):
    """One step of the rules, site by site, resolving divisions from each free
    target's point of view (pull) instead of scattering proposals (push)."""
    H, W = cells.shape
    st = [[int(cells[y, x]) & 3 for x in range(W)] for y in range(H)]
    ag = [[(int(cells[y, x]) >> 2) & 0xFF for x in range(W)] for y in range(H)]

    def env(y, x):
        O, G, Hh = fields[0][y, x], fields[1][y, x], fields[2][y, x]
        if G < params.th_Gd or O < params.th_Od or Hh > params.th_Hd:
            return DEAD
        if O < params.th_Oq or G < params.th_Gq:
            return QUIESC
        return PROLIF

    def free_dirs(y, x):
        out = []
        for d, (dy, dx) in enumerate(NB):
            yy, xx = y + dy, x + dx
            if 0 <= yy < H and 0 <= xx < W and st[yy][xx] == EMPTY:
                out.append(d)
        return out

    def proposal(y, x):
        """Target (ty, tx) and key of the cell at (y, x), or None."""
        if st[y][x] not in (PROLIF, QUIESC) or env(y, x) != PROLIF or ag[y][x] < params.T_min:
            return None
        fd = free_dirs(y, x)
        if not fd:
            return None
        w0, _, w2, w3 = (int(v) for v in words[:, y * W + x])
        if w3 >= params.T_div:
            return None
        d = fd[(w0 * len(fd)) >> 32]
        ty, tx = y + NB[d][0], x + NB[d][1]
        back = (d + 2) % 4          # direction of (y, x) seen from the target
        return ty, tx, ((w2 >> 3) << 2) | back

    new = np.zeros((H, W), dtype=np.int64)
    for y in range(H):
        for x in range(W):
            s, a = st[y][x], ag[y][x]
            if s == EMPTY:
                best = None
                for d, (dy, dx) in enumerate(NB):
                    yy, xx = y + dy, x + dx
                    if 0 <= yy < H and 0 <= xx < W:
                        pr = proposal(yy, xx)
                        if pr is not None and pr[:2] == (y, x):
                            best = pr[2] if best is None else min(best, pr[2])
                new[y, x] = pack(PROLIF, 0) if best is not None else 0
            elif s == DEAD:
                a2 = min(a + 1, AGE_MAX)
                new[y, x] = 0 if a2 >= params.T_lys else pack(DEAD, a2)
            else:
                e = env(y, x)
                if e == DEAD:
                    new[y, x] = pack(DEAD, 0)
                elif e == QUIESC:
                    new[y, x] = pack(QUIESC, a)
                else:
                    pr = proposal(y, x)
                    won = False
                    if pr is not None:
                        ty, tx, key = pr
                        rivals = []
                        for dy, dx in NB:
                            yy, xx = ty + dy, tx + dx
                            if 0 <= yy < H and 0 <= xx < W:
                                q = proposal(yy, xx)
                                if q is not None and q[:2] == (ty, tx):
                                    rivals.append(q[2])
                        won = key == min(rivals)
                    new[y, x] = pack(PROLIF, 0 if won else min(a + 1, AGE_MAX))
    return new


def forced(words):
    return lambda sites: words[:, np.asarray(sites)]


KINDS = [(EMPTY, 0), (PROLIF, 3), (PROLIF, 20), (QUIESC, 30), (DEAD, 23), (DEAD, 4)]


def _good_fields(H, W):
    return np.stack([np.full((H, W), 0.9), np.full((H, W), 0.9), np.full((H, W), 0.1)])


@pytest.mark.parametrize("shape", [(2, 2), (1, 4), (4, 1)])
def test_exhaustive_tiny_lattices(params, shape, rng):
    H, W = shape
    n = H * W
    checked = 0
    for combo in itertools.product(range(len(KINDS)), repeat=n):
        st = np.array([KINDS[k][0] for k in combo]).reshape(H, W)
        ag = np.array([KINDS[k][1] for k in combo]).reshape(H, W)
        cells = pack(st, ag)
        for trial in range(3):
            words = rng.integers(0, 2**32, size=(4, n), dtype=np.uint64)
            if trial == 0:
                words[3] = 0                    # everybody ready
            if trial == 1:                      # equal top bits: direction breaks ties
                words[2] = words[2, 0]
                words[3] = 0
            fields = _good_fields(H, W)
            got = cell_update(cells, fields, forced(words), params)
            ref = scalar_reference(cells, fields, words, params)
            assert np.array_equal(got, ref), (combo, trial)
            checked += 1
    assert checked == 3 * len(KINDS) ** n


def test_random_3x3_and_5x5_with_environment(params, rng):
    for trial in range(400):
        H = W = 3 if trial < 300 else 5
        st = rng.integers(0, 4, size=(H, W))
        ag = rng.integers(0, 40, size=(H, W))
        cells = pack(st, ag)
        fields = np.stack([rng.uniform(0, 1, (H, W)), rng.uniform(0, 1, (H, W)), rng.uniform(0, 1, (H, W))])
        words = rng.integers(0, 2**32, size=(4, H * W), dtype=np.uint64)
        if trial % 2:
            words[3] = rng.integers(0, 2**31, size=H * W)
        got = cell_update(cells, fields, forced(words), params)
        assert np.array_equal(got, scalar_reference(cells, fields, words, params)), trial


@pytest.mark.parametrize("O,G,H,expect", [
    (0.9, 0.9, 0.1, PROLIF),
    (0.19, 0.9, 0.1, QUIESC),   # low oxygen
    (0.9, 0.19, 0.1, QUIESC),   # low glucose
    (0.019, 0.9, 0.1, DEAD),    # anoxia
    (0.9, 0.049, 0.1, DEAD),    # glucose starvation
    (0.9, 0.9, 0.91, DEAD),     # acidity
    (0.2, 0.2, 0.9, PROLIF),    # strict comparisons at the thresholds
    (0.02, 0.05, 0.9, QUIESC),
])
@pytest.mark.parametrize("start", [PROLIF, QUIESC])
def test_environment_rule_table(params, O, G, H, expect, start):
    """Single isolated live site (no free neighbours on a 1x1 lattice)."""
    O, G, H = (float(np.float32(v)) for v in (O, G, H))
    cells = pack(np.array([[start]]), np.array([[15]]))
    fields = np.array([[[O]], [[G]], [[H]]])
    new = cell_update(cells, fields, forced(np.zeros((4, 1), np.uint64)), params)
    st, ag = unpack(new)
    assert st[0, 0] == expect
    want_age = {PROLIF: 16, QUIESC: 15, DEAD: 0}[expect]
    assert ag[0, 0] == want_age


def test_dead_cells_age_then_lyse(params):
    cells = pack(np.array([[DEAD, DEAD, DEAD]]), np.array([[0, params.T_lys - 2, params.T_lys - 1]]))
    new = cell_update(cells, _good_fields(1, 3), forced(np.zeros((4, 3), np.uint64)), params)
    st, ag = unpack(new)
    assert list(st[0]) == [DEAD, DEAD, EMPTY] and list(ag[0]) == [1, params.T_lys - 1, 0]


def test_ages_saturate(params):
    cells = pack(np.array([[PROLIF]]), np.array([[AGE_MAX]]))
    new = cell_update(cells, _good_fields(1, 1), forced(np.zeros((4, 1), np.uint64)), params)
    assert unpack(new)[1][0, 0] == AGE_MAX


def _step_with_accounting(fields, cells, n, thr, p, r, seed, params):
    """One oracle step, also returning (RT kills, necrosis, births)."""
    from oracle.philox import site_words
    draw = lambda s: site_words(s, n, r, p, seed)
    st0, _ = unpack(cells)
    live0 = (st0 == PROLIF) | (st0 == QUIESC)
    c1 = sim.irradiate(cells, thr, draw, params) if thr is not None else cells
    st1, _ = unpack(c1)
    kills = int(np.count_nonzero(live0 & (st1 == DEAD)))
    act = sim.activity(c1, params)
    f = fields
    for _ in range(10):
        f = sim.diffuse_substep(f, act, params)
    c2 = sim.cell_update(c1, f, draw, params)
    st2, _ = unpack(c2)
    live1 = (st1 == PROLIF) | (st1 == QUIESC)
    necro = int(np.count_nonzero(live1 & (st2 == DEAD)))
    births = int(np.count_nonzero((st1 == EMPTY) & (st2 == PROLIF)))
    return f, c2, kills, necro, births


def test_count_balance_over_a_trajectory(params):
    """n(t+1) = n(t) + births - RT kills - necrosis, every step; one cell per site;
    every birth has exactly one winning parent whose age restarts."""
    from oracle.protocol import lq_threshold
    L = 40
    fields, cells = sim.init_state(params, L, 0, 0, 3)
    thr = [lq_threshold(2.0, params.m[c], params.alpha, params.beta) for c in range(4)]
    n = sim.live_count(cells)
    tot_births = 0
    for step in range(120):
        fields, new, kills, necro, births = _step_with_accounting(
            fields, cells, step, thr if step in (30, 60) else None, 0, 0, 3, params)
        st_old, ag_old = unpack(cells)
        st_new, ag_new = unpack(new)
        n_new = sim.live_count(new)
        assert n_new == n + births - kills - necro
        # winners: PROLIF before and after whose age restarted at 0
        restarted = np.count_nonzero((st_old == PROLIF) & (st_new == PROLIF) & (ag_new == 0) & (ag_old >= params.T_min))
        if not (step in (30, 60)):
            assert restarted == births
        tot_births += births
        n, cells = n_new, new
    assert tot_births > 50
