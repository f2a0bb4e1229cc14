"""Pins of initialisation and unirradiated growth."""
import numpy as np
from scipy.stats import chisquare

from oracle import sim
from oracle.model import PROLIF, Params
from oracle.sim import pack, unpack


def test_seed_spheroid_has_gauss_circle_count(params):
    """Radius-6 disc: N(6) = 113 lattice points (Gauss circle problem)."""
    for L in (64, 128, 30):
        fields, cells = sim.init_state(params, L, 0, 0, 0)
        st, ag = unpack(cells)
        assert np.count_nonzero(st == PROLIF) == 113 == sim.live_count(cells)
        assert np.all(ag[st == PROLIF] < params.A0)
        for f in range(3):
            assert np.all(fields[f] == params.init[f])
        ys, xs = np.nonzero(st == PROLIF)
        assert ys.mean() == L // 2 and xs.mean() == L // 2


def test_initial_ages_are_uniform(params):
    ages = np.concatenate([unpack(sim.init_state(params, 32, p, r, 4)[1])[1][
        unpack(sim.init_state(params, 32, p, r, 4)[1])[0] == PROLIF] for p in range(6) for r in range(6)])
    counts = np.bincount(ages, minlength=params.A0)
    assert len(counts) == params.A0 and chisquare(counts).pvalue > 1e-3


def _no_environment(params):
    d = dict(params.__dict__)
    d.update(th_Oq=-1.0, th_Gq=-1.0, th_Od=-1.0, th_Gd=-1.0, th_Hd=1e30)
    return Params(**d)


def test_unirradiated_growth_without_environment_never_shrinks(params):
    p2 = _no_environment(params)
    _, _, traj = sim.run_instance(p2, 48, 150, 10, [], 0, 0, 1)
    assert np.all(np.diff(traj) >= 0) and traj[-1] > 2 * 113


def test_isolated_cell_first_division_is_geometric(params):
    """One PROLIF cell of age 0 on an open lattice first divides at step
    T_min + G, G ~ Geometric(P_div) on {0, 1, ...} (it ages one hour per step)."""
    p2 = _no_environment(params)
    L = 5
    firsts = []
    for r in range(1500):
        cells = np.zeros((L, L), np.int64)
        cells[2, 2] = pack(PROLIF, 0)
        fields = np.stack([np.ones((L, L)), np.ones((L, L)), np.zeros((L, L))])
        for n in range(60):
            fields, cells = sim.step(fields, cells, n, None, 0, r, 77, p2, 1)
            if sim.live_count(cells) == 2:
                firsts.append(n)
                break
    firsts = np.array(firsts)
    assert firsts.min() >= params.T_min
    j = firsts - params.T_min
    bins = 10
    obs = np.bincount(np.minimum(j, bins), minlength=bins + 1)
    q = params.P_div
    pmf = np.array([(1 - q) ** i * q for i in range(bins)] + [(1 - q) ** bins])
    exp = pmf * len(firsts) * (len(j) / len(firsts))
    assert len(firsts) >= 1490
    assert chisquare(obs, exp * obs.sum() / exp.sum()).pvalue > 1e-3
