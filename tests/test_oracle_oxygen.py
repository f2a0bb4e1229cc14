"""Pins of the oracle's oxygen effect on radiosensitivity (oer_max > 1): the
dose a cell sees is scaled by the oxygen modification factor of its oxygen
bin.  Checked against the limits and the half-effect point of the oxygen
enhancement law, the bin edges, the plain law when the effect is off,
monotonicity in oxygen, and binomial survivors through the simulation step
in a lattice with a hypoxic and a well-oxygenated half."""
import copy
import math

import numpy as np

from oracle import sim
from oracle.model import DEAD, OER_BINS, PROLIF, Params
from oracle.protocol import (events, lq_survival, lq_threshold, oxygen_bin, oxygen_modification,
                             oxygen_thresholds)
from oracle.sim import pack, unpack


def oxic(md, oer_max=3.0, oer_k=0.05):
    d = copy.deepcopy(md)
    d["oer_max"], d["oer_k"] = oer_max, oer_k
    return Params.from_dict(d)


def test_no_oxygen_effect_is_the_plain_law(model_dict, params):
    assert not params.oxygen_effect
    p1 = oxic(model_dict, oer_max=1.0)
    assert not p1.oxygen_effect
    for b in range(OER_BINS):
        assert oxygen_modification(b, p1) == 1.0
    tab = oxygen_thresholds(2.0, 0.5, oxic(model_dict, oer_max=1.0))
    for c in range(4):
        assert tab[c] == [lq_threshold(2.0, params.m[c], params.alpha, params.beta, 0.5)] * OER_BINS


def test_limits_and_half_effect_point(model_dict):
    m = 2.8
    # a tiny K: even the first bin is well oxygenated; a huge K: every bin is anoxic
    p = oxic(model_dict, oer_max=m, oer_k=1e-9)
    assert math.isclose(oxygen_modification(OER_BINS - 1, p), 1.0, rel_tol=1e-7)
    p = oxic(model_dict, oer_max=m, oer_k=1e9)
    assert math.isclose(oxygen_modification(0, p), 1.0 / m, rel_tol=1e-7)
    # at O = K the effect is half way: OMF = (m + 1) / (2 m)
    b = 5
    K = (b + 0.5) * float(p.ghost[0]) / OER_BINS
    p = oxic(model_dict, oer_max=m, oer_k=K)
    assert math.isclose(oxygen_modification(b, p), (m + 1) / (2 * m), rel_tol=1e-15)


def test_survival_rises_as_oxygen_falls(model_dict):
    p = oxic(model_dict)
    tab = oxygen_thresholds(2.5, 0.0, p)
    for c in range(4):
        assert all(tab[c][b] > tab[c][b + 1] for b in range(OER_BINS - 1))
        # the oxic bin's survival lies above the plain law's (OMF < 1 at the midpoint)
        assert tab[c][-1] >= lq_threshold(2.5, p.m[c], p.alpha, p.beta)


def test_oxygen_bins_at_their_edges(model_dict):
    p = oxic(model_dict)
    ref = float(p.ghost[0])
    assert oxygen_bin(0.0, p) == 0 and oxygen_bin(ref, p) == OER_BINS - 1 and oxygen_bin(2 * ref, p) == OER_BINS - 1
    for b in range(1, OER_BINS):
        edge = b * ref / OER_BINS
        assert oxygen_bin(edge, p) == b and oxygen_bin(np.nextafter(edge, 0.0), p) == b - 1


def test_hypoxic_cells_survive_more(model_dict):
    """Young proliferating cells fill a lattice whose left half sits at O in
    bin 1 and right half in bin 14; one 3 Gy fraction: each half's survivors
    follow the binomial law of its bin's dose-modified survival."""
    p = oxic(model_dict)
    L = 100
    cells = pack(np.full((L, L), PROLIF), np.full((L, L), 1))
    fields = np.empty((3, L, L))
    for f in range(3):
        fields[f] = p.init[f]
    ref = float(p.ghost[0])
    fields[0][:, :L // 2] = 1.5 * ref / OER_BINS
    fields[0][:, L // 2:] = 14.5 * ref / OER_BINS
    ev = events(np.float32([3.0]), np.int32([0]), 1, 1, p)
    out = sim.irradiate(cells, ev[0][1], lambda s: sim.site_words(s, 0, 0, 0, 3), p, fields)
    alive = unpack(out)[0] != DEAD
    m0 = p.m[0]
    for half, b in ((alive[:, :L // 2], 1), (alive[:, L // 2:], 14)):
        o = (b + 0.5) * ref / OER_BINS
        omf = (p.oer_max * o + p.oer_k) / (p.oer_max * (o + p.oer_k))
        s = lq_survival(3.0 * omf, m0, p.alpha, p.beta)
        n = half.size
        assert abs(int(half.sum()) - n * s) < 4.5 * math.sqrt(n * s * (1 - s)), (b, int(half.sum()), n * s)
    assert alive[:, :L // 2].mean() > alive[:, L // 2:].mean() + 0.05
