"""Helpers for comparing the HIP path with the oracle.

Parity regime for one step from identical state: float32 fields within 1e-5
relative (floored at 1e-3); cell words equal except at *counted* sites.  A site
is counted when the oracle sees one of the field values it compares (live
sites only) within 4e-5 * max(|theta|, 1e-3) of that threshold, or lies within
Manhattan distance 2 of such a site (a flipped site changes its own proposal,
its target's winner and so that target's other proposers).  Irradiation and
division decisions are integer comparisons and are never counted.
"""
import numpy as np

from oracle import sim
from oracle.model import PROLIF, QUIESC
from oracle.philox import site_words

FIELD_RTOL = 1e-5
FIELD_FLOOR = 1e-3
WINDOW = 4e-5
MAX_COUNTED_FRACTION = 1e-3


def field_units(prm):
    """(g, rho) of the HIP path's field representation: its state buffers hold
    c^ = (c - g_f) / rho_f with g_f the Dirichlet boundary value and
    rho_f = kappa'_f / kappa'_O, kappa' = (-kappa_O, -kappa_G, +kappa_H)."""
    k = np.array(prm.kappa, np.float64)
    kp = np.array([-k[0], -k[1], k[2]])
    return np.array(prm.ghost, np.float64).reshape(3, 1, 1), (kp / kp[0]).reshape(3, 1, 1)


def to_field_units(fields, prm):
    """Physical fields [..., 3, L, L] -> the HIP path's float32 representation."""
    g, rho = field_units(prm)
    return ((np.asarray(fields, np.float64) - g) / rho).astype(np.float32)


def from_field_units(fields, prm):
    """The HIP path's representation -> physical fields, float64."""
    g, rho = field_units(prm)
    return np.asarray(fields, np.float64) * rho + g


def field_error(got, ref):
    return float(np.max(np.abs(got.astype(np.float64) - ref) / np.maximum(np.abs(ref), FIELD_FLOOR)))


def near_threshold(fields, cells, params, window=WINDOW, radius=2, abs_window=0.0):
    """Boolean map of counted sites for a cell update that sees `fields` (after
    diffusion) and the snapshot `cells` (after irradiation).  `abs_window`
    widens the window to an absolute floor where the test's own field bound
    is absolute."""
    st, _ = sim.unpack(cells)
    live = (st == PROLIF) | (st == QUIESC)
    O, G, H = fields
    near = np.zeros(cells.shape, dtype=bool)
    for f, th in ((O, params.th_Od), (O, params.th_Oq), (G, params.th_Gd), (G, params.th_Gq),
                  (H, params.th_Hd)):
        near |= live & (np.abs(f - th) <= max(window * max(abs(th), 1e-3), abs_window))
    return dilate(near, radius)


def dilate(mask, radius):
    """Sites within Manhattan distance `radius` of a marked site."""
    out = mask.copy()
    ys, xs = np.nonzero(mask)
    Hh, W = mask.shape
    for dy in range(-radius, radius + 1):
        for dx in range(-(radius - abs(dy)), radius - abs(dy) + 1):
            yy, xx = ys + dy, xs + dx
            ok = (yy >= 0) & (yy < Hh) & (xx >= 0) & (xx < W)
            out[yy[ok], xx[ok]] = True
    return out


def oracle_step_detail(fields, cells, n, thr, p, r, seed, params, substeps, abs_window=0.0, thr_mid=None):
    """One oracle step (thr_mid: a fraction at the half hour); returns
    (fields, cells, counted-site map)."""
    draw = lambda s: site_words(s, n, r, p, seed)
    c1 = sim.irradiate(cells, thr, draw, params, fields) if thr is not None else cells
    act = sim.activity(c1, params)
    f = fields
    first = substeps // 2 if thr_mid is not None else substeps
    edge = np.zeros(cells.shape, bool)
    if params.oxygen_effect and thr is not None:
        edge |= near_oxygen_edge(fields, cells, params)
    for _ in range(first):
        f = sim.diffuse_substep(f, act, params)
    if thr_mid is not None:
        if params.oxygen_effect:
            edge |= near_oxygen_edge(f, c1, params)
        c1 = sim.irradiate(c1, thr_mid, lambda s: site_words(s, sim.MID_STEP | n, r, p, seed), params, f)
        act = sim.activity(c1, params)
        for _ in range(substeps - first):
            f = sim.diffuse_substep(f, act, params)
    c2 = sim.cell_update(c1, f, draw, params)
    return f, c2, near_threshold(f, c1, params, abs_window=abs_window) | dilate(edge, 2)


def near_oxygen_edge(fields, cells, params, window=WINDOW):
    """Live sites whose oxygen level lies within `window` (relative) of an
    oxygen-bin edge: float32 rounding may put them in the other bin."""
    from oracle.model import OER_BINS
    state = cells & 3
    live = (state == 1) | (state == 2)
    q = fields[0] / float(params.ghost[0]) * OER_BINS
    return live & (np.abs(q - np.round(q)) < window * np.maximum(np.abs(q), 1.0)) & (q > 0.5) & (q < OER_BINS - 0.5)


def oracle_certain_prefix(params, L, nsteps, substeps, ev, p, r, seed, half_hour=False):
    """Oracle trajectory plus the number of leading steps whose outcome no
    float32 rounding can change (no counted site yet); event times in
    half-hours with half_hour."""
    fields, cells = sim.init_state(params, L, p, r, seed)
    evmap = {(t if half_hour else 2 * t): thr for t, thr in ev}
    traj = np.zeros(nsteps, np.int64)
    certain = nsteps
    for n in range(nsteps):
        fields, cells, near = oracle_step_detail(fields, cells, n, evmap.get(2 * n), p, r, seed, params, substeps,
                                                 thr_mid=evmap.get(2 * n + 1))
        traj[n] = sim.live_count(cells)
        if certain == nsteps and near.any():
            certain = n
    return traj, certain


def compare_cells(got, ref, counted):
    """(number of mismatches outside the counted set, counted fraction)."""
    bad = (got.astype(np.int64) != ref.astype(np.int64)) & ~counted
    return int(bad.sum()), float(counted.mean())
