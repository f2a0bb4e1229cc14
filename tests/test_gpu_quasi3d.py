"""The quasi-3D variant (C cell slots per site) against the oracle and the 2D
kernels, through the C ABI (needs an MI355X).

With one slot per site the variant's arithmetic is the 2D kernels' operation
for operation, so trajectories and states equal gga_simulate's bit for bit,
with every option.  With several slots, single steps from grown oracle states
match the oracle (fields within 1e-5, cell words exactly outside the counted
near-threshold sites, all slots of a counted site excluded), and whole
trajectories match over their certain prefix.
"""
import copy

import numpy as np
import pytest
import torch

from oracle import protocol, quasi3d, sim
from oracle.model import PROLIF, QUIESC, Params
from parity_helpers import (FIELD_RTOL, MAX_COUNTED_FRACTION, dilate, field_error, from_field_units,
                            near_oxygen_edge, near_threshold, to_field_units)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gga():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2303_08123_amd as g
    return g


def _dev(*arrays):
    return [torch.from_numpy(np.ascontiguousarray(a)).cuda() for a in arrays]


def with_options(md, **kw):
    d = copy.deepcopy(md)
    d.update(kw)
    return d


OPTIONS = {
    "plain": ({}, False),
    "half_repair": ({"repair_half_time": 2.0}, True),
    "oxygen": ({"oer_max": 3.0, "oer_k": 0.1, "kappa": [4.0e-3, 2.0e-3, 2.0e-3]}, False),
    "mitotic_half": ({"mitotic_death": 1}, True),
}


def protocols(half):
    dose = np.array([[2.0, 3.0, 1.5, 2.5], [4.0, 4.0, 0.0, 0.0], [30.0, 0.0, 0.0, 0.0]], np.float32)
    gap = np.array([[20, 9, 13, 7], [30, 24, 0, 0], [0, 0, 0, 0]], np.int32)
    if half:
        gap[0] = [41, 17, 25, 15]
        gap[1] = [61, 47, 0, 0]
    nfrac = np.array([4, 2, 1], np.int32)             # the last breaks the 20 Gy cap
    return dose, gap, nfrac


@pytest.mark.parametrize("L", [64, 128])
@pytest.mark.parametrize("name", list(OPTIONS))
def test_one_slot_equals_the_2d_kernel(gga, model_dict, L, name):
    opts, half = OPTIONS[name]
    md = with_options(model_dict, **opts)
    H, R = 110, 3
    print(f"quasi-3D C=1 vs 2D L={L} {name}", flush=True)
    dose, gap, nfrac = protocols(half)
    dd = _dev(dose, gap, nfrac)
    cfg = gga.make_cfg(L, H, R, seed=11, dose_cap=20.0, half_hour=half)
    live2, fit2, tr2 = gga.simulate(md, cfg, *dd, traj=True)
    live3, fit3, tr3 = gga.simulate_q3(md, cfg, 1, *dd, traj=True)
    torch.cuda.synchronize()
    assert torch.equal(live2, live3) and torch.equal(tr2[:2], tr3[:2])
    assert (live3[2] == -1).all() and (tr3[2] == -1).all() and torch.isnan(fit3[2])
    assert torch.equal(fit2[:2], fit3[:2])
    assert len(set(tr3[0, 0].tolist())) > 20                   # a growing, irradiated tumour
    # stepping a state: the same words and fields as the 2D kernel
    f2, c2 = gga.state_init(md, cfg, 3)
    f3, c3 = gga.q3_init(md, cfg, 1, 3)
    assert torch.equal(f2, f3) and torch.equal(c2, c3[:, 0])
    gga.state_run(md, cfg, *dd, 0, 60, f2, c2)
    gga.q3_run(md, cfg, 1, *dd, 0, 60, f3, c3)
    torch.cuda.synchronize()
    assert torch.equal(f2[:6], f3[:6]) and torch.equal(c2[:6], c3[:6, 0])
    # invalid protocols leave their states untouched
    f0, c0 = gga.q3_init(md, cfg, 1, 3)
    assert torch.equal(f3[6:], f0[6:]) and torch.equal(c3[6:], c0[6:])


def site_live(cells):
    """PROLIF at sites with any live slot: the 2D live map of the helpers."""
    st = cells & 3
    return np.where(((st == PROLIF) | (st == QUIESC)).any(axis=0), PROLIF, 0)


def q3_step_detail(fields, cells, n, thr, thr_mid, p, r, seed, prm, substeps):
    """One oracle step; returns (fields, cells, counted-site map)."""
    L = cells.shape[1]
    draw = quasi3d.slot_draw(n, r, p, seed, L)
    c1 = quasi3d.irradiate(cells, thr, draw, prm, fields) if thr is not None else cells
    act = quasi3d.activity(c1, prm)
    edge = np.zeros((L, L), bool)
    if prm.oxygen_effect and thr is not None:
        edge |= near_oxygen_edge(fields, site_live(cells), prm)
    f = fields
    first = substeps // 2 if thr_mid is not None else substeps
    for _ in range(first):
        f = sim.diffuse_substep(f, act, prm)
    if thr_mid is not None:
        if prm.oxygen_effect:
            edge |= near_oxygen_edge(f, site_live(c1), prm)
        c1 = quasi3d.irradiate(c1, thr_mid, quasi3d.slot_draw(sim.MID_STEP | n, r, p, seed, L), prm, f)
        act = quasi3d.activity(c1, prm)
        for _ in range(substeps - first):
            f = sim.diffuse_substep(f, act, prm)
    c2 = quasi3d.cell_update(c1, f, draw, prm)
    return f, c2, near_threshold(f, site_live(c1), prm) | dilate(edge, 2)


STEP_CASES = [(32, 2, "plain", "start"), (32, 4, "half_repair", "mid"), (48, 8, "oxygen", "start"),
              (40, 5, "mitotic_half", "both"), (64, 3, "plain", "none")]


@pytest.mark.parametrize("L,C,name,kind", STEP_CASES)
def test_single_step_against_the_oracle(gga, model_dict, L, C, name, kind):
    opts, half = OPTIONS[name]
    if kind != "start" and kind != "none":
        half = True
    md = with_options(model_dict, **opts)
    prm = Params.from_dict(md)
    R, seed, warm = 2, 4, 90
    print(f"quasi-3D single step L={L} C={C} {name} {kind}", flush=True)
    states = [quasi3d.run_instance(prm, L, C, warm, 10, [], 0, r, seed)[:2] for r in range(R)]
    fields = to_field_units(np.stack([s[0] for s in states]), prm)
    start = from_field_units(fields, prm)
    cells = np.stack([s[1].astype(np.uint16) for s in states])
    assert (((cells & 3) == 1) | ((cells & 3) == 2)).sum(axis=1).max() >= 2      # columns hold several cells
    if kind == "start":
        dose, gap = np.array([[3.0, 2.0]], np.float32), np.array([[warm, 5]], np.int32)
    elif kind == "mid":
        dose, gap = np.array([[3.0, 2.0]], np.float32), np.array([[2 * warm - 5, 6]], np.int32)
    elif kind == "both":
        dose, gap = np.array([[2.0, 1.5, 2.5]], np.float32), np.array([[2 * warm - 4, 4, 1]], np.int32)
    else:
        dose, gap = np.array([[2.0]], np.float32), np.array([[warm + 50]], np.int32)
    nfrac = np.array([dose.shape[1]], np.int32)
    cfg = gga.make_cfg(L, warm + 1, R, seed=seed, dose_cap=20.0, half_hour=half)
    f_d, c_d = _dev(fields, cells.view(np.int16))
    live, _ = gga.q3_run(md, cfg, C, *_dev(dose, gap, nfrac), warm, 1, f_d, c_d)
    ev = protocol.events(dose[0], gap[0], nfrac[0], warm + 1, prm, half_hour=half)
    evh = {(t if half else 2 * t): thr for t, thr in ev}
    if kind != "none":
        assert (2 * warm in evh) or (2 * warm + 1 in evh)
    got_f, got_c = from_field_units(f_d.cpu().numpy(), prm), c_d.cpu().numpy().view(np.uint16)
    live = live.cpu().numpy()
    for r in range(R):
        f_ref, c_ref, counted = q3_step_detail(start[r], cells[r].astype(np.int64), warm, evh.get(2 * warm),
                                               evh.get(2 * warm + 1), 0, r, seed, prm, 10)
        assert field_error(got_f[r], f_ref) <= FIELD_RTOL
        bad = sum(int(((got_c[r, z].astype(np.int64) != c_ref[z]) & ~counted).sum()) for z in range(C))
        assert bad == 0 and counted.mean() <= MAX_COUNTED_FRACTION, (r, bad, counted.mean())
        if not counted.any():
            assert live[0, r] == quasi3d.live_count(c_ref)


def test_trajectories_over_the_certain_prefix(gga, model_dict):
    """Whole runs from the initial state (L = 40, 4 slots, fractions at 30 h
    and 54 h): every step's live count equals the oracle's until the first step
    with a counted site."""
    prm = Params.from_dict(model_dict)
    L, C, R, seed, H = 40, 4, 2, 6, 90
    dose = np.array([[2.5, 2.0]], np.float32)
    gap = np.array([[30, 24]], np.int32)
    nfrac = np.array([2], np.int32)
    cfg = gga.make_cfg(L, H, R, seed=seed, dose_cap=20.0)
    live, fit, traj = gga.simulate_q3(model_dict, cfg, C, *_dev(dose, gap, nfrac), traj=True)
    traj = traj.cpu().numpy()[0]
    ev = dict((2 * t, thr) for t, thr in protocol.events(dose[0], gap[0], 2, H, prm))
    for r in range(R):
        f, c = quasi3d.init_state(prm, L, C, 0, r, seed)
        certain, ref = H, np.zeros(H, np.int64)
        for n in range(H):
            f, c, near = q3_step_detail(f, c, n, ev.get(2 * n), None, 0, r, seed, prm, 10)
            ref[n] = quasi3d.live_count(c)
            if certain == H and near.any():
                certain = n
        assert certain >= 40, certain
        assert np.array_equal(traj[r, :certain], ref[:certain]), r
        if certain == H:
            assert live[0, r].item() == ref[-1]
    assert ref.max() > ref[0] + 50 and len(set(ref.tolist())) > 30


def test_ragged_lattice_and_batch(gga, model_dict):
    """L = 24 (576 sites: a partial block per instance) and 3 x 3 instances
    (not a multiple of the 8 XCDs): the horizon-0 count, and C = 1 against the
    2D oracle's whole trajectories (the oracle's fields in float64 can flip a
    decision, so only its certain prefix is compared)."""
    prm = Params.from_dict(model_dict)
    L, R, seed, H = 24, 3, 8, 50
    dose = np.array([[2.0], [3.0], [0.0]], np.float32)
    gap = np.array([[20], [25], [0]], np.int32)
    nfrac = np.array([1, 1, 0], np.int32)
    dd = _dev(dose, gap, nfrac)
    live0, fit0, _ = gga.simulate_q3(model_dict, gga.make_cfg(L, 0, R, seed=seed), 3, *dd)
    disc = [sim.live_count(sim.init_state(prm, L, p, r, seed)[1]) for p in range(3) for r in range(R)]
    assert live0.cpu().numpy().reshape(-1).tolist() == disc
    live, _, traj = gga.simulate_q3(model_dict, gga.make_cfg(L, H, R, seed=seed), 1, *dd, traj=True)
    traj = traj.cpu().numpy()
    for p in range(3):
        ev = protocol.events(dose[p], gap[p], nfrac[p], H, prm)
        for r in range(R):
            from parity_helpers import oracle_certain_prefix
            ref, certain = oracle_certain_prefix(prm, L, H, 10, ev, p, r, seed)
            assert certain >= 20
            assert np.array_equal(traj[p, r, :certain], ref[:certain]), (p, r)


@pytest.mark.parametrize("substeps,half", [(13, False), (16, False), (20, False), (25, True), (37, False)])
def test_sub_step_counts_and_chunks(gga, model_dict, substeps, half):
    """More sub-steps per hour than one launch of the fused kernel takes at
    the narrow tile (over 10: the wide tile; over 16: several launches per
    run of sub-steps; with the half-hour split 12 + 13): still the 2D kernel's
    results bit for bit at C = 1."""
    L, H, R = 64, 60, 2
    print(f"quasi-3D C=1 vs 2D, {substeps} sub-steps, half={half}", flush=True)
    dose, gap, nfrac = protocols(half)
    dd = _dev(dose, gap, nfrac)
    cfg = gga.make_cfg(L, H, R, seed=21, substeps=substeps, dose_cap=20.0, half_hour=half)
    live2, _, tr2 = gga.simulate(model_dict, cfg, *dd, traj=True)
    live3, _, tr3 = gga.simulate_q3(model_dict, cfg, 1, *dd, traj=True)
    torch.cuda.synchronize()
    assert torch.equal(live2[:2], live3[:2]) and torch.equal(tr2[:2], tr3[:2])
    f2, c2 = gga.state_init(model_dict, cfg, 3)
    f3, c3 = gga.q3_init(model_dict, cfg, 1, 3)
    gga.state_run(model_dict, cfg, *dd, 0, 30, f2, c2)
    gga.q3_run(model_dict, cfg, 1, *dd, 0, 30, f3, c3)
    torch.cuda.synchronize()
    assert torch.equal(f2[:4], f3[:4]) and torch.equal(c2[:4], c3[:4, 0])
