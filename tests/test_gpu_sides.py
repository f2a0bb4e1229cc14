"""Lattice sides between the kernel's row pitches of 64, 128 and 256 columns
(96, 160, 192, 224): the lanes past the lattice hold padding sites.  Through
the C ABI against the oracle, against the other variants of the side, and in
one uneven batch of all seven sides 64 .. 256 (needs an MI355X)."""
import copy

import numpy as np
import pytest
import torch

from oracle import protocol, sim
from oracle.model import Params
from paper_2303_08123_amd import workloads
from parity_helpers import (FIELD_RTOL, MAX_COUNTED_FRACTION, compare_cells, field_error, from_field_units,
                            oracle_certain_prefix, oracle_step_detail, to_field_units)

pytestmark = pytest.mark.gpu

DEFAULTS = ((64, 0), (96, 9), (128, 2), (160, 22), (192, 24), (224, 16), (256, 6))


@pytest.fixture(scope="module")
def gga():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2303_08123_amd as g
    yield g
    for L, v in DEFAULTS:
        g.set_variant(L, v)


def _dev(*arrays):
    return [torch.from_numpy(np.ascontiguousarray(a)).cuda() for a in arrays]


def high_uptake(md):
    d = copy.deepcopy(md)
    d["kappa"] = [4.0e-3, 2.0e-3, 2.0e-3]
    return d


def _oracle_init(prm, L, P, R, seed):
    fields, cells = [], []
    for p in range(P):
        for r in range(R):
            f, c = sim.init_state(prm, L, p, r, seed)
            fields.append(to_field_units(f, prm))
            cells.append(c.astype(np.uint16))
    return np.stack(fields), np.stack(cells)


PROTOS = (np.array([[2.0, 3.0, 1.0], [1.5, 0.0, 2.5]], np.float32),
          np.array([[10, 20, 5], [0, 7, 24]], np.int32),
          np.array([3, 3], np.int32))


@pytest.mark.parametrize("L,variant,event", [
    (96, 9, False), (96, 9, True), (96, 10, True), (96, 17, True),
    (160, 11, True), (192, 14, True), (224, 15, False), (224, 15, True), (224, 16, True),
    (160, 18, True), (160, 19, False), (160, 19, True), (192, 20, True), (192, 21, False), (192, 21, True),
    (160, 22, True), (192, 23, True), (192, 24, False), (192, 24, True),
])
def test_single_step_parity(gga, model_dict, L, variant, event):
    """One step from an identical grown state: fields within 1e-5 relative,
    cells bit-exact outside the counted near-threshold set."""
    print(f"single step L={L} variant={variant} event={event}", flush=True)
    md = high_uptake(model_dict)
    prm = Params.from_dict(md)
    # Seed 6: on a 96 x 96 lattice one near-threshold site with its radius-2
    # neighbourhood (13 sites) is 1.4e-3 of the sites, above the regime's
    # 1e-3 cap; under seed 6 no state of these cases has such a site (the
    # oracle alone decides that), so every site is compared bit for bit.
    R, seed, warm = 2, 6, 200
    states = [sim.run_instance(prm, L, warm, 10, [], 0, r, seed)[:2] for r in range(R)]
    fields = to_field_units(np.stack([s[0] for s in states]), prm)
    start = from_field_units(fields, prm)
    cells = np.stack([s[1].astype(np.uint16) for s in states])
    dose, gap, nfrac = (np.array([[2.5]], np.float32), np.array([[warm if event else warm + 5]], np.int32),
                        np.array([1], np.int32))
    cfg = gga.make_cfg(L, warm + 1, R, seed=seed, dose_cap=20.0)
    f_d, c_d = _dev(fields, cells.view(np.int16))
    live = gga.state_run_variant(md, cfg, variant, *_dev(dose, gap, nfrac), warm, 1, f_d, c_d).cpu().numpy()
    got_f, got_c = from_field_units(f_d.cpu().numpy(), prm), c_d.cpu().numpy().view(np.uint16)
    ev = dict(protocol.events(dose[0], gap[0], 1, warm + 1, prm))
    assert (warm in ev) == event
    for r in range(R):
        f_ref, c_ref, counted = oracle_step_detail(start[r], cells[r].astype(np.int64), warm,
                                                   ev.get(warm), 0, r, seed, prm, 10)
        assert field_error(got_f[r], f_ref) <= FIELD_RTOL
        bad, frac = compare_cells(got_c[r], c_ref, counted)
        assert bad == 0 and frac <= MAX_COUNTED_FRACTION
        if not counted.any():
            assert live[0, r] == sim.live_count(c_ref)
    assert ((cells & 3) == 2).any() and ((cells & 3) == 3).any()   # quiescent and dead cells took part


@pytest.mark.parametrize("L,variants", [(96, (9, 10, 17)), (160, (11, 12, 18, 19, 22)), (192, (13, 14, 20, 21, 23, 24)),
                                        (224, (15, 16))])
def test_variants_agree_bit_for_bit(gga, model_dict, L, variants):
    """Resident and slab variants of one side, from one state, over two
    segments of steps: identical fields, cells and counts."""
    print(f"variants L={L} {variants}", flush=True)
    md = high_uptake(model_dict)
    prm = Params.from_dict(md)
    P, R, seed = 2, 2, 13
    f0, c0 = _oracle_init(prm, L, P, R, seed)
    cfg = gga.make_cfg(L, 200, R, seed=seed, dose_cap=100.0)
    states = {}
    for v in variants:
        f_d, c_d = _dev(f0, c0.view(np.int16))
        out = []
        for n0, n in ((0, 50), (50, 150)):              # dead cells at step 50, quiescent ones by 200
            live = gga.state_run_variant(md, cfg, v, *_dev(*PROTOS), n0, n, f_d, c_d)
            out.append((f_d.cpu().numpy().copy(), c_d.cpu().numpy().copy(), live.cpu().numpy()))
        states[v] = out
    for v in variants[1:]:
        for seg_a, seg_b in zip(states[variants[0]], states[v]):
            for a, b in zip(seg_a, seg_b):
                assert np.array_equal(a, b), v
    st50, st200 = (states[variants[0]][k][1].view(np.uint16) & 3 for k in (0, 1))
    assert (st50 == 3).any() and (st200 == 2).any()


@pytest.mark.parametrize("L", [96, 160, 224])
def test_trajectory_matches_oracle(gga, model_dict, L):
    """gga_simulate (resident at 96, slabs through its workspace at 160, with
    three columns per lane, and 224): the
    live count of every step agrees with the oracle's until the oracle first
    meets a near-threshold site."""
    print(f"trajectory L={L}", flush=True)
    prm = Params.from_dict(model_dict)
    R, seed, H = 2, 0, 120
    dose, gap, nfrac = workloads.config1_protocols()
    cfg = gga.make_cfg(L, H, R, seed=seed, dose_cap=20.0)
    assert (gga.workspace_bytes(cfg, 1) > 0) == (L > 128)
    live, fit, traj = gga.simulate(model_dict, cfg, *_dev(dose, gap, nfrac), traj=True)
    traj = traj.cpu().numpy()[0]
    assert np.array_equal(live.cpu().numpy()[0], traj[:, -1])
    ev = protocol.events(dose[0], gap[0], nfrac[0], H, prm)
    for r in range(R):
        ref, certain = oracle_certain_prefix(prm, L, H, 10, ev, 0, r, seed)
        assert certain >= 60, certain
        assert np.array_equal(traj[r, :certain], ref[:certain]), r


@pytest.mark.parametrize("L", [160, 192, 256])
def test_slab_simulate_equals_step_runs(gga, model_dict, L):
    """gga_simulate's slab path equals the same steps run one at a time from
    the oracle's initial state; invalid protocols give -1 / NaN; the
    trajectory's last entry is the final count."""
    print(f"slab simulate L={L}", flush=True)
    md = high_uptake(model_dict)
    prm = Params.from_dict(md)
    P, R, seed, H = 3, 2, 9, 30
    dose = np.array([[2.0, 3.0, 1.0], [1.5, 0.0, 2.5], [-1.0, 1.0, 1.0]], np.float32)
    gap = np.array([[3, 10, 5], [0, 7, 9], [0, 1, 1]], np.int32)
    nfrac = np.array([3, 3, 3], np.int32)
    dd = _dev(dose, gap, nfrac)
    cfg = gga.make_cfg(L, H, R, seed=seed, dose_cap=100.0)
    live, fit, traj = gga.simulate(md, cfg, *dd, traj=True)
    live, fit, traj = live.cpu().numpy(), fit.cpu().numpy(), traj.cpu().numpy()
    f0, c0 = _oracle_init(prm, L, P, R, seed)
    f_d, c_d = _dev(f0, c0.view(np.int16))
    v = gga.get_variant(L)
    steps = np.stack([gga.state_run_variant(md, cfg, v, *dd, n, 1, f_d, c_d).cpu().numpy() for n in range(H)], -1)
    assert np.array_equal(traj[:2], steps[:2]) and np.array_equal(live[:2], steps[:2, :, -1])
    assert np.all(live[2] == -1) and np.isnan(fit[2]) and np.allclose(fit[:2], live[:2].mean(1))


def test_uneven_batch_of_all_seven_sides(gga, model_dict):
    """One uneven call mixing every side 64 .. 256 (resident and slab forms),
    horizons (one of them 0) and fraction counts equals gga_simulate per
    (side, horizon)."""
    md = high_uptake(model_dict)
    P, K, R, seed = 14, 6, 2, 31
    dose, gap, nfrac = workloads.random_protocols(P, K, seed=7, kmin=1)
    lattice = np.array([64, 96, 128, 160, 192, 224, 256] * 2, np.int32)
    horizon = np.array([30, 24, 18, 26, 20, 16, 12, 0, 30, 22, 14, 0, 20, 10], np.int32)
    cfg = gga.make_cfg(64, 0, R, seed=seed, dose_cap=100.0)
    dd = _dev(dose, gap, nfrac)
    live, fit = gga.simulate_uneven(md, cfg, *dd, lattice, horizon)
    live, fit = live.cpu().numpy(), fit.cpu().numpy()
    ref = np.zeros((P, R), np.int64)
    for L, H in sorted(set(zip(lattice.tolist(), horizon.tolist()))):
        rows = np.nonzero((lattice == L) & (horizon == H))[0]
        lv = gga.simulate(md, gga.make_cfg(L, H, R, seed=seed, dose_cap=100.0), *dd)[0].cpu().numpy()
        ref[rows] = lv[rows]
    assert np.array_equal(live, ref)
    assert np.allclose(fit, ref.mean(1))
    assert live[7, 0] == 113 and live[11, 1] == 113            # horizon 0: the seed disc



@pytest.mark.parametrize("L,variant", [(160, 12), (160, 19), (160, 22), (192, 14), (192, 21), (192, 23), (192, 24),
                                       (224, 16), (256, 6)])
def test_teams_equal_one_launch_per_step(gga, model_dict, L, variant):
    """The team form (slabs co-resident for the whole horizon, halo rows
    exchanged through device memory) gives the per-step slab form's results
    bit for bit: live counts, fitness and every step's count."""
    print(f"teams vs per-step L={L} variant={variant}", flush=True)
    gga.set_variant(L, variant)
    md = high_uptake(model_dict)
    P, K, R = 5, 4, 3
    dose, gap, nfrac = workloads.random_protocols(P, K, seed=L, kmin=1)
    dd = _dev(dose, gap, nfrac)
    cfg = gga.make_cfg(L, 40, R, seed=4, dose_cap=100.0)
    out = {}
    try:
        for teams in (True, False):
            gga.set_team_options(teams)
            out[teams] = [x.cpu().numpy() for x in gga.simulate(md, cfg, *dd, traj=True)]
    finally:
        gga.set_team_options(True)
        for side, v in DEFAULTS:
            gga.set_variant(side, v)
    for a, b in zip(out[True], out[False]):
        assert np.array_equal(a, b, equal_nan=True)
    assert np.all(out[True][0] > 0)


@pytest.mark.parametrize("teams", [True, False])
@pytest.mark.parametrize("L", [160, 256])
def test_slab_sides_zero_horizon_empty_batch_and_no_fractions(gga, model_dict, L, teams):
    """Degenerate calls on the slab sides, as teams and one launch per step:
    an empty batch returns empty outputs; a zero-step horizon returns the
    initial disc's count (113 sites within radius 6 of the centre) for valid
    protocols and marks an invalid one (-1 live, NaN fitness); protocols with
    no fraction equal the oracle's unirradiated trajectory."""
    print(f"slab degenerate cases L={L} teams={teams}", flush=True)
    try:
        gga.set_team_options(teams)
        cfg = gga.make_cfg(L, 10, 2, seed=0)
        e = torch.zeros((0, 3), dtype=torch.float32, device="cuda")
        live, fit, _ = gga.simulate(model_dict, cfg, e, e.int(), torch.zeros(0, dtype=torch.int32, device="cuda"))
        assert live.numel() == 0 and fit.numel() == 0
        dose = np.array([[2.0, 0.0], [0.0, 0.0], [30.0, 30.0]], np.float32)
        gap = np.zeros((3, 2), np.int32)
        nfrac = np.array([1, 0, 2], np.int32)                # the last breaks the 20 Gy cap
        live, fit, _ = gga.simulate(model_dict, gga.make_cfg(L, 0, 2, seed=0, dose_cap=20.0), *_dev(dose, gap, nfrac))
        live, fit = live.cpu().numpy(), fit.cpu().numpy()
        assert np.all(live[:2] == 113) and np.all(live[2] == -1)
        assert np.all(fit[:2] == 113.0) and np.isnan(fit[2])
        H = 30
        z = np.zeros((2, 0), np.float32)
        live, fit, traj = gga.simulate(model_dict, gga.make_cfg(L, H, 2, seed=5), *_dev(z, z.astype(np.int32),
                                                                                           np.zeros(2, np.int32)),
                                       traj=True)
        traj = traj.cpu().numpy()
    finally:
        gga.set_team_options(True)
    prm = Params.from_dict(model_dict)
    for p in range(2):
        for r in range(2):
            ref, certain = oracle_certain_prefix(prm, L, H, 10, [], p, r, 5)
            assert certain == H, (p, r, certain)
            assert np.array_equal(traj[p, r], ref), (p, r)



def test_team_uneven_batch_with_slab_choices_everywhere(gga, model_dict):
    """With the slab variants chosen for every side (64, 96 and 128 too), an
    uneven batch run as teams equals the same batch run one launch per step
    and the resident runs of the resident sides."""
    md = high_uptake(model_dict)
    P, K, R, seed = 14, 5, 2, 41
    dose, gap, nfrac = workloads.random_protocols(P, K, seed=8, kmin=1)
    lattice = np.array([64, 96, 128, 160, 192, 224, 256] * 2, np.int32)
    horizon = np.array([20, 18, 16, 14, 12, 10, 8, 0, 20, 1, 2, 14, 3, 9], np.int32)
    cfg = gga.make_cfg(64, 0, R, seed=seed, dose_cap=100.0)
    dd = _dev(dose, gap, nfrac)
    resident = gga.simulate_uneven(md, cfg, *dd, lattice, horizon)[0].cpu().numpy()
    runs = []
    try:
        for L, v in ((64, 1), (96, 17), (128, 4)):
            gga.set_variant(L, v)
        for teams in (True, False):
            gga.set_team_options(teams)
            runs.append(gga.simulate_uneven(md, cfg, *dd, lattice, horizon)[0].cpu().numpy())
    finally:
        gga.set_team_options(True)
        for L, v in DEFAULTS:
            gga.set_variant(L, v)
    assert np.array_equal(runs[0], runs[1]) and np.array_equal(runs[0], resident)


def test_team_wait_that_runs_out_is_reported_and_every_workgroup_exits(gga, model_dict):
    """A team whose bounded wait fails (forced from the host: every wait fails)
    leaves negative live counts and NaN fitness for instances that needed a
    wait (horizon >= 2), correct results for those that did not, and the
    device keeps working: the next call with the default limit is correct."""
    P, K, R = 3, 3, 2
    dose, gap, nfrac = workloads.random_protocols(P, K, seed=5, kmin=1)
    dd = _dev(dose, gap, nfrac)
    cfg = gga.make_cfg(64, 0, R, seed=2, dose_cap=100.0)
    lattice = np.array([256, 224, 160], np.int32)
    horizon = np.array([6, 1, 0], np.int32)
    ref = gga.simulate_uneven(model_dict, cfg, *dd, lattice, horizon)
    try:
        gga.set_team_options(True, -1)
        live, fit = gga.simulate_uneven(model_dict, cfg, *dd, lattice, horizon)
        live, fit = live.cpu().numpy(), fit.cpu().numpy()
    finally:
        gga.set_team_options(True)
    assert np.all(live[0] < 0) and np.isnan(fit[0])
    assert np.array_equal(live[1:], ref[0].cpu().numpy()[1:])
    again = gga.simulate_uneven(model_dict, cfg, *dd, lattice, horizon)
    assert torch.equal(again[0], ref[0])
