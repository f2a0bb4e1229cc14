"""Protocols timed in 30-minute units (GGA_SIM_HALF_HOUR) against the oracle,
through the C ABI (needs an MI355X): even half-hour times reproduce the hourly
protocol bit for bit; single steps with a fraction at the half hour (alone and
after one at the start of the same hour) on the resident 64 x 64 and
128 x 128 kernels and on the 256 x 256 slabs; the trajectory of a protocol
shifted by 30 minutes over its certain prefix; and one generation of the GA
over the paper's 30-minute slot genome."""
import copy

import numpy as np
import pytest
import torch

from oracle import ga_slots as ogs
from oracle import protocol, sim
from oracle.model import Params
from parity_helpers import (FIELD_RTOL, MAX_COUNTED_FRACTION, compare_cells, field_error, from_field_units,
                            oracle_certain_prefix, oracle_step_detail, to_field_units)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gga():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2303_08123_amd as g
    yield g
    for L, v in ((64, 0), (128, 2), (256, 6)):      # the library's defaults
        g.set_variant(L, v)


def _dev(*arrays):
    return [torch.from_numpy(np.ascontiguousarray(a)).cuda() for a in arrays]


def high_uptake(md):
    d = copy.deepcopy(md)
    d["kappa"] = [4.0e-3, 2.0e-3, 2.0e-3]
    return d


@pytest.mark.parametrize("L", [64, 128])
def test_even_half_hours_equal_the_hourly_protocol(gga, model_dict, L):
    rng = np.random.default_rng(L)
    P, K, R, H = 6, 5, 2, 60
    dose = rng.choice(np.float32([0.5, 1.0, 2.0, 3.0]), (P, K)).astype(np.float32)
    gap = rng.integers(1, 14, (P, K)).astype(np.int32)
    gap[:, 0] -= 1                                         # first fraction at t >= 0
    nfrac = np.full(P, K, np.int32)
    out = []
    for half, g in ((False, gap), (True, 2 * gap)):
        cfg = gga.make_cfg(L, H, R, seed=3, dose_cap=100.0, half_hour=half)
        live, fit, traj = gga.simulate(model_dict, cfg, *_dev(dose, g, nfrac), traj=True)
        out.append([x.cpu().numpy() for x in (live, fit, traj)])
    for a, b in zip(*out):
        assert np.array_equal(a, b)


def _steps(L, warm, kind):
    """Protocol of one or two fractions at step `warm`: 'mid' one at its half
    hour, 'both' one at the start and one at the half hour (half-hour units)."""
    if kind == "mid":
        return np.array([[2.5]], np.float32), np.array([[2 * warm + 1]], np.int32), np.array([1], np.int32)
    return (np.array([[1.5, 2.0]], np.float32), np.array([[2 * warm, 1]], np.int32), np.array([2], np.int32))


def _check_step(prm, md, start, cells, got_f, got_c, live, warm, ev, R, seed):
    for r in range(R):
        f_ref, c_ref, counted = oracle_step_detail(start[r], cells[r].astype(np.int64), warm, ev.get(2 * warm),
                                                   0, r, seed, prm, 10, thr_mid=ev.get(2 * warm + 1))
        assert field_error(got_f[r], f_ref) <= FIELD_RTOL
        bad, frac = compare_cells(got_c[r], c_ref, counted)
        assert bad == 0 and frac <= MAX_COUNTED_FRACTION, (r, bad, frac)
        if not counted.any():
            assert live[0, r] == sim.live_count(c_ref)


@pytest.mark.parametrize("L,warm,kind", [(64, 150, "mid"), (64, 150, "both"), (128, 260, "mid"),
                                         (128, 260, "both")])
def test_single_step_with_a_half_hour_fraction(gga, model_dict, L, warm, kind):
    md = high_uptake(model_dict)
    prm = Params.from_dict(md)
    R, seed = 2, 5
    print(f"half-hour single step L={L} {kind}", flush=True)
    states = [sim.run_instance(prm, L, warm, 10, [], 0, r, seed)[:2] for r in range(R)]
    fields = to_field_units(np.stack([s[0] for s in states]), prm)
    start = from_field_units(fields, prm)
    cells = np.stack([s[1].astype(np.uint16) for s in states])
    dose, gap, nfrac = _steps(L, warm, kind)
    cfg = gga.make_cfg(L, warm + 1, R, seed=seed, dose_cap=20.0, half_hour=True)
    f_d, c_d = _dev(fields, cells.view(np.int16))
    live, _ = gga.state_run(md, cfg, *_dev(dose, gap, nfrac), warm, 1, f_d, c_d)
    ev = dict(protocol.events(dose[0], gap[0], nfrac[0], warm + 1, prm, half_hour=True))
    assert (2 * warm + 1) in ev and ((2 * warm) in ev) == (kind == "both")
    _check_step(prm, md, start, cells, from_field_units(f_d.cpu().numpy(), prm), c_d.cpu().numpy().view(np.uint16),
                live.cpu().numpy(), warm, ev, R, seed)


@pytest.mark.parametrize("variant,kind", [(5, "mid"), (6, "both")])
def test_L256_slab_single_step_with_a_half_hour_fraction(gga, model_dict, variant, kind):
    md = high_uptake(model_dict)
    prm = Params.from_dict(md)
    L, R, seed, warm = 256, 2, 5, 200
    print(f"half-hour single step L=256 variant {variant} {kind}", flush=True)
    states = [sim.run_instance(prm, L, warm, 10, [], 0, r, seed)[:2] for r in range(R)]
    fields = to_field_units(np.stack([s[0] for s in states]), prm)
    start = from_field_units(fields, prm)
    cells = np.stack([s[1].astype(np.uint16) for s in states])
    dose, gap, nfrac = _steps(L, warm, kind)
    cfg = gga.make_cfg(L, warm + 1, R, seed=seed, dose_cap=20.0, half_hour=True)
    f_d, c_d = _dev(fields, cells.view(np.int16))
    live = gga.state_run_variant(md, cfg, variant, *_dev(dose, gap, nfrac), warm, 1, f_d, c_d).cpu().numpy()
    ev = dict(protocol.events(dose[0], gap[0], nfrac[0], warm + 1, prm, half_hour=True))
    _check_step(prm, md, start, cells, from_field_units(f_d.cpu().numpy(), prm), c_d.cpu().numpy().view(np.uint16),
                live, warm, ev, R, seed)


def test_trajectory_of_a_half_hour_protocol(gga, model_dict):
    """BMII shifted by 30 minutes (2 Gy at 0.5, 24.5, ..., 96.5 h) on 64 x 64:
    every step's live count equals the oracle's over the certain prefix, and
    the uneven call on 256 x 256 slabs equals its step-by-step run."""
    prm = Params.from_dict(model_dict)
    L, R, seed, H = 64, 4, 0, 240
    dose = np.full((1, 5), 2.0, np.float32)
    gap = np.array([[1, 48, 48, 48, 48]], np.int32)
    nfrac = np.array([5], np.int32)
    cfg = gga.make_cfg(L, H, R, seed=seed, dose_cap=20.0, half_hour=True)
    _, _, traj = gga.simulate(model_dict, cfg, *_dev(dose, gap, nfrac), traj=True)
    traj = traj.cpu().numpy()[0]
    ev = protocol.events(dose[0], gap[0], 5, H, prm, half_hour=True)
    assert [t for t, _ in ev] == [1, 49, 97, 145, 193]
    for r in range(R):
        ref, certain = oracle_certain_prefix(prm, L, H, 10, ev, 0, r, seed, half_hour=True)
        assert certain >= 100, certain
        assert np.array_equal(traj[r, :certain], ref[:certain]), r
    # 256 x 256 slabs: the uneven call equals stepping the same states one step at a time
    L2, H2, R2 = 256, 30, 1
    dose2 = np.array([[2.0, 1.0]], np.float32)
    gap2 = np.array([[3, 18]], np.int32)                   # 1.5 h and 10.5 h
    cfg2 = gga.make_cfg(L2, H2, R2, seed=seed, dose_cap=20.0, half_hour=True)
    dd = _dev(dose2, gap2, np.array([2], np.int32))
    f0, c0 = [], []
    for r in range(R2):
        f, c = sim.init_state(prm, L2, 0, r, seed)
        f0.append(to_field_units(f, prm))
        c0.append(c.astype(np.uint16))
    f_d, c_d = _dev(np.stack(f0), np.stack(c0).view(np.int16))
    steps = np.stack([gga.state_run_variant(model_dict, cfg2, 5, *dd, n, 1, f_d, c_d).cpu().numpy()[0]
                      for n in range(H2)], axis=1)
    live, _ = gga.simulate_uneven(model_dict, cfg2, *dd, [L2], [H2])
    assert np.array_equal(live.cpu().numpy()[0], steps[:, -1])


def test_slot_ga_generation_on_30_minute_slots(gga, model_dict):
    """One generation of the slot GA on 30-minute slots (48 slots = the first
    day, minimal interval 6 h = 12 slots): the device's fitness and next
    population equal the oracle's half-hour simulation and breeding."""
    N, S, K, R, L, H, seed = 10, 48, 4, 2, 64, 30, 9
    rng = np.random.default_rng(2)
    pop = (rng.integers(1, 9, (N, S)) * (rng.random((N, S)) < 0.2)).astype(np.uint8)
    pop = np.array([ogs.guards(v.tolist(), 12, 8, 16) for v in pop], np.uint8)
    cfg = gga.make_cfg(L, H, R, seed=seed, dose_cap=4.0, half_hour=True)
    ga_cfg = gga.make_ga(n_elite=2, tournament_k=3, p_cross=0.8, p_mut=0.5, seed=6, crossover="two_point",
                         mutation=())
    sc = gga.make_slots(S=S, g_min=12, dmax_q=8, cap_q=16)
    nxt, hist, _ = gga.slots_run(model_dict, cfg, ga_cfg, sc, torch.from_numpy(pop).cuda(), K, 1, False)
    prm = Params.from_dict(model_dict)
    fit = np.zeros(N)
    for p, v in enumerate(pop):
        d, g, n = ogs.decode(v.tolist(), np.float32(0.25), K)
        ev = protocol.events(d, g, n, H, prm, half_hour=True)
        fit[p] = np.mean([sim.run_instance(prm, L, H, 10, ev, p, r, seed, half_hour=True)[2][-1]
                          for r in range(R)])
    fit32 = fit.astype(np.float32)
    assert hist.cpu().numpy()[0, 0] == fit32.min()
    want = ogs.next_generation_slots(pop, fit32, 0, 6, 12, 8, 16, 2, 3, 0.8, 0.5, crossover_kind="two_point",
                                     mutations=("swap", "split", "time"))
    assert np.array_equal(nxt.cpu().numpy(), want)
