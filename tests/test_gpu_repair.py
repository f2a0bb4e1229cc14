"""Incomplete repair between fractions (repair_half_time > 0) against the
oracle, through the C ABI (needs an MI355X): single steps whose fraction
carries unrepaired damage from a fraction before the step range (resident
64 x 64 and 128 x 128 kernels, 256 x 256 slabs, hourly and half-hour
timing), and a trajectory over its certain prefix."""
import copy

import numpy as np
import pytest
import torch

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


def repairing(md, half_time):
    d = copy.deepcopy(md)
    d["kappa"] = [4.0e-3, 2.0e-3, 2.0e-3]
    d["repair_half_time"] = half_time
    return d


@pytest.mark.parametrize("L,variant,half", [(64, None, False), (128, None, False), (64, None, True),
                                            (256, 5, False), (256, 6, True)])
def test_single_step_with_unrepaired_damage(gga, model_dict, L, variant, half):
    md = repairing(model_dict, 2.0)
    prm = Params.from_dict(md)
    R, seed = 2, 7
    warm = {64: 150, 128: 260, 256: 200}[L]
    print(f"repair single step L={L} variant={variant} half={half}", flush=True)
    states = [sim.run_instance(prm, L, warm, 10, [], 0, r, seed)[:2] for r in range(R)]
    fields = to_field_units(np.stack([s[0] for s in states]), prm)
    start = from_field_units(fields, prm)
    cells = np.stack([s[1].astype(np.uint16) for s in states])
    u = 2 if half else 1
    # 3 Gy three hours before the step range, 2.5 Gy at its start (and 1 Gy at
    # its half hour with half-hour timing)
    if half:
        dose = np.array([[3.0, 2.5, 1.0]], np.float32)
        gap = np.array([[u * (warm - 3), u * 3, 1]], np.int32)
    else:
        dose = np.array([[3.0, 2.5]], np.float32)
        gap = np.array([[warm - 3, 3]], np.int32)
    nfrac = np.array([dose.shape[1]], np.int32)
    cfg = gga.make_cfg(L, warm + 1, R, seed=seed, dose_cap=20.0, half_hour=half)
    f_d, c_d = _dev(fields, cells.view(np.int16))
    dd = _dev(dose, gap, nfrac)
    if variant is None:
        live = gga.state_run(md, cfg, *dd, warm, 1, f_d, c_d)[0].cpu().numpy()
    else:
        live = gga.state_run_variant(md, cfg, variant, *dd, warm, 1, f_d, c_d).cpu().numpy()
    ev = dict(protocol.events(dose[0], gap[0], nfrac[0], warm + 1, prm, half_hour=half))
    key = (lambda t: t) if half else (lambda t: 2 * t)
    evh = {key(t): thr for t, thr in ev.items()}
    plain = dict(protocol.events(dose[0], gap[0], nfrac[0], warm + 1, Params.from_dict(repairing(model_dict, 0.0)),
                                 half_hour=half))
    assert ev[u * warm] != plain[u * warm]        # the unrepaired damage changes the thresholds
    got_f, got_c = from_field_units(f_d.cpu().numpy(), prm), c_d.cpu().numpy().view(np.uint16)
    for r in range(R):
        f_ref, c_ref, counted = oracle_step_detail(start[r], cells[r].astype(np.int64), warm, evh.get(2 * warm), 0, r,
                                                   seed, prm, 10, thr_mid=evh.get(2 * warm + 1))
        assert field_error(got_f[r], f_ref) <= FIELD_RTOL
        bad, frac = compare_cells(got_c[r], c_ref, counted)
        assert bad == 0 and frac <= MAX_COUNTED_FRACTION, (r, bad, frac)
        if not counted.any():
            assert live[0, r] == sim.live_count(c_ref)


def test_trajectory_with_incomplete_repair(gga, model_dict):
    """BMI (1.25 Gy, alternately 6 h and 18 h apart) with a 3-hour repair
    half-time on 64 x 64: every step's live count equals the oracle's over the
    certain prefix, and the final counts differ from those without repair."""
    md = copy.deepcopy(model_dict)
    md["repair_half_time"] = 3.0
    prm = Params.from_dict(md)
    L, R, seed, H = 64, 4, 1, 200
    dose = np.full((1, 8), 1.25, np.float32)
    gap = np.array([[0, 6, 18, 6, 18, 6, 18, 6]], np.int32)
    nfrac = np.array([8], np.int32)
    cfg = gga.make_cfg(L, H, R, seed=seed, dose_cap=20.0)
    live, _, traj = gga.simulate(md, cfg, *_dev(dose, gap, nfrac), traj=True)
    traj = traj.cpu().numpy()[0]
    ev = protocol.events(dose[0], gap[0], 8, H, prm)
    for r in range(R):
        ref, certain = oracle_certain_prefix(prm, L, H, 10, ev, 0, r, seed)
        assert certain >= 50, certain
        assert np.array_equal(traj[r, :certain], ref[:certain]), r
    live0, _, _ = gga.simulate(model_dict, cfg, *_dev(dose, gap, nfrac))
    assert not np.array_equal(live.cpu().numpy(), live0.cpu().numpy())
