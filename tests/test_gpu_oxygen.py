"""The oxygen effect on radiosensitivity (oer_max > 1) against the oracle,
through the C ABI (needs an MI355X): single steps with a fraction on
hypoxic, grown tumours (resident 64 x 64 and 128 x 128 kernels, 256 x 256
slabs), also at the half hour and with incomplete repair, and a trajectory
over its certain prefix.  The kernel reads each site's oxygen bin from the
same float32 field the oracle converts exactly, so start-of-step decisions
match bit for bit; later ones exclude sites within rounding of a bin edge."""
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


def oxygenated(md, repair=0.0):
    d = copy.deepcopy(md)
    d["kappa"] = [4.0e-3, 2.0e-3, 2.0e-3]            # hypoxic cores on small lattices
    d["oer_max"], d["oer_k"] = 3.0, 0.1
    d["repair_half_time"] = repair
    return d


CASES = [(64, None, "start", 0.0), (128, None, "start", 0.0), (64, None, "mid", 2.0), (128, None, "both", 1.5),
         (256, 5, "start", 0.0), (256, 6, "both", 2.0)]


@pytest.mark.parametrize("L,variant,kind,repair", CASES)
def test_single_step_with_the_oxygen_effect(gga, model_dict, L, variant, kind, repair):
    md = oxygenated(model_dict, repair)
    prm = Params.from_dict(md)
    R, seed = 2, 3
    warm = {64: 150, 128: 260, 256: 200}[L]
    print(f"oxygen single step L={L} variant={variant} {kind} repair={repair}", flush=True)
    states = [sim.run_instance(prm, L, warm, 10, [], 0, r, seed)[:2] for r in range(R)]
    fields = to_field_units(np.stack([s[0] for s in states]), prm)
    start = from_field_units(fields, prm)
    cells = np.stack([s[1].astype(np.uint16) for s in states])
    half = kind != "start"
    if kind == "start":
        dose, gap = np.array([[2.0, 3.0]], np.float32), np.array([[warm - 4, 4]], np.int32)
    elif kind == "mid":
        dose, gap = np.array([[2.0, 3.0]], np.float32), np.array([[2 * warm - 5, 6]], np.int32)
    else:
        dose, gap = np.array([[2.0, 1.5, 2.5]], np.float32), np.array([[2 * warm - 4, 4, 1]], np.int32)
    nfrac = np.array([dose.shape[1]], np.int32)
    cfg = gga.make_cfg(L, warm + 1, R, seed=seed, dose_cap=20.0, half_hour=half)
    f_d, c_d = _dev(fields, cells.view(np.int16))
    dd = _dev(dose, gap, nfrac)
    if variant is None:
        live = gga.state_run(md, cfg, *dd, warm, 1, f_d, c_d)[0].cpu().numpy()
    else:
        live = gga.state_run_variant(md, cfg, variant, *dd, warm, 1, f_d, c_d).cpu().numpy()
    ev = protocol.events(dose[0], gap[0], nfrac[0], warm + 1, prm, half_hour=half)
    evh = {(t if half else 2 * t): thr for t, thr in ev}
    assert (2 * warm in evh) or (2 * warm + 1 in evh)
    got_f, got_c = from_field_units(f_d.cpu().numpy(), prm), c_d.cpu().numpy().view(np.uint16)
    st = cells[0] & 3
    o = start[0][0][(st == 1) | (st == 2)]
    assert o.min() < 0.6 * float(prm.ghost[0])        # the tumour spans several oxygen bins
    for r in range(R):
        f_ref, c_ref, counted = oracle_step_detail(start[r], cells[r].astype(np.int64), warm, evh.get(2 * warm), 0, r,
                                                   seed, prm, 10, thr_mid=evh.get(2 * warm + 1))
        assert field_error(got_f[r], f_ref) <= FIELD_RTOL
        bad, frac = compare_cells(got_c[r], c_ref, counted)
        assert bad == 0 and frac <= MAX_COUNTED_FRACTION, (r, bad, frac)
        if not counted.any():
            assert live[0, r] == sim.live_count(c_ref)
        # no oxygen-bin bits are left in the cell words
        assert not (got_c[r] & 0xFC00).any()


def test_trajectory_with_the_oxygen_effect(gga, model_dict):
    """BMII on 64 x 64 with oer_max = 3: every step's live count equals the
    oracle's over the certain prefix; the effect changes the outcome."""
    md = copy.deepcopy(model_dict)
    md["oer_max"], md["oer_k"] = 3.0, 0.1
    prm = Params.from_dict(md)
    L, R, seed, H = 64, 4, 2, 240
    dose = np.full((1, 5), 2.0, np.float32)
    gap = np.array([[0, 24, 24, 24, 24]], np.int32)
    nfrac = np.array([5], np.int32)
    cfg = gga.make_cfg(L, H, R, seed=seed, dose_cap=20.0)
    live, _, traj = gga.simulate(md, cfg, *_dev(dose, gap, nfrac), traj=True)
    traj = traj.cpu().numpy()[0]
    ev = protocol.events(dose[0], gap[0], 5, H, prm)
    for r in range(R):
        ref, certain = oracle_certain_prefix(prm, L, H, 10, ev, 0, r, seed)
        # sites within rounding of an oxygen-bin edge end the prefix at a fraction
        # step; it must still hold the fractions at 0 h and 24 h
        assert certain >= 30, certain
        assert np.array_equal(traj[r, :certain], ref[:certain]), r
    live0, _, _ = gga.simulate(model_dict, cfg, *_dev(dose, gap, nfrac))
    assert not np.array_equal(live.cpu().numpy(), live0.cpu().numpy())
