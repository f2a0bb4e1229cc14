"""Mitotic (delayed) death (mitotic_death = 1) against the oracle, through
the C ABI (needs an MI355X): single steps from states holding marked cells,
with and without a further fraction (resident 64 x 64 and 128 x 128
kernels, 256 x 256 slabs, also with the oxygen effect), and a trajectory over
its certain prefix."""
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


def delayed(md, oer=False):
    d = copy.deepcopy(md)
    d["kappa"] = [4.0e-3, 2.0e-3, 2.0e-3]
    d["mitotic_death"] = 1
    if oer:
        d["oer_max"], d["oer_k"] = 3.0, 0.1
    return d


@pytest.mark.parametrize("L,variant,event,oer", [(64, None, False, False), (64, None, True, False),
                                                 (128, None, True, True), (256, 5, False, False),
                                                 (256, 6, True, True)])
def test_single_step_with_marked_cells(gga, model_dict, L, variant, event, oer):
    md = delayed(model_dict, oer)
    prm = Params.from_dict(md)
    R, seed = 2, 13
    warm = {64: 150, 128: 260, 256: 200}[L]
    print(f"mitotic single step L={L} variant={variant} event={event} oer={oer}", flush=True)
    # a 2.5 Gy fraction six hours before the step marks cells (the oracle's state)
    pre = [(warm - 6, protocol.events(np.float32([2.5]), np.int32([0]), 1, 1, prm)[0][1])]
    states = [sim.run_instance(prm, L, warm, 10, pre, 0, r, seed)[:2] for r in range(R)]
    fields = to_field_units(np.stack([s[0] for s in states]), prm)
    start = from_field_units(fields, prm)
    cells = np.stack([s[1].astype(np.uint16) for s in states])
    assert ((cells >> 14) & 1).sum() > 20                  # marked cells are in the state
    dose = np.array([[2.5, 2.0]], np.float32)
    gap = np.array([[warm - 6, 6 if event else 9]], np.int32)
    nfrac = np.array([2], np.int32)
    cfg = gga.make_cfg(L, warm + 1, R, seed=seed, dose_cap=20.0)
    f_d, c_d = _dev(fields, cells.view(np.int16))
    dd = _dev(dose, gap, nfrac)
    if variant is None:
        live = gga.state_run(md, cfg, *dd, warm, 1, f_d, c_d)[0].cpu().numpy()
    else:
        live = gga.state_run_variant(md, cfg, variant, *dd, warm, 1, f_d, c_d).cpu().numpy()
    ev = dict(protocol.events(dose[0], gap[0], 2, warm + 1, prm))
    assert (warm in ev) == event
    got_f, got_c = from_field_units(f_d.cpu().numpy(), prm), c_d.cpu().numpy().view(np.uint16)
    for r in range(R):
        f_ref, c_ref, counted = oracle_step_detail(start[r], cells[r].astype(np.int64), warm, ev.get(warm), 0, r,
                                                   seed, prm, 10)
        assert field_error(got_f[r], f_ref) <= FIELD_RTOL
        bad, frac = compare_cells(got_c[r], c_ref, counted)
        assert bad == 0 and frac <= MAX_COUNTED_FRACTION, (r, bad, frac)
        if not counted.any():
            assert live[0, r] == sim.live_count(c_ref)
        assert not (got_c[r] & 0x3C00).any()               # no oxygen-bin bits left


def test_trajectory_with_mitotic_death(gga, model_dict):
    """BMII on 64 x 64 with delayed death: every step's live count equals the
    oracle's over the certain prefix, and delayed death changes the outcome."""
    md = copy.deepcopy(model_dict)
    md["mitotic_death"] = 1
    prm = Params.from_dict(md)
    L, R, seed, H = 64, 4, 3, 240
    dose = np.full((1, 5), 2.0, np.float32)
    gap = np.array([[0, 24, 24, 24, 24]], np.int32)
    nfrac = np.array([5], np.int32)
    cfg = gga.make_cfg(L, H, R, seed=seed, dose_cap=20.0)
    live, _, traj = gga.simulate(md, cfg, *_dev(dose, gap, nfrac), traj=True)
    traj = traj.cpu().numpy()[0]
    ev = protocol.events(dose[0], gap[0], 5, H, prm)
    for r in range(R):
        ref, certain = oracle_certain_prefix(prm, L, H, 10, ev, 0, r, seed)
        assert certain >= 50, certain
        assert np.array_equal(traj[r, :certain], ref[:certain]), r
    live0, _, _ = gga.simulate(model_dict, cfg, *_dev(dose, gap, nfrac))
    assert not np.array_equal(live.cpu().numpy(), live0.cpu().numpy())
