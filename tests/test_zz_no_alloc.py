"""gga_simulate_noalloc (the workspace in the library's fixed scratch) against
gga_simulate with a caller workspace, through the C ABI (needs an MI355X):
two calls in a row on slab-form sides, the second smaller, an invalid
protocol, a resident side, and a batch beyond the scratch refused before any
work."""
import numpy as np
import pytest
import torch

from paper_2303_08123_amd import workloads

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gga():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2303_08123_amd as g
    return g


def _dev(*arrays):
    return [torch.from_numpy(np.ascontiguousarray(a)).cuda() for a in arrays]


def _same(a, b):
    live_a, fit_a, tr_a = (x.cpu().numpy() if x is not None else None for x in a)
    live_b, fit_b, tr_b = (x.cpu().numpy() if x is not None else None for x in b)
    assert np.array_equal(live_a, live_b)
    assert np.array_equal(fit_a, fit_b, equal_nan=True)
    assert (tr_a is None) == (tr_b is None)
    if tr_a is not None:
        assert np.array_equal(tr_a, tr_b)


def test_noalloc_equals_simulate_on_two_calls_in_a_row(gga, model_dict):
    dose, gap, nfrac = workloads.random_protocols(6, 5, seed=11, kmin=1)
    dose[4, 1] = -1.0                                     # an invalid protocol: live -1, fitness NaN
    dd = _dev(dose, gap, nfrac)
    cfg = gga.make_cfg(160, 40, 4, seed=5, dose_cap=100.0)
    assert 0 < gga.workspace_bytes(cfg, 6) <= gga.NOALLOC_SCRATCH_BYTES
    print("noalloc call 1: L=160 P=6 R=4 horizon 40", flush=True)
    got = gga.simulate_noalloc(model_dict, cfg, *dd, traj=True)
    ref = gga.simulate(model_dict, cfg, *dd, traj=True)
    _same(got, ref)
    live = got[0].cpu().numpy()
    assert np.all(live[4] == -1) and np.all(np.delete(live, 4, 0) > 0)
    # a smaller second call: the scratch holds the first call's state, none of which may leak in
    small = [x[:2].contiguous() for x in dd]
    cfg2 = gga.make_cfg(160, 25, 2, seed=9, dose_cap=100.0)
    print("noalloc call 2: L=160 P=2 R=2 horizon 25", flush=True)
    got = gga.simulate_noalloc(model_dict, cfg2, *small, traj=True)
    ref = gga.simulate(model_dict, cfg2, *small, traj=True)
    _same(got, ref)
    # another slab side and a resident one (no scratch)
    for L in (224, 96):
        c = gga.make_cfg(L, 20, 2, seed=3, dose_cap=100.0)
        print(f"noalloc call: L={L} P=3 R=2 horizon 20", flush=True)
        _same(gga.simulate_noalloc(model_dict, c, *[x[:3].contiguous() for x in dd]),
              gga.simulate(model_dict, c, *[x[:3].contiguous() for x in dd]))


def test_noalloc_refuses_a_batch_beyond_the_scratch(gga, model_dict):
    P = 37                                                # 36 instances of 256 x 256 fit
    dose, gap, nfrac = workloads.random_protocols(P, 3, seed=2, kmin=1)
    dd = _dev(dose, gap, nfrac)
    cfg = gga.make_cfg(256, 10, 1, seed=0, dose_cap=100.0)
    assert gga.workspace_bytes(cfg, P) > gga.NOALLOC_SCRATCH_BYTES >= gga.workspace_bytes(cfg, 36)
    live = torch.full((P, 1), 7, dtype=torch.int32, device="cuda")
    fit = torch.zeros(P, dtype=torch.float32, device="cuda")
    with pytest.raises(gga.GGAError) as e:
        gga.simulate_noalloc(model_dict, cfg, *dd, out=(live, fit, None))
    assert e.value.code == gga.E_SCRATCH
    torch.cuda.synchronize()
    assert torch.all(live == 7)                           # nothing was enqueued
