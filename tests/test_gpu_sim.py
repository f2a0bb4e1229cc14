"""HIP path against the oracle, through the C ABI (needs an MI355X)."""
import copy

import numpy as np
import pytest
import torch

from oracle import protocol, sim
from oracle.model import Params
from oracle.philox import philox4x32_10
from paper_2303_08123_amd import workloads
from parity_helpers import (FIELD_RTOL, MAX_COUNTED_FRACTION, compare_cells, field_error, from_field_units,
                            oracle_certain_prefix, oracle_step_detail, to_field_units)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gga():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2303_08123_amd as g
    return g


def _dev(*arrays):
    return [torch.from_numpy(np.ascontiguousarray(a)).cuda() for a in arrays]


def high_uptake(md):
    """Stronger consumption so quiescence and necrosis appear on small lattices."""
    d = copy.deepcopy(md)
    d["kappa"] = [4.0e-3, 2.0e-3, 2.0e-3]
    return d


def uniform_rt(md):
    d = copy.deepcopy(md)
    d["m"] = [1.0, 1.0, 1.0, 1.0]
    return d


def test_philox_matches_oracle(gga):
    rng = np.random.default_rng(0)
    n = 1 << 20
    ctr = rng.integers(0, 2**32, size=(n, 4), dtype=np.uint64).astype(np.uint32)
    seed = 0x9E3779B97F4A7C15
    out = gga.philox_fill(torch.from_numpy(ctr.view(np.int32)).cuda(), seed).cpu().numpy().view(np.uint32)
    ref = np.stack(philox4x32_10(ctr[:, 0], ctr[:, 1], ctr[:, 2], ctr[:, 3],
                                 seed & 0xFFFFFFFF, seed >> 32), axis=1)
    assert np.array_equal(out, ref)


@pytest.mark.parametrize("L", [64, 96, 128])
def test_initial_state_is_bit_exact(gga, model_dict, L):
    prm = Params.from_dict(model_dict)
    P, R, seed = 3, 2, 11
    cfg = gga.make_cfg(L, 0, R, seed=seed)
    fields, cells = gga.state_init(model_dict, cfg, P)
    fields, cells = fields.cpu().numpy(), cells.cpu().numpy().view(np.uint16)
    for p in range(P):
        for r in range(R):
            f_ref, c_ref = sim.init_state(prm, L, p, r, seed)
            assert np.array_equal(cells[p * R + r].astype(np.int64), c_ref)
            assert np.array_equal(fields[p * R + r], to_field_units(f_ref, prm))


def _oracle_states(prm, L, steps, P, R, seed, dose, gap, nfrac, substeps=10):
    """Mid-trajectory oracle states, fields rounded to float32."""
    out = []
    for p in range(P):
        ev = protocol.events(dose[p], gap[p], nfrac[p], steps, prm)
        for r in range(R):
            f, c, _ = sim.run_instance(prm, L, steps, substeps, ev, p, r, seed)
            out.append((f.astype(np.float32), c.astype(np.uint16)))
    return out


@pytest.mark.parametrize("L,preset,warm,event", [
    (64, "high_uptake", 150, False),
    (64, "high_uptake", 150, True),
    (64, "uniform_rt", 60, True),
    (128, "high_uptake", 260, False),
    (128, "high_uptake", 260, True),
])
def test_single_step_parity(gga, model_dict, L, preset, warm, event):
    """One step from identical state: fields within 1e-5 relative (floor 1e-3),
    cell words bit-exact outside the counted near-threshold set."""
    md = {"high_uptake": high_uptake, "uniform_rt": uniform_rt}[preset](model_dict)
    prm = Params.from_dict(md)
    P, R, seed, substeps = 2, 2, 5, 10
    # fraction j of protocol p falls on step `warm` when `event`
    dose = np.array([[2.0, 3.0], [1.5, 0.0]], np.float32)
    gap = np.array([[warm if event else warm + 3, 10], [warm if event else 1, 0]], np.int32)
    nfrac = np.array([2, 1], np.int32)
    # states: oracle run of `warm` steps with no fractions
    zero = (np.zeros((P, 2), np.float32), np.zeros((P, 2), np.int32), np.zeros(P, np.int32))
    states = _oracle_states(prm, L, warm, P, R, seed, *zero, substeps=substeps)
    fields = to_field_units(np.stack([s[0] for s in states]), prm)
    start = from_field_units(fields, prm)           # the state the HIP path holds, in physical units
    cells = np.stack([s[1] for s in states])
    f_d, c_d = _dev(fields, cells.view(np.int16))
    cfg = gga.make_cfg(L, warm + 1, R, seed=seed, substeps=substeps, dose_cap=100.0)
    d_d, g_d, n_d = _dev(dose, gap, nfrac)
    live, _ = gga.state_run(md, cfg, d_d, g_d, n_d, warm, 1, f_d, c_d)
    got_f = from_field_units(f_d.cpu().numpy(), prm)
    got_c = c_d.cpu().numpy().view(np.uint16)
    live = live.cpu().numpy()
    worst_field, worst_counted = 0.0, 0.0
    for p in range(P):
        ev = dict(protocol.events(dose[p], gap[p], nfrac[p], warm + 1, prm))
        if event:
            assert warm in ev
        for r in range(R):
            i = p * R + r
            f_ref, c_ref, counted = oracle_step_detail(start[i], cells[i].astype(np.int64),
                                                       warm, ev.get(warm), p, r, seed, prm, substeps)
            worst_field = max(worst_field, field_error(got_f[i], f_ref))
            bad, frac = compare_cells(got_c[i], c_ref, counted)
            if bad:
                ys, xs = np.nonzero((got_c[i].astype(np.int64) != c_ref) & ~counted)
                print("mismatch sites", list(zip(ys.tolist(), xs.tolist()))[:10],
                      "got", got_c[i][ys, xs][:10], "ref", c_ref[ys, xs][:10],
                      "was", cells[i][ys, xs][:10], "field err", field_error(got_f[i], f_ref))
            assert bad == 0, (p, r, bad)
            worst_counted = max(worst_counted, frac)
            if not counted.any():
                assert live[p, r] == sim.live_count(c_ref)
    assert worst_field <= FIELD_RTOL, worst_field
    assert worst_counted <= MAX_COUNTED_FRACTION, worst_counted


def test_single_step_parity_white_noise_fields(gga, model_dict):
    """Cells of every kind under fields drawn independently per site: cell words
    bit-exact outside the counted set; fields to the float32 bound of the update
    (neighbours of unrelated size make the 1e-5 relative bar meaningless at
    sites near zero, so the check is absolute: 2e-6)."""
    prm = Params.from_dict(model_dict)
    L, P, R, seed = 128, 1, 3, 9
    fields, cells = [], []
    for r in range(R):
        f, c = workloads.random_state(L, 100 + r)
        fields.append(f)
        cells.append(c)
    fields, cells = to_field_units(np.stack(fields), prm), np.stack(cells)
    start = from_field_units(fields, prm)
    f_d, c_d = _dev(fields, cells.view(np.int16))
    dose, gap, nfrac = np.array([[2.5]], np.float32), np.array([[77]], np.int32), np.array([1], np.int32)
    cfg = gga.make_cfg(L, 100, R, seed=seed, dose_cap=20.0)
    gga.state_run(model_dict, cfg, *_dev(dose, gap, nfrac), 77, 1, f_d, c_d)
    got_f, got_c = from_field_units(f_d.cpu().numpy(), prm), c_d.cpu().numpy().view(np.uint16)
    thr = protocol.events(dose[0], gap[0], 1, 100, prm)[0][1]
    for r in range(R):
        f_ref, c_ref, counted = oracle_step_detail(start[r], cells[r].astype(np.int64),
                                                   77, thr, 0, r, seed, prm, 10, abs_window=2e-6)
        assert np.max(np.abs(got_f[r] - f_ref)) < 2e-6
        bad, frac = compare_cells(got_c[r], c_ref, counted)
        assert bad == 0 and frac <= MAX_COUNTED_FRACTION, (r, bad, frac)


@pytest.mark.parametrize("L,warm,event", [(64, 150, True), (128, 240, False)])
def test_single_step_parity_from_gpu_state(gga, model_dict, L, warm, event):
    """The other direction: the HIP path advances its own initial state `warm`
    steps; the oracle takes that state (fields converted to physical units in
    float64) and both sides step once.  Same bar as from oracle states."""
    md = high_uptake(model_dict)
    prm = Params.from_dict(md)
    P, R, seed, substeps = 1, 3, 21, 10
    dose = np.array([[2.0, 2.5]], np.float32)
    gap = np.array([[warm if event else warm + 7, 30]], np.int32)
    nfrac = np.array([2], np.int32)
    cfg = gga.make_cfg(L, warm + 1, R, seed=seed, substeps=substeps, dose_cap=100.0)
    dd = _dev(dose, gap, nfrac)
    f_d, c_d = gga.state_init(md, cfg, P)
    gga.state_run(md, cfg, *dd, 0, warm, f_d, c_d)
    start = from_field_units(f_d.cpu().numpy(), prm)
    cells = c_d.cpu().numpy().view(np.uint16).copy()
    live, _ = gga.state_run(md, cfg, *dd, warm, 1, f_d, c_d)
    got_f = from_field_units(f_d.cpu().numpy(), prm)
    got_c, live = c_d.cpu().numpy().view(np.uint16), live.cpu().numpy()
    ev = dict(protocol.events(dose[0], gap[0], nfrac[0], warm + 1, prm))
    assert (warm in ev) == event
    assert ((cells & 3) == 2).any()                 # quiescent cells: the environment rules act
    for r in range(R):
        f_ref, c_ref, counted = oracle_step_detail(start[r], cells[r].astype(np.int64), warm, ev.get(warm), 0, r,
                                                   seed, prm, substeps)
        assert field_error(got_f[r], f_ref) <= FIELD_RTOL
        bad, frac = compare_cells(got_c[r], c_ref, counted)
        assert bad == 0 and frac <= MAX_COUNTED_FRACTION, (r, bad, frac)
        if not counted.any():
            assert live[0, r] == sim.live_count(c_ref)


def test_multi_step_state_run_equals_simulate(gga, model_dict):
    """Running 40 steps as 40 one-step calls from the initial state gives the
    same trajectory as one simulate call (same kernel, state round trip)."""
    L, R, steps, seed = 64, 2, 40, 3
    dose, gap, nfrac = workloads.config1_protocols()
    dd = _dev(dose, gap, nfrac)
    cfg = gga.make_cfg(L, steps, R, seed=seed)
    _, _, traj = gga.simulate(model_dict, cfg, *dd, traj=True)
    f_d, c_d = gga.state_init(model_dict, cfg, 1)
    counts = []
    for n in range(steps):
        live, _ = gga.state_run(model_dict, cfg, *dd, n, 1, f_d, c_d)
        counts.append(live.cpu().numpy()[0])
    assert np.array_equal(np.stack(counts, axis=1), traj.cpu().numpy()[0])


@pytest.mark.parametrize("preset,L,steps", [("default", 64, 240), ("high_uptake", 64, 200)])
def test_trajectory_matches_over_certain_prefix(gga, model_dict, preset, L, steps):
    """Whole trajectories, same seeds: the live count of every step agrees
    exactly until the oracle first meets a near-threshold site."""
    md = model_dict if preset == "default" else high_uptake(model_dict)
    prm = Params.from_dict(md)
    R, seed = 4, 0
    dose, gap, nfrac = workloads.config1_protocols()
    cfg = gga.make_cfg(L, steps, R, seed=seed)
    live, fit, traj = gga.simulate(md, cfg, *_dev(dose, gap, nfrac), traj=True)
    traj = traj.cpu().numpy()[0]
    ev = protocol.events(dose[0], gap[0], nfrac[0], steps, prm)
    certain_steps = []
    for r in range(R):
        ref, certain = oracle_certain_prefix(prm, L, steps, 10, ev, 0, r, seed)
        assert np.array_equal(traj[r, :certain], ref[:certain]), r
        certain_steps.append(certain)
    if preset == "default":
        assert min(certain_steps) == steps     # BMII on 64x64 never nears a threshold
    assert np.isclose(fit.cpu().numpy()[0], traj[:, -1].mean())


@pytest.mark.parametrize("alpha", ["config2", "varying_k"])
def test_population_matches_oracle(gga, alpha):
    if alpha == "config2":
        a = dict(dose_quantum=0.5, dose_q=[1, 2, 3, 4, 5], gaps=list(range(6, 61, 6)), kmin=10, kmax=10, cap=20.0)
        P, K = 1024, 10
    else:
        a = dict(dose_quantum=0.5, dose_q=list(range(1, 11)), gaps=list(range(6, 61, 6)), kmin=3, kmax=40, cap=30.0)
        P, K = 300, 40
    ab = gga.make_alphabet(**a)
    dose, gap, nfrac = gga.population_random(ab, P, K, seed=42)
    rd, rg, rn = protocol.sample_population(a, P, K, seed=42)
    assert np.array_equal(nfrac.cpu().numpy(), rn)
    assert np.array_equal(gap.cpu().numpy(), rg)
    assert np.array_equal(dose.cpu().numpy(), rd)


def test_invalid_protocols_are_flagged(gga, model_dict):
    L, R = 64, 2
    dose = np.array([[1.0, 1.0], [-1.0, 1.0], [15.0, 15.0], [1.0, 1.0], [1.0, 1.0]], np.float32)
    gap = np.array([[0, 5], [0, 5], [0, 5], [0, 0], [0, 5]], np.int32)
    nfrac = np.array([2, 2, 2, 2, 3], np.int32)
    cfg = gga.make_cfg(L, 20, R, seed=1, dose_cap=20.0)
    live, fit, _ = gga.simulate(model_dict, cfg, *_dev(dose, gap, nfrac))
    live, fit = live.cpu().numpy(), fit.cpu().numpy()
    status = gga.validate(cfg, dose, gap, nfrac)
    assert list(status) == [0, gga.PROTO_DOSE, gga.PROTO_CAP, gga.PROTO_GAP, gga.PROTO_NFRAC]
    assert np.all(live[0] > 0) and np.isfinite(fit[0])
    assert np.all(live[1:] == -1) and np.all(np.isnan(fit[1:]))
    assert np.array_equal(status, protocol.validate(dose, gap, nfrac, 2, 20.0))


def test_zero_and_edge_sizes(gga, model_dict):
    cfg = gga.make_cfg(64, 10, 1, seed=0)
    empty = torch.zeros((0, 3), dtype=torch.float32, device="cuda")
    live, fit, _ = gga.simulate(model_dict, cfg, empty, empty.int(), torch.zeros(0, dtype=torch.int32, device="cuda"))
    assert live.numel() == 0 and fit.numel() == 0
    # K = 0 protocols and a zero-step horizon
    z = torch.zeros((2, 0), dtype=torch.float32, device="cuda")
    n = torch.zeros(2, dtype=torch.int32, device="cuda")
    cfg0 = gga.make_cfg(64, 0, 3, seed=0)
    live, fit, _ = gga.simulate(model_dict, cfg0, z, z.int(), n)
    assert np.all(live.cpu().numpy() == 113)
    for side in (80, 288):                                 # multiples of 32 in 64 .. 256 only
        with pytest.raises(gga.GGAError):
            gga.simulate(model_dict, gga.make_cfg(side, 10, 1), z, z.int(), n)


def test_outputs_are_deterministic(gga, model_dict):
    dose, gap, nfrac = workloads.random_protocols(16, 6, seed=4, kmin=1)
    cfg = gga.make_cfg(128, 60, 3, seed=8, dose_cap=100.0)
    dd = _dev(dose, gap, nfrac)
    a = gga.simulate(model_dict, cfg, *dd, traj=True)
    b = gga.simulate(model_dict, cfg, *dd, traj=True)
    assert all(torch.equal(x, y) for x, y in zip(a, b))


def test_library_tumours_equal_state_runs_from_the_same_states(gga, model_dict):
    """Replica r of every protocol starts from library tumour r mod n: the live
    counts equal state_run from copies of those states."""
    L, P, R, n_lib, H = 64, 5, 3, 2, 40
    lib_f, lib_c = gga.grow_library(model_dict, L, n_lib, days=4, seed=12)
    assert (lib_c.cpu().numpy().view(np.uint16) & 3 != 0).sum() > 2 * 113      # the tumours grew
    dose, gap, nfrac = workloads.random_protocols(P, 4, seed=3, kmin=1)
    dd = _dev(dose, gap, nfrac)
    cfg = gga.make_cfg(L, H, R, seed=21, dose_cap=100.0)
    live, fit = gga.simulate_library(model_dict, cfg, *dd, lib_f, lib_c)
    idx = torch.tensor([r % n_lib for p in range(P) for r in range(R)], device="cuda")
    f, c = lib_f[idx].contiguous(), lib_c[idx].contiguous()
    ref, _ = gga.state_run(model_dict, cfg, *dd, 0, H, f, c)
    assert torch.equal(live, ref)
    assert np.allclose(fit.cpu().numpy(), ref.cpu().numpy().mean(1))
    assert torch.equal(lib_f, gga.grow_library(model_dict, L, n_lib, days=4, seed=12)[0])   # read only, repeatable
