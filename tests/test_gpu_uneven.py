"""Kernel variants and uneven batches against the resident kernel and the
oracle, through the C ABI (needs an MI355X).

Every variant computes each site with the same arithmetic, so slab and
resident variants must agree bit for bit; the 256 x 256 lattices, which only
the slab form runs, are checked against the oracle by single steps and by the
trajectory's certain prefix."""
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


@pytest.fixture(scope="module")
def gga():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2303_08123_amd as g
    yield g
    for L, v in ((64, 0), (96, 9), (128, 2), (160, 22), (192, 24), (224, 16), (256, 6)):   # the library's defaults
        g.set_variant(L, v)


def _dev(*arrays):
    return [torch.from_numpy(np.ascontiguousarray(a)).cuda() for a in arrays]


def high_uptake(md):
    d = copy.deepcopy(md)
    d["kappa"] = [4.0e-3, 2.0e-3, 2.0e-3]
    return d


def _oracle_init(prm, L, P, R, seed):
    """Initial states in the HIP path's field units."""
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


@pytest.mark.parametrize("L,variant,reference", [(64, 1, 0), (64, 7, 0), (64, 8, 0), (128, 4, 2), (128, 3, 2)])
def test_variants_agree_bit_for_bit(gga, model_dict, L, variant, reference):
    md = high_uptake(model_dict)
    prm = Params.from_dict(md)
    P, R, seed = 2, 2, 13
    f0, c0 = _oracle_init(prm, L, P, R, seed)
    cfg = gga.make_cfg(L, 150, R, seed=seed, dose_cap=100.0)
    states = {}
    for v in (reference, variant):
        f_d, c_d = _dev(f0, c0.view(np.int16))
        out = []
        for n0, n in ((0, 50), (50, 200)):              # dead cells at step 50, quiescent ones by 250
            live = gga.state_run_variant(md, cfg, v, *_dev(*PROTOS), n0, n, f_d, c_d)
            out.append((f_d.cpu().numpy().copy(), c_d.cpu().numpy().copy(), live.cpu().numpy()))
        states[v] = out
    for seg_a, seg_b in zip(states[reference], states[variant]):
        for a, b in zip(seg_a, seg_b):
            assert np.array_equal(a, b)
    st50, st250 = (states[reference][k][1].view(np.uint16) & 3 for k in (0, 1))
    assert (st50 == 3).any() and (st250 == 2).any()   # dead and quiescent cells took part


def test_slab_continuation_equals_one_run(gga, model_dict):
    """Steps run as two calls (state round trip) equal one call."""
    L, P, R, seed = 256, 2, 1, 4
    prm = Params.from_dict(model_dict)
    f0, c0 = _oracle_init(prm, L, P, R, seed)
    cfg = gga.make_cfg(L, 40, R, seed=seed, dose_cap=100.0)
    dd = _dev(*PROTOS)
    fa, ca = _dev(f0, c0.view(np.int16))
    la = gga.state_run_variant(model_dict, cfg, 5, *dd, 0, 25, fa, ca)
    fb, cb = _dev(f0, c0.view(np.int16))
    gga.state_run_variant(model_dict, cfg, 5, *dd, 0, 12, fb, cb)
    lb = gga.state_run_variant(model_dict, cfg, 5, *dd, 12, 13, fb, cb)
    assert torch.equal(fa, fb) and torch.equal(ca, cb) and torch.equal(la, lb)


@pytest.mark.parametrize("variant,event", [(5, False), (5, True), (6, True)])
def test_L256_single_step_parity(gga, model_dict, variant, event):
    md = high_uptake(model_dict)
    prm = Params.from_dict(md)
    L, P, R, seed, warm = 256, 1, 2, 5, 200
    states = [sim.run_instance(prm, L, warm, 10, [], 0, r, seed)[:2] for r in range(R)]
    fields = to_field_units(np.stack([s[0] for s in states]), prm)
    start = from_field_units(fields, prm)           # the state the HIP path holds, in physical units
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
    st = cells & 3
    assert (st == 2).any()                         # the state holds quiescent cells


def test_L256_trajectory_matches_oracle(gga, model_dict):
    """Same seeds: the live count of every step agrees with the oracle's until
    the oracle first meets a near-threshold site, and the uneven call's final
    count equals the step-by-step one."""
    from parity_helpers import oracle_certain_prefix
    prm = Params.from_dict(model_dict)
    L, R, seed, H = 256, 2, 0, 120
    dose, gap, nfrac = workloads.config1_protocols()
    dd = _dev(dose, gap, nfrac)
    cfg = gga.make_cfg(L, H, R, seed=seed, dose_cap=20.0)
    f0, c0 = _oracle_init(prm, L, 1, R, seed)
    f_d, c_d = _dev(f0, c0.view(np.int16))
    traj = np.stack([gga.state_run_variant(model_dict, cfg, 5, *dd, n, 1, f_d, c_d).cpu().numpy()[0]
                     for n in range(H)], axis=1)
    ev = protocol.events(dose[0], gap[0], nfrac[0], H, prm)
    for r in range(R):
        ref, certain = oracle_certain_prefix(prm, L, H, 10, ev, 0, r, seed)
        assert certain >= 60, certain
        assert np.array_equal(traj[r, :certain], ref[:certain]), r
    live, fit = gga.simulate_uneven(model_dict, cfg, *dd, [L], [H])
    assert np.array_equal(live.cpu().numpy()[0], traj[:, -1])
    assert np.isclose(fit.cpu().numpy()[0], traj[:, -1].mean())


def test_uneven_batch_equals_uniform_runs(gga, model_dict):
    """Mixed lattice sides, horizons (one of them 0) and fraction counts in one
    call equal the same protocols run per (side, horizon); invalid protocols
    give -1 / NaN."""
    md = high_uptake(model_dict)
    prm = Params.from_dict(md)
    P, K, R, seed = 10, 6, 2, 17
    dose, gap, nfrac = workloads.random_protocols(P, K, seed=2, kmin=1)
    dose[7, 0] = -1.0                                      # invalid dose
    lattice = np.array([64, 128, 256, 64, 256, 128, 64, 256, 128, 256], np.int32)
    horizon = np.array([30, 45, 20, 0, 33, 12, 30, 20, 45, 0], np.int32)
    cfg = gga.make_cfg(64, 0, R, seed=seed, dose_cap=100.0)
    dd = _dev(dose, gap, nfrac)
    live, fit = gga.simulate_uneven(md, cfg, *dd, lattice, horizon)
    live, fit = live.cpu().numpy(), fit.cpu().numpy()
    ref = np.zeros((P, R), np.int64)
    for L, H in sorted(set(zip(lattice.tolist(), horizon.tolist()))):
        rows = np.nonzero((lattice == L) & (horizon == H))[0]
        c = gga.make_cfg(L, H, R, seed=seed, dose_cap=100.0)
        if L < 256:
            lv, _, _ = gga.simulate(md, c, *dd)
            ref[rows] = lv.cpu().numpy()[rows]
        elif H > 0:
            f0, c0 = _oracle_init(prm, L, P, R, seed)
            f_d, c_d = _dev(f0, c0.view(np.int16))
            lv = gga.state_run_variant(md, c, 5, *dd, 0, H, f_d, c_d)
            ref[rows] = lv.cpu().numpy()[rows]
        else:
            ref[rows] = sim.live_count(sim.init_state(prm, L, 0, 0, seed)[1])
    ref[7] = -1
    assert np.array_equal(live, ref)
    assert np.isnan(fit[7]) and np.allclose(np.delete(fit, 7), np.delete(ref, 7, 0).mean(1))
    assert live[3, 0] == 113 and live[9, 1] == 113        # horizon 0: the seed disc


def test_uneven_batch_with_every_option_equals_uniform_runs(gga, model_dict):
    """With delays in half-hours, incomplete repair and the oxygen effect all
    on, a mixed batch (resident and slab forms) still equals the same
    protocols run per (side, horizon)."""
    md = high_uptake(model_dict)
    md["repair_half_time"], md["oer_max"], md["oer_k"] = 2.0, 3.0, 0.1
    prm = Params.from_dict(md)
    P, K, R, seed = 8, 6, 2, 23
    dose, gap, nfrac = workloads.random_protocols(P, K, seed=5, kmin=2)
    gap[:, 1:] = np.maximum(gap[:, 1:] // 3, 1)            # half-hour delays, fractions close together
    gap[:, 0] = 2 * (gap[:, 0] % 10) + 1                   # the first fraction at an odd half-hour before 10 h
    lattice = np.array([64, 128, 256, 64, 256, 128, 256, 64], np.int32)
    horizon = np.array([30, 25, 20, 30, 20, 25, 12, 0], np.int32)
    cfg = gga.make_cfg(64, 0, R, seed=seed, dose_cap=100.0, half_hour=True)
    dd = _dev(dose, gap, nfrac)
    live = gga.simulate_uneven(md, cfg, *dd, lattice, horizon)[0].cpu().numpy()
    ref = np.zeros((P, R), np.int64)
    for L, H in sorted(set(zip(lattice.tolist(), horizon.tolist()))):
        rows = np.nonzero((lattice == L) & (horizon == H))[0]
        c = gga.make_cfg(L, H, R, seed=seed, dose_cap=100.0, half_hour=True)
        if L < 256:
            ref[rows] = gga.simulate(md, c, *dd)[0].cpu().numpy()[rows]
        elif H > 0:
            f0, c0 = _oracle_init(prm, L, P, R, seed)
            f_d, c_d = _dev(f0, c0.view(np.int16))
            ref[rows] = gga.state_run_variant(md, c, 6, *dd, 0, H, f_d, c_d).cpu().numpy()[rows]
        else:
            ref[rows] = sim.live_count(sim.init_state(prm, L, 0, 0, seed)[1])
    assert np.array_equal(live, ref)
    # the options change the outcome of the irradiated protocols
    plain = gga.simulate_uneven(high_uptake(model_dict), gga.make_cfg(64, 0, R, seed=seed, dose_cap=100.0,
                                                                      half_hour=True), *dd, lattice, horizon)[0]
    assert not np.array_equal(plain.cpu().numpy(), live)


def test_slab_variants_and_choice_do_not_change_results(gga, model_dict):
    P, K, R = 6, 5, 2
    dose, gap, nfrac = workloads.random_protocols(P, K, seed=9, kmin=1)
    lattice = np.array([256, 128, 64, 256, 128, 64], np.int32)
    horizon = np.array([24, 30, 30, 18, 10, 5], np.int32)
    cfg = gga.make_cfg(64, 0, R, seed=3, dose_cap=100.0)
    dd = _dev(dose, gap, nfrac)
    results = []
    for v256, v128 in ((5, 2), (6, 4), (5, 3)):
        gga.set_variant(256, v256)
        gga.set_variant(128, v128)
        results.append([x.cpu().numpy() for x in gga.simulate_uneven(model_dict, cfg, *dd, lattice, horizon)])
    gga.set_variant(256, 6)
    gga.set_variant(128, 2)
    for res in results[1:]:
        assert np.array_equal(res[0], results[0][0]) and np.array_equal(res[1], results[0][1], equal_nan=True)


def test_autotune_picks_a_variant_of_the_side(gga, model_dict):
    dose, gap, nfrac = workloads.random_protocols(64, 4, seed=1, kmin=1)
    dd = _dev(dose, gap, nfrac)
    cfg = gga.make_cfg(64, 24, 2, seed=0, dose_cap=100.0)
    before = gga.simulate(model_dict, cfg, *dd)[0].cpu().numpy()
    v, ms = gga.autotune(model_dict, cfg, *dd)
    assert gga.variants()[v][1] == 64 and set(ms) == {0, 1, 7, 8} and all(t > 0 for t in ms.values())
    res = min((t, i) for i, t in ms.items() if not gga.variants()[i][2])[1]
    assert gga.get_variant(64) == v and gga.get_variant(64, resident_only=True) == res
    after = gga.simulate(model_dict, cfg, *dd)[0].cpu().numpy()
    assert np.array_equal(before, after)
    gga.set_variant(64, 0)
    assert gga.get_variant(64, resident_only=True) == 0


def test_full_size_uneven_workload(gga, model_dict):
    """The uneven bench configuration (8192 protocols x 8 replicas, sides 64,
    96, .., 256, 10-40 days, 3-40 fractions) with the default variants:
    properties of every output; for the first protocol of each side, every
    replica's count equals a uniform gga_simulate of the same protocol index,
    whose trajectory equals the oracle's step by step until its first
    near-threshold site (the first 150 steps at most)."""
    wl = dict(workloads.CONFIG3)
    P, K, R = wl["P"], wl["K"], wl["R"]
    print("full-size uneven batch", flush=True)
    alpha = gga.make_alphabet(wl["dose_quantum"], wl["dose_q"], wl["gaps"], wl["kmin"], K, wl["dose_cap"])
    dose, gap, nfrac = gga.population_random(alpha, P, K, seed=3)
    lattice, horizon = workloads.config3_shapes(P, seed=wl["seed"], sides=wl["sides"], days=wl["days"])
    cfg = gga.make_cfg(64, 0, R, seed=wl["seed"], substeps=wl["substeps"], dose_cap=wl["dose_cap"])
    live, fit = gga.simulate_uneven(model_dict, cfg, dose, gap, nfrac, lattice, horizon)
    live, fit = live.cpu().numpy(), fit.cpu().numpy()
    assert live.shape == (P, R) and fit.shape == (P,)
    assert np.all(live >= 0) and np.all(live <= lattice.astype(np.int64)[:, None] ** 2)
    np.testing.assert_allclose(fit, live.mean(axis=1), rtol=1e-6)
    prm = Params.from_dict(model_dict)
    dh, gh, nh = (x.cpu().numpy() for x in (dose, gap, nfrac))
    certain = []
    for L in wl["sides"]:
        p = int(np.nonzero(lattice == L)[0][0])
        H = int(horizon[p])
        print(f"sampled protocol {p}: L={L} H={H}", flush=True)
        c1 = gga.make_cfg(L, H, R, seed=wl["seed"], substeps=wl["substeps"], dose_cap=wl["dose_cap"])
        lv, _, tr = gga.simulate(model_dict, c1, dose[:p + 1].contiguous(), gap[:p + 1].contiguous(),
                                 nfrac[:p + 1].contiguous(), traj=True)
        lv, tr = lv.cpu().numpy(), tr.cpu().numpy()
        assert np.array_equal(lv[p], live[p]), (L, p)
        ev = protocol.events(dh[p], gh[p], int(nh[p]), H, prm)
        n = min(H, 150)
        for r in (0, R - 1):
            ref, c = oracle_certain_prefix(prm, L, n, wl["substeps"], ev, p, r, wl["seed"])
            assert np.array_equal(tr[p, r, :c], ref[:c]), (L, p, r, c)
            certain.append(c)
    print("certain prefixes", certain)
    assert min(certain) >= 60
