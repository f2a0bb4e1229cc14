"""Whole-trajectory parity (needs an MI355X).

Distribution level, as the paper compared its GPU and CPU codes (Results,
"Establishing the fidelity of the GPU model": t-test of means and
Kolmogorov-Smirnov tests over replicate runs): final live counts of the HIP
path under one run seed against stored oracle replicas under another seed;
the 95 % confidence interval of the mean difference must contain 0 (Welch)
and the two-sample KS p-value must exceed 0.05.  Three cases at level 0.05
each (multiplicity stated: three tests), and a family of 16 batched-workload
protocols tested as one family at level 0.05 (combined statistics, with a
Bonferroni bound per protocol).  Same seeds: the share of replicas whose
final counts agree exactly is reported.

Full size: the batched workload (1,024 protocols x 4 replicas, 128 x 128,
480 steps) in bench.py's launch configuration, with sampled instances checked
step by step against the oracle over their certain prefix.
"""
import copy
import json
import os

import numpy as np
import pytest
import torch
from scipy import stats

from oracle import protocol
from oracle.model import Params
from paper_2303_08123_amd import workloads
from parity_helpers import oracle_certain_prefix

pytestmark = pytest.mark.gpu
HERE = os.path.dirname(os.path.abspath(__file__))
GPU_SEED = 2000


@pytest.fixture(scope="module")
def gga():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2303_08123_amd as g
    return g


@pytest.fixture(scope="module")
def golden():
    with open(os.path.join(HERE, "golden", "oracle_distributions.json")) as fh:
        return json.load(fh)


@pytest.fixture(scope="module")
def family():
    with open(os.path.join(HERE, "golden", "oracle_batched16.json")) as fh:
        return json.load(fh)


def _model(md, name):
    if name == "high_uptake":
        md = copy.deepcopy(md)
        md["kappa"] = [4.0e-3, 2.0e-3, 2.0e-3]
    return md


def _run(gga, md, case, seed):
    dose = torch.tensor([case["dose"]], dtype=torch.float32, device="cuda")
    gap = torch.tensor([case["gap"]], dtype=torch.int32, device="cuda")
    nfrac = torch.tensor([case["nfrac"]], dtype=torch.int32, device="cuda")
    cfg = gga.make_cfg(case["L"], case["horizon"], case["R"], seed=seed, substeps=10, dose_cap=100.0)
    live, fit, _ = gga.simulate(md, cfg, dose, gap, nfrac)
    return live.cpu().numpy()[0], float(fit.cpu().numpy()[0])


@pytest.mark.parametrize("name", ["plain_bmii_64", "high_uptake_bmii_64", "batched_p0_128"])
def test_final_count_distribution_matches_oracle(gga, model_dict, golden, name):
    case = golden[name]
    md = _model(model_dict, case["model"])
    ref = np.array(case["live"], dtype=np.float64)
    got, fit = _run(gga, md, case, GPU_SEED)
    assert np.isclose(fit, got.mean(), rtol=1e-6)
    t = stats.ttest_ind(got, ref, equal_var=False)
    ks = stats.ks_2samp(got, ref)
    same, _ = _run(gga, md, case, golden["seed"])
    match = float(np.mean(same == np.array(case["live"])))
    print(f"{name}: gpu mean {got.mean():.1f} sd {got.std():.1f} | oracle mean {ref.mean():.1f} sd {ref.std():.1f} | "
          f"Welch p {t.pvalue:.3f} KS p {ks.pvalue:.3f} | same-seed exact match {match:.3f}")
    assert t.pvalue > 0.05 and ks.pvalue > 0.05
    if name == "plain_bmii_64":
        assert match == 1.0     # no site ever comes near a threshold in this case
    assert match >= 0.25


def test_batched_family_distributions_match_oracle(gga, model_dict, family):
    """16 protocols of the batched workload run as one batch of 16, 200
    replicas each, against stored oracle replicas under another run seed.
    One family at family-wise level 0.05: the standardised mean differences'
    sum of squares against chi2(16) and Fisher's combination of the 16 KS
    p-values against chi2(32), each at 0.05, and every protocol's Welch and KS
    p-values above the Bonferroni level 0.05 / 16.  Same seeds: at least a
    quarter of all replicas end with the oracle's exact count."""
    cases = sorted((v for k, v in family.items() if k.startswith("batched_")), key=lambda c: c["p"])
    assert [c["p"] for c in cases] == list(range(16))
    R = cases[0]["R"]
    dd = [torch.tensor([c[k] for c in cases], dtype=dt, device="cuda")
          for k, dt in (("dose", torch.float32), ("gap", torch.int32))]
    nfrac = torch.tensor([c["nfrac"] for c in cases], dtype=torch.int32, device="cuda")

    def run(seed):
        cfg = gga.make_cfg(128, 480, R, seed=seed, substeps=10, dose_cap=100.0)
        return gga.simulate(model_dict, cfg, *dd, nfrac)[0].cpu().numpy()

    got, same = run(GPU_SEED), run(family["seed"])
    z2, fisher, matches = 0.0, 0.0, 0
    for j, c in enumerate(cases):
        ref, g = np.array(c["live"], np.float64), got[j].astype(np.float64)
        t = stats.ttest_ind(g, ref, equal_var=False)
        ks = stats.ks_2samp(g, ref)
        z = (g.mean() - ref.mean()) / np.sqrt(g.var(ddof=1) / len(g) + ref.var(ddof=1) / len(ref))
        z2 += z * z
        fisher += -2.0 * np.log(max(ks.pvalue, 1e-300))
        matches += int(np.sum(same[j] == np.array(c["live"])))
        print(f"protocol {c['sample_index']}: gpu mean {g.mean():.1f} | oracle mean {ref.mean():.1f} | "
              f"Welch p {t.pvalue:.3f} KS p {ks.pvalue:.3f}")
        assert t.pvalue > 0.05 / 16 and ks.pvalue > 0.05 / 16, c["sample_index"]
    p_mean, p_ks = stats.chi2.sf(z2, 16), stats.chi2.sf(fisher, 32)
    match = matches / (16 * R)
    print(f"family: mean chi2(16) p {p_mean:.3f}, Fisher KS chi2(32) p {p_ks:.3f}, same-seed exact match {match:.3f}")
    assert p_mean > 0.05 and p_ks > 0.05
    assert match >= 0.25


@pytest.mark.parametrize("name", ["growth_64", "growth_128"])
def test_unirradiated_growth_matches_oracle(gga, model_dict, name):
    """Untreated growth on the plain (64 x 64, 10 days) and batched (128 x 128,
    20 days) workloads' lattices: the live count after every 24th step of the
    HIP path's replicas under one run seed against stored oracle replicas under
    another.  Each day's means agree by Welch's test at the Bonferroni level
    0.05 / days, and the final counts by Welch and two-sample KS at 0.05; under
    the oracle's seed, the share of replicas whose whole growth curve equals
    the oracle's exactly is reported (at least a quarter)."""
    with open(os.path.join(HERE, "golden", "oracle_growth.json")) as fh:
        case = json.load(fh)[name]
    seed_oracle = 1000
    ref = np.array(case["live"], np.float64)                # [R][days]
    every, R = case["every"], case["R"]
    z = torch.zeros((1, 0), dtype=torch.float32, device="cuda")
    nfrac = torch.zeros(1, dtype=torch.int32, device="cuda")

    def curves(seed):
        cfg = gga.make_cfg(case["L"], case["horizon"], R, seed=seed, substeps=10, dose_cap=100.0)
        live, fit, traj = gga.simulate(model_dict, cfg, z, z.int(), nfrac, traj=True)
        tr = traj.cpu().numpy()[0]
        assert np.array_equal(tr[:, -1], live.cpu().numpy()[0])
        return tr[:, every - 1::every].astype(np.float64)

    got, same = curves(GPU_SEED), curves(seed_oracle)
    days = ref.shape[1]
    for d in range(days):
        t = stats.ttest_ind(got[:, d], ref[:, d], equal_var=False)
        assert t.pvalue > 0.05 / days, (d + 1, got[:, d].mean(), ref[:, d].mean(), t.pvalue)
    t = stats.ttest_ind(got[:, -1], ref[:, -1], equal_var=False)
    ks = stats.ks_2samp(got[:, -1], ref[:, -1])
    match = float(np.mean(np.all(same == ref, axis=1)))
    print(f"{name}: day means gpu {np.round(got.mean(0), 1).tolist()} | oracle {np.round(ref.mean(0), 1).tolist()} | "
          f"final Welch p {t.pvalue:.3f} KS p {ks.pvalue:.3f} | same-seed whole-curve match {match:.3f}")
    assert t.pvalue > 0.05 and ks.pvalue > 0.05
    assert match >= 0.25
    assert np.all(np.diff(got.mean(0)) > 0)                   # the untreated tumour grows every day


def test_full_size_batched_workload(gga, model_dict):
    """Bench configuration: sampled instances equal the oracle step by step
    until their first near-threshold site; properties of every output."""
    wl = workloads.CONFIG2
    dose, gap, nfrac = workloads.config2_protocols(wl["P"], wl["K"], seed=0, cap=wl["dose_cap"])
    cfg = gga.make_cfg(wl["L"], wl["horizon"], wl["R"], seed=wl["seed"], substeps=wl["substeps"],
                       dose_cap=wl["dose_cap"])
    dd = [torch.from_numpy(x).cuda() for x in (dose, gap, nfrac)]
    live, fit, traj = gga.simulate(model_dict, cfg, *dd, traj=True)
    live, fit, traj = live.cpu().numpy(), fit.cpu().numpy(), traj.cpu().numpy()
    L2 = wl["L"] ** 2
    assert live.shape == (wl["P"], wl["R"]) and traj.shape == (wl["P"], wl["R"], wl["horizon"])
    assert np.all(live >= 0) and np.all(live <= L2) and np.array_equal(live, traj[:, :, -1])
    np.testing.assert_allclose(fit, live.mean(axis=1), rtol=1e-6)
    prm = Params.from_dict(model_dict)
    certain = []
    for p, r in ((0, 0), (517, 2), (1023, 3)):
        ev = protocol.events(dose[p], gap[p], nfrac[p], wl["horizon"], prm)
        ref, c = oracle_certain_prefix(prm, wl["L"], wl["horizon"], wl["substeps"], ev, p, r, wl["seed"])
        assert np.array_equal(traj[p, r, :c], ref[:c]), (p, r, c)
        certain.append(c)
    print("certain prefixes", certain)
    assert min(certain) >= 100
