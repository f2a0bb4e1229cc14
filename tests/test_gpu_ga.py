"""Device GA against the oracle, through the C ABI (needs an MI355X)."""
import numpy as np
import pytest
import torch

from oracle import ga as oga
from oracle import protocol, sim
from oracle.model import Params

pytestmark = pytest.mark.gpu

ALPHA = dict(dose_quantum=0.5, dose_q=[1, 2, 3, 4, 5], gaps=list(range(6, 61, 6)), kmin=10, kmax=10, cap=20.0)
W64 = 0x9E3779B97F4A7C15


@pytest.fixture(scope="module")
def gga():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2303_08123_amd as g
    return g


def _alphabet(gga):
    return gga.make_alphabet(ALPHA["dose_quantum"], ALPHA["dose_q"], ALPHA["gaps"], 10, 10, ALPHA["cap"])


def _pop(N, K, seed, doses=(0.5, 1.0, 1.5, 2.0, 2.5)):
    rng = np.random.default_rng(seed)
    dose = rng.choice(doses, size=(N, K)).astype(np.float32)
    gap = rng.choice(ALPHA["gaps"], size=(N, K)).astype(np.int32)
    return dose, gap


@pytest.mark.parametrize("N,gen,elite,k,doses", [
    (256, 7, 4, 4, (0.5, 1.0, 1.5, 2.0, 2.5)),
    (101, 0, 3, 6, (2.0, 2.5)),            # odd pair count, k > 4, parents over the cap
    (64, 123, 0, 1, (0.5, 1.0)),
])
def test_breed_matches_oracle(gga, N, gen, elite, k, doses):
    K = 10
    dose, gap = _pop(N, K, N + gen, doses)
    rng = np.random.default_rng(gen)
    fitness = rng.integers(0, 50, size=N).astype(np.float32)         # many ties
    fitness[rng.uniform(size=N) < 0.05] = np.nan
    cfg = gga.make_ga(n_elite=elite, tournament_k=k, p_cross=0.8, p_mut=0.05, seed=0xABCDEF12345)
    g_t = torch.tensor([gen], dtype=torch.int32, device="cuda")
    order, pos, nd, ng = gga.ga_breed(cfg, _alphabet(gga), torch.from_numpy(fitness).cuda(),
                                      torch.from_numpy(dose).cuda(), torch.from_numpy(gap).cuda(), g_t)
    r_order, r_pos = oga.rank_order(fitness)
    assert np.array_equal(order.cpu().numpy(), r_order) and np.array_equal(pos.cpu().numpy(), r_pos)
    rd, rg = oga.next_generation(dose, gap, fitness, gen, 0xABCDEF12345, ALPHA, elite, k, 0.8, 0.05)
    assert np.array_equal(nd.cpu().numpy(), rd)
    assert np.array_equal(ng.cpu().numpy(), rg)


@pytest.mark.parametrize("selection,crossover,mutation,k", [
    ("rank", "middle", ("gene",), 16),
    ("roulette", "two_point", ("swap",), 1),
    ("truncation", "uniform", ("raise",), 1),
    ("tournament", "uniform", ("gene", "swap", "raise"), 4),
    ("rank", "two_point", ("gene", "raise"), 3),
])
def test_breed_variants_match_oracle(gga, selection, crossover, mutation, k):
    """The paper-style operator variants, bit-exact against the oracle (an
    odd child count, NaN fitness, parents over the cap)."""
    N, K, gen, elite = 97, 10, 5, 2
    dose, gap = _pop(N, K, 31, (1.0, 1.5, 2.0, 2.5))
    rng = np.random.default_rng(8)
    fitness = rng.uniform(100, 400, size=N).astype(np.float32)
    fitness[::17] = np.nan
    kw = dict(selection=selection, crossover=crossover, mutation=mutation, q=0.7, trunc_frac=0.3,
              roulette_base=420.0)
    cfg = gga.make_ga(n_elite=elite, tournament_k=k, p_cross=0.9, p_mut=0.3, seed=1234567, **kw)
    g_t = torch.tensor([gen], dtype=torch.int32, device="cuda")
    _, _, nd, ng = gga.ga_breed(cfg, _alphabet(gga), torch.from_numpy(fitness).cuda(),
                                torch.from_numpy(dose).cuda(), torch.from_numpy(gap).cuda(), g_t)
    rd, rg = oga.next_generation(dose, gap, fitness, gen, 1234567, ALPHA, elite, k, 0.9, 0.3, **kw)
    assert np.array_equal(nd.cpu().numpy(), rd)
    assert np.array_equal(ng.cpu().numpy(), rg)


def test_generation_matches_oracle_simulation_and_breeding(gga, model_dict):
    """One whole generation at generation counter 3: the fitness the device
    computes equals the oracle's (short horizon, no near-threshold site), and
    the next population equals the oracle's breeding of that fitness."""
    N, K, R, L, H, seed, gen = 12, 10, 2, 64, 30, 77, 3
    dose, gap = _pop(N, K, 5, (0.5, 1.0, 1.5, 2.0))
    nfrac = np.full(N, K, np.int32)
    cfg = gga.make_cfg(L, H, R, seed=seed, dose_cap=20.0)
    ga_cfg = gga.make_ga(n_elite=2, tournament_k=4, p_cross=0.8, p_mut=0.05, seed=99)
    ws = gga.ga_workspace(N, R)
    gga.ga_set_generation(ws, gen)
    hist = torch.full((8, 2), float("nan"), device="cuda")
    dd = [torch.from_numpy(x).cuda() for x in (dose, gap, nfrac)]
    nd, ng = gga.ga_generation(model_dict, cfg, ga_cfg, _alphabet(gga), *dd, ws, hist=hist, advance=True)
    torch.cuda.synchronize()
    prm = Params.from_dict(model_dict)
    key = (seed + gen * W64) % 2**64
    fit = np.zeros(N)
    for p in range(N):
        ev = protocol.events(dose[p], gap[p], K, H, prm)
        fit[p] = np.mean([sim.run_instance(prm, L, H, 10, ev, p, r, key)[2][-1] for r in range(R)])
    fit32 = fit.astype(np.float32)
    h = hist.cpu().numpy()
    assert h[gen, 0] == fit32.min()
    assert np.isclose(h[gen, 1], fit.mean(), rtol=1e-6)
    assert np.all(np.isnan(np.delete(h, gen, axis=0)))
    rd, rg = oga.next_generation(dose, gap, fit32, gen, 99, ALPHA, 2, 4, 0.8, 0.05)
    assert np.array_equal(nd.cpu().numpy(), rd) and np.array_equal(ng.cpu().numpy(), rg)


def test_graph_replays_equal_host_driven_loop(gga, model_dict):
    """hipGraph-replayed generations give bit-identical history and populations
    to the host-driven loop, also when eager work and synchronisations run
    between two runs that continue from each other's output."""
    N, K, R, L, H = 48, 10, 2, 64, 36
    dose, gap = _pop(N, K, 8, (0.5, 1.0, 1.5, 2.0))
    cfg = gga.make_cfg(L, H, R, seed=5, dose_cap=20.0)
    ga_cfg = gga.make_ga(n_elite=2, tournament_k=4, p_cross=0.8, p_mut=0.05, seed=31)
    a = _alphabet(gga)
    d0, g0 = torch.from_numpy(dose).cuda(), torch.from_numpy(gap).cuda()
    results = {}
    for use_graph in (False, True):
        d1, g1, h1, t1 = gga.ga_run(model_dict, cfg, ga_cfg, a, d0, g0, 5, use_graph)
        # eager work in between, then continue from the result
        gga.simulate(model_dict, gga.make_cfg(L, 10, 1, seed=1), d1, g1,
                     torch.full((N,), K, dtype=torch.int32, device="cuda"))
        torch.cuda.synchronize()
        d2, g2, h2, t2 = gga.ga_run(model_dict, cfg, ga_cfg, a, d1, g1, 4, use_graph, g0=5, hist=h1)
        results[use_graph] = [x.cpu().numpy() for x in (d1, g1, h1, d2, g2, h2)]
        assert np.all(np.diff(t1) > 0) and np.all(np.diff(t2) > 0)
    for x, y in zip(results[False], results[True]):
        assert np.array_equal(x, y, equal_nan=True)
    h2 = results[True][5]
    assert h2.shape == (9, 2) and np.all(np.isfinite(h2)) and np.all(h2[:, 0] <= h2[:, 1])
    # one run of 9 generations equals the 5 + 4 continuation
    d9, g9, h9, _, (bd, bg) = gga.ga_run(model_dict, cfg, ga_cfg, a, d0, g0, 9, True, archive=True)
    assert np.array_equal(d9.cpu().numpy(), results[True][3]) and np.array_equal(h9.cpu().numpy(), h2)
    # the archive's last row is the best of generation 8, which elitism copies to row 0 of the bred population
    assert bd.shape == (9, K) and np.array_equal(bd[8].cpu().numpy(), d9[0].cpu().numpy())
    assert np.array_equal(bg[8].cpu().numpy(), g9[0].cpu().numpy())
    # and the first rows match the host-driven run's archive
    _, _, _, _, (pd, pg) = gga.ga_run(model_dict, cfg, ga_cfg, a, d0, g0, 5, False, archive=True)
    assert np.array_equal(pd.cpu().numpy(), bd[:5].cpu().numpy()) and np.array_equal(pg.cpu().numpy(), bg[:5].cpu().numpy())
