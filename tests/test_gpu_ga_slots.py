"""Device GA over the time-slot genome against the oracle, through the C ABI
(needs an MI355X).  Every comparison is bit-exact: genomes are bytes, decoded
doses are float32 products of a quantum count and the quantum."""
import numpy as np
import pytest
import torch

from oracle import ga_slots as ogs
from oracle import protocol, sim
from oracle.model import Params

pytestmark = pytest.mark.gpu

W64 = 0x9E3779B97F4A7C15
ALL = ("swap", "split", "time", "value")
DEFAULT = ("swap", "split", "time")


@pytest.fixture(scope="module")
def gga():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2303_08123_amd as g
    return g


def genomes(N, S, seed, dmax, g_min, cap, guarded=True, density=0.15):
    """Random genomes; unguarded ones hold doses up to 255 at any spacing."""
    rng = np.random.default_rng(seed)
    hi = dmax if guarded else 255
    pop = (rng.integers(1, hi + 1, (N, S)) * (rng.random((N, S)) < density)).astype(np.uint8)
    if guarded:
        pop = np.array([ogs.guards(r.tolist(), g_min, dmax, cap) for r in pop], np.uint8)
    return pop


def breed(gga, pop, fit, gen, ga_cfg, sc):
    g = torch.tensor([gen], dtype=torch.int32, device="cuda")
    _, _, nxt = gga.slots_breed(ga_cfg, sc, torch.from_numpy(fit).cuda(), torch.from_numpy(pop).cuda(), g)
    torch.cuda.synchronize()
    return nxt.cpu().numpy()


CASES = [
    # S, N, gen, elite, k, selection, crossover, mutations, guarded, g_min, dmax, cap
    (120, 256, 3, 4, 4, "tournament", "two_point", ALL, True, 6, 20, 40),       # the paper's window, 25/50/75 % cuts
    (256, 97, 0, 3, 5, "rank", "uniform", ALL, False, 12, 16, 40),             # two mask blocks, odd pair count
    (7, 40, 11, 4, 2, "roulette", "middle", ("swap", "split"), False, 2, 6, 9),  # ragged small window
    (1, 10, 2, 0, 3, "truncation", "one_point", ALL, False, 1, 4, 3),          # one slot: no crossover, no swap
    (200, 64, 5, 2, 3, "tournament", "one_point", ("time", "value"), True, 24, 8, 30),
    (120, 130, 9, 13, 4, "tournament", "two_point", DEFAULT, True, 48, 18, 40),  # default operators
    (129, 50, 1, 1, 64, "rank", "uniform", ALL, False, 3, 255, 65535),        # dmax 255, cap never binding
]


@pytest.mark.parametrize("case", CASES, ids=[f"S{c[0]}-N{c[1]}-{c[5]}-{c[6]}" for c in CASES])
def test_breed_matches_oracle(gga, case):
    S, N, gen, elite, k, selection, crossover, muts, guarded, g_min, dmax, cap = case
    print(f"slots breed S={S} N={N} {selection}/{crossover} {muts}", flush=True)
    pop = genomes(N, S, 1000 + S + N, dmax, g_min, cap, guarded)
    rng = np.random.default_rng(S * 7 + N)
    fit = rng.random(N).astype(np.float32) * 100
    fit[rng.integers(0, N, 3)] = np.nan
    fit[5] = fit[6]                                             # a tie, broken by index
    base = 120.0 if selection == "roulette" else 0.0
    ga_cfg = gga.make_ga(n_elite=elite, tournament_k=k, p_cross=0.9, p_mut=0.6, seed=4242 + S, selection=selection,
                         crossover=crossover, mutation=(), q=0.7, trunc_frac=0.4, roulette_base=base)
    sc = gga.make_slots(S=S, g_min=g_min, dmax_q=dmax, cap_q=cap, quantum=0.25,
                        mutation=() if muts == DEFAULT else muts)
    got = breed(gga, pop, fit, gen, ga_cfg, sc)
    want = ogs.next_generation_slots(pop, fit, gen, 4242 + S, g_min, dmax, cap, elite, k, 0.9, 0.6,
                                     selection=selection, crossover_kind=crossover, mutations=muts, q=0.7,
                                     trunc_frac=0.4, roulette_base=base)
    assert got.shape == want.shape
    bad = np.nonzero(np.any(got != want, axis=1))[0]
    assert bad.size == 0, f"rows {bad[:8]} differ"
    # every child meets the constraints
    for r in got[elite:]:
        slots = np.nonzero(r)[0]
        assert r.max(initial=0) <= dmax and int(r.sum()) <= cap and np.all(np.diff(slots) >= g_min)


def test_breed_full_population_sampled(gga):
    """A population of 2,048 genomes of the paper's 120-hour window: 256
    sampled rows, the elites and the last row equal the oracle's."""
    S, N, g_min, dmax, cap, gen, seed = 120, 2048, 6, 20, 40, 17, 99
    pop = genomes(N, S, 5, dmax, g_min, cap)
    fit = np.random.default_rng(6).random(N).astype(np.float32)
    ga_cfg = gga.make_ga(n_elite=204, tournament_k=4, p_cross=0.8, p_mut=0.3, seed=seed, crossover="two_point",
                         mutation=())
    sc = gga.make_slots(S=S, g_min=g_min, dmax_q=dmax, cap_q=cap, mutation=ALL)
    got = breed(gga, pop, fit, gen, ga_cfg, sc)
    rows = sorted(set(np.random.default_rng(7).integers(204, N, 256).tolist()) | {204, 205, N - 1})
    want = ogs.next_generation_slots(pop, fit, gen, seed, g_min, dmax, cap, 204, 4, 0.8, 0.3,
                                     crossover_kind="two_point", mutations=ALL, rows=rows)
    assert np.array_equal(got[:204], want[:204])
    assert np.array_equal(got[rows], want[rows])


@pytest.mark.parametrize("S,K,guarded", [(120, 20, True), (256, 64, False), (3, 5, False), (120, 4, False)])
def test_decode_matches_oracle(gga, S, K, guarded):
    N = 300
    pop = genomes(N, S, S + K, 20, 6, 40, guarded, density=0.1)
    pop[0] = 0                                                  # an empty genome
    pop[1, :] = 0
    pop[1, S - 1] = 7                                           # a dose in the last slot
    sc = gga.make_slots(S=S, g_min=1, dmax_q=255, cap_q=65535, quantum=0.3)
    d, g, n = gga.slots_decode(sc, torch.from_numpy(pop).cuda(), K)
    torch.cuda.synchronize()
    d, g, n = d.cpu().numpy(), g.cpu().numpy(), n.cpu().numpy()
    for p in range(N):
        wd, wg, wn = ogs.decode(pop[p].tolist(), np.float32(0.3), K)
        assert n[p] == wn and np.array_equal(d[p], wd) and np.array_equal(g[p], wg), p


def test_encode_matches_oracle(gga):
    """Protocols on and off the quantum grid, fractions past the window,
    negative, NaN and infinite doses, negative delays and nfrac outside 0 .. K."""
    P, K, S = 400, 12, 120
    rng = np.random.default_rng(3)
    dose = (rng.integers(0, 14, (P, K)) * 0.25).astype(np.float32)
    dose[::7] += np.float32(0.1)                                # off the grid
    dose[3, 2], dose[4, 0], dose[5, 1] = np.nan, -1.0, np.inf
    gap = rng.integers(0, 30, (P, K)).astype(np.int32)
    gap[9, 3] = -50
    nfrac = rng.integers(0, K + 1, P).astype(np.int32)
    nfrac[10], nfrac[11] = K + 5, -3
    sc = gga.make_slots(S=S, g_min=6, dmax_q=16, cap_q=40, quantum=0.25)
    pop = gga.slots_encode(sc, *[torch.from_numpy(x).cuda() for x in (dose, gap, nfrac)])
    torch.cuda.synchronize()
    got = pop.cpu().numpy()
    for p in range(P):
        want = ogs.encode(dose[p], gap[p], nfrac[p], S, np.float32(0.25), 6, 16, 40)
        assert got[p].tolist() == want, p


def test_decode_encode_round_trip_on_device(gga):
    S, K, N = 120, 20, 512
    pop = genomes(N, S, 77, 20, 6, 40)
    sc = gga.make_slots(S=S, g_min=6, dmax_q=20, cap_q=40)
    d, g, n = gga.slots_decode(sc, torch.from_numpy(pop).cuda(), K)
    back = gga.slots_encode(sc, d, g, n)
    torch.cuda.synchronize()
    assert np.array_equal(back.cpu().numpy(), pop)


def _fitness(model_dict, pop, K, L, H, R, key, quantum):
    prm = Params.from_dict(model_dict)
    fit = np.zeros(len(pop))
    for p, v in enumerate(pop):
        dose, gap, n = ogs.decode(v.tolist(), quantum, K)
        ev = protocol.events(dose, gap, n, H, prm)
        fit[p] = np.mean([sim.run_instance(prm, L, H, 10, ev, p, r, key)[2][-1] for r in range(R)])
    return fit.astype(np.float32)


def test_generation_matches_oracle_simulation_and_breeding(gga, model_dict):
    """One whole slot-GA generation: the device decodes, simulates, reduces and
    breeds; the oracle simulates the decoded protocols (short horizon) and
    breeds the same fitness to the same population."""
    N, S, K, R, L, H, seed = 12, 24, 8, 2, 64, 30, 77
    pop = genomes(N, S, 21, 8, 3, 16, density=0.4)
    cfg = gga.make_cfg(L, H, R, seed=seed, dose_cap=4.0)
    ga_cfg = gga.make_ga(n_elite=2, tournament_k=3, p_cross=0.8, p_mut=0.5, seed=5, crossover="two_point",
                         mutation=())
    sc = gga.make_slots(S=S, g_min=3, dmax_q=8, cap_q=16, mutation=ALL)
    nxt, hist, _ = gga.slots_run(model_dict, cfg, ga_cfg, sc, torch.from_numpy(pop).cuda(), K, 1, False)
    torch.cuda.synchronize()
    fit = _fitness(model_dict, pop, K, L, H, R, seed, np.float32(0.25))
    h = hist.cpu().numpy()
    assert h[0, 0] == fit.min() and np.isclose(h[0, 1], fit.astype(np.float64).mean(), rtol=1e-6)
    want = ogs.next_generation_slots(pop, fit, 0, 5, 3, 8, 16, 2, 3, 0.8, 0.5, crossover_kind="two_point",
                                     mutations=ALL)
    assert np.array_equal(nxt.cpu().numpy(), want)


def test_graph_replays_equal_host_driven_loop(gga, model_dict):
    """hipGraph replays and the host-driven loop give identical populations
    and histories; 5 + 4 generations continued equal 9 in one run; the archive
    holds the decoded best protocol of each generation."""
    N, S, K, R, L, H = 48, 120, 20, 2, 64, 36
    pop = torch.from_numpy(genomes(N, S, 8, 20, 6, 40)).cuda()
    cfg = gga.make_cfg(L, H, R, seed=5, dose_cap=10.0)
    ga_cfg = gga.make_ga(n_elite=4, tournament_k=4, p_cross=0.8, p_mut=0.2, seed=31, crossover="two_point",
                         mutation=())
    sc = gga.make_slots()
    out = {}
    for use_graph in (False, True):
        p5, h5, t5 = gga.slots_run(model_dict, cfg, ga_cfg, sc, pop, K, 5, use_graph)
        gga.slots_decode(sc, p5, K)                             # eager work in between
        torch.cuda.synchronize()
        p9, h9, t9 = gga.slots_run(model_dict, cfg, ga_cfg, sc, p5, K, 4, use_graph, g0=5)
        out[use_graph] = [x.cpu().numpy() for x in (p5, h5, p9, h9)]
        assert np.all(np.diff(t5) > 0) and np.all(np.diff(t9) > 0)
    for x, y in zip(out[False], out[True]):
        assert np.array_equal(x, y, equal_nan=True)
    full, hf, _, (bd, bg) = gga.slots_run(model_dict, cfg, ga_cfg, sc, pop, K, 9, True, archive=True)
    assert np.array_equal(full.cpu().numpy(), out[True][2])
    assert np.array_equal(hf.cpu().numpy()[5:], out[True][3][5:])
    assert np.array_equal(hf.cpu().numpy()[:5], out[True][1])
    # the last archived protocol is the best of generation 8, copied by elitism to row 0 of the result
    d0, g0, n0 = gga.slots_decode(sc, full[:1].contiguous(), K)
    assert np.array_equal(bd[8].cpu().numpy(), d0[0].cpu().numpy())
    assert np.array_equal(bg[8].cpu().numpy(), g0[0].cpu().numpy())
