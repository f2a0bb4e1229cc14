"""Surrogate-screened GA on the device (needs an MI355X): one generation
against the oracle (random screen), graph replays against the host-driven
loop, and the gain of the trained surrogate over the same loop without it."""
import numpy as np
import pytest
import torch

from oracle import sga as osga
from oracle.model import Params

pytestmark = pytest.mark.gpu
ALPHA = dict(dose_quantum=0.5, dose_q=[1, 2, 3, 4, 5], gaps=list(range(6, 61, 6)), kmin=10, kmax=10, cap=20.0)


@pytest.fixture(scope="module")
def gga():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2303_08123_amd as g
    return g


def _alphabet(gga):
    return gga.make_alphabet(0.5, [1, 2, 3, 4, 5], list(range(6, 61, 6)), 10, 10, 20.0)


def _pop(N, K, seed):
    rng = np.random.default_rng(seed)
    return (rng.choice([0.5, 1.0, 1.5, 2.0], size=(N, K)).astype(np.float32),
            rng.choice(ALPHA["gaps"], size=(N, K)).astype(np.int32))


def test_random_screen_generation_matches_oracle(gga, model_dict):
    N, K, R, L, H, C, S = 24, 10, 2, 64, 30, 60, 8
    run_seed, ga_seed = 21, 5
    dose, gap = _pop(N, K, 3)
    cfg = gga.make_cfg(L, H, R, seed=run_seed, dose_cap=20.0)
    ga_cfg = gga.make_ga(n_elite=0, tournament_k=4, p_cross=0.8, p_mut=0.05, seed=ga_seed)
    sga = gga.SurrogateGA(model_dict, cfg, ga_cfg, _alphabet(gga), gga.make_sga(C, S, screen=False), None,
                          torch.from_numpy(dose).cuda(), torch.from_numpy(gap).cuda())
    sga.init()
    sga.run(2, use_graph=False)
    prm = Params.from_dict(model_dict)
    f = osga.simulate_fitness(prm, L, H, 10, R, run_seed, dose, gap)
    d, g = dose, gap
    for gen in range(2):
        d, g, f = osga.generation_random_screen(prm, L, H, 10, R, run_seed, d, g, f, gen, ga_seed, ALPHA,
                                                4, 0.8, 0.05, C, S)
    assert np.array_equal(sga.dose[:N].cpu().numpy(), d)
    assert np.array_equal(sga.gap[:N].cpu().numpy(), g)
    assert np.array_equal(sga.fit[:N].cpu().numpy(), f)
    h = sga.hist.cpu().numpy()
    assert h[1, 0] == f[0] and np.isclose(h[1, 1], f.astype(np.float64).mean(), rtol=1e-6)


def test_graph_equals_host_driven(gga, model_dict):
    N, K, R, L, H, C, S = 32, 10, 2, 64, 24, 128, 8
    dose, gap = _pop(N, K, 4)
    cfg = gga.make_cfg(L, H, R, seed=2, dose_cap=20.0)
    ga_cfg = gga.make_ga(n_elite=0, tournament_k=4, p_cross=0.8, p_mut=0.05, seed=6)
    net0 = gga.mlp_net(seed=1)
    out = []
    for use_graph in (False, True):
        net = net0.clone()                  # online refinement trains the net during the run
        s = gga.SurrogateGA(model_dict, cfg, ga_cfg, _alphabet(gga),
                            gga.make_sga(C, S, screen=True, refine_steps=2, refine_lr=1e-4), net,
                            torch.from_numpy(dose).cuda(), torch.from_numpy(gap).cuda(), archive=True)
        s.init()
        s.run(3, use_graph)
        torch.cuda.synchronize()
        s.run(2, use_graph)
        out.append([x.cpu().numpy() for x in (s.dose[:N], s.gap[:N], s.fit[:N], s.hist, *s.archive,
                                              gga.mlp_block(net, "p"))])
        assert not torch.equal(gga.mlp_block(net, "p"), gga.mlp_block(net0, "p"))   # the net was refined
        assert np.array_equal(out[-1][4][-1], out[-1][0][0]) and np.array_equal(out[-1][5][-1], out[-1][1][0])
    for a, b in zip(*out):
        assert np.array_equal(a, b, equal_nan=True)
    f = out[1][2]
    assert np.all(np.diff(f) >= 0) and np.all(np.diff(out[1][3][:, 0]) <= 0)


def test_surrogate_screen_beats_random_screen(gga, model_dict):
    """Same simulation budget per generation: offspring picked by the trained
    surrogate reach a fitter population than offspring picked at random."""
    L, H, R, K = 64, 240, 2, 10
    cfg = gga.make_cfg(L, H, R, seed=11, dose_cap=20.0)
    alpha = _alphabet(gga)
    # training pairs: random protocols of the same alphabet, simulated
    n_train = 8192
    td, tg, tn = gga.population_random(alpha, n_train, K, seed=123)
    live, tf, _ = gga.simulate(model_dict, gga.make_cfg(L, H, R, seed=99, dose_cap=20.0), td, tg, tn)
    net = gga.mlp_net(seed=2)
    gga.mlp_set_norm(net, tf)
    work = gga.mlp_work(512)
    rng = torch.Generator(device="cpu").manual_seed(0)
    step = 0
    for epoch in range(15):
        perm = torch.randperm(n_train, generator=rng).cuda()
        for b in range(0, n_train, 512):
            idx = perm[b:b + 512]
            step += 1
            gga.mlp_train_step(net, td[idx].contiguous(), tg[idx].contiguous(), tn[idx].contiguous(),
                               tf[idx].contiguous(), step, 1e-3, work=work)
    # held-out quality
    vd, vg, vn = gga.population_random(alpha, 1024, K, seed=321)
    _, vf, _ = gga.simulate(model_dict, gga.make_cfg(L, H, R, seed=98, dose_cap=20.0), vd, vg, vn)
    pred = gga.mlp_predict(net, vd, vg, vn).cpu().numpy()
    corr = np.corrcoef(pred, vf.cpu().numpy())[0, 1]
    print("surrogate held-out correlation", corr)
    assert corr > 0.4          # the targets are 2-replica means: noisy
    # the two loops
    N, C, S, G = 64, 1024, 16, 25
    d0, g0, _ = gga.population_random(alpha, N, K, seed=7)
    ga_cfg = gga.make_ga(n_elite=0, tournament_k=4, p_cross=0.8, p_mut=0.05, seed=8)
    res = {}
    for screen in (True, False):
        sga = gga.make_sga(C, S, screen=screen, refine_steps=2 if screen else 0, refine_lr=1e-4)
        s = gga.SurrogateGA(model_dict, cfg, ga_cfg, alpha, sga, net.clone(), d0, g0)
        s.init()
        s.run(G, use_graph=True)
        res[screen] = s.fit[:N].cpu().numpy()
    print("final population mean fitness: surrogate", res[True].mean(), "random", res[False].mean())
    assert res[True].mean() < res[False].mean()
    assert res[True][:8].mean() <= res[False][:8].mean()
