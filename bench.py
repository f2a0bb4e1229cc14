"""Benchmark: protocols/s and lattice-site-steps/s of the batched simulator.

One step = gga_simulate over the whole batch: every (protocol, replica)
instance simulated from its initial state over the horizon, live counts
reduced and the per-protocol fitness written.  Default workload: 1,024 random
protocols x 4 replicas on a 128 x 128 lattice over 20 days (480 steps of one
hour, 10 diffusion sub-steps each), doses {0.5..2.5} Gy, delays {6..60} h,
total dose <= 20 Gy.  Inputs are resident in HBM before timing starts.

Prints one JSON line with the throughput, the roofline of the simulation
kernel (VALU-bound: its state never leaves the compute unit) and the CPU
oracle timed on a bounded sample of the same workload.
"""
import argparse
import json
import multiprocessing as mp
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# Algorithmic VALU work of one site-substep: per field the neighbour sum
# (3 adds), the centre-and-reaction multiply-add, the lambda multiply-add,
# plus the non-negativity clamp of O and G: 6 + 6 + 5 operations.
OPS_PER_SITE_SUBSTEP = 17
# MI355X: 256 CUs x 4 SIMD x 16 lanes issue one full-rate 32-bit VALU
# operation per lane per clock at 2.4 GHz (packed FP32 excluded).
VALU_PEAK_OPS = 256 * 64 * 2.4e9


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def _oracle_instance(args):
    md, L, horizon, substeps, dose, gap, nfrac, p, r, seed = args
    from oracle import protocol, sim
    from oracle.model import Params
    prm = Params.from_dict(md)
    ev = protocol.events(dose, gap, nfrac, horizon, prm)
    t0 = time.perf_counter()
    _, _, traj = sim.run_instance(prm, L, horizon, substeps, ev, p, r, seed)
    return int(traj[-1]), time.perf_counter() - t0


def cpu_baseline(md, wl, dose, gap, nfrac, n_protocols=2):
    """The oracle on the first n_protocols protocols x R replicas, one instance
    per worker process."""
    R = wl["R"]
    jobs = [(md, wl["L"], wl["horizon"], wl["substeps"], dose[p], gap[p], int(nfrac[p]), p, r, wl["seed"])
            for p in range(n_protocols) for r in range(R)]
    workers = min(len(jobs), os.cpu_count() or 1)
    t0 = time.perf_counter()
    with mp.get_context("spawn").Pool(workers) as pool:
        res = pool.map(_oracle_instance, jobs)
    wall = time.perf_counter() - t0
    cpu_s = sum(t for _, t in res)
    inst_per_s = len(jobs) / wall
    return {
        "value": inst_per_s / R, "unit": "protocols/s", "cores": workers, "kind": "oracle",
        "sample": f"{n_protocols} protocols x {R} replicas of the same workload, whole horizon, "
                  f"one instance per process; {wall:.1f} s wall, {cpu_s:.1f} s CPU",
        "site_steps_per_s": len(jobs) * wl["L"] ** 2 * wl["horizon"] / wall,
    }


def time_to_best(hist_best, t_end_s, tol=0.01):
    """Seconds until the best-so-far fitness is within tol of the run's final
    best (fitness is minimised), and that final best."""
    best_so_far = np.minimum.accumulate(hist_best)
    final = float(best_so_far[-1])
    hit = int(np.argmax(best_so_far <= final * (1.0 + tol)))
    return float(t_end_s[hit]), final, hit


def ga_bench(gga, workloads, md, args):
    """GA on the device: population 2048 x 4 replicas on 128 x 128 over 20 days,
    tournament k = 4, one-point crossover 0.8, per-gene mutation 0.05 over the
    batched workload's alphabets, 10 % elites; host-driven loop vs replayed
    hipGraph generations, time-to-best from the per-generation history."""
    import torch
    wl = workloads.CONFIG2
    N, K, R, G = 2048, 10, wl["R"], args.generations
    cfg = gga.make_cfg(wl["L"], wl["horizon"], R, seed=wl["seed"], substeps=wl["substeps"], dose_cap=wl["dose_cap"])
    alpha = gga.make_alphabet(0.5, [1, 2, 3, 4, 5], list(range(6, 61, 6)), K, K, wl["dose_cap"])
    ga_cfg = gga.make_ga(n_elite=N // 10, tournament_k=4, p_cross=0.8, p_mut=0.05, seed=1)
    params = gga.make_params(md)
    dose0, gap0, _ = gga.population_random(alpha, N, K, seed=0)
    torch.cuda.synchronize()
    out = {}
    for mode, use_graph in (("plain", False), ("batched", True)):
        d, g = dose0, gap0
        hist, times, t_off = None, [], 0.0
        for g0 in range(0, G, args.chunk):
            n = min(args.chunk, G - g0)
            t0 = time.perf_counter()
            d, g, hist, gen_ms = gga.ga_run(params, cfg, ga_cfg, alpha, d, g, n, use_graph, g0=g0, hist=hist)
            wall = time.perf_counter() - t0
            times.extend(t_off + gen_ms.astype(np.float64) / 1000.0)
            t_off += wall
            h = hist.cpu().numpy()
            log(f"{mode}: generations {g0}..{g0 + n - 1} done in {wall:.1f} s, best so far {np.nanmin(h[:, 0]):.1f}")
        h = hist.cpu().numpy()
        ttb, final, hit = time_to_best(h[:, 0], np.array(times))
        out[mode] = {"time_to_best_s": ttb, "generation_of_best": hit, "final_best_fitness": final,
                     "total_s": t_off, "s_per_generation": t_off / G,
                     "best_first_generation": float(h[0, 0]), "mean_last_generation": float(h[-1, 1])}
    return {
        "metric": "GA time-to-best-fitness, batched (hipGraph generations) vs plain (host-driven loop)",
        "value": out["batched"]["time_to_best_s"], "unit": "s", "n_gpus": 1, "higher_is_better": False,
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "ga-2048x4-128x128-20d", "population": N, "replicas": R, "generations": G,
                   "lattice": wl["L"], "horizon_h": wl["horizon"], "tournament_k": 4, "p_cross": 0.8,
                   "p_mut": 0.05, "elites": N // 10},
        "plain": out["plain"], "batched": out["batched"],
        "speedup_time_to_best": out["plain"]["time_to_best_s"] / max(out["batched"]["time_to_best_s"], 1e-9),
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="batched", choices=["batched", "plain", "ga"])
    ap.add_argument("--generations", type=int, default=200, help="GA workload: generations")
    ap.add_argument("--chunk", type=int, default=20, help="GA workload: generations per progress line")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a plain 1 GiB device-to-device copy, to scale HBM counters")
    args = ap.parse_args()
    if args.calibrate_copy:
        import torch
        x = torch.ones(1 << 28, dtype=torch.float32, device="cuda")   # 1 GiB
        y = torch.empty_like(x)
        for _ in range(3):
            y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_per_launch": x.numel() * 4, "launches": 3}))
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU: the simulator shards by instance with no "
              "inter-GPU traffic, and this build runs and reports a single MI355X only.",
              file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2303_08123_amd as gga
    from paper_2303_08123_amd import workloads

    md = gga.load_model()
    if args.workload == "ga":
        print(json.dumps(ga_bench(gga, workloads, md, args)), flush=True)
        return
    if args.workload == "batched":
        wl = dict(workloads.CONFIG2)
        dose, gap, nfrac = workloads.config2_protocols(wl["P"], wl["K"], seed=0, cap=wl["dose_cap"])
    else:
        wl = dict(workloads.CONFIG1)
        dose, gap, nfrac = workloads.config1_protocols()
        wl["P"], wl["K"] = 1, dose.shape[1]
    P, R, L, N, S = wl["P"], wl["R"], wl["L"], wl["horizon"], wl["substeps"]
    cfg = gga.make_cfg(L, N, R, seed=wl["seed"], substeps=S, dose_cap=wl["dose_cap"])
    params = gga.make_params(md)
    dev = torch.device("cuda:0")
    d_d = torch.from_numpy(dose).to(dev)
    g_d = torch.from_numpy(gap).to(dev)
    n_d = torch.from_numpy(nfrac).to(dev)
    out = (torch.empty((P, R), dtype=torch.int32, device=dev),
           torch.empty((P,), dtype=torch.float32, device=dev), None)
    stream = torch.cuda.current_stream()

    for i in range(args.warmup):
        gga.simulate(params, cfg, d_d, g_d, n_d, out=out, stream=stream)
        torch.cuda.synchronize()
        log(f"warmup step {i + 1}/{args.warmup} done")

    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        ev[i][0].record(stream)
        gga.simulate(params, cfg, d_d, g_d, n_d, out=out, stream=stream)
        ev[i][1].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    launch_ms = [a.elapsed_time(b) for a, b in ev]
    log(f"timed {args.steps} steps: wall {wall:.3f} s, per launch {np.mean(launch_ms):.3f} ms")

    live = out[0].cpu().numpy()
    fit = out[1].cpu().numpy()
    assert np.all(live >= 0) and np.all(np.isfinite(fit))

    ms_per_step = 1000.0 * wall / args.steps
    site_steps = P * R * L * L * N
    kernel_s = float(np.mean(launch_ms)) / 1000.0
    achieved = OPS_PER_SITE_SUBSTEP * site_steps * S / kernel_s
    result = {
        "metric": "protocols/sec (batched simulation: 1024 protocols x 4 replicas, 128x128, 20 days)",
        "value": P / (ms_per_step / 1000.0),
        "unit": "protocols/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": wl["name"], "protocols": P, "replicas": R, "lattice": L,
                   "horizon_h": N, "substeps_per_h": S, "fractions": wl["K"], "dose_cap_gy": wl["dose_cap"]},
        "site_steps_per_s": site_steps / (ms_per_step / 1000.0),
        "mean_fitness": float(fit.mean()),
        "roofline": {"bound": "alu", "achieved": achieved / 1e12, "peak": VALU_PEAK_OPS / 1e12,
                     "unit": "Top/s", "frac": achieved / VALU_PEAK_OPS, "traffic": None,
                     "kernel": "sim_kernel", "kernel_ms": kernel_s * 1000.0},
    }
    if not args.no_cpu_baseline:
        log("timing the CPU oracle on a bounded sample")
        result["cpu_baseline"] = cpu_baseline(md, wl, dose, gap, nfrac, n_protocols=min(2, P))
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
