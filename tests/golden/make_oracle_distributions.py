"""Write tests/golden/oracle_distributions.json: final live counts of many
independent oracle replicas for a few protocols (with --batched16:
tests/golden/oracle_batched16.json, 16 batched-workload protocols as one
batch; with --growth: tests/golden/oracle_growth.json, the live count every
24 steps of untreated tumours on the plain and batched workloads' lattices).

Calls only the oracle and the seeded input generators.  Run from the
repository root:  python tests/golden/make_oracle_distributions.py
"""
import copy
import json
import multiprocessing as mp
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

from oracle import protocol, sim  # noqa: E402
from oracle.model import Params  # noqa: E402
from paper_2303_08123_amd import workloads  # noqa: E402

ORACLE_SEED = 1000


def model(name):
    with open(os.path.join(ROOT, "paper_2303_08123_amd", "data", "model_default.json")) as fh:
        md = json.load(fh)
    if name == "high_uptake":
        md = copy.deepcopy(md)
        md["kappa"] = [4.0e-3, 2.0e-3, 2.0e-3]
    return md


def cases():
    d1, g1, n1 = workloads.config1_protocols()
    d2, g2, n2 = workloads.config2_protocols(1024, 10, seed=0, cap=20.0)
    return {
        "plain_bmii_64": dict(model="default", L=64, horizon=240, R=256,
                              dose=d1[0].tolist(), gap=g1[0].tolist(), nfrac=int(n1[0])),
        "high_uptake_bmii_64": dict(model="high_uptake", L=64, horizon=240, R=256,
                                    dose=d1[0].tolist(), gap=g1[0].tolist(), nfrac=int(n1[0])),
        "batched_p0_128": dict(model="default", L=128, horizon=480, R=200,
                               dose=d2[0].tolist(), gap=g2[0].tolist(), nfrac=int(n2[0])),
    }


# The batched family: 16 protocols of the batched workload's sample (indices
# 32, 96, ..., 992), simulated as one batch of 16 (batch position j is the
# Philox protocol index), 200 replicas each.
FAMILY_INDICES = [32 + 64 * j for j in range(16)]
FAMILY_R = 200


def one(args):
    name, c, r = args
    prm = Params.from_dict(model(c["model"]))
    ev = protocol.events(np.array(c["dose"], np.float32), np.array(c["gap"]), c["nfrac"], c["horizon"], prm)
    # protocol index c["p"] of the batch (0 unless given), replica r, under the oracle's own run seed
    traj = sim.run_instance(prm, c["L"], c["horizon"], 10, ev, c.get("p", 0), r, ORACLE_SEED)[2]
    if c.get("every"):
        return name, r, [int(v) for v in traj[c["every"] - 1::c["every"]]]
    return name, r, int(traj[-1])


# Unirradiated growth: the plain workload's 64 x 64 lattice over 10 days and
# the batched workload's 128 x 128 lattice over 20 days, no fraction; the live
# count after every 24th step.
def growth_cases():
    return {
        "growth_64": dict(model="default", L=64, horizon=240, R=256, dose=[], gap=[], nfrac=0, every=24),
        "growth_128": dict(model="default", L=128, horizon=480, R=200, dose=[], gap=[], nfrac=0, every=24),
    }


def family_cases():
    d2, g2, n2 = workloads.config2_protocols(1024, 10, seed=0, cap=20.0)
    return {f"batched_{i}": dict(model="default", L=128, horizon=480, R=FAMILY_R, p=j, sample_index=i,
                                 dose=d2[i].tolist(), gap=g2[i].tolist(), nfrac=int(n2[i]))
            for j, i in enumerate(FAMILY_INDICES)}


def main():
    family = "--batched16" in sys.argv
    growth = "--growth" in sys.argv
    cs = family_cases() if family else growth_cases() if growth else cases()
    jobs = [(name, c, r) for name, c in cs.items() for r in range(c["R"])]
    t0 = time.time()
    with mp.Pool(os.cpu_count()) as pool:
        res = pool.map(one, jobs, chunksize=4)
    if growth:
        about = ("live counts after every 24th step (days 1, 2, ..) of independent untreated oracle replicas "
                 f"(protocol index 0, no fraction, replica r = 0..R-1, run seed {ORACLE_SEED}); written by "
                 "tests/golden/make_oracle_distributions.py --growth")
    elif family:
        about = ("final live counts of independent oracle replicas of 16 batched-workload protocols simulated "
                 f"as one batch (batch position p, replica r = 0..R-1, run seed {ORACLE_SEED}); written by "
                 "tests/golden/make_oracle_distributions.py --batched16")
    else:
        about = ("final live counts of independent oracle replicas (protocol index 0, replica r = 0..R-1, "
                 f"run seed {ORACLE_SEED}); written by tests/golden/make_oracle_distributions.py")
    out = {"_about": about, "seed": ORACLE_SEED}
    for name, c in cs.items():
        live = [0] * c["R"]
        for n, r, v in res:
            if n == name:
                live[r] = v
        out[name] = dict(c, live=live)
    fname = "oracle_batched16.json" if family else "oracle_growth.json" if growth else "oracle_distributions.json"
    with open(os.path.join(ROOT, "tests", "golden", fname), "w") as fh:
        json.dump(out, fh, indent=1)
    print(f"done in {time.time() - t0:.0f} s")


if __name__ == "__main__":
    main()
