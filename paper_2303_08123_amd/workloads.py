"""Seeded synthetic inputs shared by the tests, the benchmark and the smoke check.

Holds none of the simulated method's arithmetic: it only draws protocols and
lattice states from NumPy generators.  The paper's own workload (a private
library of ten pre-grown tumours, Materials and Methods, "The tumour case
library") is not available; a seed spheroid of radius 6 stands in for it.
"""
import numpy as np

# Benchmark II of the paper (Results, "Defining the search problem"): five
# 2 Gy fractions, the first at t = 0 and then every 24 h.
BMII = (np.array([2.0, 2.0, 2.0, 2.0, 2.0], np.float32), np.array([0, 24, 24, 24, 24], np.int32))
# Benchmark I: 1.25 Gy twice a day, 6 h / 18 h apart, eight fractions.
BMI = (np.full(8, 1.25, np.float32), np.array([0, 6, 18, 6, 18, 6, 18, 6], np.int32))

CONFIG1 = dict(name="plain-64x64-bmii", L=64, R=4, horizon=240, substeps=10, seed=0, dose_cap=20.0)
CONFIG2 = dict(name="batched-1024x4-128x128-20d", L=128, R=4, horizon=480, substeps=10, seed=0,
               dose_cap=20.0, P=1024, K=10)
# Uneven batch: lattice side uniform over {64, 96, .., 256} per protocol, 3-40
# fractions of 0.5-5 Gy (0.5 Gy steps) with delays from the batched workload's
# alphabet, total <= 30 Gy (drawn on the device, uniform over the feasible set
# for each fraction count), horizon uniform over 10-40 whole days.
CONFIG3 = dict(name="uneven-8192x8-64to256-10to40d", R=8, substeps=10, seed=0, dose_cap=30.0, P=8192, K=40,
               kmin=3, dose_quantum=0.5, dose_q=list(range(1, 11)), gaps=list(range(6, 61, 6)),
               sides=(64, 96, 128, 160, 192, 224, 256), days=(10, 40))
# Quasi-3D variant: the batched workload's protocols (first 256) on 128 x 128
# sites with 8 cell slots each, 20 days.
CONFIG_Q3 = dict(name="quasi3d-256x4-128x128x8-20d", L=128, C=8, R=4, horizon=480, substeps=10, seed=0,
                 dose_cap=20.0, P=256, K=10)
CONFIG2_DOSES = np.array([0.5, 1.0, 1.5, 2.0, 2.5], np.float32)
CONFIG2_GAPS = np.arange(6, 61, 6, dtype=np.int32)


def config1_protocols():
    dose, gap = BMII
    return dose[None, :].copy(), gap[None, :].copy(), np.array([5], np.int32)


def config2_protocols(P=1024, K=10, seed=0, cap=20.0):
    """Doses iid uniform over {0.5, ..., 2.5} Gy, delays iid uniform over
    {6, 12, ..., 60} h (the first one included), total dose <= cap by
    rejection of whole protocols."""
    rng = np.random.default_rng(seed)
    dose = np.zeros((P, K), np.float32)
    gap = np.zeros((P, K), np.int32)
    for p in range(P):
        while True:
            d = rng.choice(CONFIG2_DOSES, size=K)
            if float(d.astype(np.float64).sum()) <= cap:
                break
        dose[p] = d
        gap[p] = rng.choice(CONFIG2_GAPS, size=K)
    return dose, gap, np.full(P, K, np.int32)


def random_protocols(P, K, seed, dose_max=3.0, gap_max=48, kmin=0):
    """Unconstrained random protocols for parity tests (may exceed any cap)."""
    rng = np.random.default_rng(seed)
    nfrac = rng.integers(kmin, K + 1, size=P).astype(np.int32)
    dose = np.round(rng.uniform(0.25, dose_max, size=(P, K)) * 4) / 4
    gap = rng.integers(1, gap_max + 1, size=(P, K))
    gap[:, 0] = rng.integers(0, gap_max + 1, size=P)
    for p in range(P):
        dose[p, nfrac[p]:] = 0
        gap[p, nfrac[p]:] = 0
    return dose.astype(np.float32), gap.astype(np.int32), nfrac


def random_state(L, seed, tumour_radius=None, field_lo=0.0, field_hi=1.0):
    """A lattice state with every cell state and age, and fields spread over
    [field_lo, field_hi] so that all environment thresholds are exercised.
    Returns (fields[3, L, L] float32, cells[L, L] uint16)."""
    rng = np.random.default_rng(seed)
    yy, xx = np.mgrid[0:L, 0:L]
    r = tumour_radius if tumour_radius is not None else L // 3
    inside = (xx - L // 2) ** 2 + (yy - L // 2) ** 2 <= r * r
    state = np.where(inside, rng.choice([1, 1, 2, 3, 0], size=(L, L)), 0)
    age = rng.integers(0, 40, size=(L, L))
    age[rng.uniform(size=(L, L)) < 0.02] = 255
    cells = np.where(state == 0, 0, state | (age << 2)).astype(np.uint16)
    fields = rng.uniform(field_lo, field_hi, size=(3, L, L)).astype(np.float32)
    return fields, cells


def config3_shapes(P, seed=0, sides=(64, 96, 128, 160, 192, 224, 256), days=(10, 40)):
    """Per-protocol lattice side and horizon (steps) of the uneven batch."""
    rng = np.random.default_rng(seed)
    lattice = rng.choice(np.asarray(sides, np.int32), size=P).astype(np.int32)
    horizon = (24 * rng.integers(days[0], days[1] + 1, size=P)).astype(np.int32)
    return lattice, horizon
