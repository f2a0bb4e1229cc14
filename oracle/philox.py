"""Philox4x32-10 counter-based generator, written from its published definition.

Source: J. K. Salmon, M. A. Moraes, R. O. Dror, D. E. Shaw, "Parallel Random
Numbers: As Easy as 1, 2, 3", SC'11, Section 4 (the Philox S-box: two 32x32->64
multiplications per round, the high halves XOR-ed with the other counter words
and the round key, a Weyl sequence bumping the key between rounds).

Test infrastructure: this module belongs to the CPU oracle.  It shares no code
with the HIP library and is imported only by the tests, the package smoke check
and the CPU-baseline leg of the benchmark.

The simulation keys one 4-word block per (site, step, replica, protocol):
counter = (site, step, replica, protocol), key = (seed_lo, seed_hi).  Word use:
w0 division target, w1 irradiation survival, w2 division priority, w3 division
readiness; at initialisation (step 0xFFFFFFFF) w0 draws the starting age.
"""
import numpy as np

MASK32 = np.uint64(0xFFFFFFFF)
# Multipliers and Weyl increments of Philox4x32 (SC'11, Table 2 / Section 4.2).
M0 = np.uint64(0xD2511F53)
M1 = np.uint64(0xCD9E8D57)
W0 = np.uint64(0x9E3779B9)
W1 = np.uint64(0xBB67AE85)
INIT_STEP = 0xFFFFFFFF


def philox4x32_10(c0, c1, c2, c3, k0, k1):
    """Return the four output words of Philox4x32 with 10 rounds.

    Arguments broadcast against each other; every value is taken modulo 2**32.
    Returns four uint32 arrays.
    """
    c0, c1, c2, c3, k0, k1 = (np.asarray(v, dtype=np.uint64) & MASK32
                              for v in np.broadcast_arrays(c0, c1, c2, c3, k0, k1))
    for rnd in range(10):
        if rnd:
            k0 = (k0 + W0) & MASK32
            k1 = (k1 + W1) & MASK32
        p0 = M0 * c0          # < 2**64, exact in uint64
        p1 = M1 * c2
        hi0, lo0 = p0 >> np.uint64(32), p0 & MASK32
        hi1, lo1 = p1 >> np.uint64(32), p1 & MASK32
        c0, c1, c2, c3 = hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0
    return tuple(v.astype(np.uint32) for v in (c0, c1, c2, c3))


def site_words(sites, step, replica, protocol, seed):
    """Philox words for an array of site indices at one (step, replica, protocol).

    Returns a (4, len(sites)) uint32 array (w0, w1, w2, w3).
    """
    seed = int(seed)
    k0, k1 = seed & 0xFFFFFFFF, (seed >> 32) & 0xFFFFFFFF
    sites = np.asarray(sites, dtype=np.uint64)
    w = philox4x32_10(sites, int(step) & 0xFFFFFFFF, int(replica), int(protocol), k0, k1)
    return np.stack(w)
