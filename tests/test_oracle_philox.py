"""Pins of the oracle's Philox4x32-10 against published and library values."""
import os
import shutil
import subprocess

import numpy as np
import pytest

from oracle.philox import philox4x32_10, site_words

HERE = os.path.dirname(os.path.abspath(__file__))


def _kat():
    rows = []
    with open(os.path.join(HERE, "golden", "philox4x32_10_kat.txt")) as fh:
        for line in fh:
            if line.strip() and not line.startswith("#"):
                rows.append([int(t, 16) for t in line.split()])
    return rows


def test_known_answer_vectors():
    rows = _kat()
    assert len(rows) == 3
    for row in rows:
        out = philox4x32_10(*row[:6])
        assert [int(v) for v in out] == row[6:]


ROCRAND_PROG = r"""
#include <rocrand/rocrand_philox4x32_10.h>
#include <cstdio>
int main() {
  unsigned c0, c1, c2, c3, k0, k1;
  while (std::scanf("%x %x %x %x %x %x", &c0, &c1, &c2, &c3, &k0, &k1) == 6) {
    unsigned long long seed = ((unsigned long long)k1 << 32) | k0;
    unsigned long long sub = ((unsigned long long)c3 << 32) | c2;
    unsigned long long off = (((unsigned long long)c1 << 32) | c0) * 4ull;
    rocrand_device::philox4x32_10_engine e(seed, sub, off);
    uint4 r = e.next4();
    std::printf("%08x %08x %08x %08x\n", r.x, r.y, r.z, r.w);
  }
  return 0;
}
"""


@pytest.mark.skipif(shutil.which("g++") is None or
                    not os.path.exists("/opt/rocm/include/rocrand/rocrand_philox4x32_10.h"),
                    reason="needs g++ and the rocRAND headers")
def test_matches_rocrand_library(tmp_path):
    """rocRAND's philox4x32_10 engine, started at counter (c0, c1, c2, c3) via
    its (seed, subsequence, offset) arguments, returns the same blocks."""
    src = tmp_path / "rr.cpp"
    src.write_text(ROCRAND_PROG)
    exe = tmp_path / "rr"
    subprocess.run(["g++", "-O1", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include", str(src),
                    "-o", str(exe)], check=True, capture_output=True)
    rng = np.random.default_rng(7)
    ins = rng.integers(0, 2**32, size=(2000, 6), dtype=np.uint64)
    # keep c0 * 4 from overflowing the 64-bit offset: c1 < 2**30
    ins[:, 1] &= np.uint64(0x3FFFFFFF)
    text = "\n".join(" ".join(f"{int(v):x}" for v in row) for row in ins) + "\n"
    res = subprocess.run([str(exe)], input=text, capture_output=True, text=True, check=True)
    got = np.array([[int(t, 16) for t in line.split()] for line in res.stdout.splitlines()],
                   dtype=np.uint64)
    ref = np.stack(philox4x32_10(*[ins[:, i] for i in range(6)]), axis=1).astype(np.uint64)
    assert got.shape == ref.shape
    assert np.array_equal(got, ref)


def test_site_words_layout():
    """site_words uses counter (site, step, replica, protocol), key (seed lo, hi)."""
    seed = 0x0123456789ABCDEF
    w = site_words(np.array([5, 9]), 17, 3, 11, seed)
    for j, s in enumerate((5, 9)):
        ref = philox4x32_10(s, 17, 3, 11, seed & 0xFFFFFFFF, seed >> 32)
        assert [int(v) for v in ref] == [int(w[i, j]) for i in range(4)]


def test_threshold_decisions_are_unbiased():
    """P(w < T) = T / 2**32 for the comparisons the model makes (binomial CI)."""
    w = site_words(np.arange(400000), 3, 1, 2, 99)
    for T in (2**30, 1234567890, 3 * 2**30):
        for i in range(4):
            frac = np.mean(w[i] < T)
            p = T / 2**32
            assert abs(frac - p) < 5 * np.sqrt(p * (1 - p) / w.shape[1])


def test_multiply_shift_index_is_uniform():
    """floor(w * m / 2**32) is uniform on 0..m-1 (chi-square, m = 1..4)."""
    from scipy.stats import chisquare
    w = site_words(np.arange(200000), 8, 0, 0, 5)[0].astype(np.uint64)
    for m in (2, 3, 4):
        k = (w * np.uint64(m)) >> np.uint64(32)
        counts = np.bincount(k.astype(np.int64), minlength=m)
        assert counts.sum() == len(w) and len(counts) == m
        assert chisquare(counts).pvalue > 1e-4
