"""Host-side checks of the C ABI: the library loads, exports every declared
symbol, its structs match the Python mirrors, and the host validator agrees
with the oracle's.  No GPU work is launched."""
import ctypes
import os
import re
import shutil
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "gga.h")


@pytest.fixture(scope="module")
def gga():
    import torch  # noqa: F401  (the HIP runtime comes from torch's libraries)
    import paper_2303_08123_amd as g
    return g


def declared_functions():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+\*?\s+\*?(gga_\w+)\s*\(", text, re.M)))


def test_every_declared_symbol_is_exported(gga):
    names = declared_functions()
    assert len(names) == 26
    for n in names:
        assert hasattr(gga.LIB, n), n
    assert set(names) == set(gga.EXPORTS)
    if shutil.which("nm"):
        out = subprocess.run(["nm", "-D", "--defined-only", gga.LIB_PATH], capture_output=True, text=True).stdout
        exported = set(re.findall(r"\bT (gga_\w+)", out))
        assert set(names) <= exported


STRUCT_PROBE = r"""
#include <stdio.h>
#include <stddef.h>
#include "gga.h"
int main(void) {
  printf("%zu %zu %zu %zu %zu %zu %zu %zu %zu\n", sizeof(gga_params), sizeof(gga_sim_cfg), sizeof(gga_alphabet),
         offsetof(gga_params, P_div), offsetof(gga_params, m), offsetof(gga_sim_cfg, seed),
         offsetof(gga_alphabet, gaps), sizeof(gga_ga_cfg), offsetof(gga_ga_cfg, seed));
  return 0;
}
"""


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
def test_struct_layout_matches_python_mirror(gga, tmp_path):
    src = tmp_path / "probe.c"
    src.write_text(STRUCT_PROBE)
    exe = tmp_path / "probe"
    subprocess.run(["gcc", "-D__HIP_PLATFORM_AMD__", "-I", os.path.join(ROOT, "include"),
                    "-I", "/opt/rocm/include", str(src), "-o", str(exe)], check=True)
    vals = [int(v) for v in subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split()]
    assert vals == [ctypes.sizeof(gga.Params), ctypes.sizeof(gga.SimCfg), ctypes.sizeof(gga.Alphabet),
                    gga.Params.P_div.offset, gga.Params.m.offset, gga.SimCfg.seed.offset,
                    gga.Alphabet.gaps.offset, ctypes.sizeof(gga.GaCfg), gga.GaCfg.seed.offset]


def test_version_and_errors(gga):
    assert gga.version() == 1
    for code in (0, -1, -2, -3, -4, -5, -6, -99):
        assert gga.LIB.gga_strerror(code)


def test_host_validator_matches_oracle(gga):
    from oracle.protocol import validate
    from paper_2303_08123_amd import workloads
    rng = np.random.default_rng(3)
    for trial in range(20):
        P, K = 200, 8
        dose, gap, nfrac = workloads.random_protocols(P, K, seed=trial)
        dose[rng.uniform(size=dose.shape) < 0.01] = -0.5
        dose[rng.uniform(size=dose.shape) < 0.005] = np.nan
        gap[rng.uniform(size=gap.shape) < 0.02] = 0
        nfrac[rng.uniform(size=P) < 0.03] = K + 1
        cap = float(rng.uniform(5, 20))
        cfg = gga.make_cfg(64, 10, 1, dose_cap=cap)
        assert np.array_equal(gga.validate(cfg, dose, gap, nfrac), validate(dose, gap, nfrac, K, cap))


def test_abi_argument_errors(gga):
    cfg = gga.make_cfg(64, 10, 1)
    bad = gga.make_cfg(64, 10, 1)
    bad.struct_size = 3
    z = np.zeros((1, 1), np.float32)
    st = np.zeros(1, np.int32)
    vp = lambda a: a.ctypes.data_as(ctypes.c_void_p)
    assert gga.LIB.gga_validate(ctypes.byref(bad), vp(z), vp(st), vp(st), 1, 1, vp(st)) == -2
    assert gga.LIB.gga_validate(ctypes.byref(cfg), vp(z), vp(st), vp(st), -1, 1, vp(st)) == -1
    prm = gga.make_params(gga.load_model())
    prm.lambda_[0] = 0.3
    n = ctypes.c_void_p(0)
    assert gga.LIB.gga_simulate(ctypes.byref(prm), ctypes.byref(cfg), n, n, n, 1, 1, n, n, n, n) == -5
    prm = gga.make_params(gga.load_model())
    assert gga.LIB.gga_simulate(ctypes.byref(prm), ctypes.byref(cfg), n, n, n, 1, 1, n, n, n, n) == -1
    cfg96 = gga.make_cfg(96, 10, 1)
    assert gga.LIB.gga_simulate(ctypes.byref(prm), ctypes.byref(cfg96), n, n, n, 1, 1, n, n, n, n) == -3
    ab = gga.make_alphabet(0.5, [1, 2], [6], 5, 5, 2.0)   # 5 fractions of >= 0.5 Gy exceed 2 Gy
    assert gga.LIB.gga_population_random(ctypes.byref(ab), 0, 5, 0, n, n, n, n) == -6
    assert gga.LIB.gga_population_random(ctypes.byref(ab), 1, 5, 0, n, n, n, n) == -1


def test_mlp_layout_matches_library(gga):
    lay = gga.mlp_layout()
    assert lay["p"] == 256 and lay["g"] > lay["v"] > lay["m"] > lay["p"]
    assert gga.MLP_PARAMS == 591873
    total = lay["g"] + gga._align256(4 * gga.MLP_PARAMS)
    for k in (128, 512, 512):
        total += 2 * gga._align256(2 * k * 512)
    assert gga.LIB.gga_mlp_net_bytes() == total
