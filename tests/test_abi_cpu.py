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
    assert len(names) >= 51               # the pattern finds every declaration
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
  printf("%zu %zu %zu\n", offsetof(gga_ga_cfg, selection), offsetof(gga_ga_cfg, q), offsetof(gga_ga_cfg, roulette_base));
  printf("%zu %zu\n", sizeof(gga_sga_cfg), offsetof(gga_sga_cfg, refine_lr));
  printf("%zu %zu %zu\n", sizeof(gga_slot_cfg), offsetof(gga_slot_cfg, quantum), offsetof(gga_slot_cfg, reserved));
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
                    gga.Alphabet.gaps.offset, ctypes.sizeof(gga.GaCfg), gga.GaCfg.seed.offset,
                    gga.GaCfg.selection.offset, gga.GaCfg.q.offset, gga.GaCfg.roulette_base.offset,
                    ctypes.sizeof(gga.SgaCfg), gga.SgaCfg.refine_lr.offset,
                    ctypes.sizeof(gga.SlotCfg), gga.SlotCfg.quantum.offset, gga.SlotCfg.reserved.offset]


def test_version_and_errors(gga):
    assert gga.version() == 2
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
    assert gga.LIB.gga_simulate(ctypes.byref(prm), ctypes.byref(cfg), n, n, n, 1, 1, n, 0, n, n, n, n) == -5
    for f, v in ((1, 0.0), (2, 0.0), (2, 1e-20), (1, 1e20)):   # rates must be positive, ratios in [1e-12, 1e12]
        prm = gga.make_params(gga.load_model())
        prm.kappa[f] = v
        assert gga.LIB.gga_simulate(ctypes.byref(prm), ctypes.byref(cfg), n, n, n, 1, 1, n, 0, n, n, n, n) == -5, (f, v)
    prm = gga.make_params(gga.load_model())
    assert gga.LIB.gga_simulate(ctypes.byref(prm), ctypes.byref(cfg), n, n, n, 1, 1, n, 0, n, n, n, n) == -1
    for side in (48, 80, 100, 288):                # multiples of 32 in 64 .. 256 only
        cfgx = gga.make_cfg(side, 10, 1)
        assert gga.LIB.gga_simulate(ctypes.byref(prm), ctypes.byref(cfgx), n, n, n, 1, 1, n, 0, n, n, n, n) == -3
        assert gga.LIB.gga_workspace_bytes(ctypes.byref(cfgx), 1) == 0
    # sides without a resident variant need the workspace: a missing one is an argument error
    cfg160 = gga.make_cfg(160, 10, 1)
    assert gga.LIB.gga_simulate(ctypes.byref(prm), ctypes.byref(cfg160), n, n, n, 1, 1, n, 0, n, n, n, n) == -1
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


def test_mlp_work_layout_fits_the_work_buffer(gga):
    """The work-buffer views the gradient tests read lie inside
    gga_mlp_work_bytes(B), in order, 256-byte aligned and disjoint."""
    for B in (0, 1, 300, 16600):
        off = (ctypes.c_size_t * 12)()
        assert gga.LIB.gga_mlp_work_layout(B, off) == 0
        sizes = [2 * B * 128] + [4 * B * 512] * 3 + [2 * B * 512] * 3 + [4 * B] * 2 + [2 * B * 512] * 2 + [4 * 64 * 513]
        at = 0
        for o, n in zip(off, sizes):
            assert o == at and o % 256 == 0
            at = o + gga._align256(n)
        assert at == gga.LIB.gga_mlp_work_bytes(B)
    assert gga.LIB.gga_mlp_work_layout(-1, off) == -1
    assert gga.LIB.gga_mlp_work_layout(4, None) == -1


def test_variant_table_and_choices(gga):
    vs = gga.variants()
    assert [v[1] for v in vs] == [64, 64, 128, 128, 128, 256, 256, 64, 64, 96, 96, 160, 160, 192, 192, 224, 224, 96,
                                  160, 160, 192, 192, 160, 192, 192]
    assert [v[2] for v in vs] == [False, True, False, False, True, True, True, False, False,
                                  False, False, True, True, True, True, True, True, True, True, True, True, True,
                                  True, True, True]
    assert gga.get_variant(64) == 0 and gga.get_variant(128) == 2 and gga.get_variant(256) == 6
    assert [gga.get_variant(L) for L in (96, 160, 192, 224)] == [9, 22, 24, 16]
    assert gga.get_variant(128, resident_only=True) == 2 and gga.get_variant(96, resident_only=True) == 9
    for L in (160, 192, 224, 256):
        with pytest.raises(gga.GGAError):
            gga.get_variant(L, resident_only=True)          # no resident form above 128
    with pytest.raises(gga.GGAError):
        gga.get_variant(80)                                  # not a multiple of 32
    with pytest.raises(gga.GGAError):
        gga.set_variant(64, 2)                               # a variant of another side
    gga.set_variant(128, 4)
    assert gga.get_variant(128) == 4 and gga.get_variant(128, resident_only=True) == 2
    gga.set_variant(128, 3)
    assert gga.get_variant(128) == 3 and gga.get_variant(128, resident_only=True) == 3
    gga.set_variant(128, 2)
    assert gga.LIB.gga_variant_side(99) == -1 and gga.LIB.gga_variant_is_slab(-1) == -1


def _uneven_bytes(gga, lattice, horizon, K, R):
    lat = np.ascontiguousarray(lattice, np.int32)
    hor = np.ascontiguousarray(horizon, np.int32)
    return gga.LIB.gga_uneven_workspace_bytes(lat.ctypes.data_as(ctypes.c_void_p), hor.ctypes.data_as(ctypes.c_void_p),
                                              len(lat), K, R, 10)


def test_uneven_workspace_holds_two_states_per_slab_instance(gga):
    state = 256 * 256 * 14                                   # 3 float fields + one uint16 word per site
    small = _uneven_bytes(gga, [64, 128, 64], [10, 20, 30], 8, 4)
    big = _uneven_bytes(gga, [64, 128, 256], [10, 20, 30], 8, 4)
    assert 0 < small < 1 << 20
    assert big - small >= 2 * 4 * state - (1 << 20) and big >= 2 * 4 * state
    # a slab choice for 128 needs state buffers too
    gga.set_variant(128, 4)
    try:
        assert _uneven_bytes(gga, [64, 128, 64], [10, 20, 30], 8, 4) >= 2 * 4 * 128 * 128 * 14
    finally:
        gga.set_variant(128, 2)
    assert _uneven_bytes(gga, [64, 96], [10, 10], 8, 1) > 0      # 96 is resident: lists and tables only
    assert _uneven_bytes(gga, [64, 96], [10, 10], 8, 1) < 1 << 20
    assert _uneven_bytes(gga, [64, 160], [10, 10], 8, 1) >= 2 * 160 * 160 * 14
    # teams hold at most 128 instances of a slab side at once; one launch per step holds all
    lat, hor = [256] * 50, [10] * 50
    try:
        assert 2 * 128 * 256 * 256 * 14 <= _uneven_bytes(gga, lat, hor, 8, 4) < 2 * 129 * 256 * 256 * 14
        gga.set_team_options(False)
        assert _uneven_bytes(gga, lat, hor, 8, 4) >= 2 * 200 * 256 * 256 * 14
    finally:
        gga.set_team_options(True)
    assert _uneven_bytes(gga, [64, 80], [10, 10], 8, 1) == 0     # unsupported side
    assert _uneven_bytes(gga, [64, 64], [10, -1], 8, 1) == 0     # negative horizon


def test_uneven_argument_errors_before_any_launch(gga):
    p = gga.make_params(gga.load_model())
    cfg = gga.make_cfg(64, 0, 1)
    fake = ctypes.c_void_p(0x1000)
    lat = np.array([64, 80], np.int32)
    hor = np.array([5, 5], np.int32)
    rc = gga.LIB.gga_simulate_uneven(ctypes.byref(p), ctypes.byref(cfg), fake, fake, fake, 2, 1,
                                     lat.ctypes.data_as(ctypes.c_void_p), hor.ctypes.data_as(ctypes.c_void_p),
                                     fake, 1 << 30, fake, fake, None)
    assert rc == -3
    lat[1] = 64
    rc = gga.LIB.gga_simulate_uneven(ctypes.byref(p), ctypes.byref(cfg), fake, fake, fake, 2, 1,
                                     lat.ctypes.data_as(ctypes.c_void_p), hor.ctypes.data_as(ctypes.c_void_p),
                                     fake, 16, fake, fake, None)
    assert rc == -1                                           # workspace too small
    rc = gga.LIB.gga_state_run_variant(ctypes.byref(p), ctypes.byref(cfg), 5, fake, fake, fake, 2, 1, 0, 1,
                                       fake, fake, fake, fake, fake, 1 << 20, fake, None)
    assert rc == -1                                           # a 256 variant on a 64 lattice


def test_quasi3d_arguments_are_checked_before_any_launch(gga):
    p = gga.make_params(gga.load_model())
    fake, odd = ctypes.c_void_p(0x1000), ctypes.c_void_p(0x1008)
    ws = gga.LIB.gga_q3_workspace_bytes(128, 8, 4, 2, 3)
    # event table, then per instance and site: fields twice, reaction term, the
    # EMPTY, targeted (two) and proposer masks, the 2-bit slot states, and per
    # slot a word, a 64-bit key and a 32-bit proposal
    per = 128 * 128 * (12 * 2 + 4 + 4 * 4 + 8 + 8 * (2 + 8 + 4))
    assert per * 8 <= ws <= per * 8 + 12 * 256 + 4 * 3 * 24
    for L, C in ((128, 0), (128, 33), (4, 1), (1024, 8)):
        assert gga.LIB.gga_q3_workspace_bytes(L, C, 4, 2, 3) == 0
    call = lambda cfg, C, ws_ptr, nbytes: gga.LIB.gga_simulate_q3(
        ctypes.byref(p), ctypes.byref(cfg), C, fake, fake, fake, 4, 3, ws_ptr, nbytes, fake, fake, None, None)
    cfg = gga.make_cfg(128, 10, 2)
    assert call(cfg, 0, fake, ws) == -1                           # no slots
    assert call(cfg, 33, fake, ws) == -1                          # too many slots
    assert call(cfg, 8, fake, ws - 1) == -1                       # workspace too small
    assert call(cfg, 8, odd, ws) == -1                            # misaligned workspace
    assert call(gga.make_cfg(4, 10, 2), 1, fake, ws) == -3        # lattice too small
    assert call(gga.make_cfg(512, 10, 2), 64, fake, ws) == -1
    assert call(gga.make_cfg(128, 10, 2, substeps=65), 8, fake, ws) == -3
    rc = gga.LIB.gga_q3_run(ctypes.byref(p), ctypes.byref(cfg), 8, fake, fake, fake, 4, 3, (1 << 30) - 4, 5, fake,
                            fake, fake, ws, fake, None, None)
    assert rc == -1                                               # n0 + nsteps beyond 2^30
    bad = gga.make_params(dict(gga.load_model(), mitotic_death=2))
    assert gga.LIB.gga_q3_init(ctypes.byref(bad), ctypes.byref(cfg), 8, 4, fake, fake, None) == -5


def test_ga_operator_settings_are_checked_before_any_launch(gga):
    fake = ctypes.c_void_p(0x1000)
    a = gga.make_alphabet(0.5, [1, 2, 3, 4, 5], list(range(6, 61, 6)), 10, 10, 20.0)
    for kw in (dict(selection="rank", q=0.0), dict(selection="truncation", trunc_frac=1.5),
               dict(selection="roulette", roulette_base=float("inf"))):
        g = gga.make_ga(**kw)
        rc = gga.LIB.gga_ga_breed(ctypes.byref(g), ctypes.byref(a), fake, fake, fake, 16, 10, fake, fake, fake,
                                  fake, fake, None)
        assert rc == -1, kw
    g = gga.make_ga()
    g.selection = 7
    assert gga.LIB.gga_ga_breed(ctypes.byref(g), ctypes.byref(a), fake, fake, fake, 16, 10, fake, fake, fake,
                                fake, fake, None) == -1
    g = gga.make_ga(mutation=("gene", "swap", "raise"), crossover="uniform")
    assert g.mutation == 7 and g.crossover == 3


def test_slot_ga_settings_are_checked_before_any_launch(gga):
    """The slot GA's settings, sizes and pointers are refused on the host."""
    fake = ctypes.c_void_p(0x1000)
    g = gga.make_ga()
    ok = gga.make_slots()

    def breed(sc, ga=g, N=16, next_=ctypes.c_void_p(0x2000)):
        return gga.LIB.gga_slots_breed(ctypes.byref(ga), ctypes.byref(sc), fake, fake, N, fake, fake, fake, next_,
                                       None)

    for field, value in (("S", 0), ("S", 257), ("g_min", 0), ("g_min", 121), ("dmax_q", 0), ("dmax_q", 256),
                         ("cap_q", -1), ("cap_q", 65536), ("mutation", 16), ("reserved", 1),
                         ("quantum", 0.0), ("quantum", float("nan"))):
        sc = gga.make_slots()
        setattr(sc, field, value)
        assert breed(sc) == -1, field
    sc = gga.make_slots()
    sc.struct_size = 4
    assert breed(sc) == -2
    assert breed(ok, N=1) == -1                                   # a population of at least 2
    assert breed(ok, next_=fake) == -1                            # next population may not alias the current one
    gm = gga.make_ga(mutation=("swap",))
    assert breed(ok, ga=gm) == -1                                 # operators of the slot GA live in gga_slot_cfg
    for K in (0, 65):
        assert gga.LIB.gga_slots_decode(ctypes.byref(ok), fake, 4, K, fake, fake, fake, None) == -1
        assert gga.LIB.gga_slots_encode(ctypes.byref(ok), fake, fake, fake, 4, K, fake, None) == -1
    assert gga.LIB.gga_slots_decode(ctypes.byref(ok), None, 4, 8, fake, fake, fake, None) == -1
    assert gga.LIB.gga_slots_workspace_bytes(40, 8, 0) == 0
    assert gga.LIB.gga_slots_workspace_bytes(40, 8, 20) >= gga.LIB.gga_ga_workspace_bytes(40, 8) + 2 * 40 * 20 * 4
    # a run needs K >= ceil(S / g_min) fraction slots and a cap within the simulation's dose cap
    params = gga.make_params(gga.load_model())
    cfg = gga.make_cfg(L=64, horizon=24, R=2)
    big = ctypes.c_size_t(1 << 30)

    def run(sc, K):
        return gga.LIB.gga_slots_run(ctypes.byref(params), ctypes.byref(cfg), ctypes.byref(g), ctypes.byref(sc),
                                     fake, ctypes.c_void_p(0x3000), 16, K, 0, 1, 0, fake, big, fake, None, None,
                                     None, None)

    assert run(ok, 19) == -1
    capped = gga.make_slots(cap_q=80)                               # 20 Gy against a 10 Gy cap
    cfg.dose_cap = 10.0
    assert run(capped, 20) == -1
    assert gga.make_slots(mutation=("swap", "split", "time", "value")).mutation == 15


def test_mlp_buffers_must_be_16_byte_aligned(gga):
    """Net, work and screened-GA workspace pointers off a 16-byte boundary are
    refused before any launch (the MLP kernels load and store 16 bytes at a time)."""
    ok, off = ctypes.c_void_p(0x10000), ctypes.c_void_p(0x10008)
    B, K = 4, 10
    wb = gga.LIB.gga_mlp_work_bytes(B)
    assert gga.LIB.gga_mlp_init(off, 1, None) == -1
    assert gga.LIB.gga_mlp_set_norm(off, ok, 4, None) == -1
    assert gga.LIB.gga_mlp_predict(off, ok, ok, ok, B, K, ok, wb, ok, None) == -1
    assert gga.LIB.gga_mlp_predict(ok, ok, ok, ok, B, K, off, wb, ok, None) == -1
    assert gga.LIB.gga_mlp_grad(ok, ok, ok, ok, ok, B, K, off, wb, None, None) == -1
    assert gga.LIB.gga_mlp_train_step(off, ok, ok, ok, ok, B, K, 1, ctypes.c_float(1e-3), ok, wb, None,
                                      None) == -1


def test_measure_peaks_checks_its_buffer_before_any_launch(gga):
    d = ctypes.c_double()
    ok, off = ctypes.c_void_p(0x100000), ctypes.c_void_p(0x100008)
    big = (256 << 20) + 256
    assert gga.LIB.gga_measure_peaks(ok, big - 16, ctypes.byref(d), ctypes.byref(d), ctypes.byref(d), None) == -1
    assert gga.LIB.gga_measure_peaks(off, big, ctypes.byref(d), ctypes.byref(d), ctypes.byref(d), None) == -1
    assert gga.LIB.gga_measure_peaks(ok, big, None, ctypes.byref(d), ctypes.byref(d), None) == -1
    assert gga.LIB.gga_measure_peaks(None, big, ctypes.byref(d), ctypes.byref(d), ctypes.byref(d), None) == -1


def test_params_from_json_reads_the_model_file(gga, tmp_path):
    """The library's own reader gives the same struct as the binding's, byte for
    byte; malformed files, missing keys, non-integral integers and refused
    values return the documented codes and leave the struct unwritten."""
    import json
    import os
    path = os.path.join(gga.DATA, "model_default.json")
    got = gga.params_from_json(path)
    want = gga.make_params(gga.load_model())
    assert bytes(got) == bytes(want)
    p = gga.Params()
    p.struct_size = ctypes.sizeof(gga.Params)
    before = bytes(p)
    bad = tmp_path / "bad.json"
    model = gga.load_model()
    cases = [("{ not json", -1), (json.dumps({k: v for k, v in model.items() if k != "kappa"}), -5),
             (json.dumps(dict(model, T_min=12.5)), -5), (json.dumps(dict(model, lambda_=1)), 0),
             (json.dumps(dict(model, **{"lambda": [0.3, 0.1, 0.1]})), -5), (json.dumps(dict(model, m=[1, 2])), -5),
             (json.dumps(model) + " trailing", -1),
             (json.dumps(dict(model, repair_half_time=-1.0)), -5),
             (json.dumps(dict(model, oer_max=0.5)), -5), (json.dumps(dict(model, oer_k=0.0)), -5),
             (json.dumps(dict(model, oer_max=3.0, ghost=[0.0, 1.0, 0.0])), -5),
             (json.dumps(dict(model, oer_max=3.0, oer_k=0.1)), 0),
             (json.dumps(dict(model, mitotic_death=2)), -5), (json.dumps(dict(model, mitotic_death=1)), 0),
             (json.dumps(dict(model, repair_half_time=float("inf"))), -1)]
    for text, rc in cases:
        bad.write_text(text)
        assert gga.LIB.gga_params_from_json(str(bad).encode(), ctypes.byref(p)) == rc, text[:40]
        if rc:
            assert bytes(p) == before
        p = gga.Params()
        p.struct_size = ctypes.sizeof(gga.Params)
    # the repair half-time is optional (0 when absent) and read when present
    bad.write_text(json.dumps({k: v for k, v in model.items() if k != "repair_half_time"}))
    assert gga.LIB.gga_params_from_json(str(bad).encode(), ctypes.byref(p)) == 0 and p.repair_half_time == 0.0
    bad.write_text(json.dumps(dict(model, repair_half_time=2.5)))
    assert gga.LIB.gga_params_from_json(str(bad).encode(), ctypes.byref(p)) == 0 and p.repair_half_time == 2.5
    assert bytes(p) == bytes(gga.make_params(dict(model, repair_half_time=2.5)))
    # the oxygen effect: off (1, 0.05) when absent, read when present
    bad.write_text(json.dumps({k: v for k, v in model.items() if k not in ("oer_max", "oer_k")}))
    assert gga.LIB.gga_params_from_json(str(bad).encode(), ctypes.byref(p)) == 0
    assert (p.oer_max, p.oer_k) == (1.0, 0.05)
    bad.write_text(json.dumps(dict(model, oer_max=2.5, oer_k=0.02)))
    assert gga.LIB.gga_params_from_json(str(bad).encode(), ctypes.byref(p)) == 0
    assert bytes(p) == bytes(gga.make_params(dict(model, oer_max=2.5, oer_k=0.02)))
    assert gga.LIB.gga_params_from_json(b"/nonexistent/model.json", ctypes.byref(p)) == -1
    p.struct_size = 4
    assert gga.LIB.gga_params_from_json(path.encode(), ctypes.byref(p)) == -2


def test_simulate_workspace_sizes(gga):
    """gga_workspace_bytes: none for the resident sides; for the slab sides the
    event table and two state buffers, of at most 128 instances as teams (one
    cooperative launch's worth, plus the instance list and step counts) or of
    every instance with one launch per step."""
    for L in (64, 96, 128):
        assert gga.workspace_bytes(gga.make_cfg(L, 10, 4), 100) == 0
    table = 100 * (8 + 20 * 64)
    try:
        for teams, rows in ((True, 128), (False, 400)):
            gga.set_team_options(teams)
            for L in (160, 192, 224, 256):
                cfg = gga.make_cfg(L, 10, 4)
                n = gga.workspace_bytes(cfg, 100)
                state = 2 * rows * L * L * 14
                extra = table + (400 * 4 + 128 * 16 * 4 if teams else 0) + 8 * 256
                assert state <= n <= state + extra, (teams, L, n)
                assert gga.workspace_bytes(cfg, 0) < 1 << 14
                small = gga.workspace_bytes(cfg, 2)                       # 8 instances either way
                assert 2 * 8 * L * L * 14 <= small <= 2 * 8 * L * L * 14 + 2 * (1 << 14)
    finally:
        gga.set_team_options(True)
    bad = gga.make_cfg(160, 10, 4)
    bad.struct_size = 3
    assert gga.workspace_bytes(bad, 10) == 0 and gga.workspace_bytes(gga.make_cfg(160, 10, 4), -1) == 0


def test_noalloc_checks_its_scratch_before_any_launch(gga):
    """gga_simulate_noalloc: a batch whose workspace exceeds the fixed scratch
    is refused with GGA_E_SCRATCH, and a bad cfg with GGA_E_ABI / GGA_E_ARG,
    before anything touches a device."""
    p = gga.make_params(gga.load_model())
    fake = ctypes.c_void_p(0x1000)
    cfg = gga.make_cfg(256, 10, 1)
    assert gga.workspace_bytes(cfg, 36) <= gga.NOALLOC_SCRATCH_BYTES < gga.workspace_bytes(cfg, 37)
    rc = gga.LIB.gga_simulate_noalloc(ctypes.byref(p), ctypes.byref(cfg), fake, fake, fake, 37, 3, fake, fake,
                                      None, None)
    assert rc == gga.E_SCRATCH and "scratch" in gga.LIB.gga_strerror(rc).decode()
    bad = gga.make_cfg(256, 10, 1)
    bad.struct_size = 3
    assert gga.LIB.gga_simulate_noalloc(ctypes.byref(p), ctypes.byref(bad), fake, fake, fake, 1, 3, fake, fake,
                                        None, None) == -2
    assert gga.LIB.gga_simulate_noalloc(ctypes.byref(p), None, fake, fake, fake, 1, 3, fake, fake, None, None) == -1
