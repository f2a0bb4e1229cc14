"""MI355X (gfx950) simulator of tumour growth under fractionated radiotherapy.

Python binding of the C ABI in include/gga.h (libgga.so, built in-tree by
``python -m paper_2303_08123_amd.build``).  The binding only marshals
arguments: every step of the simulation runs in the library's HIP kernels.
PyTorch provides device memory and streams.  Importing this package without
the built library raises, there is no other code path.
"""
import ctypes
import json
import os

import numpy as np
import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libgga.so")
DATA = os.path.join(HERE, "data")

GGA_OK = 0
KMAX = 64
ERRORS = {-1: "GGA_E_ARG", -2: "GGA_E_ABI", -3: "GGA_E_UNSUPPORTED", -4: "GGA_E_HIP",
          -5: "GGA_E_PARAM", -6: "GGA_E_ALPHABET", -7: "GGA_E_SCRATCH"}
E_SCRATCH = -7
NOALLOC_SCRATCH_BYTES = 64 << 20     # GGA_NOALLOC_SCRATCH_BYTES
PROTO_OK, PROTO_NFRAC, PROTO_DOSE, PROTO_CAP, PROTO_GAP = 0, 1, 2, 3, 4


class Params(ctypes.Structure):
    _fields_ = [
        ("struct_size", ctypes.c_uint32),
        ("lambda_", ctypes.c_float * 3), ("kappa", ctypes.c_float * 3),
        ("ghost", ctypes.c_float * 3), ("init", ctypes.c_float * 3),
        ("activity", ctypes.c_float * 4),
        ("theta_O_quiesce", ctypes.c_float), ("theta_G_quiesce", ctypes.c_float),
        ("theta_O_death", ctypes.c_float), ("theta_G_death", ctypes.c_float),
        ("theta_H_death", ctypes.c_float),
        ("T_min", ctypes.c_int32), ("T_lys", ctypes.c_int32), ("A0", ctypes.c_int32),
        ("seed_radius", ctypes.c_int32), ("class_age", ctypes.c_int32 * 2),
        ("P_div", ctypes.c_double), ("alpha", ctypes.c_double), ("beta", ctypes.c_double),
        ("m", ctypes.c_double * 4), ("repair_half_time", ctypes.c_double),
        ("oer_max", ctypes.c_double), ("oer_k", ctypes.c_double),
        ("mitotic_death", ctypes.c_int32), ("reserved", ctypes.c_int32),
    ]


class SimCfg(ctypes.Structure):
    _fields_ = [
        ("struct_size", ctypes.c_uint32), ("L", ctypes.c_int32), ("horizon", ctypes.c_int32),
        ("substeps", ctypes.c_int32), ("R", ctypes.c_int32), ("flags", ctypes.c_uint32),
        ("seed", ctypes.c_uint64), ("dose_cap", ctypes.c_double),
    ]


class Alphabet(ctypes.Structure):
    _fields_ = [
        ("struct_size", ctypes.c_uint32), ("n_dose", ctypes.c_int32), ("n_gap", ctypes.c_int32),
        ("kmin", ctypes.c_int32), ("kmax", ctypes.c_int32),
        ("dose_quantum", ctypes.c_float), ("cap", ctypes.c_float),
        ("dose_q", ctypes.c_int32 * 64), ("gaps", ctypes.c_int32 * 64),
    ]


class SgaCfg(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_uint32), ("n_candidates", ctypes.c_int32),
                ("n_simulated", ctypes.c_int32), ("screen", ctypes.c_int32), ("refine_steps", ctypes.c_int32),
                ("refine_lr", ctypes.c_float)]


class GaCfg(ctypes.Structure):
    _fields_ = [
        ("struct_size", ctypes.c_uint32), ("n_elite", ctypes.c_int32), ("tournament_k", ctypes.c_int32),
        ("p_cross", ctypes.c_double), ("p_mut", ctypes.c_double), ("seed", ctypes.c_uint64),
        ("selection", ctypes.c_int32), ("crossover", ctypes.c_int32), ("mutation", ctypes.c_int32),
        ("reserved", ctypes.c_int32), ("q", ctypes.c_double), ("trunc_frac", ctypes.c_double),
        ("roulette_base", ctypes.c_double),
    ]


class SlotCfg(ctypes.Structure):
    _fields_ = [
        ("struct_size", ctypes.c_uint32), ("S", ctypes.c_int32), ("g_min", ctypes.c_int32),
        ("dmax_q", ctypes.c_int32), ("cap_q", ctypes.c_int32), ("mutation", ctypes.c_int32),
        ("quantum", ctypes.c_float), ("reserved", ctypes.c_int32),
    ]


SELECTIONS = {"tournament": 0, "rank": 1, "roulette": 2, "truncation": 3}
CROSSOVERS = {"one_point": 0, "middle": 1, "two_point": 2, "uniform": 3}
MUTATIONS = {"gene": 1, "swap": 2, "raise": 4}
SLOT_MUTATIONS = {"swap": 1, "split": 2, "time": 4, "value": 8}
SLOTS_MAX = 256


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with "
                          "`python paper_2303_08123_amd/build.py` (hipcc, gfx950)")
    lib = ctypes.CDLL(LIB_PATH)
    vp, i32, i64, u64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64
    sig = {
        "gga_version": ([], ctypes.c_int),
        "gga_strerror": ([ctypes.c_int], ctypes.c_char_p),
        "gga_last_hip_error": ([], ctypes.c_int),
        "gga_validate": ([vp, vp, vp, vp, i32, i32, vp], ctypes.c_int),
        "gga_population_random": ([vp, i32, i32, u64, vp, vp, vp, vp], ctypes.c_int),
        "gga_workspace_bytes": ([vp, i32], ctypes.c_size_t),
        "gga_simulate": ([vp, vp, vp, vp, vp, i32, i32, vp, ctypes.c_size_t, vp, vp, vp, vp], ctypes.c_int),
        "gga_simulate_noalloc": ([vp, vp, vp, vp, vp, i32, i32, vp, vp, vp, vp], ctypes.c_int),
        "gga_state_init": ([vp, vp, i32, vp, vp, vp], ctypes.c_int),
        "gga_state_run": ([vp, vp, vp, vp, vp, i32, i32, i32, i32, vp, vp, vp, vp, vp], ctypes.c_int),
        "gga_philox_fill": ([vp, u64, vp, i64, vp], ctypes.c_int),
        "gga_ga_breed": ([vp, vp, vp, vp, vp, i32, i32, vp, vp, vp, vp, vp, vp], ctypes.c_int),
        "gga_ga_workspace_bytes": ([i32, i32], ctypes.c_size_t),
        "gga_ga_set_generation": ([vp, i32, vp], ctypes.c_int),
        "gga_ga_generation": ([vp, vp, vp, vp, vp, vp, vp, i32, i32, vp, vp, vp, ctypes.c_size_t, vp, i32,
                               i32, vp], ctypes.c_int),
        "gga_ga_run": ([vp, vp, vp, vp, vp, vp, vp, vp, vp, i32, i32, i32, i32, i32, vp, ctypes.c_size_t, vp,
                        vp, vp, vp, vp], ctypes.c_int),
        "gga_mlp_net_bytes": ([], ctypes.c_size_t),
        "gga_mlp_work_bytes": ([i32], ctypes.c_size_t),
        "gga_mlp_work_layout": ([i32, vp], ctypes.c_int),
        "gga_mlp_init": ([vp, u64, vp], ctypes.c_int),
        "gga_mlp_set_norm": ([vp, vp, i32, vp], ctypes.c_int),
        "gga_mlp_predict": ([vp, vp, vp, vp, i32, i32, vp, ctypes.c_size_t, vp, vp], ctypes.c_int),
        "gga_mlp_grad": ([vp, vp, vp, vp, vp, i32, i32, vp, ctypes.c_size_t, vp, vp], ctypes.c_int),
        "gga_mlp_train_step": ([vp, vp, vp, vp, vp, i32, i32, i32, ctypes.c_float, vp, ctypes.c_size_t, vp, vp],
                               ctypes.c_int),
        "gga_mlp_gemm": ([i32, i32, i32, vp, i32, vp, i32, vp, vp], ctypes.c_int),
        "gga_sga_workspace_bytes": ([i32, i32, i32, i32, i32], ctypes.c_size_t),
        "gga_sga_init": ([vp, vp, vp, vp, vp, vp, i32, i32, vp, ctypes.c_size_t, vp], ctypes.c_int),
        "gga_sga_generation": ([vp, vp, vp, vp, vp, vp, vp, vp, vp, i32, i32, vp, ctypes.c_size_t, vp, i32, vp],
                               ctypes.c_int),
        "gga_sga_run": ([vp, vp, vp, vp, vp, vp, vp, vp, vp, i32, i32, i32, i32, i32, vp, ctypes.c_size_t, vp, vp,
                         vp, vp, vp], ctypes.c_int),
        "gga_simulate_library": ([vp, vp, vp, vp, vp, i32, i32, vp, vp, i32, vp, vp, vp], ctypes.c_int),
        "gga_variant_count": ([], ctypes.c_int),
        "gga_variant_side": ([i32], i32),
        "gga_variant_is_slab": ([i32], i32),
        "gga_variant_name": ([i32], ctypes.c_char_p),
        "gga_get_variant": ([i32, i32], ctypes.c_int),
        "gga_set_variant": ([i32, i32], ctypes.c_int),
        "gga_uneven_workspace_bytes": ([vp, vp, i32, i32, i32, i32], ctypes.c_size_t),
        "gga_set_team_options": ([i32, i32], ctypes.c_int),
        "gga_simulate_uneven": ([vp, vp, vp, vp, vp, i32, i32, vp, vp, vp, ctypes.c_size_t, vp, vp, vp],
                                ctypes.c_int),
        "gga_event_table_bytes": ([i32, i32], ctypes.c_size_t),
        "gga_state_run_variant": ([vp, vp, i32, vp, vp, vp, i32, i32, i32, i32, vp, vp, vp, vp, vp,
                                   ctypes.c_size_t, vp, vp], ctypes.c_int),
        "gga_autotune_workspace_bytes": ([i32, i32, i32, i32, i32, i32], ctypes.c_size_t),
        "gga_autotune": ([vp, vp, vp, vp, vp, i32, i32, vp, ctypes.c_size_t, vp, vp, vp, vp], ctypes.c_int),
        "gga_measure_peaks": ([vp, ctypes.c_size_t, vp, vp, vp, vp], ctypes.c_int),
        "gga_params_from_json": ([ctypes.c_char_p, vp], ctypes.c_int),
        "gga_slots_breed": ([vp, vp, vp, vp, i32, vp, vp, vp, vp, vp], ctypes.c_int),
        "gga_slots_decode": ([vp, vp, i32, i32, vp, vp, vp, vp], ctypes.c_int),
        "gga_slots_encode": ([vp, vp, vp, vp, i32, i32, vp, vp], ctypes.c_int),
        "gga_slots_workspace_bytes": ([i32, i32, i32], ctypes.c_size_t),
        "gga_slots_run": ([vp, vp, vp, vp, vp, vp, i32, i32, i32, i32, i32, vp, ctypes.c_size_t, vp, vp, vp, vp,
                           vp], ctypes.c_int),
        "gga_q3_workspace_bytes": ([i32, i32, i32, i32, i32], ctypes.c_size_t),
        "gga_q3_init": ([vp, vp, i32, i32, vp, vp, vp], ctypes.c_int),
        "gga_q3_run": ([vp, vp, i32, vp, vp, vp, i32, i32, i32, i32, vp, vp, vp, ctypes.c_size_t, vp, vp, vp],
                       ctypes.c_int),
        "gga_simulate_q3": ([vp, vp, i32, vp, vp, vp, i32, i32, vp, ctypes.c_size_t, vp, vp, vp, vp],
                            ctypes.c_int),
    }
    for name, (args, res) in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    return lib


LIB = _load()
EXPORTS = ("gga_version", "gga_strerror", "gga_last_hip_error", "gga_validate",
           "gga_population_random", "gga_workspace_bytes", "gga_simulate", "gga_simulate_noalloc", "gga_state_init", "gga_state_run",
           "gga_philox_fill", "gga_ga_breed", "gga_ga_workspace_bytes", "gga_ga_set_generation",
           "gga_ga_generation", "gga_ga_run", "gga_mlp_net_bytes", "gga_mlp_work_bytes", "gga_mlp_work_layout",
           "gga_mlp_init",
           "gga_mlp_set_norm", "gga_mlp_predict", "gga_mlp_grad", "gga_mlp_train_step", "gga_mlp_gemm",
           "gga_sga_workspace_bytes", "gga_sga_init", "gga_sga_generation", "gga_sga_run",
           "gga_variant_count", "gga_variant_side", "gga_variant_is_slab", "gga_variant_name", "gga_get_variant",
           "gga_set_variant", "gga_set_team_options", "gga_uneven_workspace_bytes", "gga_simulate_uneven", "gga_event_table_bytes",
           "gga_state_run_variant", "gga_autotune_workspace_bytes", "gga_autotune", "gga_simulate_library",
           "gga_measure_peaks", "gga_params_from_json", "gga_slots_breed", "gga_slots_decode",
           "gga_slots_encode", "gga_slots_workspace_bytes", "gga_slots_run", "gga_q3_workspace_bytes",
           "gga_q3_init", "gga_q3_run", "gga_simulate_q3")


class GGAError(RuntimeError):
    def __init__(self, msg, code=None):
        super().__init__(msg)
        self.code = code


def _check(rc):
    if rc != GGA_OK:
        msg = LIB.gga_strerror(rc).decode()
        if rc == -4:
            msg += f" (hipError {LIB.gga_last_hip_error()})"
        raise GGAError(f"{ERRORS.get(rc, rc)}: {msg}", rc)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


def _stream(stream):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def version():
    return LIB.gga_version()


# ---------------------------------------------------------------- parameters

def load_model(name="model_default"):
    with open(os.path.join(DATA, name + ".json")) as fh:
        return json.load(fh)


def make_params(d):
    p = Params()
    p.struct_size = ctypes.sizeof(Params)
    p.lambda_[:] = [float(v) for v in d["lambda"]]
    p.kappa[:] = [float(v) for v in d["kappa"]]
    p.ghost[:] = [float(v) for v in d["ghost"]]
    p.init[:] = [float(v) for v in d["init_fields"]]
    p.activity[:] = [float(v) for v in d["activity"]]
    p.theta_O_quiesce = d["theta_O_quiesce"]
    p.theta_G_quiesce = d["theta_G_quiesce"]
    p.theta_O_death = d["theta_O_death"]
    p.theta_G_death = d["theta_G_death"]
    p.theta_H_death = d["theta_H_death"]
    p.T_min, p.T_lys, p.A0 = int(d["T_min"]), int(d["T_lys"]), int(d["A0"])
    p.seed_radius = int(d["seed_radius"])
    p.class_age[:] = [int(v) for v in d["class_age"]]
    p.P_div, p.alpha, p.beta = float(d["P_div"]), float(d["alpha"]), float(d["beta"])
    p.m[:] = [float(v) for v in d["m"]]
    p.repair_half_time = float(d.get("repair_half_time", 0.0))
    p.oer_max, p.oer_k = float(d.get("oer_max", 1.0)), float(d.get("oer_k", 0.05))
    p.mitotic_death = int(d.get("mitotic_death", 0))
    return p


def params_from_json(path):
    """gga_params read by the library from a model file (gga_params_from_json)."""
    p = Params()
    p.struct_size = ctypes.sizeof(Params)
    _check(LIB.gga_params_from_json(os.fsencode(path), ctypes.byref(p)))
    return p


SIM_HALF_HOUR = 1


def make_cfg(L, horizon, R, seed=0, substeps=10, dose_cap=20.0, half_hour=False):
    """Simulation settings; half_hour=True counts protocol delays in 30-minute
    units (GGA_SIM_HALF_HOUR)."""
    c = SimCfg()
    c.struct_size = ctypes.sizeof(SimCfg)
    c.L, c.horizon, c.substeps, c.R = int(L), int(horizon), int(substeps), int(R)
    c.flags, c.seed, c.dose_cap = SIM_HALF_HOUR if half_hour else 0, int(seed), float(dose_cap)
    return c


def make_alphabet(dose_quantum, dose_q, gaps, kmin, kmax, cap):
    a = Alphabet()
    a.struct_size = ctypes.sizeof(Alphabet)
    a.n_dose, a.n_gap = len(dose_q), len(gaps)
    a.kmin, a.kmax = int(kmin), int(kmax)
    a.dose_quantum, a.cap = float(dose_quantum), float(cap)
    for i, v in enumerate(dose_q):
        a.dose_q[i] = int(v)
    for i, v in enumerate(gaps):
        a.gaps[i] = int(v)
    return a


def _as_params(params):
    return params if isinstance(params, Params) else make_params(params)


# ---------------------------------------------------------------- calls

def validate(cfg, dose, gap, nfrac):
    """Host validator: per-protocol GGA_PROTO_* codes (numpy in, numpy out)."""
    dose = np.ascontiguousarray(dose, dtype=np.float32)
    gap = np.ascontiguousarray(gap, dtype=np.int32)
    nfrac = np.ascontiguousarray(nfrac, dtype=np.int32).reshape(-1)
    P = len(nfrac)
    K = dose.shape[1] if dose.ndim == 2 else 0
    status = np.zeros(P, dtype=np.int32)
    _check(LIB.gga_validate(ctypes.byref(cfg), dose.ctypes.data_as(ctypes.c_void_p),
                            gap.ctypes.data_as(ctypes.c_void_p), nfrac.ctypes.data_as(ctypes.c_void_p),
                            P, K, status.ctypes.data_as(ctypes.c_void_p)))
    return status


def population_random(alphabet, P, K, seed, device="cuda", stream=None):
    """Device-drawn random protocols: (dose[P, K] f32, gap[P, K] i32, nfrac[P] i32)."""
    dose = torch.empty((P, K), dtype=torch.float32, device=device)
    gap = torch.empty((P, K), dtype=torch.int32, device=device)
    nfrac = torch.empty((P,), dtype=torch.int32, device=device)
    _check(LIB.gga_population_random(ctypes.byref(alphabet), P, K, int(seed), _ptr(dose),
                                     _ptr(gap), _ptr(nfrac), _stream(stream)))
    return dose, gap, nfrac


def _protocols(dose, gap, nfrac):
    for t, dt in ((dose, torch.float32), (gap, torch.int32), (nfrac, torch.int32)):
        if not (t.is_cuda and t.dtype == dt and t.is_contiguous()):
            raise ValueError("protocol tensors must be contiguous CUDA tensors (f32, i32, i32)")
    P = nfrac.numel()
    K = dose.shape[1] if dose.dim() == 2 else 0
    if dose.shape != (P, K) or gap.shape != (P, K):
        raise ValueError("dose and gap must have shape [P, K]")
    return P, K


def workspace_bytes(cfg, P):
    """Device workspace gga_simulate needs (0 for the resident sides 64, 96, 128)."""
    return int(LIB.gga_workspace_bytes(ctypes.byref(cfg), int(P)))


def workspace(cfg, P, device="cuda"):
    """A workspace tensor for gga_simulate, or None when it needs none."""
    n = workspace_bytes(cfg, P)
    return torch.empty(n, dtype=torch.uint8, device=device) if n else None


def simulate(params, cfg, dose, gap, nfrac, traj=False, out=None, ws=None, stream=None):
    """Simulate every (protocol, replica) instance; returns (live[P, R], fitness[P], traj).
    Sides without a resident variant need a workspace (allocated here unless given)."""
    P, K = _protocols(dose, gap, nfrac)
    dev = dose.device
    if out is None:
        live = torch.empty((P, cfg.R), dtype=torch.int32, device=dev)
        fit = torch.empty((P,), dtype=torch.float32, device=dev)
        tr = torch.empty((P, cfg.R, cfg.horizon), dtype=torch.int32, device=dev) if traj else None
    else:
        live, fit, tr = out
    if ws is None:
        ws = workspace(cfg, P, dev)
    nws = 0 if ws is None else ws.numel() * ws.element_size()
    _check(LIB.gga_simulate(ctypes.byref(_as_params(params)), ctypes.byref(cfg), _ptr(dose), _ptr(gap),
                            _ptr(nfrac), P, K, _ptr(ws), nws, _ptr(live), _ptr(fit), _ptr(tr), _stream(stream)))
    return live, fit, tr


def simulate_noalloc(params, cfg, dose, gap, nfrac, traj=False, out=None, stream=None):
    """gga_simulate_noalloc: as simulate, with the library's fixed scratch in
    place of a workspace (the call itself allocates no device memory; the
    outputs are allocated here unless given)."""
    P, K = _protocols(dose, gap, nfrac)
    dev = dose.device
    if out is None:
        live = torch.empty((P, cfg.R), dtype=torch.int32, device=dev)
        fit = torch.empty((P,), dtype=torch.float32, device=dev)
        tr = torch.empty((P, cfg.R, cfg.horizon), dtype=torch.int32, device=dev) if traj else None
    else:
        live, fit, tr = out
    _check(LIB.gga_simulate_noalloc(ctypes.byref(_as_params(params)), ctypes.byref(cfg), _ptr(dose), _ptr(gap),
                                    _ptr(nfrac), P, K, _ptr(live), _ptr(fit), _ptr(tr), _stream(stream)))
    return live, fit, tr


def state_init(params, cfg, P, device="cuda", stream=None):
    """Initial states: (fields[P*R, 3, L, L] f32, cells[P*R, L, L] int16 holding uint16 words)."""
    n = P * cfg.R
    fields = torch.empty((n, 3, cfg.L, cfg.L), dtype=torch.float32, device=device)
    cells = torch.empty((n, cfg.L, cfg.L), dtype=torch.int16, device=device)
    _check(LIB.gga_state_init(ctypes.byref(_as_params(params)), ctypes.byref(cfg), P, _ptr(fields),
                              _ptr(cells), _stream(stream)))
    return fields, cells


def state_run(params, cfg, dose, gap, nfrac, n0, nsteps, fields, cells, traj=False, stream=None):
    """Advance states in place by nsteps from step n0; returns (live[P, R], traj)."""
    P, K = _protocols(dose, gap, nfrac)
    n = P * cfg.R
    if fields.shape != (n, 3, cfg.L, cfg.L) or fields.dtype != torch.float32 or not fields.is_contiguous():
        raise ValueError("fields must be a contiguous float32 [P*R, 3, L, L] tensor")
    if cells.shape != (n, cfg.L, cfg.L) or cells.dtype != torch.int16 or not cells.is_contiguous():
        raise ValueError("cells must be a contiguous int16 [P*R, L, L] tensor")
    live = torch.empty((P, cfg.R), dtype=torch.int32, device=dose.device)
    tr = torch.empty((P, cfg.R, max(nsteps, 0)), dtype=torch.int32, device=dose.device) if traj else None
    _check(LIB.gga_state_run(ctypes.byref(_as_params(params)), ctypes.byref(cfg), _ptr(dose), _ptr(gap),
                             _ptr(nfrac), P, K, int(n0), int(nsteps), _ptr(fields), _ptr(cells),
                             _ptr(live), _ptr(tr), _stream(stream)))
    return live, tr


def grow_library(params, L, n, days, seed=0, substeps=10, stream=None):
    """n untreated tumours grown from the seed disc for `days` days (replica
    streams 0 .. n-1 of protocol 0 under `seed`): (fields, cells) for
    simulate_library."""
    cfg = make_cfg(L, 24 * days, n, seed=seed, substeps=substeps)
    fields, cells = state_init(params, cfg, 1, stream=stream)
    z = torch.zeros((1, 1), dtype=torch.float32, device=fields.device)
    state_run(params, cfg, z, z.int(), torch.zeros(1, dtype=torch.int32, device=fields.device), 0, 24 * days,
              fields, cells, stream=stream)
    return fields, cells


def simulate_library(params, cfg, dose, gap, nfrac, lib_fields, lib_cells, stream=None):
    """Simulate each protocol's replica r from library tumour r mod n_lib;
    returns (live[P, R], fitness[P])."""
    P, K = _protocols(dose, gap, nfrac)
    n_lib = lib_fields.shape[0]
    if lib_fields.shape != (n_lib, 3, cfg.L, cfg.L) or lib_cells.shape != (n_lib, cfg.L, cfg.L):
        raise ValueError("library states must be [n, 3, L, L] fields and [n, L, L] cells")
    if not (lib_fields.is_contiguous() and lib_cells.is_contiguous()):
        raise ValueError("library states must be contiguous")
    live = torch.empty((P, cfg.R), dtype=torch.int32, device=dose.device)
    fit = torch.empty((P,), dtype=torch.float32, device=dose.device)
    _check(LIB.gga_simulate_library(ctypes.byref(_as_params(params)), ctypes.byref(cfg), _ptr(dose), _ptr(gap),
                                    _ptr(nfrac), P, K, _ptr(lib_fields), _ptr(lib_cells),
                                    n_lib, _ptr(live), _ptr(fit), _stream(stream)))
    return live, fit


def philox_fill(ctr, seed, stream=None):
    """Device Philox4x32-10 blocks for counters ctr[n, 4] (int32 tensor holding uint32)."""
    if not (ctr.is_cuda and ctr.dtype == torch.int32 and ctr.is_contiguous() and ctr.shape[-1] == 4):
        raise ValueError("ctr must be a contiguous int32 CUDA tensor [n, 4]")
    out = torch.empty_like(ctr)
    _check(LIB.gga_philox_fill(_ptr(ctr), int(seed), _ptr(out), ctr.shape[0], _stream(stream)))
    return out


# ---------------------------------------------------------------- kernel variants, uneven batches

def variants():
    """[(id, lattice side, slab form, name)] of the simulation kernel variants."""
    return [(v, int(LIB.gga_variant_side(v)), bool(LIB.gga_variant_is_slab(v)), LIB.gga_variant_name(v).decode())
            for v in range(LIB.gga_variant_count())]


def get_variant(L, resident_only=False):
    v = LIB.gga_get_variant(int(L), int(bool(resident_only)))
    _check(min(v, 0))
    return v


def set_variant(L, v):
    _check(LIB.gga_set_variant(int(L), int(v)))


def _host_i32(x, P, what):
    a = np.ascontiguousarray(np.broadcast_to(np.asarray(x, dtype=np.int32), (P,)))
    if a.shape != (P,):
        raise ValueError(f"{what} must hold one value per protocol")
    return a


def set_team_options(use_teams=True, spin_limit=1 << 21):
    """Test hook: slab groups as teams (default) or one launch per step; the
    teams' bounded wait in polls (negative: every wait fails)."""
    _check(LIB.gga_set_team_options(int(bool(use_teams)), int(spin_limit)))


def uneven_workspace(lattice, horizon, P, K, R, device="cuda", substeps=10):
    lat, hor = _host_i32(lattice, P, "lattice"), _host_i32(horizon, P, "horizon")
    n = LIB.gga_uneven_workspace_bytes(lat.ctypes.data_as(ctypes.c_void_p), hor.ctypes.data_as(ctypes.c_void_p),
                                       P, K, R, int(substeps))
    if n == 0 and P > 0:
        raise GGAError("no uneven plan: lattice sides must be multiples of 32 in 64 .. 256 and horizons >= 0")
    return torch.empty(int(n), dtype=torch.uint8, device=device)


def simulate_uneven(params, cfg, dose, gap, nfrac, lattice, horizon, ws=None, out=None, stream=None):
    """Simulate protocol p on a lattice[p] x lattice[p] lattice for horizon[p]
    steps (host arrays or scalars; cfg.L and cfg.horizon are not used).
    Returns (live[P, R], fitness[P])."""
    P, K = _protocols(dose, gap, nfrac)
    lat, hor = _host_i32(lattice, P, "lattice"), _host_i32(horizon, P, "horizon")
    if ws is None:
        ws = uneven_workspace(lat, hor, P, K, cfg.R, dose.device, substeps=cfg.substeps)
    if out is None:
        out = (torch.empty((P, cfg.R), dtype=torch.int32, device=dose.device),
               torch.empty((P,), dtype=torch.float32, device=dose.device))
    live, fit = out
    _check(LIB.gga_simulate_uneven(ctypes.byref(_as_params(params)), ctypes.byref(cfg), _ptr(dose), _ptr(gap),
                                   _ptr(nfrac), P, K, lat.ctypes.data_as(ctypes.c_void_p),
                                   hor.ctypes.data_as(ctypes.c_void_p), _ptr(ws), ws.numel(), _ptr(live), _ptr(fit),
                                   _stream(stream)))
    return live, fit


def state_run_variant(params, cfg, variant, dose, gap, nfrac, n0, nsteps, fields, cells, stream=None):
    """state_run with a given kernel variant (slab variants step through a second
    state buffer); advances (fields, cells) in place, returns live[P, R]."""
    P, K = _protocols(dose, gap, nfrac)
    live = torch.empty((P, cfg.R), dtype=torch.int32, device=dose.device)
    f2, c2 = torch.empty_like(fields), torch.empty_like(cells)
    ws = torch.empty(max(int(LIB.gga_event_table_bytes(P, K)), 1), dtype=torch.uint8, device=dose.device)
    _check(LIB.gga_state_run_variant(ctypes.byref(_as_params(params)), ctypes.byref(cfg), int(variant), _ptr(dose),
                                     _ptr(gap), _ptr(nfrac), P, K, int(n0), int(nsteps), _ptr(fields), _ptr(cells),
                                     _ptr(f2), _ptr(c2), _ptr(ws), ws.numel(), _ptr(live), _stream(stream)))
    return live


def autotune(params, cfg, dose, gap, nfrac, stream=None):
    """Time every kernel variant for cfg.L on these protocols (cfg.horizon steps)
    and make the fastest the choice for cfg.L.  Returns (variant, {variant: ms})."""
    P, K = _protocols(dose, gap, nfrac)
    n = LIB.gga_autotune_workspace_bytes(cfg.L, P, K, cfg.R, cfg.horizon, cfg.substeps)
    ws = torch.empty(max(int(n), 1), dtype=torch.uint8, device=dose.device)
    live = torch.empty((P, cfg.R), dtype=torch.int32, device=dose.device)
    fit = torch.empty((P,), dtype=torch.float32, device=dose.device)
    ms = np.zeros(LIB.gga_variant_count(), dtype=np.float32)
    v = LIB.gga_autotune(ctypes.byref(_as_params(params)), ctypes.byref(cfg), _ptr(dose), _ptr(gap), _ptr(nfrac),
                         P, K, _ptr(ws), ws.numel(), _ptr(live), _ptr(fit), ms.ctypes.data_as(ctypes.c_void_p),
                         _stream(stream))
    _check(min(v, 0))
    return v, {i: float(t) for i, t in enumerate(ms) if np.isfinite(t)}


# ---------------------------------------------------------------- quasi-3D variant

def q3_workspace(cfg, C, P, K, device="cuda"):
    """Device workspace of the quasi-3D calls for P protocols x cfg.R replicas."""
    n = LIB.gga_q3_workspace_bytes(cfg.L, int(C), P, cfg.R, K)
    if n == 0:
        raise GGAError(f"no quasi-3D workspace for L={cfg.L}, C={C}, P={P}, R={cfg.R}, K={K}")
    return torch.empty(int(n), dtype=torch.uint8, device=device)


def q3_init(params, cfg, C, P, device="cuda", stream=None):
    """Initial quasi-3D states: (fields[P*R, 3, L, L] f32, cells[P*R, C, L, L] int16 holding uint16 words)."""
    n = P * cfg.R
    fields = torch.empty((n, 3, cfg.L, cfg.L), dtype=torch.float32, device=device)
    cells = torch.empty((n, int(C), cfg.L, cfg.L), dtype=torch.int16, device=device)
    _check(LIB.gga_q3_init(ctypes.byref(_as_params(params)), ctypes.byref(cfg), int(C), P, _ptr(fields),
                           _ptr(cells), _stream(stream)))
    return fields, cells


def q3_run(params, cfg, C, dose, gap, nfrac, n0, nsteps, fields, cells, traj=False, ws=None, stream=None):
    """Advance quasi-3D states in place by nsteps from step n0; returns (live[P, R], traj)."""
    P, K = _protocols(dose, gap, nfrac)
    n = P * cfg.R
    if fields.shape != (n, 3, cfg.L, cfg.L) or fields.dtype != torch.float32 or not fields.is_contiguous():
        raise ValueError("fields must be a contiguous float32 [P*R, 3, L, L] tensor")
    if cells.shape != (n, int(C), cfg.L, cfg.L) or cells.dtype != torch.int16 or not cells.is_contiguous():
        raise ValueError("cells must be a contiguous int16 [P*R, C, L, L] tensor")
    ws = q3_workspace(cfg, C, P, K, dose.device) if ws is None else ws
    live = torch.empty((P, cfg.R), dtype=torch.int32, device=dose.device)
    tr = torch.empty((P, cfg.R, max(nsteps, 0)), dtype=torch.int32, device=dose.device) if traj else None
    _check(LIB.gga_q3_run(ctypes.byref(_as_params(params)), ctypes.byref(cfg), int(C), _ptr(dose), _ptr(gap),
                          _ptr(nfrac), P, K, int(n0), int(nsteps), _ptr(fields), _ptr(cells), _ptr(ws), ws.numel(),
                          _ptr(live), _ptr(tr), _stream(stream)))
    return live, tr


def simulate_q3(params, cfg, C, dose, gap, nfrac, traj=False, ws=None, out=None, stream=None):
    """simulate() for the quasi-3D variant with C cell slots per site; returns (live[P, R], fitness[P], traj)."""
    P, K = _protocols(dose, gap, nfrac)
    dev = dose.device
    ws = q3_workspace(cfg, C, P, K, dev) if ws is None else ws
    if out is None:
        live = torch.empty((P, cfg.R), dtype=torch.int32, device=dev)
        fit = torch.empty((P,), dtype=torch.float32, device=dev)
        tr = torch.empty((P, cfg.R, cfg.horizon), dtype=torch.int32, device=dev) if traj else None
    else:
        live, fit, tr = out
    _check(LIB.gga_simulate_q3(ctypes.byref(_as_params(params)), ctypes.byref(cfg), int(C), _ptr(dose), _ptr(gap),
                               _ptr(nfrac), P, K, _ptr(ws), ws.numel(), _ptr(live), _ptr(fit), _ptr(tr),
                               _stream(stream)))
    return live, fit, tr


# ---------------------------------------------------------------- GA

def make_ga(n_elite=2, tournament_k=4, p_cross=0.8, p_mut=0.05, seed=0, selection="tournament",
            crossover="one_point", mutation=("gene",), q=0.9, trunc_frac=0.4, roulette_base=0.0):
    """GA settings; selection, crossover and mutation name the operator
    variants (see GGA_SEL_*, GGA_X_*, GGA_MUT_* in gga.h)."""
    g = GaCfg()
    g.struct_size = ctypes.sizeof(GaCfg)
    g.n_elite, g.tournament_k = int(n_elite), int(tournament_k)
    g.p_cross, g.p_mut, g.seed = float(p_cross), float(p_mut), int(seed)
    g.selection, g.crossover = SELECTIONS[selection], CROSSOVERS[crossover]
    g.mutation = sum(MUTATIONS[m] for m in set(mutation))
    g.q, g.trunc_frac, g.roulette_base = float(q), float(trunc_frac), float(roulette_base)
    return g


def ga_breed(ga, alphabet, fitness, dose, gap, generation, stream=None):
    """One breeding step; generation is an int32 CUDA tensor of one element.
    Returns (order, position, next_dose, next_gap)."""
    N, K = dose.shape
    order = torch.empty(N, dtype=torch.int32, device=dose.device)
    pos = torch.empty(N, dtype=torch.int32, device=dose.device)
    nd, ng = torch.empty_like(dose), torch.empty_like(gap)
    _check(LIB.gga_ga_breed(ctypes.byref(ga), ctypes.byref(alphabet), _ptr(fitness), _ptr(dose), _ptr(gap),
                            N, K, _ptr(generation), _ptr(order), _ptr(pos), _ptr(nd), _ptr(ng), _stream(stream)))
    return order, pos, nd, ng


def ga_workspace(N, R, device="cuda"):
    return torch.empty(int(LIB.gga_ga_workspace_bytes(N, R)), dtype=torch.uint8, device=device)


def ga_set_generation(ws, g, stream=None):
    _check(LIB.gga_ga_set_generation(_ptr(ws), int(g), _stream(stream)))


def ga_generation(params, cfg, ga, alphabet, dose, gap, nfrac, ws, hist=None, advance=True, stream=None):
    """Enqueue one GA generation; returns (next_dose, next_gap)."""
    N, K = _protocols(dose, gap, nfrac)
    nd, ng = torch.empty_like(dose), torch.empty_like(gap)
    cap = hist.shape[0] if hist is not None else 0
    _check(LIB.gga_ga_generation(ctypes.byref(_as_params(params)), ctypes.byref(cfg), ctypes.byref(ga),
                                 ctypes.byref(alphabet), _ptr(dose), _ptr(gap), _ptr(nfrac), N, K, _ptr(nd),
                                 _ptr(ng), _ptr(ws), ws.numel(), _ptr(hist), cap, int(bool(advance)),
                                 _stream(stream)))
    return nd, ng


def _archive(archive, rows, K, device):
    """Best-protocol archive (dose [rows][K], gap [rows][K]) grown to rows,
    keeping what an earlier archive held."""
    d = torch.zeros((rows, K), dtype=torch.float32, device=device)
    g = torch.zeros((rows, K), dtype=torch.int32, device=device)
    if archive is not None:
        n = min(rows, archive[0].shape[0])
        d[:n], g[:n] = archive[0][:n], archive[1][:n]
    return d, g


def ga_run(params, cfg, ga, alphabet, dose, gap, n_gen, use_graph, g0=0, hist=None, archive=None):
    """Run generations g0 .. g0+n_gen-1 from (dose, gap) (not modified).
    Returns (final dose, final gap, hist[g0+n_gen, 2] (best, mean), gen_ms[n_gen]).
    Pass the previous hist to keep filling it when continuing a run.  With
    archive=True (or a previous archive), the best protocol of every
    generation is kept too and a fifth value (best_dose, best_gap) returned."""
    N, K = dose.shape
    nfrac = torch.full((N,), K, dtype=torch.int32, device=dose.device)
    da, ga_ = dose.clone(), gap.clone()
    db, gb = torch.empty_like(dose), torch.empty_like(gap)
    ws = ga_workspace(N, cfg.R, dose.device)
    rows = max(g0 + n_gen, 1)
    h = torch.full((rows, 2), float("nan"), dtype=torch.float32, device=dose.device)
    if hist is not None:
        h[:min(rows, hist.shape[0])] = hist[:rows]
    gen_ms = np.zeros(max(n_gen, 1), dtype=np.float32)
    arc = _archive(None if archive is True else archive, rows, K, dose.device) if archive is not None else None
    # a captured stream must not be the legacy default stream
    side = torch.cuda.Stream(device=dose.device)
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        _check(LIB.gga_ga_run(ctypes.byref(_as_params(params)), ctypes.byref(cfg), ctypes.byref(ga),
                              ctypes.byref(alphabet), _ptr(da), _ptr(ga_), _ptr(db), _ptr(gb), _ptr(nfrac), N, K,
                              int(g0), int(n_gen), int(bool(use_graph)), _ptr(ws), ws.numel(), _ptr(h),
                              _ptr(arc[0]) if arc else None, _ptr(arc[1]) if arc else None,
                              gen_ms.ctypes.data_as(ctypes.c_void_p), ctypes.c_void_p(side.cuda_stream)))
    torch.cuda.current_stream().wait_stream(side)
    final = (da, ga_) if n_gen % 2 == 0 else (db, gb)
    if arc is not None:
        return final[0], final[1], h[:g0 + n_gen], gen_ms[:n_gen], (arc[0][:g0 + n_gen], arc[1][:g0 + n_gen])
    return final[0], final[1], h[:g0 + n_gen], gen_ms[:n_gen]


# ---------------------------------------------------------------- time-slot GA

def make_slots(S=120, g_min=6, dmax_q=20, cap_q=40, quantum=0.25, mutation=()):
    """Slot-genome settings: S hourly slots, minimal interval g_min hours,
    single doses up to dmax_q quanta, total up to cap_q quanta of `quantum`
    Gy; mutation names GGA_SMUT_* operators (empty: swap, split, time)."""
    c = SlotCfg()
    c.struct_size = ctypes.sizeof(SlotCfg)
    c.S, c.g_min, c.dmax_q, c.cap_q = int(S), int(g_min), int(dmax_q), int(cap_q)
    c.mutation = sum(SLOT_MUTATIONS[m] for m in set(mutation))
    c.quantum = float(quantum)
    return c


def _genomes(pop, sc):
    if not (pop.is_cuda and pop.dtype == torch.uint8 and pop.is_contiguous() and pop.dim() == 2
            and pop.shape[1] == sc.S):
        raise ValueError("genomes must be a contiguous uint8 CUDA tensor of shape [P, S]")
    return pop.shape[0]


def slots_breed(ga, sc, fitness, pop, generation, stream=None):
    """One breeding step over uint8 genomes pop [N][S]; generation is an int32
    CUDA tensor of one element.  Returns (order, position, next_pop)."""
    N = _genomes(pop, sc)
    if not (fitness.is_cuda and fitness.dtype == torch.float32 and fitness.numel() == N and fitness.is_contiguous()):
        raise ValueError("fitness must be a contiguous float32 CUDA tensor of N values")
    if not (generation.is_cuda and generation.dtype == torch.int32 and generation.numel() >= 1):
        raise ValueError("generation must be an int32 CUDA tensor")
    order = torch.empty(N, dtype=torch.int32, device=pop.device)
    pos = torch.empty(N, dtype=torch.int32, device=pop.device)
    nxt = torch.empty_like(pop)
    _check(LIB.gga_slots_breed(ctypes.byref(ga), ctypes.byref(sc), _ptr(fitness), _ptr(pop), N, _ptr(generation),
                               _ptr(order), _ptr(pos), _ptr(nxt), _stream(stream)))
    return order, pos, nxt


def slots_decode(sc, pop, K, stream=None):
    """(dose [P][K], gap [P][K], nfrac [P]) of genomes pop [P][S]."""
    P = _genomes(pop, sc)
    dose = torch.empty((P, K), dtype=torch.float32, device=pop.device)
    gap = torch.empty((P, K), dtype=torch.int32, device=pop.device)
    nfrac = torch.empty(P, dtype=torch.int32, device=pop.device)
    _check(LIB.gga_slots_decode(ctypes.byref(sc), _ptr(pop), P, int(K), _ptr(dose), _ptr(gap), _ptr(nfrac),
                                _stream(stream)))
    return dose, gap, nfrac


def slots_encode(sc, dose, gap, nfrac, stream=None):
    """Guarded uint8 genomes [P][S] of protocols (dose, gap, nfrac)."""
    P, K = _protocols(dose, gap, nfrac)
    pop = torch.empty((P, sc.S), dtype=torch.uint8, device=dose.device)
    _check(LIB.gga_slots_encode(ctypes.byref(sc), _ptr(dose), _ptr(gap), _ptr(nfrac), P, K, _ptr(pop),
                                _stream(stream)))
    return pop


def slots_run(params, cfg, ga, sc, pop, K, n_gen, use_graph, g0=0, archive=False):
    """Run slot-GA generations g0 .. g0+n_gen-1 from genomes pop (not
    modified), simulating K fraction slots per protocol.  Returns (final pop,
    hist[g0+n_gen, 2] (best, mean), gen_ms[n_gen]) and, with archive=True, a
    fourth value (best_dose, best_gap) per generation."""
    N = _genomes(pop, sc)
    a, b = pop.clone(), torch.empty_like(pop)
    ws = torch.empty(int(LIB.gga_slots_workspace_bytes(N, cfg.R, int(K))), dtype=torch.uint8, device=pop.device)
    rows = max(g0 + n_gen, 1)
    h = torch.full((rows, 2), float("nan"), dtype=torch.float32, device=pop.device)
    gen_ms = np.zeros(max(n_gen, 1), dtype=np.float32)
    arc = _archive(None, rows, int(K), pop.device) if archive else None
    side = torch.cuda.Stream(device=pop.device)
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        _check(LIB.gga_slots_run(ctypes.byref(_as_params(params)), ctypes.byref(cfg), ctypes.byref(ga),
                                 ctypes.byref(sc), _ptr(a), _ptr(b), N, int(K), int(g0), int(n_gen),
                                 int(bool(use_graph)), _ptr(ws), ws.numel(), _ptr(h),
                                 _ptr(arc[0]) if arc else None, _ptr(arc[1]) if arc else None,
                                 gen_ms.ctypes.data_as(ctypes.c_void_p), ctypes.c_void_p(side.cuda_stream)))
    torch.cuda.current_stream().wait_stream(side)
    final = a if n_gen % 2 == 0 else b
    if arc is not None:
        return final, h[:g0 + n_gen], gen_ms[:n_gen], (arc[0][:g0 + n_gen], arc[1][:g0 + n_gen])
    return final, h[:g0 + n_gen], gen_ms[:n_gen]


# ---------------------------------------------------------------- surrogate MLP

MLP_IN, MLP_HID = 128, 512
MLP_SHAPES = [(MLP_IN, MLP_HID), (MLP_HID,), (MLP_HID, MLP_HID), (MLP_HID,), (MLP_HID, MLP_HID), (MLP_HID,),
              (MLP_HID,), (1,)]
MLP_PARAMS = sum(int(np.prod(s)) for s in MLP_SHAPES)


def _align256(x):
    return (x + 255) & ~255


def mlp_layout():
    """Byte offsets of the net buffer's blocks (norm, params, m, v, grads)."""
    off, out = 0, {}
    for name, size in (("norm", 12), ("p", 4 * MLP_PARAMS), ("m", 4 * MLP_PARAMS), ("v", 4 * MLP_PARAMS),
                       ("g", 4 * MLP_PARAMS)):
        out[name] = off
        off += _align256(size)
    return out


def mlp_net(seed=0, device="cuda", stream=None):
    net = torch.empty(int(LIB.gga_mlp_net_bytes()), dtype=torch.uint8, device=device)
    _check(LIB.gga_mlp_init(_ptr(net), int(seed), _stream(stream)))
    return net


def mlp_block(net, name):
    """float32 view of a block of the net buffer (norm, p, m, v or g)."""
    off = mlp_layout()[name]
    n = 2 if name == "norm" else MLP_PARAMS
    return net[off:off + 4 * n].view(torch.float32)


def mlp_split(flat):
    """Split a flat parameter-ordered vector into the per-tensor shapes."""
    out, i = [], 0
    for s in MLP_SHAPES:
        n = int(np.prod(s))
        out.append(flat[i:i + n].reshape(s))
        i += n
    return out


def mlp_work(B, device="cuda"):
    return torch.empty(max(int(LIB.gga_mlp_work_bytes(B)), 1), dtype=torch.uint8, device=device)


MLP_WORK_PARTS = ("X", "Z1", "Z2", "Z3", "H1", "H2", "H3", "y", "dy", "dZa", "dZb")


def mlp_work_views(work, B):
    """Views of what the MLP passes leave in a work buffer of batch B (test
    hook): X, H1..H3, dZa, dZb as bfloat16, the rest float32 (layout from
    gga_mlp_work_layout)."""
    off = (ctypes.c_size_t * 12)()
    _check(LIB.gga_mlp_work_layout(int(B), off))
    shapes = {"X": (B, MLP_IN), "y": (B,), "dy": (B,)}
    out = {}
    for i, name in enumerate(MLP_WORK_PARTS):
        shape = shapes.get(name, (B, MLP_HID))
        half = name in ("X", "H1", "H2", "H3", "dZa", "dZb")
        n = int(np.prod(shape)) * (2 if half else 4)
        out[name] = work[off[i]:off[i] + n].view(torch.bfloat16 if half else torch.float32).view(shape)
    return out


def mlp_set_norm(net, target, stream=None):
    _check(LIB.gga_mlp_set_norm(_ptr(net), _ptr(target), target.numel(), _stream(stream)))


def mlp_predict(net, dose, gap, nfrac, work=None, out=None, stream=None):
    B, K = _protocols(dose, gap, nfrac)
    work = work if work is not None else mlp_work(B, dose.device)
    pred = out if out is not None else torch.empty(B, dtype=torch.float32, device=dose.device)
    _check(LIB.gga_mlp_predict(_ptr(net), _ptr(dose), _ptr(gap), _ptr(nfrac), B, K, _ptr(work), work.numel(),
                               _ptr(pred), _stream(stream)))
    return pred


def mlp_grad(net, dose, gap, nfrac, target, work=None, stream=None):
    B, K = _protocols(dose, gap, nfrac)
    work = work if work is not None else mlp_work(B, dose.device)
    loss = torch.empty(1, dtype=torch.float32, device=dose.device)
    _check(LIB.gga_mlp_grad(_ptr(net), _ptr(dose), _ptr(gap), _ptr(nfrac), _ptr(target), B, K, _ptr(work),
                            work.numel(), _ptr(loss), _stream(stream)))
    return loss


def mlp_train_step(net, dose, gap, nfrac, target, step, lr, work=None, loss=None, stream=None):
    B, K = _protocols(dose, gap, nfrac)
    work = work if work is not None else mlp_work(B, dose.device)
    loss = loss if loss is not None else torch.empty(1, dtype=torch.float32, device=dose.device)
    _check(LIB.gga_mlp_train_step(_ptr(net), _ptr(dose), _ptr(gap), _ptr(nfrac), _ptr(target), B, K, int(step),
                                  float(lr), _ptr(work), work.numel(), _ptr(loss), _stream(stream)))
    return loss


def mlp_gemm(A, B, a_trans=False, b_trans=False, stream=None):
    """C = op(A) op(B) with the MLP's MFMA kernel (bf16 in, f32 out)."""
    if A.dtype != torch.bfloat16 or B.dtype != torch.bfloat16:
        raise ValueError("A and B must be bfloat16")
    M, K = (A.shape[1], A.shape[0]) if a_trans else A.shape
    K2, N = (B.shape[1], B.shape[0]) if b_trans else B.shape
    if K != K2:
        raise ValueError("inner dimensions differ")
    C = torch.empty((M, N), dtype=torch.float32, device=A.device)
    _check(LIB.gga_mlp_gemm(M, N, K, _ptr(A.contiguous()), int(a_trans), _ptr(B.contiguous()), int(b_trans),
                            _ptr(C), _stream(stream)))
    return C


# ---------------------------------------------------------------- surrogate-screened GA

def make_sga(n_candidates, n_simulated, screen=True, refine_steps=0, refine_lr=1e-4):
    c = SgaCfg()
    c.struct_size = ctypes.sizeof(SgaCfg)
    c.n_candidates, c.n_simulated, c.screen = int(n_candidates), int(n_simulated), int(bool(screen))
    c.refine_steps, c.refine_lr = int(refine_steps), float(refine_lr)
    return c


class SurrogateGA:
    """Population (N + S rows) and workspace of a surrogate-screened GA run.

    init() simulates the initial population; run() advances generations (in
    chunks if wanted: continuing with g0 reproduces one longer run).  With
    archive=True the best protocol of every generation is kept in
    self.archive = (best_dose, best_gap)."""

    def __init__(self, params, cfg, ga, alphabet, sga, net, dose, gap, archive=False):
        self.params, self.cfg, self.ga, self.alphabet, self.sga, self.net = _as_params(params), cfg, ga, alphabet, sga, net
        N, K = dose.shape
        S = sga.n_simulated
        self.N, self.K = N, K
        dev = dose.device
        self.dose = torch.zeros((N + S, K), dtype=torch.float32, device=dev)
        self.gap = torch.zeros((N + S, K), dtype=torch.int32, device=dev)
        self.fit = torch.full((N + S,), float("nan"), dtype=torch.float32, device=dev)
        self.dose[:N] = dose
        self.gap[:N] = gap
        self.ws = torch.empty(int(LIB.gga_sga_workspace_bytes(N, K, cfg.R, sga.n_candidates, S)),
                              dtype=torch.uint8, device=dev)
        self.hist = None
        self.keep_archive = bool(archive)
        self.archive = None
        self.g = 0
        self.stream = torch.cuda.Stream(device=dev)     # capturable (not the legacy default stream)

    def init(self):
        self.stream.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(self.stream):
            _check(LIB.gga_sga_init(ctypes.byref(self.params), ctypes.byref(self.cfg), ctypes.byref(self.sga),
                                    _ptr(self.dose), _ptr(self.gap), _ptr(self.fit), self.N, self.K, _ptr(self.ws),
                                    self.ws.numel(), ctypes.c_void_p(self.stream.cuda_stream)))
        torch.cuda.current_stream().wait_stream(self.stream)

    def run(self, n_gen, use_graph=True):
        rows = self.g + n_gen
        h = torch.full((max(rows, 1), 2), float("nan"), dtype=torch.float32, device=self.dose.device)
        if self.hist is not None:
            h[:self.hist.shape[0]] = self.hist
        gen_ms = np.zeros(max(n_gen, 1), dtype=np.float32)
        arc = _archive(self.archive, max(rows, 1), self.K, self.dose.device) if self.keep_archive else None
        self.stream.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(self.stream):
            _check(LIB.gga_sga_run(ctypes.byref(self.params), ctypes.byref(self.cfg), ctypes.byref(self.ga),
                                   ctypes.byref(self.alphabet), ctypes.byref(self.sga), _ptr(self.net),
                                   _ptr(self.dose), _ptr(self.gap), _ptr(self.fit), self.N, self.K, self.g, n_gen,
                                   int(bool(use_graph)), _ptr(self.ws), self.ws.numel(), _ptr(h),
                                   _ptr(arc[0]) if arc else None, _ptr(arc[1]) if arc else None,
                                   gen_ms.ctypes.data_as(ctypes.c_void_p), ctypes.c_void_p(self.stream.cuda_stream)))
        torch.cuda.current_stream().wait_stream(self.stream)
        self.hist = h[:rows]
        if arc is not None:
            self.archive = (arc[0][:rows], arc[1][:rows])
        self.g = rows
        return gen_ms[:n_gen]


# ---------------------------------------------------------------- measurement

def measure_peaks(nbytes=1 << 30, stream=None):
    """Microbenchmarks on the current device: {"valu_lane_ops_per_s",
    "lds_read_bytes_per_s", "hbm_read_bytes_per_s"} (gga_measure_peaks over a
    buffer of nbytes)."""
    buf = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    v, l, h = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
    _check(LIB.gga_measure_peaks(_ptr(buf), nbytes, ctypes.byref(v), ctypes.byref(l), ctypes.byref(h),
                                 _stream(stream)))
    return {"valu_lane_ops_per_s": v.value, "lds_read_bytes_per_s": l.value, "hbm_read_bytes_per_s": h.value}
