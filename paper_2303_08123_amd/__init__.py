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
          -5: "GGA_E_PARAM", -6: "GGA_E_ALPHABET"}
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
        ("m", ctypes.c_double * 4),
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


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with "
                          "`python -m paper_2303_08123_amd.build` (hipcc, gfx950)")
    lib = ctypes.CDLL(LIB_PATH)
    vp, i32, i64, u64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64
    sig = {
        "gga_version": ([], ctypes.c_int),
        "gga_strerror": ([ctypes.c_int], ctypes.c_char_p),
        "gga_last_hip_error": ([], ctypes.c_int),
        "gga_validate": ([vp, vp, vp, vp, i32, i32, vp], ctypes.c_int),
        "gga_population_random": ([vp, i32, i32, u64, vp, vp, vp, vp], ctypes.c_int),
        "gga_simulate": ([vp, vp, vp, vp, vp, i32, i32, vp, vp, vp, vp], ctypes.c_int),
        "gga_state_init": ([vp, vp, i32, vp, vp, vp], ctypes.c_int),
        "gga_state_run": ([vp, vp, vp, vp, vp, i32, i32, i32, i32, vp, vp, vp, vp, vp], ctypes.c_int),
        "gga_philox_fill": ([vp, u64, vp, i64, vp], ctypes.c_int),
    }
    for name, (args, res) in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    return lib


LIB = _load()
EXPORTS = ("gga_version", "gga_strerror", "gga_last_hip_error", "gga_validate",
           "gga_population_random", "gga_simulate", "gga_state_init", "gga_state_run",
           "gga_philox_fill")


class GGAError(RuntimeError):
    pass


def _check(rc):
    if rc != GGA_OK:
        msg = LIB.gga_strerror(rc).decode()
        if rc == -4:
            msg += f" (hipError {LIB.gga_last_hip_error()})"
        raise GGAError(f"{ERRORS.get(rc, rc)}: {msg}")


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
    return p


def make_cfg(L, horizon, R, seed=0, substeps=10, dose_cap=20.0):
    c = SimCfg()
    c.struct_size = ctypes.sizeof(SimCfg)
    c.L, c.horizon, c.substeps, c.R = int(L), int(horizon), int(substeps), int(R)
    c.flags, c.seed, c.dose_cap = 0, int(seed), float(dose_cap)
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


def simulate(params, cfg, dose, gap, nfrac, traj=False, out=None, stream=None):
    """Simulate every (protocol, replica) instance; returns (live[P, R], fitness[P], traj)."""
    P, K = _protocols(dose, gap, nfrac)
    dev = dose.device
    if out is None:
        live = torch.empty((P, cfg.R), dtype=torch.int32, device=dev)
        fit = torch.empty((P,), dtype=torch.float32, device=dev)
        tr = torch.empty((P, cfg.R, cfg.horizon), dtype=torch.int32, device=dev) if traj else None
    else:
        live, fit, tr = out
    _check(LIB.gga_simulate(ctypes.byref(_as_params(params)), ctypes.byref(cfg), _ptr(dose), _ptr(gap),
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


def philox_fill(ctr, seed, stream=None):
    """Device Philox4x32-10 blocks for counters ctr[n, 4] (int32 tensor holding uint32)."""
    if not (ctr.is_cuda and ctr.dtype == torch.int32 and ctr.is_contiguous() and ctr.shape[-1] == 4):
        raise ValueError("ctr must be a contiguous int32 CUDA tensor [n, 4]")
    out = torch.empty_like(ctr)
    _check(LIB.gga_philox_fill(_ptr(ctr), int(seed), _ptr(out), ctr.shape[0], _stream(stream)))
    return out
