"""ctypes declarations of include/ibschur.h (argument marshalling only)."""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libibschur.so")

SIM_OK = 0
SIM_EINVAL = -1
SIM_ESTATE = -2
SIM_ENOTCONV = -3
SIM_ENONFINITE = -4
SIM_EDEVICE = -5
SIM_ENOMEM = -6
STATUS_NAMES = {0: "SIM_OK", -1: "SIM_EINVAL", -2: "SIM_ESTATE", -3: "SIM_ENOTCONV",
                -4: "SIM_ENONFINITE", -5: "SIM_EDEVICE", -6: "SIM_ENOMEM"}

OPS = dict(laplacian=0, schur=1, precond=2, grad=3, div=4, interp=5, spread=6, helmholtz=7,
           convection=8, helm_solve=9, schur_rhs=10, schur_exact=11)

EXPORTS = ["sim_config_check", "sim_workspace_bytes", "sim_create", "sim_destroy", "sim_set_bodies", "sim_set_fields",
           "sim_get_fields", "sim_step", "sim_solve_schur", "sim_solve_schur_noalloc", "sim_get_forces",
           "sim_get_points",
           "sim_get_body_state", "sim_set_time",
           "sim_step_adjoint", "sim_step_adjoint_two_way", "sim_apply", "sim_schur_spectrum", "sim_probe_enable", "sim_probe_read", "sim_last_error"]

PROBES = dict(smooth=0, smooth_first=1, restrict=2, prolong=3, laplacian=4,
              spread_div=5, spread_face=6, interp_grad=7, interp_face=8, multidot=9,
              update_norm=10, coarse=11, helm_sweep=12, helm_resid=13, vcycle=14, mom_rhs=15,
              helm_first=16, tile_down=17, tile_up=18)


class SimConfig(C.Structure):
    _fields_ = [("n", C.c_int32 * 3), ("len", C.c_double * 3), ("bc", C.c_int32 * 3),
                ("nu", C.c_double), ("dt", C.c_double), ("g", C.c_double * 3),
                ("delta", C.c_int32), ("lump_c", C.c_double),
                ("precision", C.c_int32), ("krylov_restart", C.c_int32), ("krylov_maxit", C.c_int32),
                ("krylov_rtol", C.c_double), ("helm_maxit", C.c_int32), ("helm_rtol", C.c_double),
                ("mg_coarsest", C.c_int32), ("mg_pre", C.c_int32), ("mg_post", C.c_int32),
                ("mg_coarse_sweeps", C.c_int32), ("precond", C.c_int32), ("krylov", C.c_int32),
                ("outer_iters", C.c_int32), ("outer_tol", C.c_double),
                ("xi", C.c_double), ("record_two_way", C.c_int32), ("device", C.c_int32),
                ("stream", C.c_void_p)]


class SimBody(C.Structure):
    _fields_ = [("center", C.c_double * 3), ("vel", C.c_double * 3), ("omega", C.c_double * 3),
                ("radius", C.c_double), ("density_ratio", C.c_double), ("osc_amp", C.c_double * 3),
                ("osc_omega", C.c_double), ("motion", C.c_int32), ("n_points", C.c_int32)]


class SolveStats(C.Structure):
    _fields_ = [("iters", C.c_int32), ("rel_res", C.c_double), ("seconds", C.c_double),
                ("nhist", C.c_int32), ("hist", C.c_double * 64)]


class StepStats(C.Structure):
    _fields_ = [("outer", C.c_int32), ("helm", SolveStats), ("schur", SolveStats),
                ("div_rel", C.c_double), ("slip_rel", C.c_double), ("outer_crit", C.c_double),
                ("seconds", C.c_double), ("total_schur_iters", C.c_int32)]


_lib = None


def load(path: str = LIB_PATH):
    """Load the HIP library; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"libibschur.so not built ({path}); run __graft_entry__.build()")
    lib = C.CDLL(path)
    P, D, I32, I64, VP = C.POINTER, C.c_double, C.c_int32, C.c_int64, C.c_void_p
    sim_t = C.c_void_p
    lib.sim_config_check.argtypes = [P(SimConfig), I64, C.c_char_p, I32]
    lib.sim_workspace_bytes.argtypes = [P(SimConfig), I64]
    lib.sim_workspace_bytes.restype = C.c_size_t
    lib.sim_create.argtypes = [P(SimConfig), VP, C.c_size_t, I64, P(sim_t)]
    lib.sim_destroy.argtypes = [sim_t]
    lib.sim_set_bodies.argtypes = [sim_t, I32, P(SimBody), P(D)]
    lib.sim_set_fields.argtypes = [sim_t, I32, VP, VP, VP, VP, VP]
    lib.sim_get_fields.argtypes = [sim_t, VP, VP, VP, VP]
    lib.sim_step.argtypes = [sim_t, I32, P(StepStats)]
    lib.sim_solve_schur.argtypes = [sim_t, VP, VP, VP, VP, P(SolveStats)]
    lib.sim_solve_schur_noalloc.argtypes = [sim_t, VP, VP, VP, VP, P(SolveStats)]
    lib.sim_get_forces.argtypes = [sim_t, VP, P(D)]
    lib.sim_get_points.argtypes = [sim_t, VP, VP]
    lib.sim_get_body_state.argtypes = [sim_t, P(D)]
    lib.sim_set_time.argtypes = [sim_t, D]
    lib.sim_step_adjoint.argtypes = [sim_t, VP, VP, VP, VP, VP, VP, P(D), VP, VP, VP, VP]
    lib.sim_apply.argtypes = [sim_t, I32, VP, VP, VP]
    lib.sim_step_adjoint_two_way.argtypes = [sim_t, VP, VP, VP, VP, VP, P(D), VP, VP, VP, VP, P(D)]
    lib.sim_schur_spectrum.argtypes = [sim_t, I32, VP, I32, D, P(D), P(D), P(I32), P(D), P(D)]
    lib.sim_probe_enable.argtypes = [sim_t, I32, I32]
    lib.sim_probe_read.argtypes = [sim_t, I32, P(I64), P(D), P(D), I32]
    lib.sim_last_error.argtypes = [sim_t]
    lib.sim_last_error.restype = C.c_char_p
    for name in EXPORTS:
        if name not in ("sim_workspace_bytes", "sim_last_error"):
            getattr(lib, name).restype = C.c_int
    _lib = lib
    return lib
