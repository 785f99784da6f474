"""Python front end of libibschur: a thin wrapper that marshals torch device
tensors and the current HIP stream into the C ABI of include/ibschur.h.

Every computation runs in the HIP library; this module only allocates the
device workspace and the argument tensors (PyTorch is used for device memory
and streams) and converts layouts of Python objects into the C structs.
"""
from __future__ import annotations

import ctypes as C

import numpy as np
import torch

from . import _lib
from .workloads import Body, Config, Workload


class SimError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{_lib.STATUS_NAMES.get(code, code)}: {msg}")
        self.code = code


def _ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None else C.c_void_p(0)


def config_check(cfg: Config, max_points: int = 0) -> str:
    """The first rule of the C ABI's configuration check that cfg breaks, or
    "" (host-only: needs the built library but no GPU)."""
    lib = _lib.load()
    msg = C.create_string_buffer(256)
    lib.sim_config_check(C.byref(make_config(cfg, 0)), max_points, msg, 256)
    return msg.value.decode()


def make_config(cfg: Config, stream=None) -> _lib.SimConfig:
    c = _lib.SimConfig()
    c.n[:] = list(cfg.n)
    c.len[:] = list(cfg.length)
    c.bc[:] = list(cfg.bc)
    c.nu, c.dt = cfg.nu, cfg.dt
    c.g[:] = list(cfg.g)
    c.delta, c.lump_c = cfg.delta, cfg.lump_c
    c.precision, c.krylov_restart, c.krylov_maxit = cfg.precision, cfg.krylov_restart, cfg.krylov_maxit
    c.krylov_rtol = cfg.krylov_rtol
    c.helm_maxit, c.helm_rtol = cfg.helm_maxit, cfg.helm_rtol
    c.mg_coarsest, c.mg_pre, c.mg_post = cfg.mg_coarsest, cfg.mg_pre, cfg.mg_post
    c.mg_coarse_sweeps = cfg.mg_coarse_sweeps
    c.precond = cfg.precond
    c.krylov = cfg.krylov
    c.outer_iters, c.outer_tol, c.xi = cfg.outer_iters, cfg.outer_tol, cfg.xi
    c.record_two_way = cfg.record_two_way
    c.device = cfg.device
    c.stream = stream if stream is not None else torch.cuda.current_stream(cfg.device).cuda_stream
    return c


def make_bodies(bodies):
    arr = (_lib.SimBody * max(1, len(bodies)))()
    for i, b in enumerate(bodies):
        sb = arr[i]
        sb.center[:] = [float(x) for x in b.center]
        sb.vel[:] = [float(x) for x in b.vel]
        sb.omega[:] = [float(x) for x in b.omega]
        sb.radius = float(b.radius)
        sb.density_ratio = float(b.density_ratio)
        sb.osc_amp[:] = [float(x) for x in b.osc_amp]
        sb.osc_omega = float(b.osc_omega)
        sb.motion = int(b.motion)
        sb.n_points = int(b.n_points)
    return arr


class Sim:
    """One solver instance on one GPU (one handle, one stream)."""

    def __init__(self, cfg: Config, max_points: int, device: int = 0):
        if not torch.cuda.is_available():
            raise RuntimeError("the IB Schur solver needs a HIP device")
        self.lib = _lib.load()
        cfg.device = device
        self.cfg = cfg
        self.dev = torch.device("cuda", device)
        self.stream = torch.cuda.current_stream(self.dev)
        self.ccfg = make_config(cfg, self.stream.cuda_stream)
        msg = C.create_string_buffer(256)
        if self.lib.sim_config_check(C.byref(self.ccfg), max_points, msg, 256) != 0:
            raise SimError(_lib.SIM_EINVAL, f"invalid configuration: {msg.value.decode()}")
        nbytes = self.lib.sim_workspace_bytes(C.byref(self.ccfg), max_points)
        if nbytes == 0:
            raise SimError(_lib.SIM_EINVAL, "invalid configuration")
        self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.dev)
        h = C.c_void_p()
        rc = self.lib.sim_create(C.byref(self.ccfg), _ptr(self.workspace), nbytes + 256, max_points,
                                 C.byref(h))
        if rc != 0:
            raise SimError(rc, "sim_create failed")
        self.h = h
        self.K = 0
        self.nb = 0
        self.n = tuple(cfg.n)

    def _check(self, rc, allow_notconv=False):
        if rc == 0 or (allow_notconv and rc == _lib.SIM_ENOTCONV):
            return rc
        raise SimError(rc, self.lib.sim_last_error(self.h).decode())

    def close(self):
        if getattr(self, "h", None):
            self.lib.sim_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- state ------------------------------------------------------------
    def set_bodies(self, bodies, offsets):
        off = np.ascontiguousarray(offsets, dtype=np.float64)
        arr = make_bodies(bodies)
        self._check(self.lib.sim_set_bodies(self.h, len(bodies), arr,
                                            off.ctypes.data_as(C.POINTER(C.c_double))))
        self.K = int(off.shape[0])
        self.nb = len(bodies)
        self.bodies = list(bodies)
        self.offsets = off

    def set_time(self, t: float):
        self._check(self.lib.sim_set_time(self.h, float(t)))

    def set_workload(self, w: Workload):
        self.set_bodies(w.bodies, w.offsets)
        u0 = torch.as_tensor(w.u0, device=self.dev)
        self.set_fields(0, u0)
        self.set_fields(1, u0)

    def _t(self, x):
        if x is None:
            return None
        return torch.as_tensor(x, dtype=torch.float64, device=self.dev).contiguous()

    def set_fields(self, level, u3=None, p=None, phi=None):
        u3 = self._t(u3)
        comps = [u3[d] if u3 is not None else None for d in range(3)]
        p, phi = self._t(p), self._t(phi)
        self._check(self.lib.sim_set_fields(self.h, level, *[_ptr(c) for c in comps], _ptr(p), _ptr(phi)))

    def get_fields(self):
        u = torch.empty((3,) + self.n, dtype=torch.float64, device=self.dev)
        p = torch.empty(self.n, dtype=torch.float64, device=self.dev)
        self._check(self.lib.sim_get_fields(self.h, _ptr(u[0]), _ptr(u[1]), _ptr(u[2]), _ptr(p)))
        return u, p

    def get_points(self):
        X = torch.empty((max(self.K, 1), 3), dtype=torch.float64, device=self.dev)
        U = torch.empty_like(X)
        self._check(self.lib.sim_get_points(self.h, _ptr(X), _ptr(U)))
        return X[:self.K], U[:self.K]

    def get_body_state(self):
        """Per body: dict(center, vel, omega, R) at the current time."""
        buf = (C.c_double * (18 * max(self.nb, 1)))()
        self._check(self.lib.sim_get_body_state(self.h, buf))
        a = np.array(buf[:18 * self.nb]).reshape(self.nb, 18)
        return [dict(center=r[0:3], vel=r[3:6], omega=r[6:9], R=r[9:18].reshape(3, 3)) for r in a]

    def get_forces(self):
        f = torch.empty((max(self.K, 1), 3), dtype=torch.float64, device=self.dev)
        ft = (C.c_double * (6 * max(self.nb, 1)))()
        self._check(self.lib.sim_get_forces(self.h, _ptr(f), ft))
        return f[:self.K], np.array(ft[:6 * self.nb]).reshape(self.nb, 6)

    # -- compute ----------------------------------------------------------
    def step(self, nsteps=1, allow_notconv=False):
        st = _lib.StepStats()
        rc = self._check(self.lib.sim_step(self.h, nsteps, C.byref(st)), allow_notconv)
        return st, rc

    def solve_schur(self, rhs_p, rhs_f, allow_notconv=False):
        rp, rf = self._t(rhs_p), self._t(rhs_f)
        p = torch.empty(self.n, dtype=torch.float64, device=self.dev)
        phi = torch.empty((max(self.K, 1), 3), dtype=torch.float64, device=self.dev)
        st = _lib.SolveStats()
        rc = self._check(self.lib.sim_solve_schur(self.h, _ptr(rp), _ptr(rf), _ptr(p), _ptr(phi),
                                                  C.byref(st)), allow_notconv)
        return p, phi[:self.K], st

    def solve_schur_noalloc(self, rhs_p, rhs_f, allow_notconv=False):
        """sim_solve_schur_noalloc: the solve with its work arrays in the
        library's static device scratch (the output tensors are allocated
        here, by the caller, as the C ABI expects)."""
        rp, rf = self._t(rhs_p), self._t(rhs_f)
        p = torch.empty(self.n, dtype=torch.float64, device=self.dev)
        phi = torch.empty((max(self.K, 1), 3), dtype=torch.float64, device=self.dev)
        st = _lib.SolveStats()
        rc = self._check(self.lib.sim_solve_schur_noalloc(self.h, _ptr(rp), _ptr(rf), _ptr(p), _ptr(phi),
                                                          C.byref(st)), allow_notconv)
        return p, phi[:self.K], st

    def apply(self, op, x, x2=None):
        opid = _lib.OPS[op]
        x = self._t(x)
        x2 = self._t(x2)
        cells, faces, points = self.n, (3,) + self.n, (max(self.K, 1), 3)
        out_shape = {"laplacian": cells, "schur": cells, "precond": cells, "grad": faces,
                     "div": cells, "interp": points, "spread": faces, "helmholtz": faces,
                     "convection": faces, "helm_solve": faces, "schur_rhs": cells, "schur_exact": cells}[op]
        out = torch.empty(out_shape, dtype=torch.float64, device=self.dev)
        self._check(self.lib.sim_apply(self.h, opid, _ptr(x), _ptr(x2), _ptr(out)))
        return out[:self.K] if op == "interp" else out

    def schur_spectrum(self, v0, exact=False, steps=60, lap_rtol=1e-12):
        """Lanczos estimate of spec(L^+ S) (S = S~, or S_p if exact): dict with
        the tridiagonal coefficients alpha, beta, its order and the extreme
        Ritz values lmin, lmax."""
        v = self._t(v0)
        a = (C.c_double * steps)()
        b = (C.c_double * steps)()
        m = C.c_int32()
        lo, hi = C.c_double(), C.c_double()
        self._check(self.lib.sim_schur_spectrum(self.h, int(bool(exact)), _ptr(v), int(steps), float(lap_rtol),
                                                a, b, C.byref(m), C.byref(lo), C.byref(hi)))
        k = int(m.value)
        return dict(alpha=np.array(a[:k]), beta=np.array(b[:k]), steps=k, lmin=float(lo.value),
                    lmax=float(hi.value))

    def probe(self, name, on=True):
        self._check(self.lib.sim_probe_enable(self.h, _lib.PROBES[name], int(on)))

    def probe_read(self, name, reset=True):
        """(launches, milliseconds, algorithmic bytes) of a probe's kernel class."""
        n = C.c_int64()
        ms = C.c_double()
        nb = C.c_double()
        self._check(self.lib.sim_probe_read(self.h, _lib.PROBES[name], C.byref(n), C.byref(ms), C.byref(nb),
                                            int(reset)))
        return int(n.value), float(ms.value), float(nb.value)

    BODY_OUT = ("xc", "us", "w", "I", "J")
    BODY_IN = ("xc", "xc_m", "us", "us_m", "w", "w_m", "I_n", "I_m", "J_n", "J_m")

    def step_adjoint_two_way(self, gu=None, gp=None, gphi=None, gbodies=None):
        """Reverse mode of the last two-way step.  gbodies: per body a dict with
        any of xc, us, w, I, J (cotangents of the step's body outputs).
        Returns dict(gu, gum, gp, gphi, bodies=[dict(xc, xc_m, us, ...)])."""
        gu = self._t(gu)
        comps = [gu[d] if gu is not None else None for d in range(3)]
        gp, gphi = self._t(gp), self._t(gphi)
        gout = (C.c_double * (15 * max(self.nb, 1)))()
        for i, gb in enumerate(gbodies or []):
            for j, key in enumerate(self.BODY_OUT):
                if gb.get(key) is not None:
                    gout[15 * i + 3 * j:15 * i + 3 * j + 3] = [float(x) for x in gb[key]]
        gin = (C.c_double * (30 * max(self.nb, 1)))()
        outs = [torch.zeros((3,) + self.n, dtype=torch.float64, device=self.dev),
                torch.zeros((3,) + self.n, dtype=torch.float64, device=self.dev),
                torch.zeros(self.n, dtype=torch.float64, device=self.dev),
                torch.zeros((max(self.K, 1), 3), dtype=torch.float64, device=self.dev)]
        self._check(self.lib.sim_step_adjoint_two_way(self.h, *[_ptr(c) for c in comps], _ptr(gp), _ptr(gphi),
                                                      gout, *[_ptr(o) for o in outs], gin))
        g30 = np.array(gin[:30 * self.nb]).reshape(self.nb, 10, 3)
        bodies = [{k: g30[i, j].copy() for j, k in enumerate(self.BODY_IN)} for i in range(self.nb)]
        return dict(gu=outs[0], gum=outs[1], gp=outs[2], gphi=outs[3][:self.K], bodies=bodies)

    def step_adjoint(self, gu=None, gp=None, gphi=None, want_inputs=False):
        gu = self._t(gu)
        comps = [gu[d] if gu is not None else None for d in range(3)]
        gp, gphi = self._t(gp), self._t(gphi)
        gX = torch.zeros((max(self.K, 1), 3), dtype=torch.float64, device=self.dev)
        gU = (C.c_double * (6 * max(self.nb, 1)))()
        outs = [None] * 4
        if want_inputs:
            outs = [torch.zeros((3,) + self.n, dtype=torch.float64, device=self.dev),
                    torch.zeros((3,) + self.n, dtype=torch.float64, device=self.dev),
                    torch.zeros(self.n, dtype=torch.float64, device=self.dev),
                    torch.zeros((max(self.K, 1), 3), dtype=torch.float64, device=self.dev)]
        self._check(self.lib.sim_step_adjoint(self.h, *[_ptr(c) for c in comps], _ptr(gp), _ptr(gphi),
                                              _ptr(gX), gU, *[_ptr(o) for o in outs]))
        g6 = np.array(gU[:6 * self.nb]).reshape(self.nb, 6)
        res = dict(gX=gX[:self.K], gU=g6[:, :3], gW=g6[:, 3:])
        if want_inputs:
            res.update(gu=outs[0], gum=outs[1], gp=outs[2], gphi=outs[3][:self.K])
        return res
