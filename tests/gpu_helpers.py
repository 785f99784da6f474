"""Shared set-up for the GPU parity tests: the same seeded workload goes to the
HIP library (through the C ABI) and to the CPU oracle."""
import numpy as np

from oracle import bodies as obd
from oracle import delta as odelta
from oracle import mac as omac
from oracle import schur as oschur
from paper_2501_15314_amd import workloads as wl


def oracle_for(w: wl.Workload, t: float = 0.0):
    cfg = w.cfg
    g = omac.Grid(cfg.n, cfg.h, cfg.bc)
    Xs = []
    for b, o in zip(w.bodies, np.split(w.offsets, np.cumsum([b.n_points for b in w.bodies])[:-1])):
        c = obd.prescribed_center(b.center, b.vel, b.osc_amp, b.osc_omega, t)
        R = obd.prescribed_rotation(b.omega, t)
        Xs.append(obd.points(c, R, o))
    X = np.concatenate(Xs) if Xs else np.zeros((0, 3))
    W = odelta.regularization_matrix(g, X, cfg.delta)
    S = oschur.SchurSystem(g, W, cfg.lump_c)
    return g, X, W, S


def rel(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


def walls_workload(n=32, pts=260, seed=3):
    return wl.make_c3(seed=seed, n=n, points_per_sphere=pts)


def mixed_workload(seed=12):
    """Non-cubic grid (16 x 24 x 32 cells of width 1/32), no-slip along x only,
    two spheres."""
    rng = np.random.default_rng(seed)
    n = (16, 24, 32)
    h = 1.0 / 32
    length = (16 * h, 24 * h, 32 * h)
    radius = 0.12
    K = 150
    cfg = wl.Config(n=n, length=length, bc=(wl.BC_NOSLIP, wl.BC_PERIODIC, wl.BC_PERIODIC),
                    nu=0.02, dt=0.005, delta=wl.DELTA_PESKIN4,
                    lump_c=wl.lump_constant(wl.DELTA_PESKIN4, h, K, radius), krylov_rtol=1e-12)
    c1 = np.array([0.25, 0.3, 0.3]) + rng.uniform(-0.01, 0.01, 3)
    c2 = np.array([0.25, 0.5, 0.75]) + rng.uniform(-0.01, 0.01, 3)
    bodies = [wl.Body(center=c1, vel=rng.normal(0, 0.1, 3), omega=np.array([0.0, 0.0, 1.0]),
                      radius=radius, n_points=K),
              wl.Body(center=c2, vel=rng.normal(0, 0.1, 3), omega=np.zeros(3), radius=radius,
                      n_points=K)]
    off = np.concatenate([wl.fibonacci_offsets(K, radius)] * 2)
    return wl.Workload("mixed_16x24x32", cfg, bodies, off, np.zeros((3,) + n), steps=1, seed=seed)
