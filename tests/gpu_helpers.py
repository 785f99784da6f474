"""Shared set-up for the GPU parity tests: the same seeded workload goes to the
HIP library (through the C ABI) and to the CPU oracle."""
import contextlib
import os

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


def freeslip_workload(n=32, pts=260, seed=3):
    """The wall-bounded spheres of walls_workload in a box with free-slip
    walls normal to x and y and no-slip walls normal to z, so that both
    ghost rules of the viscous stencil meet in one grid."""
    w = walls_workload(n, pts, seed)
    w.cfg.bc = (wl.BC_FREESLIP, wl.BC_FREESLIP, wl.BC_NOSLIP)
    w.name = w.name.replace("noslip", "freeslip_xy_noslip_z")
    return w


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


def odd_tiles_workload(seed=13):
    """A grid whose point-tile counts are odd along two axes (20 x 24 x 28
    cells of width 1/28: 5 x 6 x 7 tiles of 4^3 cells), so the spreading runs
    on 4^3-cell band tiles instead of 8^3; periodic, no-slip and free-slip
    axes; one sphere; the multigrid hierarchy stops at 10 x 12 x 14."""
    rng = np.random.default_rng(seed)
    n = (20, 24, 28)
    h = 1.0 / 28
    radius = 0.17
    K = 220
    cfg = wl.Config(n=n, length=tuple(x * h for x in n), bc=(wl.BC_PERIODIC, wl.BC_NOSLIP, wl.BC_FREESLIP),
                    nu=0.02, dt=0.005, delta=wl.DELTA_PESKIN4,
                    lump_c=wl.lump_constant(wl.DELTA_PESKIN4, h, K, radius), krylov_rtol=1e-12, mg_coarsest=14)
    c = np.array([0.3, 0.43, 0.5]) + rng.uniform(-0.01, 0.01, 3)
    bodies = [wl.Body(center=c, vel=rng.normal(0, 0.1, 3), omega=np.array([0.0, 1.0, 0.0]), radius=radius,
                      n_points=K)]
    return wl.Workload("odd_tiles_20x24x28", cfg, bodies, wl.fibonacci_offsets(K, radius), np.zeros((3,) + n),
                       steps=1, seed=seed)


def wrap16_workload(seed=14):
    """A 16^3 periodic box (two 8^3-cell band tiles per axis) with one sphere
    centred near a corner, so that point supports wrap across the x and z
    boundaries and reach the last face position of a band tile's box from
    the far side."""
    rng = np.random.default_rng(seed)
    n = (16, 16, 16)
    h = 1.0 / 16
    radius = 0.2
    K = 130
    cfg = wl.Config(n=n, length=(1.0, 1.0, 1.0), bc=(wl.BC_PERIODIC,) * 3, nu=0.02, dt=0.005,
                    delta=wl.DELTA_PESKIN4, lump_c=wl.lump_constant(wl.DELTA_PESKIN4, h, K, radius),
                    krylov_rtol=1e-12)
    c = np.array([0.97, 0.5, 0.03]) + rng.uniform(-0.01, 0.01, 3)
    bodies = [wl.Body(center=c, vel=rng.normal(0, 0.1, 3), omega=np.array([1.0, 0.0, 0.0]), radius=radius,
                      n_points=K)]
    return wl.Workload("wrap16_periodic", cfg, bodies, wl.fibonacci_offsets(K, radius), np.zeros((3,) + n),
                       steps=1, seed=seed)


def free_workload(n=32, bc=wl.BC_PERIODIC, seed=21, precision=wl.PREC_FP64, xi=0.6, outer_iters=3):
    """Two free spheres (a = 0.15, theta 1.5 and 2.5) under gravity, with small
    random initial velocities and spins in a random solenoidal flow (periodic)
    or in fluid at rest (no-slip walls)."""
    rng = np.random.default_rng(seed)
    h = 1.0 / n
    radius = 0.15
    K = int(round(4 * np.pi * radius ** 2 / h ** 2))
    cfg = wl.Config(n=(n, n, n), length=(1.0, 1.0, 1.0), bc=(bc,) * 3, nu=0.01, dt=0.002,
                    delta=wl.DELTA_PESKIN4, lump_c=wl.lump_constant(wl.DELTA_PESKIN4, h, K, radius),
                    precision=precision, krylov_rtol=1e-12 if precision == wl.PREC_FP64 else 1e-11,
                    helm_rtol=1e-12 if precision == wl.PREC_FP64 else 1e-11,
                    outer_iters=outer_iters, outer_tol=0.0, xi=xi)
    cfg.g = (0.0, 0.0, -1.0)
    centers = [np.array([0.3, 0.35, 0.6]), np.array([0.68, 0.62, 0.4])]
    bodies = []
    for c, theta in zip(centers, (1.5, 2.5)):
        bodies.append(wl.Body(center=c + rng.uniform(-0.01, 0.01, 3), vel=rng.normal(0, 0.05, 3),
                              omega=rng.normal(0, 0.5, 3), radius=radius, density_ratio=theta,
                              motion=wl.MOTION_FREE, n_points=K))
    off = np.concatenate([wl.fibonacci_offsets(K, radius)] * 2)
    if bc == wl.BC_PERIODIC:
        u0 = wl.solenoidal_field(rng, (n, n, n), h, 0.05)
    else:
        u0 = np.zeros((3, n, n, n))
    kind = {wl.BC_PERIODIC: "periodic", wl.BC_NOSLIP: "walls", wl.BC_FREESLIP: "freeslip"}[bc]
    return wl.Workload(f"free_{n}_{kind}", cfg, bodies, off, u0, steps=2, seed=seed)


def oracle_free_bodies(w: wl.Workload):
    from oracle import step as ostep
    out, k0 = [], 0
    for b in w.bodies:
        out.append(ostep.free_body(b.center, b.vel, b.omega, b.radius, b.density_ratio,
                                   w.offsets[k0:k0 + b.n_points], w.cfg.dt))
        k0 += b.n_points
    return out


def prescribed_points(w: wl.Workload, t: float):
    """Point positions and velocities of prescribed bodies at time t
    (X_k = X_c + R X~_k, U_k = u_s + omega x R X~_k)."""
    Xs, Us, k0 = [], [], 0
    for b in w.bodies:
        o = w.offsets[k0:k0 + b.n_points]
        c = obd.prescribed_center(b.center, b.vel, b.osc_amp, b.osc_omega, t)
        R = obd.prescribed_rotation(b.omega, t)
        lever = o @ R.T
        Xs.append(c[None, :] + lever)
        Us.append(obd.point_velocities(obd.prescribed_velocity(b.vel, b.osc_amp, b.osc_omega, t), b.omega, lever))
        k0 += b.n_points
    return np.concatenate(Xs), np.concatenate(Us)


# The plane-marching kernels run shorter chunks of planes per workgroup on
# small grids; the library reads IBSCHUR_MARCH_FULL_CHUNKS when a handle is
# created, and "1" gives every grid the full 8-plane chunks of the
# benchmark-size grids.  Parity tests run both launch shapes.
CHUNKS = ["auto", "full"]


@contextlib.contextmanager
def march_chunks(mode: str):
    """Environment for sim_create: mode "full" forces 8-plane chunks."""
    old = os.environ.get("IBSCHUR_MARCH_FULL_CHUNKS")
    if mode == "full":
        os.environ["IBSCHUR_MARCH_FULL_CHUNKS"] = "1"
    else:
        os.environ.pop("IBSCHUR_MARCH_FULL_CHUNKS", None)
    try:
        yield
    finally:
        if old is None:
            os.environ.pop("IBSCHUR_MARCH_FULL_CHUNKS", None)
        else:
            os.environ["IBSCHUR_MARCH_FULL_CHUNKS"] = old


@contextlib.contextmanager
def mg_tile_cells(cells):
    """Environment for sim_create: multigrid levels of at most `cells` cells
    run as tile levels (0: none; None: the library's default)."""
    old = os.environ.get("IBSCHUR_MG_TILE_CELLS")
    if cells is None:
        os.environ.pop("IBSCHUR_MG_TILE_CELLS", None)
    else:
        os.environ["IBSCHUR_MG_TILE_CELLS"] = str(int(cells))
    try:
        yield
    finally:
        if old is None:
            os.environ.pop("IBSCHUR_MG_TILE_CELLS", None)
        else:
            os.environ["IBSCHUR_MG_TILE_CELLS"] = old


def make_sim(cfg, max_points, chunks: str = "auto"):
    """A Sim created under the given plane-march chunking."""
    from paper_2501_15314_amd.sim import Sim
    with march_chunks(chunks):
        return Sim(cfg, max_points)
