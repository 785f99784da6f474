"""Seeded synthetic inputs shared by the GPU path, the tests and the benchmark.

This module only draws numbers: grid and physical parameters, sphere centres,
radii, velocities and density ratios, Lagrangian point offsets on a Fibonacci
(golden-angle) sphere lattice, random initial velocity fields and random
right-hand sides.  It contains none of the solver's arithmetic (no stencils,
no delta kernels, no Krylov or multigrid code), so both the HIP path and the
CPU reference consume exactly the same arrays.

The workloads stand in for the paper's own sphere-in-box experiments
(Sec. 6.1.1, oscillating sphere; Sec. 6.1.2, porous sphere arrays; Sec. 6.1.3,
sedimentation): no dataset is involved.

Array layout conventions (identical on both sides):
  * grid fields are float64 arrays of shape (n0, n1, n2), axis 2 contiguous;
  * cell (i,j,k) is centred at ((i+1/2)h, (j+1/2)h, (k+1/2)h);
  * velocity component d at index (i,j,k) sits on the face of cell (i,j,k)
    that is lower along axis d; on a no-slip axis d that index-0 face is the
    wall and always holds 0;
  * Lagrangian arrays are (K, 3) float64, bodies stored one after another.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional

import numpy as np

BC_PERIODIC = 0
BC_NOSLIP = 1
BC_FREESLIP = 2
DELTA_PESKIN4 = 0
DELTA_ROMA3 = 1
PREC_FP64 = 0
PREC_FP32MG = 1
MOTION_PRESCRIBED = 0
MOTION_FREE = 1
PRECOND_VCYCLE = 0
PRECOND_FASTDIAG = 1
PRECOND_FASTDIAG_EXACT = 2
KRYLOV_FGMRES = 0
KRYLOV_BICGSTAB = 1

# Sum over integer shifts j of phi(r - j)^2 for the two kernels (independent of
# r for both).  Used only to size the scalar lumping constant of C = W^T W.
_SUM_PHI_SQ = {DELTA_PESKIN4: 3.0 / 8.0, DELTA_ROMA3: 1.0 / 2.0}


@dataclasses.dataclass
class Config:
    n: tuple = (32, 32, 32)
    length: tuple = (1.0, 1.0, 1.0)
    bc: tuple = (BC_PERIODIC, BC_PERIODIC, BC_PERIODIC)
    nu: float = 0.01
    dt: float = 0.01
    g: tuple = (0.0, 0.0, 0.0)
    delta: int = DELTA_PESKIN4
    lump_c: float = 0.375
    precision: int = PREC_FP64
    krylov_restart: int = 20
    krylov_maxit: int = 200
    krylov_rtol: float = 1e-10
    helm_maxit: int = 50
    helm_rtol: float = 1e-10
    # V(2,1) down to 8^3, solved there exactly by fast diagonalisation
    # (mg_coarse_sweeps = 0; k > 0 runs k LDS V-cycles instead): the fastest
    # setting measured for the 256^3 solves (11 FGMRES iterations)
    mg_coarsest: int = 8
    mg_pre: int = 2
    mg_post: int = 1
    mg_coarse_sweeps: int = 0
    precond: int = 0            # PRECOND_VCYCLE or PRECOND_FASTDIAG
    krylov: int = 0             # KRYLOV_FGMRES or KRYLOV_BICGSTAB
    outer_iters: int = 1
    outer_tol: float = 0.0
    xi: float = 1.0
    record_two_way: int = 0     # keep the outer passes for the reverse-mode two-way step
    device: int = 0

    @property
    def h(self) -> float:
        return self.length[0] / self.n[0]

    @property
    def ncell(self) -> int:
        return self.n[0] * self.n[1] * self.n[2]


@dataclasses.dataclass
class Body:
    center: np.ndarray          # (3,) centre at t = 0
    vel: np.ndarray             # (3,) translational velocity
    omega: np.ndarray           # (3,) angular velocity (inertial frame)
    radius: float
    density_ratio: float = 1.0
    motion: int = MOTION_PRESCRIBED
    n_points: int = 0
    osc_amp: np.ndarray = dataclasses.field(default_factory=lambda: np.zeros(3))
    osc_omega: float = 0.0


@dataclasses.dataclass
class Workload:
    name: str
    cfg: Config
    bodies: List[Body]
    offsets: np.ndarray         # (K, 3) body-frame offsets, bodies in order
    u0: np.ndarray              # (3, n0, n1, n2) initial velocity (level n)
    steps: int = 1
    seed: int = 0

    @property
    def n_points(self) -> int:
        return int(self.offsets.shape[0])


def fibonacci_offsets(n_points: int, radius: float) -> np.ndarray:
    """Golden-angle (Fibonacci) lattice on a sphere of the given radius.

    z_q = 1 - (2q+1)/N, rho_q = sqrt(1 - z_q^2), azimuth q*pi*(3 - sqrt 5).
    Every point carries the same share of the surface area, as the paper's
    equal-area partition does (Sec. 6.1.1)."""
    q = np.arange(n_points, dtype=np.float64)
    z = 1.0 - (2.0 * q + 1.0) / n_points
    rho = np.sqrt(np.maximum(0.0, 1.0 - z * z))
    th = q * math.pi * (3.0 - math.sqrt(5.0))
    return radius * np.stack([rho * np.cos(th), rho * np.sin(th), z], axis=1)


def lump_constant(delta: int, h: float, n_points: int, radius: float) -> float:
    """Scalar c in C = W^T W ~ c I, rescaled by the marker density.

    At Lagrangian spacing equal to h the row sums of W^T W equal the sum of
    the squared 1-D kernel weights (1/2 for the 3-point kernel, which is the
    paper's C ~ I/2 of Sec. 4.1); at other spacings they scale with
    (h / h_L)^2 (Appendix A, rescaled lumping)."""
    area_per_point = 4.0 * math.pi * radius * radius / n_points
    return _SUM_PHI_SQ[delta] * h * h / area_per_point


def solenoidal_field(rng: np.random.Generator, n, h: float, sigma: float) -> np.ndarray:
    """Random periodic MAC velocity field that is discretely divergence-free.

    Built as the staggered curl of a random edge-centred vector potential, so
    no pressure solve is needed to make it solenoidal; the per-face standard
    deviation is about sigma."""
    n0, n1, n2 = n
    a = rng.standard_normal((3, n0, n1, n2)) * (sigma * h / 2.0)
    ax, ay, az = a

    def fwd(f, axis):  # f(idx + e_axis) - f(idx)
        return np.roll(f, -1, axis=axis) - f

    u = np.empty((3, n0, n1, n2))
    # u_x(i,j,k) = [Az(i,j+1,k)-Az(i,j,k) - (Ay(i,j,k+1)-Ay(i,j,k))]/h
    u[0] = (fwd(az, 1) - fwd(ay, 2)) / h
    u[1] = (fwd(ax, 2) - fwd(az, 0)) / h
    u[2] = (fwd(ay, 0) - fwd(ax, 1)) / h
    return u


def _cfg(n, bc, nu, dt, n_points, radius, delta=DELTA_PESKIN4, **kw) -> Config:
    h = 1.0 / n
    return Config(n=(n, n, n), length=(1.0, 1.0, 1.0), bc=(bc, bc, bc), nu=nu, dt=dt,
                  delta=delta, lump_c=lump_constant(delta, h, n_points, radius), **kw)


def make_c1(seed: int = 1, n: int = 32, n_points: int = 300) -> Workload:
    """One sphere (a = 0.15) translating at (0.1, 0, 0) in a periodic unit box."""
    rng = np.random.default_rng(seed)
    radius = 0.15
    center = 0.5 + rng.uniform(-0.02, 0.02, 3)
    cfg = _cfg(n, BC_PERIODIC, 0.01, 0.01, n_points, radius, krylov_rtol=1e-10)
    body = Body(center=center, vel=np.array([0.1, 0.0, 0.0]), omega=np.zeros(3),
                radius=radius, n_points=n_points)
    u0 = solenoidal_field(rng, cfg.n, cfg.h, 1e-3)
    return Workload("c1_32cube_periodic_1sphere", cfg, [body],
                    fibonacci_offsets(n_points, radius), u0, steps=1, seed=seed)


def make_c2(seed: int = 2, n: int = 128, n_points: int = 5000) -> Workload:
    """One sphere (a = 0.1) oscillating along x (amplitude 0.05, period 1)."""
    radius = 0.1
    cfg = _cfg(n, BC_PERIODIC, 0.01, 0.005, n_points, radius, krylov_rtol=1e-8,
               precision=PREC_FP32MG)
    body = Body(center=np.array([0.5, 0.5, 0.5]), vel=np.zeros(3), omega=np.zeros(3),
                radius=radius, n_points=n_points,
                osc_amp=np.array([0.05, 0.0, 0.0]), osc_omega=2.0 * math.pi)
    u0 = np.zeros((3, n, n, n))
    return Workload("c2_128cube_periodic_oscillating_sphere", cfg, [body],
                    fibonacci_offsets(n_points, radius), u0, steps=50, seed=seed)


def random_centers(rng, count, lo, hi, min_sep, max_tries=100000):
    centers = []
    tries = 0
    while len(centers) < count:
        tries += 1
        if tries > max_tries:
            raise RuntimeError("could not place non-overlapping centres")
        c = rng.uniform(lo, hi, 3)
        if all(np.linalg.norm(c - o) >= min_sep for o in centers):
            centers.append(c)
    return centers


def make_c3(seed: int = 3, n: int = 256, points_per_sphere: int = 18000,
            n_spheres: int = 8, radius: float = 0.06) -> Workload:
    """Eight spheres (a = 0.06) with constant random velocities, no-slip box."""
    rng = np.random.default_rng(seed)
    centers = random_centers(rng, n_spheres, 0.16, 0.84, 0.15)
    vels = [rng.normal(0.0, 0.05, 3) for _ in range(n_spheres)]
    cfg = _cfg(n, BC_NOSLIP, 0.005, 0.002, points_per_sphere, radius, krylov_rtol=1e-8,
               precision=PREC_FP32MG)
    bodies = [Body(center=c, vel=v, omega=np.zeros(3), radius=radius,
                   n_points=points_per_sphere) for c, v in zip(centers, vels)]
    off = np.concatenate([fibonacci_offsets(points_per_sphere, radius)] * n_spheres)
    u0 = np.zeros((3, n, n, n))
    return Workload("c3_256cube_noslip_8spheres", cfg, bodies, off, u0, steps=20, seed=seed)


def make_c4(seed: int = 4, n: int = 128, points_per_sphere: int = 5000) -> Workload:
    """Two spheres (a = 0.1) 0.3 apart with random velocities, periodic box."""
    rng = np.random.default_rng(seed)
    radius = 0.1
    c1 = rng.uniform(0.35, 0.65, 3)
    d = rng.standard_normal(3)
    d /= np.linalg.norm(d)
    c2 = np.mod(c1 + 0.3 * d, 1.0)
    v1 = rng.normal(0.0, 0.1, 3)
    v2 = rng.normal(0.0, 0.1, 3)
    cfg = _cfg(n, BC_PERIODIC, 0.01, 0.005, points_per_sphere, radius, krylov_rtol=1e-12)
    bodies = [Body(center=c1, vel=v1, omega=np.zeros(3), radius=radius, n_points=points_per_sphere),
              Body(center=c2, vel=v2, omega=np.zeros(3), radius=radius, n_points=points_per_sphere)]
    off = np.concatenate([fibonacci_offsets(points_per_sphere, radius)] * 2)
    u0 = np.zeros((3, n, n, n))
    return Workload("c4_128cube_periodic_2spheres_adjoint", cfg, bodies, off, u0, steps=1,
                    seed=seed)


def make_c5(seed: int = 5, n: int = 384, points_per_sphere: int = 18000,
            radius: float = 0.04) -> Workload:
    """27 free spheres (a = 0.04) on a jittered 3x3x3 lattice under gravity."""
    rng = np.random.default_rng(seed)
    centers = []
    for x in (0.25, 0.5, 0.75):
        for y in (0.25, 0.5, 0.75):
            for z in (0.25, 0.5, 0.75):
                centers.append(np.array([x, y, z]))
    centers = [c + rng.uniform(-0.02, 0.02, 3) for c in centers]
    thetas = rng.uniform(0.8, 1.5, len(centers))
    cfg = _cfg(n, BC_NOSLIP, 0.002, 0.001, points_per_sphere, radius, krylov_rtol=1e-8,
               precision=PREC_FP32MG, outer_iters=3, outer_tol=1e-3, xi=0.6)
    cfg.g = (0.0, 0.0, -1.0)
    bodies = [Body(center=c, vel=np.zeros(3), omega=np.zeros(3), radius=radius,
                   density_ratio=float(t), motion=MOTION_FREE, n_points=points_per_sphere)
              for c, t in zip(centers, thetas)]
    off = np.concatenate([fibonacci_offsets(points_per_sphere, radius)] * len(centers))
    u0 = np.zeros((3, n, n, n))
    return Workload("c5_384cube_noslip_27free_spheres", cfg, bodies, off, u0, steps=100,
                    seed=seed)


# Porous sphere of diameter D modelled by solid sub-spheres packed inside it
# (Sec. 6.1.2): sub-sphere radius r D and centres in units of D / 10, from the
# paper's table of the 7- and 14-sub-sphere configurations.
POROUS_CONFIGS = {
    7: (0.193, [(1.1140, -1.9296, -2.1126), (-2.2281, 0.0, -2.1126), (1.1140, 1.9296, -2.1126),
                (-1.5009, -2.5997, 0.64522), (3.0019, 0.0, 0.64522), (-1.5009, 2.5997, 0.64522),
                (0.0, 0.0, 3.0704)]),
    14: (0.161, [(0.0, -2.287, -2.4917), (-2.2875, 0.0, -2.4917), (2.2875, 0.0, -2.4917), (0.0, 2.2875, -2.4917),
                 (-2.3820, -2.3820, -0.30478), (2.3820, -2.3820, -0.30478), (-2.3820, 2.3820, -0.30478),
                 (2.3820, 2.3820, -0.30478), (0.0, 0.0, 0.0), (0.0, -2.8412, 1.8355), (-2.8412, 0.0, 1.8355),
                 (2.8412, 0.0, 1.8355), (0.0, 2.8412, 1.8355), (0.0, 0.0, 3.3825)]),
}


def make_porous(n_sub: int = 7, cells_per_d: int = 32, re: float = 100.0, amp: float = 1.0,
                precision: int = PREC_FP64) -> Workload:
    """Oscillating porous sphere (Sec. 6.1.2, the oscillation law of Sec. 6.1.1):
    bounding sphere of diameter D = 1 at the centre of a 4D x 4D x 6D no-slip
    box, n_sub rigid sub-spheres of radius r D - h/2 at the tabulated centres,
    all moving with z(t) = -A cos(t / A) (u_z = sin(t / A), U_max = 1), nu =
    1/Re, Roma 3-point kernel, markers at spacing ~h, time step at CFL 0.1.
    The grid is (4, 4, 6) x cells_per_d (multiples of 8 so that every
    multigrid level keeps the plane-march layout)."""
    r, centres = POROUS_CONFIGS[n_sub]
    n = (4 * cells_per_d, 4 * cells_per_d, 6 * cells_per_d)
    h = 1.0 / cells_per_d
    radius = r - 0.5 * h
    n_points = max(8, int(round(4.0 * math.pi * radius * radius / (h * h))))
    box_centre = np.array([2.0, 2.0, 3.0])
    cfg = Config(n=n, length=(4.0, 4.0, 6.0), bc=(BC_NOSLIP,) * 3, nu=1.0 / re, dt=0.1 * h,
                 delta=DELTA_ROMA3, lump_c=lump_constant(DELTA_ROMA3, h, n_points, radius),
                 precision=precision, krylov_rtol=1e-8)
    bodies = []
    for c in centres:
        # centre(t) = centre - A cos(t / A) e_z: the stroke z in [-A, A] about
        # the box centre, starting at its lowest point
        bodies.append(Body(center=box_centre + 0.1 * np.array(c), vel=np.zeros(3),
                           omega=np.zeros(3), radius=radius, n_points=n_points,
                           osc_amp=np.array([0.0, 0.0, amp]), osc_omega=1.0 / amp))
    offsets = np.concatenate([fibonacci_offsets(n_points, radius) for _ in centres])
    u0 = np.zeros((3,) + n)
    return Workload(f"porous{n_sub}_{n[0]}x{n[1]}x{n[2]}", cfg, bodies, offsets, u0, steps=1, seed=0)



def make_oscillating_sphere(cells_per_d: int = 16, re: float = 100.0, amp: float = 1.0,
                            precision: int = PREC_FP64) -> Workload:
    """The oscillating sphere of Sec. 6.1.1: a solid sphere of diameter D = 1
    at the centre of a 4D x 4D x 6D no-slip box moving with
    z(t) = -A cos(t / A) (u_z = sin(t / A), U_max = 1), nu = 1/Re, Roma
    3-point kernel, markers at spacing ~h on the sphere retracted by h/2,
    time step at CFL 0.1."""
    n = (4 * cells_per_d, 4 * cells_per_d, 6 * cells_per_d)
    h = 1.0 / cells_per_d
    radius = 0.5 - 0.5 * h
    n_points = max(8, int(round(4.0 * math.pi * radius * radius / (h * h))))
    cfg = Config(n=n, length=(4.0, 4.0, 6.0), bc=(BC_NOSLIP,) * 3, nu=1.0 / re, dt=0.1 * h,
                 delta=DELTA_ROMA3, lump_c=lump_constant(DELTA_ROMA3, h, n_points, radius),
                 precision=precision, krylov_rtol=1e-8)
    body = Body(center=np.array([2.0, 2.0, 3.0]), vel=np.zeros(3), omega=np.zeros(3), radius=radius,
                n_points=n_points, osc_amp=np.array([0.0, 0.0, amp]), osc_omega=1.0 / amp)
    u0 = np.zeros((3,) + n)
    return Workload(f"oscillating_sphere_{n[0]}x{n[1]}x{n[2]}", cfg, [body],
                    fibonacci_offsets(n_points, radius), u0, steps=1, seed=0)

# Settling sphere in a quiescent fluid (Sec. 6.1.3): density ratio,
# particle Reynolds number Re_p = U D / nu and Froude number Fr = U / sqrt(g D)
# of the two cases of the paper's settling figure.
SEDIMENTATION_CASES = {
    "re11": (1.164, 11.6, 0.237),
    "re32": (1.167, 31.9, 0.334),
}


def make_sedimentation(case: str = "re11", cells_per_d: int = 16,
                       precision: int = PREC_FP32MG, spacing_ratio: float = 1.0,
                       lump_c: Optional[float] = None) -> Workload:
    """Free sphere of diameter D = 1 released from rest on the vertical centre
    line at height 8.5 D of a 10D x 10D x 15D box with free-slip walls on all
    faces (Sec. 6.1.3).  Units D = 1 and |g| = 1, so that the terminal velocity
    is Fr and nu = Fr / Re_p.  Markers on a sphere of radius D/2 - h/2 (the
    regularised force layer reaches about half a cell outside the markers),
    spacing ~h; the body itself (mass, buoyancy and the volume integrals of
    Newton-Euler) keeps its physical radius D/2;
    Roma 3-point kernel, time step at CFL 0.1 for a unit velocity, relaxation
    0.6 (the paper's value for the smallest density ratios), outer loop until
    the relative l1 change of the force density drops below 1e-3 (the paper's
    tolerance) or after 3 passes (the count the paper reports; with the
    lumped W^T W ~ c I the criterion levels off near 1e-2, set by marker
    modes that the grid barely sees).  The grid is
    (10, 10, 15) x cells_per_d; cells_per_d a multiple of 8 keeps every axis
    a multiple of 8 for the fast-diagonalisation preconditioner, which the
    workload uses (the 15 D axis does not halve to the multigrid coarse size).
    spacing_ratio = h / h_L sets the marker spacing h_L (the sweep of
    Appendix A: markers ~ 4 pi a^2 / h_L^2); lump_c overrides the lumping
    constant, which otherwise is rescaled by the marker density."""
    theta, re, fr = SEDIMENTATION_CASES[case]
    n = (10 * cells_per_d, 10 * cells_per_d, 15 * cells_per_d)
    h = 1.0 / cells_per_d
    radius = 0.5 - 0.5 * h
    n_points = int(round(4.0 * math.pi * radius * radius * (spacing_ratio / h) ** 2))
    c = lump_constant(DELTA_ROMA3, h, n_points, radius) if lump_c is None else float(lump_c)
    cfg = Config(n=n, length=(10.0, 10.0, 15.0), bc=(BC_FREESLIP,) * 3, nu=fr / re, dt=0.1 * h,
                 delta=DELTA_ROMA3, lump_c=c,
                 precision=precision, krylov_rtol=1e-8, precond=PRECOND_FASTDIAG,
                 outer_iters=3, outer_tol=1e-3, xi=0.6)
    cfg.g = (0.0, 0.0, -1.0)
    body = Body(center=np.array([5.0, 5.0, 8.5]), vel=np.zeros(3), omega=np.zeros(3), radius=0.5,
                density_ratio=theta, motion=MOTION_FREE, n_points=n_points)
    u0 = np.zeros((3,) + n)
    return Workload(f"sedimentation_{case}_{n[0]}x{n[1]}x{n[2]}_freeslip", cfg, [body],
                    fibonacci_offsets(n_points, radius), u0, steps=1, seed=0)


def scaled(make, n: int, **kw) -> Workload:
    """The same geometry on an n^3 grid with the marker count scaled as h^-2."""
    w0 = make()
    ratio = (n / w0.cfg.n[0]) ** 2
    if make is make_c1:
        return make_c1(n=n, n_points=max(8, int(round(300 * ratio))), **kw)
    if make is make_c3:
        return make_c3(n=n, points_per_sphere=max(8, int(round(18000 * ratio))), **kw)
    if make is make_c4:
        return make_c4(n=n, points_per_sphere=max(8, int(round(5000 * ratio))), **kw)
    if make is make_c2:
        return make_c2(n=n, n_points=max(8, int(round(5000 * ratio))), **kw)
    if make is make_c5:
        return make_c5(n=n, points_per_sphere=max(8, int(round(18000 * ratio))), **kw)
    raise ValueError(make)


def body_positions_at(w: Workload, t: float) -> np.ndarray:
    """Centres of prescribed bodies at time t (constant velocity plus the
    paper's oscillation law x_c = x_0 - A cos(omega t), Sec. 6.1.1)."""
    out = []
    for b in w.bodies:
        out.append(b.center + b.vel * t - b.osc_amp * math.cos(b.osc_omega * t))
    return np.array(out)


def random_schur_rhs(seed: int, n, n_points: int):
    """Random right-hand side for a pressure-force solve: rhs_p ~ N(0,1) with its
    mean removed, rhs_f ~ N(0,1) per point and component (the paper's
    random-RHS experiment, Sec. 6.2)."""
    rng = np.random.default_rng(seed)
    rp = rng.standard_normal(tuple(n))
    rp -= rp.mean()
    rf = rng.standard_normal((n_points, 3))
    return rp, rf


def random_fields(seed: int, n, n_points: int, scale: float = 1.0):
    """Random state (u^n, u^{n-1}, p^n, Phi^n) for operator-level parity tests."""
    rng = np.random.default_rng(seed)
    u = rng.standard_normal((3,) + tuple(n)) * scale
    um = rng.standard_normal((3,) + tuple(n)) * scale
    p = rng.standard_normal(tuple(n)) * scale
    phi = rng.standard_normal((n_points, 3)) * scale
    return u, um, p, phi
