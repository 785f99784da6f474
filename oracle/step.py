"""One-way and two-way time steps of the SIMPLE-IBM scheme, FP64.

Paper Sec. 3.1 (eqs. ustar, utag, unplus1, divfree, modified_poisson,
u_n_plus_1, Saddle) and Sec. 3.2.1 (Steps 1-3, eqs. particle_position,
ustar_two_way, bdy_linear_vel_iter, bdy_angular_vel_iter,
kinematic_constraint_iterative, pressure_force_iterative_system, the relaxed
update with xi and eq. convergence_criterion).

Readings:
  * tau = 2 dt / 3 (the BDF2 factor of eq. u_n_plus_1);
  * RHS_p = -D u* / tau and RHS_F = (W^T u* - U) / tau (below eq. Saddle);
  * all body data (points X_k, velocities U_k) and hence W are taken at
    t^{n+1}; the force of the previous level, Phi^n, is spread with that W;
  * BDF2 from the first step with u^{-1} = u^0, p^0 = 0, Phi^0 = 0;
  * Phi is the solver's force unknown: the paper's force density times the
    shell volume, divided by h^3, so that the spread force on the grid is W Phi.
"""
from __future__ import annotations

import dataclasses

import numpy as np

from . import bodies as bd
from . import delta, mac
from .schur import SchurSystem


@dataclasses.dataclass
class State:
    u: np.ndarray        # (3, n0, n1, n2) at t^n
    um: np.ndarray       # (3, n0, n1, n2) at t^{n-1}
    p: np.ndarray        # (n0, n1, n2)
    phi: np.ndarray      # (K, 3)
    t: float = 0.0

    def copy(self):
        return State(self.u.copy(), self.um.copy(), self.p.copy(), self.phi.copy(), self.t)


def cg(matvec, b, rtol=1e-14, maxit=1000):
    """Plain conjugate gradients for the SPD momentum operator."""
    x = np.zeros_like(b)
    r = b.copy()
    p = r.copy()
    rr = r @ r
    bn = np.sqrt(b @ b)
    if bn == 0.0:
        return x, 0
    for it in range(1, maxit + 1):
        Ap = matvec(p)
        alpha = rr / (p @ Ap)
        x += alpha * p
        r -= alpha * Ap
        rr_new = r @ r
        if np.sqrt(rr_new) <= rtol * bn:
            return x, it
        p = r + (rr_new / rr) * p
        rr = rr_new
    return x, maxit


def momentum_rhs(g: mac.Grid, dt, u, um, p, phi, W):
    """(4u^n - u^{n-1})/(2dt) - G p^n + W Phi^n - N(u^n), eq. ustar without the
    implicit viscous term (which is in the operator A)."""
    G = mac.gradient(g)
    mask = g.face_dof_mask()
    rhs = (4.0 * u - um) / (2.0 * dt) - (G @ p.ravel()).reshape(u.shape) \
        + delta.spread(W, phi, g.n) - mac.convection(g, u)
    return rhs * mask


def helmholtz_solve(g: mac.Grid, nu, dt, rhs, rtol=1e-14):
    """u* = A^{-1} rhs on the unknown faces (A = 3/(2dt) I - nu Delta_h)."""
    A = mac.helmholtz(g, nu, dt)
    mask = g.face_dof_mask().ravel()
    Ad = A[mask][:, mask]
    x, its = cg(lambda v: Ad @ v, rhs.ravel()[mask], rtol=rtol)
    out = np.zeros(3 * g.N)
    out[mask] = x
    return out.reshape((3,) + g.n), its


def correction(sys: SchurSystem, ustar, U, dt, xi=1.0, rtol=1e-13):
    """One pressure / force correction (eqs. Saddle, ApproxSchurPrimalP/F,
    u_n_plus_1): returns (u_new, p', Phi', info)."""
    g = sys.g
    tau = 2.0 * dt / 3.0
    mask = g.face_dof_mask()
    rhs_p = -(sys.D @ ustar.ravel()).reshape(g.n) / tau
    rhs_f = (delta.interpolate(sys.W, ustar) - U) / tau
    pp, phip, its, hist = sys.solve(rhs_p, rhs_f, rtol=rtol)
    du = -(sys.G @ pp.ravel()).reshape(ustar.shape) + delta.spread(sys.W, phip, g.n)
    unew = (ustar + xi * tau * du) * mask
    return unew, pp, phip, dict(iters=its, hist=hist, rhs_p=rhs_p, rhs_f=rhs_f)


def one_way_step(g: mac.Grid, nu, dt, state: State, X, U, kernel, c, xi=1.0,
                 helm_rtol=1e-14, schur_rtol=1e-13):
    """Prescribed-motion step: predictor, one correction (footnote of Sec. 3.1)."""
    W = delta.regularization_matrix(g, X, kernel)
    rhs = momentum_rhs(g, dt, state.u, state.um, state.p, state.phi, W)
    ustar, hits = helmholtz_solve(g, nu, dt, rhs, helm_rtol)
    sys = SchurSystem(g, W, c)
    unew, pp, phip, info = correction(sys, ustar, U, dt, xi, schur_rtol)
    new = State(unew, state.u.copy(), state.p + xi * pp, state.phi + xi * phip,
                state.t + dt)
    info.update(ustar=ustar, pprime=pp, phiprime=phip, helm_iters=hits, W=W, sys=sys)
    return new, info


# ---------------------------------------------------------------------------
# two-way coupling

@dataclasses.dataclass
class FreeBody:
    radius: float
    theta: float
    offsets: np.ndarray          # (k, 3) body frame
    xc: np.ndarray               # X_c^n
    xc_m: np.ndarray             # X_c^{n-1}
    us: np.ndarray               # u_s^n
    us_m: np.ndarray             # u_s^{n-1}
    w: np.ndarray                # omega^n (inertial)
    w_m: np.ndarray              # omega^{n-1}
    R: np.ndarray                # R^n
    I_n: np.ndarray = None       # sum alpha u h^3 at level n
    I_m: np.ndarray = None       # ... at level n-1
    J_n: np.ndarray = None
    J_m: np.ndarray = None

    def copy(self):
        return dataclasses.replace(self, **{f.name: (getattr(self, f.name).copy()
                                                      if isinstance(getattr(self, f.name), np.ndarray)
                                                      else getattr(self, f.name))
                                            for f in dataclasses.fields(self)})


def free_body(center, vel, omega, radius, theta, offsets, dt):
    """A free sphere entering the first step in steady motion: u_s^{-1} = u_s^0,
    omega^{-1} = omega^0, and the consistent centre X_c^{-1} = X_c^0 - dt u_s^0
    (so that Step 1's BDF2 prediction advances a steadily moving body by
    dt u_s); orientation R^0 = I."""
    c = np.asarray(center, dtype=np.float64)
    v = np.asarray(vel, dtype=np.float64)
    w = np.asarray(omega, dtype=np.float64)
    return FreeBody(radius=float(radius), theta=float(theta),
                    offsets=np.asarray(offsets, dtype=np.float64), xc=c.copy(), xc_m=c - dt * v,
                    us=v.copy(), us_m=v.copy(), w=w.copy(), w_m=w.copy(), R=np.eye(3))


def domain_length(g: mac.Grid):
    return tuple(n * g.h for n in g.n)


def init_volume_history(g: mac.Grid, u, bodies):
    for b in bodies:
        I, J = bd.volume_integrals(g, u, b.xc, b.radius, domain_length(g))
        b.I_n, b.J_n = I, J
        b.I_m, b.J_m = I.copy(), J.copy()


def two_way_step(g: mac.Grid, nu, dt, gvec, state: State, bodies, kernel, c, xi,
                 n_outer, outer_tol=0.0, schur_rtol=1e-13, helm_rtol=1e-14):
    """Sec. 3.2.1.  n_outer fixes the number of Step-3 iterations; with
    outer_tol > 0 the loop also stops on eq. convergence_criterion."""
    nb = len(bodies)
    # Step 1: explicit prediction of positions and orientations
    xc1 = [(4.0 * b.xc - b.xc_m) / 3.0 + (2.0 * dt / 3.0) * b.us for b in bodies]
    R1 = [bd.rotation_step(b.R, b.w, b.w_m, dt) for b in bodies]
    levers = [b.offsets @ R.T for b, R in zip(bodies, R1)]
    X = np.concatenate([x[None, :] + lv for x, lv in zip(xc1, levers)])
    counts = [b.offsets.shape[0] for b in bodies]
    starts = np.concatenate([[0], np.cumsum(counts)])
    W = delta.regularization_matrix(g, X, kernel)
    # Step 2: Eulerian predictor
    rhs = momentum_rhs(g, dt, state.u, state.um, state.p, state.phi, W)
    uk, _ = helmholtz_solve(g, nu, dt, rhs, helm_rtol)
    sys = SchurSystem(g, W, c)
    p = state.p.copy()
    phi = state.phi.copy()
    h3 = g.h ** 3
    crit_hist, iters = [], []
    us_k = [b.us.copy() for b in bodies]
    w_k = [b.w.copy() for b in bodies]
    used = [None] * nb
    # per-pass record for the reverse-mode step (no arithmetic of its own)
    rec = dict(u=[], phi=[], pp=[], phip=[], rhs_f=[], U=[], us=[], w=[], u0=uk.copy())
    for k in range(n_outer):
        U = np.empty_like(X)
        for ib, b in enumerate(bodies):
            s0, s1 = starts[ib], starts[ib + 1]
            F = h3 * phi[s0:s1].sum(axis=0)
            T = h3 * np.cross(levers[ib], phi[s0:s1]).sum(axis=0)
            Ik, Jk = bd.volume_integrals(g, uk, xc1[ib], b.radius, domain_length(g))
            us_k[ib], w_k[ib] = bd.newton_euler(b.theta, b.radius, dt, b.us, b.us_m, b.w, b.w_m,
                                                F, T, Ik, b.I_n, b.I_m, Jk, b.J_n, b.J_m, gvec)
            U[s0:s1] = bd.point_velocities(us_k[ib], w_k[ib], levers[ib])
            used[ib] = dict(F=F, T=T, I=Ik, J=Jk)
        rec["u"].append(uk.copy())
        rec["phi"].append(phi.copy())
        rec["U"].append(U.copy())
        rec["us"].append([v.copy() for v in us_k])
        rec["w"].append([v.copy() for v in w_k])
        uk, pp, phip, info = correction(sys, uk, U, dt, xi, schur_rtol)
        rec["pp"].append(pp)
        rec["phip"].append(phip)
        rec["rhs_f"].append(info["rhs_f"])
        p = p + xi * pp
        phi = phi + xi * phip
        iters.append(info["iters"])
        denom = np.abs(phi).sum()
        crit = np.abs(phip).sum() / denom if denom > 0 else np.inf
        crit_hist.append(crit)
        if outer_tol > 0.0 and crit < outer_tol:
            break
    new_bodies = []
    for ib, b in enumerate(bodies):
        nbody = b.copy()
        nbody.xc_m, nbody.xc = b.xc.copy(), xc1[ib]
        nbody.us_m, nbody.us = b.us.copy(), us_k[ib]
        nbody.w_m, nbody.w = b.w.copy(), w_k[ib]
        nbody.R = R1[ib]
        I1, J1 = bd.volume_integrals(g, uk, xc1[ib], b.radius, domain_length(g))
        nbody.I_m, nbody.I_n = b.I_n.copy(), I1
        nbody.J_m, nbody.J_n = b.J_n.copy(), J1
        new_bodies.append(nbody)
    new = State(uk, state.u.copy(), p, phi, state.t + dt)
    return new, new_bodies, dict(crit=crit_hist, iters=iters, X=X, W=W, used=used, sys=sys,
                                 xc1=xc1, R1=R1, levers=levers, starts=starts, rec=rec)
