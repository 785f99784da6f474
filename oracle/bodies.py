"""Rigid spherical bodies: kinematics, rotation update, Newton-Euler, volume
fractions.

Paper Sec. 2.1 (eq. kinematic_constraint: U = u_s + omega x L~), Sec. 2.2
(rotation update: AB2 angle, Rodrigues formula, R^{n+1} = R^n R_Delta),
Sec. 3.2 (eq. volume_integrals with the volume fractions of Kempe & Uhlmann),
Sec. 3.2.1 (Step 1 position prediction, Step 3 discrete linear / angular
momentum equations).

Readings:
  * Newton-Euler is written dimensionally with fluid density 1:
      theta V_p du/dt = -h^3 sum Phi + d/dt sum alpha u h^3 + (theta - 1) V_p g
      theta I_p dw/dt = -h^3 sum L~ x Phi + d/dt sum alpha r x u h^3
    with V_p = 4 pi a^3 / 3 and I_p = 2/5 V_p a^2; at D = 1 these reduce to the
    printed non-dimensional coefficients 6/(pi theta) and 60/(pi theta);
  * the lever arm of the angular volume integral is r = x - X_c at each level;
  * the garbled position prediction is read as
      X_c^{n+1} = (4 X_c^n - X_c^{n-1}) / 3 + (2 dt / 3) u_s^n,
    and the points as X_k = X_c^{n+1} + R^{n+1} X~_k^0;
  * the volume fraction of a velocity node is that of the cell-sized box centred
    on it, from the signed distance s = |x - X_c| - a at its 8 corners:
      alpha = sum(-s, s < 0) / sum |s|.
"""
from __future__ import annotations

import math

import numpy as np

from .mac import PERIODIC, Grid


def skew(v):
    return np.array([[0.0, -v[2], v[1]], [v[2], 0.0, -v[0]], [-v[1], v[0], 0.0]])


def rodrigues(axis_unit, gamma):
    """R_Delta = I + sin(gamma) W + (1 - cos(gamma)) W^2 (Sec. 2.2)."""
    W = skew(axis_unit)
    return np.eye(3) + math.sin(gamma) * W + (1.0 - math.cos(gamma)) * (W @ W)


def rotation_step(R, omega_n, omega_nm1, dt):
    """R^{n+1} = R^n R_Delta with the AB2 angle
    gamma = dt (3/2 |w^n| - 1/2 |w^{n-1}|) about the body-frame axis of w^n."""
    wn = np.linalg.norm(omega_n)
    if wn == 0.0:
        return R.copy()
    gamma = dt * (1.5 * wn - 0.5 * np.linalg.norm(omega_nm1))
    axis_body = R.T @ (omega_n / wn)
    return R @ rodrigues(axis_body, gamma)


def prescribed_center(center0, vel, amp, w, t):
    """Constant translation plus the oscillation law x = x_0 - A cos(w t)."""
    return center0 + vel * t - amp * math.cos(w * t)


def prescribed_velocity(vel, amp, w, t):
    return vel + amp * w * math.sin(w * t)


def prescribed_rotation(omega, t):
    """Rotation by a constant angular velocity over time t."""
    wn = np.linalg.norm(omega)
    if wn == 0.0:
        return np.eye(3)
    return rodrigues(omega / wn, wn * t)


def points(center, R, offsets):
    """X_k = X_c + R X~_k."""
    return center[None, :] + offsets @ R.T


def point_velocities(u_s, omega, lever):
    """U_k = u_s + omega x L~_k (eq. kinematic_constraint)."""
    return u_s[None, :] + np.cross(omega[None, :], lever)


# ---------------------------------------------------------------------------
# volume fractions and integrals

def face_positions(g: Grid, d: int):
    """Coordinates of the component-d velocity nodes, (3, n0, n1, n2)."""
    ii = np.indices(g.n).astype(np.float64)
    pos = (ii + 0.5) * g.h
    pos[d] -= 0.5 * g.h
    return pos


def _rel(g: Grid, pos, center, length):
    r = pos - center.reshape(3, 1, 1, 1)
    for a in range(3):
        if g.bc[a] == PERIODIC:
            L = length[a]
            r[a] -= L * np.round(r[a] / L)
    return r


def volume_fraction(g: Grid, d: int, center, radius, length=(1.0, 1.0, 1.0)):
    """alpha at every component-d node for one sphere."""
    pos = face_positions(g, d)
    r = _rel(g, pos, np.asarray(center), length)
    num = np.zeros(g.n)
    den = np.zeros(g.n)
    for sx in (-0.5, 0.5):
        for sy in (-0.5, 0.5):
            for sz in (-0.5, 0.5):
                cx = r[0] + sx * g.h
                cy = r[1] + sy * g.h
                cz = r[2] + sz * g.h
                s = np.sqrt(cx * cx + cy * cy + cz * cz) - radius
                num += np.where(s < 0.0, -s, 0.0)
                den += np.abs(s)
    return np.where(den > 0.0, num / np.where(den > 0, den, 1.0), 0.0)


def volume_fraction_grad(g: Grid, d: int, center, radius, length=(1.0, 1.0, 1.0)):
    """Derivative of volume_fraction with respect to the sphere centre,
    (3, n0, n1, n2): with s_i = |c_i - X_c| - a at the 8 corners c_i,
    d s_i / d X_c = -(c_i - X_c) / |c_i - X_c|, and alpha = num / den with
    num = sum(-s_i, s_i < 0), den = sum |s_i| (piecewise smooth; the branch of
    each s_i is taken at its value)."""
    pos = face_positions(g, d)
    r = _rel(g, pos, np.asarray(center), length)
    num = np.zeros(g.n)
    den = np.zeros(g.n)
    dnum = np.zeros((3,) + g.n)
    dden = np.zeros((3,) + g.n)
    for sx in (-0.5, 0.5):
        for sy in (-0.5, 0.5):
            for sz in (-0.5, 0.5):
                c = np.stack([r[0] + sx * g.h, r[1] + sy * g.h, r[2] + sz * g.h])
                dist = np.sqrt((c * c).sum(axis=0))
                s = dist - radius
                ds = -c / np.where(dist > 0, dist, 1.0)
                inside = s < 0.0
                num += np.where(inside, -s, 0.0)
                den += np.abs(s)
                dnum -= np.where(inside, ds, 0.0)
                dden += np.sign(s) * ds
    ok = den > 0.0
    safe = np.where(ok, den, 1.0)
    return np.where(ok, (dnum * safe - num * dden) / (safe * safe), 0.0)


def volume_integrals(g: Grid, u, center, radius, length=(1.0, 1.0, 1.0)):
    """(sum alpha u h^3, sum alpha r x u h^3) for one sphere (eq. volume_integrals)."""
    h3 = g.h ** 3
    lin = np.zeros(3)
    ang = np.zeros(3)
    for d in range(3):
        a = volume_fraction(g, d, center, radius, length)
        r = _rel(g, face_positions(g, d), np.asarray(center), length)
        au = a * u[d] * h3
        lin[d] = au.sum()
        # u_d enters (r x u) as +r_{d+2} u_d in component d+1 and -r_{d+1} u_d
        # in component d+2
        e1, e2 = (d + 1) % 3, (d + 2) % 3
        ang[e1] += (r[e2] * au).sum()
        ang[e2] -= (r[e1] * au).sum()
    return lin, ang


def newton_euler(theta, radius, dt, us_n, us_nm1, w_n, w_nm1, force_sum, torque_sum,
                 I_k, I_n, I_nm1, J_k, J_n, J_nm1, g):
    """Discrete BDF2 momentum balances of Step 3 (eqs. bdy_linear_vel_iter,
    bdy_angular_vel_iter); force_sum = h^3 sum Phi, torque_sum = h^3 sum L~ x Phi."""
    Vp = 4.0 / 3.0 * math.pi * radius ** 3
    Ip = 0.4 * Vp * radius ** 2
    c = 2.0 * dt / 3.0
    us = (4.0 * us_n - us_nm1) / 3.0 + c / (theta * Vp) * (
        -force_sum + (3.0 * I_k - 4.0 * I_n + I_nm1) / (2.0 * dt)
        + (theta - 1.0) * Vp * np.asarray(g))
    w = (4.0 * w_n - w_nm1) / 3.0 + c / (theta * Ip) * (
        -torque_sum + (3.0 * J_k - 4.0 * J_n + J_nm1) / (2.0 * dt))
    return us, w
