"""Discrete delta kernels and the regularization / interpolation matrix.

Paper Sec. 2.3: the regularization R spreads Lagrangian forces to the Eulerian
velocity nodes and the interpolation R^T gathers velocities at the Lagrangian
points, both built from the same discrete delta, so that they are exact
transposes (eqs. interpolation, regularization).  Here W is that matrix with
dimensionless entries w_ik = h^3 delta_h(x_i - X_k) = phi(dx/h) phi(dy/h) phi(dz/h).

Kernels (1-D, argument in cell widths):
  * ROMA3: the 3-point kernel printed as eq. delta (support 1.5 cells);
  * PESKIN4: the standard 4-point kernel (support 2 cells); the paper prints
    only the 3-point one, the 4-point formula is Peskin's (Acta Numerica 2002).

Periodic axes wrap with the minimum image; on a wall axis (either kind) the support of a
point must stay inside the domain (Appendix B), otherwise ValueError.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from .mac import PERIODIC, Grid

PESKIN4 = 0
ROMA3 = 1


def phi_roma3(r):
    """eq. delta with Delta r = 1 (multiplied by Delta r: dimensionless)."""
    a = np.abs(np.asarray(r, dtype=np.float64))
    out = np.zeros_like(a)
    inner = a <= 0.5
    outer = (a > 0.5) & (a <= 1.5)
    out[inner] = (1.0 + np.sqrt(1.0 - 3.0 * a[inner] ** 2)) / 3.0
    out[outer] = (5.0 - 3.0 * a[outer] - np.sqrt(np.maximum(0.0, 1.0 - 3.0 * (1.0 - a[outer]) ** 2))) / 6.0
    return out


def phi_peskin4(r):
    a = np.abs(np.asarray(r, dtype=np.float64))
    out = np.zeros_like(a)
    m1 = a <= 1.0
    m2 = (a > 1.0) & (a < 2.0)
    out[m1] = (3.0 - 2.0 * a[m1] + np.sqrt(1.0 + 4.0 * a[m1] - 4.0 * a[m1] ** 2)) / 8.0
    out[m2] = (5.0 - 2.0 * a[m2] - np.sqrt(np.maximum(0.0, -7.0 + 12.0 * a[m2] - 4.0 * a[m2] ** 2))) / 8.0
    return out


def dphi_roma3(r):
    """d phi / d r of the 3-point kernel."""
    r = np.asarray(r, dtype=np.float64)
    a = np.abs(r)
    s = np.sign(r)
    out = np.zeros_like(a)
    inner = a <= 0.5
    outer = (a > 0.5) & (a < 1.5)
    q = np.sqrt(np.maximum(1e-300, 1.0 - 3.0 * a[inner] ** 2))
    out[inner] = (-3.0 * a[inner] / q) / 3.0 * s[inner]
    t = 1.0 - a[outer]
    q2 = np.sqrt(np.maximum(1e-300, 1.0 - 3.0 * t * t))
    # d/da [5 - 3a - sqrt(1 - 3(1-a)^2)]/6 = [-3 - 3(1-a)/sqrt(...)]/6
    out[outer] = (-3.0 - 3.0 * t / q2) / 6.0 * s[outer]
    return out


def dphi_peskin4(r):
    r = np.asarray(r, dtype=np.float64)
    a = np.abs(r)
    s = np.sign(r)
    out = np.zeros_like(a)
    m1 = a <= 1.0
    m2 = (a > 1.0) & (a < 2.0)
    q1 = np.sqrt(1.0 + 4.0 * a[m1] - 4.0 * a[m1] ** 2)
    out[m1] = (-2.0 + (2.0 - 4.0 * a[m1]) / q1) / 8.0 * s[m1]
    q2 = np.sqrt(np.maximum(1e-300, -7.0 + 12.0 * a[m2] - 4.0 * a[m2] ** 2))
    out[m2] = (-2.0 - (6.0 - 4.0 * a[m2]) / q2) / 8.0 * s[m2]
    return out


PHI = {PESKIN4: phi_peskin4, ROMA3: phi_roma3}
DPHI = {PESKIN4: dphi_peskin4, ROMA3: dphi_roma3}
WIDTH = {PESKIN4: 4, ROMA3: 3}


def _stencil(g: Grid, X: np.ndarray, d: int, kernel: int):
    """For component d, the node indices (K, 3, w) and offsets r (K, 3, w) in
    cell units of every point's support."""
    w = WIDTH[kernel]
    K = X.shape[0]
    idx = np.empty((K, 3, w), dtype=np.int64)
    r = np.empty((K, 3, w))
    for a in range(3):
        o = 0.0 if a == d else 0.5          # face nodes along d, centres otherwise
        s = X[:, a] / g.h - o
        if w == 4:
            i0 = np.floor(s).astype(np.int64) - 1
        else:
            i0 = np.floor(s + 0.5).astype(np.int64) - 1
        for t in range(w):
            idx[:, a, t] = i0 + t
            r[:, a, t] = s - (i0 + t)
    return idx, r


def check_support(g: Grid, X: np.ndarray, kernel: int):
    """Appendix B: near a wall (either kind) the whole support must lie on
    interior nodes; raise ValueError otherwise."""
    for d in range(3):
        idx, _ = _stencil(g, X, d, kernel)
        for a in range(3):
            if g.bc[a] == PERIODIC:
                continue
            lo = 1 if a == d else 0
            hi = g.n[a] - 1
            if (idx[:, a, :] < lo).any() or (idx[:, a, :] > hi).any():
                raise ValueError("delta support of a Lagrangian point crosses a wall")


def regularization_matrix(g: Grid, X: np.ndarray, kernel: int = PESKIN4,
                          deriv_axis: int | None = None) -> sp.csr_matrix:
    """W of shape (3N, 3K): row d*N + cell, column 3k + d, w_ik as above.

    With deriv_axis = a, returns dW/dX_{k,a} with the same sparsity (the
    derivative of each weight with respect to its own point's coordinate a)."""
    check_support(g, X, kernel)
    K = X.shape[0]
    phi, dphi = PHI[kernel], DPHI[kernel]
    w = WIDTH[kernel]
    rows, cols, vals = [], [], []
    for d in range(3):
        idx, r = _stencil(g, X, d, kernel)
        f = [phi(r[:, a, :]) for a in range(3)]
        if deriv_axis is not None:
            # r = X/h - node, so d/dX = (1/h) d/dr
            f[deriv_axis] = dphi(r[:, deriv_axis, :]) / g.h
        wk = f[0][:, :, None, None] * f[1][:, None, :, None] * f[2][:, None, None, :]
        ii = [np.mod(idx[:, a, :], g.n[a]) for a in range(3)]
        cell = (ii[0][:, :, None, None] * g.n[1] + ii[1][:, None, :, None]) * g.n[2] \
            + ii[2][:, None, None, :]
        rows.append((d * g.N + cell).ravel())
        cols.append(np.repeat(3 * np.arange(K) + d, w ** 3))
        vals.append(wk.ravel())
    return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                         shape=(3 * g.N, 3 * K))


def interpolate(W: sp.csr_matrix, u: np.ndarray) -> np.ndarray:
    """W^T u: (3, n0, n1, n2) -> (K, 3) (eq. interpolation)."""
    return (W.T @ u.ravel()).reshape(-1, 3)


def spread(W: sp.csr_matrix, f: np.ndarray, n) -> np.ndarray:
    """W f: (K, 3) -> (3, n0, n1, n2) (eq. regularization)."""
    return (W @ f.ravel()).reshape((3,) + tuple(n))
