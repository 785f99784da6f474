"""Staggered (MAC) grid operators, FP64, as explicit sparse matrices.

Paper: Sec. 2.1 (the discretization cell figure: velocities on faces, pressure
at centres) and Sec. 3.1 (central finite-volume differences in space, BDF2 in
time).  The paper does not print the stencils;
the reading taken here is the classical MAC scheme:

  * (G p) on the face of component d at index (i,j,k) = (p[idx] - p[idx-e_d]) / h;
    on a wall axis d the index-0 face is the wall, its row of G is zero;
  * D = -G^T exactly (the symmetry the spectral theorem of Sec. 5 needs);
  * L = G^T G, the positive semi-definite Neumann/periodic Laplacian "-nabla^2"
    of eq. modified_poisson (no Dirichlet point: its null space is the constants);
  * the viscous Laplacian on each velocity component is the 7-point stencil on
    that component's face grid; a normal wall neighbour is the wall face, 0;
    a tangential wall neighbour is a ghost half a cell beyond the wall: -u on
    a no-slip wall (zero tangential velocity at the wall), +u on a free-slip
    wall (zero normal derivative of the tangential velocity, the box
    condition of the sedimentation runs of Sec. 6.1.3);
  * both wall kinds carry zero normal velocity, so G, D, L and the
    convective fluxes through the wall are the same for both;
  * the convection term (u . grad u) of eq. ustar is taken in divergence form
    div(u u) with arithmetic averaging to the control-volume faces.

Layout: natural (n0, n1, n2) C order; a face field is (3, n0, n1, n2).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

PERIODIC = 0
NOSLIP = 1
FREESLIP = 2


def is_wall(b: int) -> bool:
    """Either wall kind: the box ends on this axis, normal velocity zero."""
    return b != PERIODIC


class Grid:
    def __init__(self, n, h, bc):
        self.n = tuple(int(x) for x in n)
        self.h = float(h)
        self.bc = tuple(int(b) for b in bc)
        self.N = self.n[0] * self.n[1] * self.n[2]

    def idx(self):
        return np.indices(self.n)

    def lin(self, i, j, k):
        return (i * self.n[1] + j) * self.n[2] + k

    def face_dof_mask(self):
        """(3, n0, n1, n2) bool: False on wall faces (index 0 of a wall axis d
        for component d), which are not unknowns and always hold zero."""
        m = np.ones((3,) + self.n, dtype=bool)
        for d in range(3):
            if is_wall(self.bc[d]):
                sl = [d, slice(None), slice(None), slice(None)]
                sl[1 + d] = 0
                m[tuple(sl)] = False
        return m


def _shift(ii, a, s, n, bc):
    """Index array shifted by s along axis a; returns (shifted, valid mask)."""
    out = [x.copy() for x in ii]
    out[a] = ii[a] + s
    if bc[a] == PERIODIC:
        out[a] %= n[a]
        valid = np.ones(ii[0].shape, dtype=bool)
    else:
        valid = (out[a] >= 0) & (out[a] < n[a])
        out[a] = np.clip(out[a], 0, n[a] - 1)
    return out, valid


def gradient(g: Grid) -> sp.csr_matrix:
    """G: cells -> faces, shape (3N, N)."""
    ii = [x.ravel() for x in g.idx()]
    rows, cols, vals = [], [], []
    for d in range(3):
        lo, valid = _shift(ii, d, -1, g.n, g.bc)
        if is_wall(g.bc[d]):
            valid = valid & (ii[d] > 0)
        r = d * g.N + g.lin(*ii)
        rows += [r[valid], r[valid]]
        cols += [g.lin(*ii)[valid], g.lin(*lo)[valid]]
        vals += [np.full(valid.sum(), 1.0 / g.h), np.full(valid.sum(), -1.0 / g.h)]
    return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                         shape=(3 * g.N, g.N))


def divergence(g: Grid) -> sp.csr_matrix:
    """D = -G^T: faces -> cells, (Du)[c] = sum_d (u_d[c+e_d] - u_d[c]) / h."""
    return (-gradient(g).T).tocsr()


def laplacian(g: Grid) -> sp.csr_matrix:
    """L = G^T G (positive semi-definite, constant null space)."""
    G = gradient(g)
    return (G.T @ G).tocsr()


def viscous_laplacian(g: Grid) -> sp.csr_matrix:
    """Delta_h on the three face grids, block diagonal (3N, 3N); rows and
    columns of wall faces are empty."""
    ii = [x.ravel() for x in g.idx()]
    lin = g.lin(*ii)
    mask = g.face_dof_mask().reshape(3, -1)
    rows, cols, vals = [], [], []
    h2 = 1.0 / (g.h * g.h)
    for d in range(3):
        dof = mask[d]
        base = d * g.N
        diag = np.zeros(g.N)
        for a in range(3):
            for s in (-1, 1):
                nb, valid = _shift(ii, a, s, g.n, g.bc)
                if g.bc[a] == PERIODIC:
                    ok = valid
                    diag -= h2
                elif a == d:
                    # normal direction: neighbours are faces; faces 0 and n are walls (0)
                    nbi = ii[a] + s
                    ok = (nbi >= 1) & (nbi <= g.n[a] - 1)
                    diag -= h2
                else:
                    # tangential: outside the box the ghost value is -u on a
                    # no-slip wall (adds -1/h^2 to the diagonal) and +u on a
                    # free-slip wall (cancels the -1/h^2 of the centre)
                    ok = valid
                    diag -= h2
                    if g.bc[a] == FREESLIP:
                        diag[~valid] += h2
                    else:
                        diag[~valid] -= h2
                ok = ok & dof & mask[d][g.lin(*nb)]
                rows.append(base + lin[ok])
                cols.append(base + g.lin(*nb)[ok])
                vals.append(np.full(ok.sum(), h2))
        rows.append(base + lin[dof])
        cols.append(base + lin[dof])
        vals.append(diag[dof])
    return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                         shape=(3 * g.N, 3 * g.N))


def helmholtz(g: Grid, nu: float, dt: float) -> sp.csr_matrix:
    """Momentum operator of eq. ustar for BDF2: A = (3/(2 dt)) I - nu Delta_h,
    on the unknown faces (identity rows on wall faces keep them at zero)."""
    m = g.face_dof_mask().ravel().astype(np.float64)
    I = sp.diags(1.5 / dt * m + (1.0 - m))
    return (I - nu * viscous_laplacian(g)).tocsr()


def convection(g: Grid, u: np.ndarray) -> np.ndarray:
    """N(u) = div(u u) at the faces, central, arithmetic averages (reading of
    Sec. 3.1: explicit at t^n).  u: (3, n0, n1, n2).  Fluxes through walls
    of either kind vanish (normal velocity zero there)."""
    n, h, bc = g.n, g.h, g.bc
    out = np.zeros_like(u)
    mask = g.face_dof_mask()
    uu = u * mask

    def sh(f, a, s):
        """f(idx + s e_a), zero outside a wall box."""
        r = np.roll(f, -s, axis=a)
        if is_wall(bc[a]):
            sl = [slice(None)] * 3
            if s > 0:
                sl[a] = slice(n[a] - s, n[a])
            else:
                sl[a] = slice(0, -s)
            r[tuple(sl)] = 0.0
        return r

    idx = np.indices(n)
    for d in range(3):
        ud = uu[d]
        acc = np.zeros(n)
        for a in range(3):
            if a == d:
                # flux at cell centres: (mean of u_d over the cell)^2
                cp = 0.5 * (ud + sh(ud, d, 1))     # centre of cell idx
                cm = 0.5 * (sh(ud, d, -1) + ud)    # centre of cell idx - e_d
                acc += (cp * cp - cm * cm) / h
            else:
                ua = uu[a]
                # edge at face(idx) + h/2 e_a
                ud_e = 0.5 * (ud + sh(ud, a, 1))
                ua_e = 0.5 * (sh(ua, a, 1) + sh(sh(ua, a, 1), d, -1))
                fp = ud_e * ua_e
                if is_wall(bc[a]):
                    fp = np.where(idx[a] == n[a] - 1, 0.0, fp)
                fm = sh(fp, a, -1)
                if is_wall(bc[a]):
                    fm = np.where(idx[a] == 0, 0.0, fm)
                acc += (fp - fm) / h
        out[d] = acc
    return out * mask


# ----------------------------------------------------------------------------
# An independent stencil (np.roll) formulation of G, D, L, used only to check
# the sparse matrices above against a second derivation.

def grad_stencil(g: Grid, p: np.ndarray) -> np.ndarray:
    out = np.empty((3,) + g.n)
    for d in range(3):
        gd = (p - np.roll(p, 1, axis=d)) / g.h
        if is_wall(g.bc[d]):
            sl = [slice(None)] * 3
            sl[d] = 0
            gd[tuple(sl)] = 0.0
        out[d] = gd
    return out


def div_stencil(g: Grid, u: np.ndarray) -> np.ndarray:
    out = np.zeros(g.n)
    for d in range(3):
        ud = u[d].copy()
        if is_wall(g.bc[d]):
            sl = [slice(None)] * 3
            sl[d] = 0
            ud[tuple(sl)] = 0.0
        up = np.roll(ud, -1, axis=d)
        if is_wall(g.bc[d]):
            sl = [slice(None)] * 3
            sl[d] = g.n[d] - 1
            up[tuple(sl)] = 0.0
        out += (up - ud) / g.h
    return out


def lap_stencil(g: Grid, p: np.ndarray) -> np.ndarray:
    return -div_stencil(g, grad_stencil(g, p))
