"""Reverse-mode derivative (vector-Jacobian product) of the one-way time step.

The step of Sec. 3.1 (one correction, prescribed bodies) maps
(u^n, u^{n-1}, p^n, Phi^n, X, U) to (u^{n+1}, p^{n+1}, Phi^{n+1}) through

    rhs  = M[(4 u^n - u^{n-1}) / (2 dt) - G p^n + W Phi^n - N(u^n)]   (eq. ustar)
    u*   = A^-1 rhs
    RHS_p = -D u* / tau,   RHS_F = (W^T u* - U) / tau
    b    = P(RHS_p + c^-1 D W RHS_F)                    (eq. ApproxSchurPrimalP)
    p'   = S~^+ b,  S~ = L + c^-1 G^T W W^T G           (eq. tildeSp)
    Phi' = c^-1 (-W^T G p' - RHS_F)                     (eq. ApproxSchurPrimalF)
    u^{n+1} = M[u* + xi tau (-G p' + W Phi')],  p^{n+1} = p^n + xi p',
    Phi^{n+1} = Phi^n + xi Phi'                         (eq. u_n_plus_1)

with W = W(X) the regularization matrix, M the mask of the unknown faces, P
the projection to mean zero, tau = 2 dt / 3.  Every step is transposed in the
reverse order below; A and S~ are symmetric, so their transposed solves are
solves with the same operators.  The derivative of W with respect to the point
coordinates comes from delta.regularization_matrix(..., deriv_axis=e).  N is
quadratic, and its Jacobian is assembled from the same flux definition as
mac.convection.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from . import delta, mac
from . import step as ostep
from .mac import is_wall


def _shift(g: mac.Grid, a: int, s: int) -> sp.csr_matrix:
    """(S f)(x) = f(x + s e_a); zero outside a wall box, wrapped otherwise."""
    ii = [x.ravel() for x in g.idx()]
    jj = [x.copy() for x in ii]
    jj[a] = ii[a] + s
    if is_wall(g.bc[a]):
        ok = (jj[a] >= 0) & (jj[a] < g.n[a])
    else:
        jj[a] %= g.n[a]
        ok = np.ones(g.N, dtype=bool)
    rows = g.lin(*ii)[ok]
    cols = g.lin(*[np.where(ok, x, 0) for x in jj])[ok]
    return sp.csr_matrix((np.ones(ok.sum()), (rows, cols)), shape=(g.N, g.N))


def convection_jacobian(g: mac.Grid, u: np.ndarray) -> sp.csr_matrix:
    """dN/du at u (3N x 3N) for the flux form of mac.convection:
    N_d = sum_a (F_ad(x) - F_ad(x - e_a)) / h with F_dd = C^2, C the cell mean
    of u_d, and F_ad = E1 E2 (a != d), E1 = mean of u_d across the edge,
    E2 = mean of u_a along d at the edge; fluxes through walls are 0."""
    N, h = g.N, g.h
    mask = g.face_dof_mask().reshape(3, N).astype(np.float64)
    uu = (u.reshape(3, N) * mask)
    idx = [x.ravel() for x in g.idx()]
    I = sp.identity(N, format="csr")
    blocks = [[sp.csr_matrix((N, N)) for _ in range(3)] for _ in range(3)]
    for d in range(3):
        for a in range(3):
            Sp, Sm = _shift(g, a, 1), _shift(g, a, -1)
            if a == d:
                Cop = 0.5 * (I + Sp)                       # C(x) = (u_d(x) + u_d(x+e_d)) / 2
                C = Cop @ uu[d]
                dF = sp.diags(2.0 * C) @ Cop               # d(C^2) / du_d
                blocks[d][d] = blocks[d][d] + (dF - Sm @ dF) / h
            else:
                Sd_m = _shift(g, d, -1)
                E1op = 0.5 * (I + Sp)                      # acts on u_d
                E2op = 0.5 * (Sp + Sd_m @ Sp)              # acts on u_a
                E1, E2 = E1op @ uu[d], E2op @ uu[a]
                zp = np.ones(N)
                zm = np.ones(N)
                if is_wall(g.bc[a]):
                    zp[idx[a] == g.n[a] - 1] = 0.0
                    zm[idx[a] == 0] = 0.0
                Zp, Zm = sp.diags(zp), sp.diags(zm)
                dF_dd = Zp @ sp.diags(E2) @ E1op
                dF_da = Zp @ sp.diags(E1) @ E2op
                blocks[d][d] = blocks[d][d] + (dF_dd - Zm @ Sm @ dF_dd) / h
                blocks[d][a] = blocks[d][a] + (dF_da - Zm @ Sm @ dF_da) / h
    J = sp.bmat(blocks, format="csr")
    Mk = sp.diags(mask.ravel())
    return (Mk @ J @ Mk).tocsr()


def _dx(dW, a_faces, b_points):
    """Gradient with respect to the point coordinates of a^T W(X) b, (K, 3)."""
    K = b_points.shape[0]
    out = np.empty((K, 3))
    for e in range(3):
        out[:, e] = ((dW[e].T @ a_faces.ravel()).reshape(K, 3) * b_points).sum(axis=1)
    return out


def one_way_step_vjp(g: mac.Grid, nu, dt, state: ostep.State, X, U, kernel, c, xi,
                     gu, gp, gphi, helm_rtol=1e-14, schur_rtol=1e-13):
    """Cotangents of (u^{n+1}, p^{n+1}, Phi^{n+1}) -> cotangents of the inputs.

    Returns dict(u=..., um=..., p=..., phi=..., X=(K,3), U=(K,3)) and the
    forward result."""
    new, info = ostep.one_way_step(g, nu, dt, state, X, U, kernel, c, xi, helm_rtol, schur_rtol)
    W, sysm = info["W"], info["sys"]
    ustar, pp, phip, rhs_f = info["ustar"], info["pprime"], info["phiprime"], info["rhs_f"]
    K = X.shape[0]
    tau = 2.0 * dt / 3.0
    mask = g.face_dof_mask().ravel().astype(np.float64)
    G, D = mac.gradient(g), mac.divergence(g)
    dW = [delta.regularization_matrix(g, X, kernel, deriv_axis=e) for e in range(3)]

    gu = np.zeros(3 * g.N) if gu is None else np.asarray(gu, dtype=np.float64).ravel()
    gp = np.zeros(g.N) if gp is None else np.asarray(gp, dtype=np.float64).ravel()
    gphi = np.zeros((K, 3)) if gphi is None else np.asarray(gphi, dtype=np.float64).reshape(K, 3)

    # update: u+ = M[u* + xi tau (-G p' + W Phi')], p+ = p + xi p', Phi+ = Phi + xi Phi'
    ub = gu * mask
    p_n_bar = gp.copy()
    phi_n_bar = gphi.copy()
    ppb = xi * gp - xi * tau * (G.T @ ub)
    phipb = xi * gphi + xi * tau * (W.T @ ub).reshape(K, 3)
    gX = xi * tau * _dx(dW, ub, phip)
    ustarb = ub.copy()
    # force recovery: Phi' = c^-1 (-W^T G p' - RHS_F)
    Gpp = G @ pp.ravel()
    ppb = ppb - (G.T @ (W @ phipb.ravel())) / c
    rhsfb = -phipb / c
    gX -= _dx(dW, Gpp, phipb) / c
    # Schur solve p' = S~^+ b: bbar = S~^+ P pbar'; dS~ = c^-1 G^T (dW W^T + W dW^T) G
    bbar, _, _, _ = sysm.solve(ppb.reshape(g.n), np.zeros((K, 3)), rtol=schur_rtol)
    bbar = bbar.ravel()
    Gbb = G @ bbar
    gX -= (_dx(dW, Gbb, (W.T @ Gpp).reshape(K, 3)) + _dx(dW, Gpp, (W.T @ Gbb).reshape(K, 3))) / c
    # right-hand side b = P(RHS_p + c^-1 D W RHS_F)
    rhspb = bbar - bbar.mean()
    DTb = D.T @ rhspb
    rhsfb = rhsfb + (W.T @ DTb).reshape(K, 3) / c
    gX += _dx(dW, DTb, rhs_f) / c
    # RHS_p = -D u* / tau, RHS_F = (W^T u* - U) / tau
    ustarb = ustarb - (D.T @ rhspb) / tau + (W @ rhsfb.ravel()) / tau
    Ubar = -rhsfb / tau
    gX += _dx(dW, ustar.ravel(), rhsfb) / tau
    # u* = A^-1 rhs on the unknown faces (A symmetric)
    rhsb, _ = ostep.helmholtz_solve(g, nu, dt, (ustarb * mask).reshape((3,) + g.n), helm_rtol)
    rhsb = rhsb.ravel() * mask
    # rhs = M[(4 u^n - u^{n-1})/(2 dt) - G p^n + W Phi^n - N(u^n)]
    Jn = convection_jacobian(g, state.u)
    u_n_bar = (2.0 / dt * rhsb - Jn.T @ rhsb) * mask
    um_bar = -rhsb / (2.0 * dt) * mask
    p_n_bar = p_n_bar - G.T @ rhsb
    phi_n_bar = phi_n_bar + (W.T @ rhsb).reshape(K, 3)
    gX += _dx(dW, rhsb, state.phi)
    grads = dict(u=u_n_bar.reshape((3,) + g.n), um=um_bar.reshape((3,) + g.n),
                 p=p_n_bar.reshape(g.n), phi=phi_n_bar, X=gX, U=Ubar)
    return grads, new, info
