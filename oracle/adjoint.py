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


# ---------------------------------------------------------------------------
# two-way step (Sec. 3.2.1) with a fixed number of outer passes

def _vol_vjp(g: mac.Grid, u, center, radius, Ibar, Jbar, length):
    """Transpose of bodies.volume_integrals at (u, center): the cotangents
    (Ibar, Jbar) of (sum alpha u h^3, sum alpha r x u h^3) give the face-field
    cotangent alpha h^3 (Ibar + Jbar x r) and the centre cotangent, through
    alpha (volume_fraction_grad) and through r = x - X_c."""
    from . import bodies as bd
    h3 = g.h ** 3
    ubar = np.zeros((3,) + g.n)
    cbar = np.zeros(3)
    for d in range(3):
        a = bd.volume_fraction(g, d, center, radius, length)
        da = bd.volume_fraction_grad(g, d, center, radius, length)
        r = bd._rel(g, bd.face_positions(g, d), np.asarray(center), length)
        e1, e2 = (d + 1) % 3, (d + 2) % 3
        wgt = h3 * (Ibar[d] + Jbar[e1] * r[e2] - Jbar[e2] * r[e1])
        ubar[d] = a * wgt
        cbar += (da * (u[d] * wgt)).reshape(3, -1).sum(axis=1)
        cbar += np.cross(Jbar, np.eye(3)[d]) * h3 * (a * u[d]).sum()
    return ubar, cbar


def _left_jacobian(psi):
    """Left Jacobian of the rotation exponential: exp([psi + dpsi]) =
    exp([J_l(psi) dpsi]) exp([psi]) to first order."""
    from . import bodies as bd
    th = np.linalg.norm(psi)
    S = bd.skew(psi)
    if th < 1e-8:
        return np.eye(3) + 0.5 * S
    return np.eye(3) + (1.0 - np.cos(th)) / th ** 2 * S + (th - np.sin(th)) / th ** 3 * (S @ S)


def two_way_step_vjp(g: mac.Grid, nu, dt, gvec, state: ostep.State, bodies, kernel, c, xi, n_outer,
                     gu=None, gp=None, gphi=None, gbodies=None, helm_rtol=1e-14, schur_rtol=1e-13):
    """Reverse mode of ostep.two_way_step with n_outer passes (no early stop).

    Cotangents of the outputs: gu, gp, gphi for (u^{n+1}, p^{n+1}, Phi^{n+1});
    gbodies[i] a dict with any of xc, us, w, I, J for the body's X_c^{n+1},
    u_s^{n+1}, omega^{n+1} and the volume integrals of u^{n+1} at X_c^{n+1}.
    The orientation R^n is held fixed (its cotangent is not formed).

    Returns (grads, new_state, new_bodies, info): grads has the fluid
    cotangents u, um, p, phi and, per body, xc, xc_m, us, us_m, w, w_m, I_n,
    I_m, J_n, J_m.

    Reverse order: the outer passes k = n_outer-1 .. 0, each the transposed
    correction (as in one_way_step_vjp, with u* replaced by u^k and U by
    U^k), then the kinematic constraint U^k = u_s^k + omega^k x L~, then
    Newton-Euler (linear in the force, torque and volume integrals), the
    force / torque sums and the volume integrals of u^k; then the predictor;
    then the points X = X_c^{n+1} + R^{n+1} X~ and Step 1 (the BDF2 centre
    prediction and R^{n+1} = exp([psi]) R^n, psi = gamma omega^n/|omega^n|)."""
    from . import bodies as bd
    new, nbod, info = ostep.two_way_step(g, nu, dt, gvec, state, bodies, kernel, c, xi, n_outer, 0.0,
                                         schur_rtol, helm_rtol)
    rec, W, sysm, X = info["rec"], info["W"], info["sys"], info["X"]
    xc1, levers, starts, R1 = info["xc1"], info["levers"], info["starts"], info["R1"]
    nb = len(bodies)
    K = X.shape[0]
    tau = 2.0 * dt / 3.0
    h3 = g.h ** 3
    length = ostep.domain_length(g)
    mask = g.face_dof_mask().ravel().astype(np.float64)
    G, D = mac.gradient(g), mac.divergence(g)
    dW = [delta.regularization_matrix(g, X, kernel, deriv_axis=e) for e in range(3)]
    gb = [dict() for _ in range(nb)] if gbodies is None else gbodies

    def z3(v):
        return np.zeros(3) if v is None else np.asarray(v, dtype=np.float64)

    ub = np.zeros(3 * g.N) if gu is None else np.asarray(gu, dtype=np.float64).ravel() * mask
    pb = np.zeros(g.N) if gp is None else np.asarray(gp, dtype=np.float64).ravel().copy()
    phib = np.zeros((K, 3)) if gphi is None else np.asarray(gphi, dtype=np.float64).reshape(K, 3).copy()
    gX = np.zeros((K, 3))
    Lb = np.zeros((K, 3))                       # cotangent of the levers L~ = R^{n+1} X~
    out_b = [dict(xc=np.zeros(3), xc_m=np.zeros(3), us=np.zeros(3), us_m=np.zeros(3), w=np.zeros(3),
                  w_m=np.zeros(3), I_n=np.zeros(3), I_m=np.zeros(3), J_n=np.zeros(3), J_m=np.zeros(3))
             for _ in range(nb)]
    xc1b = [z3(gb[i].get("xc")).copy() for i in range(nb)]
    # volume integrals of u^{n+1} at X_c^{n+1}
    for i, b in enumerate(bodies):
        if gb[i].get("I") is not None or gb[i].get("J") is not None:
            u_b, c_b = _vol_vjp(g, new.u, xc1[i], b.radius, z3(gb[i].get("I")), z3(gb[i].get("J")), length)
            ub += u_b.ravel() * mask
            xc1b[i] += c_b
    usb = [z3(gb[i].get("us")).copy() for i in range(nb)]
    wb = [z3(gb[i].get("w")).copy() for i in range(nb)]

    for k in reversed(range(n_outer)):
        uk, pp, phip, rhs_f = rec["u"][k], rec["pp"][k], rec["phip"][k], rec["rhs_f"][k]
        # update u^{k+1} = M[u^k + xi tau (-G p' + W Phi')], p += xi p', Phi += xi Phi'
        ppb = xi * pb - xi * tau * (G.T @ ub)
        phipb = xi * phib + xi * tau * (W.T @ ub).reshape(K, 3)
        gX += xi * tau * _dx(dW, ub, phip)
        ukb = ub.copy()
        # force recovery Phi' = c^-1 (-W^T G p' - RHS_F)
        Gpp = G @ pp.ravel()
        ppb = ppb - (G.T @ (W @ phipb.ravel())) / c
        rhsfb = -phipb / c
        gX -= _dx(dW, Gpp, phipb) / c
        # Schur solve and the dependence of S~ on the points
        bbar, _, _, _ = sysm.solve(ppb.reshape(g.n), np.zeros((K, 3)), rtol=schur_rtol)
        bbar = bbar.ravel()
        Gbb = G @ bbar
        gX -= (_dx(dW, Gbb, (W.T @ Gpp).reshape(K, 3)) + _dx(dW, Gpp, (W.T @ Gbb).reshape(K, 3))) / c
        # b = P(RHS_p + c^-1 D W RHS_F)
        rhspb = bbar - bbar.mean()
        DTb = D.T @ rhspb
        rhsfb = rhsfb + (W.T @ DTb).reshape(K, 3) / c
        gX += _dx(dW, DTb, rhs_f) / c
        # RHS_p = -D u^k / tau, RHS_F = (W^T u^k - U^k) / tau
        ukb = ukb - (D.T @ rhspb) / tau + (W @ rhsfb.ravel()) / tau
        Ub = -rhsfb / tau
        gX += _dx(dW, uk.ravel(), rhsfb) / tau
        ub = ukb * mask
        # U^k = u_s^k + omega^k x L~ (per body), then Newton-Euler and the sums
        for i, b in enumerate(bodies):
            s0, s1 = starts[i], starts[i + 1]
            lev = levers[i]
            wk = rec["w"][k][i]
            usb_k = usb[i] + Ub[s0:s1].sum(axis=0)
            wb_k = wb[i] + np.cross(lev, Ub[s0:s1]).sum(axis=0)
            Lb[s0:s1] += np.cross(Ub[s0:s1], wk[None, :])
            usb[i] = np.zeros(3)
            wb[i] = np.zeros(3)
            Vp = 4.0 / 3.0 * np.pi * b.radius ** 3
            Ip = 0.4 * Vp * b.radius ** 2
            cu, cw = tau / (b.theta * Vp), tau / (b.theta * Ip)
            ob = out_b[i]
            ob["us"] += 4.0 / 3.0 * usb_k
            ob["us_m"] -= usb_k / 3.0
            ob["w"] += 4.0 / 3.0 * wb_k
            ob["w_m"] -= wb_k / 3.0
            Fb, Tb = -cu * usb_k, -cw * wb_k
            Ikb, Jkb = cu * 1.5 / dt * usb_k, cw * 1.5 / dt * wb_k
            ob["I_n"] -= cu * 2.0 / dt * usb_k
            ob["I_m"] += cu * 0.5 / dt * usb_k
            ob["J_n"] -= cw * 2.0 / dt * wb_k
            ob["J_m"] += cw * 0.5 / dt * wb_k
            # F = h^3 sum Phi^(k), T = h^3 sum L~ x Phi^(k)
            phik = rec["phi"][k][s0:s1]
            phib[s0:s1] += h3 * Fb[None, :] + h3 * np.cross(Tb[None, :], lev)
            Lb[s0:s1] += h3 * np.cross(phik, Tb[None, :])
            # volume integrals of u^k at X_c^{n+1}
            u_b, c_b = _vol_vjp(g, uk, xc1[i], b.radius, Ikb, Jkb, length)
            ub += u_b.ravel() * mask
            xc1b[i] += c_b

    # predictor: u^0 = A^-1 M[(4u^n - u^{n-1})/(2dt) - G p^n + W Phi^n - N(u^n)]
    rhsb, _ = ostep.helmholtz_solve(g, nu, dt, ub.reshape((3,) + g.n), helm_rtol)
    rhsb = rhsb.ravel() * mask
    Jn = convection_jacobian(g, state.u)
    u_n_bar = (2.0 / dt * rhsb - Jn.T @ rhsb) * mask
    um_bar = -rhsb / (2.0 * dt) * mask
    p_n_bar = pb - G.T @ rhsb
    phi_n_bar = phib + (W.T @ rhsb).reshape(K, 3)
    gX += _dx(dW, rhsb, state.phi)
    # points X = X_c^{n+1} + L~, L~ = R^{n+1} X~; Step 1
    for i, b in enumerate(bodies):
        s0, s1 = starts[i], starts[i + 1]
        xc1b[i] += gX[s0:s1].sum(axis=0)
        Lb[s0:s1] += gX[s0:s1]
        phibar = np.cross(levers[i], Lb[s0:s1]).sum(axis=0)
        ob = out_b[i]
        wn = np.linalg.norm(b.w)
        if wn > 0.0:
            what = b.w / wn
            gam = dt * (1.5 * wn - 0.5 * np.linalg.norm(b.w_m))
            psib = _left_jacobian(gam * what).T @ phibar
            dpsi_dw = 1.5 * dt * np.outer(what, what) + gam * (np.eye(3) - np.outer(what, what)) / wn
            ob["w"] += dpsi_dw.T @ psib
            wmn = np.linalg.norm(b.w_m)
            if wmn > 0.0:
                ob["w_m"] += (-0.5 * dt * np.outer(what, b.w_m / wmn)).T @ psib
        ob["xc"] += 4.0 / 3.0 * xc1b[i]
        ob["xc_m"] -= xc1b[i] / 3.0
        ob["us"] += tau * xc1b[i]
    grads = dict(u=u_n_bar.reshape((3,) + g.n), um=um_bar.reshape((3,) + g.n), p=p_n_bar.reshape(g.n),
                 phi=phi_n_bar, bodies=out_b)
    return grads, new, nbod, info
