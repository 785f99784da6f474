"""Right-preconditioned restarted GMRES in FP64 (plain, unfused).

The paper solves the Schur system with a Krylov method preconditioned by the
Laplacian (Sec. 4.2: BiCGStab or GMRES, left preconditioning).  The oracle
uses right preconditioning so that the stopping test is on the true residual
||b - A x|| / ||b||; the converged solution is the same up to the tolerance.
Arnoldi uses modified Gram-Schmidt; the small least-squares problem is solved
with Givens rotations.
"""
from __future__ import annotations

import numpy as np


def gmres(matvec, b, precond=None, rtol=1e-13, restart=30, maxit=500, x0=None):
    """Returns (x, iterations, relative true residual history per restart)."""
    M = precond if precond is not None else (lambda v: v)
    x = np.zeros_like(b) if x0 is None else x0.copy()
    bnorm = np.linalg.norm(b)
    if bnorm == 0.0:
        return x, 0, [0.0]
    hist = []
    it = 0
    while it < maxit:
        r = b - matvec(x)
        beta = np.linalg.norm(r)
        hist.append(beta / bnorm)
        if beta / bnorm <= rtol:
            break
        m = min(restart, maxit - it)
        V = np.zeros((m + 1,) + b.shape)
        Z = np.zeros((m,) + b.shape)
        H = np.zeros((m + 1, m))
        cs = np.zeros(m)
        sn = np.zeros(m)
        gvec = np.zeros(m + 1)
        gvec[0] = beta
        V[0] = r / beta
        j_done = 0
        for j in range(m):
            Z[j] = M(V[j])
            w = matvec(Z[j])
            for i in range(j + 1):
                H[i, j] = np.vdot(V[i], w)
                w = w - H[i, j] * V[i]
            H[j + 1, j] = np.linalg.norm(w)
            if H[j + 1, j] > 0:
                V[j + 1] = w / H[j + 1, j]
            for i in range(j):
                t = cs[i] * H[i, j] + sn[i] * H[i + 1, j]
                H[i + 1, j] = -sn[i] * H[i, j] + cs[i] * H[i + 1, j]
                H[i, j] = t
            den = np.hypot(H[j, j], H[j + 1, j])
            cs[j] = H[j, j] / den
            sn[j] = H[j + 1, j] / den
            H[j, j] = den
            H[j + 1, j] = 0.0
            gvec[j + 1] = -sn[j] * gvec[j]
            gvec[j] = cs[j] * gvec[j]
            it += 1
            j_done = j + 1
            if abs(gvec[j + 1]) / bnorm <= rtol * 0.1 or it >= maxit:
                break
        y = np.linalg.solve(np.triu(H[:j_done, :j_done]), gvec[:j_done])
        x = x + np.tensordot(y, Z[:j_done], axes=1)
    r = b - matvec(x)
    hist.append(np.linalg.norm(r) / bnorm)
    return x, it, hist


def bicgstab(matvec, b, precond=None, rtol=1e-13, maxit=500, x0=None):
    """Right-preconditioned BiCGStab (van der Vorst, 1992), the Krylov method
    the paper pairs with the Laplacian preconditioner (Sec. 4.2, Sec. 6.2).
    One iteration applies the preconditioner and the operator twice.  The
    recursive residual is used for the stopping test; the returned history
    ends with the true residual.  Returns (x, iterations, history)."""
    M = precond if precond is not None else (lambda v: v)
    x = np.zeros_like(b) if x0 is None else x0.copy()
    bnorm = np.linalg.norm(b)
    if bnorm == 0.0:
        return x, 0, [0.0]
    r = b - matvec(x)
    rhat = r.copy()
    p = np.zeros_like(b)
    v = np.zeros_like(b)
    rho_old = alpha = omega = 1.0
    hist = [np.linalg.norm(r) / bnorm]
    it = 0
    while hist[-1] > rtol and it < maxit:
        rho = np.vdot(rhat, r)
        beta = (rho / rho_old) * (alpha / omega) if it > 0 else 0.0
        p = r + beta * (p - omega * v)
        phat = M(p)
        v = matvec(phat)
        alpha = rho / np.vdot(rhat, v)
        s = r - alpha * v
        it += 1
        if np.linalg.norm(s) / bnorm <= rtol:
            x = x + alpha * phat
            hist.append(np.linalg.norm(s) / bnorm)
            break
        shat = M(s)
        t = matvec(shat)
        omega = np.vdot(t, s) / np.vdot(t, t)
        x = x + alpha * phat + omega * shat
        r = s - omega * t
        rho_old = rho
        hist.append(np.linalg.norm(r) / bnorm)
    hist.append(np.linalg.norm(b - matvec(x)) / bnorm)
    return x, it, hist
