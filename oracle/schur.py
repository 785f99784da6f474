"""The pressure / force-density correction system and its lumped Schur solve.

Paper Sec. 3.1 (eq. Saddle), Sec. 4.1 (eqs. SchurPrimal, tildeSp,
ApproxSchurPrimalP, ApproxSchurPrimalF, the Laplacian as preconditioner),
Sec. 4.2 (its direct solve).

Reading of the signs (the printed saddle matrix is not consistent with the
printed update and eq. modified_poisson): B^T is taken as the divergence of
the spread force, B^T = D W, so B = (D W)^T = -W^T G.  Then

    S~ = L + c^-1 B^T B = G^T (I + c^-1 W W^T) G          (SPD on mean-zero p)
    b  = RHS_p + c^-1 B^T RHS_F = RHS_p + c^-1 D W RHS_F
    Phi' = c^-1 (B p' - RHS_F) = c^-1 (-W^T G p' - RHS_F)

where c is the scalar of the lumping C = W^T W ~ c I (the paper's 1/2 for its
3-point kernel at spacing h).  With this choice the first block row,
L p' + B^T Phi' = RHS_p, holds to solver tolerance, which makes the projected
velocity discretely divergence-free.  S~ only involves B^T B, so the Krylov
problem is the same under either sign reading.

The Laplacian and S~ are singular on the constants (pressure is defined up to
a constant); b is projected to mean zero and the mean-zero p' is returned.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import krylov, mac, poisson


class SchurSystem:
    def __init__(self, g: mac.Grid, W: sp.csr_matrix, c: float):
        self.g = g
        self.W = W
        self.c = float(c)
        self.G = mac.gradient(g)
        self.D = (-self.G.T).tocsr()
        self.L = (self.G.T @ self.G).tocsr()

    # operators -------------------------------------------------------------
    def B(self, p):
        """B p = -W^T G p, (K, 3)."""
        return -(self.W.T @ (self.G @ p.ravel())).reshape(-1, 3)

    def BT(self, q):
        """B^T q = D W q, shape g.n."""
        return (self.D @ (self.W @ q.ravel())).reshape(self.g.n)

    def matvec(self, p):
        """S~ p = L p + c^-1 B^T B p."""
        return (self.L @ p.ravel()).reshape(self.g.n) + self.BT(self.B(p)) / self.c

    def rhs(self, rhs_p, rhs_f):
        """b = RHS_p + c^-1 B^T RHS_F (eq. ApproxSchurPrimalP), projected to mean 0."""
        b = rhs_p + self.BT(rhs_f) / self.c
        return b - b.mean()

    def force(self, p, rhs_f):
        """Phi' = c^-1 (B p' - RHS_F) (eq. ApproxSchurPrimalF)."""
        return (self.B(p) - rhs_f) / self.c

    # solves ------------------------------------------------------------------
    def solve(self, rhs_p, rhs_f, rtol=1e-13, restart=30, maxit=400, workers=None, method="gmres"):
        """Krylov solve of S~ p' = b preconditioned by the exact L^+ (Sec. 4.1-4.2),
        by restarted GMRES or by BiCGStab (method="bicgstab").

        Returns (p', Phi', iterations, residual history)."""
        b = self.rhs(rhs_p, rhs_f)
        pre = lambda v: poisson.solve_laplacian(self.g, v, workers)
        if method == "bicgstab":
            p, its, hist = krylov.bicgstab(self.matvec, b, precond=pre, rtol=rtol, maxit=maxit)
        else:
            p, its, hist = krylov.gmres(self.matvec, b, precond=pre, rtol=rtol,
                                        restart=restart, maxit=maxit)
        p = p - p.mean()
        return p, self.force(p, rhs_f), its, hist

    def solve_direct(self, rhs_p, rhs_f):
        """Sparse LU of the bordered system [[S~, 1], [1^T, 0]] (small grids)."""
        N = self.g.N
        S = self.L + (self.G.T @ (self.W @ (self.W.T @ self.G))) / self.c
        one = sp.csr_matrix(np.ones((N, 1)))
        A = sp.bmat([[S, one], [one.T, None]], format="csc")
        b = self.rhs(rhs_p, rhs_f).ravel()
        x = spla.splu(A).solve(np.concatenate([b, [0.0]]))
        p = x[:N].reshape(self.g.n)
        return p, self.force(p, rhs_f)


def exact_schur_dense(G: np.ndarray, W: np.ndarray):
    """Dense L and the exact primal Schur complement L + B^T C^-1 B with
    C = W^T W (eq. SchurPrimal), for the spectral checks of Sec. 5."""
    L = G.T @ G
    C = W.T @ W
    B = W.T @ G
    Sp = L + B.T @ np.linalg.solve(C, B)
    return L, Sp, C


def preconditioned_spectrum(sys: SchurSystem, exact: bool, workers=None):
    """Eigenvalues of L^+ S on mean-zero pressures, the quantity bounded by
    the theorem of Sec. 5 and measured in Sec. 6.2: S = S~ = L + c^-1 B^T B
    (exact = False) or S_p = L + B^T C^-1 B with C = W^T W (exact = True).

    L^+ S = I + L^+ B^T M B with M = I/c or C^-1, and a product of two
    matrices has the same nonzero eigenvalues in either order, so apart from
    the eigenvalue 1 (on the mean-zero vectors that B annihilates) the
    spectrum is 1 + eig(M K) with the 3K x 3K matrix K = B L^+ B^T, formed
    column by column with the exact Poisson solve.  Returns those 3K values,
    ascending (the remaining eigenvalues are all 1)."""
    g = sys.g
    m = sys.W.shape[1]
    K = np.empty((m, m))
    for i in range(m):
        e = np.zeros(m)
        e[i] = 1.0
        z = poisson.solve_laplacian(g, sys.BT(e.reshape(-1, 3)), workers)
        K[:, i] = sys.B(z).ravel()
    K = 0.5 * (K + K.T)
    if exact:
        import scipy.linalg as sla
        C = (sys.W.T @ sys.W).toarray()
        ev = sla.eigh(K, C, eigvals_only=True)
    else:
        ev = np.linalg.eigvalsh(K) / sys.c
    return 1.0 + np.sort(ev)
