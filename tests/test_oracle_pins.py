"""Pins of the CPU oracle against facts fixed outside the oracle itself:
closed-form spectra, kernel moment identities, brute-force definitions on tiny
inputs, the spectral theorem, printed tables of the paper, and a second
(stencil) formulation of the grid operators."""
import math
import os

import numpy as np
import pytest
import scipy.sparse as sp

from oracle import bodies as bd
from oracle import delta, mac, poisson, schur
from oracle import step as ostep
from paper_2501_15314_amd import workloads as wl

P, W_, F_ = mac.PERIODIC, mac.NOSLIP, mac.FREESLIP


def _grid(n, bc, L=1.0):
    n = (n, n, n) if np.isscalar(n) else n
    return mac.Grid(n, L / n[0], bc)


# --------------------------------------------------------------------------
# P1: closed-form spectra of L and of the momentum operator

def _basis_1d(n, bc, k):
    i = np.arange(n)
    if bc == P:
        return np.cos(2 * np.pi * k * (i + 0.5) / n)
    return np.cos(np.pi * k * (i + 0.5) / n)        # DCT-II


@pytest.mark.parametrize("bc", [(P, P, P), (W_, W_, W_), (P, W_, P), (W_, P, W_), (F_, F_, F_),
                                (P, F_, W_)])
def test_laplacian_symbol(bc):
    g = _grid((6, 8, 10), bc)
    L = mac.laplacian(g)
    rng = np.random.default_rng(0)
    for _ in range(6):
        ks = [rng.integers(0, g.n[a]) for a in range(3)]
        v = np.einsum("i,j,k->ijk", *[_basis_1d(g.n[a], bc[a], ks[a]) for a in range(3)])
        lam = sum(poisson.eigenvalues_1d(g.n[a], g.h, bc[a])[ks[a]] for a in range(3))
        Lv = (L @ v.ravel()).reshape(g.n)
        assert np.allclose(Lv, lam * v, rtol=0, atol=1e-12 * max(1.0, lam))


def test_lap_symbol_closed_form_values():
    # (4/h^2) sin^2(pi k/n): for n = 4, k = 1 periodic -> 2/h^2; k = 2 -> 4/h^2
    e = poisson.eigenvalues_1d(4, 1.0, P)
    assert np.allclose(e, [0.0, 2.0, 4.0, 2.0])
    e = poisson.eigenvalues_1d(2, 1.0, W_)
    assert np.allclose(e, [0.0, 2.0])


@pytest.mark.parametrize("bc", [(P, P, P), (W_, W_, W_), (W_, P, W_), (F_, F_, F_), (F_, P, W_),
                                (W_, F_, F_)])
def test_momentum_operator_symbol(bc):
    """A = 3/(2dt) - nu Delta_h on each face grid.  Eigenvectors per axis:
    periodic Fourier; tangential no-slip (ghost = -u): DST-II with eigenvalue
    (4/h^2) sin^2(pi (k+1)/(2n)); tangential free-slip (ghost = +u): DCT-II
    with eigenvalue (4/h^2) sin^2(pi k/(2n)), k = 0 included (a uniform
    tangential flow is not damped); normal wall of either kind (Dirichlet on
    faces 0, n): DST-I on faces 1..n-1 with eigenvalue (4/h^2) sin^2(pi k/(2n))."""
    g = _grid((6, 8, 6), bc)
    nu, dt = 0.03, 0.01
    A = mac.helmholtz(g, nu, dt)
    rng = np.random.default_rng(1)
    for d in range(3):
        for _ in range(4):
            vecs, lam = [], 0.0
            for a in range(3):
                n = g.n[a]
                i = np.arange(n)
                if bc[a] == P:
                    k = rng.integers(0, n)
                    vecs.append(np.cos(2 * np.pi * k * (i + (0.0 if a == d else 0.5)) / n))
                    lam += 4 / g.h ** 2 * np.sin(np.pi * k / n) ** 2
                elif a == d:
                    k = rng.integers(1, n)
                    vecs.append(np.sin(np.pi * k * i / n))
                    lam += 4 / g.h ** 2 * np.sin(np.pi * k / (2 * n)) ** 2
                elif bc[a] == F_:
                    k = rng.integers(0, n) if _ else 0
                    vecs.append(np.cos(np.pi * k * (i + 0.5) / n))
                    lam += 4 / g.h ** 2 * np.sin(np.pi * k / (2 * n)) ** 2
                else:
                    k = rng.integers(0, n)
                    vecs.append(np.sin(np.pi * (k + 1) * (i + 0.5) / n))
                    lam += 4 / g.h ** 2 * np.sin(np.pi * (k + 1) / (2 * n)) ** 2
            v = np.zeros((3,) + g.n)
            v[d] = np.einsum("i,j,k->ijk", *vecs)
            Av = (A @ v.ravel()).reshape(v.shape)
            expect = (1.5 / dt + nu * lam) * v
            assert np.allclose(Av, expect, atol=1e-10 * (1.5 / dt + nu * lam))


# --------------------------------------------------------------------------
# P2 / P16: G, D, L consistency and a second formulation

@pytest.mark.parametrize("bc", [(P, P, P), (W_, W_, W_), (P, W_, W_), (F_, P, W_), (F_, F_, F_)])
def test_sparse_vs_stencil(bc):
    g = _grid((5, 6, 8), bc)
    rng = np.random.default_rng(2)
    p = rng.standard_normal(g.n)
    u = rng.standard_normal((3,) + g.n) * g.face_dof_mask()
    G, D, L = mac.gradient(g), mac.divergence(g), mac.laplacian(g)
    assert np.allclose((G @ p.ravel()).reshape(u.shape), mac.grad_stencil(g, p), atol=1e-12)
    assert np.allclose((D @ u.ravel()).reshape(g.n), mac.div_stencil(g, u), atol=1e-12)
    assert np.allclose((L @ p.ravel()).reshape(g.n), mac.lap_stencil(g, p), atol=1e-10)
    # adjointness <Du, q> = -<u, Gq> and -DG == L
    q = rng.standard_normal(g.n)
    assert abs(np.vdot(D @ u.ravel(), q.ravel()) + np.vdot(u.ravel(), G @ q.ravel())) < 1e-10
    assert abs(-(D @ G) - L).max() < 1e-10
    # constants are the null space of L and D maps into mean-zero fields
    assert np.abs(L @ np.ones(g.N)).max() < 1e-10
    assert abs((D @ u.ravel()).sum()) < 1e-9


def test_fast_poisson_inverse():
    for bc in [(P, P, P), (W_, W_, W_), (W_, P, W_)]:
        g = _grid((8, 6, 10), bc)
        rng = np.random.default_rng(3)
        b = rng.standard_normal(g.n)
        x = poisson.solve_laplacian(g, b)
        L = mac.laplacian(g)
        assert abs(x.mean()) < 1e-12
        assert np.allclose((L @ x.ravel()).reshape(g.n), b - b.mean(), atol=1e-10)


# --------------------------------------------------------------------------
# convection: conservation identities and second-order consistency

def test_convection_momentum_and_energy_periodic():
    g = _grid(12, (P, P, P))
    rng = np.random.default_rng(4)
    u = wl.solenoidal_field(rng, g.n, g.h, 1.0)
    assert np.abs(mac.div_stencil(g, u)).max() < 1e-10
    N = mac.convection(g, u)
    # discrete momentum is conserved (flux form)
    for d in range(3):
        assert abs(N[d].sum()) < 1e-9 * np.abs(N[d]).max() * N[d].size
    # with Du = 0 the divergence form on the staggered grid conserves energy
    assert abs(np.vdot(u, N)) < 1e-10 * np.abs(u).max() * np.abs(N).sum()


def test_convection_second_order():
    def field(n):
        g = _grid(n, (P, P, P))
        errs = []
        pos = [bd.face_positions(g, d) for d in range(3)]
        tp = 2 * np.pi
        u = np.empty((3,) + g.n)
        u[0] = np.sin(tp * pos[0][0]) * np.cos(tp * pos[0][1]) * np.cos(tp * pos[0][2])
        u[1] = np.cos(tp * pos[1][0]) * np.sin(tp * pos[1][1]) * np.cos(tp * pos[1][2])
        u[2] = -2 * np.cos(tp * pos[2][0]) * np.cos(tp * pos[2][1]) * np.sin(tp * pos[2][2])
        N = mac.convection(g, u)
        # analytic div(u u)_x = d(uu)/dx + d(vu)/dy + d(wu)/dz for this field
        x, y, z = pos[0]
        s, c = np.sin, np.cos
        uu = lambda x, y, z: s(tp*x)*c(tp*y)*c(tp*z)
        vv = lambda x, y, z: c(tp*x)*s(tp*y)*c(tp*z)
        ww = lambda x, y, z: -2*c(tp*x)*c(tp*y)*s(tp*z)
        eps = 1e-5
        def ddx(f, a):
            e = [0, 0, 0]; e[a] = eps
            return (f(x+e[0], y+e[1], z+e[2]) - f(x-e[0], y-e[1], z-e[2])) / (2*eps)
        ex = ddx(lambda x, y, z: uu(x, y, z)**2, 0) + ddx(lambda x, y, z: vv(x, y, z)*uu(x, y, z), 1) \
            + ddx(lambda x, y, z: ww(x, y, z)*uu(x, y, z), 2)
        return np.abs(N[0] - ex).max()
    e1, e2 = field(16), field(32)
    assert 3.5 < e1 / e2 < 4.5


# --------------------------------------------------------------------------
# P3: delta-kernel identities

@pytest.mark.parametrize("kernel", [delta.PESKIN4, delta.ROMA3])
def test_kernel_moments(kernel):
    phi = delta.PHI[kernel]
    r = np.random.default_rng(5).uniform(0, 1, 10000)
    j = np.arange(-4, 5)
    vals = phi(r[:, None] - j[None, :])
    off = r[:, None] - j[None, :]
    assert np.abs(vals.sum(1) - 1).max() < 1e-14                      # partition of unity
    assert np.abs((off * vals).sum(1)).max() < 1e-14                  # zero first moment
    s2 = 3 / 8 if kernel == delta.PESKIN4 else 1 / 2
    assert np.abs((vals ** 2).sum(1) - s2).max() < 1e-14              # sum of squares
    if kernel == delta.PESKIN4:
        even = (j % 2 == 0)
        assert np.abs(vals[:, even].sum(1) - 0.5).max() < 1e-14
    else:
        assert abs(phi(np.array([0.0]))[0] - 2 / 3) < 1e-15           # eq. delta at r = 0
        assert abs(phi(np.array([1.0]))[0] - 1 / 6) < 1e-15           # and at r = h
        assert phi(np.array([1.5]))[0] == 0.0


@pytest.mark.parametrize("kernel", [delta.PESKIN4, delta.ROMA3])
def test_kernel_derivative_matches_finite_differences(kernel):
    r = np.random.default_rng(6).uniform(-2.2, 2.2, 2000)
    # stay away from the kinks at half-integers (ROMA3) where phi is only C^1
    r = r[np.min(np.abs(r[:, None] - np.array([-1.5, -0.5, 0.5, 1.5, -2, -1, 0, 1, 2])[None]), 1) > 1e-3]
    e = 1e-6
    fd = (delta.PHI[kernel](r + e) - delta.PHI[kernel](r - e)) / (2 * e)
    assert np.abs(fd - delta.DPHI[kernel](r)).max() < 1e-6


# --------------------------------------------------------------------------
# P4 / P5: W against its definition by brute force, interpolation consistency

def _brute_W(g, X, kernel, d):
    phi = delta.PHI[kernel]
    pos = bd.face_positions(g, d).reshape(3, -1).T
    out = np.zeros((g.N, X.shape[0]))
    for k in range(X.shape[0]):
        r = (pos - X[k]) / g.h
        for a in range(3):
            if g.bc[a] == P:
                r[:, a] -= g.n[a] * np.round(r[:, a] / g.n[a])
        out[:, k] = phi(r[:, 0]) * phi(r[:, 1]) * phi(r[:, 2])
    return out


@pytest.mark.parametrize("kernel", [delta.PESKIN4, delta.ROMA3])
@pytest.mark.parametrize("bc", [(P, P, P), (W_, W_, W_)])
def test_W_brute_force(kernel, bc):
    g = _grid(8, bc)
    rng = np.random.default_rng(7)
    lo, hi = (0.0, 1.0) if bc[0] == P else (0.3, 0.7)
    X = rng.uniform(lo, hi, (5, 3))
    Wm = delta.regularization_matrix(g, X, kernel).toarray()
    for d in range(3):
        ref = _brute_W(g, X, kernel, d)
        blk = Wm[d * g.N:(d + 1) * g.N, d::3]
        assert np.abs(blk - ref).max() < 1e-15
        # off-component blocks are empty
        for e in range(3):
            if e != d:
                assert np.abs(Wm[d * g.N:(d + 1) * g.N, e::3]).max() == 0.0


def test_interpolation_consistency_and_adjoint():
    g = _grid(16, (P, P, P))
    rng = np.random.default_rng(8)
    X = rng.uniform(0.3, 0.7, (40, 3))
    Wm = delta.regularization_matrix(g, X, delta.PESKIN4)
    # constants and linear fields are interpolated exactly
    for d in range(3):
        u = np.zeros((3,) + g.n)
        u[d] = 1.0
        assert np.abs(delta.interpolate(Wm, u)[:, d] - 1.0).max() < 1e-14
        pos = bd.face_positions(g, d)
        u[d] = 0.3 * pos[0] - 0.7 * pos[1] + 0.2 * pos[2]
        ref = 0.3 * X[:, 0] - 0.7 * X[:, 1] + 0.2 * X[:, 2]
        assert np.abs(delta.interpolate(Wm, u)[:, d] - ref).max() < 1e-14
    # <W f, u> = <f, W^T u> (spreading and interpolation are transposes)
    f = rng.standard_normal((40, 3))
    u = rng.standard_normal((3,) + g.n)
    lhs = np.vdot(delta.spread(Wm, f, g.n), u)
    rhs = np.vdot(f, delta.interpolate(Wm, u))
    assert abs(lhs - rhs) < 1e-14 * abs(lhs) * 100


@pytest.mark.parametrize("bc", [(W_, W_, W_), (F_, P, P)])
def test_support_crossing_wall_rejected(bc):
    g = _grid(16, bc)
    with pytest.raises(ValueError):
        delta.regularization_matrix(g, np.array([[0.05, 0.5, 0.5]]), delta.PESKIN4)
    delta.regularization_matrix(g, np.array([[0.2, 0.5, 0.5]]), delta.PESKIN4)


# --------------------------------------------------------------------------
# P6: the paper's Appendix A table of R^T R row sums

def _load_table(path):
    rows = []
    for line in open(path):
        line = line.strip()
        if line and not line.startswith("#"):
            rows.append([float(x) for x in line.split()])
    return np.array(rows)


def test_rtr_row_sums_match_appendix_table(golden_dir):
    tab = _load_table(os.path.join(golden_dir, "table_a1_rtr_rowsums.txt"))
    n = 32
    g = _grid(n, (P, P, P))
    a = 10 * g.h                                   # D / h = 20
    for ratio, mn, mx, avg in tab:
        K = int(round(4 * np.pi * (a / g.h) ** 2 * ratio ** 2))
        X = 0.5 + 0.13 * g.h + wl.fibonacci_offsets(K, a)
        Wm = delta.regularization_matrix(g, X, delta.ROMA3)
        W0 = Wm[:g.N, 0::3]
        rs = np.asarray((W0.T @ W0).sum(axis=1)).ravel()
        assert abs(rs.mean() - avg) < 0.012 * max(1.0, avg), (ratio, rs.mean(), avg)
        assert abs(rs.min() - mn) < 0.03 * max(1.0, mn), (ratio, rs.min(), mn)
        assert abs(rs.max() - mx) < 0.03 * max(1.0, mx), (ratio, rs.max(), mx)


def test_lumping_constant_tracks_row_sums():
    w = wl.make_c1()
    g = _grid(w.cfg.n[0], (P, P, P))
    X = w.bodies[0].center + w.offsets
    Wm = delta.regularization_matrix(g, X, delta.PESKIN4)
    W0 = Wm[:g.N, 0::3]
    rs = np.asarray((W0.T @ W0).sum(axis=1)).ravel()
    assert abs(rs.mean() / w.cfg.lump_c - 1) < 0.05


# --------------------------------------------------------------------------
# P7 / P8: Schur solve vs direct LU, block-row identity, spectral theorem

def _small_system(n=12, bc=(P, P, P), K=60, kernel=delta.PESKIN4, seed=9):
    g = _grid(n, bc)
    rng = np.random.default_rng(seed)
    a = 0.25
    X = 0.5 + rng.uniform(-0.02, 0.02, 3) + wl.fibonacci_offsets(K, a)
    Wm = delta.regularization_matrix(g, X, kernel)
    c = wl.lump_constant(kernel, g.h, K, a)
    return g, X, Wm, c


@pytest.mark.parametrize("bc", [(P, P, P), (W_, W_, W_)])
def test_schur_krylov_vs_direct(bc):
    g, X, Wm, c = _small_system(16, bc, 200)
    S = schur.SchurSystem(g, Wm, c)
    rp, rf = wl.random_schur_rhs(10, g.n, X.shape[0])
    p1, f1, its, hist = S.solve(rp, rf, rtol=1e-13)
    p2, f2 = S.solve_direct(rp, rf)
    assert np.linalg.norm(p1 - p2) / np.linalg.norm(p2) < 1e-11
    assert np.linalg.norm(f1 - f2) / np.linalg.norm(f2) < 1e-11
    assert its < 20
    # first block row L p' + B^T Phi' = RHS_p (projected) holds
    r1 = (S.L @ p1.ravel()).reshape(g.n) + S.BT(f1) - (rp - rp.mean())
    assert np.abs(r1).max() < 1e-9 * np.abs(rp).max()


@pytest.mark.parametrize("bc", [(P, P, P), (W_, P, W_)])
def test_schur_bicgstab_vs_direct(bc):
    """BiCGStab with the exact L^+ (the paper's pairing, Sec. 4.2) reaches the
    LU solution; with a spectrum of L^+ S~ inside [1, 2] it needs only a few
    iterations (two operator applications each)."""
    g, X, Wm, c = _small_system(16, bc, 200)
    S = schur.SchurSystem(g, Wm, c)
    rp, rf = wl.random_schur_rhs(11, g.n, X.shape[0])
    p1, f1, its, hist = S.solve(rp, rf, rtol=1e-12, method="bicgstab")
    p2, f2 = S.solve_direct(rp, rf)
    assert np.linalg.norm(p1 - p2) / np.linalg.norm(p2) < 1e-10
    assert np.linalg.norm(f1 - f2) / np.linalg.norm(f2) < 1e-10
    assert hist[-1] < 1e-11
    assert its <= 12


def test_bicgstab_closed_forms():
    """A = a I converges in one iteration to b / a; on a diagonal SPD matrix
    with k distinct eigenvalues the iterates reach the solution, and the result
    matches scipy's BiCGStab."""
    from oracle import krylov
    import scipy.sparse.linalg as spla
    rng = np.random.default_rng(3)
    b = rng.standard_normal(50)
    x, its, _ = krylov.bicgstab(lambda v: 2.5 * v, b, rtol=1e-14)
    assert its == 1 and np.abs(x - b / 2.5).max() < 1e-15
    d = np.repeat([1.0, 3.0, 7.0], [20, 20, 10])
    x, its, hist = krylov.bicgstab(lambda v: d * v, b, rtol=1e-13)
    assert np.abs(x - b / d).max() < 1e-11 and its <= 4
    A = np.diag(d) + 0.1 * np.diag(np.ones(49), 1)
    x, its, hist = krylov.bicgstab(lambda v: A @ v, b, rtol=1e-13, maxit=200)
    xs, info = spla.bicgstab(A, b, rtol=1e-13, maxiter=200)
    assert info == 0
    assert np.abs(x - np.linalg.solve(A, b)).max() < 1e-10
    assert np.abs(xs - np.linalg.solve(A, b)).max() < 1e-9


def test_spectral_theorem_bounds():
    """spec(L^-1 (L + B^T C^-1 B)) in [1, 2] on the mean-zero subspace
    (theorem of Sec. 5), and the lumped operator is bounded by
    1 + lambda_max(C)/c."""
    g, X, Wm, c = _small_system(8, (P, P, P), 40, delta.ROMA3)
    G = mac.gradient(g).toarray()
    Wd = Wm.toarray()
    L, Sp, C = schur.exact_schur_dense(G, Wd)
    # restrict to mean-zero vectors with an orthonormal basis Q
    N = g.N
    Q, _ = np.linalg.qr(np.eye(N)[:, 1:] - 1.0 / N)
    Lq, Sq = Q.T @ L @ Q, Q.T @ Sp @ Q
    ev = np.linalg.eigvals(np.linalg.solve(Lq, Sq)).real
    assert ev.min() > 1 - 1e-8 and ev.max() < 2 + 1e-8
    St = Q.T @ (L + G.T @ Wd @ Wd.T @ G / c) @ Q
    ev2 = np.linalg.eigvals(np.linalg.solve(Lq, St)).real
    lmax = np.linalg.eigvalsh(C).max()
    assert ev2.min() > 1 - 1e-8 and ev2.max() < 1 + lmax / c + 1e-8


# --------------------------------------------------------------------------
# P9 / P10: one-way step properties, flat iteration counts

@pytest.mark.parametrize("bc", [(P, P, P), (W_, F_, W_)])
def test_preconditioned_spectrum_matches_dense(bc):
    """The reduced 3K x 3K form of spec(L^+ S) equals the dense spectrum of
    the mean-zero pencil: 1 with multiplicity N - 1 - 3K and the 3K reduced
    values, for the lumped and for the exact primal Schur complement."""
    g, X, Wm, c = _small_system(8, bc, 30, delta.ROMA3)
    sysm = schur.SchurSystem(g, Wm, c)
    G = mac.gradient(g).toarray()
    Wd = Wm.toarray()
    L, Sp, C = schur.exact_schur_dense(G, Wd)
    N = g.N
    Q, _ = np.linalg.qr(np.eye(N)[:, 1:] - 1.0 / N)
    Lq = Q.T @ L @ Q
    for exact, S in ((True, Sp), (False, L + G.T @ Wd @ Wd.T @ G / c)):
        dense = np.sort(np.linalg.eigvals(np.linalg.solve(Lq, Q.T @ S @ Q)).real)
        red = schur.preconditioned_spectrum(sysm, exact)
        m = red.size
        assert np.allclose(dense[-m:], red, rtol=0, atol=1e-9)
        assert np.allclose(dense[:-m], 1.0, rtol=0, atol=1e-9)
        if exact:
            assert red.min() > 1 - 1e-9 and red.max() < 2 + 1e-9


def test_one_way_step_divergence_free_and_slip():
    w = wl.make_c1(n=16, n_points=80)
    cfg = w.cfg
    g = mac.Grid(cfg.n, cfg.h, cfg.bc)
    b = w.bodies[0]
    st = ostep.State(w.u0.copy(), w.u0.copy(), np.zeros(g.n), np.zeros((w.n_points, 3)))
    t1 = cfg.dt
    X = bd.points(bd.prescribed_center(b.center, b.vel, b.osc_amp, b.osc_omega, t1),
                  np.eye(3), w.offsets)
    U = np.tile(bd.prescribed_velocity(b.vel, b.osc_amp, b.osc_omega, t1), (w.n_points, 1))
    new, info = ostep.one_way_step(g, cfg.nu, cfg.dt, st, X, U, cfg.delta, cfg.lump_c)
    D = mac.divergence(g)
    div_star = np.linalg.norm(D @ info["ustar"].ravel())
    div_new = np.linalg.norm(D @ new.u.ravel())
    # row 1 of the saddle system makes D u^{n+1} vanish to solver tolerance
    assert div_new < 1e-10 * max(div_star, np.linalg.norm(new.u) / g.h)
    assert div_new < 1e-3 * div_star
    # the slip is reduced by the correction
    slip0 = np.linalg.norm(delta.interpolate(info["W"], info["ustar"]) - U)
    slip1 = np.linalg.norm(delta.interpolate(info["W"], new.u) - U)
    assert slip1 < 0.7 * slip0


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_one_way_steps_advect_a_transverse_wave_downstream(axis):
    """Sign and placement of the convection term in the momentum predictor
    (Sec. 3.1, eq. ustar: the material derivative du/dt + u.grad u on the
    left, so N(u^n) enters the right-hand side with a minus sign).

    A uniform stream U0 along `axis` carries a small transverse wave
    v = eps sin(2 pi x_axis / L) whose velocity points along the next axis;
    the field is divergence-free, p stays constant and no body is present.
    The exact solution of the continuous equations is the wave moved
    downstream by U0 t and damped by exp(-nu k^2 t).  After k steps the
    oracle's wave must have moved +U0 k dt (to the O(h^2) phase error of
    central differences and the O(dt) of the explicit term) and kept
    the viscous amplitude; with the sign of N flipped it moves upstream."""
    n = [8, 8, 8]
    n[axis] = 32
    h = 1.0 / 32
    g = mac.Grid(tuple(n), h, (P, P, P))
    U0, eps, nu, dt, k = 1.0, 1e-3, 0.01, 0.002, 25
    tr = (axis + 1) % 3
    x = (np.arange(32) + 0.5) * h          # transverse component sits at cell centres along `axis`
    shape = [1, 1, 1]
    shape[axis] = 32
    u = np.zeros((3,) + g.n)
    u[axis] = U0
    u[tr] = eps * np.sin(2 * np.pi * x).reshape(shape)
    st = ostep.State(u.copy(), u.copy(), np.zeros(g.n), np.zeros((0, 3)))
    none = np.zeros((0, 3))
    for _ in range(k):
        st, _ = ostep.one_way_step(g, nu, dt, st, none, none, delta.PESKIN4, 0.375)
    line = [0, 0, 0]
    line[axis] = slice(None)
    v = st.u[tr][tuple(line)]
    a = 2.0 / 32 * np.sum(v * np.sin(2 * np.pi * x))
    b = 2.0 / 32 * np.sum(v * np.cos(2 * np.pi * x))
    shift = np.arctan2(-b, a) / (2 * np.pi)  # v = A sin(2 pi (x - shift))
    amp = np.hypot(a, b) / eps
    assert abs(shift - U0 * k * dt) < 0.05 * U0 * k * dt, shift
    assert abs(amp - np.exp(-nu * (2 * np.pi) ** 2 * k * dt)) < 0.01, amp
    # the stream itself is untouched and no other component appears
    assert np.abs(st.u[axis] - U0).max() < 1e-12
    assert np.abs(st.u[3 - axis - tr]).max() < 1e-12
    assert np.ptp(st.p) < 1e-10


def test_iteration_count_flat_under_refinement():
    """Spectral equivalence (Sec. 5, Sec. 6.2): with the exact Laplacian as
    preconditioner the Krylov count does not grow with resolution."""
    counts = []
    for n in (16, 32, 48):
        g = _grid(n, (P, P, P))
        K = int(round(300 * (n / 32) ** 2))
        X = np.array([0.5, 0.49, 0.51]) + wl.fibonacci_offsets(K, 0.15)
        Wm = delta.regularization_matrix(g, X, delta.PESKIN4)
        S = schur.SchurSystem(g, Wm, wl.lump_constant(delta.PESKIN4, g.h, K, 0.15))
        rp, rf = wl.random_schur_rhs(11, g.n, K)
        _, _, its, _ = S.solve(rp, rf, rtol=1e-10)
        counts.append(its)
    assert max(counts) - min(counts) <= 2, counts
    assert max(counts) <= 15, counts


# --------------------------------------------------------------------------
# P15 + two-way pieces

def test_volume_fraction_total_volume():
    g = _grid(32, (P, P, P))
    a = 0.2
    for d in range(3):
        al = bd.volume_fraction(g, d, np.array([0.5, 0.47, 0.52]), a)
        vol = al.sum() * g.h ** 3
        assert abs(vol / (4 / 3 * np.pi * a ** 3) - 1) < 0.01


def test_volume_integrals_of_rigid_motion():
    """For u = U + w x r inside the sphere, the integrals equal V U and I_f w
    (I_f = 2/5 V a^2 for unit density) up to O(h)."""
    g = _grid(40, (P, P, P))
    a, c = 0.25, np.array([0.5, 0.5, 0.5])
    U, w = np.array([0.3, -0.2, 0.1]), np.array([0.5, 0.2, -0.4])
    u = np.empty((3,) + g.n)
    for d in range(3):
        r = bd.face_positions(g, d) - c.reshape(3, 1, 1, 1)
        u[d] = U[d] + np.cross(w, r, axisa=0, axisb=0, axisc=0)[d]
    lin, ang = bd.volume_integrals(g, u, c, a)
    V = 4 / 3 * np.pi * a ** 3
    assert np.allclose(lin, V * U, rtol=0.02)
    assert np.allclose(ang, 0.4 * V * a * a * w, rtol=0.05)


def test_rotation_update_orthonormal_and_angle():
    R = np.eye(3)
    w = np.array([0.0, 0.0, 2.0])
    R1 = bd.rotation_step(R, w, w, 0.1)
    assert np.allclose(R1.T @ R1, np.eye(3), atol=1e-15)
    assert np.allclose(R1[:2, :2], [[np.cos(0.2), -np.sin(0.2)], [np.sin(0.2), np.cos(0.2)]])


def test_newton_euler_free_fall_limit():
    """No fluid force and no added mass: u_s^{k} follows BDF2 of du/dt =
    (theta - 1)/theta g exactly."""
    us, w = bd.newton_euler(2.0, 0.1, 0.01, np.zeros(3), np.zeros(3), np.zeros(3), np.zeros(3),
                            np.zeros(3), np.zeros(3), np.zeros(3), np.zeros(3), np.zeros(3),
                            np.zeros(3), np.zeros(3), np.zeros(3), (0, 0, -1.0))
    assert np.allclose(us, [0, 0, -2 / 3 * 0.01 * 0.5])
    assert np.allclose(w, 0)


# --------------------------------------------------------------------------
# two-way coupling (Sec. 3.2.1)

def _two_way(n, bc, a, theta, gvec, u0=None, v0=(0, 0, 0), w0=(0, 0, 0), nsteps=1, n_outer=3,
             xi=0.6, nu=0.002, dt=0.002, center=(0.5, 0.5, 0.5)):
    g = _grid(n, (bc,) * 3)
    K = int(round(4 * np.pi * a * a / g.h ** 2))
    off = wl.fibonacci_offsets(K, a)
    c = wl.lump_constant(delta.PESKIN4, g.h, K, a)
    fb = [ostep.free_body(np.array(center, float), np.array(v0, float), np.array(w0, float),
                          a, theta, off, dt)]
    u0 = np.zeros((3,) + g.n) if u0 is None else u0
    st = ostep.State(u0.copy(), u0.copy(), np.zeros(g.n), np.zeros((K, 3)))
    ostep.init_volume_history(g, st.u, fb)
    out = []
    for _ in range(nsteps):
        new, nbod, info = ostep.two_way_step(g, nu, dt, np.array(gvec, float), st, fb, delta.PESKIN4,
                                             c, xi, n_outer)
        out.append((st, fb, new, nbod, info))
        st, fb = new, nbod
    return g, out


def test_two_way_fluid_momentum_balance():
    """Periodic box: convection (divergence form), viscosity and the pressure
    gradient sum to zero over the grid and the delta weights of a point sum to
    one, so the BDF2 change of the fluid momentum equals the total spread force
    h^3 sum Phi^{n+1} exactly, whatever the outer iterations did."""
    n = 16
    rng = np.random.default_rng(4)
    u0 = wl.solenoidal_field(rng, (n, n, n), 1.0 / n, 0.05)
    g, out = _two_way(n, P, 0.25, 1.5, (0, 0, -1.0), u0=u0, v0=(0.02, 0, 0), nsteps=2, n_outer=2)
    for st, _, new, _, _ in out:
        h3 = g.h ** 3
        dm = h3 * (3 * new.u - 4 * st.u + st.um).sum(axis=(1, 2, 3)) / (2 * 0.002)
        f = h3 * new.phi.sum(axis=0)
        assert np.allclose(dm, f, rtol=1e-9, atol=1e-12 * np.abs(f).max())


def test_two_way_ballistic_heavy_body():
    """theta -> infinity without gravity: the fluid cannot change the body's
    motion, so Step 1 must advance the centre by dt u_s and the orientation by
    the angle dt |omega| about the fixed spin axis."""
    v0, w0, dt = np.array([0.3, -0.2, 0.1]), np.array([0.0, 0.0, 2.0]), 0.002
    g, out = _two_way(16, P, 0.25, 1e12, (0, 0, 0), v0=v0, w0=w0, nsteps=3, n_outer=2, dt=dt)
    c0 = np.array([0.5, 0.5, 0.5])
    for s, (_, _, _, nb, info) in enumerate(out, start=1):
        b = nb[0]
        assert np.allclose(b.us, v0, atol=1e-9) and np.allclose(b.w, w0, atol=1e-9)
        assert np.allclose(b.xc, c0 + s * dt * v0, atol=1e-12)
        ang = s * dt * 2.0
        Rz = np.array([[np.cos(ang), -np.sin(ang), 0], [np.sin(ang), np.cos(ang), 0], [0, 0, 1]])
        assert np.allclose(b.R, Rz, atol=1e-12)
        assert np.allclose(info["X"], b.xc + b.offsets @ b.R.T, atol=1e-14)


def test_two_way_settling_from_rest():
    """A sphere released from rest (theta = 2) accelerates along g, slower than
    free fall (theta - 1)/theta g because the fluid inside and around it must be
    accelerated too; the inviscid added-mass value is (theta - 1)/(theta + 1/2) g.
    At 4.8 cells per radius the regularised sphere is effectively larger than a,
    which adds inertia, so the bracket is loose."""
    theta, dt = 2.0, 0.002
    g, out = _two_way(24, W_, 0.2, theta, (0, 0, -1.0), nsteps=1, n_outer=16, dt=dt)
    b = out[0][3][0]
    acc = 3 * b.us / (2 * dt)          # BDF2 from rest
    free = (theta - 1) / theta
    added = (theta - 1) / (theta + 0.5)
    assert -free < acc[2] < -0.55 * added
    assert np.abs(acc[:2]).max() < 1e-3 * abs(acc[2])
    # the outer iterations contract
    crit = out[0][4]["crit"]
    assert crit[-1] < 0.05 * crit[0]


def test_two_way_spin_down():
    """A sphere spinning in fluid at rest (theta = 10): the first step shares its
    angular momentum with the fluid it must carry (at least the enclosed fluid,
    moment of inertia I_p / theta relative to the body's), after the start-up
    transient the surrounding fluid keeps slowing it down, and the spin axis
    stays put."""
    theta, w0 = 10.0, np.array([0.0, 0.0, 3.0])
    g, out = _two_way(16, P, 0.25, theta, (0, 0, 0), w0=w0, nsteps=6, n_outer=4)
    wz = [o[3][0].w[2] for o in out]
    # theta I_p w0 = (theta I_p + X I_p) w1 with the carried inertia X I_p, X > 1
    X = theta * (w0[2] / wz[0] - 1.0)
    assert 1.0 < X < 4.0
    assert wz[3] > wz[4] > wz[5] > 0
    for o in out:
        assert np.abs(o[3][0].w[:2]).max() < 1e-3 * wz[0]


def test_two_way_drag_along():
    """A body at rest in a uniformly moving periodic fluid is dragged along:
    0 < u_s < U0 along the flow."""
    n, U0 = 16, 0.1
    u0 = np.zeros((3, n, n, n))
    u0[0] = U0
    g, out = _two_way(n, P, 0.25, 2.0, (0, 0, 0), u0=u0, nsteps=2, n_outer=4)
    us = [o[3][0].us for o in out]
    assert 0 < us[0][0] < us[1][0] < U0
    assert np.abs(us[1][1:]).max() < 1e-2 * us[1][0]


def test_two_way_steady_translation():
    """Galilean consistency: a sphere moving with a uniform periodic flow stays
    in it (the BDF2 weights of the enclosed-fluid momentum sum to zero for a
    steady state); only the small change of the discrete enclosed volume as the
    sphere crosses cells perturbs it."""
    n, U0 = 16, 0.1
    u0 = np.zeros((3, n, n, n))
    u0[0] = U0
    g, out = _two_way(n, P, 0.25, 2.0, (0, 0, 0), u0=u0, v0=(U0, 0, 0), nsteps=2, n_outer=3)
    for _, _, new, nb, _ in out:
        assert np.abs(nb[0].us - [U0, 0, 0]).max() < 2e-3 * U0
        assert np.abs(new.u[0] - U0).max() < 2e-2 * U0
