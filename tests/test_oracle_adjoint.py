"""Pins of the oracle's reverse-mode step (oracle/adjoint.py) against the
forward step itself: the polarization identity of the quadratic convection
term, the dot-product test on the inputs the step is affine in, exact central
differences along u^n (the step is quadratic in u^n), and central differences
along the point coordinates."""
import numpy as np
import pytest

from oracle import adjoint as oadj
from oracle import bodies as bd
from oracle import mac
from oracle import step as ostep
from paper_2501_15314_amd import workloads as wl

P, W_, F_ = mac.PERIODIC, mac.NOSLIP, mac.FREESLIP


@pytest.mark.parametrize("bc", [(P, P, P), (W_, W_, W_), (W_, P, P), (P, W_, W_), (F_, F_, W_)])
def test_convection_jacobian_polarization(bc):
    """N is quadratic with N(0) = 0, so J(u) v = N(u + v) - N(u) - N(v)."""
    g = mac.Grid((6, 8, 10), 0.125, bc)
    rng = np.random.default_rng(1)
    m = g.face_dof_mask()
    u = rng.standard_normal((3,) + g.n) * m
    v = rng.standard_normal((3,) + g.n) * m
    J = oadj.convection_jacobian(g, u)
    lhs = (J @ v.ravel()).reshape(v.shape)
    rhs = mac.convection(g, u + v) - mac.convection(g, u) - mac.convection(g, v)
    assert np.abs(lhs - rhs).max() < 1e-11 * np.abs(rhs).max()


def _setup(case, seed=7):
    rng = np.random.default_rng(seed)
    if case == "periodic":
        w = wl.make_c1(n=16, n_points=80)
        u0 = wl.solenoidal_field(rng, w.cfg.n, w.cfg.h, 0.3)
    else:
        w = wl.make_c3(seed=seed, n=16, points_per_sphere=40)
        w.bodies = w.bodies[:2]
        w.offsets = w.offsets[:80]
        g0 = mac.Grid(w.cfg.n, w.cfg.h, w.cfg.bc)
        u0 = rng.standard_normal((3,) + w.cfg.n) * 0.1 * g0.face_dof_mask()
    cfg = w.cfg
    g = mac.Grid(cfg.n, cfg.h, cfg.bc)
    mask = g.face_dof_mask()
    K = w.offsets.shape[0]
    um = u0 + 0.05 * rng.standard_normal(u0.shape) * mask
    st = ostep.State(u0 * mask, um * mask, rng.standard_normal(g.n), 0.3 * rng.standard_normal((K, 3)))
    Xs, k0 = [], 0
    for b in w.bodies:
        Xs.append(bd.points(b.center, bd.prescribed_rotation(b.omega, cfg.dt), w.offsets[k0:k0 + b.n_points]))
        k0 += b.n_points
    X = np.concatenate(Xs)
    U = 0.1 * rng.standard_normal((K, 3))
    return cfg, g, st, X, U


def _fwd(cfg, g, st, X, U):
    new, _ = ostep.one_way_step(g, cfg.nu, cfg.dt, st, X, U, cfg.delta, cfg.lump_c, 0.8)
    return new


def _pair(cfg, g, st, X, U, ybar):
    gu, gp, gphi = ybar
    grads, new, _ = oadj.one_way_step_vjp(g, cfg.nu, cfg.dt, st, X, U, cfg.delta, cfg.lump_c, 0.8,
                                          gu, gp, gphi)
    return grads, new


def _ydot(new, base, ybar):
    return sum(float(np.vdot(a - b, c)) for a, b, c in
               zip((new.u, new.p, new.phi), (base.u, base.p, base.phi), ybar))


@pytest.mark.parametrize("case", ["periodic", "walls"])
def test_step_vjp_dot_product_affine_inputs(case):
    """The step is affine in (u^{n-1}, p^n, Phi^n, U): step(x + xdot) - step(x)
    = J xdot, so <ybar, J xdot> must equal <J^T ybar, xdot>."""
    cfg, g, st, X, U = _setup(case)
    rng = np.random.default_rng(3)
    mask = g.face_dof_mask()
    ybar = (rng.standard_normal((3,) + g.n) * mask, rng.standard_normal(g.n),
            rng.standard_normal(st.phi.shape))
    grads, base = _pair(cfg, g, st, X, U, ybar)
    dirs = dict(um=rng.standard_normal(st.u.shape) * mask, p=rng.standard_normal(g.n),
                phi=rng.standard_normal(st.phi.shape), U=rng.standard_normal(U.shape))
    for name, xd in dirs.items():
        s2 = st.copy()
        U2 = U
        if name == "um":
            s2.um = st.um + xd
        elif name == "p":
            s2.p = st.p + xd
        elif name == "phi":
            s2.phi = st.phi + xd
        else:
            U2 = U + xd
        lhs = _ydot(_fwd(cfg, g, s2, X, U2), base, ybar)
        rhs = float(np.vdot(grads[name], xd))
        assert abs(lhs - rhs) < 1e-8 * (abs(lhs) + abs(rhs)), (name, lhs, rhs)


@pytest.mark.parametrize("case", ["periodic", "walls"])
def test_step_vjp_velocity_central_difference(case):
    """Along u^n the step is quadratic (through N only), so the central
    difference equals the directional derivative exactly."""
    cfg, g, st, X, U = _setup(case)
    rng = np.random.default_rng(4)
    mask = g.face_dof_mask()
    ybar = (rng.standard_normal((3,) + g.n) * mask, rng.standard_normal(g.n),
            rng.standard_normal(st.phi.shape))
    grads, base = _pair(cfg, g, st, X, U, ybar)
    v = rng.standard_normal(st.u.shape) * mask
    eps = 0.05
    sp_, sm_ = st.copy(), st.copy()
    sp_.u = st.u + eps * v
    sm_.u = st.u - eps * v
    fd = (_ydot(_fwd(cfg, g, sp_, X, U), base, ybar) - _ydot(_fwd(cfg, g, sm_, X, U), base, ybar)) / (2 * eps)
    an = float(np.vdot(grads["u"], v))
    assert abs(fd - an) < 1e-8 * abs(an), (fd, an)


@pytest.mark.parametrize("case", ["periodic", "walls"])
def test_step_vjp_positions_central_difference(case):
    cfg, g, st, X, U = _setup(case)
    rng = np.random.default_rng(5)
    mask = g.face_dof_mask()
    ybar = (rng.standard_normal((3,) + g.n) * mask, rng.standard_normal(g.n),
            rng.standard_normal(st.phi.shape))
    grads, base = _pair(cfg, g, st, X, U, ybar)
    for trial in range(2):
        Xd = rng.standard_normal(X.shape)
        eps = 1e-4 * g.h
        fp = _ydot(_fwd(cfg, g, st, X + eps * Xd, U), base, ybar)
        fm = _ydot(_fwd(cfg, g, st, X - eps * Xd, U), base, ybar)
        fd = (fp - fm) / (2 * eps)
        an = float(np.vdot(grads["X"], Xd))
        assert abs(fd - an) < 1e-5 * abs(an), (fd, an)


# --------------------------------------------------------------------------
# two-way step (fixed number of outer passes)

def _two_way_setup(bc, seed=11):
    rng = np.random.default_rng(seed)
    n, a, theta = 16, 0.17, (1.6, 2.4)
    g = mac.Grid((n, n, n), 1.0 / n, (bc,) * 3)
    K = int(round(4 * np.pi * a * a / g.h ** 2))
    off = wl.fibonacci_offsets(K, a)
    c = wl.lump_constant(wl.DELTA_PESKIN4, g.h, K, a)
    dt = 0.004
    fb = []
    for cen, th in zip(((0.38, 0.38, 0.6), (0.64, 0.62, 0.4)), theta):
        b = ostep.free_body(np.array(cen) + rng.uniform(-0.01, 0.01, 3), rng.normal(0, 0.1, 3),
                            rng.normal(0, 1.0, 3), a, th, off, dt)
        b.xc_m = b.xc - dt * b.us + rng.normal(0, 1e-4, 3)
        b.us_m = b.us + rng.normal(0, 0.01, 3)
        b.w_m = b.w + rng.normal(0, 0.1, 3)
        fb.append(b)
    mask = g.face_dof_mask()
    u0 = rng.standard_normal((3,) + g.n) * 0.05 * mask
    st = ostep.State(u0, u0 + 0.01 * rng.standard_normal(u0.shape) * mask, rng.standard_normal(g.n),
                     0.2 * rng.standard_normal((2 * K, 3)))
    ostep.init_volume_history(g, st.u, fb)
    for b in fb:
        b.I_m = b.I_m + rng.normal(0, 1e-4, 3)
        b.J_m = b.J_m + rng.normal(0, 1e-5, 3)
    return g, st, fb, c, dt


_BODY_IN = ("xc", "xc_m", "us", "us_m", "w", "w_m", "I_n", "I_m", "J_n", "J_m")


@pytest.mark.parametrize("bc", [P, W_, F_])
def test_two_way_step_vjp_central_differences(bc):
    """<ybar, (step(x + e d) - step(x - e d)) / 2e> = <J^T ybar, d> along a
    random direction of every input group, fluid and body."""
    g, st, fb, c, dt = _two_way_setup(bc)
    nu, xi, n_outer, gvec = 0.01, 0.6, 3, np.array([0.0, 0.0, -1.0])
    rng = np.random.default_rng(5)
    mask = g.face_dof_mask()
    K = st.phi.shape[0]
    gu = rng.standard_normal((3,) + g.n) * mask
    gp = rng.standard_normal(g.n)
    gphi = rng.standard_normal((K, 3))
    gbod = [dict(xc=rng.standard_normal(3), us=rng.standard_normal(3), w=rng.standard_normal(3),
                 I=rng.standard_normal(3), J=rng.standard_normal(3)) for _ in fb]
    grads, _, _, _ = oadj.two_way_step_vjp(g, nu, dt, gvec, st, fb, wl.DELTA_PESKIN4, c, xi, n_outer,
                                           gu, gp, gphi, gbod)

    def ell(s, bodies):
        new, nb, _ = ostep.two_way_step(g, nu, dt, gvec, s, bodies, wl.DELTA_PESKIN4, c, xi, n_outer,
                                        0.0, 1e-13, 1e-14)
        v = float(np.vdot(gu, new.u) + np.vdot(gp, new.p) + np.vdot(gphi, new.phi))
        for b, y in zip(nb, gbod):
            v += float(y["xc"] @ b.xc + y["us"] @ b.us + y["w"] @ b.w + y["I"] @ b.I_n + y["J"] @ b.J_n)
        return v

    groups = {"u": 1e-4, "um": 1e-4, "p": 1e-4, "phi": 1e-4}
    groups.update({f"b{i}.{k}": 1e-6 for i in range(len(fb)) for k in _BODY_IN})
    for name, eps in groups.items():
        if name.startswith("b"):
            i, key = int(name[1]), name[3:]
            d = rng.standard_normal(3)
            d *= {"I_n": 1e-3, "I_m": 1e-3, "J_n": 1e-4, "J_m": 1e-4}.get(key, 1.0)
            an = float(grads["bodies"][i][key] @ d)

            def shifted(sgn):
                bs = [b.copy() for b in fb]
                setattr(bs[i], key, getattr(bs[i], key) + sgn * eps * d)
                return ell(st, bs)
        else:
            shape = {"u": st.u.shape, "um": st.u.shape, "p": g.n, "phi": st.phi.shape}[name]
            d = rng.standard_normal(shape) * (mask if name in ("u", "um") else 1.0)
            an = float(np.vdot(grads[name], d))

            def shifted(sgn):
                s2 = st.copy()
                setattr(s2, name, getattr(st, name) + sgn * eps * d)
                return ell(s2, [b.copy() for b in fb])
        fd = (shifted(1.0) - shifted(-1.0)) / (2 * eps)
        assert abs(fd - an) < 2e-6 * max(abs(an), abs(fd), 1e-3), (name, fd, an)
