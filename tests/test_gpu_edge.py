"""Degenerate inputs through the C ABI, against the oracle: no Lagrangian
points at all (the step reduces to a projection method and S~ to L), a
single point, a zero right-hand side, and a non-cubic grid with walls on one
axis and a ragged number of tiles."""
import numpy as np
import pytest

from oracle import mac as omac
from oracle import poisson as opoisson
from oracle import step as ostep
from paper_2501_15314_amd import workloads as wl

from .conftest import gpu_available
from .gpu_helpers import oracle_for, rel

pytestmark = pytest.mark.gpu

if gpu_available():
    from paper_2501_15314_amd.sim import Sim


def _empty(n=(16, 24, 48), bc=(wl.BC_NOSLIP, wl.BC_PERIODIC, wl.BC_FREESLIP), precision=wl.PREC_FP64):
    h = 1.0 / 32
    cfg = wl.Config(n=n, length=tuple(x * h for x in n), bc=bc, nu=0.02, dt=0.005, precision=precision,
                    krylov_rtol=1e-12 if precision == wl.PREC_FP64 else 1e-11,
                    helm_rtol=1e-12 if precision == wl.PREC_FP64 else 1e-11)
    rng = np.random.default_rng(3)
    g = omac.Grid(cfg.n, cfg.h, cfg.bc)
    u0 = rng.standard_normal((3,) + cfg.n) * 0.05 * g.face_dof_mask()
    return wl.Workload("empty", cfg, [], np.zeros((0, 3)), u0, steps=1, seed=3)


@pytest.mark.parametrize("prec", [wl.PREC_FP64, wl.PREC_FP32MG])
def test_step_without_points_is_a_projection(prec):
    w = _empty(precision=prec)
    cfg = w.cfg
    print(f"no points, n={cfg.n} bc={cfg.bc} prec {prec}", flush=True)
    sim = Sim(cfg, 0)
    sim.set_workload(w)
    st, _ = sim.step(1)
    u, p = sim.get_fields()
    g = omac.Grid(cfg.n, cfg.h, cfg.bc)
    state = ostep.State(w.u0, w.u0, np.zeros(g.n), np.zeros((0, 3)))
    new, _ = ostep.one_way_step(g, cfg.nu, cfg.dt, state, np.zeros((0, 3)), np.zeros((0, 3)), cfg.delta,
                                cfg.lump_c, cfg.xi)
    tol = 1e-9 if prec == wl.PREC_FP64 else 1e-7
    eu = rel(u.cpu().numpy(), new.u)
    ep = rel(p.cpu().numpy() - p.cpu().numpy().mean(), new.p - new.p.mean())
    print(f"  err u={eu:.2e} p={ep:.2e} div_rel={st.div_rel:.1e} schur iters {st.schur.iters}", flush=True)
    assert eu < tol and ep < tol
    assert st.div_rel < 1e-8
    sim.close()


def test_schur_without_points_is_the_laplacian():
    w = _empty()
    sim = Sim(w.cfg, 0)
    sim.set_workload(w)
    g = omac.Grid(w.cfg.n, w.cfg.h, w.cfg.bc)
    rp, rf = wl.random_schur_rhs(5, g.n, 0)
    p, phi, st = sim.solve_schur(rp, rf)
    ref = opoisson.solve_laplacian(g, rp - rp.mean())
    err = rel(p.cpu().numpy(), ref - ref.mean())
    print(f"S~ = L: err {err:.2e}, {st.iters} iterations", flush=True)
    assert err < 1e-10 and phi.shape[0] == 0
    sim.close()


def test_zero_right_hand_side():
    w = wl.make_c1(n=16, n_points=80)
    sim = Sim(w.cfg, w.n_points)
    sim.set_bodies(w.bodies, w.offsets)
    p, phi, st = sim.solve_schur(np.zeros(w.cfg.n), np.zeros((w.n_points, 3)))
    assert st.iters == 0 and not p.abs().max().item() and not phi.abs().max().item()
    sim.close()


def test_single_point():
    w = wl.make_c1(n=16, n_points=1)
    w.offsets = np.array([[0.1, 0.0, 0.0]])
    sim = Sim(w.cfg, 1)
    sim.set_bodies(w.bodies, w.offsets)
    g, X, W, S = oracle_for(w)
    rp, rf = wl.random_schur_rhs(6, g.n, 1)
    p, phi, st = sim.solve_schur(rp, rf)
    pr, phir, _, _ = S.solve(rp, rf, rtol=1e-13)
    ep, ef = rel(p.cpu().numpy(), pr), rel(phi.cpu().numpy(), phir)
    print(f"one point: err p={ep:.2e} phi={ef:.2e}", flush=True)
    assert ep < 1e-9 and ef < 1e-9
    sim.close()
