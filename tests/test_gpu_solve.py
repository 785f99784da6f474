"""Parity of the pressure-force Schur solve (sim_solve_schur) and of one time
step (sim_step) with the CPU oracle, plus determinism and error paths."""
import numpy as np
import pytest

from oracle import bodies as obd
from oracle import mac as omac
from oracle import step as ostep
from paper_2501_15314_amd import workloads as wl

from .conftest import gpu_available
from .gpu_helpers import (CHUNKS, freeslip_workload, make_sim, mixed_workload, odd_tiles_workload, oracle_for, rel,
                          walls_workload)

pytestmark = pytest.mark.gpu

if gpu_available():
    from paper_2501_15314_amd.sim import Sim, SimError


CASES = {
    "c1_periodic": lambda: wl.make_c1(n=32, n_points=300),
    "walls": lambda: walls_workload(32, 260),
    "mixed": mixed_workload,
    "c1_48_roma": lambda: _roma(wl.make_c1(n=48, n_points=700)),
    "freeslip": freeslip_workload,
    "odd_tiles": odd_tiles_workload,
}


def _roma(w):
    w.cfg.delta = wl.DELTA_ROMA3
    w.cfg.lump_c = wl.lump_constant(wl.DELTA_ROMA3, w.cfg.h, w.n_points, w.bodies[0].radius)
    return w


@pytest.mark.parametrize("chunks", CHUNKS)
@pytest.mark.parametrize("case", list(CASES))
@pytest.mark.parametrize("prec", [wl.PREC_FP64, wl.PREC_FP32MG])
@pytest.mark.parametrize("precond", [wl.PRECOND_VCYCLE, wl.PRECOND_FASTDIAG])
def test_schur_solve_matches_oracle(case, prec, precond, chunks):
    if case == "odd_tiles" and precond == wl.PRECOND_FASTDIAG:
        pytest.skip("the bfloat16 fast diagonalisation takes axis sizes that are multiples of 8")
    w = CASES[case]()
    w.cfg.precision = prec
    w.cfg.precond = precond
    w.cfg.krylov_rtol = 1e-12 if prec == wl.PREC_FP64 else 1e-11
    print(f"case {case} prec {prec} precond {precond} chunks {chunks} n={w.cfg.n} K={w.n_points}", flush=True)
    sim = make_sim(w.cfg, w.n_points, chunks)
    sim.set_bodies(w.bodies, w.offsets)
    g, X, W, S = oracle_for(w)
    rp, rf = wl.random_schur_rhs(21, g.n, w.n_points)
    p, phi, st = sim.solve_schur(rp, rf)
    p_ref, phi_ref, its, _ = S.solve(rp, rf, rtol=1e-13)
    ep = rel(p.cpu().numpy(), p_ref)
    ef = rel(phi.cpu().numpy(), phi_ref)
    print(f"  iters gpu={st.iters} oracle={its} rel_res={st.rel_res:.2e} err p={ep:.2e} phi={ef:.2e}")
    tol = 1e-10 if prec == wl.PREC_FP64 else 1e-8
    assert ep < tol and ef < tol
    assert st.rel_res <= w.cfg.krylov_rtol
    assert abs(p.cpu().numpy().mean()) < 1e-12 * np.abs(p_ref).max()
    sim.close()


@pytest.mark.parametrize("case", ["c1_periodic", "walls", "mixed"])
@pytest.mark.parametrize("prec", [wl.PREC_FP64, wl.PREC_FP32MG])
@pytest.mark.parametrize("precond", [wl.PRECOND_VCYCLE, wl.PRECOND_FASTDIAG])
def test_schur_bicgstab_matches_oracle(case, prec, precond):
    """BiCGStab (the paper's Krylov method) reaches the same unique mean-zero
    solution as the oracle's BiCGStab with the exact L^+."""
    w = CASES[case]()
    w.cfg.precision = prec
    w.cfg.precond = precond
    w.cfg.krylov = wl.KRYLOV_BICGSTAB
    w.cfg.krylov_rtol = 1e-12 if prec == wl.PREC_FP64 else 1e-11
    print(f"case {case} prec {prec} precond {precond} bicgstab n={w.cfg.n} K={w.n_points}", flush=True)
    sim = Sim(w.cfg, w.n_points)
    sim.set_bodies(w.bodies, w.offsets)
    g, X, W, S = oracle_for(w)
    rp, rf = wl.random_schur_rhs(24, g.n, w.n_points)
    p, phi, st = sim.solve_schur(rp, rf)
    p_ref, phi_ref, its, _ = S.solve(rp, rf, rtol=1e-13, method="bicgstab")
    ep = rel(p.cpu().numpy(), p_ref)
    ef = rel(phi.cpu().numpy(), phi_ref)
    print(f"  iters gpu={st.iters} oracle={its} rel_res={st.rel_res:.2e} err p={ep:.2e} phi={ef:.2e}")
    tol = 1e-10 if prec == wl.PREC_FP64 else 1e-8
    assert ep < tol and ef < tol
    assert st.rel_res <= w.cfg.krylov_rtol
    sim.close()


@pytest.mark.parametrize("prec", [wl.PREC_FP64, wl.PREC_FP32MG])
def test_constant_in_pressure_rhs_is_projected_out(prec):
    """S~ annihilates the constants (L and B^T B both do: Sec. 4.1), so the
    solve takes RHS_p to mean zero (inside the pass that starts each Krylov
    cycle) and returns a mean-free p': a large constant added to RHS_p must
    leave p' and Phi' as they are."""
    w = walls_workload(32, 260)
    w.cfg.precision = prec
    w.cfg.krylov_rtol = 1e-12 if prec == wl.PREC_FP64 else 1e-11
    sim = Sim(w.cfg, w.n_points)
    sim.set_bodies(w.bodies, w.offsets)
    rp, rf = wl.random_schur_rhs(23, w.cfg.n, w.n_points)
    p1, f1, _ = sim.solve_schur(rp, rf)
    p2, f2, _ = sim.solve_schur(rp + 7.0, rf)
    p1, p2, f1, f2 = (t.cpu().numpy() for t in (p1, p2, f1, f2))
    tol = 1e-10 if prec == wl.PREC_FP64 else 1e-8
    print(f"  prec {prec}: shift changes p' by {rel(p2, p1):.1e}, Phi' by {rel(f2, f1):.1e}", flush=True)
    assert rel(p2, p1) < tol and rel(f2, f1) < tol
    assert abs(p2.mean()) < 1e-12 * np.abs(p1).max()
    sim.close()


def test_schur_solve_bitwise_repeatable():
    w = walls_workload(32, 260)
    w.cfg.precision = wl.PREC_FP32MG
    w.cfg.krylov_rtol = 1e-10
    sim = Sim(w.cfg, w.n_points)
    sim.set_bodies(w.bodies, w.offsets)
    rp, rf = wl.random_schur_rhs(22, w.cfg.n, w.n_points)
    p1, f1, _ = sim.solve_schur(rp, rf)
    p2, f2, _ = sim.solve_schur(rp, rf)
    assert np.array_equal(p1.cpu().numpy(), p2.cpu().numpy())
    assert np.array_equal(f1.cpu().numpy(), f2.cpu().numpy())
    sim.close()


@pytest.mark.parametrize("prec", [wl.PREC_FP64, wl.PREC_FP32MG])
def test_zero_and_constant_rhs_give_zero_solution(prec):
    """b = 0 (or a constant RHS_p, whose projection is 0) has the solution
    p' = 0 and, with RHS_F = 0, Phi' = 0; the solve returns it without an
    iteration.  Run twice on one handle, after a nonzero solve, so nothing
    of the earlier solution survives in the outputs."""
    w = walls_workload(32, 260)
    w.cfg.precision = prec
    sim = Sim(w.cfg, w.n_points)
    sim.set_bodies(w.bodies, w.offsets)
    rp, rf = wl.random_schur_rhs(24, w.cfg.n, w.n_points)
    sim.solve_schur(rp, rf)
    for const in (0.0, 3.0):
        p, phi, st = sim.solve_schur(np.full(w.cfg.n, const), np.zeros((w.n_points, 3)))
        p, phi = p.cpu().numpy(), phi.cpu().numpy()
        print(f"  prec {prec} RHS_p = {const}: iters {st.iters}, max |p'| {np.abs(p).max():.1e}, "
              f"max |Phi'| {np.abs(phi).max():.1e}", flush=True)
        assert st.iters == 0
        assert np.abs(p).max() <= 1e-12 * max(const, 1.0) and np.abs(phi).max() <= 1e-12 * max(const, 1.0)
    sim.close()


def test_unaligned_caller_buffers_give_the_same_solve():
    """The boundary takes any 8-byte aligned device pointers: RHS_p and p'
    one double past a 16-byte boundary take the per-cell layout conversions
    instead of the paired ones, with the same values bit for bit."""
    import ctypes as C
    import torch
    from paper_2501_15314_amd import _lib
    w = walls_workload(32, 260)
    w.cfg.precision = wl.PREC_FP32MG
    sim = Sim(w.cfg, w.n_points)
    sim.set_bodies(w.bodies, w.offsets)
    rp, rf = wl.random_schur_rhs(25, w.cfg.n, w.n_points)
    p1, f1, _ = sim.solve_schur(rp, rf)
    n = int(np.prod(w.cfg.n))
    rbuf = torch.zeros(n + 1, dtype=torch.float64, device=sim.dev)
    rbuf[1:] = torch.as_tensor(rp.ravel(), device=sim.dev)
    pbuf = torch.zeros(n + 1, dtype=torch.float64, device=sim.dev)
    rft = torch.as_tensor(rf, dtype=torch.float64, device=sim.dev).contiguous()
    phi = torch.empty((w.n_points, 3), dtype=torch.float64, device=sim.dev)
    assert (rbuf[1:].data_ptr() % 16, pbuf[1:].data_ptr() % 16) == (8, 8)
    st = _lib.SolveStats()
    rc = sim.lib.sim_solve_schur(sim.h, C.c_void_p(rbuf[1:].data_ptr()), C.c_void_p(rft.data_ptr()),
                                 C.c_void_p(pbuf[1:].data_ptr()), C.c_void_p(phi.data_ptr()), C.byref(st))
    torch.cuda.synchronize()
    assert rc == 0
    assert np.array_equal(pbuf[1:].cpu().numpy(), p1.cpu().numpy().ravel())
    assert np.array_equal(phi.cpu().numpy(), f1.cpu().numpy())
    sim.close()


def test_notconv_reports_best_iterate():
    w = wl.make_c1(n=32, n_points=300)
    w.cfg.krylov_maxit = 1
    w.cfg.krylov_rtol = 1e-14
    sim = Sim(w.cfg, w.n_points)
    sim.set_bodies(w.bodies, w.offsets)
    rp, rf = wl.random_schur_rhs(23, w.cfg.n, w.n_points)
    with pytest.raises(SimError) as e:
        sim.solve_schur(rp, rf)
    assert "ENOTCONV" in str(e.value)
    p, phi, st = sim.solve_schur(rp, rf, allow_notconv=True)
    assert st.iters == 1 and 0 < st.rel_res < 1
    sim.close()


def test_restart_at_its_maximum_runs_a_full_cycle():
    """krylov_restart = 64, the largest the header allows: with a tolerance
    out of reach the iteration cap ends the first cycle after all 64 Arnoldi
    steps (the last one forms the 65th basis scale), and the iterate still
    matches the oracle's solution."""
    w = wl.make_c1(n=32, n_points=300)
    w.cfg.krylov_restart = 64
    w.cfg.krylov_maxit = 64
    w.cfg.krylov_rtol = 1e-300
    sim = Sim(w.cfg, w.n_points)
    sim.set_bodies(w.bodies, w.offsets)
    g, X, W, S = oracle_for(w)
    rp, rf = wl.random_schur_rhs(26, g.n, w.n_points)
    p, phi, st = sim.solve_schur(rp, rf, allow_notconv=True)
    p_ref, phi_ref, _, _ = S.solve(rp, rf, rtol=1e-13)
    ep, ef = rel(p.cpu().numpy(), p_ref), rel(phi.cpu().numpy(), phi_ref)
    print(f"  iters {st.iters} rel_res {st.rel_res:.2e} err p={ep:.2e} phi={ef:.2e}")
    assert st.iters == 64 and st.nhist == 64
    assert st.rel_res < 1e-12 and ep < 1e-10 and ef < 1e-10
    sim.close()


def test_nonfinite_rhs_rejected():
    w = wl.make_c1(n=32, n_points=300)
    sim = Sim(w.cfg, w.n_points)
    sim.set_bodies(w.bodies, w.offsets)
    rp, rf = wl.random_schur_rhs(24, w.cfg.n, w.n_points)
    rp[3, 4, 5] = np.nan
    with pytest.raises(SimError) as e:
        sim.solve_schur(rp, rf)
    assert "ENONFINITE" in str(e.value)
    sim.close()


@pytest.mark.parametrize("field,value", [("precond", 7), ("krylov", 5), ("n", (20, 20, 20))])
def test_bad_solver_options_rejected(field, value):
    """Unknown preconditioner or Krylov codes, and a fast-diagonalisation grid
    whose sizes are not multiples of 8 (one multigrid level, so that only that
    rule applies), are refused at creation."""
    w = wl.make_c1(n=32, n_points=300)
    cfg = w.cfg
    if field == "n":
        cfg.n, cfg.length, cfg.precond, cfg.mg_coarsest = value, (1.0, 1.0, 1.0), wl.PRECOND_FASTDIAG, 32
    else:
        setattr(cfg, field, value)
    with pytest.raises(SimError) as e:
        Sim(cfg, w.n_points)
    assert "EINVAL" in str(e.value)


def test_bicgstab_notconv_reports_best_iterate():
    w = wl.make_c1(n=32, n_points=300)
    w.cfg.krylov = wl.KRYLOV_BICGSTAB
    w.cfg.krylov_maxit = 1
    w.cfg.krylov_rtol = 1e-14
    sim = Sim(w.cfg, w.n_points)
    sim.set_bodies(w.bodies, w.offsets)
    rp, rf = wl.random_schur_rhs(25, w.cfg.n, w.n_points)
    with pytest.raises(SimError) as e:
        sim.solve_schur(rp, rf)
    assert "ENOTCONV" in str(e.value)
    p, phi, st = sim.solve_schur(rp, rf, allow_notconv=True)
    assert st.iters == 1 and 0 < st.rel_res < 1
    sim.close()


@pytest.mark.parametrize("bc", [wl.BC_NOSLIP, wl.BC_FREESLIP])
def test_support_crossing_wall_rejected(bc):
    w = walls_workload(32, 260)
    w.cfg.bc = (bc,) * 3
    w.bodies[0].center = np.array([0.07, 0.5, 0.5])
    sim = Sim(w.cfg, w.n_points)
    with pytest.raises(SimError) as e:
        sim.set_bodies(w.bodies, w.offsets)
    assert "EINVAL" in str(e.value)
    sim.close()


# ---------------------------------------------------------------------------
# one-way time step

def _oracle_step(w, state, t1):
    cfg = w.cfg
    g, X, W, S = oracle_for(w, t1)
    U = []
    for b in w.bodies:
        v = obd.prescribed_velocity(b.vel, b.osc_amp, b.osc_omega, t1)
        U.append(np.tile(v, (b.n_points, 1)))
    U = np.concatenate(U)
    # rotating bodies: U = v + omega x (R X~)
    k0 = 0
    for b in w.bodies:
        if np.any(b.omega):
            R = obd.prescribed_rotation(b.omega, t1)
            lever = w.offsets[k0:k0 + b.n_points] @ R.T
            U[k0:k0 + b.n_points] = obd.point_velocities(
                obd.prescribed_velocity(b.vel, b.osc_amp, b.osc_omega, t1), b.omega, lever)
        k0 += b.n_points
    return ostep.one_way_step(g, cfg.nu, cfg.dt, state, X, U, cfg.delta, cfg.lump_c, cfg.xi)


@pytest.mark.parametrize("chunks", CHUNKS)
@pytest.mark.parametrize("case", ["c1_periodic", "walls", "mixed", "freeslip", "odd_tiles"])
@pytest.mark.parametrize("prec", [wl.PREC_FP64, wl.PREC_FP32MG])
def test_one_way_steps_match_oracle(case, prec, chunks):
    w = CASES[case]()
    cfg = w.cfg
    cfg.precision = prec
    cfg.krylov_rtol = 1e-12 if prec == wl.PREC_FP64 else 1e-11
    cfg.helm_rtol = 1e-12 if prec == wl.PREC_FP64 else 1e-11
    if case in ("walls", "freeslip"):
        rng = np.random.default_rng(5)
        mask = omac.Grid(cfg.n, cfg.h, cfg.bc).face_dof_mask()
        w.u0 = rng.standard_normal(w.u0.shape) * 1e-2 * mask
    print(f"case {case} prec {prec} chunks {chunks}", flush=True)
    sim = make_sim(cfg, w.n_points, chunks)
    sim.set_workload(w)
    g = omac.Grid(cfg.n, cfg.h, cfg.bc)
    mask = g.face_dof_mask()
    state = ostep.State(w.u0 * mask, w.u0 * mask, np.zeros(g.n), np.zeros((w.n_points, 3)))
    tol = 1e-10 if prec == wl.PREC_FP64 else 1e-8
    for n in range(2):
        st, _ = sim.step(1)
        t1 = (n + 1) * cfg.dt
        state, info = _oracle_step(w, state, t1)
        u, p = sim.get_fields()
        f, ft = sim.get_forces()
        eu = rel(u.cpu().numpy(), state.u)
        ep = rel(p.cpu().numpy() - p.cpu().numpy().mean(), state.p - state.p.mean())
        ef = rel(f.cpu().numpy(), state.phi * cfg.h ** 3)
        print(f"  step {n}: helm {st.helm.iters} schur {st.schur.iters} div_rel {st.div_rel:.1e} "
              f"err u={eu:.2e} p={ep:.2e} phi={ef:.2e}")
        assert eu < tol and ep < tol and ef < tol
        assert st.div_rel < 1e-6
    sim.close()
