"""Parity of the two-way coupled step (free bodies, Sec. 3.2.1) with the CPU
oracle: fluid state, forces and the rigid-body state after two steps with a
fixed number of outer iterations."""
import numpy as np
import pytest

from oracle import mac as omac
from oracle import step as ostep
from paper_2501_15314_amd import workloads as wl

from .conftest import gpu_available
from .gpu_helpers import CHUNKS, free_workload, make_sim, oracle_free_bodies, rel

pytestmark = pytest.mark.gpu

if gpu_available():
    from paper_2501_15314_amd.sim import Sim, SimError


def _body_err(gpu_state, bodies):
    e = 0.0
    for s, b in zip(gpu_state, bodies):
        e = max(e, np.abs(s["center"] - b.xc).max(), np.abs(s["vel"] - b.us).max() / max(np.abs(b.us).max(), 1e-3),
                np.abs(s["omega"] - b.w).max() / max(np.abs(b.w).max(), 1e-3), np.abs(s["R"] - b.R).max())
    return e


@pytest.mark.parametrize("chunks", CHUNKS)
@pytest.mark.parametrize("bc", [wl.BC_PERIODIC, wl.BC_NOSLIP, wl.BC_FREESLIP])
@pytest.mark.parametrize("prec", [wl.PREC_FP64, wl.PREC_FP32MG])
def test_two_way_steps_match_oracle(bc, prec, chunks):
    w = free_workload(32, bc, precision=prec)
    cfg = w.cfg
    print(f"two-way bc {bc} prec {prec} chunks {chunks} n={cfg.n} K={w.n_points}", flush=True)
    sim = make_sim(cfg, w.n_points, chunks)
    sim.set_workload(w)
    g = omac.Grid(cfg.n, cfg.h, cfg.bc)
    mask = g.face_dof_mask()
    state = ostep.State(w.u0 * mask, w.u0 * mask, np.zeros(g.n), np.zeros((w.n_points, 3)))
    fb = oracle_free_bodies(w)
    ostep.init_volume_history(g, state.u, fb)
    tol = 1e-10 if prec == wl.PREC_FP64 else 1e-8
    for n in range(2):
        st, _ = sim.step(1)
        state, fb, info = ostep.two_way_step(g, cfg.nu, cfg.dt, np.array(cfg.g), state, fb, cfg.delta,
                                             cfg.lump_c, cfg.xi, cfg.outer_iters)
        u, p = sim.get_fields()
        f, ft = sim.get_forces()
        bs = sim.get_body_state()
        eu = rel(u.cpu().numpy(), state.u)
        ep = rel(p.cpu().numpy() - p.cpu().numpy().mean(), state.p - state.p.mean())
        ef = rel(f.cpu().numpy(), state.phi * cfg.h ** 3)
        eb = _body_err(bs, fb)
        ec = abs(st.outer_crit - info["crit"][-1]) / info["crit"][-1]
        print(f"  step {n}: outer {st.outer} crit {st.outer_crit:.3e}/{info['crit'][-1]:.3e} "
              f"schur {st.total_schur_iters} err u={eu:.2e} p={ep:.2e} phi={ef:.2e} body={eb:.2e}",
              flush=True)
        assert st.outer == cfg.outer_iters
        assert eu < tol and ep < tol and ef < tol and eb < tol and ec < 1e3 * tol
        # per-body force and torque agree with the point forces
        Xg, _ = sim.get_points()
        assert np.allclose(Xg.cpu().numpy(), info["X"], atol=1e-12)
    sim.close()


def test_two_way_outer_tolerance_stops_early():
    w = free_workload(32, wl.BC_NOSLIP, outer_iters=12)
    w.cfg.outer_tol = 1e-1
    sim = Sim(w.cfg, w.n_points)
    sim.set_workload(w)
    st, _ = sim.step(1)
    print(f"outer {st.outer} crit {st.outer_crit:.3e}", flush=True)
    assert 1 <= st.outer < 12 and st.outer_crit < 1e-1
    sim.close()


def test_two_way_bitwise_repeatable():
    outs = []
    for _ in range(2):
        w = free_workload(32, wl.BC_PERIODIC, precision=wl.PREC_FP32MG)
        sim = Sim(w.cfg, w.n_points)
        sim.set_workload(w)
        sim.step(2)
        u, p = sim.get_fields()
        outs.append((u.cpu().numpy(), p.cpu().numpy(), np.array([list(b["vel"]) + list(b["omega"])
                                                                 for b in sim.get_body_state()])))
        sim.close()
    for a, b in zip(outs[0], outs[1]):
        assert np.array_equal(a, b)


def test_mixed_motion_rejected():
    w = free_workload(32, wl.BC_PERIODIC)
    w.bodies[1].motion = wl.MOTION_PRESCRIBED
    sim = Sim(w.cfg, w.n_points)
    with pytest.raises(SimError, match="all prescribed or all free"):
        sim.set_bodies(w.bodies, w.offsets)
    sim.close()
