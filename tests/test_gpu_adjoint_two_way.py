"""Reverse mode of the two-way step (free bodies, Sec. 3.2.1, three outer
passes) on the GPU through the C ABI (sim_step_adjoint_two_way), matched
against the oracle's two_way_step_vjp, itself pinned by central differences
of the forward step."""
import numpy as np
import pytest

from oracle import adjoint as oadj
from oracle import mac as omac
from oracle import step as ostep
from paper_2501_15314_amd import workloads as wl

from .conftest import gpu_available
from .gpu_helpers import free_workload, oracle_free_bodies, rel

pytestmark = pytest.mark.gpu

if gpu_available():
    from paper_2501_15314_amd.sim import Sim, SimError


@pytest.mark.parametrize("bc", [wl.BC_PERIODIC, wl.BC_NOSLIP, wl.BC_FREESLIP])
@pytest.mark.parametrize("prec", [wl.PREC_FP64, wl.PREC_FP32MG])
def test_two_way_adjoint_matches_oracle(bc, prec):
    w = free_workload(32, bc, precision=prec)
    cfg = w.cfg
    cfg.record_two_way = 1
    print(f"two-way adjoint bc {bc} prec {prec} n={cfg.n} K={w.n_points}", flush=True)
    g = omac.Grid(cfg.n, cfg.h, cfg.bc)
    mask = g.face_dof_mask()
    rng = np.random.default_rng(23)
    K = w.n_points
    gu = rng.standard_normal((3,) + g.n) * mask
    gp = rng.standard_normal(g.n)
    gphi = rng.standard_normal((K, 3))
    gbod = [dict(xc=rng.standard_normal(3), us=rng.standard_normal(3), w=rng.standard_normal(3),
                 I=rng.standard_normal(3), J=rng.standard_normal(3)) for _ in w.bodies]
    sim = Sim(cfg, K)
    sim.set_workload(w)
    sim.step(1)
    res = sim.step_adjoint_two_way(gu, gp, gphi, gbod)
    state = ostep.State(w.u0 * mask, w.u0 * mask, np.zeros(g.n), np.zeros((K, 3)))
    fb = oracle_free_bodies(w)
    ostep.init_volume_history(g, state.u, fb)
    ref, _, _, _ = oadj.two_way_step_vjp(g, cfg.nu, cfg.dt, np.array(cfg.g), state, fb, cfg.delta, cfg.lump_c,
                                         cfg.xi, cfg.outer_iters, gu, gp, gphi, gbod)
    tol = 1e-8 if prec == wl.PREC_FP64 else 1e-6
    errs = dict(u=rel(res["gu"].cpu().numpy(), ref["u"]), um=rel(res["gum"].cpu().numpy(), ref["um"]),
                p=rel(res["gp"].cpu().numpy(), ref["p"]), phi=rel(res["gphi"].cpu().numpy(), ref["phi"]))
    for i in range(len(w.bodies)):
        for key in Sim.BODY_IN:
            errs[f"b{i}.{key}"] = rel(res["bodies"][i][key], ref["bodies"][i][key])
    print("  " + " ".join(f"{k}={v:.1e}" for k, v in errs.items()), flush=True)
    for k, v in errs.items():
        assert v < tol, (k, v)
    sim.close()


def test_two_way_adjoint_needs_a_recorded_step():
    w = free_workload(32, wl.BC_PERIODIC)
    sim = Sim(w.cfg, w.n_points)            # record_two_way = 0
    sim.set_workload(w)
    sim.step(1)
    with pytest.raises(SimError, match="ESTATE"):
        sim.step_adjoint_two_way()
    sim.close()
    w.cfg.record_two_way = 1
    w.cfg.outer_tol = 1e-3                  # early stop: the pass count is not fixed
    sim = Sim(w.cfg, w.n_points)
    sim.set_workload(w)
    sim.step(1, allow_notconv=True)
    with pytest.raises(SimError, match="ESTATE"):
        sim.step_adjoint_two_way()
    sim.close()
