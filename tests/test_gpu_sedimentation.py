"""Settling sphere in a free-slip box (Sec. 6.1.3), coarse grid, two-way
coupling with three outer passes per step.  The checks are properties any
correct run has, not values of the paper's figure (which needs its far longer
runs and finer grids): the sphere starts to fall, never faster than
buoyancy-reduced free fall, stays on the centre line, each relaxed pass
removes its share of the divergence, and the outer passes stay contracting
(the force-density change of the last pass small against the force density).  Two-way steps in a
free-slip box are matched against the oracle in the two-way parity tests."""
import numpy as np
import pytest

from paper_2501_15314_amd import workloads as wl

from .conftest import gpu_available

pytestmark = pytest.mark.gpu

if gpu_available():
    from paper_2501_15314_amd.sim import Sim


@pytest.mark.parametrize("case", ["re11", "re32"])
def test_settling_sphere_coarse(case):
    w = wl.make_sedimentation(case, cells_per_d=8)
    cfg = w.cfg
    theta = w.bodies[0].density_ratio
    gmag = abs(cfg.g[2])
    print(f"sedimentation {case} n={cfg.n} K={w.n_points} theta={theta}", flush=True)
    sim = Sim(cfg, w.n_points)
    sim.set_workload(w)
    vz_prev = 0.0
    for n in range(24):
        st, _ = sim.step(1, allow_notconv=True)
        b = sim.get_body_state()[0]
        t = (n + 1) * cfg.dt
        vz = float(b["vel"][2])
        print(f"  step {n}: outer {st.outer} crit {st.outer_crit:.2e} schur {st.total_schur_iters} "
              f"vel {b['vel'][0]:+.2e} {b['vel'][1]:+.2e} {vz:+.4e} div {st.div_rel:.1e}", flush=True)
        assert st.outer == cfg.outer_iters or st.outer_crit < cfg.outer_tol
        assert st.outer_crit < 0.5
        # every pass removes the fraction xi of the divergence left
        assert st.div_rel < 1.01 * (1.0 - cfg.xi) ** st.outer + 1e-6
        # falling and accelerating from rest, never faster than free fall with
        # buoyancy (drag and added mass only slow the sphere down)
        assert vz < vz_prev
        assert -vz <= 1.02 * (1.0 - 1.0 / theta) * gmag * t
        # the box and the release point are symmetric about the vertical line
        assert max(abs(b["vel"][0]), abs(b["vel"][1])) < 0.05 * abs(vz)
        assert np.abs(b["center"][:2] - 5.0).max() < 1e-3
        vz_prev = vz
    sim.close()


@pytest.mark.parametrize("case", ["re11", "re32"])
def test_settling_velocity_reaches_the_measured_terminal_velocity(case):
    """The paper's settling figure compares with experiments at Re_p = 11.6,
    Fr = 0.237 and Re_p = 31.9, Fr = 0.334: in units of D and |g| the
    measured terminal velocity is Fr (the workload sets nu = Fr / Re_p).
    After 15 time units (1200 steps at D/h = 8; the sphere falls about 2.5 D)
    the settling velocity has nearly levelled off and must lie within 8 % of
    Fr (the paper reports 7 % between its two grids); D/h = 16 gives the same
    velocity to 1 % (measured: 0.2250 against 0.2259 at Re_p = 11.6)."""
    w = wl.make_sedimentation(case, cells_per_d=8)
    cfg = w.cfg
    fr = wl.SEDIMENTATION_CASES[case][2]
    sim = Sim(cfg, w.n_points)
    sim.set_workload(w)
    nsteps = int(round(15.0 / cfg.dt))
    vz = []
    for n in range(nsteps):
        sim.step(1, allow_notconv=True)
        if n >= nsteps - 40:
            vz.append(float(sim.get_body_state()[0]["vel"][2]))
    print(f"{case}: settling velocity {vz[-1]:+.5f} at t = 15 ({-vz[-1] / fr:.3f} of Fr = {fr})", flush=True)
    assert 0.92 * fr < -vz[-1] < 1.02 * fr
    # nearly terminal: the last 40 steps (0.5 time units) change it by under 1 %
    assert abs(vz[-1] - vz[0]) < 0.01 * abs(vz[-1])
    sim.close()
