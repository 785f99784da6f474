"""The paper-literal solver variant: the lumped Schur system of Sec. 4.1 with
the Roma 3-point kernel and c = 1/2 at marker spacing h, solved by BiCGStab
to 1e-12 preconditioned by the exact L^-1 (the direct fast-diagonalisation
solve of Sec. 4.2, here in float64 on the device), on the oscillating
sphere (Sec. 6.1.1) and the porous sphere arrays (Sec. 6.1.2).

The device's iteration counts must equal those of the oracle's own BiCGStab
with its exact FFT/DCT L^+ on the same system (to one iteration, rounding
can move the 1e-12 crossing), its solution must match the oracle's, and the
counts must stay flat from D/h = 8 to D/h = 16.  The paper's tables print
4.0-5.0 average iterations for its runs; the same method on these systems
needs 7-9 in the oracle as well (left or right preconditioning alike), so
that gap is not a property of the device code."""
import numpy as np
import pytest

from oracle import bodies as obd
from paper_2501_15314_amd import workloads as wl

from .conftest import gpu_available
from .gpu_helpers import oracle_for, rel

pytestmark = pytest.mark.gpu

if gpu_available():
    import torch

    from paper_2501_15314_amd.sim import Sim

GEOMS = {
    "sphere": lambda cpd: wl.make_oscillating_sphere(cpd),
    "porous7": lambda cpd: wl.make_porous(7, cpd),
    "porous14": lambda cpd: wl.make_porous(14, cpd),
}


def _at_time(w, t):
    """The workload with its bodies frozen at their positions at time t and
    the impulsive right-hand side of a step that starts there from rest
    (RHS_p = 0, RHS_F = -U(t) / tau)."""
    U = []
    for b in w.bodies:
        c = obd.prescribed_center(b.center, b.vel, b.osc_amp, b.osc_omega, t)
        U.append(np.tile(obd.prescribed_velocity(b.vel, b.osc_amp, b.osc_omega, t), (b.n_points, 1)))
        b.center, b.osc_amp = c, np.zeros(3)
    tau = 2.0 * w.cfg.dt / 3.0
    return np.zeros(w.cfg.n), -np.concatenate(U) / tau


@pytest.mark.parametrize("geom", list(GEOMS))
def test_paper_variant_iterations_match_oracle_and_stay_flat(geom):
    counts = {}
    for cpd in (8, 16):
        w = GEOMS[geom](cpd)
        cfg = w.cfg
        cfg.precision, cfg.precond, cfg.krylov = wl.PREC_FP64, wl.PRECOND_FASTDIAG_EXACT, wl.KRYLOV_BICGSTAB
        cfg.krylov_rtol, cfg.lump_c = 1e-12, 0.5
        rp, rf = _at_time(w, 0.3)
        sim = Sim(cfg, w.n_points)
        sim.set_bodies(w.bodies, w.offsets)
        p, phi, st = sim.solve_schur(torch.as_tensor(rp, device="cuda"), torch.as_tensor(rf, device="cuda"))
        g, X, W, S = oracle_for(w)
        p_ref, phi_ref, its, _ = S.solve(rp, rf, rtol=1e-12, method="bicgstab")
        ep, ef = rel(p.cpu().numpy(), p_ref - p_ref.mean()), rel(phi.cpu().numpy(), phi_ref)
        print(f"{geom} D/h={cpd} n={cfg.n} K={w.n_points}: BiCGStab iterations device {st.iters} "
              f"oracle {its}, rel_res {st.rel_res:.1e}, err p {ep:.1e} phi {ef:.1e}", flush=True)
        assert st.rel_res <= 1e-12
        assert abs(st.iters - its) <= 1
        assert ep < 1e-10 and ef < 1e-10
        counts[cpd] = st.iters
        sim.close()
    assert abs(counts[16] - counts[8]) <= 1, counts
