"""The benchmark configuration itself: the 256^3 no-slip box with 8 spheres
and 144,000 points, in both precision forms, as bench.py times it.  The
oracle cannot solve a system this large within a test, but its own sparse
operators check what the GPU returns: the true relative residual of p' under
the oracle's S~ and right-hand side (eqs. tildeSp, ApproxSchurPrimalP) must
meet the tolerance, Phi' must equal the oracle's force recovery from that p'
(eq. ApproxSchurPrimalF), and a full time step must leave a velocity field
that the oracle's divergence finds solenoidal to the solver tolerance."""
import numpy as np
import pytest

from oracle import mac as omac
from paper_2501_15314_amd import workloads as wl

from .conftest import gpu_available
from .gpu_helpers import oracle_for, rel

pytestmark = pytest.mark.gpu

if gpu_available():
    from paper_2501_15314_amd.sim import Sim


@pytest.mark.parametrize("prec", [wl.PREC_FP32MG, wl.PREC_FP64])
def test_full_size_solve_checked_by_the_oracle(prec):
    w = wl.make_c3()
    cfg = w.cfg
    cfg.precision = prec
    cfg.krylov_rtol = 1e-8
    cfg.helm_rtol = 1e-8
    K = w.n_points
    print(f"full size n={cfg.n} K={K} prec {prec}", flush=True)
    sim = Sim(cfg, K)
    sim.set_bodies(w.bodies, w.offsets)
    rp, rf = wl.random_schur_rhs(31, cfg.n, K)
    p, phi, st = sim.solve_schur(rp, rf)
    p, phi = p.cpu().numpy(), phi.cpu().numpy()
    g, X, W, S = oracle_for(w)
    b = S.rhs(rp, rf)
    res = float(np.linalg.norm(b - S.matvec(p)) / np.linalg.norm(b))
    ef = rel(phi, S.force(p, rf))
    print(f"  {st.iters} iterations: oracle residual {res:.2e} (device {st.rel_res:.2e}), force {ef:.1e}",
          flush=True)
    assert st.rel_res <= 1e-8 and res < 1.5e-8 and ef < 1e-12
    # one full time step from rest with the bodies moving
    sim.set_workload(w)
    st, _ = sim.step(1)
    u, _ = sim.get_fields()
    u = u.cpu().numpy()
    du = (omac.divergence(g) @ u.ravel()) * g.h
    ratio = float(np.linalg.norm(du) / np.linalg.norm(u))
    print(f"  step: div_rel {st.div_rel:.1e}, |h D u| / |u| = {ratio:.1e}", flush=True)
    assert st.div_rel < 1e-6 and ratio < 1e-8
    sim.close()
