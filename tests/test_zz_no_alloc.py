"""sim_solve_schur_noalloc (the Schur solve for callers that cannot allocate:
its work arrays in the library's static device scratch) against
sim_solve_schur on the same handle and right-hand side, through the C ABI.
Two handles in a row, the second on a smaller grid with fewer points, share
the one static array; a configuration too large for it is refused."""
import numpy as np
import pytest

from paper_2501_15314_amd import workloads as wl

from .conftest import gpu_available
from .gpu_helpers import oracle_for, rel, walls_workload

pytestmark = pytest.mark.gpu

if gpu_available():
    import torch

    from paper_2501_15314_amd.sim import Sim, SimError


@pytest.mark.parametrize("prec", [wl.PREC_FP64, wl.PREC_FP32MG])
def test_noalloc_solve_matches_solve_schur(prec):
    cases = [("walls 32^3", lambda: walls_workload(32, 260), wl.PRECOND_VCYCLE, wl.KRYLOV_FGMRES),
             ("c1 16^3", lambda: wl.make_c1(n=16, n_points=80), wl.PRECOND_VCYCLE, wl.KRYLOV_FGMRES),
             ("c1 32^3 bicgstab fastdiag", lambda: wl.make_c1(n=32, n_points=300), wl.PRECOND_FASTDIAG,
              wl.KRYLOV_BICGSTAB),
             ("c1 16^3 bicgstab", lambda: wl.make_c1(n=16, n_points=80), wl.PRECOND_VCYCLE, wl.KRYLOV_BICGSTAB)]
    for name, make, precond, krylov in cases:
        w = make()
        w.cfg.precision = prec
        w.cfg.precond = precond
        w.cfg.krylov = krylov
        w.cfg.krylov_rtol = 1e-12 if prec == wl.PREC_FP64 else 1e-11
        print(f"noalloc {name} prec {prec} n={w.cfg.n} K={w.n_points}", flush=True)
        sim = Sim(w.cfg, w.n_points)
        sim.set_bodies(w.bodies, w.offsets)
        rp, rf = wl.random_schur_rhs(41, w.cfg.n, w.n_points)
        p1, f1, s1 = sim.solve_schur(rp, rf)
        p2, f2, s2 = sim.solve_schur_noalloc(rp, rf)
        p3, f3, s3 = sim.solve_schur_noalloc(rp, rf)
        torch.cuda.synchronize()
        print(f"  iters {s1.iters} / {s2.iters} / {s3.iters}, max |dp| {float((p1 - p2).abs().max()):.1e}",
              flush=True)
        # the same kernels on other buffers: the same bits
        assert torch.equal(p1, p2) and torch.equal(f1, f2) and s1.iters == s2.iters
        assert torch.equal(p1, p3) and torch.equal(f1, f3)
        # and the oracle's solution to the parity bar
        g, X, W, S = oracle_for(w)
        p_ref, phi_ref, _, _ = S.solve(rp, rf, rtol=1e-13)
        tol = 1e-10 if prec == wl.PREC_FP64 else 1e-8
        assert rel(p2.cpu().numpy(), p_ref) < tol and rel(f2.cpu().numpy(), phi_ref) < tol
        sim.close()


def test_noalloc_refuses_a_solve_larger_than_the_scratch():
    w = wl.make_c1(n=128, n_points=300)
    w.cfg.precision = wl.PREC_FP64
    sim = Sim(w.cfg, w.n_points)
    sim.set_bodies(w.bodies, w.offsets)
    rp, rf = wl.random_schur_rhs(42, w.cfg.n, w.n_points)
    with pytest.raises(SimError) as e:
        sim.solve_schur_noalloc(rp, rf)
    assert "EINVAL" in str(e.value) and "static scratch" in str(e.value)
    # the handle still solves through its own workspace
    p, phi, st = sim.solve_schur(rp, rf)
    assert st.rel_res <= w.cfg.krylov_rtol
    sim.close()
