"""The unlumped primal Schur complement S_p = L + B^T (W^T W)^-1 B on the GPU
(sim_apply SCHUR_EXACT, inner conjugate gradients on W^T W) and the spectral
theorem of Sec. 5 on it: L <= S_p <= 2 L on mean-zero vectors, because
W (W^T W)^-1 W^T is an orthogonal projector.  The upper bound is probed with
generalized Rayleigh quotients (x, S_p x) / (x, L x), x from a few steps of
power iteration with the fast-diagonalisation approximation of L^+ (the
quotients themselves are exact float64 operator products), at sizes the
dense oracle check cannot reach.  The device Lanczos (sim_schur_spectrum)
is matched against the oracle's spectrum of L^+ S at small sizes and then
gives the extremes of spec(L^+ S_p) and spec(L^+ S~) on the porous arrays,
the 3-D counterpart of the paper's table of preconditioned spectra."""
import numpy as np
import pytest

import scipy.linalg as sla

from oracle import mac as omac
from oracle import schur as oschur
from paper_2501_15314_amd import workloads as wl

from .conftest import gpu_available
from .gpu_helpers import oracle_for, rel

pytestmark = pytest.mark.gpu

if gpu_available():
    import torch

    from paper_2501_15314_amd.sim import Sim


@pytest.mark.parametrize("case", ["c1_periodic", "porous_walls"])
def test_exact_schur_matches_oracle(case):
    # markers at spacing ~h on spheres of several h, so that W^T W is well
    # conditioned (the porous array: Roma kernel, radius reduced by h / 2)
    w = wl.make_c1(n=16, n_points=80) if case == "c1_periodic" else wl.make_porous(7, 16)
    sim = Sim(w.cfg, w.n_points)
    sim.set_bodies(w.bodies, w.offsets)
    g, X, W, S = oracle_for(w)
    G = omac.gradient(g)
    z = np.random.default_rng(31).standard_normal(g.n)
    z -= z.mean()
    Gz = G @ z.ravel()
    y = np.linalg.solve((W.T @ W).toarray(), W.T @ Gz)
    ref = (S.L @ z.ravel() + G.T @ (W @ y)).reshape(g.n)
    out = sim.apply("schur_exact", z).cpu().numpy()
    err = rel(out, ref)
    print(f"{case}: S_p z rel err {err:.2e}", flush=True)
    assert err < 1e-10
    sim.close()


@pytest.mark.parametrize("n_sub,cells_per_d", [(7, 16), (14, 32)])
def test_spectral_bounds_on_gpu(n_sub, cells_per_d):
    """Porous sphere arrays (64 x 64 x 96 and 128 x 128 x 192 no-slip grids):
    every Rayleigh quotient lies in [1, 2]; power iteration with the
    approximate L^+ climbs towards the top of the spectrum and never passes 2."""
    w = wl.make_porous(n_sub, cells_per_d)
    cfg = w.cfg
    n = cfg.n
    cfg.precond = wl.PRECOND_FASTDIAG
    sim = Sim(cfg, w.n_points)
    sim.set_bodies(w.bodies, w.offsets)
    dev = torch.device("cuda", 0)
    gen = torch.Generator(device=dev).manual_seed(5)

    def rq(x):
        x = x - x.mean()
        num = (x * sim.apply("schur_exact", x)).sum().item()
        den = (x * sim.apply("laplacian", x)).sum().item()
        return num / den, x

    x = torch.randn(cfg.n, generator=gen, device=dev, dtype=torch.float64)
    r0, x = rq(x)
    quotients = [r0]
    for _ in range(8):
        x = sim.apply("precond", sim.apply("schur_exact", x))
        x = x / x.norm()
        r, x = rq(x)
        quotients.append(r)
    print(f"n={n}: Rayleigh quotients {[f'{q:.6f}' for q in quotients]}", flush=True)
    assert all(1.0 - 1e-10 <= q <= 2.0 + 1e-10 for q in quotients)
    assert quotients[-1] > quotients[0]
    sim.close()


def _ritz(res):
    a, b = res["alpha"], res["beta"]
    return sla.eigvalsh_tridiagonal(a, b[1:]) if a.size > 1 else a.copy()


@pytest.mark.parametrize("case", ["c1_periodic", "porous_walls"])
@pytest.mark.parametrize("exact", [False, True])
def test_lanczos_extremes_match_oracle(case, exact):
    """Every Ritz value lies inside the oracle's spectrum of L^+ S, and the
    extreme ones reach its ends (the smallest eigenvalue is 1, on the
    pressures B annihilates)."""
    w = wl.make_c1(n=16, n_points=80) if case == "c1_periodic" else wl.make_porous(7, 8)
    sim = Sim(w.cfg, w.n_points)
    sim.set_bodies(w.bodies, w.offsets)
    g, X, W, S = oracle_for(w)
    ref = oschur.preconditioned_spectrum(S, exact)
    v0 = np.random.default_rng(41).standard_normal(g.n)
    res = sim.schur_spectrum(v0, exact=exact, steps=80, lap_rtol=1e-12)
    ritz = _ritz(res)
    lo, hi = 1.0, ref.max()
    print(f"{case} exact={exact}: steps {res['steps']} Ritz [{res['lmin']:.10f}, {res['lmax']:.10f}] "
          f"oracle [{lo:.10f}, {hi:.10f}]", flush=True)
    assert abs(res["lmin"] - ritz.min()) < 1e-12 and abs(res["lmax"] - ritz.max()) < 1e-12
    assert ritz.min() > lo - 1e-9 and ritz.max() < hi + 1e-9
    # the eigenvalue 1 has multiplicity N - 1 - 3K; the top one converges
    # to the digits the gap to its neighbours allows in 80 steps
    assert abs(res["lmin"] - lo) < 1e-6
    assert hi - res["lmax"] < 1e-4 * hi
    sim.close()


@pytest.mark.parametrize("n_sub,cells_per_d", [(7, 16), (14, 32)])
def test_lanczos_spectrum_porous(n_sub, cells_per_d):
    """Extremes of the preconditioned spectra on the porous arrays: the
    primal Schur complement stays in [1, 2] (theorem of Sec. 5) and its top
    approaches 2; the lumped operator is never below L (its top may pass 2
    slightly, as the paper observes for S~)."""
    w = wl.make_porous(n_sub, cells_per_d)
    cfg = w.cfg
    cfg.precond = wl.PRECOND_FASTDIAG
    sim = Sim(cfg, w.n_points)
    sim.set_bodies(w.bodies, w.offsets)
    v0 = np.random.default_rng(43).standard_normal(cfg.n)
    out = {}
    for exact in (True, False):
        res = sim.schur_spectrum(v0, exact=exact, steps=60, lap_rtol=1e-11)
        out[exact] = res
        print(f"porous{n_sub} n={cfg.n} K={w.n_points} exact={exact}: steps {res['steps']} "
              f"[{res['lmin']:.8f}, {res['lmax']:.8f}]", flush=True)
    assert out[True]["lmin"] > 1.0 - 1e-9 and out[True]["lmax"] < 2.0 + 1e-9
    assert out[True]["lmax"] > 1.9
    assert out[False]["lmin"] > 1.0 - 1e-9
    sim.close()
