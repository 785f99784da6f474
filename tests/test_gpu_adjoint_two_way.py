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
from .gpu_helpers import CHUNKS, free_workload, make_sim, oracle_free_bodies, rel

pytestmark = pytest.mark.gpu

if gpu_available():
    from paper_2501_15314_amd.sim import Sim, SimError


@pytest.mark.parametrize("chunks", CHUNKS)
@pytest.mark.parametrize("bc", [wl.BC_PERIODIC, wl.BC_NOSLIP, wl.BC_FREESLIP])
@pytest.mark.parametrize("prec", [wl.PREC_FP64, wl.PREC_FP32MG])
def test_two_way_adjoint_matches_oracle(bc, prec, chunks):
    w = free_workload(32, bc, precision=prec)
    cfg = w.cfg
    cfg.record_two_way = 1
    print(f"two-way adjoint bc {bc} prec {prec} chunks {chunks} n={cfg.n} K={w.n_points}", flush=True)
    g = omac.Grid(cfg.n, cfg.h, cfg.bc)
    mask = g.face_dof_mask()
    rng = np.random.default_rng(23)
    K = w.n_points
    gu = rng.standard_normal((3,) + g.n) * mask
    gp = rng.standard_normal(g.n)
    gphi = rng.standard_normal((K, 3))
    gbod = [dict(xc=rng.standard_normal(3), us=rng.standard_normal(3), w=rng.standard_normal(3),
                 I=rng.standard_normal(3), J=rng.standard_normal(3)) for _ in w.bodies]
    sim = make_sim(cfg, K, chunks)
    sim.set_workload(w)
    sim.step(1)
    res = sim.step_adjoint_two_way(gu, gp, gphi, gbod)
    state = ostep.State(w.u0 * mask, w.u0 * mask, np.zeros(g.n), np.zeros((K, 3)))
    fb = oracle_free_bodies(w)
    ostep.init_volume_history(g, state.u, fb)
    ref, _, _, _ = oadj.two_way_step_vjp(g, cfg.nu, cfg.dt, np.array(cfg.g), state, fb, cfg.delta, cfg.lump_c,
                                         cfg.xi, cfg.outer_iters, gu, gp, gphi, gbod)
    tol = 1e-10 if prec == wl.PREC_FP64 else 1e-8
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


def test_two_way_adjoint_dot_product_full_size():
    """The 27 settling spheres at 384^3 (486 000 points), three outer passes:
    with the body state fixed the two-way step is affine in (u^{n-1}, p^n,
    Phi^n), so <ybar, step(x + xdot) - step(x)> must equal <J^T ybar, xdot>
    for each of them (ybar on the fluid outputs and on the bodies' X_c, u_s,
    omega)."""
    import torch
    w = wl.make_c5()
    cfg = w.cfg
    cfg.precision = wl.PREC_FP64
    cfg.krylov_rtol = 1e-12
    cfg.helm_rtol = 1e-12
    cfg.outer_tol = 0.0
    cfg.record_two_way = 1
    dev = torch.device("cuda", 0)
    gen = torch.Generator(device=dev).manual_seed(7)
    n = cfg.n
    K = w.n_points
    print(f"two-way adjoint dot product n={n} K={K} bodies={len(w.bodies)}", flush=True)

    def rnd(*shape, scale=1.0):
        return torch.randn(*shape, generator=gen, device=dev, dtype=torch.float64) * scale

    u0, um, p0, phi0 = rnd(3, *n, scale=0.02), rnd(3, *n, scale=0.02), rnd(*n), rnd(K, 3, scale=0.2)
    ybar = (rnd(3, *n), rnd(*n), rnd(K, 3))
    rng = np.random.default_rng(8)
    gbod = [dict(xc=rng.standard_normal(3), us=rng.standard_normal(3), w=rng.standard_normal(3))
            for _ in w.bodies]

    def run(du=None, dp=None, dphi=None):
        s = Sim(cfg, K)
        s.set_bodies(w.bodies, w.offsets)
        s.set_fields(0, u0, p0 + (dp if dp is not None else 0), phi0 + (dphi if dphi is not None else 0))
        s.set_fields(1, um + (du if du is not None else 0))
        s.step(1)
        u, p = s.get_fields()
        f, _ = s.get_forces()
        bs = s.get_body_state()
        return s, (u, p, f / cfg.h ** 3, bs)

    def pairing(out, base):
        v = sum(float((a - b).mul(y).sum()) for a, b, y in zip(out[:3], base[:3], ybar))
        for bo, bb, y in zip(out[3], base[3], gbod):
            v += float(y["xc"] @ (bo["center"] - bb["center"]) + y["us"] @ (bo["vel"] - bb["vel"])
                       + y["w"] @ (bo["omega"] - bb["omega"]))
        return v

    base_sim, base = run()
    res = base_sim.step_adjoint_two_way(*ybar, gbodies=gbod)
    base_sim.close()
    dirs = dict(um=rnd(3, *n), p=rnd(*n), phi=rnd(K, 3))
    for name, xd in dirs.items():
        s2, out = run(du=xd if name == "um" else None, dp=xd if name == "p" else None,
                      dphi=xd if name == "phi" else None)
        s2.close()
        lhs = pairing(out, base)
        rhs = float((res[dict(um="gum", p="gp", phi="gphi")[name]] * xd).sum())
        print(f"  {name}: <ybar, J xdot> = {lhs:.12e}  <J^T ybar, xdot> = {rhs:.12e}", flush=True)
        assert abs(lhs - rhs) < 1e-8 * (abs(lhs) + abs(rhs))
