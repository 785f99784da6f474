"""Reverse-mode step (sim_step_adjoint) against the oracle's transposed step,
and the dot-product identity at the full 128^3 adjoint workload."""
import numpy as np
import pytest

from oracle import adjoint as oadj
from oracle import bodies as obd
from oracle import mac as omac
from oracle import step as ostep
from paper_2501_15314_amd import workloads as wl

from .conftest import gpu_available
from .gpu_helpers import CHUNKS, freeslip_workload, make_sim, prescribed_points, rel, walls_workload

pytestmark = pytest.mark.gpu

if gpu_available():
    import torch

    from paper_2501_15314_amd.sim import Sim, SimError


def _case(name, prec):
    if name == "c4_32":
        w = wl.scaled(wl.make_c4, 32)
    else:
        w = walls_workload(32, 200) if name == "walls" else freeslip_workload(32, 200)
        w.bodies = w.bodies[:3]
        w.offsets = w.offsets[:600]
        w.bodies[1].omega = np.array([0.0, 1.5, -0.5])
    cfg = w.cfg
    cfg.precision = prec
    cfg.krylov_rtol = 1e-12 if prec == wl.PREC_FP64 else 1e-11
    cfg.helm_rtol = 1e-12 if prec == wl.PREC_FP64 else 1e-11
    cfg.xi = 0.8
    rng = np.random.default_rng(17)
    g = omac.Grid(cfg.n, cfg.h, cfg.bc)
    mask = g.face_dof_mask()
    u0 = rng.standard_normal((3,) + cfg.n) * 0.05 * mask
    um = u0 + rng.standard_normal(u0.shape) * 0.01 * mask
    p0 = rng.standard_normal(cfg.n)
    phi0 = 0.2 * rng.standard_normal((w.n_points, 3))
    ybar = (rng.standard_normal((3,) + cfg.n) * mask, rng.standard_normal(cfg.n),
            rng.standard_normal((w.n_points, 3)))
    return w, g, ostep.State(u0, um, p0, phi0), ybar


def _gpu(w, state, ybar, chunks="auto"):
    sim = make_sim(w.cfg, w.n_points, chunks)
    sim.set_bodies(w.bodies, w.offsets)
    sim.set_fields(0, state.u, state.p, state.phi)
    sim.set_fields(1, state.um)
    st, _ = sim.step(1)
    res = sim.step_adjoint(ybar[0], ybar[1], ybar[2], want_inputs=True)
    return sim, res


@pytest.mark.parametrize("chunks", CHUNKS)
@pytest.mark.parametrize("name", ["c4_32", "walls", "freeslip"])
@pytest.mark.parametrize("prec", [wl.PREC_FP64, wl.PREC_FP32MG])
def test_step_adjoint_matches_oracle(name, prec, chunks):
    w, g, state, ybar = _case(name, prec)
    cfg = w.cfg
    print(f"adjoint {name} prec {prec} chunks {chunks} n={cfg.n} K={w.n_points}", flush=True)
    sim, res = _gpu(w, state, ybar, chunks)
    X, U = prescribed_points(w, cfg.dt)
    ref, new, info = oadj.one_way_step_vjp(g, cfg.nu, cfg.dt, state, X, U, cfg.delta, cfg.lump_c, cfg.xi,
                                           ybar[0], ybar[1], ybar[2])
    tol = 1e-10 if prec == wl.PREC_FP64 else 1e-8
    errs = dict(X=rel(res["gX"].cpu().numpy(), ref["X"]),
                u=rel(res["gu"].cpu().numpy(), ref["u"]),
                um=rel(res["gum"].cpu().numpy(), ref["um"]),
                p=rel(res["gp"].cpu().numpy(), ref["p"]),
                phi=rel(res["gphi"].cpu().numpy(), ref["phi"]))
    # per-body dl/du_s and dl/domega from the point cotangents of U
    k0, gUs, gWs = 0, [], []
    for b in w.bodies:
        sl = slice(k0, k0 + b.n_points)
        R = obd.prescribed_rotation(b.omega, cfg.dt)
        lever = w.offsets[sl] @ R.T
        gUs.append(ref["U"][sl].sum(axis=0))
        gWs.append(np.cross(lever, ref["U"][sl]).sum(axis=0))
        k0 += b.n_points
    errs["U"] = rel(res["gU"], np.array(gUs))
    errs["W"] = rel(res["gW"], np.array(gWs))
    print("  " + " ".join(f"{k}={v:.2e}" for k, v in errs.items()), flush=True)
    for k, v in errs.items():
        assert v < tol, (k, v)
    # repeatable and non-destructive: a second call gives the same result
    res2 = sim.step_adjoint(ybar[0], ybar[1], ybar[2], want_inputs=True)
    assert torch.equal(res["gX"], res2["gX"]) and torch.equal(res["gu"], res2["gu"])
    # any state change invalidates the record
    sim.set_fields(1, state.um)
    with pytest.raises(SimError, match="ESTATE"):
        sim.step_adjoint(ybar[0], ybar[1], ybar[2])
    sim.close()


def _pairing(sim_out, base, ybar):
    u, p, f = sim_out
    return (float((u - base[0]).mul(ybar[0]).sum()) + float((p - base[1]).mul(ybar[1]).sum()) +
            float((f - base[2]).mul(ybar[2]).sum()))


def test_step_adjoint_dot_product_full_size():
    """128^3, two spheres of 5000 points (the adjoint workload): the step is
    affine in (u^{n-1}, p^n, Phi^n), so <ybar, step(x + xdot) - step(x)> must
    equal <J^T ybar, xdot> for each of them."""
    w = wl.make_c4()
    cfg = w.cfg
    cfg.krylov_rtol = 1e-12
    cfg.helm_rtol = 1e-12
    dev = torch.device("cuda", 0)
    gen = torch.Generator(device=dev).manual_seed(5)
    n = cfg.n
    print(f"adjoint dot product n={n} K={w.n_points}", flush=True)

    def rnd(*shape, scale=1.0):
        return torch.randn(*shape, generator=gen, device=dev, dtype=torch.float64) * scale

    u0, um, p0, phi0 = rnd(3, *n, scale=0.05), rnd(3, *n, scale=0.05), rnd(*n), rnd(w.n_points, 3, scale=0.2)
    ybar = (rnd(3, *n), rnd(*n), rnd(w.n_points, 3))
    # base step and its adjoint
    base_sim = Sim(cfg, w.n_points)
    base_sim.set_bodies(w.bodies, w.offsets)
    base_sim.set_fields(0, u0, p0, phi0)
    base_sim.set_fields(1, um)
    base_sim.step(1)
    ub, pb = base_sim.get_fields()
    fb, _ = base_sim.get_forces()
    base = (ub, pb, fb / cfg.h ** 3)
    res = base_sim.step_adjoint(*ybar, want_inputs=True)
    dirs = dict(um=rnd(3, *n), p=rnd(*n), phi=rnd(w.n_points, 3))
    for name, xd in dirs.items():
        s2 = Sim(cfg, w.n_points)
        s2.set_bodies(w.bodies, w.offsets)
        s2.set_fields(0, u0, p0 + (xd if name == "p" else 0), phi0 + (xd if name == "phi" else 0))
        s2.set_fields(1, um + (xd if name == "um" else 0))
        s2.step(1)
        u2, p2 = s2.get_fields()
        f2, _ = s2.get_forces()
        lhs = _pairing((u2, p2, f2 / cfg.h ** 3), base, ybar)
        key = dict(um="gum", p="gp", phi="gphi")[name]
        rhs = float((res[key] * xd).sum())
        print(f"  {name}: <ybar, J xdot> = {lhs:.12e}  <J^T ybar, xdot> = {rhs:.12e}", flush=True)
        assert abs(lhs - rhs) < 1e-8 * (abs(lhs) + abs(rhs))
        s2.close()
    base_sim.close()
