"""torch.autograd through the HIP step on the 128^3 adjoint workload (two
spheres of radius 0.1, 5000 points each, seeded velocities, periodic box):
a 16-step unroll whose loss is the x-drag of sphere 1, h^3 times the sum of
its points' Phi_x after the last step.  Gradients with respect to both
bodies' centres and velocities and to individual point positions come from
the hand-written transposed step (per-step checkpointing: each backward
recomputes its step from the saved inputs) and are checked by central
finite differences of the GPU forward with eps = 1e-6 on 20 seeded
coordinates."""
import numpy as np
import pytest

from paper_2501_15314_amd import workloads as wl

from .conftest import gpu_available

pytestmark = pytest.mark.gpu

if gpu_available():
    import torch

    from paper_2501_15314_amd.autograd import ib_step
    from paper_2501_15314_amd.sim import Sim

NSTEPS = 16
EPS = 1e-6


def _setup():
    w = wl.make_c4()
    cfg = w.cfg
    cfg.krylov_rtol = 1e-13
    cfg.helm_rtol = 1e-13
    sim = Sim(cfg, w.n_points)
    sim.set_bodies(w.bodies, w.offsets)
    dev = torch.device("cuda", 0)
    t = lambda a: torch.tensor(np.asarray(a), device=dev, dtype=torch.float64)
    d = dict(c0=t([b.center for b in w.bodies]), v0=t([b.vel for b in w.bodies]),
             om0=torch.zeros(2, 3, device=dev, dtype=torch.float64), off=t(w.offsets))
    return w, sim, d


def _loss(sim, c0, v0, om0, off):
    """x-drag of sphere 1 after the unroll: h^3 sum_{k in body 1} Phi_{k,x}."""
    cfg = sim.cfg
    dev = c0.device
    u = torch.zeros(3, *cfg.n, device=dev, dtype=torch.float64)
    um, p = u, torch.zeros(cfg.n, device=dev, dtype=torch.float64)
    phi = torch.zeros(off.shape[0], 3, device=dev, dtype=torch.float64)
    for s in range(NSTEPS):
        centers = c0 + (s + 1) * cfg.dt * v0
        u1, p1, phi1 = ib_step(sim, u, um, p, phi, centers, v0, om0, off)
        u, um, p, phi = u1, u, p1, phi1
    k1 = sim.bodies[0].n_points
    return cfg.h ** 3 * phi[:k1, 0].sum()


def test_unrolled_drag_gradient_matches_finite_differences():
    w, sim, d = _setup()
    args = {k: v.clone().requires_grad_(k != "om0") for k, v in d.items()}
    loss = _loss(sim, args["c0"], args["v0"], args["om0"], args["off"])
    loss.backward()
    print(f"16-step x-drag of sphere 1: {loss.item():.12e}", flush=True)
    grads = {k: v.grad.clone() for k, v in args.items() if v.grad is not None}
    rng = np.random.default_rng(20)
    K1 = w.bodies[0].n_points
    coords = [("v0", (b, a)) for b in range(2) for a in range(3)]
    coords += [("c0", (b, a)) for b in range(2) for a in range(3)]
    pts = list(rng.integers(0, K1, 4)) + list(rng.integers(K1, w.n_points, 4))
    coords += [("off", (int(k), int(a))) for k, a in zip(pts, rng.integers(0, 3, 8))]
    assert len(coords) == 20
    worst = 0.0
    with torch.no_grad():
        for name, idx in coords:
            vals = []
            for sgn in (1.0, -1.0):
                a = {k: v.clone() for k, v in d.items()}
                a[name][idx] += sgn * EPS
                vals.append(_loss(sim, a["c0"], a["v0"], a["om0"], a["off"]).item())
            fd = (vals[0] - vals[1]) / (2 * EPS)
            an = grads[name][idx].item()
            err = abs(fd - an) / max(abs(an), 1e-300)
            worst = max(worst, err)
            print(f"  {name}{idx}: autograd {an:+.10e}  fd {fd:+.10e}  rel {err:.1e}", flush=True)
            assert err < 1e-5, (name, idx, an, fd)
    print(f"worst relative error {worst:.2e}", flush=True)
    sim.close()
