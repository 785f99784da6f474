"""torch.autograd through the HIP step: a 16-step unroll on the 128^3 adjoint
workload (two spheres of 5000 points), gradients checked by central finite
differences of the GPU forward on 20 seeded coordinates."""
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


def _setup():
    w = wl.make_c4()
    cfg = w.cfg
    cfg.krylov_rtol = 1e-13
    cfg.helm_rtol = 1e-13
    sim = Sim(cfg, w.n_points)
    sim.set_bodies(w.bodies, w.offsets)
    dev = torch.device("cuda", 0)
    gen = torch.Generator(device=dev).manual_seed(9)
    n = cfg.n
    wu = torch.randn(3, *n, generator=gen, device=dev, dtype=torch.float64) / np.sqrt(3 * np.prod(n))
    wp = torch.randn(*n, generator=gen, device=dev, dtype=torch.float64) / np.sqrt(np.prod(n))
    z3 = torch.zeros(3, *n, device=dev, dtype=torch.float64)
    c0 = torch.tensor(np.array([b.center for b in w.bodies]), device=dev)
    v0 = torch.tensor(np.array([b.vel for b in w.bodies]), device=dev)
    om0 = torch.tensor([[0.0, 0.0, 0.5], [0.3, 0.0, 0.0]], device=dev, dtype=torch.float64)
    phi0 = torch.zeros(w.n_points, 3, device=dev, dtype=torch.float64)
    return w, sim, dict(wu=wu, wp=wp, z3=z3, c0=c0, v0=v0, om0=om0, phi0=phi0)


def _loss(sim, d, c0, v0, om0, phi0):
    cfg = sim.cfg
    u, um = d["z3"], d["z3"]
    p = torch.zeros(cfg.n, device=d["z3"].device, dtype=torch.float64)
    phi = phi0
    for s in range(NSTEPS):
        centers = c0 + (s + 1) * cfg.dt * v0
        u1, p1, phi1 = ib_step(sim, u, um, p, phi, centers, v0, om0)
        u, um, p, phi = u1, u, p1, phi1
    return (d["wu"] * u).sum() + (d["wp"] * (p - p.mean())).sum() + 1e-3 * phi.sum()


def test_unrolled_gradient_matches_finite_differences():
    w, sim, d = _setup()
    c0 = d["c0"].clone().requires_grad_(True)
    v0 = d["v0"].clone().requires_grad_(True)
    om0 = d["om0"].clone().requires_grad_(True)
    phi0 = d["phi0"].clone().requires_grad_(True)
    loss = _loss(sim, d, c0, v0, om0, phi0)
    loss.backward()
    print(f"16-step loss {loss.item():.12e}", flush=True)
    grads = dict(c0=c0.grad.clone(), v0=v0.grad.clone(), om0=om0.grad.clone(), phi0=phi0.grad.clone())
    rng = np.random.default_rng(20)
    coords = [("c0", (b, a)) for b in range(2) for a in range(3)]
    coords += [("v0", (b, a)) for b in range(2) for a in range(3)]
    coords += [("om0", (b, a)) for b, a in [(0, 2), (1, 0), (0, 0), (1, 1)]]
    coords += [("phi0", (int(k), int(a))) for k, a in zip(rng.integers(0, w.n_points, 4), rng.integers(0, 3, 4))]
    assert len(coords) == 20
    eps = dict(c0=2e-6, v0=1e-5, om0=1e-5, phi0=2e-2)
    worst = 0.0
    with torch.no_grad():
        for name, idx in coords:
            vals = []
            for sgn in (1.0, -1.0):
                args = dict(c0=d["c0"].clone(), v0=d["v0"].clone(), om0=d["om0"].clone(), phi0=d["phi0"].clone())
                args[name][idx] += sgn * eps[name]
                vals.append(_loss(sim, d, args["c0"], args["v0"], args["om0"], args["phi0"]).item())
            fd = (vals[0] - vals[1]) / (2 * eps[name])
            an = grads[name][idx].item()
            err = abs(fd - an) / max(abs(an), 1e-12)
            worst = max(worst, err)
            print(f"  {name}{idx}: autograd {an:+.10e}  fd {fd:+.10e}  rel {err:.1e}", flush=True)
            assert err < 1e-5, (name, idx, an, fd)
    print(f"worst relative error {worst:.2e}", flush=True)
    sim.close()
