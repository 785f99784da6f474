"""Operator-level parity of the HIP kernels with the CPU oracle, through the C
ABI (sim_apply).  FP64 operators must agree to rounding."""
import numpy as np
import pytest

from oracle import mac as omac
from paper_2501_15314_amd import workloads as wl

from .conftest import gpu_available
from .gpu_helpers import (CHUNKS, freeslip_workload, make_sim, mg_tile_cells, mixed_workload, odd_tiles_workload,
                          oracle_for, rel, walls_workload, wrap16_workload)

pytestmark = pytest.mark.gpu

if gpu_available():
    from paper_2501_15314_amd.sim import Sim


def _cases():
    return {
        "c1_periodic": lambda: wl.make_c1(n=32, n_points=300),
        "walls": lambda: walls_workload(32, 260),
        "mixed": mixed_workload,
        "freeslip": freeslip_workload,
        "odd_tiles": odd_tiles_workload,
        "wrap16": wrap16_workload,
    }


@pytest.fixture(scope="module", params=[(c, m) for c in ["c1_periodic", "walls", "mixed", "freeslip", "odd_tiles",
                                                                  "wrap16"]
                                        for m in CHUNKS], ids=lambda p: f"{p[0]}-{p[1]}")
def setup(request):
    case, chunks = request.param
    w = _cases()[case]()
    w.cfg.precision = wl.PREC_FP64
    print(f"case {case} chunks {chunks} n={w.cfg.n} K={w.n_points}", flush=True)
    sim = make_sim(w.cfg, w.n_points, chunks)
    sim.set_bodies(w.bodies, w.offsets)
    g, X, W, S = oracle_for(w)
    yield case, w, sim, g, X, W, S
    sim.close()


def _rand(seed, shape, mask=None):
    x = np.random.default_rng(seed).standard_normal(shape)
    return x * mask if mask is not None else x


def test_points(setup):
    _, w, sim, g, X, W, S = setup
    Xg, Ug = sim.get_points()
    assert np.abs(Xg.cpu().numpy() - X).max() < 1e-14


def test_laplacian_grad_div(setup):
    _, w, sim, g, X, W, S = setup
    p = _rand(1, g.n)
    u = _rand(2, (3,) + g.n, g.face_dof_mask())
    assert rel(sim.apply("laplacian", p).cpu().numpy(), (S.L @ p.ravel()).reshape(g.n)) < 1e-14
    assert rel(sim.apply("grad", p).cpu().numpy(), (S.G @ p.ravel()).reshape(u.shape)) < 1e-14
    assert rel(sim.apply("div", u).cpu().numpy(), (S.D @ u.ravel()).reshape(g.n)) < 1e-14


def test_helmholtz_and_convection(setup):
    _, w, sim, g, X, W, S = setup
    mask = g.face_dof_mask()
    u = _rand(3, (3,) + g.n, mask)
    A = omac.helmholtz(g, w.cfg.nu, w.cfg.dt)
    ref = (A @ u.ravel()).reshape(u.shape) * mask
    assert rel(sim.apply("helmholtz", u).cpu().numpy(), ref) < 1e-14
    ref = omac.convection(g, u)
    assert rel(sim.apply("convection", u).cpu().numpy(), ref) < 1e-13


def test_interp_spread(setup):
    _, w, sim, g, X, W, S = setup
    mask = g.face_dof_mask()
    u = _rand(4, (3,) + g.n, mask)
    f = _rand(5, (w.n_points, 3))
    gi = sim.apply("interp", u).cpu().numpy()
    assert rel(gi, (W.T @ u.ravel()).reshape(-1, 3)) < 1e-14
    gs = sim.apply("spread", f).cpu().numpy()
    assert rel(gs, (W @ f.ravel()).reshape(u.shape)) < 1e-14
    # adjoint identity <W f, u> = <f, W^T u> on the GPU operators
    assert abs(np.vdot(gs, u) - np.vdot(f, gi)) < 1e-12 * abs(np.vdot(gs, u))


def test_spread_interp_bitwise_repeatable(setup):
    _, w, sim, g, X, W, S = setup
    f = _rand(6, (w.n_points, 3))
    u = _rand(7, (3,) + g.n, g.face_dof_mask())
    a1 = sim.apply("spread", f).cpu().numpy()
    a2 = sim.apply("spread", f).cpu().numpy()
    b1 = sim.apply("interp", u).cpu().numpy()
    b2 = sim.apply("interp", u).cpu().numpy()
    assert np.array_equal(a1, a2) and np.array_equal(b1, b2)


def test_schur_operator_and_rhs(setup):
    _, w, sim, g, X, W, S = setup
    p = _rand(8, g.n)
    assert rel(sim.apply("schur", p).cpu().numpy(), S.matvec(p)) < 1e-13
    rp, rf = wl.random_schur_rhs(9, g.n, w.n_points)
    assert rel(sim.apply("schur_rhs", rp, rf).cpu().numpy(), S.rhs(rp, rf)) < 1e-13


@pytest.mark.parametrize("chunks", CHUNKS)
@pytest.mark.parametrize("prec", [wl.PREC_FP64, wl.PREC_FP32MG])
@pytest.mark.parametrize("case", ["c1_periodic", "walls", "mixed", "freeslip"])
def test_helm_solve_matches_oracle(case, prec, chunks):
    """The momentum (A-block) solve alone, A u* = rhs with
    A = 3/(2 dt) - nu Delta_h (Sec. 3.1, eq. ustar), against the oracle's
    conjugate-gradient solve on its sparse A: FP64 defect correction whose
    red-black SOR relaxations run in the precision form's type."""
    from oracle import step as ostep
    w = _cases()[case]()
    cfg = w.cfg
    cfg.precision = prec
    cfg.helm_rtol = 1e-12 if prec == wl.PREC_FP64 else 1e-11
    g = omac.Grid(cfg.n, cfg.h, cfg.bc)
    rhs = _rand(16, (3,) + g.n, g.face_dof_mask())
    ref, _ = ostep.helmholtz_solve(g, cfg.nu, cfg.dt, rhs, rtol=1e-14)
    sim = make_sim(cfg, w.n_points, chunks)
    out = sim.apply("helm_solve", rhs).cpu().numpy()
    err = rel(out, ref)
    print(f"  {case} prec {prec} chunks {chunks}: helm_solve err {err:.2e}", flush=True)
    assert err < (1e-11 if prec == wl.PREC_FP64 else 1e-10)
    sim.close()


@pytest.mark.parametrize("prec", [wl.PREC_FP64, wl.PREC_FP32MG])
@pytest.mark.parametrize("case", ["c1_periodic", "walls", "mixed", "freeslip"])
def test_full_chunks_give_the_same_operators(case, prec):
    """The 8-plane chunks of the large grids and the shorter chunks of the
    small ones compute the same values: every red-black half sweep, residual,
    restriction and prolongation updates a cell from the other colour only,
    so the V-cycle, the Laplacian, the momentum operator, the momentum solve
    and the Schur operator agree to the last bit between the two launch
    shapes."""
    w = _cases()[case]()
    w.cfg.precision = prec
    g = omac.Grid(w.cfg.n, w.cfg.h, w.cfg.bc)
    mask = g.face_dof_mask()
    b = _rand(17, g.n)
    b -= b.mean()
    u = _rand(18, (3,) + g.n, mask)
    outs = {}
    for mode in CHUNKS:
        sim = make_sim(w.cfg, w.n_points, mode)
        sim.set_bodies(w.bodies, w.offsets)
        outs[mode] = [sim.apply("precond", b).cpu().numpy(), sim.apply("laplacian", b).cpu().numpy(),
                      sim.apply("helmholtz", u).cpu().numpy(), sim.apply("helm_solve", u).cpu().numpy(),
                      sim.apply("schur", b).cpu().numpy()]
        sim.close()
    for name, a, c in zip(["precond", "laplacian", "helmholtz", "helm_solve", "schur"], outs["auto"],
                          outs["full"]):
        print(f"  {case} prec {prec} {name}: max |auto - full| = {np.abs(a - c).max():.1e}", flush=True)
        assert np.array_equal(a, c), name


@pytest.mark.parametrize("prec", [wl.PREC_FP64, wl.PREC_FP32MG])
@pytest.mark.parametrize("case", ["c1_periodic", "walls", "mixed", "freeslip", "walls64", "periodic64_v22",
                                  "freeslip64_v11", "thin64x64x16"])
def test_tile_levels_give_the_same_bits(case, prec):
    """Tile levels (a level's pre-smoothing, residual and restriction in one
    launch, its prolongation and post-smoothing in another, each 8^3 tile
    recomputing its halo) give every cell the operations of the march
    kernels in the same order: the V-cycle and a whole Schur solve agree to
    the last bit with the tile levels switched off.  The 64^3 cases tile two
    levels (64^3 and 32^3 above the 16^3 + 8^3 subcycle); V(2,2) and V(1,1)
    take the other halo widths.  The thin 64 x 64 x 16 box tiles two levels
    whose coarse grids are 4 cells deep along the periodic axis, so a tile's
    coarse block wraps across most of that axis."""
    cases = dict(_cases())
    cases["thin64x64x16"] = thin_workload
    cases["walls64"] = lambda: walls_workload(64, 260)
    cases["periodic64_v22"] = lambda: wl.make_c1(n=64, n_points=300)
    cases["freeslip64_v11"] = lambda: freeslip_workload(64, 260)
    w = cases[case]()
    w.cfg.precision = prec
    w.cfg.krylov_rtol = 1e-10
    if case == "periodic64_v22":
        w.cfg.mg_pre, w.cfg.mg_post = 2, 2
    if case == "freeslip64_v11":
        w.cfg.mg_pre, w.cfg.mg_post = 1, 1
    g = omac.Grid(w.cfg.n, w.cfg.h, w.cfg.bc)
    b = _rand(31, g.n)
    b -= b.mean()
    rp, rf = wl.random_schur_rhs(32, w.cfg.n, w.n_points)
    outs = {}
    for cells in (0, 1 << 40):
        with mg_tile_cells(cells):
            sim = Sim(w.cfg, w.n_points)
        sim.set_bodies(w.bodies, w.offsets)
        sim.probe("tile_down")
        z = sim.apply("precond", b).cpu().numpy()
        p, f, st = sim.solve_schur(rp, rf)
        ntile = sim.probe_read("tile_down")[0]
        outs[cells] = (z, p.cpu().numpy(), f.cpu().numpy(), st.iters, ntile)
        sim.close()
    (z0, p0, f0, it0, n0), (z1, p1, f1, it1, n1) = outs[0], outs[1 << 40]
    print(f"  {case} prec {prec}: tile launches {n0} / {n1}, iterations {it0} / {it1}, "
          f"max |dz| {np.abs(z1 - z0).max():.1e}, |dp| {np.abs(p1 - p0).max():.1e}", flush=True)
    assert n0 == 0 and n1 > 0
    assert np.array_equal(z0, z1)
    assert it0 == it1 and np.array_equal(p0, p1) and np.array_equal(f0, f1)


def thin_workload(seed=15):
    """A 64 x 64 x 16 box of cells of width 1/64, no-slip along x and y,
    periodic along z, one sphere."""
    rng = np.random.default_rng(seed)
    n = (64, 64, 16)
    h = 1.0 / 64
    radius = 0.07
    K = 200
    cfg = wl.Config(n=n, length=tuple(x * h for x in n), bc=(wl.BC_NOSLIP, wl.BC_NOSLIP, wl.BC_PERIODIC),
                    nu=0.02, dt=0.005, delta=wl.DELTA_PESKIN4,
                    lump_c=wl.lump_constant(wl.DELTA_PESKIN4, h, K, radius), krylov_rtol=1e-12)
    c = np.array([0.5, 0.45, 0.125]) + rng.uniform(-0.01, 0.01, 3)
    bodies = [wl.Body(center=c, vel=rng.normal(0, 0.1, 3), omega=np.zeros(3), radius=radius, n_points=K)]
    return wl.Workload("thin_64x64x16", cfg, bodies, wl.fibonacci_offsets(K, radius), np.zeros((3,) + n),
                       steps=1, seed=seed)


def test_vcycle_contracts(setup):
    """One V-cycle is a good approximate inverse of L: the residual of a
    mean-zero right-hand side drops by a large factor."""
    _, w, sim, g, X, W, S = setup
    b = _rand(10, g.n)
    b -= b.mean()
    z = sim.apply("precond", b).cpu().numpy()
    r = b - (S.L @ z.ravel()).reshape(g.n)
    assert np.linalg.norm(r) / np.linalg.norm(b) < 0.25


def test_vcycle_fp32_contracts():
    w = walls_workload(32, 260)
    w.cfg.precision = wl.PREC_FP32MG
    sim = Sim(w.cfg, w.n_points)
    g = omac.Grid(w.cfg.n, w.cfg.h, w.cfg.bc)
    L = omac.laplacian(g)
    b = _rand(11, g.n)
    b -= b.mean()
    z = sim.apply("precond", b).cpu().numpy()
    r = b - (L @ z.ravel()).reshape(g.n)
    assert np.linalg.norm(r) / np.linalg.norm(b) < 0.25
    sim.close()


@pytest.mark.parametrize("bc", [(0, 0, 0), (1, 1, 1), (1, 0, 0), (0, 1, 1)])
@pytest.mark.parametrize("prec", [wl.PREC_FP64, wl.PREC_FP32MG])
def test_exact_coarse_solve_is_pseudo_inverse(bc, prec):
    """A 16^3 grid is its own coarsest grid: the preconditioner is then the
    fast-diagonalisation solve alone and must equal L^+ (the oracle's
    FFT/DCT pseudo-inverse) to the working precision."""
    from oracle import poisson as opoisson
    n = 16
    cfg = wl.Config(n=(n, n, n), length=(1.0, 1.0, 1.0), bc=bc, precision=prec, mg_coarsest=16,
                    mg_coarse_sweeps=0)
    sim = Sim(cfg, 1)
    g = omac.Grid(cfg.n, cfg.h, cfg.bc)
    b = _rand(12, g.n)
    z = sim.apply("precond", b).cpu().numpy()
    ref = opoisson.solve_laplacian(g, b)
    err = rel(z - z.mean(), ref)
    print(f"bc {bc} prec {prec}: rel err {err:.2e}", flush=True)
    assert err < (1e-12 if prec == wl.PREC_FP64 else 1e-5)
    sim.close()


@pytest.mark.parametrize("case", ["c1_periodic", "walls", "mixed"])
def test_fastdiag_preconditioner_is_pseudo_inverse(case):
    """The whole-grid fast-diagonalisation preconditioner approximates L^+ to
    the bfloat16 rounding of its six transforms."""
    from oracle import poisson as opoisson
    w = _cases()[case]()
    w.cfg.precond = wl.PRECOND_FASTDIAG
    sim = Sim(w.cfg, w.n_points)
    g = omac.Grid(w.cfg.n, w.cfg.h, w.cfg.bc)
    b = _rand(13, g.n)
    z = sim.apply("precond", b).cpu().numpy()
    ref = opoisson.solve_laplacian(g, b)
    err = rel(z - z.mean(), ref)
    print(f"{case}: fast-diagonalisation rel err {err:.2e}", flush=True)
    assert err < 2e-2
    sim.close()


@pytest.mark.parametrize("bc", [(0, 0, 0), (1, 1, 1), (1, 0, 1)])
def test_exact_coarse_solve_on_matrix_cores(bc):
    """A 32^3 coarsest grid is too large for the single-workgroup solver, so
    the exact coarse solve runs the bfloat16 matrix-core fast diagonalisation:
    it must equal L^+ to that rounding."""
    from oracle import poisson as opoisson
    n = 32
    cfg = wl.Config(n=(n, n, n), length=(1.0, 1.0, 1.0), bc=bc, precision=wl.PREC_FP32MG, mg_coarsest=32,
                    mg_coarse_sweeps=0)
    sim = Sim(cfg, 1)
    g = omac.Grid(cfg.n, cfg.h, cfg.bc)
    b = _rand(14, g.n)
    z = sim.apply("precond", b).cpu().numpy()
    ref = opoisson.solve_laplacian(g, b)
    err = rel(z - z.mean(), ref)
    print(f"bc {bc}: matrix-core coarse solve rel err {err:.2e}", flush=True)
    assert err < 2e-2
    sim.close()


@pytest.mark.parametrize("n,bc", [((16, 24, 272), (0, 1, 1)), ((264, 16, 48), (1, 0, 1))])
def test_fastdiag_long_axis(n, bc):
    """Axes longer than 256 take the eight-tile-per-wavefront variant of the
    transform kernel; sizes not a multiple of 16 or 64 exercise the padding."""
    from oracle import poisson as opoisson
    cfg = wl.Config(n=n, length=tuple(x / 64.0 for x in n), bc=bc, precision=wl.PREC_FP32MG,
                    precond=wl.PRECOND_FASTDIAG)
    sim = Sim(cfg, 1)
    g = omac.Grid(cfg.n, cfg.h, cfg.bc)
    b = _rand(15, g.n)
    z = sim.apply("precond", b).cpu().numpy()
    ref = opoisson.solve_laplacian(g, b)
    err = rel(z - z.mean(), ref)
    print(f"n {n} bc {bc}: fast-diagonalisation rel err {err:.2e}", flush=True)
    assert err < 2e-2
    sim.close()


@pytest.mark.parametrize("n,bc", [((32, 32, 32), (0, 0, 0)), ((32, 32, 32), (1, 1, 1)), ((16, 24, 40), (1, 0, 2)),
                                  ((20, 28, 36), (0, 1, 0)), ((64, 48, 96), (1, 1, 1))])
def test_exact_fastdiag_is_pseudo_inverse(n, bc):
    """The float64 fast-diagonalisation preconditioner is the exact L^+ of
    the direct solve of Sec. 4.2 (the oracle's FFT/DCT pseudo-inverse) to
    rounding, on any axis sizes (multiples of 4 that are not multiples of
    the 64-wide transform tiles included) and every boundary kind."""
    from oracle import poisson as opoisson
    cfg = wl.Config(n=n, length=tuple(x / 32.0 for x in n), bc=bc, precision=wl.PREC_FP64,
                    precond=wl.PRECOND_FASTDIAG_EXACT)
    sim = Sim(cfg, 1)
    g = omac.Grid(cfg.n, cfg.h, cfg.bc)
    b = _rand(19, g.n)
    z = sim.apply("precond", b).cpu().numpy()
    ref = opoisson.solve_laplacian(g, b)
    err = rel(z, ref)
    print(f"n {n} bc {bc}: exact fast-diagonalisation rel err {err:.2e}, mean {z.mean():.1e}", flush=True)
    assert err < 1e-12 and abs(z.mean()) < 1e-12 * np.abs(ref).max()
    sim.close()


def test_exact_fastdiag_needs_fp64():
    cfg = wl.Config(n=(32, 32, 32), precision=wl.PREC_FP32MG, precond=wl.PRECOND_FASTDIAG_EXACT)
    with pytest.raises(Exception) as e:
        Sim(cfg, 1)
    assert "EINVAL" in str(e.value)
