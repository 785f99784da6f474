#!/usr/bin/env python3
"""Throughput benchmark of the coupled IB pressure-force Schur solve on one MI355X.

Unit of work (one timed step): one sim_solve_schur -- the lumped Schur solve
S~ p' = b (FGMRES right-preconditioned by one V-cycle per iteration) plus
the force recovery Phi' (paper Sec. 4.1) -- in the FP32-preconditioned form,
on the right-hand side of the first time step of the 256^3 workload: a
no-slip box, eight spheres of radius 0.06 with seeded constant velocities
and 18,000 Lagrangian points each (144,000 points), nu = 0.005, dt = 0.002,
fluid at rest.  From rest the momentum predictor gives u* = 0, so the
first step's system is RHS_p = -D u*/tau = 0 and RHS_F = (W^T u* - U)/tau =
-U/tau with the points at t = dt.  Inputs are resident in HBM before the
timed region; value = Schur solves per second at the Krylov tolerance that
keeps the solution within 1e-8 of the oracle's (METRIC_RTOL).

Printed: one JSON line with the solve rate of the FP32-MG form (value) and
of the FP64 form, both forms' relative L2 error against the FP64 CPU
oracle's own solution of the same 256^3 system (GMRES to 1e-13 with its
exact L^+), the roofline of the dominant kernel of the solve (HIP events and
algorithmic bytes of every launch of that kernel inside the timed region),
the whole preconditioner application as an aggregate, the per-kernel table
of an untimed instrumented pass, solver variants, whole time steps of the
workloads at 128^3, 256^3 and 384^3, and the CPU oracle baseline rows.
"""
import argparse
import hashlib
import json
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0   # MI355X HBM3E peak
# Krylov tolerance of the metric's solves: the largest relative residual at
# which both forms' p' and Phi' stay within 1e-8 of the oracle's solution
# (the relative error runs about twice the relative residual here), and the
# tolerance of the FP64 row held to the 1e-10 accuracy of the FP64 form
METRIC_RTOL = 3e-9
FP64_ACCURATE_RTOL = 3e-11
PROBED_SOLVES = 2       # timed solves (the last ones) whose dominant-kernel launches carry HIP events
SINGLE_KERNEL_CLASSES = ("smooth", "smooth_first", "restrict", "prolong", "coarse", "laplacian",
                         "spread_div", "interp_grad", "multidot", "update_norm")


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def sources_digest(srcs):
    """sha256 over the concatenated bytes of the given repository files."""
    h = hashlib.sha256()
    for src in srcs:
        with open(os.path.join(ROOT, src), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def traffic_record(kernel):
    """Counter-measured HBM bytes per launch from profiles/, if they were
    taken on the current kernel source (matching source hash)."""
    path = os.path.join(ROOT, "profiles", "traffic_counters.txt")
    if not os.path.exists(path):
        return None
    rec = {}
    for line in open(path):
        line = line.strip()
        if not line or line.startswith("#") or "=" not in line:
            continue
        k, v = line.split("=", 1)
        rec[k.strip()] = v.strip()
    if rec.get("kernel") != kernel:
        return None
    srcs = [x.strip() for x in rec.get("source", "").split(",") if x.strip()]
    if not srcs or rec.get("source_sha256") != sources_digest(srcs):
        return None
    try:
        return float(rec["bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or "unknown"


def first_step(w):
    """The workload with its bodies moved to their positions at t = dt, and
    the first step's Schur right-hand side (RHS_p = 0, RHS_F = -U / tau)."""
    import copy
    import numpy as np
    w1 = copy.deepcopy(w)
    dt = w.cfg.dt
    for b in w1.bodies:
        b.center = b.center + b.vel * dt - b.osc_amp * np.cos(b.osc_omega * dt)
        b.osc_amp = np.zeros(3)
        assert not np.any(b.omega), "the benchmark bodies do not rotate"
    U = np.concatenate([np.tile(b.vel, (b.n_points, 1)) for b in w.bodies])
    tau = 2.0 * dt / 3.0
    return w1, np.zeros(w.cfg.n), -U / tau


def oracle_points(w):
    import numpy as np
    out, k0 = [], 0
    for b in w.bodies:
        out.append(b.center - b.osc_amp + w.offsets[k0:k0 + b.n_points])
        k0 += b.n_points
    return np.concatenate(out)


def oracle_solve(w, rp, rf, workers, rtol=1e-13):
    """The FP64 oracle's own Schur solve (sparse S~, GMRES preconditioned by
    the exact L^+ by FFT/DCT): returns (p', Phi', iterations, seconds of
    the solve, seconds of the operator assembly)."""
    import scipy.fft
    from oracle import delta, mac, schur
    cfg = w.cfg
    t0 = time.perf_counter()
    g = mac.Grid(cfg.n, cfg.h, cfg.bc)
    S = schur.SchurSystem(g, delta.regularization_matrix(g, oracle_points(w), cfg.delta), cfg.lump_c)
    t1 = time.perf_counter()
    with scipy.fft.set_workers(workers):
        p, phi, its, _ = S.solve(rp, rf, rtol=rtol, workers=workers)
    t2 = time.perf_counter()
    return p, phi, its, t2 - t1, t1 - t0


def cpu_rows(make_first, workers_all):
    """Full oracle Schur solves of the first-step system at 32^3 and 128^3,
    on one core and on all cores."""
    rows = []
    for n in (32, 128):
        w1, rp, rf = make_first(n)
        for workers in (1, workers_all):
            p, phi, its, ts, ta = oracle_solve(w1, rp, rf, workers)
            rows.append({"grid": n, "cores": workers, "iters_to_1e-13": its, "solve_s": round(ts, 3),
                         "assembly_s": round(ta, 3), "solves_per_s": round(1.0 / ts, 4)})
            log(f"oracle {n}^3 on {workers} core(s): {its} iterations, {ts:.2f} s")
    return rows


def rel(a, b):
    import numpy as np
    nb = float(np.linalg.norm(b))
    return float(np.linalg.norm(a - b) / (nb if nb > 0 else 1.0))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20, help="timed Schur solves")
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--n", type=int, default=256)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle (errors and baseline)")
    ap.add_argument("--no-fp64", action="store_true", help="skip the FP64-form solve rate")
    ap.add_argument("--no-variants", action="store_true",
                    help="skip the solver variants (fast-diagonalisation preconditioner, BiCGStab)")
    ap.add_argument("--no-steps", action="store_true",
                    help="skip the whole-time-step timings (128^3, 256^3, 384^3 two-way)")
    ap.add_argument("--step-workloads", default="c3,c2,c5",
                    help="comma-separated whole-time-step timings to run (c3: 256^3, c2: 128^3 oscillating "
                         "sphere, c5: 384^3 two-way)")
    ap.add_argument("--c5-steps", type=int, default=100, help="timed two-way steps at 384^3")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 1 GiB device-to-device copy three times (the reference "
                         "kernel for scaling HBM byte counters) and exit")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (the solver runs on a single MI355X); "
              f"--gpus {args.gpus} is not supported", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    if args.copy_calibration:
        nbytes = 1 << 30
        a = torch.empty(nbytes // 8, dtype=torch.float64, device="cuda").fill_(1.0)
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": nbytes, "copy_bytes_written": nbytes, "launches": 3}), flush=True)
        return
    from paper_2501_15314_amd import _lib
    from paper_2501_15314_amd import workloads as wl
    from paper_2501_15314_amd.sim import Sim

    n = args.n
    pps = int(round(18000 * (n / 256) ** 2))

    def make_first(nn):
        return first_step(wl.make_c3(n=nn, points_per_sphere=int(round(18000 * (nn / 256) ** 2))))

    w1, rp, rf = make_first(n)
    K = w1.n_points
    N = int(np.prod(w1.cfg.n))
    rpt = torch.as_tensor(rp, device="cuda")
    rft = torch.as_tensor(rf, device="cuda")

    def make_sim(prec, precond=wl.PRECOND_VCYCLE, krylov=wl.KRYLOV_FGMRES, rtol=METRIC_RTOL):
        cfg = wl.make_c3(n=n, points_per_sphere=pps).cfg
        cfg.precision, cfg.precond, cfg.krylov, cfg.krylov_rtol = prec, precond, krylov, rtol
        s = Sim(cfg, K)
        s.set_bodies(w1.bodies, w1.offsets)
        return s

    log(f"workload c3 first-step system n={n} K={K} steps={args.steps} warmup={args.warmup}")
    sim = make_sim(wl.PREC_FP32MG)
    for _ in range(args.warmup):
        sim.solve_schur(rpt, rft)
    # untimed instrumented pass: every kernel class probed (HIP events and
    # algorithmic bytes of every launch) over three solves
    probes = list(_lib.PROBES)
    for p in probes:
        sim.probe(p, True)
        sim.probe_read(p, reset=True)
    for _ in range(3):
        sim.solve_schur(rpt, rft)
    kern = {}
    for p in probes:
        cnt, ms, nb = sim.probe_read(p, reset=True)
        sim.probe(p, False)
        if cnt:
            kern[p] = (cnt, ms, nb)
    singles = {k: v for k, v in kern.items() if k in SINGLE_KERNEL_CLASSES}
    dom = max(singles, key=lambda k: singles[k][1]) if singles else None
    probed = ([dom] if dom else []) + ["vcycle"]
    for p in probed:
        sim.probe_read(p, reset=True)
    # timed region: K solves; in the last PROBED_SOLVES of them the launches
    # of the dominant kernel and every preconditioner application are
    # bracketed by HIP events on the solver's stream (the events cost about
    # a microsecond per launch, so the other solves run without them)
    its = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        if k == max(args.steps - PROBED_SOLVES, 0):
            for p in probed:
                sim.probe(p, True)
        p32, phi32, st = sim.solve_schur(rpt, rft)
        its.append(st.iters)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    dom_timed = sim.probe_read(dom, reset=True) if dom else None
    vc_timed = sim.probe_read("vcycle", reset=True)
    for p in ([dom] if dom else []) + ["vcycle"]:
        sim.probe(p, False)
    res32 = st.rel_res
    p32, phi32 = p32.cpu().numpy(), phi32.cpu().numpy()
    sim.close()
    del sim
    torch.cuda.empty_cache()
    log(f"{args.steps} FP32-MG solves in {elapsed:.3f} s ({its[-1]} iterations each)")

    def solve_rate(s, reps=5):
        s.solve_schur(rpt, rft)
        torch.cuda.synchronize()
        a = time.perf_counter()
        for _ in range(reps):
            p, phi, st2 = s.solve_schur(rpt, rft)
        torch.cuda.synchronize()
        t = (time.perf_counter() - a) / reps  # before the copies to the host below
        return p.cpu().numpy(), phi.cpu().numpy(), t, st2

    forms = {}
    gp, gphi = {"fp32mg": p32, }, {"fp32mg": phi32}
    forms["fp32mg"] = {"solves_per_s": round(args.steps / elapsed, 2), "ms": round(1e3 * elapsed / args.steps, 3),
                       "iters": its[-1], "krylov_rtol": METRIC_RTOL, "rel_res": res32,
                       "cell_updates_per_s": round(N * its[-1] * args.steps / elapsed, 1)}
    variants = [("fp64", wl.PREC_FP64, wl.PRECOND_VCYCLE, wl.KRYLOV_FGMRES, METRIC_RTOL),
                ("fp64_rtol_3e-11", wl.PREC_FP64, wl.PRECOND_VCYCLE, wl.KRYLOV_FGMRES, FP64_ACCURATE_RTOL)] \
        if not args.no_fp64 else []
    if not args.no_variants:
        variants += [("fp32mg_fgmres_fastdiag", wl.PREC_FP32MG, wl.PRECOND_FASTDIAG, wl.KRYLOV_FGMRES, METRIC_RTOL),
                     ("fp32mg_bicgstab_vcycle", wl.PREC_FP32MG, wl.PRECOND_VCYCLE, wl.KRYLOV_BICGSTAB, METRIC_RTOL),
                     ("fp64_bicgstab_vcycle", wl.PREC_FP64, wl.PRECOND_VCYCLE, wl.KRYLOV_BICGSTAB, METRIC_RTOL),
                     # the paper's own solver: BiCGStab with the exact L^-1 (float64 fast diagonalisation)
                     ("fp64_bicgstab_exact_fastdiag_rtol_1e-12", wl.PREC_FP64, wl.PRECOND_FASTDIAG_EXACT,
                      wl.KRYLOV_BICGSTAB, 1e-12)]
    for form, prec, precond, krylov, rtol in variants:
        s2 = make_sim(prec, precond, krylov, rtol)
        gp[form], gphi[form], tsol, st2 = solve_rate(s2)
        forms[form] = {"solves_per_s": round(1.0 / tsol, 2), "ms": round(1e3 * tsol, 3), "iters": st2.iters,
                       "krylov_rtol": rtol, "rel_res": st2.rel_res,
                       "cell_updates_per_s": round(N * st2.iters / tsol, 1)}
        log(f"{form}: {1e3 * tsol:.2f} ms, {st2.iters} iterations")
        s2.close()
        del s2
        torch.cuda.empty_cache()

    # random right-hand side (the paper's random-RHS experiment, Sec. 6.2)
    rrp, rrf = wl.random_schur_rhs(31, w1.cfg.n, K)
    rand_rhs = {}
    for form, prec in (("fp32mg", wl.PREC_FP32MG), ("fp64", wl.PREC_FP64)):
        if form == "fp64" and args.no_fp64:
            continue
        s2 = make_sim(prec)
        a, b = torch.as_tensor(rrp, device="cuda"), torch.as_tensor(rrf, device="cuda")
        s2.solve_schur(a, b)
        torch.cuda.synchronize()
        t = time.perf_counter()
        _, _, st2 = s2.solve_schur(a, b)
        torch.cuda.synchronize()
        rand_rhs[form] = {"ms": round(1e3 * (time.perf_counter() - t), 3), "iters": st2.iters}
        s2.close()
        del s2
        torch.cuda.empty_cache()

    # whole time steps: the 256^3 workload (one-way, both forms), the
    # oscillating sphere at 128^3 (50 steps, FP64 then FP32-MG) and the 27
    # settling spheres at 384^3 (two-way, three outer passes, FP32-MG)
    steps = {}
    if not args.no_steps:
        for tag, make, nsteps, forms_ in (("c3_256cube_8spheres", lambda: wl.make_c3(n=n, points_per_sphere=pps), 10,
                                           (wl.PREC_FP32MG, wl.PREC_FP64)),
                                          ("c2_128cube_oscillating_sphere", wl.make_c2, 50,
                                           (wl.PREC_FP64, wl.PREC_FP32MG)),
                                          ("c5_384cube_27free_spheres", wl.make_c5, args.c5_steps,
                                           (wl.PREC_FP32MG,))):
            if tag.split("_")[0] not in args.step_workloads.split(","):
                continue
            for prec in forms_:
                wt = make()
                wt.cfg.precision = prec
                if tag.startswith("c5"):
                    wt.cfg.outer_tol = 0.0      # every step runs all three passes
                fname = "fp32mg" if prec == wl.PREC_FP32MG else "fp64"
                log(f"time steps {tag} {fname} n={wt.cfg.n} K={wt.n_points}")
                st3 = Sim(wt.cfg, wt.n_points)
                st3.set_workload(wt)
                st3.step(1, allow_notconv=True)
                schur_its = []
                torch.cuda.synchronize()
                a = time.perf_counter()
                for _ in range(nsteps):
                    sst, _ = st3.step(1, allow_notconv=True)
                    schur_its.append(sst.total_schur_iters)
                torch.cuda.synchronize()
                steps[f"{tag}_{fname}"] = {"ms_per_step": round(1e3 * (time.perf_counter() - a) / nsteps, 3),
                                           "steps": nsteps, "schur_iters_per_step": float(np.mean(schur_its)),
                                           "outer_passes": int(sst.outer), "grid": list(wt.cfg.n),
                                           "points": wt.n_points, "bodies": len(wt.bodies)}
                st3.close()
                del st3, wt
                torch.cuda.empty_cache()

    # kernel table of the instrumented pass
    kinfo = {}
    for name, (cnt, ms, nb) in kern.items():
        avg_us = 1e3 * ms / cnt
        gbs = nb / (ms * 1e-3) / 1e9 if nb > 0 else None
        kinfo[name] = {"launches": cnt, "avg_us": round(avg_us, 2), "total_ms": round(ms, 3),
                       "alg_bytes_per_launch": round(nb / cnt), "alg_GBs": round(gbs, 1) if gbs else None,
                       "frac": round(gbs / HBM_PEAK_GBS, 4) if gbs else None}
    roof = None
    if dom and dom_timed and dom_timed[0]:
        cnt, ms, nb = dom_timed
        avg_s = ms * 1e-3 / cnt
        ach = nb / (ms * 1e-3) / 1e9
        roof = {"bound": "hbm", "kernel": dom, "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(ach / HBM_PEAK_GBS, 4), "traffic": traffic_record(dom),
                "alg_bytes_per_launch": round(nb / cnt), "avg_launch_us": round(avg_s * 1e6, 2), "launches": cnt}
    vagg = None
    if vc_timed and vc_timed[0]:
        cnt, ms, nb = vc_timed
        vagg = {"launches": cnt, "avg_us": round(1e3 * ms / cnt, 2), "alg_bytes_per_application": round(nb / cnt),
                "achieved_GBs": round(nb / (ms * 1e-3) / 1e9, 1),
                "frac": round(nb / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}

    cpu, errors = None, {}
    if not args.no_cpu:
        workers = len(os.sched_getaffinity(0))
        log(f"CPU oracle: the same {n}^3 system on {workers} cores")
        pref, phiref, oits, ts, ta = oracle_solve(w1, rp, rf, workers)
        log(f"oracle {n}^3: {oits} iterations, {ts:.1f} s (assembly {ta:.1f} s)")
        pm = pref - pref.mean()
        for form in gp:
            q = gp[form] - gp[form].mean()
            errors[form] = {"p_rel_err": rel(q, pm), "phi_rel_err": rel(gphi[form], phiref)}
        rows = cpu_rows(make_first, workers)
        cpu = {"value": round(1.0 / ts, 5), "unit": "Schur solves/s", "cores": workers, "kind": "oracle",
               "cpu": cpu_model(),
               "sample": f"one full FP64 NumPy/SciPy oracle solve of the same {n}^3 first-step system "
                         f"(sparse S~, GMRES to 1e-13 preconditioned by the exact L^+ by FFT/DCT: "
                         f"{oits} iterations, {ts:.1f} s; operator assembly {ta:.1f} s excluded); baseline only",
               "rows": rows}
        for form, e in errors.items():
            forms[form].update(e)

    value = args.steps / elapsed
    line = {
        "metric": "Schur solves/s & HBM-roofline % at 256^3, FP32-MG vs FP64, at 1e-8 rel err",
        "value": round(value, 3),
        "unit": "Schur solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(1e3 * elapsed / args.steps, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64+f32mg",
        "data": "synthetic",
        "config": {"workload": f"c3 first-step Schur system, {n}^3 no-slip box, 8 spheres, {K} points",
                   "grid": list(w1.cfg.n), "bodies": len(w1.bodies), "points": K, "form": "fp32mg",
                   "krylov": "fgmres(20)", "precond": "vcycle", "krylov_rtol": METRIC_RTOL, "nu": w1.cfg.nu,
                   "dt": w1.cfg.dt},
        "solves": forms,
        "random_rhs": rand_rhs,
        "time_steps": steps,
        "roofline": roof,
        "precond_aggregate": vagg,
        "kernels": kinfo,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
