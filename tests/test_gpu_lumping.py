"""The lumping C = W^T W ~ c I against the Euler / Lagrange spacing ratio
(Appendix A), on the settling sphere in its free-slip box (Sec. 6.1.3):

  * the row sums of W^T W on the device equal the oracle's, point by point,
    and sit at the paper's printed (min, max, avg) for every ratio;
  * with the paper's fixed c = 1/2, dense marker sets (ratio 2) make the time
    integration diverge within a few steps while ratio 1.33 stays stable,
    and the lumping rescaled to the marker density is stable at ratio 2 too,
    with the same Schur iteration counts and the same settling velocity."""
import os

import numpy as np
import pytest

from paper_2501_15314_amd import workloads as wl

from .conftest import gpu_available
from .gpu_helpers import oracle_for

pytestmark = pytest.mark.gpu

if gpu_available():
    import torch

    from paper_2501_15314_amd.sim import Sim, SimError


def _table(golden_dir):
    rows = []
    for line in open(os.path.join(golden_dir, "table_a1_rtr_rowsums.txt")):
        line = line.strip()
        if line and not line.startswith("#"):
            rows.append([float(x) for x in line.split()])
    return rows


def test_rtr_row_sums_on_device(golden_dir):
    for ratio, mn, mx, avg in _table(golden_dir):
        w = wl.make_sedimentation("re11", cells_per_d=16, spacing_ratio=ratio)
        sim = Sim(w.cfg, w.n_points)
        sim.set_workload(w)
        ones = torch.ones((w.n_points, 3), dtype=torch.float64, device="cuda")
        rs = sim.apply("interp", sim.apply("spread", ones)).cpu().numpy()
        g, X, W, S = oracle_for(w)
        ref = (W.T @ (W @ np.ones(3 * w.n_points))).reshape(-1, 3)
        err = np.abs(rs - ref).max() / np.abs(ref).max()
        r = rs[:, 0]
        print(f"ratio {ratio}: K={w.n_points} row sums [{r.min():.3f}, {r.max():.3f}, {r.mean():.3f}] "
              f"paper [{mn}, {mx}, {avg}] vs oracle {err:.1e}", flush=True)
        assert err < 1e-13
        assert abs(r.mean() - avg) < 0.012 * max(1.0, avg)
        assert abs(r.min() - mn) < 0.03 * max(1.0, mn) and abs(r.max() - mx) < 0.03 * max(1.0, mx)
        sim.close()


def _run(ratio, lump_c, nsteps=40):
    w = wl.make_sedimentation("re11", cells_per_d=16, spacing_ratio=ratio, lump_c=lump_c)
    print(f"ratio {ratio} c={w.cfg.lump_c:.4f} K={w.n_points}", flush=True)
    sim = Sim(w.cfg, w.n_points)
    sim.set_workload(w)
    its, vz, ok = [], 0.0, True
    try:
        for _ in range(nsteps):
            st, _ = sim.step(1, allow_notconv=True)
            its.append(st.total_schur_iters / st.outer)
            vz = float(sim.get_body_state()[0]["vel"][2])
            if not np.isfinite(vz) or abs(vz) > 10.0:
                ok = False
                break
    except SimError as e:
        assert "ENONFINITE" in str(e)
        ok = False
    sim.close()
    print(f"  {'stable' if ok else 'diverged'} after {len(its)} steps, vz {vz:+.5f}, "
          f"Schur iterations per solve {np.mean(its):.1f}", flush=True)
    return ok, vz, its


def test_fixed_lumping_breaks_down_for_dense_markers():
    ok_ref, vz_ref, its_ref = _run(1.0, None)
    ok_dense, _, _ = _run(2.0, 0.5)
    ok_mid, vz_mid, _ = _run(1.33, 0.5)
    ok_resc, vz_resc, its_resc = _run(2.0, None)
    assert ok_ref and ok_mid and ok_resc
    assert not ok_dense
    assert abs(vz_mid - vz_ref) < 0.02 * abs(vz_ref)
    assert abs(vz_resc - vz_ref) < 0.02 * abs(vz_ref)
    assert max(its_resc) <= max(its_ref) + 2
