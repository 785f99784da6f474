"""CPU checks of the C ABI: the library loads, exports every function the
header declares, the ctypes structs match the C layout, and configuration
validation (sim_workspace_bytes) behaves.  No device work is launched."""
import ctypes as C
import os
import re
import subprocess
import tempfile

import pytest

from paper_2501_15314_amd import _lib
from paper_2501_15314_amd import workloads as wl

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ibschur.h")


def _lib_or_skip():
    if not os.path.exists(_lib.LIB_PATH):
        pytest.skip("library not built")
    return _lib.load()


def header_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(sim_[a-z_]+)\s*\(", src)))


def test_header_and_binding_agree():
    assert header_functions() == sorted(_lib.EXPORTS)


def test_library_exports_every_symbol():
    lib = _lib_or_skip()
    out = subprocess.run(["nm", "-D", "--defined-only", _lib.LIB_PATH], capture_output=True, text=True).stdout
    syms = set(re.findall(r" T (sim_\w+)", out))
    for name in header_functions():
        assert name in syms, name
        getattr(lib, name)


def test_struct_layouts_match_c():
    prog = r"""
#include <stdio.h>
#include <stddef.h>
#include "ibschur.h"
int main(void) {
  printf("%zu %zu %zu %zu\n", sizeof(sim_config), sizeof(sim_body), sizeof(sim_solve_stats), sizeof(sim_step_stats));
  printf("%zu %zu %zu\n", offsetof(sim_config, stream), offsetof(sim_config, xi), offsetof(sim_config, lump_c));
  printf("%zu %zu\n", offsetof(sim_body, motion), offsetof(sim_step_stats, schur));
  return 0;
}
"""
    with tempfile.TemporaryDirectory() as d:
        c = os.path.join(d, "t.c")
        exe = os.path.join(d, "t")
        open(c, "w").write(prog)
        subprocess.check_call(["gcc", "-I", os.path.join(ROOT, "include"), c, "-o", exe])
        vals = [int(x) for x in subprocess.check_output([exe]).split()]
    assert vals[:4] == [C.sizeof(_lib.SimConfig), C.sizeof(_lib.SimBody), C.sizeof(_lib.SolveStats),
                        C.sizeof(_lib.StepStats)]
    assert vals[4] == _lib.SimConfig.stream.offset
    assert vals[5] == _lib.SimConfig.xi.offset
    assert vals[6] == _lib.SimConfig.lump_c.offset
    assert vals[7] == _lib.SimBody.motion.offset
    assert vals[8] == _lib.StepStats.schur.offset


def _cfg(**kw):
    from paper_2501_15314_amd.sim import make_config
    w = wl.make_c1()
    for k, v in kw.items():
        setattr(w.cfg, k, v)
    return make_config(w.cfg, stream=0)


def test_workspace_bytes_validation():
    lib = _lib_or_skip()
    good = lib.sim_workspace_bytes(C.byref(_cfg()), 300)
    assert good > 32 ** 3 * 8 * 20
    assert lib.sim_workspace_bytes(C.byref(_cfg(lump_c=0.0)), 300) == 0
    assert lib.sim_workspace_bytes(C.byref(_cfg(n=(30, 32, 32))), 300) == 0      # not a multiple of 4
    assert lib.sim_workspace_bytes(C.byref(_cfg(length=(1.0, 2.0, 1.0))), 300) == 0  # non-cubic cells
    assert lib.sim_workspace_bytes(C.byref(_cfg(krylov_restart=65)), 300) == 0
    assert lib.sim_workspace_bytes(C.byref(_cfg(mg_pre=0)), 300) == 0
    # FP32 preconditioned form stores Z in float32: smaller workspace
    assert lib.sim_workspace_bytes(C.byref(_cfg(precision=wl.PREC_FP32MG)), 300) < good
    # 256^3 FP32-MG form with FGMRES(20) fits easily in one GPU's 288 GB
    w3 = _cfg(n=(256, 256, 256), precision=wl.PREC_FP32MG)
    assert 4e9 < lib.sim_workspace_bytes(C.byref(w3), 144000) < 16e9


def test_config_check_names_the_broken_rule():
    """sim_config_check runs on the host: the rules of the configuration,
    each reported by name, without a GPU."""
    import copy

    from paper_2501_15314_amd import workloads as wl
    from paper_2501_15314_amd.sim import config_check

    good = wl.make_c1(n=32, n_points=300).cfg
    assert config_check(good, 300) == ""
    cases = [
        (dict(n=(30, 32, 32)), "multiple of 4"),
        (dict(bc=(3, 0, 0)), "bad bc"),
        (dict(length=(1.0, 1.0, 2.0)), "cubic"),
        (dict(dt=0.0), "dt"),
        (dict(lump_c=0.0), "lump_c"),
        (dict(krylov_restart=65), "krylov_restart"),
        (dict(precond=wl.PRECOND_FASTDIAG, n=(36, 36, 36), length=(1.0, 1.0, 1.0)), "multiples of 8"),
        (dict(krylov=7), "krylov"),
        (dict(outer_iters=0), "outer_iters"),
    ]
    for change, words in cases:
        cfg = copy.deepcopy(good)
        for k, v in change.items():
            setattr(cfg, k, v)
        msg = config_check(cfg, 300)
        assert words in msg, (change, msg)
    assert "max_points" in config_check(good, -1)
