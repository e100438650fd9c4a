"""The C ABI: the library loads, exports every function include/aux.h declares,
and rejects invalid input from the host-side setup path (no GPU needed)."""
import ctypes
import os
import re
import subprocess

import numpy as np
import pytest

import paper_1204_2586_amd as aux
import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "aux.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\*?\s*([a-z_][a-z0-9_]*)\s*\(", src, flags=re.M)
    return sorted(set(names))


def test_every_declared_symbol_is_exported():
    names = _declared()
    assert "aux_setup" in names and "pcg_solve" in names and "aux_apply" in names
    lib = ctypes.CDLL(aux.library_path())
    for n in names:
        assert hasattr(lib, n), n
    out = subprocess.run(["nm", "-D", "--defined-only", aux.library_path()], capture_output=True, text=True).stdout
    exported = {l.split()[-1] for l in out.splitlines() if " T " in l}
    assert set(names) <= exported


def test_no_cpu_fallback_symbols():
    """The product path has no host implementation of the solve phase."""
    out = subprocess.run(["nm", "-D", "--defined-only", aux.library_path()], capture_output=True, text=True).stdout
    assert "orc_" not in out


def _mesh():
    return W.kuhn_mesh(2)


@pytest.mark.parametrize("case", ["order", "kappa_zero", "kappa_nan", "xyz_nan", "vertex_range", "flat_tet",
                                  "theta", "nu", "sell_window", "batch_tiles", "fuse_cycle", "cycle_lanes",
                                  "cycle_lanes_neg", "dense_cycle_rows", "no_interior"])
def test_setup_rejects_bad_input(case):
    xyz, tets = _mesh()
    kappa = np.ones(len(tets))
    kw = dict(host_only=True)
    order = 2
    if case == "order":
        order = 5
    elif case == "kappa_zero":
        kappa[3] = 0.0
    elif case == "kappa_nan":
        kappa[1] = np.nan
    elif case == "xyz_nan":
        xyz = xyz.copy()
        xyz[4, 1] = np.nan
    elif case == "vertex_range":
        tets = tets.copy()
        tets[0, 2] = len(xyz)
    elif case == "flat_tet":
        tets = tets.copy()
        tets[5, 3] = tets[5, 2]
    elif case == "theta":
        kw["theta"] = 1.5
    elif case == "nu":
        kw["nu"] = 0
    elif case == "sell_window":
        kw["sell_window"] = -5
    elif case == "batch_tiles":
        kw["batch_tiles"] = 3
    elif case == "fuse_cycle":
        kw["fuse_cycle"] = 2
    elif case == "cycle_lanes":
        kw["cycle_lanes"] = 3
    elif case == "cycle_lanes_neg":
        kw["cycle_lanes"] = -64
    elif case == "dense_cycle_rows":
        kw["dense_cycle_rows"] = -1
    elif case == "no_interior":                 # one tet: every node on the boundary
        xyz = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1.0]])
        tets = np.array([[0, 1, 2, 3]], dtype=np.int32)
        kappa = None
    with pytest.raises(aux.AuxError) as e:
        aux.Solver(xyz, tets, order, kappa, **kw)
    assert e.value.code == -1


def test_host_only_handle_refuses_device_calls():
    xyz, tets = _mesh()
    s = aux.Solver(xyz, tets, 2, host_only=True)
    lib = aux.load_library()
    rc = lib.aux_apply(s._h, None, None)
    assert rc == -7 and b"host-only" in lib.aux_last_error()


def test_fgmres_entry_checks_handle():
    lib = aux.load_library()
    assert lib.fgmres_solve(None, None, None, 1e-6, 30, 0, None, None) == -1
    xyz, tets = _mesh()
    s = aux.Solver(xyz, tets, 2, host_only=True)
    assert lib.fgmres_solve(s._h, None, None, 1e-6, 30, 0, None, None) == -7
