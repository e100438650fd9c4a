"""Host-side builders checked on the CPU: the row-split sliced ELL layout of
the V-cycle operators (entry placement, padding and the wavefront's product
against the CSR product), the Morton order and column renumbering of the
batched layout, and the dense sub-cycle matrix (against the V(1,1)
cycle evaluated step by step on every unit vector, Alg. 2.1's coarse solve).
The C++ harness tests/host_formats_check.cpp is compiled with the library's
host sources."""
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HOST = os.path.join(ROOT, "paper_1204_2586_amd", "csrc", "host")


@pytest.fixture(scope="module")
def results(tmp_path_factory):
    exe = tmp_path_factory.mktemp("hostfmt") / "check"
    srcs = [os.path.join(ROOT, "tests", "host_formats_check.cpp")] + \
           [os.path.join(HOST, f) for f in ("fem.cpp", "amg.cpp", "formats.cpp", "fuse.cpp")]
    subprocess.run(["g++", "-O1", "-std=c++17", "-I", HOST] + srcs + ["-o", str(exe)], check=True)
    run = subprocess.run([str(exe)], capture_output=True, text=True)
    assert run.returncode == 0, run.stdout + run.stderr
    out = {"ell": [], "dense": [], "morton": [], "renum": []}
    for line in run.stdout.splitlines():
        kind, size, err = line.split()
        out[kind].append((int(size), float(err)))
    return out


def test_row_split_ell_layout_and_product(results):
    assert sorted({l for l, _ in results["ell"]}) == [1, 2, 4, 8, 16, 32]
    for lanes, err in results["ell"]:
        assert err <= 1e-14, (lanes, err)


def test_dense_sub_cycle_equals_stepwise_cycle(results):
    assert [n for n, _ in results["dense"]] == [2, 3, 4]
    for nlev, err in results["dense"]:
        assert err <= 1e-12, (nlev, err)


def test_morton_order(results):
    """A permutation whose interleaved-bit codes never decrease; on 2^k
    lattices every aligned run of 8 and 64 points is a 2- and 4-cube."""
    assert [k for k, _ in results["morton"]] == [1, 3, 4]
    assert all(v == 0 for _, v in results["morton"]), results["morton"]


def test_renumber_cols(results):
    assert len(results["renum"]) == 3
    assert all(err == 0.0 for _, err in results["renum"]), results["renum"]
