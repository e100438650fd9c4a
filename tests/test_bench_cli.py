"""The benchmark's command-line contract, checked on the CPU: requests it
cannot honour end with exit status 2 and one JSON line naming the reason,
before any device is touched; the byte model of the dominant kernel follows
its stated formula."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _run(*args):
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args], capture_output=True, text=True,
                       timeout=120)
    return r.returncode, json.loads(r.stdout.strip().splitlines()[-1])


@pytest.mark.parametrize("gpus", ["2", "8"])
def test_more_than_one_gpu_refused(gpus):
    rc, out = _run("--gpus", gpus)
    assert rc == 2 and "one GPU" in out["error"]


@pytest.mark.parametrize("workload", ["p2_n64_32rhs", "p2_n40_adjoint"])
def test_fgmres_only_on_single_vector_solves(workload):
    rc, out = _run("--krylov", "fgmres", "--workload", workload)
    assert rc == 2 and "FGMRES" in out["error"]


def test_sweep_bytes_formula():
    sys.path.insert(0, ROOT)
    import bench
    n, nnz = 857375, 23881263
    nslices = (n + 63) // 64
    # (s + i) nnz + 8 bytes of metadata per slice + 4 s n, FP32 values, 32-bit columns
    assert bench.algorithmic_bytes("pk_sweep", n, nnz, 4, (4, 8 * nslices)) == 8 * nnz + 8 * nslices + 16 * n
    assert bench.algorithmic_bytes("pk_sweep", n, nnz, 4, (4, 8 * nslices)) == 204875280
