"""GPU parity at the benchmark sizes, in the configuration bench.py times
(default options: autotuned layout, each CG iteration replayed as a HIP
graph), against the CPU oracle solving the same systems.

* P2, 48^3 cubes x 6 tets, interior vertices jittered +-0.2h (857,375
  unknowns), manufactured source: one preconditioner application in FP64
  (1e-12) and FP32 (2e-6, and more than 1e-9 away from FP64); FP64 CG with the iteration count fixed to
  the oracle's agrees to 1e-10; free-running counts within +-1 (FP64 against
  the oracle's FP64, mixed against the oracle's FP32 mode); the mixed solution
  within 1e-7 of the oracle's FP64 solution; the same with the matrix-free
  operator.
* P3, 32^3 cubes, kappa = exp(GRF) (857,375 unknowns): the same bars for the
  assembled and the matrix-free operator.
* P4, 24^3 cubes, kappa = 1 (857,375 unknowns): the same bars for the
  assembled and the matrix-free operator.
* 32 sources in lock-step on P2, 64^3 cubes (2,048,383 unknowns): the
  columns the oracle can afford (sources 0 and 31) are solved by the oracle
  and compared at the mixed bar; every column's true residual meets the
  tolerance.

The oracle runs single-threaded here, about 10 to 40 s per system.
"""
import numpy as np
import pytest
import torch

import oracle
import paper_1204_2586_amd as aux
import workloads as W

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def _t(x):
    return torch.tensor(np.asarray(x), dtype=torch.float64, device=DEV)


def _rel(a, b):
    a, b = np.asarray(a), np.asarray(b)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def _system(k, n, jitter, grf):
    xyz, tets = W.kuhn_mesh(n, jitter=jitter, seed=0)
    kappa = np.exp(W.grf_log_kappa(xyz, tets, seed=1)) if grf else None
    return xyz, tets, kappa


@pytest.mark.parametrize("name,k,n,jitter,grf,operator", [
    ("p2_n48_jitter", 2, 48, 0.2, False, "assembled"),
    ("p2_n48_jitter", 2, 48, 0.2, False, "matfree"),
    ("p3_n32_grf", 3, 32, 0.0, True, "assembled"),
    ("p3_n32_grf", 3, 32, 0.0, True, "matfree"),
    ("p4_n24", 4, 24, 0.0, False, "assembled"),
    ("p4_n24", 4, 24, 0.0, False, "matfree"),
])
def test_full_size_solve_matches_oracle(name, k, n, jitter, grf, operator):
    print(f"[full size {name} {operator}]", flush=True)
    xyz, tets, kappa = _system(k, n, jitter, grf)
    orc = oracle.Problem(xyz, tets, k, kappa).setup_amg()
    b = orc.load(W.manufactured_f)
    x64, it64, _, st = orc.pcg(b, tol=1e-8)
    assert st == 0
    x32, it32, _, st = orc.pcg(b, tol=1e-8, fp32=True)
    assert st == 0

    lib = aux.Solver(xyz, tets, k, kappa, device=DEV, operator=operator)
    assert np.array_equal(lib.dof_keys(), orc.dof_keys())
    f = _t(b)
    # one preconditioner application in both precisions against the oracle's;
    # the FP32 form must visibly differ from the FP64 one (FP32 ran)
    r = W.random_vector(lib.n, 7)
    lib.set_precision("fp64")
    z64 = lib.apply(_t(r)).cpu().numpy()
    lib.set_precision("mixed")
    z32 = lib.apply(_t(r)).cpu().numpy()
    o64 = orc.apply(r)
    assert _rel(z64, o64) <= 1e-12
    assert _rel(z32, orc.apply(r, fp32=True)) <= 2e-6 and _rel(z32, o64) <= 2e-6
    assert _rel(z32, o64) > 1e-9 and _rel(z32, z64) > 1e-9
    lib.set_precision("fp64")
    u, info = lib.solve(f, tol=1e-8)
    assert abs(info.iterations - it64) <= 1
    u, info = lib.solve(f, tol=0.0, maxit=it64, check=False)
    assert info.iterations == it64
    assert _rel(u.cpu().numpy(), x64) <= 1e-10
    lib.set_precision("mixed")
    u, info = lib.solve(f, tol=1e-8)
    assert abs(info.iterations - it32) <= 1
    assert _rel(u.cpu().numpy(), x64) <= 1e-7
    true_res = torch.linalg.norm(f - lib.matvec(u)) / torch.linalg.norm(f)
    assert float(true_res) <= 1e-8 * 1.05


def test_full_size_batched_columns_match_oracle():
    print("[full size p2_n64_32rhs]", flush=True)
    xyz, tets, _ = _system(2, 64, 0.0, False)
    lib = aux.Solver(xyz, tets, 2, None, device=DEV, precision="mixed")
    F = _t(lib.load_many(W.fourier_fields(range(32)), 32, threads=16))
    U, infos = lib.solve_batched(F, tol=1e-8)
    assert all(i.converged for i in infos)
    for c in range(32):
        r = torch.linalg.norm(F[:, c] - lib.matvec(U[:, c].contiguous())) / torch.linalg.norm(F[:, c])
        assert float(r) <= 1e-8 * 1.05, c
    orc = oracle.Problem(xyz, tets, 2).setup_amg()
    for c in (0, 31):
        src = W.fourier_fields([c])

        def f(p):
            out = np.empty(p.shape[0])
            for i in range(0, p.shape[0], 1 << 22):
                out[i:i + (1 << 22)] = src(p[i:i + (1 << 22)])[0]
            return out

        b = orc.load(f)
        # the device load vector is the library's host assembly of the same source
        assert _rel(F[:, c].cpu().numpy(), b) <= 1e-13
        x, it, _, st = orc.pcg(b, tol=1e-8, fp32=True)
        assert st == 0 and abs(infos[c].iterations - it) <= 1
        assert _rel(U[:, c].cpu().numpy(), orc.pcg(b, tol=1e-8)[0]) <= 1e-7
