"""GPU block preconditioned CG (O'Leary 1980) through the C ABI against the
oracle's block CG and its single-column solves.

Bars (from the arithmetic, as for single-vector CG):
* FP64, step count fixed to the oracle's: the block within 1e-10 (relative
  Frobenius norm) of the oracle's block CG after the same steps;
* free-running: the step count within +-1 of the oracle's block CG (FP64
  against FP64, mixed against the oracle's FP32-preconditioner form); every
  column within 1e-7 of the oracle's single-column FP64 solution and its
  true residual within the tolerance;
* widths padded to the block (5 columns in a block of 8, 12 in 16) and one
  column (which is CG).
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


def _relf(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b)))


CASES = {
    "p2_n8_jitter_5rhs": dict(k=2, n=8, jitter=0.2, nrhs=5),
    "p3_n5_12rhs": dict(k=3, n=5, jitter=0.0, nrhs=12),
    "p2_n6_1rhs": dict(k=2, n=6, jitter=0.2, nrhs=1),
}


@pytest.fixture(scope="module", params=list(CASES), ids=list(CASES))
def case(request):
    c = CASES[request.param]
    print(f"[block cg {request.param}]", flush=True)
    xyz, tets = W.kuhn_mesh(c["n"], jitter=c["jitter"], seed=0)
    kappa = np.exp(np.random.default_rng(4).normal(size=len(tets)))
    orc = oracle.Problem(xyz, tets, c["k"], kappa).setup_amg()
    lib = aux.Solver(xyz, tets, c["k"], kappa, device=DEV)
    assert np.array_equal(lib.dof_keys(), orc.dof_keys())
    F = np.stack([orc.load(W.fourier_f(j)) for j in range(c["nrhs"])], axis=1)
    return lib, orc, F


def test_block_fixed_steps_fp64(case):
    lib, orc, F = case
    lib.set_precision("fp64")
    X, it, rel, st = orc.block_pcg(F, tol=1e-8)
    assert st == 0
    for k in sorted({1, 3, it}):
        Xk, _, _, _ = orc.block_pcg(F, tol=0.0, maxit=k)
        U, infos = lib.solve_block(_t(F), tol=0.0, maxit=k, check=False)
        assert all(i.iterations == k for i in infos)
        assert _relf(U.cpu().numpy(), Xk) <= 1e-10, k


def test_block_free_running(case):
    lib, orc, F = case
    for prec in ("fp64", "mixed"):
        lib.set_precision(prec)
        X, it, rel, st = orc.block_pcg(F, tol=1e-8, fp32=(prec == "mixed"))
        assert st == 0
        Ft = _t(F)
        U, infos = lib.solve_block(Ft, tol=1e-8)
        assert all(i.converged for i in infos)
        assert abs(infos[0].iterations - it) <= 1, (prec, infos[0].iterations, it)
        for j in range(F.shape[1]):
            xj, _, _, _ = orc.pcg(F[:, j], tol=1e-10)
            assert _relf(U[:, j].cpu().numpy(), xj) <= 1e-7, (prec, j)
            res = torch.linalg.norm(Ft[:, j] - lib.matvec(U[:, j].contiguous())) / torch.linalg.norm(Ft[:, j])
            assert float(res) <= 1e-8 * 1.05, (prec, j)
            assert infos[j].rel_residual <= 1e-8
    lib.set_precision("fp64")


def test_block_one_column_equals_cg():
    xyz, tets = W.kuhn_mesh(6, jitter=0.2, seed=1)
    lib = aux.Solver(xyz, tets, 2, device=DEV)
    b = _t(lib.load(W.manufactured_f))
    u, info = lib.solve(b, tol=1e-8)
    U, infos = lib.solve_block(b[:, None].contiguous(), tol=1e-8)
    assert abs(infos[0].iterations - info.iterations) <= 1
    # the same iterates up to rounding: 1e-10 at the same step count
    bar = 1e-10 if infos[0].iterations == info.iterations else 1e-7
    assert _relf(U[:, 0].cpu().numpy(), u.cpu().numpy()) <= bar


def test_block_limits():
    xyz, tets = W.kuhn_mesh(4, seed=0)
    lib = aux.Solver(xyz, tets, 2, device=DEV)
    F = torch.zeros(lib.n, 65, dtype=torch.float64, device=DEV)
    with pytest.raises(aux.AuxError) as e:
        lib.solve_block(F)
    assert e.value.code == aux.EINVAL
    U, infos = lib.solve_block(torch.zeros(lib.n, 3, dtype=torch.float64, device=DEV))
    assert all(i.converged and i.iterations == 0 for i in infos) and not torch.any(U)
