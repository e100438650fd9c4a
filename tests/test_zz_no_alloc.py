"""The allocation-free CG entry point pcg_solve_noalloc against pcg_solve.

pcg_solve_noalloc runs the same kernels in the same order as pcg_solve with
its reduction partials, CG state and histories in the library's fixed
per-GPU scratch array instead of the handle's buffers (and without graph
replay, which launches the same kernels).  Checked through the C ABI, to the
FP64 parity bar (1e-10 relative 2-norm; the same iteration count and status;
the mixed form to the same bar against its own pcg_solve): two calls in a
row, the second on a smaller problem (another handle sharing the array), and
the argument limits.
"""
import ctypes

import numpy as np
import pytest
import torch

import paper_1204_2586_amd as aux
import workloads as W

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def _rel(a, b):
    return float(torch.linalg.norm(a - b) / torch.linalg.norm(b))


def _system(k, n, precision, operator="assembled"):
    xyz, tets = W.kuhn_mesh(n, jitter=0.2, seed=0)
    s = aux.Solver(xyz, tets, k, device=DEV, precision=precision, operator=operator)
    f = torch.tensor(s.load(W.manufactured_f), dtype=torch.float64, device=DEV)
    return s, f


@pytest.mark.parametrize("precision,operator", [("fp64", "assembled"), ("mixed", "assembled"),
                                                ("mixed", "matfree")])
def test_noalloc_matches_pcg_solve_two_calls(precision, operator):
    cases = [(2, 12), (2, 6)] if operator == "assembled" else [(3, 8), (3, 4)]
    for k, n in cases:                      # the second call is on a smaller problem
        print(f"[no-alloc {precision} {operator} P{k} {n}^3]", flush=True)
        s, f = _system(k, n, precision, operator)
        u_ref, i_ref = s.solve(f, tol=1e-8)
        u = torch.zeros_like(f)
        info = s.solve_noalloc(f, u, tol=1e-8)
        torch.cuda.synchronize()
        assert info.status == i_ref.status == 0
        assert info.iterations == i_ref.iterations
        assert _rel(u, u_ref) <= 1e-10
        assert abs(info.rel_residual - i_ref.rel_residual) <= 1e-6 * i_ref.rel_residual
        # fixed iteration count (tol = 0), from a non-zero initial guess
        u0 = torch.tensor(W.random_vector(s.n, 3), device=DEV)
        u_ref, i_ref = s.solve(f, tol=0.0, maxit=5, u0=u0, check=False)
        u = u0.clone()
        info = s.solve_noalloc(f, u, tol=0.0, maxit=5, check=False)
        assert info.iterations == i_ref.iterations == 5 and info.status == i_ref.status == aux.ENOTCONV
        assert _rel(u, u_ref) <= 1e-10
        s.close()


def test_noalloc_limits():
    s, f = _system(2, 4, "fp64")
    u = torch.zeros_like(f)
    with pytest.raises(aux.AuxError) as e:
        s.solve_noalloc(f, u, tol=1e-8, maxit=5000)
    assert e.value.code == aux.EINVAL
    info = s.solve_noalloc(f, u, tol=1e-8, maxit=4094)
    assert info.converged
    lib = aux.load_library()
    rc = lib.pcg_solve_noalloc(None, ctypes.c_void_p(f.data_ptr()), ctypes.c_void_p(u.data_ptr()), 1e-8, 0, None)
    assert rc == aux.EINVAL
    s.close()
