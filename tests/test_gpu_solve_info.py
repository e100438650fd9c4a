"""Solve metrics and the failure path on the GPU, through the C ABI.

* The option true_residual reports ||f - A_h u|| / ||f|| of the returned
  iterate (checked against a product recomputed here); without it the field
  is -1.
* aux_residual_history returns ||r_k|| / ||f|| for k = 0 .. iterations of the
  last single-vector CG solve, equal step by step to the oracle's CG stopped
  after k iterations; after the allocation-free solve as well.
* The smoother weight omega (G_h = omega D_l1^-1) against the oracle with the
  same weight (P2, P3, and the intermediate P^2 space at P4); a negative
  weight makes B indefinite and CG returns AUX_EBREAKDOWN (the breakdown
  status, reached here from the host with valid input).
"""
import numpy as np
import pytest
import torch

import oracle
import paper_1204_2586_amd as aux
import workloads as W

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def _mesh(n, jitter=0.2):
    return W.kuhn_mesh(n, jitter=jitter, seed=0)


def _t(x):
    return torch.tensor(np.asarray(x), dtype=torch.float64, device=DEV)


def _rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def test_true_residual():
    xyz, tets = _mesh(6)
    f = None
    for flag in (False, True):
        s = aux.Solver(xyz, tets, 2, device=DEV, precision="mixed", true_residual=flag)
        if f is None:
            f = _t(s.load(W.manufactured_f))
        u, info = s.solve(f, tol=1e-8)
        if not flag:
            assert info.true_rel_residual == -1.0
            continue
        ref = float(torch.linalg.norm(f - s.matvec(u)) / torch.linalg.norm(f))
        assert abs(info.true_rel_residual - ref) <= 1e-10 * ref
        assert info.true_rel_residual <= 1.01e-8
        info2 = s.solve_noalloc(f, torch.zeros_like(f), tol=1e-8)
        assert abs(info2.true_rel_residual - ref) <= 1e-6 * ref


@pytest.mark.parametrize("k,n", [(2, 6), (3, 4)])
def test_residual_history_matches_oracle(k, n):
    xyz, tets = _mesh(n)
    s = aux.Solver(xyz, tets, k, device=DEV)
    orc = oracle.Problem(xyz, tets, k).setup_amg()
    b = orc.load(W.manufactured_f)
    u, info = s.solve(_t(b), tol=1e-8)
    h = s.residual_history()
    assert len(h) == info.iterations + 1
    assert abs(h[0] - 1.0) <= 1e-15
    assert abs(h[-1] - info.rel_residual) <= 1e-15 * max(info.rel_residual, 1e-300)
    for it in range(1, info.iterations + 1):
        _, k_it, rr, _ = orc.pcg(b, tol=0.0, maxit=it)
        assert k_it == it
        assert abs(h[it] - rr) <= 1e-8 * rr, (it, h[it], rr)
    # the allocation-free solve keeps its history in the GPU's scratch array
    u2 = torch.zeros_like(u)
    info2 = s.solve_noalloc(_t(b), u2, tol=1e-8)
    h2 = s.residual_history()
    assert len(h2) == info2.iterations + 1
    assert np.max(np.abs(h2 - h[:len(h2)])) <= 1e-12


@pytest.mark.parametrize("k,n,omega", [(2, 6, 0.7), (3, 5, 0.8)])
def test_smoother_weight_parity(k, n, omega):
    xyz, tets = _mesh(n)
    s = aux.Solver(xyz, tets, k, device=DEV, smoother_weight=omega)
    orc = oracle.Problem(xyz, tets, k).set_smoother_weight(omega).setup_amg()
    r = W.random_vector(s.n, 4)
    z = s.apply(_t(r)).cpu().numpy()
    assert _rel(z, orc.apply(r)) <= 1e-12
    assert _rel(z, oracle.Problem(xyz, tets, k).setup_amg().apply(r)) > 1e-3
    s.set_precision("mixed")
    z32 = s.apply(_t(r)).cpu().numpy()
    assert _rel(z32, orc.apply(r, fp32=True)) <= 2e-6
    s.set_precision("fp64")
    b = orc.load(W.manufactured_f)
    x, it, _, _ = orc.pcg(b, tol=1e-8)
    u, info = s.solve(_t(b), tol=0.0, maxit=it, check=False)
    assert _rel(u.cpu().numpy(), x) <= 1e-10


def test_smoother_weight_nested():
    xyz, tets = _mesh(3)
    s = aux.Solver(xyz, tets, 4, device=DEV, smoother_weight=0.8, aux_space=2)
    orc = oracle.Problem(xyz, tets, 4).set_smoother_weight(0.8).setup_nested()
    r = W.random_vector(s.n, 6)
    assert _rel(s.apply(_t(r)).cpu().numpy(), orc.apply_nested(r)) <= 1e-12


def test_negative_weight_reports_breakdown():
    xyz, tets = _mesh(4)
    s = aux.Solver(xyz, tets, 2, device=DEV, smoother_weight=-1.0, coarse_max=8)
    orc = oracle.Problem(xyz, tets, 2).set_smoother_weight(-1.0).setup_amg(coarse_max=8)
    b = orc.load(W.manufactured_f)
    _, it, _, st = orc.pcg(b, tol=1e-8)
    assert st == 2
    u, info = s.solve(_t(b), tol=1e-8, check=False)
    assert info.status == aux.EBREAKDOWN
    assert info.iterations == it
    with pytest.raises(aux.AuxError, match="AUX_EBREAKDOWN"):
        s.solve(_t(b), tol=1e-8)


def test_invalid_weight_rejected():
    xyz, tets = _mesh(3)
    for w in (0.0, float("nan"), float("inf")):
        with pytest.raises(aux.AuxError, match="smoother_weight"):
            aux.Solver(xyz, tets, 2, device=DEV, smoother_weight=w)
