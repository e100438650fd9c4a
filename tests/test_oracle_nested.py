"""Pins of the oracle's intermediate auxiliary space (Remark 6.2): P^2 on the
same mesh in place of P^1 for a P^k problem (k = 3, 4), its own problem
solved by one application of the P^2 auxiliary-space preconditioner.

* The transfer I_2 is the embedding of P^2 in P^k: the identity for k = 2;
  P^k nodal values of every quadratic at nodes whose key vertices are all
  interior (the P^2 nodes of their sub-simplex are then unknowns).
* Nested spaces with exact integration: I_2^T A_k I_2 = A_2 (the P^2
  stiffness assembled on its own), for any coefficient.
* The preconditioner is symmetric positive definite with spectrum of B A_k
  in (0, 1] (a symmetric two-level method whose coarse solve B_2 satisfies
  0 < B_2 A_2 <= 1), also with a multi-level inner AMG.
* PCG with it converges in fewer steps than with P^1 as the auxiliary space,
  and in about as many on finer meshes; in the fp32 mode the result differs
  from FP64 by single-precision rounding only.
"""
import numpy as np
import pytest

import oracle
import workloads as W


def _problem(k, n, jitter=0.2, kappa=None, coarse_max=100, nested=True, seed=0):
    xyz, tets = W.kuhn_mesh(n, jitter=jitter, seed=seed)
    kap = None
    if kappa == "grf":
        kap = np.exp(W.grf_log_kappa(xyz, tets, seed=1))
    elif kappa == "rand":
        kap = np.exp(np.random.default_rng(3).normal(size=len(tets)))
    P = oracle.Problem(xyz, tets, k, kap)
    if nested:
        P.setup_nested(coarse_max=coarse_max)
    return P


def _node_xyz(P):
    keys = P.dof_keys()
    return P.xyz[keys].mean(axis=1)


def test_transfer_is_identity_for_p2():
    P = _problem(2, 4)
    I2 = P.csr("I2")
    assert I2.shape == (P.n, P.aux2.n)
    assert abs(I2 - np.eye(P.n)).max() == 0.0


@pytest.mark.parametrize("k", [3, 4])
def test_transfer_reproduces_quadratics(k):
    P = _problem(k, 4)
    I2 = P.csr("I2")
    assert I2.shape == (P.n, P.aux2.n)
    X, X2 = _node_xyz(P), _node_xyz(P.aux2)
    keys = P.dof_keys()
    interior = np.zeros(P.xyz.shape[0], dtype=bool)
    interior[np.all((P.xyz > 1e-12) & (P.xyz < 1 - 1e-12), axis=1)] = True
    rows = np.flatnonzero(interior[keys].all(axis=1))
    assert len(rows) > P.n // 8
    for q in (lambda x: 1.0 + 0 * x[:, 0], lambda x: x[:, 0] - 2 * x[:, 1] + 0.5 * x[:, 2],
              lambda x: x[:, 0] * x[:, 1] - 3 * x[:, 2] ** 2 + x[:, 1]):
        v = I2 @ q(X2)
        assert np.max(np.abs(v[rows] - q(X)[rows])) < 1e-13


@pytest.mark.parametrize("k,kappa", [(3, None), (3, "grf"), (4, "rand")])
def test_galerkin_product_is_the_p2_stiffness(k, kappa):
    P = _problem(k, 3, kappa=kappa)
    I2 = P.csr("I2")
    G = (I2.T @ P.csr("A") @ I2).toarray()
    A2 = P.aux2.csr("A").toarray()
    assert np.max(np.abs(G - A2)) < 1e-12 * np.max(np.abs(A2))


@pytest.mark.parametrize("k,n,coarse_max", [(3, 3, 100), (3, 4, 8), (4, 2, 100), (4, 3, 1)])
def test_nested_preconditioner_spd(k, n, coarse_max):
    P = _problem(k, n, coarse_max=coarse_max)
    if coarse_max < 100:
        assert P.aux2.nlev >= 3                      # the inner B_2 runs a multi-level cycle
    m = P.n
    B = np.column_stack([P.apply_nested(np.eye(m)[:, j]) for j in range(m)])
    assert np.max(np.abs(B - B.T)) <= 1e-13 * np.max(np.abs(B))
    assert np.linalg.eigvalsh(0.5 * (B + B.T))[0] > 0
    A = P.csr("A").toarray()
    ev = np.linalg.eigvals(B @ A).real
    assert ev.min() > 0 and ev.max() <= 1 + 1e-12


# (k, meshes): steps to 1e-8 measured (jittered, GRF kappa) P3 24, 21, 21
# (P^1 space 43, 38, 36); P4 37, 39, 39 (P^1 space 71, 82, 69)
@pytest.mark.parametrize("k,ns", [(3, (5, 7, 9)), (4, (3, 4, 6))])
def test_nested_pcg_beats_p1_space_and_is_flat(k, ns):
    steps, base = [], []
    for n in ns:
        P = _problem(k, n, kappa="grf")
        P.setup_amg()
        b = P.load(W.manufactured_f)
        x, it, rr, st = P.pcg_nested(b, tol=1e-8)
        assert st == 0 and rr <= 1e-8
        A = P.csr("A")
        assert np.linalg.norm(b - A @ x) <= 1.01e-8 * np.linalg.norm(b)
        x1, it1, _, st1 = P.pcg(b, tol=1e-8)
        assert st1 == 0
        assert np.linalg.norm(x - x1) <= 1e-6 * np.linalg.norm(x1)
        steps.append(it)
        base.append(it1)
    assert all(a < 0.7 * b for a, b in zip(steps, base)), (steps, base)
    assert steps[-1] <= steps[0] + 3, steps


def test_nested_fp32_mode():
    P = _problem(3, 4, kappa="grf")
    r = np.random.default_rng(5).standard_normal(P.n)
    z64, z32 = P.apply_nested(r), P.apply_nested(r, fp32=True)
    d = np.linalg.norm(z32 - z64) / np.linalg.norm(z64)
    assert 1e-10 < d < 1e-5
