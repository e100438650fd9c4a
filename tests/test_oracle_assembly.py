"""Pins of the oracle's global discretisation (Sec. 2 of the paper).

* sizes: (kn-1)^3 interior P^k nodes and (n-1)^3 interior vertices on the
  n^3-cube Kuhn mesh;
* A_h symmetric, and consistent: for a polynomial q of degree <= k and a node
  whose basis support avoids the boundary, (A_h q)_i = int (-Laplace q) phi_i,
  which the load vector computes independently;
* A_H on the unjittered mesh is h times the 7-point Laplacian;
* the Galerkin relation A_H = I_R A_h I_P with I_R = I_P^T (Sec. 2, after
  eq. "Prol"), for jittered meshes and per-tet kappa;
* I_P transfers P^1 functions exactly: c_j^i = psi_j(x_i^h) (Sec. 2).
"""
import numpy as np
import pytest
import scipy.sparse as sp

import oracle
import workloads as W


def _node_positions(P, xyz):
    keys = P.dof_keys()
    return xyz[keys].mean(axis=1), keys


@pytest.mark.parametrize("k,n", [(2, 3), (2, 5), (3, 3), (3, 4), (4, 2), (4, 3)])
def test_sizes(k, n):
    xyz, tets = W.kuhn_mesh(n)
    P = oracle.Problem(xyz, tets, k)
    assert P.n == (k * n - 1) ** 3
    assert P.nH == (n - 1) ** 3
    assert P.nnode == (k * n + 1) ** 3
    keys = P.dof_keys()
    assert np.all(np.diff(keys, axis=1) >= 0)                   # sorted multisets
    # numbered in lexicographic key order
    assert all(tuple(keys[i]) < tuple(keys[i + 1]) for i in range(len(keys) - 1))


@pytest.mark.parametrize("k,jit", [(2, 0.0), (2, 0.2), (3, 0.0), (3, 0.15), (4, 0.0), (4, 0.15)])
def test_stiffness_consistency_with_load(k, jit):
    n = 6
    xyz, tets = W.kuhn_mesh(n, jitter=jit, seed=11)
    P = oracle.Problem(xyz, tets, k)
    A = P.csr("A")
    assert abs(A - A.T).max() < 1e-13 * abs(A).max()
    x, keys = _node_positions(P, xyz)
    lattice, _ = _node_positions(P, W.kuhn_mesh(n)[0])
    far = np.all((lattice > 1.99 / n) & (lattice < 1 - 1.99 / n), axis=1)
    assert far.sum() > 50

    if k == 2:
        def q(p):
            return p[..., 0] ** 2 + 2 * p[..., 1] ** 2 - p[..., 2] ** 2 + p[..., 0] * p[..., 1] + p[..., 2]

        def minus_lap(p):
            return np.full(p.shape[:-1], -4.0)
    else:
        def q(p):
            return p[..., 0] ** 3 - 2 * p[..., 0] * p[..., 1] * p[..., 2] + p[..., 1] ** 2 * p[..., 2]

        def minus_lap(p):
            return -(6 * p[..., 0] + 2 * p[..., 2])

    lhs = A @ q(x)
    rhs = P.load(minus_lap)
    assert np.max(np.abs(lhs[far] - rhs[far])) < 1e-11 * np.max(np.abs(rhs[far]))


@pytest.mark.parametrize("n", [4, 7])
def test_P1_matrix_is_scaled_7_point_laplacian(n):
    xyz, tets = W.kuhn_mesh(n)
    P = oracle.Problem(xyz, tets, 2)
    AH = P.csr("AH")
    h = 1.0 / n
    L1 = sp.diags([-np.ones(n - 2), 2 * np.ones(n - 1), -np.ones(n - 2)], [-1, 0, 1])
    I = sp.identity(n - 1)
    L7 = sp.kron(sp.kron(L1, I), I) + sp.kron(sp.kron(I, L1), I) + sp.kron(sp.kron(I, I), L1)
    assert abs(AH - h * L7).max() < 1e-14


@pytest.mark.parametrize("k", [2, 3, 4])
def test_galerkin_relation(k):
    xyz, tets = W.kuhn_mesh(5, jitter=0.2, seed=2)
    kappa = np.exp(2.0 * np.random.default_rng(9).normal(size=tets.shape[0]))
    P = oracle.Problem(xyz, tets, k, kappa)
    A, AH, IP = P.csr("A"), P.csr("AH"), P.csr("IP")
    G = (IP.T @ A @ IP).toarray()
    assert np.max(np.abs(G - AH.toarray())) < 1e-13 * np.max(np.abs(AH.toarray()))


@pytest.mark.parametrize("k", [2, 3, 4])
def test_transfer_of_linear_functions(k):
    xyz, tets = W.kuhn_mesh(4, jitter=0.2, seed=5)
    P = oracle.Problem(xyz, tets, k)
    IP = P.csr("IP")
    x, keys = _node_positions(P, xyz)
    interior_vertex = np.all((xyz > 1e-9 + 0.5 / 4) & (xyz < 1 - 0.5 / 4), axis=1)
    vid = np.cumsum(interior_vertex) - 1
    rows_ok = np.all(interior_vertex[keys], axis=1)      # carrier away from the boundary
    assert rows_ok.sum() > 10
    c = np.array([0.3, -1.2, 0.7])
    ell_v = 0.5 + xyz[interior_vertex] @ c
    ell_nodes = 0.5 + x @ c
    assert np.max(np.abs((IP @ ell_v)[rows_ok] - ell_nodes[rows_ok])) < 1e-14
    rs = np.asarray(IP.sum(axis=1)).ravel()
    assert np.max(np.abs(rs[rows_ok] - 1.0)) < 1e-15
    assert np.all(np.abs(IP.data * k - np.round(IP.data * k)) == 0)   # multiples of 1/k
    # each row couples only to the vertices of the node's own carrier
    for i in np.flatnonzero(rows_ok)[:50]:
        cols = IP.indices[IP.indptr[i]:IP.indptr[i + 1]]
        assert set(cols) == set(vid[np.unique(keys[i])])
