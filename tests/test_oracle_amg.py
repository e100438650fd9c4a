"""Pins of the oracle's AMG setup on the auxiliary P^1 matrix.

The paper uses PMIS coarsening and extended+i interpolation with the
strength rule of Sec. 6.2.  Checked here: the published splitmix64 test
vector behind the PMIS random measure; the PMIS splitting property (every F
point influences nobody or depends strongly on a C point); interpolation
identity rows at C points; the extended+i property that rows of P sum to one
where the row sums of A vanish; Galerkin coarse operators symmetric positive
definite; the distance-two reach of interpolation; and the hierarchy shape.
"""
import os

import numpy as np
import pytest

import oracle
import oracle_pins as pins
import workloads as W

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def test_splitmix64_published_vector():
    vals = [int(l, 16) for l in open(os.path.join(GOLD, "splitmix64_seed0.txt"))
            if l.strip() and not l.startswith("#")]
    g = 0x9E3779B97F4A7C15
    assert [oracle.splitmix64((i * g) % 2 ** 64) for i in range(3)] == vals


@pytest.fixture(scope="module")
def hier():
    xyz, tets = W.kuhn_mesh(12, jitter=0.2, seed=0)
    P = oracle.Problem(xyz, tets, 2)
    P.setup_amg(theta=0.8, coarse_max=100)
    return P


def _strong(A, theta):
    """Strength sets by the rule of Sec. 6.2 (for checking the splitting only)."""
    S = []
    for i in range(A.shape[0]):
        cols = A.indices[A.indptr[i]:A.indptr[i + 1]]
        vals = A.data[A.indptr[i]:A.indptr[i + 1]]
        off = cols != i
        m = np.max(-vals[off]) if off.any() else -np.inf
        S.append(set(cols[off][-vals[off] > theta * m + 1e-12 * m]) if m > 0 else set())
    return S


def test_hierarchy_shape(hier):
    assert hier.nlev >= 3 and hier.ncoarse <= 100
    sizes = [hier.csr("Alev", l).shape[0] for l in range(hier.nlev)]
    assert sizes[0] == hier.nH and all(b < a for a, b in zip(sizes, sizes[1:]))
    L = hier.coarse_cholesky()
    Ac = hier.csr("Alev", hier.nlev - 1).toarray()
    assert np.max(np.abs(L @ L.T - Ac)) < 1e-13 * np.max(np.abs(Ac))


def test_pmis_splitting_property(hier):
    for l in range(hier.nlev - 1):
        A = hier.csr("Alev", l)
        cf = hier.level_cf(l)
        assert set(np.unique(cf)) <= {-1, 1}
        S = _strong(A, 0.8)
        influences = np.zeros(A.shape[0], dtype=int)
        for i, s in enumerate(S):
            for j in s:
                influences[j] += 1
        for i in range(A.shape[0]):
            if cf[i] > 0:
                assert influences[i] > 0          # C points influence someone
            elif influences[i] > 0:
                assert any(cf[j] > 0 for j in S[i]), (l, i)


def test_interpolation_properties(hier):
    for l in range(hier.nlev - 1):
        A = hier.csr("Alev", l)
        P = hier.csr("P", l)
        cf = hier.level_cf(l)
        cidx = np.cumsum(cf > 0) - 1
        assert P.shape == (A.shape[0], int((cf > 0).sum()))
        for i in np.flatnonzero(cf > 0):
            row = P.getrow(i)
            assert row.nnz == 1 and row.indices[0] == cidx[i] and row.data[0] == 1.0
        rs_A = np.abs(np.asarray(A.sum(axis=1)).ravel())
        zero_rows = rs_A < 1e-12 * np.abs(A.diagonal())
        rs_P = np.asarray(P.sum(axis=1)).ravel()
        if l == 0:
            assert zero_rows.sum() > 0
        if zero_rows.any():
            assert np.max(np.abs(rs_P[zero_rows] - 1.0)) < 1e-12
        # distance two: P_ij != 0 only for C points j within two graph steps of i
        A2 = (abs(A) @ abs(A)).tocsr()
        Pc = P.tocoo()
        cpts = np.flatnonzero(cf > 0)
        for i, j in zip(Pc.row, Pc.col):
            assert A2[i, cpts[j]] != 0 or i == cpts[j]


def test_coarse_operators_spd(hier):
    for l in range(1, hier.nlev):
        A = hier.csr("Alev", l).toarray()
        assert np.max(np.abs(A - A.T)) < 1e-13 * np.max(np.abs(A))
        if A.shape[0] <= 2000:
            assert np.linalg.eigvalsh(A)[0] > 0
        P = hier.csr("P", l - 1)
        Af = hier.csr("Alev", l - 1)
        assert abs(P.T @ Af @ P - hier.csr("Alev", l)).max() < 1e-13 * np.abs(A).max()


def test_unjittered_level0_stencil_all_axis_neighbours_strong():
    xyz, tets = W.kuhn_mesh(8)
    P = oracle.Problem(xyz, tets, 2)
    P.setup_amg(theta=0.8)
    A = P.csr("Alev", 0)
    S = _strong(A, 0.8)
    n1 = 7
    for i in range(A.shape[0]):
        a, r = divmod(i, n1 * n1)
        b, c = divmod(r, n1)
        axis_nb = sum(0 <= v + d < n1 for v in (a, b, c) for d in (-1, 1))
        assert len(S[i]) == axis_nb


@pytest.mark.parametrize("theta,seed", [(0.8, 0), (0.25, 7)])
def test_pmis_rounds(theta, seed):
    """Each PMIS round: the new C points are exactly the undecided local
    maxima of the measure over S u S^T (independent there), and exactly the
    undecided points depending strongly on one of them become F."""
    pins.check_pmis_rounds(theta=theta, seed=seed)


def test_ext_i_harmonic_1d():
    """Extended+i reproduces the harmonic extension -A_FF^{-1} A_FC on
    tridiagonal M-matrices with F runs of length <= 2 (plain extended
    interpolation does not)."""
    pins.check_ext_i_harmonic_1d()


def test_ext_i_exact_rationals():
    """Extended+i weights on random small matrices (positive off-diagonals,
    weak couplings, d_k = 0 cases, distance-two C points) equal the published
    formula evaluated in exact rationals."""
    pins.check_ext_i_rational()
