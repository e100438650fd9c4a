"""Host assembly of the library's Stokes blocks (Hood-Taylor P2-P1, Sec. 5)
against the oracle's, on host-only handles (no GPU).

The library integrates B = -div and the pressure mass matrix M_p exactly by
barycentric moments; the oracle by a degree-2 quadrature rule, exact for
these integrands.  Same patterns, values within 1e-14 of the largest entry.
"""
import numpy as np
import pytest

import oracle
import paper_1204_2586_amd as aux
import workloads as W


@pytest.mark.parametrize("n,jitter,rand", [(3, 0.2, True), (5, 0.2, False), (4, 0.0, True)])
def test_blocks_match_oracle(n, jitter, rand):
    xyz, tets = W.kuhn_mesh(n, jitter=jitter, seed=2)
    kap = np.exp(np.random.default_rng(1).normal(size=len(tets))) if rand else None
    s = aux.Solver(xyz, tets, 2, kap, host_only=True)
    assert s.stokes_setup() == xyz.shape[0]
    P = oracle.Problem(xyz, tets, 2, kap).stokes_setup()
    assert np.array_equal(s.dof_keys(), P.dof_keys())
    for which in ("B", "Mp"):
        a, b = s.export_csr(which), P.csr(which)
        assert a.shape == b.shape
        assert np.array_equal(a.indptr, b.indptr) and np.array_equal(a.indices, b.indices), which
        assert np.max(np.abs(a.data - b.data)) <= 1e-14 * np.max(np.abs(b.data)), which


def test_blocks_properties():
    """Independent of the oracle: B^T 1 = 0 (constants are the pressure null
    space), the mass matrix integrates 1 and x exactly (1 and 1/3)."""
    xyz, tets = W.kuhn_mesh(4, jitter=0.2, seed=3)
    s = aux.Solver(xyz, tets, 2, host_only=True)
    s.stokes_setup()
    B, M = s.export_csr("B"), s.export_csr("Mp")
    assert B.shape == (xyz.shape[0], 3 * s.n)
    assert np.max(np.abs(B.T @ np.ones(B.shape[0]))) <= 1e-14 * np.abs(B).max()
    one = np.ones(M.shape[0])
    assert abs(one @ M @ one - 1.0) <= 1e-14
    for c in range(3):
        assert abs(xyz[:, c] @ M @ xyz[:, c] - 1.0 / 3.0) <= 1e-14


@pytest.mark.parametrize("order", [3, 4])
def test_other_orders_rejected(order):
    xyz, tets = W.kuhn_mesh(2)
    s = aux.Solver(xyz, tets, order, host_only=True)
    with pytest.raises(aux.AuxError) as e:
        s.stokes_setup()
    assert e.value.code == aux.EINVAL
    with pytest.raises(aux.AuxError):
        s.export_csr("B")
