"""Host setup of the intermediate auxiliary space (Remark 6.2) against the
oracle (no GPU needed): the library's P^2 handle on the same mesh numbers
its dofs like the oracle's P^2 problem, and the transfer I_2 (the embedding
of P^2 in P^k) is entry for entry the oracle's."""
import numpy as np
import pytest

import oracle
import paper_1204_2586_amd as aux
import workloads as W


@pytest.mark.parametrize("k,n,jitter", [(3, 4, 0.2), (4, 3, 0.0), (3, 5, 0.0)])
def test_transfer_equals_oracle(k, n, jitter):
    xyz, tets = W.kuhn_mesh(n, jitter=jitter, seed=0)
    lib = aux.Solver(xyz, tets, k, host_only=True, aux_space=2)
    orc = oracle.Problem(xyz, tets, k).setup_nested()
    assert lib.info.aux_space == 2
    a, b = lib.export_csr("I2"), orc.csr("I2")
    assert a.shape == b.shape == (orc.n, orc.aux2.n)
    assert np.array_equal(a.indptr, b.indptr) and np.array_equal(a.indices, b.indices)
    assert np.max(np.abs(a.data - b.data)) == 0.0


def test_order_two_rejected():
    xyz, tets = W.kuhn_mesh(3, seed=0)
    with pytest.raises(Exception, match="aux_space 2 needs order 3 or 4"):
        aux.Solver(xyz, tets, 2, host_only=True, aux_space=2)
