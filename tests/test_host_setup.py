"""Host setup of the GPU library against the oracle (no GPU needed).

The library's C++ setup and the oracle are independent implementations of
the same definitions: the dof numbering, A_h, A_H, I_P, the l1 norms, the
load vector, the PMIS splittings and the whole AMG hierarchy must agree.
"""
import numpy as np
import pytest

import oracle
import paper_1204_2586_amd as aux
import workloads as W


def _rel(a, b):
    return abs(a - b).max() / max(abs(b).max(), 1e-300)


CASES = [(2, 6, 0.2, None), (3, 5, 0.15, "grf"), (2, 10, 0.0, None), (2, 9, 0.2, "rand"), (4, 4, 0.2, "rand")]


@pytest.fixture(scope="module", params=CASES, ids=lambda c: f"P{c[0]}-n{c[1]}-j{c[2]}-{c[3]}")
def pair(request):
    k, n, jit, kap = request.param
    xyz, tets = W.kuhn_mesh(n, jitter=jit, seed=0)
    kappa = None
    if kap == "grf":
        kappa = np.exp(W.grf_log_kappa(xyz, tets, seed=1))
    elif kap == "rand":
        kappa = np.exp(np.random.default_rng(2).normal(size=len(tets)))
    lib = aux.Solver(xyz, tets, k, kappa, host_only=True)
    orc = oracle.Problem(xyz, tets, k, kappa).setup_amg()
    return lib, orc


def test_dofs_and_operators(pair):
    lib, orc = pair
    assert lib.n == orc.n and lib.nH == orc.nH
    assert np.array_equal(lib.dof_keys(), orc.dof_keys())
    for name in ("A", "AH", "IP"):
        a, b = lib.export_csr(name), orc.csr(name)
        assert a.shape == b.shape
        assert _rel(a, b) < 1e-13, name
    assert _rel(lib.export_csr("IP"), orc.csr("IP")) == 0.0


def test_dof_xyz_reproduced_by_linear_transfer(pair):
    """Node positions: I_P carries a linear function at the P^1 vertices to its
    values at the P^k nodes (Sec. 2), so rows whose vertices are all interior
    reproduce g(x_i) for g linear."""
    lib, orc = pair
    X = lib.dof_xyz()
    assert X.shape == (lib.n, 3)
    interior = np.flatnonzero(np.all((orc.xyz > 1e-12) & (orc.xyz < 1 - 1e-12), axis=1))
    assert len(interior) == lib.nH
    coef = np.array([0.3, -1.7, 2.2])
    g = orc.xyz[interior] @ coef + 0.5
    IP = orc.csr("IP")
    full = np.isclose(np.asarray(IP.sum(axis=1)).ravel(), 1.0)
    assert full.sum() > lib.n // 8          # enough rows away from the boundary to test
    assert np.max(np.abs((IP @ g)[full] - (X[full] @ coef + 0.5))) < 1e-12
    # nodes lie inside the cube, vertices of the key averaged
    assert np.all((X > 0) & (X < 1))


def test_load_vector(pair):
    lib, orc = pair
    b1, b2 = lib.load(W.manufactured_f), orc.load(W.manufactured_f)
    assert np.max(np.abs(b1 - b2)) < 1e-13 * np.max(np.abs(b2))


def test_load_many_matches_oracle_per_column(pair):
    lib, orc = pair
    rs = [0, 5, 9]
    B = lib.load_many(W.fourier_fields(rs), len(rs), chunk=37, threads=3)
    assert B.shape == (lib.n, 3)
    for c, r in enumerate(rs):
        b = orc.load(W.fourier_f(r))
        assert np.max(np.abs(B[:, c] - b)) < 1e-13 * np.max(np.abs(b))


def test_amg_hierarchy_identical(pair):
    lib, orc = pair
    assert lib.info.levels == orc.nlev and lib.info.ncoarse == orc.ncoarse
    for l in range(orc.nlev - 1):
        assert np.array_equal(lib.export_cf(l), orc.level_cf(l)), l
        assert _rel(lib.export_csr("P", l), orc.csr("P", l)) < 1e-12
        assert _rel(lib.export_csr("Alev", l + 1), orc.csr("Alev", l + 1)) < 1e-12


def test_operator_complexity_reported(pair):
    lib, orc = pair
    tot = sum(orc.csr("Alev", l).nnz for l in range(orc.nlev))
    assert abs(lib.info.amg_complexity - tot / orc.nnz_AH) < 1e-12
    assert abs(lib.info.op_complexity - (orc.nnz_A + tot) / orc.nnz_A) < 1e-12


@pytest.mark.parametrize("theta,coarse_max,max_levels,seed", [(0.25, 100, 25, 0), (0.8, 20, 25, 7),
                                                              (0.5, 100, 2, 0), (0.8, 500, 25, 123)])
def test_hierarchy_options_identical(theta, coarse_max, max_levels, seed):
    """The strength threshold, the coarsest size, the level cap and the PMIS
    seed give the oracle's hierarchy level by level."""
    xyz, tets = W.kuhn_mesh(10, jitter=0.2, seed=0)
    lib = aux.Solver(xyz, tets, 2, host_only=True, theta=theta, coarse_max=coarse_max, max_levels=max_levels,
                     seed=seed)
    orc = oracle.Problem(xyz, tets, 2).setup_amg(theta=theta, coarse_max=coarse_max, max_levels=max_levels,
                                                 seed=seed)
    assert lib.info.levels == orc.nlev and lib.info.ncoarse == orc.ncoarse
    assert orc.nlev <= max_levels and (orc.ncoarse <= coarse_max or orc.nlev == max_levels)
    for l in range(orc.nlev - 1):
        assert np.array_equal(lib.export_cf(l), orc.level_cf(l)), l
        assert _rel(lib.export_csr("P", l), orc.csr("P", l)) < 1e-12
        assert _rel(lib.export_csr("Alev", l + 1), orc.csr("Alev", l + 1)) < 1e-12
