"""A new coefficient on the same mesh (aux_set_kappa): the device assembly
against a new setup and against the oracle.

* The operators the device assembles for kappa_2 on a handle set up with
  kappa_1 (A_h, A_H, the l1 norms behind the smoother) equal those of a new
  setup with kappa_2 bit for bit (the same arithmetic in the same order), so
  the AMG hierarchy (C/F splits, interpolation, coarse operators) is the same,
  and with rule-based layouts every application and solve is bitwise equal.
* Against the oracle for kappa_2: apply 1e-12, CG at the oracle's iteration
  count 1e-10, mixed mode 1e-7; the matrix-free operator and the batched
  solve after the update; several updates in a row.
* A failed update leaves the handle refusing solves until the next update.
"""
import time

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
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b)))


def _kappas(xyz, tets, seeds):
    return [np.exp(W.grf_log_kappa(xyz, tets, seed=s)) for s in seeds]


@pytest.mark.parametrize("k,n", [(2, 8), (3, 5), (4, 4)])
def test_set_kappa_equals_new_setup(k, n):
    print(f"[set_kappa vs new setup P{k} {n}^3]", flush=True)
    xyz, tets = W.kuhn_mesh(n, jitter=0.2, seed=0)
    k1, k2 = _kappas(xyz, tets, (1, 2))
    kw = dict(device=DEV, sell_window=1 << 30)           # rule-based layouts: bitwise comparable
    a = aux.Solver(xyz, tets, k, k1, **kw)
    a.set_kappa(k2)
    b = aux.Solver(xyz, tets, k, k2, **kw)
    for which in ("A", "AH"):
        ma, mb = a.export_csr(which), b.export_csr(which)
        assert np.array_equal(ma.indptr, mb.indptr) and np.array_equal(ma.indices, mb.indices)
        assert np.array_equal(ma.data, mb.data), which           # bitwise
    assert a.info.levels == b.info.levels
    for l in range(a.info.levels - 1):
        assert np.array_equal(a.export_cf(l), b.export_cf(l))
        pa, pb = a.export_csr("P", l), b.export_csr("P", l)
        assert np.array_equal(pa.data, pb.data)
    r = _t(W.random_vector(a.n, 3))
    assert torch.equal(a.apply(r), b.apply(r))
    f = _t(W.random_vector(a.n, 4))
    ua, ia = a.solve(f, tol=1e-9)
    ub, ib = b.solve(f, tol=1e-9)
    assert ia.iterations == ib.iterations and torch.equal(ua, ub)
    for prec in ("mixed",):
        a.set_precision(prec)
        b.set_precision(prec)
        assert torch.equal(a.apply(r), b.apply(r))


@pytest.mark.parametrize("lanes", [4, -8])
def test_set_kappa_forced_storage(lanes):
    """The V-cycle's level operators in a forced storage (row-split ELL with
    4 lanes per row, built again on the device from the new device-built
    operators; or CSR with 8 lanes), no dense sub-cycle: the update equals a
    new setup bitwise (composite operators, applications in both
    precisions, CG)."""
    print(f"[set_kappa forced storage {lanes}]", flush=True)
    xyz, tets = W.kuhn_mesh(10, jitter=0.2, seed=0)
    k1, k2 = _kappas(xyz, tets, (1, 2))
    kw = dict(device=DEV, sell_window=1 << 30, cycle_lanes=lanes, coarse_max=20, dense_cycle_rows=0)
    a = aux.Solver(xyz, tets, 2, k1, **kw)
    a.set_kappa(k2)
    b = aux.Solver(xyz, tets, 2, k2, **kw)
    assert a.info.levels == b.info.levels >= 3
    assert list(a.info.level_nnz_up[:a.info.levels]) == list(b.info.level_nnz_up[:b.info.levels])
    for l in range(a.info.levels - 1):
        for which in ("down", "up"):
            ma, mb = a.export_csr(which, l), b.export_csr(which, l)
            assert np.array_equal(ma.indptr, mb.indptr) and np.array_equal(ma.indices, mb.indices)
            assert np.array_equal(ma.data, mb.data), (which, l)
    r = _t(W.random_vector(a.n, 5))
    for prec in ("fp64", "mixed"):
        a.set_precision(prec)
        b.set_precision(prec)
        assert torch.equal(a.apply(r), b.apply(r)), prec
    f = _t(W.random_vector(a.n, 6))
    ua, ia = a.solve(f, tol=1e-9)
    ub, ib = b.solve(f, tol=1e-9)
    assert ia.iterations == ib.iterations and torch.equal(ua, ub)


def test_failed_update_refuses_solves(monkeypatch):
    """An update that fails after the old coefficient's device data are
    released (the device allocator refuses every allocation after the first
    dozen of the update, which lands inside the AMG build) leaves the handle
    refusing applications and solves with AUX_ESTATE instead of running on
    missing data; the next update restores it, bitwise equal to a new setup."""
    print("[set_kappa failure path]", flush=True)
    xyz, tets = W.kuhn_mesh(8, jitter=0.2, seed=0)
    k1, k2 = _kappas(xyz, tets, (1, 2))
    kw = dict(device=DEV, sell_window=1 << 30)
    s = aux.Solver(xyz, tets, 2, k1, **kw)
    s.set_kappa(k2)                                          # builds the assembly maps
    real = torch.cuda.caching_allocator_alloc
    calls = [0]

    def refusing(n, d, st):
        calls[0] += 1
        return 0 if calls[0] > 12 else real(n, d, st)

    monkeypatch.setattr(torch.cuda, "caching_allocator_alloc", refusing)
    with pytest.raises(aux.AuxError, match="AUX_ENOMEM"):
        s.set_kappa(k1)
    monkeypatch.setattr(torch.cuda, "caching_allocator_alloc", real)
    assert calls[0] > 12
    r = _t(W.random_vector(s.n, 3))
    with pytest.raises(aux.AuxError, match="AUX_ESTATE"):
        s.apply(r)
    with pytest.raises(aux.AuxError, match="AUX_ESTATE"):
        s.solve(_t(W.random_vector(s.n, 4)), tol=1e-8)
    s.set_kappa(k1)
    b = aux.Solver(xyz, tets, 2, k1, **kw)
    assert torch.equal(s.apply(r), b.apply(r))


def test_set_kappa_against_oracle_and_forms():
    print("[set_kappa against the oracle]", flush=True)
    xyz, tets = W.kuhn_mesh(8, jitter=0.2, seed=1)
    ks = _kappas(xyz, tets, (3, 4, 5))
    s = aux.Solver(xyz, tets, 2, ks[0], device=DEV, precision="mixed")
    for kap in ks[1:]:                                       # two updates in a row
        s.set_kappa(kap)
        orc = oracle.Problem(xyz, tets, 2, kap).setup_amg()
        assert np.array_equal(s.dof_keys(), orc.dof_keys())
        b = orc.load(W.manufactured_f)
        r = W.random_vector(s.n, 9)
        s.set_precision("fp64")
        assert _rel(s.apply(_t(r)).cpu().numpy(), orc.apply(r)) <= 1e-12
        x, it, rr, st = orc.pcg(b, tol=1e-8)
        u, info = s.solve(_t(b), tol=0.0, maxit=it, check=False)
        assert info.iterations == it and _rel(u.cpu().numpy(), x) <= 1e-10
        s.set_precision("mixed")
        u, info = s.solve(_t(b), tol=1e-8)
        assert info.converged and _rel(u.cpu().numpy(), x) <= 1e-7
        # the matrix-free operator (weights refreshed) and the batched solve
        s.set_operator("matfree")
        s.set_precision("fp64")
        assert _rel(s.apply(_t(r)).cpu().numpy(), orc.apply(r)) <= 1e-12
        s.set_operator("assembled")
        s.set_precision("mixed")
        F = np.stack([orc.load(W.fourier_f(c)) for c in range(3)], axis=1)
        U, infos = s.solve_batched(_t(F), tol=1e-8)
        for j in range(3):
            xj, _, _, _ = orc.pcg(F[:, j], tol=1e-10)
            assert infos[j].converged and _rel(U[:, j].cpu().numpy(), xj) <= 1e-7
        g = s.kappa_grad(_t(x), _t(x))
        assert _rel(g.cpu().numpy(), orc.kappa_grad(x, x)) <= 1e-12


def test_set_kappa_time_at_full_size():
    """P2 48^3 jittered: a coefficient update against a new setup (time
    printed; the operators checked bitwise against the new setup's)."""
    print("[set_kappa P2 48^3]", flush=True)
    xyz, tets = W.kuhn_mesh(48, jitter=0.2, seed=0)
    k1, k2 = _kappas(xyz, tets, (1, 2))
    t0 = time.perf_counter()
    a = aux.Solver(xyz, tets, 2, k1, device=DEV)
    t_setup = time.perf_counter() - t0
    a.set_kappa(k2)                                          # builds the assembly maps once
    t0 = time.perf_counter()
    a.set_kappa(k1)
    t_update = time.perf_counter() - t0
    b = aux.Solver(xyz, tets, 2, k1, device=DEV)
    assert np.array_equal(a.export_csr("A").data, b.export_csr("A").data)
    print(f"setup {t_setup:.2f} s, coefficient update {t_update:.2f} s "
          f"(library: {a.info.setup_seconds:.2f} s)", flush=True)
    f = _t(b.load(W.manufactured_f))
    ua, ia = a.solve(f, tol=1e-8)
    ub, ib = b.solve(f, tol=1e-8)
    assert abs(ia.iterations - ib.iterations) <= 1 and _rel(ua.cpu().numpy(), ub.cpu().numpy()) <= 1e-7
