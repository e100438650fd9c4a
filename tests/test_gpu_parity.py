"""GPU parity: the HIP path through the C ABI against the CPU oracle.

Bars (from the arithmetic):
* FP64 preconditioner application: relative 2-norm <= 1e-12 (the operator is
  a fixed composition of ~10^2 sparse passes; rounding-order differences stay
  near machine precision times its norm);
* CG in FP64 with the iteration count fixed to the oracle's: <= 1e-10; the
  free-running iteration count within +-1 of the oracle's;
* mixed mode (FP32 preconditioner): converged solution within 1e-7 of the
  FP64 oracle, iteration count within +-1 of the oracle's FP32 mode;
* determinism: repeated FP64 solves are bitwise identical.
"""
import numpy as np
import pytest
import torch

import oracle
import paper_1204_2586_amd as aux
import workloads as W

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def _case(k, n, jitter=0.0, kappa=None, seed=0):
    xyz, tets = W.kuhn_mesh(n, jitter=jitter, seed=seed)
    if kappa == "grf":
        kappa = np.exp(W.grf_log_kappa(xyz, tets, seed=1))
    elif kappa == "rand":
        kappa = np.exp(np.random.default_rng(3).normal(size=len(tets)))
    return xyz, tets, kappa


CASES = {
    "p2_n8": dict(k=2, n=8),                                   # the 8^3-cube P2 workload
    "p2_n10_jitter_rand": dict(k=2, n=10, jitter=0.2, kappa="rand"),
    "p3_n6_grf": dict(k=3, n=6, kappa="grf"),
    "p3_n5_jitter": dict(k=3, n=5, jitter=0.15),
    "p2_n3_single_level": dict(k=2, n=3),                      # n_H = 8: coarse solve only
    "p4_n4_jitter_rand": dict(k=4, n=4, jitter=0.2, kappa="rand"),
    "p4_n7": dict(k=4, n=7),                                   # 19,683 P^4 unknowns
}


@pytest.fixture(scope="module", params=list(CASES), ids=list(CASES))
def pair(request):
    c = CASES[request.param]
    xyz, tets, kappa = _case(c["k"], c["n"], c.get("jitter", 0.0), c.get("kappa"))
    print(f"[case {request.param}]", flush=True)
    lib = aux.Solver(xyz, tets, c["k"], kappa, device=DEV)
    orc = oracle.Problem(xyz, tets, c["k"], kappa).setup_amg()
    assert np.array_equal(lib.dof_keys(), orc.dof_keys())
    b = orc.load(W.manufactured_f)
    return lib, orc, b


def _t(x):
    return torch.tensor(np.asarray(x), dtype=torch.float64, device=DEV)


def _rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def test_matvec(pair):
    lib, orc, b = pair
    x = W.random_vector(lib.n, 5)
    y = lib.matvec(_t(x)).cpu().numpy()
    assert _rel(y, orc.csr("A") @ x) <= 1e-14


def test_apply_fp64(pair):
    lib, orc, b = pair
    lib.set_precision("fp64")
    for seed in (1, 2):
        r = W.random_vector(lib.n, seed)
        z = lib.apply(_t(r)).cpu().numpy()
        assert _rel(z, orc.apply(r)) <= 1e-12


def test_apply_mixed(pair):
    """The FP32 preconditioner agrees with the oracle's FP32 and FP64 forms to
    FP32 accuracy, and visibly differs from the FP64 form (so FP32 ran)."""
    lib, orc, b = pair
    r = W.random_vector(lib.n, 7)
    lib.set_precision("fp64")
    z64 = lib.apply(_t(r)).cpu().numpy()
    lib.set_precision("mixed")
    z = lib.apply(_t(r)).cpu().numpy()
    lib.set_precision("fp64")
    o32, o64 = orc.apply(r, fp32=True), orc.apply(r)
    print(f"mixed apply: vs oracle fp32 {_rel(z, o32):.2e}, vs oracle fp64 {_rel(z, o64):.2e}, "
          f"oracle fp32 vs fp64 {_rel(o32, o64):.2e}", flush=True)
    assert _rel(z, o32) <= 2e-6
    assert _rel(z, o64) <= 2e-6
    assert _rel(z, o64) > 1e-9 and _rel(z, z64) > 1e-9


def test_pcg_fixed_iterations_fp64(pair):
    lib, orc, b = pair
    lib.set_precision("fp64")
    x, it, rr, st = orc.pcg(b, tol=1e-8)
    assert st == 0
    u, info = lib.solve(_t(b), tol=0.0, maxit=it, check=False)
    assert info.iterations == it and info.status == -4
    assert _rel(u.cpu().numpy(), x) <= 1e-10
    assert abs(info.rel_residual - rr) <= 1e-4 * rr


def test_pcg_free_running_fp64(pair):
    lib, orc, b = pair
    lib.set_precision("fp64")
    x, it, rr, st = orc.pcg(b, tol=1e-8)
    u, info = lib.solve(_t(b), tol=1e-8)
    assert info.converged and abs(info.iterations - it) <= 1
    assert info.rel_residual <= 1e-8
    assert _rel(u.cpu().numpy(), x) <= 1e-7


def test_pcg_mixed(pair):
    lib, orc, b = pair
    lib.set_precision("mixed")
    x64, it64, _, _ = orc.pcg(b, tol=1e-8)
    x32, it32, _, _ = orc.pcg(b, tol=1e-8, fp32=True)
    u, info = lib.solve(_t(b), tol=1e-8)
    lib.set_precision("fp64")
    assert info.converged and abs(info.iterations - it32) <= 1
    assert _rel(u.cpu().numpy(), x64) <= 1e-7


def test_deterministic(pair):
    lib, orc, b = pair
    lib.set_precision("fp64")
    u1, i1 = lib.solve(_t(b), tol=1e-10)
    u2, i2 = lib.solve(_t(b), tol=1e-10)
    assert i1.iterations == i2.iterations
    assert torch.equal(u1, u2)


def test_kappa_grad(pair):
    lib, orc, b = pair
    u = W.random_vector(lib.n, 11)
    lam = W.random_vector(lib.n, 12)
    g = lib.kappa_grad(_t(u), _t(lam)).cpu().numpy()
    assert _rel(g, orc.kappa_grad(u, lam)) <= 1e-12


def test_status_codes():
    xyz, tets, _ = _case(2, 4)
    lib = aux.Solver(xyz, tets, 2, device=DEV)
    orc = oracle.Problem(xyz, tets, 2).setup_amg()
    b = orc.load(W.manufactured_f)
    u, info = lib.solve(_t(np.zeros(lib.n)), tol=1e-8)
    assert info.converged and info.iterations == 0 and not torch.any(u)
    u, info = lib.solve(_t(b), tol=1e-12, maxit=1, check=False)
    assert info.status == -4 and info.iterations == 1
    bad = b.copy()
    bad[2] = np.nan
    u, info = lib.solve(_t(bad), tol=1e-8, check=False)
    assert info.status == -6
    # initial guess: starting from the converged solution needs no iteration
    u, info = lib.solve(_t(b), tol=1e-8)
    u2, info2 = lib.solve(_t(b), tol=1e-6, u0=u)
    assert info2.iterations == 0 and torch.equal(u, u2)


@pytest.mark.parametrize("k,n", [(2, 8), (3, 5), (4, 4)])
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_batched_columns_match_single_solves(precision, k, n):
    print(f"[batched columns k={k} n={n} {precision}]", flush=True)
    xyz, tets, kappa = _case(k, n, jitter=0.2, kappa="rand")
    lib = aux.Solver(xyz, tets, k, kappa, device=DEV, precision=precision)
    orc = oracle.Problem(xyz, tets, k, kappa).setup_amg()
    nrhs = 12                                   # padded to 16 lanes internally
    F = np.stack([orc.load(W.fourier_f(r)) for r in range(nrhs)], axis=1)
    U, infos = lib.solve_batched(_t(F), tol=1e-8)
    for j in range(nrhs):
        u, info = lib.solve(_t(F[:, j]), tol=1e-8)
        assert infos[j].converged and abs(infos[j].iterations - info.iterations) <= 1
        assert _rel(U[:, j].cpu().numpy(), u.cpu().numpy()) <= 1e-8
        x, it, rr, st = orc.pcg(F[:, j], tol=1e-8, fp32=(precision == "mixed"))
        assert abs(infos[j].iterations - it) <= 1
        assert _rel(U[:, j].cpu().numpy(), x) <= 1e-7


def test_batched_fixed_iterations_fp64():
    xyz, tets, _ = _case(3, 5, jitter=0.1)
    lib = aux.Solver(xyz, tets, 3, device=DEV)
    orc = oracle.Problem(xyz, tets, 3).setup_amg()
    F = np.stack([orc.load(W.fourier_f(r)) for r in range(8)], axis=1)
    its = [orc.pcg(F[:, j], tol=1e-8)[1] for j in range(8)]
    m = min(its)
    U, infos = lib.solve_batched(_t(F), tol=0.0, maxit=m, check=False)
    for j in range(8):
        x, it, rr, st = orc.pcg(F[:, j], tol=0.0, maxit=m)
        assert infos[j].iterations == m
        assert _rel(U[:, j].cpu().numpy(), x) <= 1e-10


@pytest.mark.parametrize("k,n,jit,kap", [(3, 6, 0.0, "grf"), (2, 7, 0.2, "rand"), (3, 5, 0.15, None),
                                         (4, 4, 0.2, "rand"), (4, 3, 0.0, None)])
def test_matfree_operator(k, n, jit, kap):
    """The matrix-free element operator (MFMA) inside the preconditioner equals
    the assembled one: FP64 to rounding, FP32 to single precision."""
    xyz, tets, kappa = _case(k, n, jitter=jit, kappa=kap)
    lib = aux.Solver(xyz, tets, k, kappa, device=DEV)
    orc = oracle.Problem(xyz, tets, k, kappa).setup_amg()
    r = W.random_vector(lib.n, 3)
    for prec, tol in (("fp64", 1e-12), ("mixed", 2e-6)):
        lib.set_precision(prec)
        lib.set_operator("assembled")
        z_asm = lib.apply(_t(r)).cpu().numpy()
        lib.set_operator("matfree")
        z_mf = lib.apply(_t(r)).cpu().numpy()
        assert _rel(z_mf, z_asm) <= tol, prec
        assert _rel(z_mf, orc.apply(r, fp32=(prec == "mixed"))) <= tol, prec
    b = orc.load(W.manufactured_f)
    x, it, rr, st = orc.pcg(b, tol=1e-8, fp32=True)
    u, info = lib.solve(_t(b), tol=1e-8)
    assert info.converged and abs(info.iterations - it) <= 1
    x64, it64, _, _ = orc.pcg(b, tol=1e-8)
    assert _rel(u.cpu().numpy(), x64) <= 1e-7
    # FP64: the CG product is the element operator too; equal iteration counts
    # give the oracle's iterate to rounding
    lib.set_precision("fp64")
    u, info = lib.solve(_t(b), tol=0.0, maxit=it64, check=False)
    assert info.iterations == it64 and _rel(u.cpu().numpy(), x64) <= 1e-10


@pytest.mark.parametrize("precision,operator", [("fp64", "assembled"), ("mixed", "assembled"), ("mixed", "matfree"),
                                                ("fp64", "matfree")])
def test_graph_replay_matches_eager(precision, operator):
    """Each CG iteration replayed as a captured HIP graph gives bitwise the
    eager result; solves alternate with eager work and synchronisations."""
    xyz, tets, kappa = _case(2, 9, jitter=0.2, kappa="rand")
    # the layout window is fixed: the timing-based choice between the two
    # candidates may differ between instances, and the internal row order
    # sets the summation order of the inner products
    kw = dict(device=DEV, precision=precision, operator=operator, sell_window=4096)
    g = aux.Solver(xyz, tets, 2, kappa, graph=True, **kw)
    e = aux.Solver(xyz, tets, 2, kappa, graph=False, **kw)
    assert g.info.sell_window == e.info.sell_window == 4096
    orc = oracle.Problem(xyz, tets, 2, kappa).setup_amg()
    for r in range(3):
        b = orc.load(W.fourier_f(r))
        ug, ig = g.solve(_t(b), tol=1e-9)
        ue, ie = e.solve(_t(b), tol=1e-9)
        torch.cuda.synchronize()
        z = g.apply(_t(b))          # eager work between the replays
        assert ig.iterations == ie.iterations
        assert torch.equal(ug, ue)
        assert torch.equal(z, e.apply(_t(b)))


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_batched_graph_replay_matches_eager(precision):
    """Lock-step iterations replayed as a HIP graph give bitwise the eager
    result, also after the block width changes (buffers reallocated, graph
    recaptured) and changes back."""
    xyz, tets, kappa = _case(2, 7, jitter=0.2, kappa="rand")
    kw = dict(device=DEV, precision=precision, sell_window=4096)
    g = aux.Solver(xyz, tets, 2, kappa, graph=True, **kw)
    e = aux.Solver(xyz, tets, 2, kappa, graph=False, **kw)
    orc = oracle.Problem(xyz, tets, 2, kappa).setup_amg()
    F = np.stack([orc.load(W.fourier_f(r)) for r in range(12)], axis=1)
    for cols in (5, 12, 5):
        Fc = _t(np.ascontiguousarray(F[:, :cols]))
        Ug, ig = g.solve_batched(Fc, tol=1e-9)
        Ue, ie = e.solve_batched(Fc, tol=1e-9)
        torch.cuda.synchronize()
        assert [i.iterations for i in ig] == [i.iterations for i in ie]
        assert all(i.converged for i in ig)
        assert torch.equal(Ug, Ue)


@pytest.mark.parametrize("window", [0, 4096, 10 ** 9])
def test_index16_layout_equals_int32(window):
    """16-bit column offsets (narrow slots) and 32-bit side columns (wide
    slots) give bitwise the results of plain 32-bit columns."""
    xyz, tets, kappa = _case(2, 24, jitter=0.2, kappa="rand")     # 103,823 unknowns > 2^16
    kw = dict(device=DEV, sell_window=window)
    a = aux.Solver(xyz, tets, 2, kappa, sell_index16=True, **kw)
    b = aux.Solver(xyz, tets, 2, kappa, sell_index16=False, **kw)
    if window:
        assert a.info.sell_window == b.info.sell_window == window
    else:                                     # autotuned: the same windows for both
        a = aux.Solver(xyz, tets, 2, kappa, sell_index16=True, device=DEV, sell_window=int(a.info.sell_window))
        b = aux.Solver(xyz, tets, 2, kappa, sell_index16=False, device=DEV, sell_window=int(a.info.sell_window))
    if window == 4096:                        # every slice spans less than 2^16 columns
        assert a.info.sell_narrow_slices == a.info.sell_slices
    if window == 10 ** 9:                     # global length sort: both kinds of slices
        assert 0 < a.info.sell_narrow_slices < a.info.sell_slices
    assert b.info.sell_narrow_slices == 0
    orc = oracle.Problem(xyz, tets, 2, kappa).setup_amg()
    f = _t(orc.load(W.manufactured_f))
    r = _t(W.random_vector(a.n, 5))
    assert torch.equal(a.matvec(r), b.matvec(r))
    for prec in ("fp64", "mixed"):
        a.set_precision(prec)
        b.set_precision(prec)
        assert torch.equal(a.apply(r), b.apply(r))
        ua, ia = a.solve(f, tol=1e-9)
        ub, ib = b.solve(f, tol=1e-9)
        assert ia.iterations == ib.iterations and torch.equal(ua, ub)
    F = torch.stack([f, r], dim=1).contiguous()
    Ua, _ = a.solve_batched(F, tol=1e-9)
    Ub, _ = b.solve_batched(F, tol=1e-9)
    assert torch.equal(Ua, Ub)


@pytest.mark.parametrize("k,n,jit,kap", [(2, 10, 0.2, "rand"), (3, 6, 0.0, "grf")])
def test_fused_cycle_matches_stepwise(k, n, jit, kap):
    """The composite level operators (two passes per level) and the fused
    restricted residual give the step-by-step preconditioner up to rounding."""
    xyz, tets, kappa = _case(k, n, jitter=jit, kappa=kap)
    kw = dict(device=DEV, sell_window=4096)
    f_ = aux.Solver(xyz, tets, k, kappa, fuse_cycle=True, **kw)
    s_ = aux.Solver(xyz, tets, k, kappa, fuse_cycle=False, **kw)
    assert f_.info.nnz_restrict > 0 and s_.info.nnz_restrict == 0
    orc = oracle.Problem(xyz, tets, k, kappa).setup_amg()
    r = W.random_vector(f_.n, 11)
    for prec, tol in (("fp64", 1e-12), ("mixed", 2e-6)):
        f_.set_precision(prec)
        s_.set_precision(prec)
        zf = f_.apply(_t(r)).cpu().numpy()
        assert _rel(zf, s_.apply(_t(r)).cpu().numpy()) <= tol
        assert _rel(zf, orc.apply(r, fp32=(prec == "mixed"))) <= tol
    b = orc.load(W.manufactured_f)
    f_.set_precision("fp64")
    x, it, _, _ = orc.pcg(b, tol=1e-8)
    u, info = f_.solve(_t(b), tol=0.0, maxit=it, check=False)
    assert _rel(u.cpu().numpy(), x) <= 1e-10
    F = np.stack([b, r], axis=1)
    for prec in ("fp64", "mixed"):
        f_.set_precision(prec)
        s_.set_precision(prec)
        Uf, inf_ = f_.solve_batched(_t(F), tol=1e-9)
        Us, ins_ = s_.solve_batched(_t(F), tol=1e-9)
        for j in range(2):
            assert abs(inf_[j].iterations - ins_[j].iterations) <= 1
            assert _rel(Uf[:, j].cpu().numpy(), Us[:, j].cpu().numpy()) <= 1e-8


@pytest.mark.parametrize("k,n,lanes", [(2, 13, 1), (2, 13, 4), (2, 13, 32), (3, 9, 2), (3, 9, 8), (3, 9, 16),
                                         (2, 13, -1), (3, 9, -8)])
def test_cycle_operator_storage(k, n, lanes):
    """Every storage of the V-cycle's operators (row-split sliced ELL with L
    lanes per row, or CSR) gives the oracle's preconditioner to rounding;
    the meshes leave ragged last slices at every level."""
    print(f"[cycle storage k={k} n={n} lanes={lanes}]", flush=True)
    xyz, tets, kappa = _case(k, n, jitter=0.2, kappa="rand")
    lib = aux.Solver(xyz, tets, k, kappa, device=DEV, cycle_lanes=lanes, dense_cycle_rows=0)
    assert lib.info.dense_cycle_level == -1
    i = lib.info
    assert i.lanes_restrict == lanes and i.lanes_prolong == lanes
    assert all(i.lanes_down[l] == lanes and i.lanes_up[l] == lanes for l in range(i.levels - 1))
    orc = oracle.Problem(xyz, tets, k, kappa).setup_amg()
    r = W.random_vector(lib.n, 5)
    for prec, tol in (("fp64", 1e-12), ("mixed", 2e-6)):
        lib.set_precision(prec)
        assert _rel(lib.apply(_t(r)).cpu().numpy(), orc.apply(r, fp32=(prec == "mixed"))) <= tol, prec
    b = orc.load(W.manufactured_f)
    lib.set_precision("fp64")
    x, it, _, _ = orc.pcg(b, tol=1e-8)
    u, info = lib.solve(_t(b), tol=0.0, maxit=it, check=False)
    assert _rel(u.cpu().numpy(), x) <= 1e-10


@pytest.mark.parametrize("k,n,rows", [(2, 13, 0), (2, 13, 300), (2, 13, 1024), (2, 13, 8192), (3, 9, 1024),
                                       (3, 9, 100)])
def test_dense_cycle(k, n, rows):
    """The cycle below the first level of at most `rows` rows, formed as one
    dense matrix at setup, gives the oracle's preconditioner to rounding in
    the single-vector and the batched solve (rows = 8192 takes the whole
    cycle, 0 none)."""
    print(f"[dense cycle k={k} n={n} rows={rows}]", flush=True)
    xyz, tets, kappa = _case(k, n, jitter=0.2, kappa="rand")
    lib = aux.Solver(xyz, tets, k, kappa, device=DEV, dense_cycle_rows=rows)
    sizes = [r for r, _ in lib.levels]
    first = next((l for l in range(len(sizes) - 1) if sizes[l] <= rows), -1) if rows else -1
    assert lib.info.dense_cycle_level == first
    orc = oracle.Problem(xyz, tets, k, kappa).setup_amg()
    r = W.random_vector(lib.n, 9)
    for prec, tol in (("fp64", 1e-12), ("mixed", 2e-6)):
        lib.set_precision(prec)
        assert _rel(lib.apply(_t(r)).cpu().numpy(), orc.apply(r, fp32=(prec == "mixed"))) <= tol, prec
    b = orc.load(W.manufactured_f)
    lib.set_precision("fp64")
    x, it, _, _ = orc.pcg(b, tol=1e-8)
    u, info = lib.solve(_t(b), tol=0.0, maxit=it, check=False)
    assert _rel(u.cpu().numpy(), x) <= 1e-10
    F = np.stack([b, r], axis=1)
    for prec in ("fp64", "mixed"):
        lib.set_precision(prec)
        U, infos = lib.solve_batched(_t(F), tol=1e-8)
        for j in range(2):
            xj, itj, _, _ = orc.pcg(F[:, j], tol=1e-8, fp32=(prec == "mixed"))
            assert abs(infos[j].iterations - itj) <= 1
            assert _rel(U[:, j].cpu().numpy(), orc.pcg(F[:, j], tol=1e-8)[0]) <= 1e-7


@pytest.mark.parametrize("k,n,split", [(4, 7, 1), (2, 12, 0)])
def test_split_slices(k, n, split):
    """With 32-bit columns, wide slices (P4) are summed by two wavefronts each
    and narrow ones (P2) by one; either gives the oracle's operator,
    preconditioner and CG iterates to rounding."""
    print(f"[split slices k={k} n={n}]", flush=True)
    xyz, tets, kappa = _case(k, n, jitter=0.2, kappa="rand")
    lib = aux.Solver(xyz, tets, k, kappa, device=DEV, sell_index16=False)
    assert lib.info.sell_split == split and lib.info.sell_narrow_slices == 0
    orc = oracle.Problem(xyz, tets, k, kappa).setup_amg()
    r = W.random_vector(lib.n, 4)
    assert _rel(lib.matvec(_t(r)).cpu().numpy(), orc.csr("A") @ r) <= 1e-13
    for prec, tol in (("fp64", 1e-12), ("mixed", 2e-6)):
        lib.set_precision(prec)
        assert _rel(lib.apply(_t(r)).cpu().numpy(), orc.apply(r, fp32=(prec == "mixed"))) <= tol, prec
    b = orc.load(W.manufactured_f)
    lib.set_precision("fp64")
    x, it, _, _ = orc.pcg(b, tol=1e-8)
    u, info = lib.solve(_t(b), tol=0.0, maxit=it, check=False)
    assert _rel(u.cpu().numpy(), x) <= 1e-10


@pytest.mark.parametrize("nrhs", [5, 12, 32])
def test_batched_tiles_equal_slices(nrhs):
    """Block products from LDS-staged row tiles and from 64-row slices sum each
    row in the same order; only the grouping of the inner products' partial
    sums differs, so the lock-step solves agree to rounding."""
    xyz, tets, kappa = _case(2, 9, jitter=0.2, kappa="rand")
    kw = dict(device=DEV, sell_window=4096)
    a = aux.Solver(xyz, tets, 2, kappa, batch_tiles=2, **kw)
    b = aux.Solver(xyz, tets, 2, kappa, batch_tiles=0, **kw)
    orc = oracle.Problem(xyz, tets, 2, kappa).setup_amg()
    F = np.stack([orc.load(W.fourier_f(r)) for r in range(nrhs)], axis=1)
    for prec in ("fp64", "mixed"):
        a.set_precision(prec)
        b.set_precision(prec)
        Ua, ia = a.solve_batched(_t(F), tol=1e-9)
        Ub, ib = b.solve_batched(_t(F), tol=1e-9)
        assert min(a.info.batch_tile_rows) > 0 and max(b.info.batch_tile_rows) == 0
        for j in range(nrhs):
            assert ia[j].converged and abs(ia[j].iterations - ib[j].iterations) <= 1
            assert _rel(Ua[:, j].cpu().numpy(), Ub[:, j].cpu().numpy()) <= 1e-8


@pytest.mark.parametrize("k,n", [(2, 1), (3, 1), (2, 2), (3, 2)])
def test_degenerate_meshes(k, n):
    """One cube (no interior P^1 vertex: B is the P^k smoother alone) and two
    cubes per side (a single P^1 unknown, the coarse solve only)."""
    xyz, tets = W.kuhn_mesh(n)
    lib = aux.Solver(xyz, tets, k, device=DEV)
    orc = oracle.Problem(xyz, tets, k).setup_amg()
    assert lib.n == orc.n and lib.nH == orc.nH == (n - 1) ** 3
    r = W.random_vector(lib.n, 4)
    assert _rel(lib.apply(_t(r)).cpu().numpy(), orc.apply(r)) <= 1e-12
    b = orc.load(W.manufactured_f)
    x, it, _, st = orc.pcg(b, tol=1e-10)
    assert st == 0
    u, info = lib.solve(_t(b), tol=1e-10)
    assert info.converged and abs(info.iterations - it) <= 1
    assert _rel(u.cpu().numpy(), x) <= 1e-9
    lib.set_precision("mixed")
    u, info = lib.solve(_t(b), tol=1e-8)
    assert info.converged and _rel(u.cpu().numpy(), x) <= 1e-7
    U, infos = lib.solve_batched(_t(np.stack([b, 2 * b, r], axis=1)), tol=1e-8)
    assert all(i.converged for i in infos)
    assert _rel(U[:, 1].cpu().numpy(), 2 * x) <= 1e-7


@pytest.mark.parametrize("nu", [1, 3])
@pytest.mark.parametrize("k,n", [(2, 8), (3, 5)])
def test_smoothing_sweeps(k, n, nu):
    """nu l1-Jacobi sweeps before and after the coarse correction (the paper
    ran one of each, Remark 6.1) against the oracle with the same nu: the
    application in FP64 and FP32, CG at the oracle's iteration count, and the
    batched form."""
    print(f"[smoothing sweeps nu={nu} k={k} n={n}]", flush=True)
    xyz, tets, kappa = _case(k, n, jitter=0.2, kappa="rand")
    orc = oracle.Problem(xyz, tets, k, kappa).setup_amg(nu=nu)
    b = orc.load(W.manufactured_f)
    lib = aux.Solver(xyz, tets, k, kappa, nu=nu, device=DEV)
    r = W.random_vector(lib.n, 9)
    assert _rel(lib.apply(_t(r)).cpu().numpy(), orc.apply(r)) <= 1e-12
    x, it, rr, st = orc.pcg(b, tol=1e-8)
    u, info = lib.solve(_t(b), tol=0.0, maxit=it, check=False)
    assert st == 0 and info.iterations == it
    assert _rel(u.cpu().numpy(), x) <= 1e-10
    lib.set_precision("mixed")
    assert _rel(lib.apply(_t(r)).cpu().numpy(), orc.apply(r, fp32=True)) <= 2e-6
    F = np.stack([orc.load(W.fourier_f(c)) for c in range(6)], axis=1)
    U, infos = lib.solve_batched(_t(F), tol=1e-8)
    for j in range(6):
        xj, itj, _, _ = orc.pcg(F[:, j], tol=1e-8, fp32=True)
        assert infos[j].converged and abs(infos[j].iterations - itj) <= 1
        assert _rel(U[:, j].cpu().numpy(), xj) <= 1e-7


@pytest.mark.parametrize("opts", [dict(theta=0.25), dict(coarse_max=500), dict(max_levels=2, theta=0.5),
                                  dict(seed=7), dict(use_torch_allocator=False)],
                         ids=["theta0.25", "coarse500", "levels2", "pmis_seed7", "hipmalloc"])
def test_hierarchy_and_allocation_options(opts):
    """Non-default AMG options (a coarsest level of a few hundred rows solved
    densely, a level cap, another PMIS seed) against the oracle built with
    the same options; device buffers from hipMalloc instead of the torch
    allocator give the same bits."""
    print(f"[options {opts}]", flush=True)
    xyz, tets, kappa = _case(2, 10, jitter=0.2, kappa="rand")
    amg = {k: v for k, v in opts.items() if k != "use_torch_allocator"}
    orc = oracle.Problem(xyz, tets, 2, kappa).setup_amg(**amg)
    # a bitwise comparison of two handles needs layouts chosen by rule, not
    # by timing (a fixed window: every layout choice is then rule-based)
    fixed = dict(sell_window=1 << 30) if opts.get("use_torch_allocator") is False else {}
    lib = aux.Solver(xyz, tets, 2, kappa, device=DEV, **opts, **fixed)
    assert lib.info.levels == orc.nlev
    b = orc.load(W.manufactured_f)
    r = W.random_vector(lib.n, 10)
    assert _rel(lib.apply(_t(r)).cpu().numpy(), orc.apply(r)) <= 1e-12
    x, it, rr, st = orc.pcg(b, tol=1e-8)
    u, info = lib.solve(_t(b), tol=0.0, maxit=it, check=False)
    assert st == 0 and info.iterations == it and _rel(u.cpu().numpy(), x) <= 1e-10
    if opts.get("use_torch_allocator") is False:
        ref = aux.Solver(xyz, tets, 2, kappa, device=DEV, **fixed)
        u2, _ = ref.solve(_t(b), tol=0.0, maxit=it, check=False)
        assert torch.equal(u, u2)


@pytest.mark.parametrize("k,n", [(2, 10), (3, 6)])
def test_batched_orders_agree(k, n):
    """The batched and block solves in the spatially ordered layout (Morton
    curve, die ranges; the default) and in the single-vector order give the
    same columns up to rounding: at a fixed iteration count within 1e-10."""
    print(f"[batched orders k={k} n={n}]", flush=True)
    xyz, tets, kappa = _case(k, n, jitter=0.2, kappa="rand")
    F = _t(np.stack([W.random_vector(aux.Solver(xyz, tets, k, kappa, host_only=True).n, 20 + j)
                     for j in range(6)], axis=1))
    out = {}
    for order in (0, 1):
        lib = aux.Solver(xyz, tets, k, kappa, device=DEV, batch_order=order)
        U, infos = lib.solve_batched(F, tol=0.0, maxit=6, check=False)
        Ub, binfos = lib.solve_block(F, tol=0.0, maxit=4, check=False)
        out[order] = (U.cpu().numpy(), Ub.cpu().numpy())
        assert all(i.iterations == 6 for i in infos) and all(i.iterations == 4 for i in binfos)
        lib.close()
    for a, b in zip(out[0], out[1]):
        assert np.linalg.norm(a - b) <= 1e-10 * np.linalg.norm(b)
