"""GPU parity of the intermediate auxiliary space (Remark 6.2, aux_space = 2):
P^3 / P^4 with P^2 on the same mesh as the auxiliary space, its problem
solved by one application of the P^2 handle's own preconditioner, against
the oracle's nested preconditioner (tests/test_oracle_nested.py pins it).

Bars as in tests/test_gpu_parity.py: FP64 application <= 1e-12; CG at the
oracle's iteration count <= 1e-10, free-running count within +-1; the FP32
preconditioner within 2e-6 of the oracle's FP32 and FP64 forms and visibly
different from the GPU's FP64 form.
"""
import numpy as np
import pytest
import torch

import oracle
import paper_1204_2586_amd as aux
import workloads as W

pytestmark = pytest.mark.gpu

DEV = "cuda:0"

CASES = {
    "p3_n5_jitter": dict(k=3, n=5, jitter=0.15),
    "p3_n6_grf_cmax8": dict(k=3, n=6, kappa="grf", coarse_max=8),
    "p4_n4_rand": dict(k=4, n=4, jitter=0.2, kappa="rand"),
    "p4_n6_cmax8": dict(k=4, n=6, coarse_max=8),
}


def _kappa(kind, xyz, tets, seed=1):
    if kind == "grf":
        return np.exp(W.grf_log_kappa(xyz, tets, seed=seed))
    if kind == "rand":
        return np.exp(np.random.default_rng(seed + 2).normal(size=len(tets)))
    return None


@pytest.fixture(scope="module", params=list(CASES), ids=list(CASES))
def pair(request):
    c = CASES[request.param]
    print(f"[nested case {request.param}]", flush=True)
    xyz, tets = W.kuhn_mesh(c["n"], jitter=c.get("jitter", 0.0), seed=0)
    kappa = _kappa(c.get("kappa"), xyz, tets)
    cm = c.get("coarse_max", 100)
    lib = aux.Solver(xyz, tets, c["k"], kappa, device=DEV, aux_space=2, coarse_max=cm)
    orc = oracle.Problem(xyz, tets, c["k"], kappa).setup_nested(coarse_max=cm)
    assert lib.info.aux_space == 2
    b = orc.load(W.manufactured_f)
    return lib, orc, b, (xyz, tets, c, cm)


def _t(x):
    return torch.tensor(np.asarray(x), dtype=torch.float64, device=DEV)


def _rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def test_apply_fp64(pair):
    lib, orc, b, _ = pair
    lib.set_precision("fp64")
    for seed in (1, 2):
        r = W.random_vector(lib.n, seed)
        z = lib.apply(_t(r)).cpu().numpy()
        assert _rel(z, orc.apply_nested(r)) <= 1e-12


def test_apply_mixed(pair):
    lib, orc, b, _ = pair
    r = W.random_vector(lib.n, 7)
    lib.set_precision("fp64")
    z64 = lib.apply(_t(r)).cpu().numpy()
    lib.set_precision("mixed")
    z = lib.apply(_t(r)).cpu().numpy()
    lib.set_precision("fp64")
    o32, o64 = orc.apply_nested(r, fp32=True), orc.apply_nested(r)
    assert _rel(z, o32) <= 2e-6
    assert _rel(z, o64) <= 2e-6
    assert _rel(z, z64) > 1e-9


def test_pcg_fixed_iterations_fp64(pair):
    lib, orc, b, _ = pair
    lib.set_precision("fp64")
    x, it, rr, st = orc.pcg_nested(b, tol=1e-8)
    assert st == 0
    u, info = lib.solve(_t(b), tol=0.0, maxit=it, check=False)
    assert info.iterations == it
    assert _rel(u.cpu().numpy(), x) <= 1e-10


def test_pcg_free_running_and_mixed(pair):
    lib, orc, b, _ = pair
    x, it, _, _ = orc.pcg_nested(b, tol=1e-8)
    _, it32, _, _ = orc.pcg_nested(b, tol=1e-8, fp32=True)
    lib.set_precision("fp64")
    u, info = lib.solve(_t(b), tol=1e-8)
    assert info.converged and abs(info.iterations - it) <= 1 and info.rel_residual <= 1e-8
    assert _rel(u.cpu().numpy(), x) <= 1e-7
    lib.set_precision("mixed")
    u, info = lib.solve(_t(b), tol=1e-8)
    lib.set_precision("fp64")
    assert info.converged and abs(info.iterations - it32) <= 1
    assert _rel(u.cpu().numpy(), x) <= 1e-7


def test_matfree_operator(pair):
    lib, orc, b, _ = pair
    lib.set_precision("fp64")
    lib.set_operator("matfree")
    r = W.random_vector(lib.n, 3)
    z = lib.apply(_t(r)).cpu().numpy()
    lib.set_operator("assembled")
    assert _rel(z, orc.apply_nested(r)) <= 1e-12


def test_fgmres(pair):
    lib, orc, b, _ = pair
    lib.set_precision("fp64")
    x, info, hist = lib.fgmres(_t(b), tol=1e-8, restart=30)
    assert info.converged
    xo = orc.pcg_nested(b, tol=1e-12)[0]
    assert _rel(x.cpu().numpy(), xo) <= 1e-6


def test_batched_needs_p1_space(pair):
    lib, orc, b, _ = pair
    F = torch.zeros(lib.n, 2, dtype=torch.float64, device=DEV)
    with pytest.raises(Exception, match="P\\^1 auxiliary space"):
        lib.solve_batched(F)


def test_set_kappa(pair):
    """A new coefficient reaches both the P^k operator (and the composite
    restriction with I_2) and the P^2 handle."""
    lib, orc, b, (xyz, tets, c, cm) = pair
    kappa2 = np.exp(np.random.default_rng(17).normal(size=len(tets)))
    lib.set_kappa(kappa2)
    orc2 = oracle.Problem(xyz, tets, c["k"], kappa2).setup_nested(coarse_max=cm)
    lib.set_precision("fp64")
    r = W.random_vector(lib.n, 9)
    z = lib.apply(_t(r)).cpu().numpy()
    assert _rel(z, orc2.apply_nested(r)) <= 1e-12
    x, it, _, _ = orc2.pcg_nested(b, tol=1e-8)
    u, info = lib.solve(_t(b), tol=1e-8)
    assert abs(info.iterations - it) <= 1


@pytest.mark.parametrize("k,n", [(4, 24), (3, 32)])
def test_full_size_fewer_iterations(k, n):
    """P4 on 24^3 and P3 on 32^3 cubes (857,375 unknowns each),
    kappa = exp(GRF): the intermediate space converges to the same solution
    in fewer CG iterations than the P^1 space (timings printed)."""
    xyz, tets = W.kuhn_mesh(n, jitter=0.0, seed=0)
    kappa = np.exp(W.grf_log_kappa(xyz, tets, seed=1))
    out = {}
    for space in (1, 2):
        s = aux.Solver(xyz, tets, k, kappa, device=DEV, precision="mixed", aux_space=space)
        f = torch.tensor(s.load(W.manufactured_f), dtype=torch.float64, device=DEV)
        s.solve(f, tol=1e-8)
        torch.cuda.synchronize()
        import time
        t0 = time.perf_counter()
        u, info = s.solve(f, tol=1e-8)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3
        res = float(torch.linalg.norm(f - s.matvec(u)) / torch.linalg.norm(f))
        out[space] = (u, info.iterations, ms, res)
        print(f"[nested full size] P{k} n={n} aux_space={space}: {info.iterations} iterations, {ms:.2f} ms, "
              f"true residual {res:.2e}", flush=True)
        del s
    assert out[2][1] < out[1][1]
    assert out[1][3] <= 1.01e-8 and out[2][3] <= 1.01e-8
    u1, u2 = out[1][0], out[2][0]
    assert float(torch.linalg.norm(u1 - u2) / torch.linalg.norm(u1)) <= 1e-6
