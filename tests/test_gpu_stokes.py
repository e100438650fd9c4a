"""GPU Stokes path (Hood-Taylor P^k-P^{k-1}, k = 2, 3, 4; Sec. 5): the saddle-point operator,
the block triangular preconditioner Q_t and FGMRES with Q_t, through the C
ABI against the oracle's.

Bars (from the arithmetic):
* operator [A B^T; B 0]: FP64 products in another summation order, 1e-13;
* Q_t: the pressure mass CG runs the same steps as the oracle's (step counts
  within one); at equal counts Q_t r agrees to 1e-10 (FP64, rounding of a
  few hundred operations amplified by the mass CG and B), otherwise to the
  mass CG's own tolerance 1e-6 propagated, 1e-5; in mixed mode the FP32
  apply bar 2e-6, and the velocity part visibly differs from FP64;
* FGMRES: at a fixed step count the iterate within 1e-8 and the residual
  history within 1e-8 ||r_0|| of the oracle's; free-running to 1e-8, the
  step count within +-1 of the oracle's (FP64 against FP64, mixed against
  the oracle's FP32-preconditioner form), the true residual at the
  tolerance; in FP64 at equal step counts the solution within 1e-8 of the
  oracle's (pressure modulo constants); against the oracle's 1e-12 solve
  the velocity within 1e-6 and the pressure within 1e-3 (the residual bound
  reaches the pressure through the discrete inf-sup constant, which scales
  like the mesh size here: 3e-5 to 6e-5 measured);
* full size P2 48^3 (jittered): converged to 1e-8 with the true residual
  recomputed by the operator, B^T 1 = 0, and the growth of the step count
  from 16^3 within 1.15 times that of CG with the same A-block
  preconditioner (Q_t adds no mesh dependence of its own: S ~ M_p is
  spectrally equivalent to the Schur complement uniformly in h); P3-P2 on
  32^3 cubes (2.85M unknowns) converged with its true residual.
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
    "p2_n6_jitter": dict(k=2, n=6, jitter=0.2, kappa=False),
    "p2_n8_rand": dict(k=2, n=8, jitter=0.0, kappa=True),
    "p3_n4_jitter": dict(k=3, n=4, jitter=0.2, kappa=False),
    "p4_n3_rand": dict(k=4, n=3, jitter=0.2, kappa=True),
}


def _t(x):
    return torch.tensor(np.asarray(x), dtype=torch.float64, device=DEV)


def _rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b)))


def _rhs(P):
    return np.concatenate([P.load(W.stokes_f(c)) for c in range(3)] + [np.zeros(P.np)])


def _p_mod_const(x, m):
    p = np.asarray(x[3 * m:])
    return p - p.mean()


@pytest.fixture(scope="module", params=list(CASES), ids=list(CASES))
def pair(request):
    c = CASES[request.param]
    print(f"[stokes {request.param}]", flush=True)
    xyz, tets = W.kuhn_mesh(c["n"], jitter=c["jitter"], seed=0)
    kappa = np.exp(np.random.default_rng(5).normal(size=len(tets))) if c["kappa"] else None
    lib = aux.Solver(xyz, tets, c["k"], kappa, device=DEV)
    orc = oracle.Problem(xyz, tets, c["k"], kappa).setup_amg().stokes_setup()
    assert lib.stokes_setup() == orc.np
    assert np.array_equal(lib.dof_keys(), orc.dof_keys())
    assert np.array_equal(lib.stokes_pressure_keys(), orc.pressure_keys())
    return lib, orc


def test_operator(pair):
    lib, orc = pair
    x = W.random_vector(3 * lib.n + lib.n_p, 1)
    yo = orc.stokes_operator(x)
    for op in ("assembled", "matfree"):
        lib.set_operator(op)
        y = lib.stokes_operator(_t(x)).cpu().numpy()
        assert _rel(y, yo) <= (1e-13 if op == "assembled" else 1e-12), op
    lib.set_operator("assembled")
    # constants are the pressure null space: F [0; 1] = [B^T 1; 0] = 0
    e = np.zeros(3 * lib.n + lib.n_p)
    e[3 * lib.n:] = 1.0
    y = lib.stokes_operator(_t(e)).cpu().numpy()
    assert np.max(np.abs(y)) <= 1e-14 * np.max(np.abs(yo))


def test_qt(pair):
    lib, orc = pair
    r = W.random_vector(3 * lib.n + lib.n_p, 2)
    for prec, fp32 in (("fp64", False), ("mixed", True)):
        lib.set_precision(prec)
        z, k = lib.stokes_qt(_t(r))
        zo, ko = orc.stokes_qt(r, fp32=fp32, steps=True)
        z = z.cpu().numpy()
        print(f"{prec}: mass CG steps {k} (oracle {ko}), Q_t rel diff {_rel(z, zo):.2e}", flush=True)
        assert abs(k - ko) <= 1
        if prec == "fp64":
            assert _rel(z, zo) <= (1e-10 if k == ko else 1e-5)
        else:
            # FP32 inside B: the apply bar of the FP32 preconditioner
            assert _rel(z, zo) <= 2e-6
            nu = 3 * lib.n                                   # FP32 ran (the velocity part)
            assert _rel(z[:nu], orc.stokes_qt(r)[:nu]) > 1e-9
    lib.set_precision("fp64")


def test_qt_pressure_block(pair):
    """Zero velocity residual: z_p = -M_p^{-1} r_p to the mass CG's tolerance
    and z_u = -B (B^T z_p) component-wise."""
    lib, orc = pair
    r = np.zeros(3 * lib.n + lib.n_p)
    r[3 * lib.n:] = W.random_vector(lib.n_p, 3)
    z, k = lib.stokes_qt(_t(r))
    z = z.cpu().numpy()
    M = orc.csr("Mp")
    rp = r[3 * lib.n:]
    assert np.linalg.norm(M @ (-z[3 * lib.n:]) - rp) <= 1e-6 * np.linalg.norm(rp)
    assert k >= 1


@pytest.mark.parametrize("steps", [1, 7])
def test_fgmres_fixed_steps(pair, steps):
    lib, orc = pair
    lib.set_precision("fp64")
    b = _rhs(orc)
    xo, ito, _, _, ho = orc.stokes_fgmres(b, tol=0.0, restart=30, maxit=steps)
    x, info, h = lib.stokes_fgmres(_t(b), tol=0.0, restart=30, maxit=steps, check=False)
    assert info.status == aux.ENOTCONV and info.iterations == ito == steps
    d = _rel(x.cpu().numpy(), xo)
    print(f"fixed {steps} steps: iterate rel diff {d:.2e}", flush=True)
    assert d <= 1e-8
    np.testing.assert_allclose(h, ho, rtol=0, atol=1e-8 * ho[0])


def test_fgmres_free_running(pair):
    lib, orc = pair
    b = _rhs(orc)
    m = lib.n
    xt, _, _, st, _ = orc.stokes_fgmres(b, tol=1e-12, restart=30, maxit=3000)
    assert st == 0
    for prec, fp32 in (("fp64", False), ("mixed", True)):
        lib.set_precision(prec)
        xo, ito, _, sto, _ = orc.stokes_fgmres(b, tol=1e-8, restart=30, maxit=500, fp32=fp32)
        x, info, h = lib.stokes_fgmres(_t(b), tol=1e-8, restart=30, maxit=500)
        x = x.cpu().numpy()
        du, dp = _rel(x[:3 * m], xt[:3 * m]), _rel(_p_mod_const(x, m), _p_mod_const(xt, m))
        print(f"{prec}: {info.iterations} steps (oracle {ito}), rel res {info.rel_residual:.2e}; vs oracle "
              f"{_rel(x[:3 * m], xo[:3 * m]):.1e} / {_rel(_p_mod_const(x, m), _p_mod_const(xo, m)):.1e}; "
              f"vs the 1e-12 solve {du:.1e} / {dp:.1e}", flush=True)
        assert sto == 0 and info.status == aux.OK and abs(info.iterations - ito) <= 1
        assert info.rel_residual <= 1.01e-8
        r = b - orc.stokes_operator(x)
        assert abs(np.linalg.norm(r) / np.linalg.norm(b) - info.rel_residual) <= 1e-12
        if prec == "fp64" and info.iterations == ito:
            assert _rel(x[:3 * m], xo[:3 * m]) <= 1e-8
            assert _rel(_p_mod_const(x, m), _p_mod_const(xo, m)) <= 1e-8
        assert du <= 1e-6 and dp <= 1e-3
    lib.set_precision("fp64")


def test_fgmres_restarted(pair):
    lib, orc = pair
    b = _rhs(orc)
    _, ito, _, sto, _ = orc.stokes_fgmres(b, tol=1e-8, restart=8, maxit=1000)
    x, info, _ = lib.stokes_fgmres(_t(b), tol=1e-8, restart=8, maxit=1000)
    assert sto == 0 and info.status == aux.OK and abs(info.iterations - ito) <= 2
    assert info.rel_residual <= 1.01e-8


def test_edge_cases():
    print("[stokes edge cases]", flush=True)
    xyz, tets = W.kuhn_mesh(4, seed=0)
    lib = aux.Solver(xyz, tets, 2, device=DEV)
    N = 3 * lib.n + lib.stokes_setup()
    x, info, h = lib.stokes_fgmres(torch.zeros(N, dtype=torch.float64, device=DEV))
    assert info.status == aux.OK and info.iterations == 0 and not torch.any(x)
    z, k = lib.stokes_qt(torch.zeros(N, dtype=torch.float64, device=DEV))
    assert k == 0 and not torch.any(z)
    b = torch.ones(N, dtype=torch.float64, device=DEV)
    for m in (0, 129):
        with pytest.raises(aux.AuxError):
            lib.stokes_fgmres(b, restart=m)
    x, info, _ = lib.stokes_fgmres(b, tol=1e-14, restart=4, maxit=5, check=False)
    assert info.status == aux.ENOTCONV and info.iterations == 5
    with pytest.raises(ValueError):
        lib.stokes_operator(torch.zeros(N - 1, dtype=torch.float64, device=DEV))


def _steps_at(n, k=2):
    xyz, tets = W.kuhn_mesh(n, jitter=0.2, seed=0)
    lib = aux.Solver(xyz, tets, k, device=DEV, precision="mixed")
    npr = lib.stokes_setup()
    b = np.concatenate([lib.load(W.stokes_f(c)) for c in range(3)] + [np.zeros(npr)])
    bt = _t(b)
    x, info, h = lib.stokes_fgmres(bt, tol=1e-8, restart=30, maxit=500)
    r = bt - lib.stokes_operator(x)
    rel = float(torch.linalg.norm(r) / torch.linalg.norm(bt))
    _, pcg = lib.solve(_t(lib.load(W.manufactured_f)), tol=1e-8)
    return lib, info, rel, pcg.iterations


def test_full_size():
    """P2 48^3 jittered (2.69M unknowns), mixed precision."""
    print("[stokes P2 16^3 and 48^3]", flush=True)
    _, i16, r16, c16 = _steps_at(16)
    lib, i48, r48, c48 = _steps_at(48)
    print(f"16^3: {i16.iterations} steps (CG {c16}); 48^3: {i48.iterations} steps (CG {c48}), "
          f"{i48.seconds:.3f} s", flush=True)
    for info, rel in ((i16, r16), (i48, r48)):
        assert info.status == aux.OK and rel <= 1.05e-8 and abs(rel - info.rel_residual) <= 1e-10
    assert i48.iterations / i16.iterations <= 1.15 * c48 / c16
    e = torch.zeros(3 * lib.n + lib.n_p, dtype=torch.float64, device=DEV)
    e[3 * lib.n:] = 1.0
    assert float(torch.max(torch.abs(lib.stokes_operator(e)))) <= 1e-15


def test_full_size_p3_p2():
    """P3-P2 on 32^3 jittered cubes (2,571,375 velocity and 274,625 pressure
    unknowns), mixed precision."""
    print("[stokes P3-P2 32^3]", flush=True)
    lib, info, rel, _ = _steps_at(32, k=3)
    print(f"P3-P2 32^3: {info.iterations} steps, {info.seconds:.3f} s", flush=True)
    assert lib.n_p == 65 ** 3
    assert info.status == aux.OK and rel <= 1.05e-8 and abs(rel - info.rel_residual) <= 1e-10
