"""Pins of the oracle's Stokes discretisation and solver (Sec. 5, Sec. 6.3:
Hood-Taylor P^k-P^{k-1} for k = 2, 3, 4, block triangular preconditioner
Q_t, FGMRES).

* B^T 1 = 0: constant pressures are the null space (integration by parts,
  the interior velocity basis vanishes on the boundary).
* B^T p for a linear pressure p = x_c (its nodal values) equals the load
  vector of the constant field e_c (again by parts: -int p dphi/dx_c =
  int dp/dx_c phi); this pins the sign, the component blocks and the
  pressure basis.
* M_p: integrals of pressure-space fields are exact (1, x^2, and x^4, x^2 y^2,
  x^6 where the pressure space holds x^2 or x^3), symmetric positive
  definite.
* FGMRES with Q_t solves the saddle-point system: agreement with a dense
  least-squares solve (pressure modulo constants).
* Manufactured smooth solution: velocity L2 error O(h^{k+1}) and pressure
  L2 error O(h^k) (the textbook Hood-Taylor rates); FGMRES steps flat in h.
"""
import numpy as np
import pytest

import oracle
import workloads as W


def _stokes(n, k=2, jitter=0.2, seed=0):
    xyz, tets = W.kuhn_mesh(n, jitter=jitter, seed=seed)
    return oracle.Problem(xyz, tets, k).setup_amg().stokes_setup()


@pytest.mark.parametrize("k", [2, 3, 4])
def test_pressure_space(k):
    P = _stokes(3, k)
    keys = P.pressure_keys()
    assert keys.shape == (P.np, k - 1)
    assert np.all(np.diff(keys, axis=1) >= 0)                              # sorted multisets
    assert all(tuple(a) < tuple(b) for a, b in zip(keys[:-1], keys[1:]))   # lexicographic, unique
    assert P.np == (3 * (k - 1) + 1) ** 3                                  # every node of order k-1
    if k == 2:
        assert np.array_equal(keys[:, 0], np.arange(P.xyz.shape[0]))       # P^1: vertex order


@pytest.mark.parametrize("k", [2, 3, 4])
def test_pressure_constants_are_the_null_space(k):
    P = _stokes(3, k)
    B = P.csr("B")
    assert np.max(np.abs(B.T @ np.ones(P.np))) <= 1e-14 * abs(B).max()


@pytest.mark.parametrize("k", [2, 3, 4])
@pytest.mark.parametrize("c", [0, 1, 2])
def test_gradient_of_linear_pressure_is_a_load_vector(k, c):
    P = _stokes(3, k)
    n = P.n
    bt = P.csr("B").T @ P.pressure_xyz()[:, c]
    ones = P.load(lambda q: np.ones(q.shape[0]))
    for d in range(3):
        blk = bt[d * n:(d + 1) * n]
        if d == c:
            assert np.max(np.abs(blk - ones)) <= 1e-13 * np.max(np.abs(ones))
        else:
            assert np.max(np.abs(blk)) <= 1e-13 * np.max(np.abs(ones))


@pytest.mark.parametrize("k", [2, 3, 4])
def test_pressure_mass_matrix(k):
    P = _stokes(3, k)
    M = P.csr("Mp").toarray()
    assert np.max(np.abs(M - M.T)) <= 1e-16
    assert np.linalg.eigvalsh(M)[0] > 0
    X = P.pressure_xyz()
    one = np.ones(P.np)
    assert abs(one @ M @ one - 1.0) <= 1e-14
    for c in range(3):
        x = X[:, c]
        assert abs(x @ M @ x - 1.0 / 3.0) <= 1e-14                        # int x^2
        if k >= 3:
            assert abs((x * x) @ M @ (x * x) - 1.0 / 5.0) <= 1e-14         # int x^4
            y = X[:, (c + 1) % 3]
            assert abs((x * x) @ M @ (y * y) - 1.0 / 9.0) <= 1e-14         # int x^2 y^2
        if k >= 4:
            assert abs((x ** 3) @ M @ (x ** 3) - 1.0 / 7.0) <= 1e-14       # int x^6


@pytest.mark.parametrize("k,n", [(2, 2), (2, 3), (3, 2), (4, 2)])
def test_fgmres_qt_matches_dense_solve(k, n):
    P = _stokes(n, k, seed=1)
    A = P.csr("A").toarray()
    B = P.csr("B").toarray()
    m = P.n
    F = np.block([[np.kron(np.eye(3), A), B.T], [B, np.zeros((P.np, P.np))]])
    rng = np.random.default_rng(n)
    b = np.concatenate([rng.standard_normal(3 * m), np.zeros(P.np)])
    x, it, rr, st, hist = P.stokes_fgmres(b, tol=1e-12, maxit=2000)
    assert st == 0 and rr <= 1e-11
    xd = np.linalg.lstsq(F, b, rcond=None)[0]
    assert np.linalg.norm(x[:3 * m] - xd[:3 * m]) <= 1e-8 * np.linalg.norm(xd[:3 * m])
    dp, dd = x[3 * m:] - x[3 * m:].mean(), xd[3 * m:] - xd[3 * m:].mean()
    assert np.linalg.norm(dp - dd) <= 1e-7 * np.linalg.norm(dd)
    assert np.max(np.abs(F @ x - b)) <= 1e-10 * np.max(np.abs(b))


# (k, meshes, velocity rate bounds, pressure rate lower bound); measured on
# the last two meshes: P2 velocity 2.8-3.0, pressure 2.6 (3.1, 2.8 before);
# P3 3.84 and 3.56; P4 4.76 and 4.27 (pre-asymptotic, textbook 5 and 4)
RATES = [(2, (4, 8, 12), (2.6, 3.5), 1.8),
         (3, (3, 4, 6), (3.5, 4.5), 2.7),
         (4, (2, 3, 4), (4.2, 5.5), 3.5)]


@pytest.mark.parametrize("k,ns,ru_bounds,rp_min", RATES, ids=[f"P{r[0]}-P{r[0]-1}" for r in RATES])
def test_hood_taylor_convergence_rates_and_flat_steps(k, ns, ru_bounds, rp_min):
    """Jittered meshes: velocity L2 rate near k+1, pressure L2 rate at least
    about k, and FGMRES steps to 1e-8 nearly flat in h (P2: 39, 44, 46; P3:
    72, 78, 77; P4: 126, 140, 138), the optimality Sec. 6.3 reports for GAMG."""
    eu, ep, steps = [], [], []
    for n in ns:
        P = _stokes(n, k, jitter=0.2)
        m = P.n
        b = np.concatenate([P.load(W.stokes_f(c)) for c in range(3)] + [np.zeros(P.np)])
        x, it, rr, st, hist = P.stokes_fgmres(b, tol=1e-12, maxit=3000)
        assert st == 0
        steps.append(P.stokes_fgmres(b, tol=1e-8, maxit=3000)[1])
        eu.append(np.sqrt(sum(P.l2_error(W.stokes_u(c), x[c * m:(c + 1) * m]) ** 2 for c in range(3))))
        ph = x[3 * m:]
        M = P.csr("Mp")
        one = np.ones(P.np)
        ph = ph - (one @ (M @ ph)) / (one @ (M @ one))
        ep.append(P.pressure_l2_error(W.stokes_p, ph))
    ru = np.log(eu[-2] / eu[-1]) / np.log(ns[-1] / ns[-2])
    rp = np.log(ep[-2] / ep[-1]) / np.log(ns[-1] / ns[-2])
    assert ru_bounds[0] < ru < ru_bounds[1], (eu, ru)
    assert rp > rp_min, (ep, rp)
    assert steps[-1] <= 1.25 * steps[0] + 2, steps
