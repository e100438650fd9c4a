"""Pins of the oracle's flexible GMRES(m), the Krylov method of the paper's
experiments (Sec. 6.1; Saad's flexible variant with right preconditioning).

* Without a preconditioner, the residual after j steps is the minimum of
  ||r_0 - A K c|| over the Krylov space K_j(A, r_0) (the defining property of
  GMRES), computed here by numpy least squares on an explicit basis.
* With the fixed preconditioner B, the correction lies in B K_j(AB, r_0) and
  minimises the residual there (the same property for AB).
* GMRES(1) is the minimal-residual iteration x += alpha B r,
  alpha = (r, A B r) / (A B r, A B r), written out here.
* Full GMRES terminates within n steps; the solution equals the dense direct
  solve; the residual history does not increase within a cycle.
* The paper's protocol (zero right-hand side, random initial guess, relative
  residual 1e-6) gives iteration counts that do not grow as h -> 0.
"""
import numpy as np
import pytest

import oracle
import workloads as W


def _problem(k, n, jitter=0.0, seed=0):
    xyz, tets = W.kuhn_mesh(n, jitter=jitter, seed=seed)
    P = oracle.Problem(xyz, tets, k)
    P.setup_amg()
    return P


def _krylov_min(Aop, M, r0, j):
    """min_c ||r0 - Aop(K c)|| with K an orthonormal basis of
    span{r0, M r0, ..., M^{j-1} r0}; Aop and M are dense matrices."""
    cols = [r0 / np.linalg.norm(r0)]
    for _ in range(1, j):
        v = M @ cols[-1]
        cols.append(v / np.linalg.norm(v))
    K, _ = np.linalg.qr(np.stack(cols, 1))
    AK = Aop @ K
    c, *_ = np.linalg.lstsq(AK, r0, rcond=None)
    return np.linalg.norm(r0 - AK @ c)


def _dense_B(P):
    return np.stack([P.apply(e) for e in np.eye(P.n)], 1)


def test_gmres_minimises_residual_over_krylov_space():
    P = _problem(2, 3, jitter=0.1, seed=3)
    A = P.csr("A").toarray()
    b = np.random.default_rng(0).standard_normal(P.n)
    x, it, rr, st, hist = P.fgmres(b, tol=0.0, restart=30, maxit=6, prec="none")
    assert it == 6 and st == 1
    for j in range(1, 7):
        ref = _krylov_min(A, A, b, j)
        assert abs(hist[j] - ref) <= 1e-9 * hist[0], (j, hist[j], ref)


def test_flexible_gmres_minimises_over_preconditioned_space():
    P = _problem(2, 3, jitter=0.1, seed=4)
    A = P.csr("A").toarray()
    B = _dense_B(P)
    b = np.random.default_rng(1).standard_normal(P.n)
    x, it, rr, st, hist = P.fgmres(b, tol=0.0, restart=30, maxit=5, prec="fp64")
    assert it == 5
    AB = A @ B
    for j in range(1, 6):
        ref = _krylov_min(AB, AB, b, j)
        assert abs(hist[j] - ref) <= 1e-9 * hist[0], (j, hist[j], ref)
    # the iterate is x0 + B K_5(AB, b): its residual is the minimum itself
    assert abs(np.linalg.norm(b - A @ x) - hist[5]) <= 1e-10 * hist[0]


@pytest.mark.parametrize("k,n", [(2, 3), (3, 2)])
def test_restart_one_is_minimal_residual_iteration(k, n):
    P = _problem(k, n, jitter=0.1, seed=5)
    A = P.csr("A")
    rng = np.random.default_rng(2)
    b = rng.standard_normal(P.n)
    x0 = rng.standard_normal(P.n)
    x, it, rr, st, hist = P.fgmres(b, tol=0.0, restart=1, maxit=8, x0=x0)
    xm = x0.copy()
    r = b - A @ xm
    norms = [np.linalg.norm(r)]
    for _ in range(8):
        z = P.apply(r)
        w = A @ z
        alpha = (r @ w) / (w @ w)
        xm += alpha * z
        r -= alpha * w
        norms.append(np.linalg.norm(r))
    assert it == 8
    assert np.linalg.norm(x - xm) <= 1e-12 * np.linalg.norm(xm)
    np.testing.assert_allclose(hist, norms, rtol=1e-9, atol=1e-13 * norms[0])


@pytest.mark.parametrize("k,n,restart", [(2, 3, 30), (2, 3, 5), (3, 2, 30), (4, 2, 10)])
def test_fgmres_matches_dense_solve(k, n, restart):
    P = _problem(k, n, jitter=0.1, seed=1)
    b = P.load(W.manufactured_f)
    xd = np.linalg.solve(P.csr("A").toarray(), b)
    x, it, rr, st, hist = P.fgmres(b, tol=1e-12, restart=restart, maxit=500)
    assert st == 0 and rr <= 1e-11
    assert np.linalg.norm(x - xd) <= 1e-10 * np.linalg.norm(xd)
    # within a cycle the minimum is over a growing space
    for c0 in range(0, it, restart):
        seg = hist[c0 + 1: min(c0 + restart, it) + 1]
        assert np.all(np.diff(seg) <= 1e-12 * hist[0])


def test_full_gmres_terminates_within_n_steps():
    P = _problem(2, 2, jitter=0.1, seed=2)
    b = np.random.default_rng(3).standard_normal(P.n)
    x, it, rr, st, hist = P.fgmres(b, tol=1e-10, restart=P.n, maxit=P.n, prec="none")
    assert st == 0 and it <= P.n and rr <= 1e-9


def test_paper_protocol_iterations_flat_in_h():
    """Zero right-hand side, random initial guess, relative residual 1e-6."""
    its = []
    for n in (4, 6, 8):
        P = _problem(2, n)
        x0 = np.random.default_rng(7).uniform(-1.0, 1.0, P.n)
        x, it, rr, st, hist = P.fgmres(np.zeros(P.n), tol=1e-6, restart=30, maxit=200, x0=x0)
        assert st == 0 and rr <= 1.01e-6
        its.append(it)
    assert max(its) - min(its) <= 2, its


def test_fgmres_status_codes_and_fp32():
    P = _problem(2, 3, jitter=0.1, seed=6)
    b = P.load(W.manufactured_f)
    x, it, rr, st, hist = P.fgmres(np.zeros(P.n), tol=1e-6)
    assert (st, it, rr) == (0, 0, 0.0) and not x.any()
    x, it, rr, st, hist = P.fgmres(b, tol=1e-14, maxit=3)
    assert st == 1 and it == 3
    # an FP32 preconditioner is not exactly symmetric; the flexible method
    # still converges to the FP64 accuracy asked for
    x32, it32, rr32, st32, _ = P.fgmres(b, tol=1e-10, prec="fp32")
    x64, it64, rr64, st64, _ = P.fgmres(b, tol=1e-10, prec="fp64")
    assert st32 == st64 == 0 and rr32 <= 1.01e-10 and abs(it32 - it64) <= 1
    assert np.linalg.norm(x32 - x64) <= 1e-8 * np.linalg.norm(x64)
