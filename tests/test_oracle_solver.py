"""Pins of the oracle's preconditioner and CG.

* CG converges to the dense direct solution of A_h u = f (brute force);
* discretisation error O(h^{k+1}) in L2 and O(h^k) in H1 for the
  manufactured solution (textbook rates for P^k Lagrange elements);
* the preconditioner B is symmetric positive definite (needed by CG; the
  symmetric GAMG variant of Remark 2.1);
* the augmented-system facts of Sec. 3 (Lemma 3.1, the null space of the
  augmented matrix, Remark 3.2: Algorithm 2.1 with exact coarse solve and
  Gauss-Seidel postsmoothing is block Gauss-Seidel on the augmented system);
* Theorem 4.2: with an exact coarse solve the iteration count does not grow
  as h -> 0; Sec. 6.2: the count is insensitive to the strength threshold.
"""
import numpy as np
import pytest
import scipy.linalg as sla

import oracle
import oracle_pins as pins
import workloads as W


def _problem(k, n, jitter=0.0, seed=0, kappa=None, **amg):
    xyz, tets = W.kuhn_mesh(n, jitter=jitter, seed=seed)
    P = oracle.Problem(xyz, tets, k, kappa)
    P.setup_amg(**amg)
    return P


@pytest.mark.parametrize("k,n", [(2, 2), (2, 3), (3, 2), (2, 5), (4, 2)])
def test_pcg_matches_dense_solve(k, n):
    P = _problem(k, n, jitter=0.1, seed=1)
    b = P.load(W.manufactured_f)
    xd = np.linalg.solve(P.csr("A").toarray(), b)
    x, it, rr, st = P.pcg(b, tol=1e-13)
    assert st == 0 and rr <= 1e-13
    assert np.linalg.norm(x - xd) <= 1e-11 * np.linalg.norm(xd)


def _grad_u(p):
    s, c = np.sin(np.pi * p), np.cos(np.pi * p)
    return np.pi * np.stack([c[..., 0] * s[..., 1] * s[..., 2], s[..., 0] * c[..., 1] * s[..., 2],
                             s[..., 0] * s[..., 1] * c[..., 2]], axis=-1)


@pytest.mark.parametrize("k,ns", [(2, (4, 8, 16)), (3, (2, 4, 8)), (4, (2, 4, 8))])
def test_convergence_rates(k, ns):
    l2, h1 = [], []
    for n in ns:
        P = _problem(k, n)
        x, it, rr, st = P.pcg(P.load(W.manufactured_f), tol=1e-12)
        assert st == 0
        l2.append(P.l2_error(W.manufactured_u, x))
        h1.append(P.h1_error(_grad_u, x))
    r2 = np.log2(l2[-2] / l2[-1])
    r1 = np.log2(h1[-2] / h1[-1])
    assert k + 1 - 0.25 < r2 < k + 1 + 0.5, (l2, r2)
    assert k - 0.2 < r1 < k + 0.5, (h1, r1)


@pytest.mark.parametrize("k,n", [(2, 3), (2, 4), (3, 3), (4, 2)])
def test_preconditioner_spd(k, n):
    P = _problem(k, n, jitter=0.2, seed=3)
    E = np.eye(P.n)
    B = np.stack([P.apply(E[:, j]) for j in range(P.n)], axis=1)
    assert np.max(np.abs(B - B.T)) < 1e-13 * np.max(np.abs(B))
    ev = np.linalg.eigvalsh(0.5 * (B + B.T))
    assert ev[0] > 0
    # the preconditioned operator has spectrum in (0, 1]: B is a contraction
    # in the energy norm (the error propagator I - BA is A-nonnegative)
    A = P.csr("A").toarray()
    lam = sla.eigh(A, np.linalg.inv(0.5 * (B + B.T)), eigvals_only=True)
    assert lam[0] > 0 and lam[-1] <= 1 + 1e-10
    B32 = np.stack([P.apply(E[:, j], fp32=True) for j in range(P.n)], axis=1)
    assert np.max(np.abs(B32 - B)) < 1e-6 * np.max(np.abs(B))


def test_vcycle_spd_multilevel():
    """The AMG V(1,1) cycle alone on a 4-level hierarchy: symmetric, positive
    definite, spectrum of V A_H in (0, 1]."""
    pins.check_vcycle_spd(k=2, n=5, coarse_max=4, min_levels=4)
    pins.check_vcycle_spd(k=3, n=4, coarse_max=4, min_levels=3)


def test_vcycle_error_propagator():
    """The cycle equals the textbook product form of its error propagator,
    level by level, on a 5-level hierarchy (P2) and a 4-level one (P3)."""
    pins.check_vcycle_error_propagator(k=2, n=6, coarse_max=4, min_levels=5)
    pins.check_vcycle_error_propagator(k=3, n=5, coarse_max=6, min_levels=4)


@pytest.mark.parametrize("k,n,cmax,minl", [(2, 4, 2, 4), (2, 5, 4, 4), (3, 4, 4, 3)])
def test_preconditioner_spd_multilevel(k, n, cmax, minl):
    """B with a 3-4 level V-cycle for Step 1: symmetric positive definite,
    spectrum of B A_h in (0, 1]."""
    pins.check_precond_spd_multilevel(k=k, n=n, coarse_max=cmax, min_levels=minl)


def test_gamg_multilevel_flat_in_h():
    pins.check_gamg_multilevel_flat_in_h()


def test_augmented_system_and_block_gauss_seidel():
    P = _problem(2, 3, jitter=0.2, seed=4)
    A = P.csr("A").toarray()
    IP = P.csr("IP").toarray()
    AH = P.csr("AH").toarray()
    nh, nH = IP.shape
    Aug = np.block([[IP.T @ A @ IP, IP.T @ A], [A @ IP, A]])     # Lemma 3.1
    assert np.linalg.matrix_rank(Aug) == nh                       # singular, rank n_h
    c = np.random.default_rng(0).normal(size=nH)
    assert np.max(np.abs(Aug @ np.concatenate([c, -IP @ c]))) < 1e-12   # null space
    assert np.all(np.diag(Aug) > 0)

    # one step of Algorithm 2.1 (exact coarse solve, Gauss-Seidel post-smoothing)
    f = P.load(W.manufactured_f)
    u = np.random.default_rng(1).normal(size=nh)
    DL = np.tril(A)
    ut = u + IP @ np.linalg.solve(AH, IP.T @ (f - A @ u))
    u_next = ut + np.linalg.solve(DL, f - A @ ut)
    # one block Gauss-Seidel step on the augmented system, eq. (bgamg)
    DmL = np.block([[IP.T @ A @ IP, np.zeros((nH, nh))], [A @ IP, DL]])
    v = np.concatenate([np.zeros(nH), u])
    ft = np.concatenate([IP.T @ f, f])
    v_next = v + np.linalg.solve(DmL, ft - Aug @ v)
    assert np.max(np.abs(IP @ v_next[:nH] + v_next[nH:] - u_next)) < 1e-12 * np.max(np.abs(u_next))


@pytest.mark.parametrize("k,ns", [(2, (4, 8, 12)), (3, (4, 6, 8)), (4, (6, 8, 10))])
def test_two_level_iterations_flat_in_h(k, ns):
    its = []
    for n in ns:
        P = _problem(k, n, jitter=0.2, seed=0, coarse_max=2000)   # exact coarse solve
        assert P.nlev == 1
        its.append(P.pcg(P.load(W.manufactured_f), tol=1e-8)[1])
    assert max(its) - min(its) <= 1, its


def test_gamg_insensitive_to_theta():
    its = []
    for theta in (0.2, 0.4, 0.6, 0.8):
        P = _problem(2, 10, jitter=0.2, seed=0, theta=theta)
        assert P.nlev > 1
        its.append(P.pcg(P.load(W.manufactured_f), tol=1e-8)[1])
    assert max(its) - min(its) <= 2, its


def test_fp32_preconditioner_converges_to_same_solution():
    P = _problem(2, 8, jitter=0.2, seed=0)
    b = P.load(W.manufactured_f)
    x, it, rr, st = P.pcg(b, tol=1e-8)
    y, it32, rr32, st32 = P.pcg(b, tol=1e-8, fp32=True)
    assert st == 0 and st32 == 0 and abs(it - it32) <= 1
    assert np.linalg.norm(x - y) <= 1e-7 * np.linalg.norm(x)


def test_pcg_status_codes():
    P = _problem(2, 4)
    b = P.load(W.manufactured_f)
    x, it, rr, st = P.pcg(b, tol=1e-12, maxit=2)
    assert st == 1 and it == 2                    # not converged
    x, it, rr, st = P.pcg(np.zeros(P.n))
    assert st == 0 and it == 0 and not np.any(x)  # zero right-hand side
    bad = b.copy()
    bad[3] = np.nan
    x, it, rr, st = P.pcg(bad)
    assert st == 3                                # NaN detected
