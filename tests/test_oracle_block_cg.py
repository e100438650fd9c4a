"""Pins of the oracle's block preconditioned CG (O'Leary 1980), the second
batched form beside lock-step CG.

* One right-hand side: block CG is CG (same iterates, iteration count).
* The defining property: after k iterations from X_0 = 0 every column is the
  A-orthogonal projection of the exact solution onto the block Krylov space
  span{B F, (BA) B F, ..., (BA)^{k-1} B F} (all columns' directions
  together), computed here with numpy from the dense A and B.
* Finite termination: in exact arithmetic at most ceil(n / s) iterations.
* Status codes: iteration limit, zero right-hand side, NaN (breakdown by a
  planted mistake in test_oracle_plants.py).
* The converged block equals the dense direct solve, column by column.
"""
import numpy as np
import pytest

import oracle
import workloads as W


def _problem(k, n, jitter=0.2, seed=2):
    xyz, tets = W.kuhn_mesh(n, jitter=jitter, seed=seed)
    return oracle.Problem(xyz, tets, k).setup_amg()


def _block(P, s, seed=0):
    rng = np.random.default_rng(seed)
    return rng.standard_normal((P.n, s))


def test_one_column_is_cg():
    P = _problem(2, 5)
    b = P.load(W.manufactured_f)
    X, it, rel, st = P.block_pcg(b[:, None], tol=1e-10)
    x, it1, rr, st1 = P.pcg(b, tol=1e-10)
    assert st == st1 == 0 and it == it1
    assert np.max(np.abs(X[:, 0] - x)) <= 1e-13 * np.max(np.abs(x))
    for k in (1, 3, 6):
        X, it, rel, st = P.block_pcg(b[:, None], tol=0.0, maxit=k)
        x, _, _, _ = P.pcg(b, tol=0.0, maxit=k)
        assert it == k and np.max(np.abs(X[:, 0] - x)) <= 1e-13 * np.max(np.abs(x))


@pytest.mark.parametrize("k,n,s", [(2, 3, 3), (2, 4, 4), (3, 2, 2)])
def test_block_krylov_projection(k, n, s):
    P = _problem(k, n)
    A = P.csr("A").toarray()
    Bd = np.stack([P.apply(e) for e in np.eye(P.n)], axis=1)
    F = _block(P, s, seed=k * 10 + n)
    Xs = np.linalg.solve(A, F)
    for kk in range(1, 5):
        if kk * s >= P.n:
            break
        blocks, V = [], Bd @ F
        for _ in range(kk):
            blocks.append(V)
            V = Bd @ (A @ V)
        K, _ = np.linalg.qr(np.concatenate(blocks, axis=1))
        Xp = K @ np.linalg.solve(K.T @ A @ K, K.T @ F)
        X, it, rel, st = P.block_pcg(F, tol=0.0, maxit=kk)
        assert it == kk
        err = np.linalg.norm(X - Xp) / np.linalg.norm(Xs)
        assert err <= 1e-9, (kk, err)


def test_finite_termination_and_dense_solve():
    P = _problem(2, 2)                     # n_h = 27
    s = 4
    F = _block(P, s, seed=3)
    # (beyond ~1e-10 the block residual loses rank and gamma = Z^T R turns
    # singular in rounding: the breakdown O'Leary's method is known for)
    X, it, rel, st = P.block_pcg(F, tol=1e-9, maxit=50)
    assert st == 0 and it <= -(-P.n // s), it
    Xd = np.linalg.solve(P.csr("A").toarray(), F)
    assert np.linalg.norm(X - Xd) <= 1e-8 * np.linalg.norm(Xd)


def test_block_cg_columns_match_single_solves():
    P = _problem(2, 6, jitter=0.2, seed=0)
    F = np.stack([P.load(W.fourier_f(c)) for c in range(5)], axis=1)
    X, it, rel, st = P.block_pcg(F, tol=1e-10)
    assert st == 0 and np.all(rel <= 1e-10)
    its = []
    for j in range(5):
        x, i1, _, _ = P.pcg(F[:, j], tol=1e-10)
        its.append(i1)
        assert np.linalg.norm(X[:, j] - x) <= 1e-8 * np.linalg.norm(x)
    assert it <= max(its)
    # the FP32 preconditioner inside converges to the same block
    X32, it32, rel32, st32 = P.block_pcg(F, tol=1e-10, fp32=True)
    assert st32 == 0 and abs(it32 - it) <= 1
    assert np.linalg.norm(X32 - X) <= 1e-8 * np.linalg.norm(X)


def test_block_cg_status_codes():
    P = _problem(2, 4)
    F = _block(P, 3, seed=5)
    X, it, rel, st = P.block_pcg(F, tol=1e-12, maxit=2)
    assert st == 1 and it == 2
    F[:, 1] = 0.0                          # a zero column converges at once
    X, it, rel, st = P.block_pcg(F[:, 1:2], tol=1e-8)
    assert st == 0 and it == 0 and not np.any(X)
    F[4, 0] = np.nan
    X, it, rel, st = P.block_pcg(F, tol=1e-8)
    assert st == 3
