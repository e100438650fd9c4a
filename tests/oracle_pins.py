"""Checks of the oracle's AMG cycle, PMIS splitting and extended+i
interpolation against what the published methods and linear algebra fix.

Shared by the oracle pin tests and by ``test_oracle_plants.py``, which runs
the same checks against copies of the oracle with a planted mistake (each
must then fail).  Every function raises AssertionError on a violation.

* V(1,1) cycle on 3-5 level hierarchies (Algorithm 2.1, Step 1, by an AMG
  cycle as Remark 2.1 allows): the cycle from a zero guess is a symmetric
  positive definite operator V with spectrum of V A_H in (0, 1] (pre- and
  post-smoothing with the same l1 diagonal, R = P^T, exact coarsest solve).
* PMIS (De Sterck, Yang, Heys 2006): in every round the new C points are
  exactly the undecided points whose measure beats every undecided neighbour
  in S u S^T (so each round's set is independent there), and exactly the
  undecided points that depend strongly on a new C point become F.
* Extended+i (De Sterck, Falgout, Nolting, Yang 2008): on a tridiagonal
  M-matrix with F runs of length at most two between C points, the weights
  equal the harmonic extension -A_FF^{-1} A_FC (eliminating the strong F
  neighbour k is then exact because i is kept in k's distribution, the "+i");
  on random small matrices the weights equal the published formula
  evaluated in exact rationals.
"""
from fractions import Fraction

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp

import oracle
import workloads as W


def problem(k, n, jitter=0.2, seed=3, **amg):
    xyz, tets = W.kuhn_mesh(n, jitter=jitter, seed=seed)
    P = oracle.Problem(xyz, tets, k)
    P.setup_amg(**amg)
    return P


# ----------------------------------------------------------- V-cycle and B

def check_vcycle_spd(k=2, n=5, coarse_max=4, min_levels=4):
    P = problem(k, n, coarse_max=coarse_max)
    assert P.nlev >= min_levels, P.nlev
    E = np.eye(P.nH)
    V = np.stack([P.vcycle(E[:, j]) for j in range(P.nH)], axis=1)
    assert np.max(np.abs(V - V.T)) <= 1e-13 * np.max(np.abs(V)), "V-cycle not symmetric"
    assert np.linalg.eigvalsh(0.5 * (V + V.T))[0] > 0, "V-cycle not positive definite"
    AH = P.csr("AH").toarray()
    lam = sla.eigh(AH, np.linalg.inv(0.5 * (V + V.T)), eigvals_only=True)
    assert lam[0] > 0 and lam[-1] <= 1 + 1e-10, (lam[0], lam[-1])


def check_vcycle_error_propagator(k=2, n=6, coarse_max=4, min_levels=5):
    """A V(1,1) cycle from zero with smoother S_l = I - D_l^{-1} A_l
    (D_l = diag(sum_j |a_ij|)) has the error propagator
    I - V_l A_l = S_l (I - P_l V_{l+1} P_l^T A_l) S_l, V_L = A_L^{-1} on the
    coarsest level (the textbook product form of the multigrid cycle).
    Evaluated densely from the exported hierarchy and compared with the
    oracle's cycle."""
    P = problem(k, n, coarse_max=coarse_max)
    assert P.nlev >= min_levels, P.nlev
    L = P.nlev - 1
    V = np.linalg.inv(P.csr("Alev", L).toarray())
    for l in range(L - 1, -1, -1):
        A = P.csr("Alev", l).toarray()
        Pl = P.csr("P", l).toarray()
        S = np.eye(A.shape[0]) - A / np.abs(A).sum(axis=1)[:, None]
        E = S @ (np.eye(A.shape[0]) - Pl @ V @ Pl.T @ A) @ S
        V = (np.eye(A.shape[0]) - E) @ np.linalg.inv(A)
    Eh = np.eye(P.nH)
    Vo = np.stack([P.vcycle(Eh[:, j]) for j in range(P.nH)], axis=1)
    assert np.max(np.abs(Vo - V)) <= 1e-12 * np.max(np.abs(V)), np.max(np.abs(Vo - V)) / np.max(np.abs(V))


def check_precond_spd_multilevel(k=2, n=4, coarse_max=2, min_levels=4):
    P = problem(k, n, coarse_max=coarse_max)
    assert P.nlev >= min_levels, P.nlev
    E = np.eye(P.n)
    B = np.stack([P.apply(E[:, j]) for j in range(P.n)], axis=1)
    assert np.max(np.abs(B - B.T)) <= 1e-13 * np.max(np.abs(B)), "B not symmetric"
    assert np.linalg.eigvalsh(0.5 * (B + B.T))[0] > 0, "B not positive definite"
    A = P.csr("A").toarray()
    lam = sla.eigh(A, np.linalg.inv(0.5 * (B + B.T)), eigvals_only=True)
    assert lam[0] > 0 and lam[-1] <= 1 + 1e-10, (lam[0], lam[-1])


def check_gamg_multilevel_flat_in_h(ns=(6, 9, 12), coarse_max=8):
    """Many-level V-cycles: CG iteration counts stay flat as h -> 0 (the
    h-independence of Theorem 4.2 carried by an AMG cycle, Sec. 6)."""
    its, levels = [], []
    for n in ns:
        P = problem(2, n, jitter=0.2, seed=0, coarse_max=coarse_max)
        levels.append(P.nlev)
        its.append(P.pcg(P.load(W.manufactured_f), tol=1e-8)[1])
    assert min(levels) >= 3, levels
    assert max(its) - min(its) <= 2, its


# -------------------------------------------------------------------- PMIS

def strong_sets(A, theta):
    """S_i by the strength rule of Sec. 6.2 (strict '>', ties within 1e-12
    of the row maximum not strong)."""
    A = sp.csr_matrix(A)
    S = []
    for i in range(A.shape[0]):
        cols = A.indices[A.indptr[i]:A.indptr[i + 1]]
        vals = A.data[A.indptr[i]:A.indptr[i + 1]]
        off = cols != i
        m = np.max(-vals[off]) if off.any() else -np.inf
        S.append(set(int(c) for c in cols[off][-vals[off] > theta * m + 1e-12 * m]) if m > 0 else set())
    return S


def check_pmis_rounds(k=2, n=8, theta=0.8, seed=0, coarse_max=20):
    xyz, tets = W.kuhn_mesh(n, jitter=0.2, seed=1)
    P = oracle.Problem(xyz, tets, k)
    P.setup_amg(theta=theta, coarse_max=coarse_max, seed=seed)
    assert P.nlev >= 3
    checked_rounds = 0
    for l in range(P.nlev - 1):
        A = P.csr("Alev", l)
        cf, rd = P.level_cf(l), P.level_rounds(l)
        nn = A.shape[0]
        S = strong_sets(A, theta)
        ST = [set() for _ in range(nn)]
        for i, s in enumerate(S):
            for j in s:
                ST[j].add(i)
        nst = [len(t) for t in ST]
        w = [(nst[i], oracle.pmis_rho(seed, l, i), -i) for i in range(nn)]
        # points that influence nobody are F before the first round
        assert all((rd[i] == 0) == (nst[i] == 0) for i in range(nn))
        assert all(cf[i] == -1 for i in range(nn) if rd[i] == 0)
        for r in range(1, int(rd.max()) + 1):
            U = {i for i in range(nn) if rd[i] >= r}
            D = {i for i in U if rd[i] == r and cf[i] == 1}
            for i in D:                                  # independent in S u S^T
                assert not ((S[i] | ST[i]) & D), (l, r, i)
            for i in U:                                  # exactly the local maxima
                nb = (S[i] | ST[i]) & U
                assert all(w[i] > w[j] for j in nb) == (i in D), (l, r, i)
            for i in U - D:                              # F rule of the round
                dep = bool(S[i] & D)
                assert (rd[i] == r) == dep, (l, r, i)
                if dep:
                    assert cf[i] == -1
            checked_rounds += 1
    assert checked_rounds >= 4


# ------------------------------------------------------------- extended+i

def _tridiag_case(rng, n=40):
    """Tridiagonal M-matrix (boundary couplings included) and a C/F split
    with C at both ends and F runs of length 1 or 2 between C points."""
    cf = [1]
    while len(cf) < n - 1:
        run = int(rng.integers(1, 3))
        cf += [-1] * run + [1]
    cf = np.array(cf[:n - 1] + [1], dtype=np.int32)
    if cf[-2] == -1 and cf[-3] == -1 and cf[-4] == -1:
        cf[-3] = 1
    c = rng.uniform(1.0, 2.0, size=n + 1)               # edge coefficients
    main = c[:-1] + c[1:]
    A = sp.diags([-c[1:-1], main, -c[1:-1]], [-1, 0, 1], format="csr")
    return A, cf


def check_ext_i_harmonic_1d(seeds=range(6)):
    for s in seeds:
        rng = np.random.default_rng(s)
        A, cf = _tridiag_case(rng)
        # no F run longer than two
        runs = np.diff(np.flatnonzero(cf > 0))
        assert runs.max() <= 3
        P = oracle.interp_given(A, cf, theta=0.25).toarray()
        Fi, Ci = np.flatnonzero(cf < 0), np.flatnonzero(cf > 0)
        Ad = A.toarray()
        ref = np.zeros((A.shape[0], len(Ci)))
        ref[Ci, np.arange(len(Ci))] = 1.0
        ref[Fi] = -np.linalg.solve(Ad[np.ix_(Fi, Fi)], Ad[np.ix_(Fi, Ci)])
        assert np.max(np.abs(P - ref)) <= 1e-14, (s, np.max(np.abs(P - ref)))


def _random_case(rng, n=12):
    """Small nonsymmetric matrix with integer entries: positive diagonal,
    mostly negative off-diagonals with some positive ones, random pattern."""
    pat = rng.random((n, n)) < 0.4
    pat = pat | pat.T
    np.fill_diagonal(pat, False)
    vals = -rng.integers(1, 10, size=(n, n)).astype(float)
    flip = rng.random((n, n)) < 0.2
    vals[flip] = -vals[flip]
    M = np.where(pat, vals, 0.0)
    np.fill_diagonal(M, np.abs(M).sum(axis=1) + rng.integers(1, 5, size=n))
    cf = np.where(rng.random(n) < 0.4, 1, -1).astype(np.int32)
    if cf.max() < 0:
        cf[0] = 1
    return M, cf


def ext_i_rational(M, cf, theta):
    """Extended+i weights by the published formula in exact rationals:
    for F point i, C^_i = (S_i n C) u U_{k in S_i n F} (S_k n C);
    abar_kl = a_kl if a_kl a_kk < 0 else 0; d_k = sum_{l in C^_i u {i}} abar_kl;
    atilde_ii = a_ii + sum_{weak/other n} a_in + sum_{k, d_k != 0} a_ik abar_ki / d_k
                + sum_{k, d_k = 0} a_ik;
    w_ij = -(a_ij + sum_{k, d_k != 0} a_ik abar_kj / d_k) / atilde_ii.
    Returns (dense Fraction weights, counters of the cases met)."""
    n = M.shape[0]
    a = [[Fraction(int(M[i, j])) for j in range(n)] for i in range(n)]
    S = strong_sets(sp.csr_matrix(M), theta)
    C = [j for j in range(n) if cf[j] > 0]
    col = {c: q for q, c in enumerate(C)}
    W = [[Fraction(0)] * len(C) for _ in range(n)]
    seen = {"d_zero": 0, "plus_i": 0, "weak": 0, "distance_two": 0}
    for i in range(n):
        if cf[i] > 0:
            W[i][col[i]] = Fraction(1)
            continue
        Fs = [k for k in sorted(S[i]) if cf[k] < 0]
        Ch = {j for j in S[i] if cf[j] > 0}
        for k in Fs:
            Ch |= {j for j in S[k] if cf[j] > 0}
        seen["distance_two"] += len(Ch - S[i])

        def abar(k, l):
            return a[k][l] if a[k][l] * a[k][k] < 0 else Fraction(0)

        diag = a[i][i]
        num = {j: a[i][j] for j in Ch}
        for m in range(n):
            if m == i or a[i][m] == 0 or m in Ch:
                continue
            if m in Fs:
                k = m
                d = sum((abar(k, l) for l in Ch | {i}), Fraction(0))
                if d == 0:
                    diag += a[i][k]
                    seen["d_zero"] += 1
                    continue
                if abar(k, i) != 0:
                    seen["plus_i"] += 1
                diag += a[i][k] * abar(k, i) / d
                for j in Ch:
                    num[j] += a[i][k] * abar(k, j) / d
            else:
                diag += a[i][m]
                seen["weak"] += 1
        for j in Ch:
            W[i][col[j]] = -num[j] / diag
    return W, seen


def check_ext_i_rational(seeds=range(40), theta=0.5):
    total = {"d_zero": 0, "plus_i": 0, "weak": 0, "distance_two": 0}
    for s in seeds:
        M, cf = _random_case(np.random.default_rng(1000 + s))
        Wr, seen = ext_i_rational(M, cf, theta)
        for key in total:
            total[key] += seen[key]
        P = oracle.interp_given(sp.csr_matrix(M), cf, theta=theta).toarray()
        ref = np.array([[float(x) for x in row] for row in Wr])
        assert P.shape == ref.shape
        scale = max(1.0, float(np.max(np.abs(ref))))
        assert np.max(np.abs(P - ref)) <= 1e-14 * scale, (s, np.max(np.abs(P - ref)))
    # the corpus exercises every branch of the formula
    assert all(v > 0 for v in total.values()), total


# ---------------------------------------------------------------- statuses

def check_breakdown_status():
    """CG must stop with the breakdown status (2) when r.z <= 0: used with a
    planted preconditioner that returns -B r."""
    P = problem(2, 4, coarse_max=8)
    x, it, rr, st = P.pcg(P.load(W.manufactured_f), tol=1e-8)
    assert st == 2 and it == 0, (st, it)
