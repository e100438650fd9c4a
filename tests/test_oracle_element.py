"""Pins of the oracle's element-level pieces against closed forms.

* nodal basis: Kronecker property at the evenly spaced nodes, partition of
  unity, exact reproduction of degree-k polynomials, derivative consistency
  (the P^k Lagrange space of Sec. 2);
* quadrature: exact integrals of monomials (Dirichlet integral on the simplex);
* element stiffness: equal to the stiffness of the Lagrange basis built
  independently in exact rational arithmetic (Vandermonde inversion and
  closed-form monomial integration); symmetry, zero row sums, one-dimensional
  kernel, and the energy of interpolated linear and quadratic functions.
"""
from fractions import Fraction
from itertools import product
from math import factorial

import numpy as np
import pytest

import oracle
import workloads as W


@pytest.mark.parametrize("k", [1, 2, 3, 4])
def test_basis_kronecker_and_unity(k):
    al = oracle.multi_indices(k)
    nloc = (k + 1) * (k + 2) * (k + 3) // 6
    assert al.shape == (nloc, 4) and np.all(al.sum(1) == k)
    for a in range(nloc):
        for b in range(nloc):
            v = oracle.basis(k, al[a], al[b] / k)
            assert abs(v - (a == b)) < 1e-13
    rng = np.random.default_rng(3)
    for _ in range(20):
        lam = rng.dirichlet(np.ones(4))
        s = sum(oracle.basis(k, al[a], lam) for a in range(nloc))
        assert abs(s - 1.0) < 1e-13


@pytest.mark.parametrize("k", [2, 3, 4])
def test_basis_reproduces_degree_k(k):
    al = oracle.multi_indices(k)
    rng = np.random.default_rng(5)
    # random polynomial of degree k in the barycentric coordinates
    terms = [(tuple(e), rng.normal()) for e in product(range(k + 1), repeat=4) if sum(e) <= k]

    def p(lam):
        return sum(c * np.prod([lam[i] ** e[i] for i in range(4)]) for e, c in terms)

    nodal = [p(al[a] / k) for a in range(len(al))]
    for _ in range(10):
        lam = rng.dirichlet(np.ones(4))
        v = sum(nodal[a] * oracle.basis(k, al[a], lam) for a in range(len(al)))
        assert abs(v - p(lam)) < 1e-12


@pytest.mark.parametrize("k", [2, 3, 4])
def test_basis_derivative_matches_difference_quotient(k):
    al = oracle.multi_indices(k)
    rng = np.random.default_rng(7)
    for a in range(len(al)):
        lam = rng.uniform(0.1, 0.6, size=4)
        d = oracle.basis_dlam(k, al[a], lam)
        for p in range(4):
            e = np.zeros(4)
            e[p] = 1e-5
            fd = (oracle.basis(k, al[a], lam + e) - oracle.basis(k, al[a], lam - e)) / 2e-5
            assert abs(fd - d[p]) < 1e-7 * max(1.0, abs(d[p]))


@pytest.mark.parametrize("m", [1, 2, 3, 4, 5, 6])
@pytest.mark.parametrize("a", [0, 1, 2])
def test_gauss_jacobi_exact(m, a):
    x, w = oracle.gauss_jacobi(m, a)
    assert np.all((x > 0) & (x < 1)) and np.all(w > 0)
    for j in range(2 * m):
        exact = factorial(j) * factorial(a) / factorial(j + a + 1)   # Beta(j+1, a+1)
        assert abs(np.sum(w * x ** j) - exact) < 1e-14


@pytest.mark.parametrize("m", [1, 2, 3, 4, 5])
def test_tet_rule_integrates_monomials(m):
    lam, w = oracle.tet_rule(m)
    assert abs(w.sum() - 1.0 / 6.0) < 1e-15
    assert np.all(lam > -1e-15)
    for beta in product(range(2 * m), repeat=4):
        if sum(beta) > 2 * m - 1:
            continue
        exact = np.prod([factorial(b) for b in beta]) / factorial(sum(beta) + 3)
        approx = np.sum(w * np.prod(lam ** np.array(beta), axis=1))
        assert abs(approx - exact) < 1e-15 + 1e-13 * exact


# ---------------------------------------------------------------- exact P^k stiffness

def _poly_mul(p, q):
    r = {}
    for ea, ca in p.items():
        for eb, cb in q.items():
            e = (ea[0] + eb[0], ea[1] + eb[1], ea[2] + eb[2])
            r[e] = r.get(e, 0) + ca * cb
    return r


def _poly_diff(p, d):
    r = {}
    for e, c in p.items():
        if e[d] > 0:
            f = list(e)
            f[d] -= 1
            r[tuple(f)] = r.get(tuple(f), 0) + c * e[d]
    return r


def _int_ref_tet(p):
    # int over {x,y,z >= 0, x+y+z <= 1} of x^a y^b z^c = a! b! c! / (a+b+c+3)!
    return sum(c * Fraction(factorial(e[0]) * factorial(e[1]) * factorial(e[2]),
                            factorial(sum(e) + 3)) for e, c in p.items())


def _exact_lagrange_stiffness(k):
    """Stiffness of the Lagrange basis on the unit right tet, in exact rationals.

    The basis is obtained by inverting the Vandermonde matrix of the
    monomials x^a y^b z^c (a+b+c <= k) at the nodes (alpha_1, alpha_2, alpha_3)/k.
    """
    al = oracle.multi_indices(k)
    mons = [e for e in product(range(k + 1), repeat=3) if sum(e) <= k]
    nodes = [tuple(Fraction(int(a[p]), k) for p in (1, 2, 3)) for a in al]
    n = len(mons)
    V = [[Fraction(1) for _ in range(n)] for _ in range(n)]
    for i, x in enumerate(nodes):
        for j, e in enumerate(mons):
            V[i][j] = x[0] ** e[0] * x[1] ** e[1] * x[2] ** e[2]
    # solve V C = I by Gauss-Jordan: column b of C gives basis b's coefficients
    M = [row[:] + [Fraction(int(i == j)) for j in range(n)] for i, row in enumerate(V)]
    for c in range(n):
        piv = next(r for r in range(c, n) if M[r][c] != 0)
        M[c], M[piv] = M[piv], M[c]
        inv = 1 / M[c][c]
        M[c] = [v * inv for v in M[c]]
        for r in range(n):
            if r != c and M[r][c] != 0:
                f = M[r][c]
                M[r] = [vr - f * vc for vr, vc in zip(M[r], M[c])]
    C = [row[n:] for row in M]
    basis = [{mons[j]: C[j][b] for j in range(n) if C[j][b] != 0} for b in range(n)]
    grads = [[_poly_diff(p, d) for d in range(3)] for p in basis]
    K = [[sum(_int_ref_tet(_poly_mul(grads[a][d], grads[b][d])) for d in range(3))
          for b in range(n)] for a in range(n)]
    return np.array([[float(v) for v in row] for row in K])


@pytest.mark.parametrize("k", [2, 3, 4])
def test_element_matrix_equals_exact_rational(k):
    xyz = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1.0]])
    # a mesh made of one tet is enough for an element matrix
    P = oracle.Problem(xyz, np.array([[0, 1, 2, 3]], dtype=np.int32), k)
    K = P.element_matrix(0)
    Kx = _exact_lagrange_stiffness(k)
    assert np.max(np.abs(K - Kx)) < 1e-13 * np.max(np.abs(Kx))


@pytest.mark.parametrize("k", [2, 3, 4])
def test_element_matrix_invariants(k):
    xyz, tets = W.kuhn_mesh(2, jitter=0.2, seed=4)
    kappa = np.exp(np.random.default_rng(1).normal(size=tets.shape[0]))
    P = oracle.Problem(xyz, tets, k, kappa)
    al = oracle.multi_indices(k)
    for t in [0, 5, 17, 40]:
        K = P.element_matrix(t)
        X = xyz[tets[t]]
        nodes = (al / k) @ X                    # node positions in the tet
        vol = abs(np.linalg.det(X[1:] - X[0])) / 6.0
        assert np.max(np.abs(K - K.T)) < 1e-13 * np.max(np.abs(K))
        assert np.max(np.abs(K.sum(1))) < 1e-12 * np.max(np.abs(K))
        ev = np.linalg.eigvalsh(K)
        assert abs(ev[0]) < 1e-11 * ev[-1] and ev[1] > 1e-8 * ev[-1]
        # energy of interpolated x: kappa |T| |grad x|^2
        ux = nodes[:, 0]
        assert abs(ux @ K @ ux - kappa[t] * vol) < 1e-12 * kappa[t] * vol
        # energy of x^2: int_T 4 x^2 = 4 |T|/20 (sum x_a^2 + (sum x_a)^2)
        uq = nodes[:, 0] ** 2
        exact = 4 * kappa[t] * vol / 20 * (np.sum(X[:, 0] ** 2) + np.sum(X[:, 0]) ** 2)
        assert abs(uq @ K @ uq - exact) < 1e-12 * exact


@pytest.mark.parametrize("k", [2, 3, 4])
def test_six_term_edge_form_of_element_stiffness(k):
    """The form the matrix-free operator uses: since the barycentric gradients
    sum to zero, K_e = sum_{p<q} (-kappa G_pq) (M^pp + M^qq - M^pq - M^qp) with
    G_pq = |T| grad lam_p . grad lam_q and M^pq the reference tables."""
    al = oracle.multi_indices(k)
    nl = len(al)
    lam, w = oracle.tet_rule(k + 1)
    d = np.array([[oracle.basis_dlam(k, al[a], l) for a in range(nl)] for l in lam])   # [q][a][p]
    M = 6.0 * np.einsum("q,qap,qbr->prab", w, d, d)       # (1/|T|) int dphi_a/dlam_p dphi_b/dlam_r
    xyz, tets = W.kuhn_mesh(2, jitter=0.2, seed=3)
    kappa = np.exp(np.random.default_rng(4).normal(size=len(tets)))
    P = oracle.Problem(xyz, tets, k, kappa)
    for t in (0, 7, 30):
        X = xyz[tets[t]]
        J = (X[1:] - X[0]).T
        g = np.linalg.inv(J)                              # rows: grad lam_1..3
        grads = np.vstack([-g.sum(0), g])
        vol = abs(np.linalg.det(J)) / 6
        G = vol * grads @ grads.T
        assert np.max(np.abs(G.sum(1))) < 1e-14 * np.abs(G).max()
        K6 = sum(-kappa[t] * G[p, q] * (M[p, p] + M[q, q] - M[p, q] - M[q, p])
                 for p in range(4) for q in range(p + 1, 4))
        K = P.element_matrix(t)
        assert np.max(np.abs(K6 - K)) < 1e-12 * np.max(np.abs(K))
