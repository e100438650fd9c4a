"""Pins of the oracle's smoother weight: G_h = omega D_l1^{-1} on the P^k
level (omega = 1 is the plain l1-Jacobi of reading R1).

* omega = 1 set explicitly is the default, bit for bit.
* For 0 < omega <= 1 the damped l1-Jacobi is still convergent, so B stays
  symmetric positive definite with the spectrum of B A_h in (0, 1], also
  with a multi-level AMG cycle and with the intermediate P^2 space.
* omega < 0 makes B indefinite (the smoothing part negative definite, the
  coarse correction positive): CG must stop within the first steps with the
  breakdown status (r.z <= 0 or p.Ap <= 0), the failure path the ABI
  reports as AUX_EBREAKDOWN.
"""
import numpy as np
import pytest

import oracle
import workloads as W


def _problem(k, n, coarse_max=8, omega=None):
    xyz, tets = W.kuhn_mesh(n, jitter=0.2, seed=3)
    P = oracle.Problem(xyz, tets, k)
    if omega is not None:
        P.set_smoother_weight(omega)
    return P.setup_amg(coarse_max=coarse_max)


def test_unit_weight_is_the_default():
    a, b = _problem(2, 4), _problem(2, 4, omega=1.0)
    r = np.random.default_rng(1).standard_normal(a.n)
    assert np.array_equal(a.apply(r), b.apply(r))


@pytest.mark.parametrize("k,n,omega", [(2, 4, 0.5), (2, 4, 0.8), (3, 4, 0.7)])
def test_damped_preconditioner_spd(k, n, omega):
    P = _problem(k, n, omega=omega)
    assert P.nlev >= 2
    m = P.n
    B = np.column_stack([P.apply(np.eye(m)[:, j]) for j in range(m)])
    assert np.max(np.abs(B - B.T)) <= 1e-13 * np.max(np.abs(B))
    A = P.csr("A").toarray()
    ev = np.linalg.eigvals(B @ A).real
    assert ev.min() > 0 and ev.max() <= 1 + 1e-12
    # the weight changes B (it is not ignored)
    r = np.random.default_rng(2).standard_normal(m)
    assert np.linalg.norm(P.apply(r) - _problem(k, n).apply(r)) > 1e-3 * np.linalg.norm(P.apply(r))


def test_damped_nested_preconditioner_spd():
    xyz, tets = W.kuhn_mesh(2, jitter=0.2, seed=3)
    P = oracle.Problem(xyz, tets, 4).set_smoother_weight(0.8).setup_nested()
    assert P.aux2.omega == 0.8
    m = P.n
    B = np.column_stack([P.apply_nested(np.eye(m)[:, j]) for j in range(m)])
    assert np.max(np.abs(B - B.T)) <= 1e-13 * np.max(np.abs(B))
    ev = np.linalg.eigvals(B @ P.csr("A").toarray()).real
    assert ev.min() > 0 and ev.max() <= 1 + 1e-12


def test_negative_weight_breaks_down():
    P = _problem(2, 4, omega=-1.0)
    x, it, rr, st = P.pcg(P.load(W.manufactured_f), tol=1e-8)
    assert st == 2 and it <= 2, (st, it)
