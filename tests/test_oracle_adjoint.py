"""Pin of the oracle's kappa-gradient against finite differences.

For L(log kappa) = 0.5 ||u - u_t||^2 with A(kappa) u = f (f the load vector),
dL/dlog(kappa_t) = -lam_t^T K_t u_t where A lam = u - u_t.  Checked against
central differences of L computed with dense direct solves on a tiny mesh,
each perturbed kappa re-assembled from scratch.
"""
import numpy as np

import oracle
import workloads as W


def test_kappa_gradient_matches_central_differences():
    xyz, tets = W.kuhn_mesh(3, jitter=0.15, seed=7)
    rng = np.random.default_rng(0)
    logk = rng.normal(size=tets.shape[0])
    ut_logk = rng.normal(size=tets.shape[0])

    def solve(lk):
        P = oracle.Problem(xyz, tets, 2, np.exp(lk))
        return P, np.linalg.solve(P.csr("A").toarray(), P.load(W.manufactured_f))

    _, ut = solve(ut_logk)

    def loss(lk):
        return 0.5 * np.sum((solve(lk)[1] - ut) ** 2)

    P, u = solve(logk)
    lam = np.linalg.solve(P.csr("A").toarray(), u - ut)
    g = P.kappa_grad(u, lam)
    eps = 1e-5
    for t in rng.choice(tets.shape[0], size=8, replace=False):
        e = np.zeros_like(logk)
        e[t] = eps
        fd = (loss(logk + e) - loss(logk - e)) / (2 * eps)
        assert abs(fd - g[t]) <= 1e-6 * max(abs(g).max(), 1e-30), (t, fd, g[t])
    # a random direction
    d = rng.normal(size=logk.shape)
    d /= np.linalg.norm(d)
    fd = (loss(logk + eps * d) - loss(logk - eps * d)) / (2 * eps)
    assert abs(fd - g @ d) <= 1e-6 * abs(g @ d)
