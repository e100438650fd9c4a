"""Adjoint solve behind torch.autograd.Function, checked by finite differences.

Workload: P2 on the unit cube, 40^3 cubes x 6 tets (493,039 unknowns),
kappa = exp(g) with g a Gaussian random field (seed 1); target u_t from a
second field (seed 2); loss L = 0.5 ||u - u_t||^2 over the interior dofs.
Gradients with respect to the load vector f and to log kappa per tet come
from one adjoint CG solve (A is symmetric, same preconditioner) and the
element formula dL/dlog(kappa_t) = -lam_t^T K_t u_t; they are compared with
central differences along 16 random unit directions (each perturbed kappa is
set up from scratch), relative error <= 1e-5.  The same check runs at
P3 and P4 on small meshes.
"""
import numpy as np
import pytest
import torch

import paper_1204_2586_amd as aux
import workloads as W

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _loss(f, logk, ut, prob):
    u = aux.AuxSolveFn.apply(f, logk, prob)
    return 0.5 * torch.sum((u - ut) ** 2)


@pytest.mark.parametrize("k,n,ndir", [(2, 8, 4), (2, 40, 16), (3, 5, 4), (4, 4, 4)])
@pytest.mark.timeout(900)
def test_adjoint_gradients_match_finite_differences(k, n, ndir):
    print(f"[adjoint k={k} n={n}]", flush=True)
    xyz, tets = W.kuhn_mesh(n)
    logk = W.grf_log_kappa(xyz, tets, seed=1)
    logk_t = W.grf_log_kappa(xyz, tets, seed=2)
    prob = aux.KappaSolve(xyz, tets, k, tol=1e-12, device=DEV)
    f = torch.tensor(aux.Solver(xyz, tets, k, host_only=True).load(W.manufactured_f), device=DEV)
    with torch.no_grad():
        ut = aux.AuxSolveFn.apply(f, torch.tensor(logk_t, device=DEV), prob)
    fv = f.clone().requires_grad_(True)
    lk = torch.tensor(logk, device=DEV, requires_grad=True)
    L = _loss(fv, lk, ut, prob)
    L.backward()
    gk, gf = lk.grad.clone(), fv.grad.clone()
    assert torch.all(torch.isfinite(gk)) and torch.all(torch.isfinite(gf))
    eps = 1e-4
    with torch.no_grad():
        for i in range(ndir):
            rng = np.random.default_rng(100 + i)
            d = rng.normal(size=logk.shape)
            d /= np.linalg.norm(d)
            dt = torch.tensor(d, device=DEV)
            lp = _loss(f, torch.tensor(logk, device=DEV) + eps * dt, ut, prob)
            lm = _loss(f, torch.tensor(logk, device=DEV) - eps * dt, ut, prob)
            fd = float((lp - lm) / (2 * eps))
            an = float(gk @ dt)
            assert abs(fd - an) <= 1e-5 * abs(an), (i, fd, an)
        # L is quadratic in f: central differences are exact up to rounding
        df = torch.tensor(np.random.default_rng(7).normal(size=f.shape[0]), device=DEV)
        df /= torch.linalg.norm(df)
        h = 1e-3 * float(torch.linalg.norm(f))
        lk0 = torch.tensor(logk, device=DEV)
        fd = float((_loss(f + h * df, lk0, ut, prob) - _loss(f - h * df, lk0, ut, prob)) / (2 * h))
        an = float(gf @ df)
        assert abs(fd - an) <= 1e-5 * abs(an), (fd, an)
