"""Seeded synthetic inputs: meshes, coefficient fields and right-hand-side functions.

This module only *generates inputs* (vertex coordinates, tetrahedra, per-tet
coefficients, and point-wise source functions).  It holds none of the
discretisation or solver arithmetic, so both the CPU oracle and the GPU
library may take their inputs from it.

Workloads (the paper's model problem is -div(kappa grad u) = f on the unit
cube with u = 0 on the boundary, Sec. 2, eq. (2.1); the paper uses kappa = 1):

* ``kuhn_mesh(n, jitter, seed)`` -- the unit cube cut into n^3 cubes, each cube
  cut into 6 tetrahedra along the main diagonal (Kuhn/Freudenthal split).  It
  stands in for the unstructured tetrahedral unit-cube meshes of Sec. 6.
* ``grf_log_kappa`` -- a smooth Gaussian random field (random Fourier features
  of a squared-exponential covariance) evaluated at tet centroids.
* ``manufactured_f`` / ``manufactured_u`` -- u = sin(pi x) sin(pi y) sin(pi z),
  f = 3 pi^2 u.
* ``fourier_f(r)`` -- a smooth random source made of 16 sine modes.
* ``stokes_u`` / ``stokes_p`` / ``stokes_f`` -- a smooth divergence-free
  velocity with zero boundary values, a zero-mean pressure and the body force
  of the Stokes system (Sec. 5) they solve.
"""
from __future__ import annotations

import itertools
import math

import numpy as np

__all__ = [
    "kuhn_mesh",
    "grf_log_kappa",
    "manufactured_u",
    "manufactured_f",
    "fourier_f",
    "random_vector",
    "WORKLOADS",
    "make_config",
]

# the six permutations of the axes, in lexicographic order
_PERMS = list(itertools.permutations((0, 1, 2)))


def kuhn_mesh(n: int, jitter: float = 0.0, seed: int = 0):
    """Unit cube, n^3 cubes, 6 tets per cube.

    Vertex (i, j, l) has id (i*(n+1)+j)*(n+1)+l and position (i, j, l)/n.
    Cube c = (i, j, l) (lexicographic) gives tets 6*lex(c)+s for the axis
    permutations s in lexicographic order; the tet's vertices are the path
    c, c+e_a, c+e_a+e_b, c+e_a+e_b+e_c for the permutation (a, b, c).  All
    tets around a cube share its main diagonal, so the mesh is conforming.

    ``jitter`` moves every interior vertex independently per coordinate by
    uniform(-jitter*h, +jitter*h) drawn from ``numpy.random.default_rng(seed)``
    in vertex-id order.  The generator checks that no tet is inverted.

    Returns (xyz float64 [nv,3], tets int32 [nt,4]).
    """
    if n < 1:
        raise ValueError("n must be >= 1")
    h = 1.0 / n
    m = n + 1
    g = np.arange(m)
    I, J, L = np.meshgrid(g, g, g, indexing="ij")
    xyz = np.stack([I.ravel(), J.ravel(), L.ravel()], axis=1).astype(np.float64) * h

    ci, cj, cl = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    base = np.stack([ci.ravel(), cj.ravel(), cl.ravel()], axis=1)  # [n^3, 3]
    tets = np.empty((n ** 3, 6, 4), dtype=np.int64)
    for s, perm in enumerate(_PERMS):
        p = base.copy()
        tets[:, s, 0] = (p[:, 0] * m + p[:, 1]) * m + p[:, 2]
        for step, ax in enumerate(perm):
            p[:, ax] += 1
            tets[:, s, step + 1] = (p[:, 0] * m + p[:, 1]) * m + p[:, 2]
    tets = tets.reshape(-1, 4).astype(np.int32)

    if jitter:
        interior = np.all((xyz > 0.5 * h) & (xyz < 1.0 - 0.5 * h), axis=1)
        rng = np.random.default_rng(seed)
        off = rng.uniform(-jitter * h, jitter * h, size=(int(interior.sum()), 3))
        ref = _signed_volumes(xyz, tets)
        xyz[interior] += off
        vol = _signed_volumes(xyz, tets)
        if np.any(np.sign(vol) != np.sign(ref)) or np.any(np.abs(vol) < 1e-3 * h ** 3 / 6.0):
            raise ValueError("jitter inverted or flattened a tetrahedron")
    return xyz, tets


def _signed_volumes(xyz, tets):
    x = xyz[tets]
    e1, e2, e3 = x[:, 1] - x[:, 0], x[:, 2] - x[:, 0], x[:, 3] - x[:, 0]
    return np.einsum("ij,ij->i", e1, np.cross(e2, e3)) / 6.0


def tet_centroids(xyz, tets):
    return xyz[tets].mean(axis=1)


def grf_log_kappa(xyz, tets, sigma: float = 2.3, ell: float = 0.1, n_features: int = 1024,
                  seed: int = 1, chunk: int = 65536):
    """Smooth Gaussian random field g at tet centroids; kappa = exp(g).

    g(x) = sigma*sqrt(2/M) * sum_m cos(w_m . x + b_m), w_m ~ N(0, ell^-2 I),
    b_m ~ U[0, 2 pi), M = n_features, all drawn from default_rng(seed) (w first,
    then b).  Its covariance tends to sigma^2 exp(-|x-y|^2 / (2 ell^2)).
    """
    rng = np.random.default_rng(seed)
    w = rng.normal(0.0, 1.0 / ell, size=(n_features, 3))
    b = rng.uniform(0.0, 2.0 * math.pi, size=n_features)
    c = tet_centroids(xyz, tets)
    g = np.empty(c.shape[0])
    scale = sigma * math.sqrt(2.0 / n_features)
    for s in range(0, c.shape[0], chunk):
        g[s:s + chunk] = scale * np.cos(c[s:s + chunk] @ w.T + b).sum(axis=1)
    return g


def manufactured_u(p):
    p = np.asarray(p, dtype=np.float64)
    return np.sin(np.pi * p[..., 0]) * np.sin(np.pi * p[..., 1]) * np.sin(np.pi * p[..., 2])


def manufactured_f(p):
    """f = -Laplace(u) for u = sin(pi x) sin(pi y) sin(pi z)."""
    return 3.0 * np.pi ** 2 * manufactured_u(p)


# Stokes manufactured solution (velocity u = curl(0, 0, psi) with
# psi = sin^2(pi x) sin^2(pi y) sin^2(pi z): divergence free, u and grad psi
# vanish on the boundary; pressure p = cos(pi x) cos(pi y) cos(pi z), zero
# mean), body force f = -Laplace(u) + grad(p).
def _s2(t):
    return np.sin(np.pi * t) ** 2


def _d1(t):       # d/dt sin^2(pi t)
    return np.pi * np.sin(2 * np.pi * t)


def _d2(t):
    return 2 * np.pi ** 2 * np.cos(2 * np.pi * t)


def _d3(t):
    return -4 * np.pi ** 3 * np.sin(2 * np.pi * t)


def stokes_u(c: int):
    """Component c of the manufactured Stokes velocity."""
    def f(q):
        q = np.asarray(q, dtype=np.float64)
        x, y, z = q[..., 0], q[..., 1], q[..., 2]
        if c == 0:
            return _s2(x) * _d1(y) * _s2(z)
        if c == 1:
            return -_d1(x) * _s2(y) * _s2(z)
        return np.zeros(q.shape[:-1])
    return f


def stokes_p(q):
    q = np.asarray(q, dtype=np.float64)
    return np.cos(np.pi * q[..., 0]) * np.cos(np.pi * q[..., 1]) * np.cos(np.pi * q[..., 2])


def stokes_f(c: int):
    """Component c of the body force -Laplace(u) + grad(p) of the manufactured solution."""
    pi = np.pi

    def f(q):
        q = np.asarray(q, dtype=np.float64)
        x, y, z = q[..., 0], q[..., 1], q[..., 2]
        if c == 0:
            lap = _d2(x) * _d1(y) * _s2(z) + _s2(x) * _d3(y) * _s2(z) + _s2(x) * _d1(y) * _d2(z)
            gp = -pi * np.sin(pi * x) * np.cos(pi * y) * np.cos(pi * z)
        elif c == 1:
            lap = -(_d3(x) * _s2(y) * _s2(z) + _d1(x) * _d2(y) * _s2(z) + _d1(x) * _s2(y) * _d2(z))
            gp = -pi * np.cos(pi * x) * np.sin(pi * y) * np.cos(pi * z)
        else:
            lap = 0.0
            gp = -pi * np.cos(pi * x) * np.cos(pi * y) * np.sin(pi * z)
        return -lap + gp
    return f


def fourier_f(r: int, n_modes: int = 16, kmax: int = 4):
    """Random smooth source number r: sum of 16 products of sines.

    f_r(x) = sum_m a_m sin(pi k1 x) sin(pi k2 y) sin(pi k3 z) with a_m ~ N(0,1)
    and (k1, k2, k3) ~ U{1..kmax}^3, drawn from default_rng(1000 + r)
    (amplitudes first, then wave numbers).
    """
    rng = np.random.default_rng(1000 + r)
    a = rng.normal(size=n_modes)
    k = rng.integers(1, kmax + 1, size=(n_modes, 3))

    def f(p):
        p = np.asarray(p, dtype=np.float64)
        out = np.zeros(p.shape[:-1])
        for m in range(n_modes):
            out += a[m] * (np.sin(np.pi * k[m, 0] * p[..., 0]) * np.sin(np.pi * k[m, 1] * p[..., 1])
                           * np.sin(np.pi * k[m, 2] * p[..., 2]))
        return out

    return f


def fourier_fields(rs, n_modes: int = 16, kmax: int = 4):
    """The sources fourier_f(r) for every r in rs, evaluated together.

    Returns f(p) -> array [len(rs), ...] (one row per source).  Every mode is a product
    sin(pi k1 x) sin(pi k2 y) sin(pi k3 z) with k in 1..kmax, so all sources
    are combinations of the same kmax^3 products: those are formed once per
    call and combined by one matrix product with the [kmax^3, len(rs)]
    amplitude table (equal to fourier_f up to rounding order).
    """
    rs = list(rs)
    amp = np.zeros((kmax ** 3, len(rs)))
    for c, r in enumerate(rs):
        rng = np.random.default_rng(1000 + r)
        a = rng.normal(size=n_modes)
        k = rng.integers(1, kmax + 1, size=(n_modes, 3))
        for m in range(n_modes):
            amp[((k[m, 0] - 1) * kmax + k[m, 1] - 1) * kmax + k[m, 2] - 1, c] += a[m]
    used = np.flatnonzero(np.any(amp != 0.0, axis=1))

    def f(p):
        p = np.asarray(p, dtype=np.float64)
        flat = p.reshape(-1, 3)
        tab = [np.sin(np.pi * np.arange(1, kmax + 1)[:, None] * flat[None, :, ax]) for ax in range(3)]
        prod = np.empty((len(used), flat.shape[0]))
        for j, idx in enumerate(used):
            k1, rem = divmod(int(idx), kmax * kmax)
            k2, k3 = divmod(rem, kmax)
            np.multiply(tab[0][k1], tab[1][k2], out=prod[j])
            prod[j] *= tab[2][k3]
        return (amp[used].T @ prod).reshape((len(rs),) + p.shape[:-1])

    return f


def random_vector(n: int, seed: int, dtype=np.float64):
    """Seeded N(0,1) vector (used as a residual to precondition)."""
    return np.random.default_rng(seed).standard_normal(n).astype(dtype)


# The five workloads: (name, k, n, jitter, kappa spec, rhs spec, extra)
WORKLOADS = {
    "p2_n8": dict(k=2, n=8, jitter=0.0, kappa=None, rhs="manufactured"),
    "p2_n48_jitter": dict(k=2, n=48, jitter=0.2, jitter_seed=0, kappa=None, rhs="manufactured"),
    "p3_n32_grf": dict(k=3, n=32, jitter=0.0, kappa=("grf", 1), rhs="manufactured"),
    "p2_n64_32rhs": dict(k=2, n=64, jitter=0.0, kappa=None, rhs=("fourier", 32)),
    "p2_n40_adjoint": dict(k=2, n=40, jitter=0.0, kappa=("grf", 1), kappa_target=("grf", 2),
                           rhs="manufactured"),
}


def make_config(name: str, n: int | None = None):
    """Mesh and coefficient of a named workload (n may be overridden to shrink it).

    Returns dict(xyz, tets, kappa, k, n, rhs).
    """
    c = dict(WORKLOADS[name])
    if n is not None:
        c["n"] = n
    xyz, tets = kuhn_mesh(c["n"], c.get("jitter", 0.0), c.get("jitter_seed", 0))
    kappa = None
    if c["kappa"] is not None:
        kappa = np.exp(grf_log_kappa(xyz, tets, seed=c["kappa"][1]))
    out = dict(xyz=xyz, tets=tets, kappa=kappa, k=c["k"], n=c["n"], rhs=c["rhs"])
    if "kappa_target" in c:
        out["kappa_target"] = np.exp(grf_log_kappa(xyz, tets, seed=c["kappa_target"][1]))
    return out
