"""CPU oracle of the GAMG-preconditioned CG method (test infrastructure).

Only the tests, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` use this package.  It wraps the plain single-threaded FP64 C code
in this directory (``liboracle.so``, built by ``oracle/build.py``) and shares
no code with the GPU library.

What it computes (Lee, Leng and Zhang, arXiv:1204.2586):

* P^k Lagrange discretisation of -div(kappa grad u) = f, u = 0 on the
  boundary (Sec. 2, eq. (2.1)-(2.5)); kappa is constant per tet (the paper
  uses kappa = 1).
* the P^1 auxiliary space, I_P with c_j^i = psi_j(x_i^h) and I_R = I_P^T
  (Sec. 2, eq. "Prol");
* AMG setup on A_H: strength rule of Sec. 6.2, PMIS coarsening and
  extended+i interpolation (the BoomerAMG options named in Sec. 1 and 6.1);
* the preconditioner of Algorithm 2.1 with presmoothing (Remark 2.1),
  l1-Jacobi smoothing, one V(1,1) AMG cycle for Step 1;
* preconditioned CG, in FP64 or with the preconditioner in FP32, and the
  flexible GMRES(m) of the paper's experiments (Sec. 6.1).
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

_i32p = np.ctypeslib.ndpointer(np.int32, flags="C_CONTIGUOUS")
_f64p = np.ctypeslib.ndpointer(np.float64, flags="C_CONTIGUOUS")
_i64p = np.ctypeslib.ndpointer(np.int64, flags="C_CONTIGUOUS")


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        from . import build as _b
        _b.build()
    lib = ctypes.CDLL(_LIB_PATH)
    vp = ctypes.c_void_p
    lib.orc_create.restype = vp
    lib.orc_create.argtypes = [ctypes.c_int, _f64p, ctypes.c_int, _i32p, ctypes.c_int, vp]
    lib.orc_setup_amg.restype = ctypes.c_int
    lib.orc_setup_amg.argtypes = [vp, ctypes.c_double, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                  ctypes.c_uint64]
    lib.orc_free.argtypes = [vp]
    lib.orc_sizes.argtypes = [vp, _i64p]
    lib.orc_csr_shape.argtypes = [vp, ctypes.c_int, ctypes.c_int, _i64p]
    lib.orc_csr_copy.argtypes = [vp, ctypes.c_int, ctypes.c_int, _i32p, _i32p, _f64p]
    lib.orc_level_cf.argtypes = [vp, ctypes.c_int, _i32p]
    lib.orc_level_round.argtypes = [vp, ctypes.c_int, _i32p]
    lib.orc_apply_vcycle.argtypes = [vp, ctypes.c_int, _f64p, _f64p]
    lib.orc_interp_given.restype = ctypes.c_int
    lib.orc_interp_given.argtypes = [ctypes.c_int, _i32p, _i32p, _f64p, ctypes.c_double, _i32p, ctypes.c_int,
                                     _i32p, _i32p, _f64p]
    lib.orc_dof_keys.argtypes = [vp, _i32p]
    lib.orc_tet_dofs.argtypes = [vp, _i32p]
    lib.orc_l1.argtypes = [vp, _f64p]
    lib.orc_coarse_chol.argtypes = [vp, _f64p]
    lib.orc_element_matrix.argtypes = [vp, ctypes.c_int, _f64p]
    lib.orc_qpoints.argtypes = [vp, ctypes.c_int, _f64p]
    lib.orc_load.argtypes = [vp, ctypes.c_int, _f64p, _f64p]
    lib.orc_l2_error.restype = ctypes.c_double
    lib.orc_l2_error.argtypes = [vp, ctypes.c_int, _f64p, _f64p]
    lib.orc_h1_error.restype = ctypes.c_double
    lib.orc_h1_error.argtypes = [vp, ctypes.c_int, _f64p, _f64p]
    lib.orc_apply_precond.argtypes = [vp, ctypes.c_int, _f64p, _f64p]
    lib.orc_pcg.restype = ctypes.c_int
    lib.orc_pcg.argtypes = [vp, ctypes.c_int, _f64p, _f64p, ctypes.c_double, ctypes.c_int,
                            ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_double)]
    lib.orc_fgmres.restype = ctypes.c_int
    lib.orc_fgmres.argtypes = [vp, ctypes.c_int, _f64p, _f64p, ctypes.c_double, ctypes.c_int, ctypes.c_int,
                               vp, vp, _f64p]
    lib.orc_kappa_grad.argtypes = [vp, _f64p, _f64p, _f64p]
    lib.orc_stokes_setup.restype = ctypes.c_int
    lib.orc_stokes_setup.argtypes = [vp]
    lib.orc_set_smoother_weight.argtypes = [vp, ctypes.c_double]
    lib.orc_setup_nested.restype = ctypes.c_int
    lib.orc_setup_nested.argtypes = [vp, vp, ctypes.c_int]
    lib.orc_apply_nested.restype = ctypes.c_int
    lib.orc_apply_nested.argtypes = [vp, ctypes.c_int, _f64p, _f64p]
    lib.orc_pcg_nested.restype = ctypes.c_int
    lib.orc_pcg_nested.argtypes = [vp, ctypes.c_int, _f64p, _f64p, ctypes.c_double, ctypes.c_int,
                                   ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_double)]
    lib.orc_stokes_fgmres.restype = ctypes.c_int
    lib.orc_stokes_fgmres.argtypes = [vp, ctypes.c_int, _f64p, _f64p, ctypes.c_double, ctypes.c_int, ctypes.c_int,
                                      ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_double), _f64p]
    lib.orc_stokes_apply_operator.argtypes = [vp, _f64p, _f64p]
    lib.orc_stokes_np.restype = ctypes.c_int
    lib.orc_stokes_np.argtypes = [vp]
    lib.orc_pressure_keys.restype = ctypes.c_int
    lib.orc_pressure_keys.argtypes = [vp, _i32p]
    lib.orc_pressure_l2_error.restype = ctypes.c_double
    lib.orc_pressure_l2_error.argtypes = [vp, ctypes.c_int, _f64p, _f64p]
    lib.orc_stokes_apply_qt.restype = ctypes.c_int
    lib.orc_stokes_apply_qt.argtypes = [vp, ctypes.c_int, _f64p, _f64p]
    lib.orc_block_pcg.restype = ctypes.c_int
    lib.orc_block_pcg.argtypes = [vp, ctypes.c_int, ctypes.c_int, _f64p, _f64p, ctypes.c_double, ctypes.c_int,
                                  ctypes.POINTER(ctypes.c_int), _f64p]
    lib.orc_gauss_jacobi.argtypes = [ctypes.c_int, ctypes.c_int, _f64p, _f64p]
    lib.orc_tet_rule.argtypes = [ctypes.c_int, _f64p, _f64p]
    lib.orc_local_multi_indices.argtypes = [ctypes.c_int, _i32p]
    lib.orc_basis.restype = ctypes.c_double
    lib.orc_basis.argtypes = [ctypes.c_int, _i32p, _f64p]
    lib.orc_basis_dlam.argtypes = [ctypes.c_int, _i32p, _f64p, _f64p]
    lib.orc_splitmix64.restype = ctypes.c_uint64
    lib.orc_splitmix64.argtypes = [ctypes.c_uint64]
    lib.orc_pmis_rho.restype = ctypes.c_uint64
    lib.orc_pmis_rho.argtypes = [ctypes.c_uint64, ctypes.c_int, ctypes.c_int]
    _lib = lib
    return lib


# ------------------------------------------------------------ element level

def splitmix64(z: int) -> int:
    """Output of splitmix64 for state z (the oracle's PMIS random source)."""
    return int(_load().orc_splitmix64(z))


def pmis_rho(seed: int, level: int, i: int) -> int:
    return int(_load().orc_pmis_rho(seed, level, i))


def multi_indices(k: int) -> np.ndarray:
    """Local nodes of a P^k tet as multi-indices alpha (|alpha| = k), lexicographic."""
    nloc = (k + 1) * (k + 2) * (k + 3) // 6
    a = np.zeros(nloc * 4, dtype=np.int32)
    _load().orc_local_multi_indices(k, a)
    return a.reshape(nloc, 4)


def basis(k: int, alpha, lam) -> float:
    return _load().orc_basis(k, np.ascontiguousarray(alpha, dtype=np.int32),
                             np.ascontiguousarray(lam, dtype=np.float64))


def basis_dlam(k: int, alpha, lam) -> np.ndarray:
    d = np.zeros(4)
    _load().orc_basis_dlam(k, np.ascontiguousarray(alpha, dtype=np.int32),
                           np.ascontiguousarray(lam, dtype=np.float64), d)
    return d


def gauss_jacobi(m: int, a: int):
    """m-point rule for int_0^1 (1-x)^a g(x) dx -> (nodes, weights)."""
    x, w = np.zeros(m), np.zeros(m)
    if _load().orc_gauss_jacobi(m, a, x, w):
        raise ValueError("bad rule")
    return x, w


def tet_rule(m: int):
    """Conical-product rule on the reference tet: (lam [m^3,4], w [m^3]), sum(w) = 1/6."""
    lam, w = np.zeros(m ** 3 * 4), np.zeros(m ** 3)
    _load().orc_tet_rule(m, lam, w)
    return lam.reshape(-1, 4), w


def interp_given(A, cf, theta: float = 0.8):
    """Extended+i interpolation of the square scipy CSR matrix A for the given
    C/F splitting (cf[i] = +1 C, -1 F) with the strength sets of threshold
    theta; returns P as a scipy CSR matrix (rows of A, columns = C points in
    increasing index)."""
    import scipy.sparse as sp
    A = sp.csr_matrix(A)
    A.sort_indices()
    n = A.shape[0]
    cf = np.ascontiguousarray(cf, dtype=np.int32)
    cap = n * n + 1
    ptr, col, val = np.zeros(n + 1, dtype=np.int32), np.zeros(cap, dtype=np.int32), np.zeros(cap)
    nnz = _load().orc_interp_given(n, A.indptr.astype(np.int32), A.indices.astype(np.int32),
                                   A.data.astype(np.float64), theta, cf, cap, ptr, col, val)
    if nnz < 0:
        raise RuntimeError("interpolation larger than expected")
    return sp.csr_matrix((val[:nnz], col[:nnz], ptr), shape=(n, int((cf > 0).sum())))


# ---------------------------------------------------------------- problem

class Problem:
    """Discretisation plus (after ``setup_amg``) the AMG hierarchy."""

    def __init__(self, xyz, tets, k: int, kappa=None):
        lib = _load()
        self.xyz = np.ascontiguousarray(xyz, dtype=np.float64)
        self.tets = np.ascontiguousarray(tets, dtype=np.int32)
        self.k = k
        kap = None
        if kappa is not None:
            self._kappa = np.ascontiguousarray(kappa, dtype=np.float64)
            kap = self._kappa.ctypes.data_as(ctypes.c_void_p)
        self._h = lib.orc_create(self.xyz.shape[0], self.xyz.ravel(), self.tets.shape[0],
                                 self.tets.ravel(), k, kap)
        if not self._h:
            raise ValueError("oracle: discretisation failed")
        self._amg = False
        self.omega = 1.0
        self._refresh()

    def _refresh(self):
        s = np.zeros(16, dtype=np.int64)
        _load().orc_sizes(self._h, s)
        (self.n, self.nH, self.nnode, self.nlev, self.nnz_A, self.nnz_AH, self.nnz_IP,
         self.ncoarse, self.nloc) = [int(v) for v in s[:9]]

    def __del__(self):
        h = getattr(self, "_h", None)
        if h and _lib is not None:
            _lib.orc_free(h)
            self._h = None

    def setup_amg(self, theta=0.8, nu=2, coarse_max=100, max_levels=25, seed=0):
        rc = _load().orc_setup_amg(self._h, theta, nu, coarse_max, max_levels, seed)
        if rc:
            raise RuntimeError(f"oracle AMG setup failed ({rc})")
        self._amg = True
        self.nu = nu
        self._refresh()
        return self

    # ---- matrices
    def csr(self, which: str, level: int = 0):
        """'A' (A_h), 'AH', 'IP', 'Alev' (level operator), 'P' (level interpolation),
        'B' (Stokes divergence, after stokes_setup), 'Mp' (pressure mass matrix),
        'I2' (P^k <- P^2 transfer, after setup_nested)."""
        import scipy.sparse as sp
        code = {"A": 0, "AH": 1, "IP": 2, "Alev": 3, "P": 4, "B": 5, "Mp": 6, "I2": 7}[which]
        shp = np.zeros(3, dtype=np.int64)
        if _load().orc_csr_shape(self._h, code, level, shp):
            raise IndexError("no such matrix")
        n, m, nnz = (int(v) for v in shp)
        ptr = np.zeros(n + 1, dtype=np.int32)
        col = np.zeros(max(nnz, 1), dtype=np.int32)
        val = np.zeros(max(nnz, 1))
        _load().orc_csr_copy(self._h, code, level, ptr, col, val)
        return sp.csr_matrix((val[:nnz], col[:nnz], ptr), shape=(n, m))

    def level_cf(self, level: int) -> np.ndarray:
        n = self.csr("Alev", level).shape[0]
        cf = np.zeros(n, dtype=np.int32)
        if _load().orc_level_cf(self._h, level, cf):
            raise IndexError("coarsest level has no splitting")
        return cf

    def level_rounds(self, level: int) -> np.ndarray:
        """PMIS round in which each point of the level was decided (0: points
        influencing nobody, made F before the first round)."""
        n = self.csr("Alev", level).shape[0]
        rd = np.zeros(n, dtype=np.int32)
        if _load().orc_level_round(self._h, level, rd):
            raise IndexError("coarsest level has no splitting")
        return rd

    def dof_keys(self) -> np.ndarray:
        keys = np.zeros(self.n * self.k, dtype=np.int32)
        _load().orc_dof_keys(self._h, keys)
        return keys.reshape(self.n, self.k)

    def tet_dofs(self) -> np.ndarray:
        out = np.zeros(self.tets.shape[0] * self.nloc, dtype=np.int32)
        _load().orc_tet_dofs(self._h, out)
        return out.reshape(-1, self.nloc)

    def l1(self) -> np.ndarray:
        d = np.zeros(self.n)
        _load().orc_l1(self._h, d)
        return d

    def coarse_cholesky(self) -> np.ndarray:
        L = np.zeros(self.ncoarse * self.ncoarse)
        _load().orc_coarse_chol(self._h, L)
        return L.reshape(self.ncoarse, self.ncoarse)

    def element_matrix(self, t: int) -> np.ndarray:
        K = np.zeros(self.nloc * self.nloc)
        _load().orc_element_matrix(self._h, t, K)
        return K.reshape(self.nloc, self.nloc)

    # ---- load vector and errors
    def qpoints(self, m: int | None = None) -> np.ndarray:
        m = self.k + 2 if m is None else m
        out = np.zeros(self.tets.shape[0] * m ** 3 * 3)
        _load().orc_qpoints(self._h, m, out)
        return out.reshape(-1, 3)

    def load(self, f, m: int | None = None) -> np.ndarray:
        """b_i = <f, phi_i> by the conical-product rule with m = k+2 points per direction."""
        m = self.k + 2 if m is None else m
        fq = np.ascontiguousarray(f(self.qpoints(m)), dtype=np.float64)
        b = np.zeros(self.n)
        _load().orc_load(self._h, m, fq, b)
        return b

    def l2_error(self, u_exact, u, m: int | None = None) -> float:
        m = self.k + 3 if m is None else m
        uq = np.ascontiguousarray(u_exact(self.qpoints(m)), dtype=np.float64)
        return _load().orc_l2_error(self._h, m, uq, np.ascontiguousarray(u, dtype=np.float64))

    def h1_error(self, grad_exact, u, m: int | None = None) -> float:
        m = self.k + 3 if m is None else m
        gq = np.ascontiguousarray(grad_exact(self.qpoints(m)), dtype=np.float64)
        return _load().orc_h1_error(self._h, m, gq.ravel(), np.ascontiguousarray(u, dtype=np.float64))

    # ---- preconditioner and solver
    def apply(self, r, fp32: bool = False) -> np.ndarray:
        assert self._amg, "call setup_amg first"
        z = np.zeros(self.n)
        _load().orc_apply_precond(self._h, int(fp32), np.ascontiguousarray(r, dtype=np.float64), z)
        return z

    def vcycle(self, b, fp32: bool = False) -> np.ndarray:
        """One AMG V(1,1) cycle from zero on the P^1 system (Step 1 of
        Algorithm 2.1 on its own): x = V b, b and x of length n_H."""
        assert self._amg, "call setup_amg first"
        x = np.zeros(self.nH)
        if _load().orc_apply_vcycle(self._h, int(fp32), np.ascontiguousarray(b, dtype=np.float64), x):
            raise ValueError("no P^1 unknowns")
        return x

    def pcg(self, b, tol=1e-8, maxit=1000, x0=None, fp32: bool = False):
        """Returns (x, iterations, relative recursive residual, status)."""
        assert self._amg, "call setup_amg first"
        x = np.zeros(self.n) if x0 is None else np.array(x0, dtype=np.float64)
        it = ctypes.c_int(0)
        rr = ctypes.c_double(0.0)
        st = _load().orc_pcg(self._h, int(fp32), np.ascontiguousarray(b, dtype=np.float64), x, tol,
                             maxit, ctypes.byref(it), ctypes.byref(rr))
        return x, it.value, rr.value, st

    def set_smoother_weight(self, omega: float):
        """The P^k smoother G_h = omega D_l1^{-1} (1 = plain l1-Jacobi); also used
        by the intermediate space's P^2 problem set up afterwards."""
        _load().orc_set_smoother_weight(self._h, float(omega))
        self.omega = float(omega)
        return self

    # ---- intermediate auxiliary space (Remark 6.2)
    def setup_nested(self, theta=0.8, nu=2, coarse_max=100, max_levels=25, seed=0):
        """P^2 on the same mesh as the auxiliary space of this P^k problem
        (k >= 2), its own problem solved by one application of its
        auxiliary-space preconditioner (P^2 smoothing around the P^1 AMG
        cycle, with these AMG options).  Keeps the P^2 problem as ``aux2``."""
        kap = getattr(self, "_kappa", None)
        self.aux2 = Problem(self.xyz, self.tets, 2, kap).setup_amg(theta=theta, nu=nu, coarse_max=coarse_max,
                                                                  max_levels=max_levels, seed=seed)
        self.aux2.set_smoother_weight(self.omega)
        if _load().orc_setup_nested(self._h, self.aux2._h, nu):
            raise RuntimeError("oracle: nested transfer failed")
        self.nu = nu
        return self

    def apply_nested(self, r, fp32: bool = False) -> np.ndarray:
        """z = B r with the intermediate P^2 space (after setup_nested)."""
        z = np.zeros(self.n)
        if _load().orc_apply_nested(self._h, int(fp32), np.ascontiguousarray(r, dtype=np.float64), z):
            raise RuntimeError("call setup_nested first")
        return z

    def pcg_nested(self, b, tol=1e-8, maxit=1000, x0=None, fp32: bool = False):
        """PCG with the intermediate-space preconditioner: (x, iterations,
        relative recursive residual, status)."""
        x = np.zeros(self.n) if x0 is None else np.array(x0, dtype=np.float64)
        it = ctypes.c_int(0)
        rr = ctypes.c_double(0.0)
        st = _load().orc_pcg_nested(self._h, int(fp32), np.ascontiguousarray(b, dtype=np.float64), x, tol,
                                    maxit, ctypes.byref(it), ctypes.byref(rr))
        if st < 0:
            raise RuntimeError("call setup_nested first")
        return x, it.value, rr.value, st

    # ---- Stokes (Sec. 5), Hood-Taylor P^2-P^1
    def stokes_setup(self):
        """Hood-Taylor P^k - P^{k-1} (k = 2, 3, 4): divergence B (n_p x 3 n_h,
        -div) and pressure mass matrix M_p, the pressure on every node of
        order k-1 (vertex order for P^1)."""
        if _load().orc_stokes_setup(self._h):
            raise ValueError("Stokes needs a velocity order of 2, 3 or 4")
        self.np = _load().orc_stokes_np(self._h)
        return self

    def pressure_keys(self) -> np.ndarray:
        """Node key of each pressure unknown: [n_p][k-1] sorted vertex ids."""
        keys = np.zeros((self.np, self.k - 1), dtype=np.int32)
        _load().orc_pressure_keys(self._h, keys)
        return keys

    def pressure_xyz(self) -> np.ndarray:
        """Position of each pressure node (the mean of its key's vertices)."""
        return self.xyz[self.pressure_keys()].mean(axis=1)

    def pressure_l2_error(self, p_exact, ph, m: int | None = None) -> float:
        m = self.k + 3 if m is None else m
        pq = np.ascontiguousarray(p_exact(self.qpoints(m)), dtype=np.float64)
        return _load().orc_pressure_l2_error(self._h, m, pq, np.ascontiguousarray(ph, dtype=np.float64))

    def stokes_operator(self, x) -> np.ndarray:
        out = np.zeros(3 * self.n + self.np)
        _load().orc_stokes_apply_operator(self._h, np.ascontiguousarray(x, dtype=np.float64), out)
        return out

    def stokes_qt(self, r, fp32: bool = False, steps: bool = False):
        """Q_t r; with steps=True also the pressure mass solve's CG step count."""
        out = np.zeros(3 * self.n + self.np)
        k = _load().orc_stokes_apply_qt(self._h, int(fp32), np.ascontiguousarray(r, dtype=np.float64), out)
        return (out, k) if steps else out

    def stokes_fgmres(self, b, tol=1e-8, restart=30, maxit=500, x0=None, fp32: bool = False):
        """FGMRES(restart) with the block triangular preconditioner Q_t on the
        saddle-point system [A B^T; B 0] [u; p] = b, unknowns [u_x; u_y; u_z; p].
        Returns (x, steps, true relative residual, status, history)."""
        assert self._amg, "call setup_amg first"
        N = 3 * self.n + self.np
        x = np.zeros(N) if x0 is None else np.array(x0, dtype=np.float64)
        it = ctypes.c_int(0)
        rr = ctypes.c_double(0.0)
        hist = np.zeros(maxit + 1)
        st = _load().orc_stokes_fgmres(self._h, int(fp32), np.ascontiguousarray(b, dtype=np.float64), x, tol,
                                       restart, maxit, ctypes.byref(it), ctypes.byref(rr), hist)
        return x, it.value, rr.value, st, hist[: it.value + 1]

    def block_pcg(self, F, tol=1e-8, maxit=1000, X0=None, fp32: bool = False):
        """O'Leary's block preconditioned CG on A_h X = F (F [n, s]); stops
        when every column meets ||r_j|| <= tol ||f_j||.  Returns (X,
        iterations, per-column relative residuals, status: 0 converged,
        1 maxit, 2 breakdown, 3 NaN)."""
        assert self._amg, "call setup_amg first"
        F = np.ascontiguousarray(F, dtype=np.float64)
        s = F.shape[1]
        X = np.zeros_like(F) if X0 is None else np.array(X0, dtype=np.float64)
        it = ctypes.c_int(0)
        rel = np.zeros(s)
        st = _load().orc_block_pcg(self._h, int(fp32), s, F, X, tol, maxit, ctypes.byref(it), rel)
        return X, it.value, rel, st

    def fgmres(self, b, tol=1e-6, restart=30, maxit=1000, x0=None, prec: str = "fp64"):
        """Flexible GMRES(restart), stopping at ||r|| <= tol ||r_0||.  prec is
        'fp64', 'fp32' (B in single precision) or 'none' (B = I).  Returns
        (x, iterations, true relative residual, status, history), history[0]
        = ||r_0|| and history[j] the rotated residual norm after step j."""
        assert prec == "none" or self._amg, "call setup_amg first"
        mode = {"fp64": 0, "fp32": 1, "none": 2}[prec]
        x = np.zeros(self.n) if x0 is None else np.array(x0, dtype=np.float64)
        it = ctypes.c_int(0)
        rr = ctypes.c_double(0.0)
        hist = np.zeros(maxit + 1)
        st = _load().orc_fgmres(self._h, mode, np.ascontiguousarray(b, dtype=np.float64), x, tol, restart,
                                maxit, ctypes.byref(it), ctypes.byref(rr), hist)
        return x, it.value, rr.value, st, hist[: it.value + 1]

    def kappa_grad(self, u, lam) -> np.ndarray:
        g = np.zeros(self.tets.shape[0])
        _load().orc_kappa_grad(self._h, np.ascontiguousarray(u, dtype=np.float64),
                               np.ascontiguousarray(lam, dtype=np.float64), g)
        return g
