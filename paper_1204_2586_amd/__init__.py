"""MI355X auxiliary-space ("GAMG") preconditioned CG for P2/P3 Poisson problems.

Python binding of ``libauxprec.so`` (C ABI in ``include/aux.h``).  This module
only marshals arguments: every step of the solve runs in the library's HIP
kernels on the GPU, and the host setup (discretisation, transfer, AMG) in the
library's C++ code.  PyTorch provides device memory (its caching allocator)
and streams.  There is no CPU fallback: without the built library or a GPU,
the device entry points raise.

Method: Lee, Leng and Zhang, arXiv:1204.2586 -- CG preconditioned by
Algorithm 2.1 with presmoothing (Remark 2.1): l1-Jacobi sweeps on the P^k
system, restriction I_R = I_P^T to the P^1 space, one AMG V-cycle (PMIS,
extended+i), prolongation I_P, l1-Jacobi sweeps.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

__all__ = ["Solver", "SolveInfo", "AuxSolveFn", "KappaSolve", "library_path", "load_library",
           "FP64", "MIXED"]

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libauxprec.so")
FP64, MIXED = 0, 1
# status codes of include/aux.h
OK, EINVAL, ENOMEM, EHIP, ENOTCONV, EBREAKDOWN, ENAN, ESTATE = 0, -1, -2, -3, -4, -5, -6, -7
_OPS = {"assembled": 0, "matfree": 1}

_ERRORS = {-1: "AUX_EINVAL", -2: "AUX_ENOMEM", -3: "AUX_EHIP", -4: "AUX_ENOTCONV", -5: "AUX_EBREAKDOWN",
           -6: "AUX_ENAN", -7: "AUX_ESTATE"}


class AuxError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{_ERRORS.get(code, code)}: {msg}")
        self.code = code


class _Mesh(ctypes.Structure):
    _fields_ = [("n_vertices", ctypes.c_int32), ("xyz", ctypes.c_void_p), ("n_tets", ctypes.c_int32),
                ("tets", ctypes.c_void_p)]


class _Options(ctypes.Structure):
    _fields_ = [("nu", ctypes.c_int), ("theta", ctypes.c_double), ("coarse_max", ctypes.c_int),
                ("max_levels", ctypes.c_int), ("pmis_seed", ctypes.c_uint64), ("precision", ctypes.c_int),
                ("maxit", ctypes.c_int), ("host_only", ctypes.c_int), ("op", ctypes.c_int),
                ("sell_window", ctypes.c_int), ("graph", ctypes.c_int),
                ("sell_index16", ctypes.c_int), ("fuse_cycle", ctypes.c_int),
                ("batch_tiles", ctypes.c_int), ("cycle_lanes", ctypes.c_int), ("dense_cycle_rows", ctypes.c_int),
                ("batch_order", ctypes.c_int), ("amg_setup", ctypes.c_int), ("aux_space", ctypes.c_int),
                ("smoother_weight", ctypes.c_double), ("true_residual", ctypes.c_int),
                ("gram_schmidt", ctypes.c_int)]


_ALLOC = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
_FREE = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p)


class _Device(ctypes.Structure):
    _fields_ = [("stream", ctypes.c_void_p), ("alloc", _ALLOC), ("free", _FREE), ("ctx", ctypes.c_void_p)]


class _Info(ctypes.Structure):
    _fields_ = [("n_h", ctypes.c_int64), ("n_H", ctypes.c_int64), ("n_tets", ctypes.c_int64),
                ("nnz_A", ctypes.c_int64), ("nnz_AH", ctypes.c_int64), ("nnz_IP", ctypes.c_int64),
                ("order", ctypes.c_int32), ("levels", ctypes.c_int32), ("ncoarse", ctypes.c_int32),
                ("precision", ctypes.c_int32), ("op_complexity", ctypes.c_double),
                ("amg_complexity", ctypes.c_double), ("level_rows", ctypes.c_int64 * 32),
                ("level_nnz", ctypes.c_int64 * 32), ("setup_seconds", ctypes.c_double),
                ("device_bytes", ctypes.c_int64), ("stored_A", ctypes.c_int64), ("sell_window", ctypes.c_int64),
                ("level_nnz_P", ctypes.c_int64 * 32), ("sell_slices", ctypes.c_int64),
                ("sell_narrow_slices", ctypes.c_int64), ("sell_index_bytes", ctypes.c_int64),
                ("nnz_restrict", ctypes.c_int64), ("level_nnz_down", ctypes.c_int64 * 32),
                ("level_nnz_up", ctypes.c_int64 * 32), ("batch_tile_rows", ctypes.c_int32 * 2),
                ("sell_tune_ms", ctypes.c_double * 4), ("dense_cycle_level", ctypes.c_int32),
                ("sell_split", ctypes.c_int32),
                ("lanes_restrict", ctypes.c_int32),
                ("lanes_prolong", ctypes.c_int32), ("lanes_down", ctypes.c_int32 * 32),
                ("lanes_up", ctypes.c_int32 * 32), ("amg_setup_seconds", ctypes.c_double),
                ("aux_space", ctypes.c_int32)]


class _SolveInfo(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int32), ("status", ctypes.c_int32), ("rel_residual", ctypes.c_double),
                ("seconds", ctypes.c_double), ("true_rel_residual", ctypes.c_double)]


@dataclass
class SolveInfo:
    iterations: int
    status: int
    rel_residual: float
    seconds: float
    true_rel_residual: float = -1.0      # with the option true_residual (single-vector CG)

    @property
    def converged(self) -> bool:
        return self.status == 0


_lib = None


def library_path() -> str:
    return _LIB_PATH


def load_library():
    """Load libauxprec.so; raises if it has not been built (no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        raise ImportError(f"{_LIB_PATH} is missing: build it with `python -c 'import __graft_entry__ as g; "
                          "g.build()'` (or python paper_1204_2586_amd/build.py)")
    lib = ctypes.CDLL(_LIB_PATH)
    vp, i32, i64, dbl = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    P = ctypes.POINTER
    sig = {
        "aux_default_options": (None, [P(_Options)]),
        "aux_setup": (ctypes.c_int, [P(_Mesh), ctypes.c_int, vp, P(_Options), P(_Device), P(vp)]),
        "aux_destroy": (ctypes.c_int, [vp]),
        "aux_set_stream": (ctypes.c_int, [vp, vp]),
        "aux_set_precision": (ctypes.c_int, [vp, ctypes.c_int]),
        "aux_set_operator": (ctypes.c_int, [vp, ctypes.c_int]),
        "aux_get_info": (ctypes.c_int, [vp, P(_Info)]),
        "aux_dof_xyz": (ctypes.c_int, [vp, vp]),
        "aux_dof_keys": (ctypes.c_int, [vp, vp]),
        "aux_qpoints_per_tet": (ctypes.c_int, [vp]),
        "aux_qpoints": (ctypes.c_int, [vp, i32, i32, vp]),
        "aux_load_accumulate": (ctypes.c_int, [vp, i32, i32, vp, vp]),
        "aux_export_csr": (ctypes.c_int, [vp, ctypes.c_int, ctypes.c_int, P(i64), vp, vp, vp]),
        "aux_export_cf": (ctypes.c_int, [vp, ctypes.c_int, vp]),
        "aux_apply": (ctypes.c_int, [vp, vp, vp]),
        "pcg_solve": (ctypes.c_int, [vp, vp, vp, dbl, ctypes.c_int, P(_SolveInfo)]),
        "pcg_solve_noalloc": (ctypes.c_int, [vp, vp, vp, dbl, ctypes.c_int, P(_SolveInfo)]),
        "aux_set_kappa": (ctypes.c_int, [vp, vp]),
        "pcg_solve_block": (ctypes.c_int, [vp, vp, vp, ctypes.c_int, dbl, ctypes.c_int, P(_SolveInfo)]),
        "pcg_solve_batched": (ctypes.c_int, [vp, vp, vp, ctypes.c_int, dbl, ctypes.c_int, P(_SolveInfo)]),
        "fgmres_solve": (ctypes.c_int, [vp, vp, vp, dbl, ctypes.c_int, ctypes.c_int, vp, P(_SolveInfo)]),
        "aux_stokes_setup": (ctypes.c_int, [vp, P(i32)]),
        "aux_stokes_pressure_keys": (ctypes.c_int, [vp, vp]),
        "stokes_apply_operator": (ctypes.c_int, [vp, vp, vp]),
        "stokes_apply_qt": (ctypes.c_int, [vp, vp, vp, P(i32)]),
        "stokes_fgmres_solve": (ctypes.c_int, [vp, vp, vp, dbl, ctypes.c_int, ctypes.c_int, vp, P(_SolveInfo)]),
        "aux_matvec": (ctypes.c_int, [vp, vp, vp]),
        "aux_kappa_grad": (ctypes.c_int, [vp, vp, vp, vp]),
        "aux_profile": (ctypes.c_int, [vp, ctypes.c_int]),
        "aux_profile_read": (ctypes.c_int, [vp, ctypes.c_int, P(i64), P(dbl)]),
        "aux_last_error": (ctypes.c_char_p, []),
        "aux_residual_history": (ctypes.c_int, [vp, vp, ctypes.c_int32, P(i32)]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _check(rc, allow=(), msg=None):
    """Raise for a failed call; msg is the error text taken right after it
    (any later library call clears the text)."""
    if rc != 0 and rc not in allow:
        raise AuxError(rc, msg if msg is not None else load_library().aux_last_error().decode())
    return rc


def _np_ptr(a):
    return ctypes.c_void_p(a.ctypes.data)


class Solver:
    """One P^k problem (order 2, 3 or 4): mesh + order + per-tet kappa, set up once.

    The keyword options map one to one onto ``aux_options`` in ``include/aux.h``
    (smoothing sweeps ``nu``, strength threshold ``theta``, coarsest size,
    precision, operator, layout window, graph replay, 16-bit columns, composite
    cycle, batched layout, V-cycle operator storage ``cycle_lanes``, dense
    sub-cycle threshold ``dense_cycle_rows``, batched dof order ``batch_order``, where the AMG
    hierarchy is built ``amg_setup`` = "device" or "host", auxiliary space ``aux_space`` = 1 (P^1)
    or 2 (the intermediate P^2 space of Remark 6.2, orders 3 and 4)); the defaults are the timed
    configuration.  ``host_only=True`` runs only the host setup (no GPU
    needed); the matrices and AMG hierarchy can then be inspected with
    ``export_csr``/``export_cf``.
    """

    def __init__(self, xyz, tets, order: int, kappa=None, *, nu: int = 2, theta: float = 0.8,
                 coarse_max: int = 100, max_levels: int = 25, seed: int = 0, precision: str = "fp64",
                 maxit: int = 1000, host_only: bool = False, device=None, use_torch_allocator: bool = True,
                 operator: str = "assembled", sell_window: int = 0, graph: bool = True, sell_index16: bool = True,
                 fuse_cycle: bool = True, batch_tiles: int = 1, cycle_lanes: int = 0,
                 dense_cycle_rows: int = 2048, batch_order: int = 0, amg_setup: str = "device",
                 aux_space: int = 1, smoother_weight: float = 1.0, true_residual: bool = False,
                 gram_schmidt: int = 1):
        lib = load_library()
        self._h = ctypes.c_void_p()
        self.order = order
        self.host_only = host_only
        xyz = np.ascontiguousarray(xyz, dtype=np.float64)
        tets = np.ascontiguousarray(tets, dtype=np.int32)
        mesh = _Mesh(xyz.shape[0], xyz.ctypes.data, tets.shape[0], tets.ctypes.data)
        opt = _Options()
        lib.aux_default_options(ctypes.byref(opt))
        opt.nu, opt.theta, opt.coarse_max, opt.max_levels = nu, theta, coarse_max, max_levels
        opt.pmis_seed, opt.maxit, opt.host_only = seed, maxit, int(host_only)
        self._maxit = int(maxit)
        opt.precision = {"fp64": FP64, "mixed": MIXED}[precision]
        opt.op = _OPS[operator]
        opt.sell_window = sell_window
        opt.graph = int(graph)
        opt.sell_index16 = int(sell_index16)
        opt.fuse_cycle = int(fuse_cycle)
        opt.batch_tiles = int(batch_tiles)
        opt.cycle_lanes = int(cycle_lanes)
        opt.dense_cycle_rows = int(dense_cycle_rows)
        opt.batch_order = int(batch_order)
        opt.amg_setup = {"host": 0, "device": 1}[amg_setup]
        opt.aux_space = int(aux_space)
        opt.smoother_weight = float(smoother_weight)
        opt.true_residual = int(true_residual)
        opt.gram_schmidt = int(gram_schmidt)
        kap = None
        if kappa is not None:
            self._kappa = np.ascontiguousarray(kappa, dtype=np.float64)
            kap = _np_ptr(self._kappa)
        dev = None
        self._torch = None
        if not host_only:
            import torch
            if not torch.cuda.is_available():
                raise RuntimeError("no GPU visible: the solver runs on the device only (use host_only=True "
                                   "for the host setup)")
            self._torch = torch
            self.device = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
            torch.cuda.set_device(self.device)
            stream = torch.cuda.current_stream(self.device)
            dev = _Device()
            dev.stream = stream.cuda_stream
            if use_torch_allocator:
                dindex = self.device.index

                def _alloc(n, ctx, _t=torch, _d=dindex, _s=stream):
                    return _t.cuda.caching_allocator_alloc(int(n), _d, _s)

                def _free(p, ctx, _t=torch):
                    _t.cuda.caching_allocator_delete(p)

                self._cb = (_ALLOC(_alloc), _FREE(_free))
                dev.alloc, dev.free = self._cb
            dev = ctypes.byref(dev)
        _check(lib.aux_setup(ctypes.byref(mesh), order, kap, ctypes.byref(opt), dev, ctypes.byref(self._h)))
        self.info = self._info()
        self.n = int(self.info.n_h)
        self.nH = int(self.info.n_H)
        self.n_tets = int(self.info.n_tets)
        self.n_p = None      # pressure count, set by stokes_setup

    # ------------------------------------------------------------ lifecycle
    def close(self):
        if getattr(self, "_h", None) and self._h.value and _lib is not None:
            if self._torch is not None:
                self._torch.cuda.synchronize(self.device)
            _lib.aux_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _info(self):
        info = _Info()
        _check(load_library().aux_get_info(self._h, ctypes.byref(info)))
        return info

    def _sync_stream(self):
        s = self._torch.cuda.current_stream(self.device).cuda_stream
        _check(load_library().aux_set_stream(self._h, ctypes.c_void_p(s)))

    def set_kappa(self, kappa):
        """A new per-tet coefficient on the same mesh: the device re-assembles
        A_h, A_H and the l1 norms (bitwise as a new setup would) and builds
        the AMG hierarchy (on the host with amg_setup="host").  If the update
        fails, the handle refuses solves until a later update succeeds."""
        kap = np.ascontiguousarray(kappa, dtype=np.float64)
        if kap.shape != (self.n_tets,):
            raise ValueError(f"kappa must have shape ({self.n_tets},)")
        self._kappa = None
        _check(load_library().aux_set_kappa(self._h, _np_ptr(kap)))
        self._kappa = kap
        self.info = self._info()

    def set_precision(self, precision: str):
        _check(load_library().aux_set_precision(self._h, {"fp64": FP64, "mixed": MIXED}[precision]))
        self.info = self._info()

    def set_operator(self, operator: str):
        """'assembled' (sliced-ELL A_h) or 'matfree' (element operator on the matrix cores)
        for the preconditioner's P^k products."""
        _check(load_library().aux_set_operator(self._h, _OPS[operator]))

    @property
    def levels(self):
        i = self.info
        return [(int(i.level_rows[l]), int(i.level_nnz[l])) for l in range(i.levels)]

    # ------------------------------------------------------------ host data
    def dof_keys(self) -> np.ndarray:
        k = np.zeros((self.n, self.order), dtype=np.int32)
        _check(load_library().aux_dof_keys(self._h, _np_ptr(k)))
        return k

    def dof_xyz(self) -> np.ndarray:
        """Node position of each dof (host [n_h, 3])."""
        out = np.zeros((self.n, 3))
        _check(load_library().aux_dof_xyz(self._h, _np_ptr(out)))
        return out

    def qpoints(self, t0: int, t1: int) -> np.ndarray:
        m = load_library().aux_qpoints_per_tet(self._h)
        out = np.zeros(((t1 - t0) * m, 3))
        _check(load_library().aux_qpoints(self._h, t0, t1, _np_ptr(out)))
        return out

    def load(self, f, chunk: int = 32768) -> np.ndarray:
        """Load vector <f, phi_i> for a point-wise function f(points[..., 3]) (host array)."""
        b = np.zeros(self.n)
        for t0 in range(0, self.n_tets, chunk):
            t1 = min(self.n_tets, t0 + chunk)
            fq = np.ascontiguousarray(f(self.qpoints(t0, t1)), dtype=np.float64)
            _check(load_library().aux_load_accumulate(self._h, t0, t1, _np_ptr(fq), _np_ptr(b)))
        return b

    def load_many(self, f, ncols: int, chunk: int = 65536, threads: int = 8) -> np.ndarray:
        """Load vectors of ncols sources at once: f(points[npts, 3]) returns
        [ncols, npts].  Returns a host [n_h, ncols] array.  Each chunk of
        tets is split into `threads` tet ranges whose sources are evaluated
        in parallel; the accumulation then runs in parallel over columns
        (numpy and the library release the GIL)."""
        from concurrent.futures import ThreadPoolExecutor
        lib = load_library()
        threads = max(1, threads)
        B = np.zeros((ncols, self.n))

        def evaluate(rng):
            ta, tb = rng
            F = np.ascontiguousarray(f(self.qpoints(ta, tb)), dtype=np.float64)
            if F.shape[0] != ncols:
                raise ValueError(f"f returned {F.shape[0]} sources, expected {ncols}")
            return ta, tb, F

        with ThreadPoolExecutor(threads) as ex:
            for t0 in range(0, self.n_tets, chunk):
                t1 = min(self.n_tets, t0 + chunk)
                cuts = np.linspace(t0, t1, threads + 1).astype(int)
                parts = list(ex.map(evaluate, [(int(a), int(b)) for a, b in zip(cuts[:-1], cuts[1:]) if b > a]))

                def accumulate(c):
                    for ta, tb, F in parts:
                        _check(lib.aux_load_accumulate(self._h, ta, tb, _np_ptr(F[c]), _np_ptr(B[c])))

                list(ex.map(accumulate, range(ncols)))
        return np.ascontiguousarray(B.T)

    def export_csr(self, which: str, level: int = 0):
        import scipy.sparse as sp
        code = {"A": 0, "AH": 1, "IP": 2, "Alev": 3, "P": 4, "B": 5, "Mp": 6, "down": 7, "up": 8,
                "I2": 9}[which]
        shape = (ctypes.c_int64 * 3)()
        lib = load_library()
        _check(lib.aux_export_csr(self._h, code, level, shape, None, None, None))
        n, m, nnz = (int(v) for v in shape)
        ptr = np.zeros(n + 1, dtype=np.int32)
        col = np.zeros(max(nnz, 1), dtype=np.int32)
        val = np.zeros(max(nnz, 1))
        _check(lib.aux_export_csr(self._h, code, level, shape, _np_ptr(ptr), _np_ptr(col), _np_ptr(val)))
        return sp.csr_matrix((val[:nnz], col[:nnz], ptr), shape=(n, m))

    def export_cf(self, level: int) -> np.ndarray:
        n = int(self.info.level_rows[level])
        cf = np.zeros(n, dtype=np.int32)
        _check(load_library().aux_export_cf(self._h, level, _np_ptr(cf)))
        return cf

    # ------------------------------------------------------------ device ops
    def _vec(self, x, name, n=None, ncols=None):
        t = self._torch
        if not isinstance(x, t.Tensor):
            x = t.as_tensor(np.asarray(x, dtype=np.float64), device=self.device)
        if x.device != self.device or x.dtype != t.float64:
            raise ValueError(f"{name} must be a float64 tensor on {self.device}")
        n = self.n if n is None else n
        shape = (n,) if ncols is None else (n, ncols)
        if tuple(x.shape) != shape:
            raise ValueError(f"{name} must have shape {shape}, got {tuple(x.shape)}")
        return x.contiguous()

    def apply(self, r, out=None):
        """z = B r (device float64 vectors)."""
        r = self._vec(r, "r")
        z = self._torch.empty_like(r) if out is None else self._vec(out, "out")
        self._sync_stream()
        _check(load_library().aux_apply(self._h, ctypes.c_void_p(r.data_ptr()), ctypes.c_void_p(z.data_ptr())))
        return z

    def matvec(self, x, out=None):
        x = self._vec(x, "x")
        y = self._torch.empty_like(x) if out is None else self._vec(out, "out")
        self._sync_stream()
        _check(load_library().aux_matvec(self._h, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(y.data_ptr())))
        return y

    def solve(self, f, tol: float = 1e-8, u0=None, maxit: int = 0, out=None, check: bool = True):
        """CG on A_h u = f.  Returns (u, SolveInfo).  With check=True a status
        other than AUX_OK raises; otherwise it is reported in SolveInfo.status."""
        f = self._vec(f, "f")
        if out is not None:
            u = self._vec(out, "out")
            if u0 is None:
                u.zero_()
        else:
            u = self._torch.zeros_like(f)
        if u0 is not None:
            u.copy_(self._vec(u0, "u0"))
        info = _SolveInfo()
        self._sync_stream()
        rc = load_library().pcg_solve(self._h, ctypes.c_void_p(f.data_ptr()), ctypes.c_void_p(u.data_ptr()), tol,
                                      int(maxit), ctypes.byref(info))
        if check:
            _check(rc)
        elif rc not in (0, -4, -5, -6):
            _check(rc)
        return u, SolveInfo(info.iterations, info.status, info.rel_residual, info.seconds, info.true_rel_residual)

    def residual_history(self) -> np.ndarray:
        """||r_k|| / ||f|| for k = 0 .. iterations of the last single-vector CG solve."""
        lib = load_library()
        n = ctypes.c_int32(0)
        _check(lib.aux_residual_history(self._h, None, 0, ctypes.byref(n)))
        out = np.zeros(max(n.value, 1))
        _check(lib.aux_residual_history(self._h, _np_ptr(out), n.value, ctypes.byref(n)))
        return out[:n.value]

    def solve_noalloc(self, f, u, tol: float = 1e-8, maxit: int = 0, check: bool = True):
        """CG on A_h u = f through pcg_solve_noalloc (no allocation in the
        library: its scratch memory is a fixed array per GPU).  u is the
        caller's device vector, initial guess in and solution out; this
        method allocates nothing either.  Returns SolveInfo."""
        f = self._vec(f, "f")
        if not (isinstance(u, self._torch.Tensor) and u.is_contiguous()):
            raise ValueError("u must be a contiguous float64 device tensor (it receives the solution)")
        u = self._vec(u, "u")
        info = _SolveInfo()
        self._sync_stream()
        rc = load_library().pcg_solve_noalloc(self._h, ctypes.c_void_p(f.data_ptr()), ctypes.c_void_p(u.data_ptr()),
                                              tol, int(maxit), ctypes.byref(info))
        if check:
            _check(rc)
        elif rc not in (0, -4, -5, -6):
            _check(rc)
        return SolveInfo(info.iterations, info.status, info.rel_residual, info.seconds, info.true_rel_residual)

    def fgmres(self, b, tol: float = 1e-6, x0=None, restart: int = 30, maxit: int = 0, check: bool = True):
        """Flexible GMRES(restart) on A_h x = b with the same preconditioner,
        stopping at ||r|| <= tol ||r_0||.  Returns (x, SolveInfo, history),
        history a numpy array of ||r_0|| and the residual norm after each
        Arnoldi step."""
        import numpy as np
        b = self._vec(b, "b")
        if x0 is None:
            x = self._torch.zeros_like(b)
        else:
            x = self._torch.empty_like(b)
            x.copy_(self._vec(x0, "x0"))
        cap = (int(maxit) if maxit > 0 else self._maxit) + 1
        hist = np.zeros(cap)
        info = _SolveInfo()
        self._sync_stream()
        rc = load_library().fgmres_solve(self._h, ctypes.c_void_p(b.data_ptr()), ctypes.c_void_p(x.data_ptr()), tol,
                                         int(restart), int(maxit), hist.ctypes.data_as(ctypes.c_void_p),
                                         ctypes.byref(info))
        if check:
            _check(rc)
        elif rc not in (0, -4, -6):
            _check(rc)
        return x, SolveInfo(info.iterations, info.status, info.rel_residual, info.seconds, info.true_rel_residual), \
            hist[: info.iterations + 1]

    # ------------------------------------------------------------ Stokes
    def stokes_setup(self) -> int:
        """Build the Hood-Taylor P^k-P^{k-1} Stokes blocks B and M_p (k = the
        order); returns the pressure count n_p (the vertex count for P^1).
        Stokes vectors have 3 n_h + n_p entries: u_0, u_1, u_2 in dof order,
        then p in the order of stokes_pressure_keys()."""
        n_p = ctypes.c_int32(0)
        _check(load_library().aux_stokes_setup(self._h, ctypes.byref(n_p)))
        self.n_p = int(n_p.value)
        return self.n_p

    def stokes_pressure_keys(self) -> np.ndarray:
        """Node key of each pressure unknown: [n_p][order-1] sorted vertex ids."""
        if self.n_p is None:
            self.stokes_setup()
        keys = np.zeros((self.n_p, self.order - 1), dtype=np.int32)
        _check(load_library().aux_stokes_pressure_keys(self._h, _np_ptr(keys)))
        return keys

    def _stokes_len(self):
        if self.n_p is None:
            self.stokes_setup()
        return 3 * self.n + self.n_p

    def stokes_operator(self, x, out=None):
        """y = [A B^T; B 0] x."""
        m = self._stokes_len()
        x = self._vec(x, "x", n=m)
        y = self._torch.empty_like(x) if out is None else self._vec(out, "out", n=m)
        self._sync_stream()
        _check(load_library().stokes_apply_operator(self._h, ctypes.c_void_p(x.data_ptr()),
                                                    ctypes.c_void_p(y.data_ptr())))
        return y

    def stokes_qt(self, r, out=None):
        """z = Q_t r (block triangular preconditioner).  Returns (z, the
        pressure mass-matrix CG step count)."""
        m = self._stokes_len()
        r = self._vec(r, "r", n=m)
        z = self._torch.empty_like(r) if out is None else self._vec(out, "out", n=m)
        steps = ctypes.c_int32(0)
        self._sync_stream()
        _check(load_library().stokes_apply_qt(self._h, ctypes.c_void_p(r.data_ptr()), ctypes.c_void_p(z.data_ptr()),
                                              ctypes.byref(steps)))
        return z, int(steps.value)

    def stokes_fgmres(self, b, tol: float = 1e-8, x0=None, restart: int = 30, maxit: int = 0, check: bool = True):
        """FGMRES(restart) with Q_t on the Stokes system.  Returns (x,
        SolveInfo, history) as fgmres."""
        import numpy as np
        m = self._stokes_len()
        b = self._vec(b, "b", n=m)
        if x0 is None:
            x = self._torch.zeros_like(b)
        else:
            x = self._torch.empty_like(b)
            x.copy_(self._vec(x0, "x0", n=m))
        cap = (int(maxit) if maxit > 0 else self._maxit) + 1
        hist = np.zeros(cap)
        info = _SolveInfo()
        self._sync_stream()
        rc = load_library().stokes_fgmres_solve(self._h, ctypes.c_void_p(b.data_ptr()), ctypes.c_void_p(x.data_ptr()),
                                                tol, int(restart), int(maxit), hist.ctypes.data_as(ctypes.c_void_p),
                                                ctypes.byref(info))
        if check:
            _check(rc)
        elif rc not in (0, -4, -6):
            _check(rc)
        return x, SolveInfo(info.iterations, info.status, info.rel_residual, info.seconds, info.true_rel_residual), \
            hist[: info.iterations + 1]

    def solve_batched(self, F, tol: float = 1e-8, U0=None, maxit: int = 0, check: bool = True):
        """nrhs lock-step CG solves; F is a [n_h, nrhs] float64 device tensor."""
        t = self._torch
        if F.dim() != 2:
            raise ValueError("F must be [n_h, nrhs]")
        nrhs = F.shape[1]
        F = self._vec(F, "F", ncols=nrhs)
        U = t.zeros_like(F) if U0 is None else self._vec(U0, "U0", ncols=nrhs).clone()
        infos = (_SolveInfo * nrhs)()
        self._sync_stream()
        rc = load_library().pcg_solve_batched(self._h, ctypes.c_void_p(F.data_ptr()), ctypes.c_void_p(U.data_ptr()),
                                              nrhs, tol, int(maxit), infos)
        msg = load_library().aux_last_error().decode()
        self.info = self._info()                  # the layout chosen for this block width
        if check:
            _check(rc, msg=msg)
        return U, [SolveInfo(i.iterations, i.status, i.rel_residual, i.seconds) for i in infos]

    def solve_block(self, F, tol: float = 1e-8, U0=None, maxit: int = 0, check: bool = True):
        """O'Leary's block preconditioned CG on the nrhs columns of F
        ([n_h, nrhs] float64 device tensor, nrhs <= 64).  Returns (U, [SolveInfo])."""
        t = self._torch
        if F.dim() != 2:
            raise ValueError("F must be [n_h, nrhs]")
        nrhs = F.shape[1]
        F = self._vec(F, "F", ncols=nrhs)
        U = t.zeros_like(F) if U0 is None else self._vec(U0, "U0", ncols=nrhs).clone()
        infos = (_SolveInfo * nrhs)()
        self._sync_stream()
        rc = load_library().pcg_solve_block(self._h, ctypes.c_void_p(F.data_ptr()), ctypes.c_void_p(U.data_ptr()),
                                            nrhs, tol, int(maxit), infos)
        msg = load_library().aux_last_error().decode()
        self.info = self._info()
        if check:
            _check(rc, msg=msg)
        elif rc not in (0, -4, -5, -6):
            _check(rc, msg=msg)
        return U, [SolveInfo(i.iterations, i.status, i.rel_residual, i.seconds) for i in infos]

    PROF = {"pk_first": 0, "pk_sweep": 1, "pk_last": 2, "pk_resid": 3, "coarse": 4, "cg_spmv": 5, "apply": 6}

    def profile(self, enable=True):
        """Start (and reset) or stop HIP-event timing of the solve-phase kernels
        (enable=True: every launch; "apply": whole preconditioner applications
        only; False: stop)."""
        mode = 2 if enable == "apply" else int(bool(enable))
        _check(load_library().aux_profile(self._h, mode))

    def profile_read(self):
        """{category: (launches, total ms)} since the last profile() call."""
        out = {}
        for name, c in self.PROF.items():
            n = ctypes.c_int64(0)
            ms = ctypes.c_double(0.0)
            _check(load_library().aux_profile_read(self._h, c, ctypes.byref(n), ctypes.byref(ms)))
            out[name] = (int(n.value), float(ms.value))
        return out

    def kappa_grad(self, u, lam, out=None):
        """g_t = -lam_t^T K_t u_t: dL/dlog(kappa_t) given the adjoint solution lam."""
        u = self._vec(u, "u")
        lam = self._vec(lam, "lam")
        g = self._torch.empty(self.n_tets, dtype=self._torch.float64, device=self.device) if out is None else out
        self._sync_stream()
        _check(load_library().aux_kappa_grad(self._h, ctypes.c_void_p(u.data_ptr()), ctypes.c_void_p(lam.data_ptr()),
                                             ctypes.c_void_p(g.data_ptr())))
        return g


class KappaSolve:
    """Mesh, order and options for the differentiable solve u = A(kappa)^{-1} f.

    One solver per mesh: the first kappa runs the full setup, a new kappa
    re-assembles on the device and rebuilds the AMG hierarchy
    (Solver.set_kappa).  The solver's current kappa is tracked so a backward
    pass whose forward used another kappa re-assembles that one first.
    """

    def __init__(self, xyz, tets, order: int, tol: float = 1e-12, **options):
        self.xyz, self.tets, self.order, self.tol, self.options = xyz, tets, order, tol, options
        self._key = None
        self._solver = None

    @staticmethod
    def key_of(kappa: np.ndarray):
        return hash(kappa.tobytes())

    def solver_for(self, kappa: np.ndarray) -> Solver:
        key = self.key_of(kappa)
        if self._solver is None:
            self._solver = Solver(self.xyz, self.tets, self.order, kappa, **self.options)
        elif self._key != key:
            self._solver.set_kappa(kappa)
        self._key = key
        return self._solver


def _make_autograd():
    import torch

    class _AuxSolveFn(torch.autograd.Function):
        """u = A(exp(log_kappa))^{-1} f with an adjoint CG solve in backward.

        forward(f, log_kappa, problem): f the load vector [n_h] (device,
        float64), log_kappa [n_tets], problem a KappaSolve.
        backward: lam = A^{-1} grad_u (same SPD operator and preconditioner),
        dL/df = lam, dL/dlog(kappa_t) = -lam_t^T K_t u_t.
        """

        @staticmethod
        def forward(ctx, f, log_kappa, problem):
            kappa = torch.exp(log_kappa.detach().double()).cpu().numpy()
            s = problem.solver_for(kappa)
            u, info = s.solve(f.detach().double().contiguous(), tol=problem.tol)
            ctx.solver, ctx.tol, ctx.problem, ctx.kappa = s, problem.tol, problem, kappa
            ctx.kdtype, ctx.kdevice = log_kappa.dtype, log_kappa.device
            ctx.save_for_backward(u)
            return u

        @staticmethod
        def backward(ctx, grad_u):
            (u,) = ctx.saved_tensors
            # the operator of this forward pass (another may have run since)
            s = ctx.problem.solver_for(ctx.kappa)
            lam, _ = s.solve(grad_u.double().contiguous(), tol=ctx.tol)
            g = s.kappa_grad(u, lam)
            return lam, g.to(dtype=ctx.kdtype, device=ctx.kdevice), None

    return _AuxSolveFn


class _LazyFn:
    _fn = None

    def __getattr__(self, name):
        if _LazyFn._fn is None:
            _LazyFn._fn = _make_autograd()
        return getattr(_LazyFn._fn, name)


AuxSolveFn = _LazyFn()
