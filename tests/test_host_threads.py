"""The host setup runs its sorts, sparsity pattern, assembly and norms on
several threads with every sum kept in its sequential order, so its outputs
must not depend on the thread count: one thread and eight give the same bits
for the operators, transfer, dof numbering and AMG hierarchy."""
import hashlib
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

SCRIPT = r"""
import hashlib, sys
import numpy as np
sys.path.insert(0, {root!r})
import paper_1204_2586_amd as aux, workloads as W
k, n = {k}, {n}
xyz, tets = W.kuhn_mesh(n, jitter=0.2, seed=0)
kappa = np.exp(np.random.default_rng(3).normal(size=len(tets)))
s = aux.Solver(xyz, tets, k, kappa, host_only=True)
h = hashlib.sha1()
h.update(np.ascontiguousarray(s.dof_keys()).tobytes())
mats = [s.export_csr("A"), s.export_csr("AH"), s.export_csr("IP")]
for l in range(s.info.levels):
    mats.append(s.export_csr("Alev", l))
    if l + 1 < s.info.levels:
        mats.append(s.export_csr("P", l))
for m in mats:
    for a in (m.indptr, m.indices, m.data):
        h.update(np.ascontiguousarray(a).tobytes())
print(h.hexdigest())
"""


def _digest(k, n, threads):
    env = dict(os.environ, AUXPREC_SETUP_THREADS=str(threads))
    r = subprocess.run([sys.executable, "-c", SCRIPT.format(root=ROOT, k=k, n=n)], env=env, capture_output=True,
                       text=True, timeout=600, check=True)
    return r.stdout.strip().splitlines()[-1]


@pytest.mark.parametrize("k,n", [(2, 24), (3, 12), (4, 8)])
def test_setup_independent_of_thread_count(k, n):
    assert _digest(k, n, 1) == _digest(k, n, 8)


LIMIT_SCRIPT = r"""
import resource, sys
sys.path.insert(0, {root!r})
import paper_1204_2586_amd as aux, workloads as W
aux.load_library()
xyz, tets = W.kuhn_mesh(24, jitter=0.2, seed=0)
def vm():
    for l in open('/proc/self/status'):
        if l.startswith('VmSize'):
            return int(l.split()[1]) * 1024
lim = vm() + {mb} * 2 ** 20
resource.setrlimit(resource.RLIMIT_AS, (lim, lim))
try:
    s = aux.Solver(xyz, tets, 2, host_only=True)
    print("ok", s.info.levels)
except aux.AuxError as e:
    print("err", e.code)
except MemoryError:
    print("pyerr")       # the interpreter's own allocation hit the limit first
"""


# glibc allocates a new thread's thread-local storage for dynamically loaded
# modules on first use and aborts the process with this message when it
# cannot; no code in the process can intercept that
_TLS_ABORT = "cannot allocate memory for thread-local data"


def test_setup_out_of_memory_returns_status():
    """Under an address-space limit the threaded host setup must fail with
    AUX_ENOMEM (worker exceptions joined and rethrown, threads that cannot be
    started replaced by the calling thread), never terminate the process by
    itself: every run ends with a result, a status, the interpreter's own
    MemoryError, or the C library's thread-local-storage abort (outside the
    library's control), and some run returns AUX_ENOMEM."""
    outcomes = []
    for mb in (50, 100, 200, 300, 100, 200):
        env = dict(os.environ, AUXPREC_SETUP_THREADS="8")
        r = subprocess.run([sys.executable, "-c", LIMIT_SCRIPT.format(root=ROOT, mb=mb)], env=env,
                           capture_output=True, text=True, timeout=600)
        if r.returncode != 0 and _TLS_ABORT in r.stderr:
            outcomes.append("tls")
            continue
        assert r.returncode == 0, (mb, r.returncode, r.stderr[-500:])
        out = r.stdout.strip().splitlines()[-1].split()
        assert out[0] in ("ok", "pyerr") or (out[0] == "err" and int(out[1]) == -2), (mb, out)
        outcomes.append(out[0])
    assert "err" in outcomes, outcomes
