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
