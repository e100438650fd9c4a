"""The oracle's pins have teeth: each plausible mistake, planted in a copy of
the oracle's C sources (on the CPU), makes the named pin tests fail.

Every case copies ``oracle/*.c``/``*.h`` to a temporary directory, replaces
one or more exact snippets (each must occur exactly once, so a plant that no
longer matches the oracle fails loudly here), builds the copy with the
oracle's own build script, and runs the named tests in a child process whose
``oracle`` package loads that copy.  A plant is caught when every named test
fails.  The last case checks a status path the method cannot reach with a
correct preconditioner: with B negated, CG must report breakdown.
"""
import json
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
ORC = os.path.join(ROOT, "oracle")

# name -> (edits [(file, old, new)], tests that must all fail)
PLANTS = {
    # Algorithm 2.1 Step 1 by a V(1,1) cycle: the level post-smoothing dropped
    "vcycle_no_post_sweep": (
        [("orc_solve.c",
          "    sweep(&lv->A, B->lAval[l], B->ldinv[l], b, x, t, R);                    /* postsmooth */\n"
          "    memcpy(x, t, (size_t)n * sizeof(double));\n", "")],
        ["test_oracle_solver.py::test_vcycle_spd_multilevel",
         "test_oracle_solver.py::test_vcycle_error_propagator",
         "test_oracle_solver.py::test_preconditioner_spd_multilevel"]),
    # the next finer level's l1 diagonal used on every coarser level (the
    # cycle stays symmetric and convergent)
    "vcycle_wrong_level_diagonal": (
        [("orc_solve.c", "x[i] = R(B->ldinv[l][i] * b[i]);", "x[i] = R(B->ldinv[l > 0 ? l - 1 : 0][i] * b[i]);"),
         ("orc_solve.c", "sweep(&lv->A, B->lAval[l], B->ldinv[l], b, x, t, R);",
          "sweep(&lv->A, B->lAval[l], B->ldinv[l > 0 ? l - 1 : 0], b, x, t, R);")],
        ["test_oracle_solver.py::test_vcycle_error_propagator"]),
    # the coarse-grid correction applied on the first level only
    "vcycle_correction_level0_only": (
        [("orc_solve.c", "    matvec_add(&lv->P, B->lPval[l], ec, x, R);",
          "    if (l == 0) matvec_add(&lv->P, B->lPval[l], ec, x, R);")],
        ["test_oracle_solver.py::test_vcycle_error_propagator",
         "test_oracle_solver.py::test_gamg_multilevel_flat_in_h"]),
    # extended interpolation without the "+i": i left out of d_k and of the
    # diagonal's share of a_ik
    "interp_without_plus_i": (
        [("orc_amg.c", "if (l == i || inC[l] == i) d += abar;", "if (inC[l] == i) d += abar;"),
         ("orc_amg.c", "if (l == i) diag += aij * abar / d;", "if (0) diag += aij * abar / d;")],
        ["test_oracle_amg.py::test_ext_i_harmonic_1d",
         "test_oracle_amg.py::test_ext_i_exact_rationals"]),
    # PMIS: a new C point compared with the points it depends on only (S),
    # not with those depending on it (S^T)
    "pmis_independent_in_S_only": (
        [("orc_amg.c",
          "            for (int e = ST->ptr[i]; e < ST->ptr[i + 1] && best; e++) {\n"
          "                int j = ST->col[e];\n"
          "                if (cf[j] == 0 && !beats(nst, rho, i, j)) best = 0;\n"
          "            }\n", "")],
        ["test_oracle_amg.py::test_pmis_rounds"]),
    # block CG: the s x s step alpha = delta^{-1} gamma applied transposed
    "block_cg_alpha_transposed": (
        [("orc_solve.c", "                    px += P[(size_t)i * s + a] * coef[a * s + b];\n"
                         "                    qx += Q[(size_t)i * s + a] * coef[a * s + b];",
          "                    px += P[(size_t)i * s + a] * coef[b * s + a];\n"
          "                    qx += Q[(size_t)i * s + a] * coef[b * s + a];")],
        ["test_oracle_block_cg.py::test_block_krylov_projection"]),
    # block CG: beta = gamma_new instead of gamma^{-1} gamma_new
    "block_cg_beta_without_gamma_inverse": (
        [("orc_solve.c", "        small_cholesky_solve(s, Lg, coef);", "")],
        ["test_oracle_block_cg.py::test_block_krylov_projection",
         "test_oracle_block_cg.py::test_one_column_is_cg"]),
    # Stokes: B assembled as +div instead of -div
    "stokes_divergence_sign": (
        [("orc_fem.c", "bv[cb] = -det * Bt[p][c][a];", "bv[cb] = det * Bt[p][c][a];")],
        ["test_oracle_stokes.py::test_gradient_of_linear_pressure_is_a_load_vector"]),
    # FGMRES: sign of the rotated right-hand side
    "fgmres_givens_rhs_sign": (
        [("orc_solve.c", "g[j + 1] = -sn[j] * g[j];", "g[j + 1] = sn[j] * g[j];")],
        ["test_oracle_fgmres.py::test_fgmres_matches_dense_solve",
         "test_oracle_fgmres.py::test_flexible_gmres_minimises_over_preconditioned_space",
         "test_oracle_fgmres.py::test_full_gmres_terminates_within_n_steps"]),
    # FGMRES: sign of an earlier rotation applied to a new Hessenberg column
    "fgmres_rotation_sign": (
        [("orc_solve.c", "H[(size_t)(i + 1) * m + j] = -sn[i] * a + cs[i] * c;",
          "H[(size_t)(i + 1) * m + j] = sn[i] * a + cs[i] * c;")],
        ["test_oracle_fgmres.py::test_gmres_minimises_residual_over_krylov_space",
         "test_oracle_fgmres.py::test_fgmres_matches_dense_solve"]),
    # FGMRES: Gram-Schmidt skipping the first basis vector
    "fgmres_orthogonalise_from_v1": (
        [("orc_solve.c", "            for (int i = 0; i <= j; i++) {\n                const double *vi",
          "            for (int i = 1; i <= j; i++) {\n                const double *vi")],
        ["test_oracle_fgmres.py::test_gmres_minimises_residual_over_krylov_space",
         "test_oracle_fgmres.py::test_flexible_gmres_minimises_over_preconditioned_space",
         "test_oracle_fgmres.py::test_restart_one_is_minimal_residual_iteration"]),
    # intermediate space: the P^2 vertex function taken as lam^2 (not lam (2 lam - 1))
    "nested_vertex_function": (
        [("orc_fem.c", "double w = lam[p] * (2.0 * lam[p] - 1.0);", "double w = lam[p] * lam[p];")],
        ["test_oracle_nested.py::test_transfer_reproduces_quadratics",
         "test_oracle_nested.py::test_galerkin_product_is_the_p2_stiffness"]),
    # intermediate space: the P^2 edge function without its factor 4
    "nested_edge_function_scale": (
        [("orc_fem.c", "double w = 4.0 * lam[p] * lam[q];", "double w = 2.0 * lam[p] * lam[q];")],
        ["test_oracle_nested.py::test_transfer_reproduces_quadratics",
         "test_oracle_nested.py::test_galerkin_product_is_the_p2_stiffness"]),
    # intermediate space: the postsmoothing left out (B no longer symmetric)
    "nested_no_postsmoothing": (
        [("orc_solve.c",
          "    matvec_add(&o->I2, N->I2val, e2, z, R);\n"
          "    /* postsmoothing */\n"
          "    for (int s = 0; s < o->nu; s++) {\n",
          "    matvec_add(&o->I2, N->I2val, e2, z, R);\n"
          "    /* postsmoothing */\n"
          "    for (int s = 0; s < 0; s++) {\n")],
        ["test_oracle_nested.py::test_nested_preconditioner_spd"]),
}

_RUNNER = r"""
import json, sys
sys.path[:0] = [{root!r}, {tests!r}]
import oracle
oracle._LIB_PATH = {lib!r}
import pytest

class Rec:
    def __init__(self):
        self.out = {{}}
    def pytest_runtest_logreport(self, report):
        if report.when == "call" or report.outcome != "passed":
            prev = self.out.get(report.nodeid)
            if prev != "failed":
                self.out[report.nodeid] = report.outcome

rec = Rec()
pytest.main(["-q", "-p", "no:cacheprovider", "-p", "no:randomly", "-m", "not gpu"] + {ids!r}, plugins=[rec])
json.dump(rec.out, open({res!r}, "w"))
"""


def _planted_lib(tmp_path, edits):
    src = tmp_path / "src"
    src.mkdir()
    for f in os.listdir(ORC):
        if f.endswith((".c", ".h")):
            shutil.copy(os.path.join(ORC, f), src / f)
    for fname, old, new in edits:
        p = src / fname
        text = p.read_text()
        assert text.count(old) == 1, f"plant snippet not found exactly once in {fname}: {old!r}"
        p.write_text(text.replace(old, new))
    from oracle import build as ob
    return ob.build(src_dir=str(src), out=str(tmp_path / "liboracle_planted.so"))


def _run(tmp_path, lib, tests):
    res = tmp_path / "res.json"
    ids = [os.path.join(ROOT, "tests", t) for t in tests]
    code = _RUNNER.format(root=ROOT, tests=os.path.join(ROOT, "tests"), lib=lib, ids=ids, res=str(res))
    subprocess.run([sys.executable, "-c", code], cwd=str(tmp_path), capture_output=True, text=True,
                   timeout=600)
    out = json.loads(res.read_text())
    by_test = {}
    for nodeid, outcome in out.items():
        base = nodeid.split("[")[0]
        key = next(t for t in tests if base.endswith(t.split("::")[1]))
        by_test.setdefault(key, []).append(outcome)
    return by_test


@pytest.mark.parametrize("name", sorted(PLANTS))
def test_plant_is_caught(name, tmp_path):
    edits, tests = PLANTS[name]
    lib = _planted_lib(tmp_path, edits)
    by_test = _run(tmp_path, lib, tests)
    assert set(by_test) == set(tests), by_test
    for t, outcomes in by_test.items():
        assert "failed" in outcomes, f"{name}: {t} passed with the plant ({outcomes})"


def test_breakdown_status_with_negated_preconditioner(tmp_path):
    edits = [("orc_solve.c",
              "    /* Step 3: postsmoothing */\n"
              "    for (int s = 0; s < o->nu; s++) {\n"
              "        sweep(&o->A, B->Aval, B->dinv, r, z, t, R);\n"
              "        memcpy(z, t, (size_t)n * sizeof(double));\n"
              "    }\n",
              "    /* Step 3: postsmoothing */\n"
              "    for (int s = 0; s < o->nu; s++) {\n"
              "        sweep(&o->A, B->Aval, B->dinv, r, z, t, R);\n"
              "        memcpy(z, t, (size_t)n * sizeof(double));\n"
              "    }\n"
              "    for (int i = 0; i < n; i++) z[i] = -z[i];\n")]
    lib = _planted_lib(tmp_path, edits)
    code = (f"import sys; sys.path[:0] = [{ROOT!r}, {os.path.join(ROOT, 'tests')!r}]\n"
            f"import oracle; oracle._LIB_PATH = {lib!r}\n"
            "import oracle_pins; oracle_pins.check_breakdown_status(); print('breakdown-ok')\n")
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0 and "breakdown-ok" in r.stdout, r.stderr[-2000:]
