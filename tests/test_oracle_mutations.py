"""The pins must fail on a plausible mistake: each case plants one in a copy of the oracle (CPU only).

A copy of ``oracle/`` is written to a temporary package with one edit (a
transposed inverse Jacobian, a dropped determinant, a wrong sign, swapped
derivative tables, a wrong quadrature weight, a wrong Chebyshev coefficient,
a Chebyshev base map ignored, a wrong multigrid correction sign, a dropped
post-smoothing, wrong interpolation points),
and the pin tests are run against it with the module swapped in. Every
mutant must make at least one pin fail.
"""
import importlib
import os
import shutil
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

MUTANTS = {
    "transposed_inverse_jacobian": ("fem.py", 'np.einsum("nda,dni->ani", inv, er.dPhi)',
                                    'np.einsum("nad,dni->ani", inv, er.dPhi)'),
    "dropped_determinant": ("fem.py", "wd = er.w3 * det * kappa_eval(kappa, x)", "wd = er.w3 * kappa_eval(kappa, x)"),
    "wrong_shape_derivative_sign": ("fem.py", "dN[:, :, 1] = 0.5 * s[None, :, 1]", "dN[:, :, 1] = -0.5 * s[None, :, 1]"),
    "cofactor_sign": ("fem.py", "cof[:, 1, 2] = -(a[:, 0, 0]", "cof[:, 1, 2] = (a[:, 0, 0]"),
    "swapped_derivative_tables": ("fem.py", "outer(phi, dphi, phi), outer(dphi, phi, phi)",
                                  "outer(dphi, phi, phi), outer(phi, dphi, phi)"),
    "kappa_at_reference_points": ("fem.py", "wd = er.w3 * det * kappa_eval(kappa, x)",
                                  "wd = er.w3 * det * kappa_eval(kappa, er.r3)"),
    "kappa_axes_swapped": ("fem.py", "wd = er.w3 * det * kappa_eval(kappa, x)",
                           "wd = er.w3 * det * kappa_eval(kappa, x[:, ::-1])"),
    "lambda_max_unscaled": ("solvers.py", "S = sp.diags(s) @ Aii @ sp.diags(s)", "S = Aii"),
    "lor_subhex_corner_order": ("fem.py", "for c in (0, 1) for b in (0, 1) for a in (0, 1)]",
                                "for c in (0, 1) for a in (0, 1) for b in (0, 1)]"),
    "helmholtz_mass_scale": ("fem.py", "return (alpha * A + beta * B).tocsr()", "return (alpha * A + alpha * B).tocsr()"),
    "gll_weight_formula": ("quadrature.py", "w = 2.0 / (p * (p + 1) * Pp * Pp)", "w = 2.0 / (p * (p + 1) * Pp)"),
    "chebyshev_coefficient": ("solvers.py", "d = rho_new * rho * d + (2.0 * rho_new / delta) * M(res)",
                              "d = rho_new * d + (2.0 * rho_new / delta) * M(res)"),
    "chebyshev_base_map_ignored": ("solvers.py", "M = dinv if callable(dinv) else (lambda v: dinv * v)",
                                   "M = (lambda v: v) if callable(dinv) else (lambda v: dinv * v)"),
    "coarse_correction_sign": ("pmg.py", "x = x + (lv.P @ ec) * lv.f", "x = x - (lv.P @ ec) * lv.f"),
    "dropped_post_smoothing": ("pmg.py", "return x + chebyshev_apply(lv.A, M, t, lam_lo, lam_hi, degree)",
                               "return x"),
    "interpolation_swapped_nodes": ("pmg.py", "return lagrange_table(xc, xf)", "return lagrange_table(xc, -xf[::-1] ** 3)"),
}

PINS = {
    "fem.py": ("test_oracle_fem", ["test_mass_integrates_volume", "test_coordinate_function_forms",
                                   "test_diffusion_invariants", "test_collocated_diagonal_closed_form",
                                   "test_kappa_location_closed_form", "test_helmholtz_forms",
                                   "test_lor_invariants_and_coordinate_function"]),
    "quadrature.py": ("test_oracle_quadrature", ["test_closed_forms", "test_exactness_degrees"]),
    "solvers.py": ("test_oracle_solvers", ["test_chebyshev_recurrence_equals_polynomial",
                                           "test_chebyshev_general_base_map", "test_lambda_max_lanczos_branch"]),
    "pmg.py": ("test_oracle_pmg", ["test_interpolation_1d", "test_prolongation_reproduces_coarse_space",
                                   "test_galerkin_identity", "test_vcycle_symmetric_and_contracting"]),
}


def _run_pins(modname, names):
    """Run the listed pin tests (all their parametrizations) in-process; return the number of failures."""
    mod = importlib.import_module(modname)
    fails = 0
    for name in names:
        fn = getattr(mod, name)
        marks = getattr(fn, "pytestmark", [])
        cases = [dict()]
        for m in marks:
            if m.name != "parametrize":
                continue
            argnames = [a.strip() for a in m.args[0].split(",")] if isinstance(m.args[0], str) else list(m.args[0])
            new = []
            for c in cases:
                for v in m.args[1]:
                    vals = v if len(argnames) > 1 else (v,)
                    new.append({**c, **dict(zip(argnames, vals))})
            cases = new
        for c in cases:
            try:
                fn(**c)
            except AssertionError:
                fails += 1
            except Exception:
                fails += 1
    return fails


@pytest.mark.parametrize("mutant", sorted(MUTANTS))
def test_pins_catch_planted_mistake(mutant, tmp_path, monkeypatch):
    fname, old, new = MUTANTS[mutant]
    pkg = tmp_path / "oracle"
    shutil.copytree(os.path.join(ROOT, "oracle"), pkg, ignore=shutil.ignore_patterns("__pycache__"))
    src = (pkg / fname).read_text()
    assert old in src, "mutation anchor not found: the oracle changed, update the mutant"
    (pkg / fname).write_text(src.replace(old, new))
    saved = {k: v for k, v in sys.modules.items() if k == "oracle" or k.startswith("oracle.")}
    test_mods = {k: sys.modules.pop(k) for k in list(sys.modules) if k.startswith("test_oracle_")}
    for k in saved:
        del sys.modules[k]
    monkeypatch.syspath_prepend(str(tmp_path))
    monkeypatch.syspath_prepend(os.path.dirname(os.path.abspath(__file__)))
    try:
        import oracle  # noqa: F401  (the mutated copy)
        assert str(tmp_path) in oracle.__file__
        modname, names = PINS[fname]
        assert _run_pins(modname, names) > 0, f"no pin failed for mutant {mutant}"
    finally:
        for k in [k for k in sys.modules if k == "oracle" or k.startswith("oracle.") or k.startswith("test_oracle_")]:
            del sys.modules[k]
        sys.modules.update(saved)
        sys.modules.update(test_mods)


def test_unmutated_oracle_passes_the_same_pins():
    sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
    try:
        for modname, names in PINS.values():
            assert _run_pins(modname, names) == 0
    finally:
        sys.path.pop(0)
