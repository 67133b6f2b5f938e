"""Planted mistakes in the oracle are caught by its pins.

Each mutant below is one plausible slip in writing the method out from the
paper (a dropped term, a wrong sign, index, coefficient or comparison, a
transposed operand).  The test compiles the oracle source with that one
edit into a temporary library, points the oracle binding at it for the
duration of the check, and runs the pins of ``test_oracle_pins.py`` listed
for the mutant: at least one of them must fail.  Nothing outside this test
ever loads a mutant.
"""
from __future__ import annotations

import ctypes
import itertools
import os
import subprocess

import pytest

import oracle
import test_oracle_pins as PINS

# (name, text in wcnst_oracle.c, replacement, pins expected to catch it)
MUTANTS = [
    ("tau5-wrong-pair", "double tau5 = fabs(beta[0] - beta[2]);\n        for (int k = 0; k < 3; ++k) x[k] = p->C",
     "double tau5 = fabs(beta[0] - beta[1]);\n        for (int k = 0; k < 3; ++k) x[k] = p->C",
     ["test_step_cuts_crossing_stencils", "test_tau5_zero_keeps_all_stencils"]),
    ("power-q-minus-1", "for (int m = 0; m < p->q; ++m) g[k] *= xs;", "for (int m = 1; m < p->q; ++m) g[k] *= xs;",
     ["test_step_cuts_crossing_stencils"]),
    ("gamma-without-scaling", "double xs = ldexp(x[k], -ex);", "double xs = x[k];",
     ["test_large_gammas_keep_their_ratios"]),
    ("tie-cuts-at-threshold", "(chi_l[k] < p->CT) ? 0 : 1", "(chi_l[k] <= p->CT) ? 0 : 1",
     ["test_cutoff_threshold_is_inclusive"]),
    ("mirror-shifted", "double sr[5] = {W[5][k], W[4][k], W[3][k], W[2][k], W[1][k]};",
     "double sr[5] = {W[4][k], W[3][k], W[2][k], W[1][k], W[0][k]};",
     ["test_reflection_symmetry_scalar", "test_sod_against_exact_riemann_solution"]),
    ("mnd-coefficient", "c2 = -3.0 / 10.0", "c2 = -1.0 / 10.0", ["test_rhs_exact_for_polynomials"]),
    ("mnd-face-index", "Fm3 = Fface[(size_t)(i + 0) * nv + v]", "Fm3 = Fface[(size_t)(i + 1) * nv + v]",
     ["test_rhs_exact_for_polynomials"]),
    ("candidate-term-sign", "D1[2] = ORC_FMA(3.0, t[2], -t[3]) / 2.0;", "D1[2] = ORC_FMA(3.0, t[2], t[3]) / 2.0;",
     ["test_oracle_interpolation_reproduces_table1", "test_candidates_exact_to_degree_2"]),
    ("beta-drops-second-difference", "beta[k] = ORC_FMA(D1[k], D1[k], D2[k] * D2[k]);",
     "beta[k] = D1[k] * D1[k];", ["test_step_cuts_crossing_stencils", "test_tau5_zero_keeps_all_stencils"]),
    ("roe-dissipation-signed-speed", "R[v * nv + k] * fabs(lam[k])", "R[v * nv + k] * lam[k]",
     ["test_numerical_flux_consistency_and_upwinding", "test_sod_against_exact_riemann_solution"]),
    ("eigenvector-sign", "-0.5 * (b1 * u + ic), 0.5 * b1,\n                        1.0 - b2",
     "-0.5 * (b1 * u - ic), 0.5 * b1,\n                        1.0 - b2", ["test_eigenvectors_and_roe_property"]),
    ("rk-stage-weights", "U2[i] = 0.75 * U[i] + 0.25 * (U1[i] + dt * R[i]);",
     "U2[i] = 0.5 * U[i] + 0.5 * (U1[i] + dt * R[i]);", ["test_full_solve_order_advection"]),
    ("optimal-weights-reversed", "D_OPT[3] = {1.0 / 16.0, 10.0 / 16.0, 5.0 / 16.0}",
     "D_OPT[3] = {5.0 / 16.0, 10.0 / 16.0, 1.0 / 16.0}", ["test_linear_scheme_coefficients"]),
    ("projection-with-right-eigenvectors", "acc = ORC_FMA(L[k * nv + v], st[m * nv + v], acc);",
     "acc = ORC_FMA(R[k * nv + v], st[m * nv + v], acc);",
     ["test_characteristic_projection_is_transparent_on_smooth_data", "test_semidiscrete_order_euler_charwise_roe"]),
    ("ghost-index", "if (g < 0) return 0;\n    if (g >= n) return n - 1;",
     "if (g < 0) return 1;\n    if (g >= n) return n - 1;", ["test_ghost_cells_match_explicit_extension"]),
    ("lf-speed-min", "double al = fmax(aL, aR);", "double al = fmin(aL, aR);", ["test_lax_friedrichs_closed_form"]),
    ("cfl-swapped-spacing", "s = s + (fabs(cell[2] * ir) + a) / p->dy;", "s = s + (fabs(cell[2] * ir) + a) / p->dx;",
     ["test_cfl_speed_hand_computed"]),
    ("cfl-max-for-sum", "s = s + (fabs(cell[2] * ir) + a) / p->dy;", "s = fmax(s, (fabs(cell[2] * ir) + a) / p->dy);",
     ["test_cfl_speed_hand_computed"]),
    ("cfl-drops-sound-speed", "s = (fabs(cell[1] * ir) + a) / p->dx;", "s = fabs(cell[1] * ir) / p->dx;",
     ["test_cfl_speed_hand_computed"]),
    ("final-step-not-clipped", "if (isfinite(t_final) && dt > t_final - t) dt = t_final - t;", "",
     ["test_cfl_time_step_and_final_clip"]),
    ("differences-not-exact-on-constants", "D1[0] = ORC_FMA(3.0, t[1], -t[0]) / 2.0;",
     "D1[0] = ORC_FMA(3.0, s[2], ORC_FMA(-4.0, s[1], s[0])) / 2.0;", ["test_constant_stencil_keeps_every_candidate"]),
    ("vanleer-mass-flux", "double fm = sign * (0.25 * U[0] * c * (a * a));", "double fm = sign * (0.5 * U[0] * c * (a * a));",
     ["test_vanleer_states_at_rest_closed_form"]),
    ("hwcns-coefficient", "b3 = 1.0 / 180.0", "b3 = 1.0 / 90.0", ["test_rhs_exact_for_polynomials"]),
    ("gravity-on-momentum", "R[2 * plane + c] + U[c] * p->gravity", "R[2 * plane + c] + U[2 * plane + c] * p->gravity",
     ["test_gravity_balances_a_hydrostatic_column"]),
    ("wall-reverses-density", "if (bc == ORC_REFLECT && v == 1) return -val;",
     "if (bc == ORC_REFLECT && v == 0) return -val;", ["test_wall_and_fixed_ghosts_match_explicit_extension"]),
    ("wcns-z-ratio-inverted", "double x = tau5 / (beta[k] + p->eps_z), xp = 1.0;",
     "double x = (beta[k] + p->eps_z) / (tau5 + p->eps_z), xp = 1.0;",
     ["test_wcns_z_weights_closed_forms", "test_table2_wcns_z_column"]),
    ("wcns-z-drops-constant-term", "alpha[k] = D_OPT[k] * (1.0 + xp);", "alpha[k] = D_OPT[k] * xp;",
     ["test_wcns_z_weights_closed_forms", "test_table2_wcns_z_column"]),
]


def _source():
    import importlib
    return importlib.import_module("oracle.build").SRC


def _calls(name):
    """Every parametrisation of pin `name` as a callable of the oracle
    module."""
    fn = getattr(PINS, name)
    marks = [m for m in getattr(fn, "pytestmark", []) if m.name == "parametrize"]
    axes = []
    for m in marks:
        names = [n.strip() for n in m.args[0].split(",")] if isinstance(m.args[0], str) else list(m.args[0])
        vals = [v if len(names) > 1 else (v,) for v in m.args[1]]
        axes.append([dict(zip(names, v)) for v in vals])
    for combo in itertools.product(*axes) if axes else [()]:
        kw = {}
        for part in combo:
            kw.update(part)
        yield (lambda kw=kw: fn(oracle, **kw) if "orc" in fn.__code__.co_varnames[:fn.__code__.co_argcount]
               else fn(**kw))


@pytest.mark.parametrize("mutant", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_planted_mistake_is_caught(tmp_path, monkeypatch, mutant):
    name, old, new, pins = mutant
    src = open(_source()).read()
    assert src.count(old) == 1, f"{name}: the text to replace must occur exactly once"
    mutated = tmp_path / "wcnst_oracle.c"
    mutated.write_text(src.replace(old, new))
    lib = tmp_path / "libmutant.so"
    subprocess.run(["gcc", "-O2", "-std=c11", "-mfma", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC",
                    "-shared", "-w", "-I", os.path.dirname(_source()), "-o", str(lib), str(mutated), "-lm"],
                   check=True)
    monkeypatch.setattr(oracle, "_lib", oracle._configure(ctypes.CDLL(str(lib))))
    caught = []
    for pin in pins:
        for call in _calls(pin):
            try:
                call()
            except Exception as e:  # an assertion, or an error the mutant provokes
                caught.append((pin, type(e).__name__))
                break
        if caught:
            break
    assert caught, f"mutant {name} passed every pin in {pins}"


def test_pins_pass_on_the_unmutated_oracle():
    """The pins named above pass on the real oracle (so a failure under a
    mutant is the mutant's)."""
    for pin in sorted({p for m in MUTANTS for p in m[3]}):
        for call in _calls(pin):
            call()
