"""Planted mistakes in the oracle must break its pins.

Each case edits one line of oracle/oracle.c (a dropped term, a wrong sign,
factor, index or component, a wrong boundary copy or sweep order), builds
the mutant into a temporary library and runs the pin suite against it in a
fresh process.  The suite has to fail for every mutant: that is the
evidence that the pins constrain each part of the oracle.  Nothing here
touches the GPU path.
"""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "oracle.c")

MUTANTS = {
    "mc_factor": ("m = fmin(m, 0.5 * fabs(a + b));", "m = fmin(m, fabs(a + b));"),
    "predictor_sign": ("AD[1] = u * D[1] + D[4] / rho;", "AD[1] = u * D[1] - D[4] / rho;"),
    "predictor_half": ("double drift = 0.5 * dtdx * AD[v];", "double drift = dtdx * AD[v];"),
    "energy_flux_term": ("F[4] = u * (E + W[4]);", "F[4] = u * E;"),
    "gravity_energy_sign": ("pen[c][4] += dt * g * (0.5 * (F[c - 1][0] + F[c][0]));",
                            "pen[c][4] += dt * g * (0.5 * (F[c - 1][0] - F[c][0]));"),
    "davis_speed": ("double SL = fmin(uL - cL, uR - cR);",
                    "double SL = fmin(uL - cL, uR + cR);"),
    "periodic_ghost_index": ("case ORC_PERIODIC: src = cell_at(g, d, N - k, a, b); break;",
                             "case ORC_PERIODIC: src = cell_at(g, d, N - k - 1, a, b); break;"),
    "transverse_swap": ("pen[c][2] = src[1 + perm[1]];", "pen[c][2] = src[1 + perm[2]];"),
    "star_energy_sign": ("Us[4] = f * (E + (Ss - u) * (rho * Ss + p / (S - u)));",
                         "Us[4] = f * (E + (Ss - u) * (rho * Ss - p / (S - u)));"),
    "pressure_half": ("W[4] = (gamma - 1.0) * (U[4] - 0.5 * mm / rho);",
                      "W[4] = (gamma - 1.0) * (U[4] - mm / rho);"),
    "contact_speed_sign": ("double num = (pR - pL) + (rL * uL * (SL - uL)",
                           "double num = (pL - pR) + (rL * uL * (SL - uL)"),
    "strang_order": ("odd[3] = {2, 1, 0};", "odd[3] = {0, 1, 2};"),
    "wall_gravity_mirror": ("double kick = mirrored ? -half_dt_g : half_dt_g;",
                            "double kick = half_dt_g;"),
    "cfl_width": ("double s = (fabs(W[1 + d]) + cs) / p->dx[d];",
                  "double s = (fabs(W[1 + d]) + cs) * p->dx[d];"),
    "momentum_source_old_rho": ("pen[c][1] += dt * g * (0.5 * (rho_old + pen[c][0]));",
                                "pen[c][1] += dt * g * rho_old;"),
    "fallback_disabled": ("hancock(W[c], Z, dtdx, gamma, kick, has_g, Wm[c], Wp[c]);",
                          "(void)Z;"),
    "fallback_without_kick": ("hancock(W[c], Z, dtdx, gamma, kick, has_g, Wm[c], Wp[c]);",
                              "hancock(W[c], Z, dtdx, gamma, kick, 0, Wm[c], Wp[c]);"),
    "fallback_density_unchecked": (
        "if (Wm[c][0] <= 0.0 || Wm[c][4] <= 0.0 || Wp[c][0] <= 0.0 ||",
        "if (Wm[c][4] <= 0.0 ||"),
    "fallback_plus_pressure_unchecked": ("        Wp[c][4] <= 0.0) {", "        0) {"),
    "fallback_minus_pressure_unchecked": ("Wm[c][4] <= 0.0 || ", ""),
    "update_sign":("for (int v = 0; v < NV; ++v) pen[c][v] -= dtdx * (F[c][v] - F[c - 1][v]);",
                    "for (int v = 0; v < NV; ++v) pen[c][v] += dtdx * (F[c][v] - F[c - 1][v]);"),
}


def _reflect_negation_mutant(text):
    # drop the normal-momentum negation of the low-side mirror ghost only
    key = "        if (negate) dst[1 + d] = -dst[1 + d];\n        /* high side"
    assert text.count(key) == 1
    return text.replace(key, "        /* high side")


@pytest.mark.parametrize("name", sorted(MUTANTS) + ["reflect_negation"])
def test_pins_catch_planted_mistake(name, tmp_path):
    from oracle.build import build
    text = open(SRC).read()
    if name == "reflect_negation":
        mutated = _reflect_negation_mutant(text)
    else:
        old, new = MUTANTS[name]
        assert text.count(old) == 1, f"mutation site of {name} not unique"
        mutated = text.replace(old, new)
    src = tmp_path / "oracle_mutant.c"
    src.write_text(mutated)
    lib = build(force=True, src=str(src), lib=str(tmp_path / "liboracle_mutant.so"))
    env = dict(os.environ, HYDRO_ORACLE_LIB=lib, OMP_NUM_THREADS="1")
    cmd = [sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
           os.path.join(ROOT, "tests", "test_oracle_pins.py")]
    r = subprocess.run(cmd, cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    assert r.returncode != 0, f"mutant {name} passed every pin:\n{r.stdout[-2000:]}"
