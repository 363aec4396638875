"""Planted mistakes in the oracle's two-level step must break its pins.

Each case edits one line of oracle/amr.py (the level step) or of the
face-flux export in oracle/oracle.c, loads the mutated oracle package from
a temporary copy in a fresh process and runs tests/test_amr_step_pins.py
against it.  Every mutant has to fail at least one pin.  Nothing here
touches the GPU path.
"""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PINS = os.path.join(ROOT, "tests", "test_amr_step_pins.py")

# (file, original text, mutated text)
MUTANTS = {
    "reflux_sign": ("amr.py", "regc[i, d, side] - regf[i, d, side] if side == 0",
                    "regf[i, d, side] - regc[i, d, side] if side == 0"),
    "register_weight": ("amr.py", "r = h * _coarse_face_mean(face, d)",
                        "r = dt * _coarse_face_mean(face, d)"),
    "interpolation_fraction": ("amr.py", "theta = 0.5 * s", "theta = 1.0 * s"),
    "transposed_face_mean": ("amr.py", "s = A[:, 0::2, 0::2] + A[:, 0::2, 1::2]",
                             "A = A.swapaxes(1, 2)\n    s = A[:, 0::2, 0::2] + A[:, 0::2, 1::2]"),
    "reflux_cell": ("amr.py", "c = o[a] - 1 if side == 0 else o[a] + n[a] // 2",
                    "c = o[a] - 1 if side == 0 else o[a] + n[a] // 2 - 1"),
    "fine_face": ("amr.py", "f = g + (0 if side == 0 else n[a])",
                  "f = g + (1 if side == 0 else n[a])"),
    "substep_order": ("amr.py", "for d in order(step_f + s):", "for d in order(step_f):"),
    "flux_export_face": ("oracle.c", "const double *f = F[NG - 1 + i];",
                         "const double *f = F[NG - 1 + (i > 0 ? i - 1 : i)];"),
    "flux_export_component": ("oracle.c", "fout[(1 + perm[1]) * fplane + o] = f[2];",
                              "fout[(1 + perm[1]) * fplane + o] = f[3];"),
}

DRIVER = """
import sys
sys.path.insert(0, {tmp!r})
import oracle, oracle.amr          # the mutated package, before the tests import it
assert oracle.__file__.startswith({tmp!r})
import pytest
sys.exit(pytest.main(["-x", "-q", "-p", "no:cacheprovider", {pins!r}]))
"""


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_level_step_pins_catch_planted_mistake(name, tmp_path):
    fname, old, new = MUTANTS[name]
    pkg = tmp_path / "oracle"
    pkg.mkdir()
    for f in os.listdir(os.path.join(ROOT, "oracle")):
        if f.endswith((".py", ".c")):
            shutil.copy(os.path.join(ROOT, "oracle", f), pkg / f)
    text = (pkg / fname).read_text()
    assert text.count(old) == 1, f"mutation site of {name} not unique"
    (pkg / fname).write_text(text.replace(old, new))
    code = DRIVER.format(tmp=str(tmp_path), pins=PINS)
    env = dict(os.environ, OMP_NUM_THREADS="1")
    env.pop("HYDRO_ORACLE_LIB", None)
    r = subprocess.run([sys.executable, "-c", code], cwd=ROOT, env=env, capture_output=True,
                       text=True, timeout=600)
    assert r.returncode not in (0, 4, 5), r.stdout[-2000:] + r.stderr[-2000:]
    assert r.returncode == 1, f"mutant {name} passed every pin:\n{r.stdout[-2000:]}"


def test_unmutated_copy_passes(tmp_path):
    # the harness itself: an unmodified copy passes every pin
    pkg = tmp_path / "oracle"
    pkg.mkdir()
    for f in os.listdir(os.path.join(ROOT, "oracle")):
        if f.endswith((".py", ".c")):
            shutil.copy(os.path.join(ROOT, "oracle", f), pkg / f)
    code = DRIVER.format(tmp=str(tmp_path), pins=PINS)
    r = subprocess.run([sys.executable, "-c", code], cwd=ROOT, capture_output=True, text=True,
                       timeout=600)
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-2000:]
