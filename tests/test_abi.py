"""CPU checks of the C ABI: the library builds for gfx950, loads, and
exports every function declared in include/hydro.h (no compute calls; there
is no GPU here)."""
import ctypes
import os
import re

import pytest

from paper_1510_05061_amd import hydro

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    text = open(os.path.join(ROOT, "include", "hydro.h")).read()
    return sorted(set(re.findall(r"^\s*(?:int|const char\*)\s+(hydro_\w+)\(", text, re.M)))


def test_header_declares_the_boundary():
    names = _declared()
    for n in ("hydro_init", "hydro_step", "hydro_cfl_dt", "hydro_batch_step",
              "hydro_batch_init", "hydro_totals", "hydro_destroy"):
        assert n in names


def test_library_exports_every_declared_symbol():
    L = hydro.lib()
    for n in _declared():
        assert hasattr(L, n), n
    assert set(_declared()) == set(hydro.exported_symbols())
    assert L.hydro_abi_version() == 3


def test_status_strings_and_struct_layout():
    L = hydro.lib()
    assert b"EINVAL" in L.hydro_strerror(1)
    assert ctypes.sizeof(hydro.HydroDesc) == 4 * 4 + 8 * 5 + 8 * 3 + 4 * 6 + 4 + 4
    assert ctypes.sizeof(hydro.HydroPatch) == 8 + 4 * 4 + 8 * 3 + 8 * 4


def test_workspace_size_and_descriptor_validation_on_host():
    d = hydro.make_desc((16, 16, 16), 1 / 16, 5 / 3)
    assert hydro.hydro_workspace_bytes(d) >= 256
    bad = hydro.make_desc((16, 16, 16), 1 / 16, 1.0)   # gamma must be > 1
    with pytest.raises(hydro.HydroError) as e:
        hydro.hydro_workspace_bytes(bad)
    assert e.value.status == hydro.HYDRO_EINVAL
    half = hydro.make_desc((16, 16, 16), 1 / 16, 1.4,
                           bc=(hydro.PERIODIC, hydro.OUTFLOW, 0, 0, 0, 0))
    with pytest.raises(hydro.HydroError):
        hydro.hydro_workspace_bytes(half)
    badcfl = hydro.make_desc((16, 16, 16), 1 / 16, 1.4, cfl=1.5)
    with pytest.raises(hydro.HydroError):
        hydro.hydro_workspace_bytes(badcfl)


def test_null_pointers_are_rejected_before_any_device_call():
    d = hydro.make_desc((8, 8, 8), 1 / 8, 1.4)
    with pytest.raises(hydro.HydroError) as e:
        hydro.hydro_init(d, None, 0, None, 0, None)
    assert e.value.status == hydro.HYDRO_EINVAL


def test_product_path_does_not_touch_the_oracle():
    # the package never imports or links the oracle
    pkg = os.path.join(ROOT, "paper_1510_05061_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".cpp", ".hpp", ".h")):
                text = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in text and "from oracle" not in text, f
                assert "liboracle" not in text and "oracle.c" not in text, f
