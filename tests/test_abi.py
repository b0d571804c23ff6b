"""The C interface library: loads on the host and exports every entry
point include/htr.h declares (no compute calls, no GPU needed)."""
import os
import re

from paper_2202_02319_amd import _lib


def test_header_declares_the_entry_points():
    names = _lib.exported_symbols()
    for required in ("htr_create", "htr_destroy", "htr_rhs", "htr_rk3_step", "htr_stable_dt", "htr_check",
                     "htr_prim_to_cons", "htr_work_bytes", "htr_last_error"):
        assert required in names


def test_library_exports_every_declared_symbol():
    lib = _lib.load()
    missing = [n for n in _lib.exported_symbols() if not hasattr(lib, n)]
    assert not missing, missing


def test_error_path_without_device():
    """Argument errors return before any device work: a NULL context."""
    lib = _lib.load()
    assert lib.htr_check(None, None) == _lib.HTR_EINVAL
    assert lib.htr_rhs(None, None, None, 0.0, None, None, None, None) == _lib.HTR_EINVAL
    assert b"NULL" in lib.htr_last_error()
    assert lib.htr_destroy(None) == _lib.HTR_EINVAL
    assert lib.htr_work_bytes(None) == 0


def test_header_constants_match_binding():
    hdr = open(os.path.join(os.path.dirname(_lib.HERE), "include", "htr.h")).read()
    for name, val in (("HTR_MAX_NS", 12), ("HTR_MAX_NR", 64), ("HTR_MAX_SIDE", 3)):
        assert re.search(rf"#define {name}\s+{val}\b", hdr)
    for name, val in (("HTR_CHEM_OFF", 1), ("HTR_VISC_OFF", 2), ("HTR_FORCE_CENTRAL", 4), ("HTR_FORCE_TENO", 8)):
        assert re.search(rf"#define {name}\s+{val}u", hdr)
