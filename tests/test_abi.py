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
    for name, val in (("HTR_CHEM_OFF", 1), ("HTR_VISC_OFF", 2), ("HTR_FORCE_CENTRAL", 4), ("HTR_FORCE_TENO", 8),
                      ("HTR_WENO3Z", 16)):
        assert re.search(rf"#define {name}\s+{val}u", hdr)


def test_tile_shape_check_on_the_host():
    """Tile shapes are validated on the host against the staging limits of
    the tiled kernels (no device call)."""
    import ctypes as C
    lib = _lib.load()
    i3 = C.c_int32 * 3
    ok = [((128, 128, 128), s) for s in ((16, 4, 4), (8, 8, 4), (8, 4, 8), (4, 8, 8), (4, 16, 4), (4, 4, 16))]
    ok += [((64, 48, 1), s) for s in ((16, 16, 1), (32, 8, 1), (8, 32, 1), (64, 4, 1))]
    ok += [((1, 64, 48), (1, 16, 16)), ((300, 1, 1), (256, 1, 1))]
    for n, s in ok:
        assert lib.htr_tile_shape_check(i3(*n), i3(*s)) == _lib.HTR_OK, (n, s)
    bad = [((128, 128, 128), (32, 4, 2), b"diffusive sweep"), ((128, 128, 128), (16, 8, 2), b"diffusive sweep"),
           ((64, 48, 1), (16, 4, 4), b"inactive axis"), ((128, 128, 128), (16, 4, 2), b"256 cells"),
           ((128, 128, 128), (2, 16, 8), b"diffusive sweep")]
    for n, s, why in bad:
        assert lib.htr_tile_shape_check(i3(*n), i3(*s)) == _lib.HTR_EINVAL, (n, s)
        assert why in lib.htr_last_error(), (s, lib.htr_last_error())
