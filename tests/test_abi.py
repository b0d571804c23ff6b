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
    bad = [((128, 128, 128), (32, 4, 2), b"too large"), ((128, 128, 128), (16, 8, 2), b"too large"),
           ((64, 48, 1), (16, 4, 4), b"inactive axis"), ((128, 128, 128), (16, 4, 2), b"256 cells"),
           ((128, 128, 128), (2, 16, 8), b"too large")]
    for n, s, why in bad:
        assert lib.htr_tile_shape_check(i3(*n), i3(*s)) == _lib.HTR_EINVAL, (n, s)
        assert why in lib.htr_last_error(), (s, lib.htr_last_error())


def test_curvilinear_lattice_checked_before_device_work():
    """htr_create_curvilinear rejects an invalid grid descriptor before it
    touches the device: NULL arguments, non-finite coordinates, an inactive
    axis whose period is not along its own coordinate (or another period
    with a component along it), and linearly dependent periods."""
    import ctypes as C
    import numpy as np
    lib = _lib.load()
    out = C.c_void_p()
    md = _lib.htr_mech_desc()
    sc = _lib.htr_scheme(cfl=0.5, theta_c=0.1, psi_c=0.05, teno_CT=1e-5, flags=0)

    def desc(n, P, xyz=None):
        g = _lib.htr_curv_grid_desc()
        N = n[0] * n[1] * n[2]
        arr = np.zeros(3 * N) if xyz is None else xyz
        g._keep = arr
        g.xyz = arr.ctypes.data_as(_lib._dp)
        for a in range(3):
            g.n[a] = n[a]
            for c in range(3):
                g.period[a][c] = P[a][c]
        return g
    create = lib.htr_create_curvilinear
    assert create(C.byref(md), None, C.byref(sc), C.byref(out)) == _lib.HTR_EINVAL
    assert create(C.byref(md), C.byref(desc((2, 2, 2), np.eye(3))), C.byref(sc), None) == _lib.HTR_EINVAL
    bad_xyz = np.zeros(24)
    bad_xyz[5] = np.nan
    g = desc((2, 2, 2), np.eye(3), bad_xyz)
    assert create(C.byref(md), C.byref(g), C.byref(sc), C.byref(out)) == _lib.HTR_EINVAL
    assert b"finite" in lib.htr_last_error()
    P = np.eye(3)
    P[2, 0] = 0.5                        # inactive z period leaning into x
    assert create(C.byref(md), C.byref(desc((4, 3, 1), P)), C.byref(sc), C.byref(out)) == _lib.HTR_EINVAL
    assert b"inactive axis 2" in lib.htr_last_error()
    P = np.eye(3)
    P[0, 2] = 0.5                        # x period with a z component, z inactive
    assert create(C.byref(md), C.byref(desc((4, 3, 1), P)), C.byref(sc), C.byref(out)) == _lib.HTR_EINVAL
    P = np.array([[1.0, 0, 0], [2.0, 0, 0], [0, 0, 1.0]])   # dependent periods
    assert create(C.byref(md), C.byref(desc((4, 3, 2), P)), C.byref(sc), C.byref(out)) == _lib.HTR_EINVAL
    assert b"linearly dependent" in lib.htr_last_error()
    assert not out.value


def test_create_rejects_bad_descriptors_before_device_work():
    """htr_create validates the mechanism, the grid and the scheme on the
    host before any device call: empty or oversized mechanisms (ns = 0,
    ns > HTR_MAX_NS, nr > HTR_MAX_NR), missing tables, an empty axis,
    non-positive metrics or periods, and invalid scheme parameters."""
    import ctypes as C
    import numpy as np
    lib = _lib.load()
    keep = []

    def dp(a):
        a = np.ascontiguousarray(np.asarray(a, dtype=np.float64))
        keep.append(a)
        return a.ctypes.data_as(_lib._dp)

    def ip(a):
        a = np.ascontiguousarray(np.asarray(a, dtype=np.int32))
        keep.append(a)
        return a.ctypes.data_as(_lib._ip)

    def mech(ns=1, nr=0, tables=True, Tmin=200.0, Tmax=6000.0):
        m = _lib.htr_mech_desc()
        m.ns, m.nr = ns, nr
        if tables:
            m.W, m.nasa7 = dp(np.full(max(ns, 1), 0.029)), dp(np.tile([3.5, 0, 0, 0, 0, 0, 0], max(ns, 1)))
            m.lj_sigma, m.lj_epsk = dp(np.full(max(ns, 1), 3.6e-10)), dp(np.full(max(ns, 1), 100.0))
            m.lnA, m.beta, m.Ea = dp(np.zeros(max(nr, 1))), dp(np.zeros(max(nr, 1))), dp(np.zeros(max(nr, 1)))
            m.nu_f, m.nu_r = ip(np.zeros(max(nr, 1) * max(ns, 1))), ip(np.zeros(max(nr, 1) * max(ns, 1)))
        m.Tmin, m.Tmax = Tmin, Tmax
        return m

    def grid(n=(4, 3, 2), xi=1e4, L=1e-3):
        g = _lib.htr_grid_desc()
        for a in range(3):
            g.n[a] = n[a]
            g.xnode[a] = dp(np.arange(max(n[a], 1)) * 1e-4)
            g.xi_node[a] = dp(np.full(max(n[a], 1), xi))
            g.xi_face[a] = dp(np.full(max(n[a], 1), xi))
            g.L[a] = L
        return g

    def scheme(cfl=0.5, flags=0):
        return _lib.htr_scheme(cfl=cfl, theta_c=0.1, psi_c=0.05, teno_CT=1e-5, flags=flags)

    out = C.c_void_p()

    def create(m, g, s):
        return lib.htr_create(C.byref(m), C.byref(g), C.byref(s), C.byref(out))
    assert create(mech(ns=0), grid(), scheme()) == _lib.HTR_EINVAL
    assert create(mech(ns=_lib.HTR_MAX_NS + 1), grid(), scheme()) == 7       # HTR_EUNSUPPORTED
    assert create(mech(nr=_lib.HTR_MAX_NR + 1), grid(), scheme()) == 7
    assert create(mech(tables=False), grid(), scheme()) == _lib.HTR_EINVAL
    assert create(mech(Tmin=300.0, Tmax=300.0), grid(), scheme()) == _lib.HTR_EINVAL
    assert create(mech(), grid(n=(0, 3, 2)), scheme()) == _lib.HTR_EINVAL
    assert create(mech(), grid(xi=-1.0), scheme()) == _lib.HTR_EINVAL
    assert create(mech(), grid(L=0.0), scheme()) == _lib.HTR_EINVAL
    assert create(mech(), grid(), scheme(cfl=0.0)) == _lib.HTR_EINVAL
    assert create(mech(), grid(), scheme(flags=_lib.HTR_FORCE_CENTRAL | _lib.HTR_FORCE_TENO)) == _lib.HTR_EINVAL
    assert b"exclusive" in lib.htr_last_error()
    assert not out.value
