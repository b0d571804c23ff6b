"""ctypes binding of the C++ oracle (htr_oracle.cpp).

TEST INFRASTRUCTURE ONLY.  Host (numpy) arrays in, host arrays out.
"""
from __future__ import annotations

import contextlib
import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "htr_oracle.cpp")
LIB = os.path.join(HERE, "liboracle.so")

_dp = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
_ip = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")
_u8 = np.ctypeslib.ndpointer(dtype=np.uint8, flags="C_CONTIGUOUS")

ERRORS = {1: "EINVAL", 4: "ENONFINITE", 5: "ENEWTON", 6: "ETRANGE"}


class OracleError(RuntimeError):
    def __init__(self, code):
        super().__init__(f"oracle error {code} ({ERRORS.get(code, '?')})")
        self.code = code


def build_oracle(force: bool = False) -> str:
    """Compile the oracle with plain FP64 semantics (no contraction, no fast math)."""
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        tmp = LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["g++", "-std=c++17", "-O2", "-fopenmp", "-ffp-contract=off", "-fno-fast-math",
                               "-fPIC", "-shared", "-o", tmp, SRC])
        os.replace(tmp, LIB)
    return LIB


_lib = None


def _bind(path):
    """Opens a compiled oracle library and declares its C signatures."""
    L = C.CDLL(path)
    L.orc_case_new.restype = C.c_void_p
    L.orc_case_new.argtypes = [C.c_int, C.c_int, _dp, _dp, _dp, _dp, _dp, _dp, _dp, _ip, _ip, C.c_double,
                               C.c_double, _ip, _dp, _dp, _dp, _dp, C.c_double, C.c_double, C.c_double,
                               C.c_double, C.c_uint]
    L.orc_case_free.argtypes = [C.c_void_p]
    L.orc_case_set_curvilinear.argtypes = [C.c_void_p, _dp, _dp]
    L.orc_case_set_boundaries.argtypes = [C.c_void_p, _ip, _dp, _dp]
    L.orc_metrics.argtypes = [C.c_void_p, _dp, _dp, _dp]
    L.orc_set_flags.argtypes = [C.c_void_p, C.c_uint]
    L.orc_prim_to_cons.argtypes = [C.c_void_p, _dp, _dp, _dp, _dp, _dp]
    L.orc_cells.argtypes = [C.c_void_p, _dp, _dp, C.c_double, _dp, _dp]
    L.orc_rhs.argtypes = [C.c_void_p, _dp, _dp, C.c_double, _dp, _dp, C.c_void_p, C.c_void_p]
    L.orc_stable_dt.argtypes = [C.c_void_p, _dp, _dp, _dp]
    L.orc_rk3_step.argtypes = [C.c_void_p, _dp, _dp, C.c_double, C.c_double, _dp, C.c_void_p, _dp]
    L.orc_rk3_tangent.argtypes = [C.c_void_p, _dp, _dp, _dp, C.c_double, C.c_double, _dp, _dp, C.c_void_p,
                                  C.c_void_p, _dp, _dp]
    L.orc_rhs_tangent.argtypes = [C.c_void_p, _dp, _dp, _dp, C.c_double, _dp, _dp, C.c_void_p, _dp, _dp,
                                  _dp, _dp]
    L.orc_rates.argtypes = [C.c_void_p, _dp, _dp, _dp]
    L.orc_teno6_detail.restype = C.c_double
    L.orc_teno6_detail.argtypes = [_dp, C.c_double, _dp]
    L.orc_thermo.argtypes = [C.c_void_p, C.c_int, C.c_double, _dp]
    L.orc_teno6.restype = C.c_double
    L.orc_teno6.argtypes = [_dp, C.c_double]
    L.orc_weno3z.restype = C.c_double
    L.orc_weno3z.argtypes = [_dp]
    for f in ("orc_omega22", "orc_omega11"):
        getattr(L, f).restype = C.c_double
        getattr(L, f).argtypes = [C.c_double]
    L.orc_mu_species.restype = C.c_double
    L.orc_mu_species.argtypes = [C.c_void_p, C.c_int, C.c_double]
    L.orc_D_binary.restype = C.c_double
    L.orc_D_binary.argtypes = [C.c_void_p, C.c_int, C.c_int, C.c_double, C.c_double]
    L.orc_cell_volume.restype = C.c_double
    L.orc_cell_volume.argtypes = [C.c_void_p, C.c_longlong]
    return L


def _load():
    global _lib
    if _lib is None:
        build_oracle()
        _lib = _bind(LIB)
    return _lib


def build_variant(replacements, out_dir, name="liboracle_variant.so"):
    """Compiles a copy of the oracle source with the given (old, new) text
    replacements, each of which must match exactly once, into out_dir and
    returns the library's path.  Used only by the tests that plant a mistake
    in the oracle to show that its pins catch it."""
    src = open(SRC).read()
    for old, new in replacements:
        if src.count(old) != 1:
            raise ValueError(f"replacement target occurs {src.count(old)} times: {old!r}")
        src = src.replace(old, new)
    os.makedirs(out_dir, exist_ok=True)
    cpp = os.path.join(out_dir, name.replace(".so", ".cpp"))
    with open(cpp, "w") as fh:
        fh.write(src)
    lib = os.path.join(out_dir, name)
    subprocess.check_call(["g++", "-std=c++17", "-O2", "-fopenmp", "-ffp-contract=off", "-fno-fast-math",
                           "-fPIC", "-shared", "-o", lib, cpp])
    return lib


@contextlib.contextmanager
def use_library(path):
    """Oracle objects created inside the block use the library at path."""
    global _lib
    prev = _load()
    _lib = _bind(path)
    try:
        yield
    finally:
        _lib = prev


def _ptr(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _chk(code):
    if code:
        raise OracleError(code)


class Oracle:
    """One case: mechanism + grid + scheme parameters.  U is [nv][N] float64."""

    def __init__(self, case, flags=None):
        L = _load()
        self.L = L
        m, g = case.mech, case.grid
        self.ns, self.nr, self.N = m.ns, m.nr, g.N
        self.nv = m.ns + 4
        self.n = g.n
        self.flags = case.flags if flags is None else flags
        self._keep = []

        def f64(a):
            a = np.ascontiguousarray(np.asarray(a, dtype=np.float64))
            self._keep.append(a)
            return a

        nf = np.ascontiguousarray(m.nu_f.astype(np.int32).reshape(-1)) if m.nr else np.zeros(1, np.int32)
        nr_ = np.ascontiguousarray(m.nu_r.astype(np.int32).reshape(-1)) if m.nr else np.zeros(1, np.int32)
        self._keep += [nf, nr_]
        z1 = lambda a: f64(a) if len(a) else f64(np.zeros(1))  # noqa: E731
        self.curv = hasattr(g, "xyz")
        if self.curv:   # the rectilinear arrays are unused placeholders
            ones = f64(np.ones(int(sum(g.n))))
            xn, xi, xf, Lp = f64(np.zeros(int(sum(g.n)))), ones, ones, f64(np.ones(3))
        else:
            xn, xi, xf = f64(np.concatenate(g.xnode)), f64(np.concatenate(g.xin)), f64(np.concatenate(g.xif))
            Lp = f64(np.array(g.L))
        self.h = L.orc_case_new(
            m.ns, m.nr, f64(m.W), f64(m.nasa7.reshape(-1)), f64(m.lj_sigma), f64(m.lj_epsk), z1(m.lnA),
            z1(m.beta), z1(m.Ea), nf, nr_, float(m.Tmin), float(m.Tmax), np.array(g.n, np.int32),
            xn, xi, xf, Lp, float(case.theta_c), float(case.psi_c), float(case.teno_CT), float(case.cfl),
            int(self.flags))
        if self.curv:
            _chk(L.orc_case_set_curvilinear(self.h, f64(np.asarray(g.xyz).reshape(-1)),
                                            f64(np.asarray(g.period).reshape(-1))))
        bc = np.ascontiguousarray(np.asarray(getattr(case, "bc", ((0, 0),) * 3), dtype=np.int32).reshape(-1))
        if bc.any():
            self._keep.append(bc)
            _chk(L.orc_case_set_boundaries(self.h, bc, f64(np.asarray(case.pinf, float).reshape(-1)),
                                           f64(np.asarray(case.relax, float).reshape(-1))))
        self.case = case

    def __del__(self):
        try:
            self.L.orc_case_free(self.h)
        except Exception:
            pass

    def set_flags(self, flags):
        self.flags = flags
        self.L.orc_set_flags(self.h, int(flags))

    @staticmethod
    def _las(laser):
        return np.ascontiguousarray(laser.as_array() if hasattr(laser, "as_array") else np.asarray(laser, float))

    def prim_to_cons(self, Y=None, T=None, p=None, vel=None):
        c = self.case
        Y = np.ascontiguousarray(c.Y if Y is None else Y, dtype=np.float64)
        T = np.ascontiguousarray(c.T if T is None else T, dtype=np.float64)
        p = np.ascontiguousarray(c.p if p is None else p, dtype=np.float64)
        vel = np.ascontiguousarray(c.vel if vel is None else vel, dtype=np.float64)
        U = np.zeros((self.nv, self.N))
        _chk(self.L.orc_prim_to_cons(self.h, Y, T, p, vel, U))
        return U

    def cells(self, U, T_io, t=0.0, laser=None):
        """Per-cell rows: T, p, c, mu, lambda, D_s, wdot_s, hrr, q_L, theta."""
        nq = 5 + 2 * self.ns + 3
        out = np.zeros((nq, self.N))
        las = self._las(laser if laser is not None else self.case.laser)
        _chk(self.L.orc_cells(self.h, np.ascontiguousarray(U), T_io, float(t), las, out))
        return out

    def rhs(self, U, T_io, t=0.0, laser=None, want_mask=False, want_hrr=False):
        dUdt = np.zeros((self.nv, self.N))
        hrr = np.zeros(self.N) if want_hrr else None
        mask = np.zeros((3, self.N), np.uint8) if want_mask else None
        las = self._las(laser if laser is not None else self.case.laser)
        _chk(self.L.orc_rhs(self.h, np.ascontiguousarray(U), T_io, float(t), las, dUdt, _ptr(hrr), _ptr(mask)))
        out = [dUdt]
        if want_hrr:
            out.append(hrr)
        if want_mask:
            out.append(mask)
        return out[0] if len(out) == 1 else tuple(out)

    def rates(self, U, T_io):
        """Forward and backward rates of progress, shape [nr][2][N]."""
        out = np.zeros((self.nr, 2, self.N))
        _chk(self.L.orc_rates(self.h, np.ascontiguousarray(U), T_io, out))
        return out

    def destruction_rate(self, U, T_io):
        """Pseudo-first-order destruction rate of every species,
        sum_j (nu'_sj r_fj + nu''_sj r_bj) / c_s, shape [ns][N]."""
        r = self.rates(U, T_io)
        m = self.case.mech
        c = U[:self.ns] / m.W[:, None]
        lam = np.einsum("js,jn->sn", m.nu_f, r[:, 0]) + np.einsum("js,jn->sn", m.nu_r, r[:, 1])
        return lam / np.maximum(c, 1e-300)

    def stable_dt(self, U, T_io):
        dt = np.zeros(1)
        _chk(self.L.orc_stable_dt(self.h, np.ascontiguousarray(U), T_io, dt))
        return float(dt[0])

    def rk3_step(self, U, T_io, t, dt, laser=None, lnA=None, J=None):
        """Advances U in place; returns the updated J (time-integrated heat release)."""
        Jv = np.array([0.0 if J is None else float(J)])
        las = self._las(laser if laser is not None else self.case.laser)
        lnA = None if lnA is None else np.ascontiguousarray(lnA, dtype=np.float64)
        _chk(self.L.orc_rk3_step(self.h, U, T_io, float(t), float(dt), las, _ptr(lnA), Jv))
        return float(Jv[0])

    def rk3_tangent(self, U, dU, T_io, t, dt, laser, dlas, lnA=None, dlnA=None, J=0.0, dJ=0.0):
        Jv = np.array([float(J)])
        dJv = np.array([float(dJ)])
        las = self._las(laser)
        dlas = np.ascontiguousarray(np.asarray(dlas, float))
        lnA = None if lnA is None else np.ascontiguousarray(lnA, dtype=np.float64)
        dlnA = None if dlnA is None else np.ascontiguousarray(dlnA, dtype=np.float64)
        _chk(self.L.orc_rk3_tangent(self.h, U, dU, T_io, float(t), float(dt), las, dlas, _ptr(lnA), _ptr(dlnA),
                                    Jv, dJv))
        return float(Jv[0]), float(dJv[0])

    def rhs_tangent(self, U, dU, T_io, t, laser, dlas, dlnA=None):
        dUdt = np.zeros((self.nv, self.N))
        ddUdt = np.zeros((self.nv, self.N))
        hrr = np.zeros(self.N)
        dhrr = np.zeros(self.N)
        dlnA = None if dlnA is None else np.ascontiguousarray(dlnA, dtype=np.float64)
        _chk(self.L.orc_rhs_tangent(self.h, np.ascontiguousarray(U), np.ascontiguousarray(dU), T_io, float(t),
                                    self._las(laser), np.ascontiguousarray(np.asarray(dlas, float)), _ptr(dlnA),
                                    dUdt, ddUdt, hrr, dhrr))
        return dUdt, ddUdt, hrr, dhrr

    def metrics(self):
        """Curvilinear grids: node metric terms [3][3][N] ((d xi_d / d x_c) / J
        at [d][c]), the same at faces i+1/2 along d, and J [N]."""
        mt, mf, jac = np.zeros((9, self.N)), np.zeros((9, self.N)), np.zeros(self.N)
        self.L.orc_metrics(self.h, mt, mf, jac)
        return mt.reshape(3, 3, self.N), mf.reshape(3, 3, self.N), jac

    def cell_volume(self, q):
        return self.L.orc_cell_volume(self.h, int(q))

    # building blocks
    def teno6(self, f, CT=1e-5):
        return self.L.orc_teno6(np.ascontiguousarray(f, dtype=np.float64), CT)

    def thermo(self, s, T):
        """(c_p/R, h/(RT), s/R) of species s at T."""
        out = np.zeros(3)
        self.L.orc_thermo(self.h, int(s), float(T), out)
        return out

    def mu_species(self, s, T):
        return self.L.orc_mu_species(self.h, s, T)

    def D_binary(self, i, j, T, p):
        return self.L.orc_D_binary(self.h, i, j, T, p)


def omega22(Ts):
    return _load().orc_omega22(float(Ts))


def omega11(Ts):
    return _load().orc_omega11(float(Ts))


def teno6(f, CT=1e-5):
    return _load().orc_teno6(np.ascontiguousarray(f, dtype=np.float64), CT)


def weno3z(f):
    """WENO3-Z reconstruction at x_{i+1/2} from the six-point face stencil
    f_{i-2..i+3} (it uses f_{i-1}, f_i, f_{i+1})."""
    return _load().orc_weno3z(np.ascontiguousarray(f, dtype=np.float64))


def teno6_detail(f, CT=1e-5):
    """Returns (value, dict of beta0..3, beta6, tau, chi[4], omega[4])."""
    d = np.zeros(15)
    v = _load().orc_teno6_detail(np.ascontiguousarray(f, dtype=np.float64), CT, d)
    return v, dict(beta=d[0:4].copy(), beta6=d[4], tau=d[5], chi=d[6:10].copy(), omega=d[10:14].copy())
