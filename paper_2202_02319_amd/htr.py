"""Python binding of the C interface (include/htr.h).

Argument marshalling only: torch tensors provide device memory and the
current HIP stream; every step of the computation runs in the HIP kernels
of libhtr.so.  Functions carry the names of the C entry points.
"""
from __future__ import annotations

import ctypes as C

import numpy as np
import torch

from . import _lib
from ._lib import HTRError, check, htr_grid_desc, htr_laser, htr_mech_desc, htr_member_desc, htr_scheme  # noqa: F401,E501


def _ptr(t):
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("device tensor required")
    if t.dtype not in (torch.float64, torch.uint8):
        raise ValueError(f"float64 tensor required, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError("contiguous tensor required")
    return C.c_void_p(t.data_ptr())


def _stream(stream):
    if stream is None:
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream))


def _f64(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def make_laser(laser) -> htr_laser | None:
    """htr_laser from an object with E, center, sigma_r, t0, sigma_t, on (or None)."""
    if laser is None:
        return None
    L = htr_laser()
    L.E = float(laser.E)
    for a in range(3):
        L.center[a] = float(laser.center[a])
    L.sigma_r = float(laser.sigma_r)
    L.t0 = float(laser.t0)
    L.sigma_t = float(laser.sigma_t)
    L.on = 1 if laser.on else 0
    return L


class Context:
    """Owns an htr_ctx for one mechanism, grid and scheme."""

    def __init__(self, mech, grid, *, cfl=0.5, theta_c=0.1, psi_c=0.05, teno_CT=1e-5, flags=0):
        lib = _lib.load()
        self._keep = []
        md = htr_mech_desc()
        md.ns, md.nr = int(mech.ns), int(mech.nr)

        def dp(a):
            a = _f64(a)
            if a.size == 0:
                a = np.zeros(1)
            self._keep.append(a)
            return a.ctypes.data_as(_lib._dp)

        def ip(a):
            a = np.ascontiguousarray(np.asarray(a, dtype=np.int32)).reshape(-1)
            if a.size == 0:
                a = np.zeros(1, np.int32)
            self._keep.append(a)
            return a.ctypes.data_as(_lib._ip)
        md.W, md.nasa7 = dp(mech.W), dp(np.asarray(mech.nasa7).reshape(-1))
        md.lj_sigma, md.lj_epsk = dp(mech.lj_sigma), dp(mech.lj_epsk)
        md.lnA, md.beta, md.Ea = dp(mech.lnA), dp(mech.beta), dp(mech.Ea)
        md.nu_f, md.nu_r = ip(mech.nu_f), ip(mech.nu_r)
        md.Tmin, md.Tmax = float(mech.Tmin), float(mech.Tmax)
        sc = htr_scheme(cfl=cfl, theta_c=theta_c, psi_c=psi_c, teno_CT=teno_CT, flags=flags)
        h = C.c_void_p()
        self.curvilinear = hasattr(grid, "xyz")
        if self.curvilinear:   # node coordinates and lattice periods
            gd = _lib.htr_curv_grid_desc()
            for a in range(3):
                gd.n[a] = int(grid.n[a])
                for c in range(3):
                    gd.period[a][c] = float(grid.period[a][c])
            gd.xyz = dp(np.asarray(grid.xyz).reshape(-1))
            check(lib.htr_create_curvilinear(C.byref(md), C.byref(gd), C.byref(sc), C.byref(h)))
        else:
            gd = htr_grid_desc()
            for a in range(3):
                gd.n[a] = int(grid.n[a])
                gd.xnode[a] = dp(grid.xnode[a])
                gd.xi_node[a] = dp(grid.xin[a])
                gd.xi_face[a] = dp(grid.xif[a])
                gd.L[a] = float(grid.L[a])
            check(lib.htr_create(C.byref(md), C.byref(gd), C.byref(sc), C.byref(h)))
        self.h = h
        self.lib = lib
        self.ns, self.nr = md.ns, md.nr
        self.nv = self.ns + 4
        self.N = int(lib.htr_num_cells(h))
        self.n = tuple(int(v) for v in grid.n)
        self.flags = flags
        self._keep = []

    @classmethod
    def from_case(cls, case, flags=None):
        g = cls(case.mech, case.grid, cfl=case.cfl, theta_c=case.theta_c, psi_c=case.psi_c,
                teno_CT=case.teno_CT, flags=case.flags if flags is None else flags)
        bc = getattr(case, "bc", None)
        if bc is not None and np.any(np.asarray(bc)):
            htr_set_boundaries(g, bc, case.pinf, case.relax)
        return g

    def close(self):
        if getattr(self, "h", None):
            check(self.lib.htr_destroy(self.h))
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_flags(self, flags):
        check(self.lib.htr_set_flags(self.h, int(flags)))
        self.flags = flags

    def work_bytes(self):
        return int(self.lib.htr_work_bytes(self.h))

    def new_work(self, device="cuda"):
        return torch.empty(self.work_bytes() // 8, dtype=torch.float64, device=device)


# ------------------------------------------------------------ C-name binding
def htr_set_boundaries(ctx, bc, pinf, relax):
    """Boundary type per axis and side (HTR_BC_*), outflow far-field
    pressure and relaxation coefficient, each [3][2]."""
    b = np.ascontiguousarray(np.asarray(bc, dtype=np.int32).reshape(3, 2))
    p = np.ascontiguousarray(np.asarray(pinf, dtype=np.float64).reshape(3, 2))
    r = np.ascontiguousarray(np.asarray(relax, dtype=np.float64).reshape(3, 2))
    check(ctx.lib.htr_set_boundaries(ctx.h, b.ctypes.data, p.ctypes.data, r.ctypes.data))


def htr_prim_to_cons(ctx, Y, T, p, vel, U, stream=None):
    check(ctx.lib.htr_prim_to_cons(ctx.h, _ptr(Y), _ptr(T), _ptr(p), _ptr(vel), _ptr(U), _stream(stream)))


def htr_rhs(ctx, U, T_io, t, laser, dUdt, hrr=None, stream=None):
    L = make_laser(laser)
    check(ctx.lib.htr_rhs(ctx.h, _ptr(U), _ptr(T_io), float(t), C.byref(L) if L else None, _ptr(dUdt),
                          _ptr(hrr), _stream(stream)))


def htr_cells(ctx, U, T_io, t, laser, out, stream=None):
    L = make_laser(laser)
    check(ctx.lib.htr_cells(ctx.h, _ptr(U), _ptr(T_io), float(t), C.byref(L) if L else None, _ptr(out),
                            _stream(stream)))


def htr_stable_dt(ctx, U, T_io, dt_dev, stream=None):
    check(ctx.lib.htr_stable_dt(ctx.h, _ptr(U), _ptr(T_io), _ptr(dt_dev), _stream(stream)))


def htr_work_bytes(ctx):
    return int(ctx.lib.htr_work_bytes(ctx.h))


def htr_rk3_step(ctx, U, T_io, t_dev, dt_dev, compute_dt, laser, dlnA_dev, work, J_dev=None, stream=None):
    L = make_laser(laser)
    check(ctx.lib.htr_rk3_step(ctx.h, _ptr(U), _ptr(T_io), _ptr(t_dev), _ptr(dt_dev), int(compute_dt),
                               C.byref(L) if L else None, _ptr(dlnA_dev), _ptr(work), _ptr(J_dev), _stream(stream)))


def htr_rk3_step_noalloc(ctx, U, T_io, t_dev, dt_dev, compute_dt, laser, dlnA_dev, J_dev=None, stream=None):
    L = make_laser(laser)
    check(ctx.lib.htr_rk3_step_noalloc(ctx.h, _ptr(U), _ptr(T_io), _ptr(t_dev), _ptr(dt_dev), int(compute_dt),
                                       C.byref(L) if L else None, _ptr(dlnA_dev), _ptr(J_dev), _stream(stream)))


def htr_timing(ctx, enable):
    check(ctx.lib.htr_timing(ctx.h, int(enable)))


KERNEL_CLASSES = ("point", "sensor", "conv", "diff", "reduce", "update")


def htr_timing_read(ctx):
    """{class: (total ms, launches)} since htr_timing(ctx, 1)."""
    nc = len(KERNEL_CLASSES)
    ms = (C.c_double * nc)()
    n = (C.c_int64 * nc)()
    check(ctx.lib.htr_timing_read(ctx.h, ms, n))
    return {KERNEL_CLASSES[k]: (ms[k], n[k]) for k in range(nc)}


def htr_adjoint_work_bytes(ctx):
    return int(ctx.lib.htr_adjoint_work_bytes(ctx.h))


def new_adjoint_work(ctx, device="cuda"):
    return torch.empty(htr_adjoint_work_bytes(ctx) // 8, dtype=torch.float64, device=device)


def htr_rhs_adjoint(ctx, U, T_io, t, laser, dlnA_dev, lam, s, h, Ubar_acc, pbar_acc, adj_work, stream=None):
    L = make_laser(laser)
    check(ctx.lib.htr_rhs_adjoint(ctx.h, _ptr(U), _ptr(T_io), float(t), C.byref(L) if L else None, _ptr(dlnA_dev),
                                  _ptr(lam), float(s), float(h), _ptr(Ubar_acc), _ptr(pbar_acc), _ptr(adj_work),
                                  _stream(stream)))


def htr_rk3_step_adjoint(ctx, Un, stages, T_io, t, dt, laser, dlnA_dev, Jbar, Ubar, pbar_acc, adj_work,
                         tape=None, stream=None):
    L = make_laser(laser)
    check(ctx.lib.htr_rk3_step_adjoint(ctx.h, _ptr(Un), _ptr(stages), _ptr(T_io), float(t), float(dt),
                                       C.byref(L) if L else None, _ptr(dlnA_dev), float(Jbar), _ptr(Ubar),
                                       _ptr(pbar_acc), _ptr(adj_work), _ptr(tape), _stream(stream)))


def htr_tape_bytes(ctx):
    return int(ctx.lib.htr_tape_bytes(ctx.h))


def new_tape(ctx, device="cuda"):
    """Device buffer for the forward tape of one RK3 step."""
    return torch.empty((htr_tape_bytes(ctx) + 7) // 8, dtype=torch.float64, device=device)


def tape_switches(ctx, tape):
    """Byte views of a forward tape's discrete switches, by the layout that
    htr_tape_bytes states: the sensor flags [3 stages][N] and the TENO
    cut-off patterns [3 stages][3 axes][nv][N]."""
    b = tape.view(torch.uint8)
    N, nv = ctx.N, ctx.ns + 4
    o = 3 * (8 + ctx.ns) * N * 8
    return b[o:o + 3 * N], b[o + 3 * N:o + 3 * N + 9 * nv * N]


def htr_rk3_step_taped(ctx, U, T_io, t_dev, dt_dev, compute_dt, laser, dlnA_dev, work, J_dev, tape, stream=None):
    L = make_laser(laser)
    check(ctx.lib.htr_rk3_step_taped(ctx.h, _ptr(U), _ptr(T_io), _ptr(t_dev), _ptr(dt_dev), int(compute_dt),
                                     C.byref(L) if L else None, _ptr(dlnA_dev), _ptr(work), _ptr(J_dev), _ptr(tape),
                                     _stream(stream)))


def _i3(v):
    return (C.c_int32 * 3)(*[int(x) for x in v])


def htr_tile_shape_check(n, shape):
    """Host-only check that shape is a valid tile for a grid of n cells;
    raises HTRError with the reason otherwise."""
    check(_lib.load().htr_tile_shape_check(_i3(n), _i3(shape)))


def htr_set_tiling(ctx, shape=None, grid=0):
    check(ctx.lib.htr_set_tiling(ctx.h, _i3(shape) if shape is not None else None, int(grid)))


def htr_get_tiling(ctx):
    """(tile shape, persistent grid) of the context."""
    sh, g = (C.c_int32 * 3)(), C.c_int32()
    check(ctx.lib.htr_get_tiling(ctx.h, sh, C.byref(g)))
    return tuple(sh), g.value


def htr_set_conv_split(ctx, split):
    check(ctx.lib.htr_set_conv_split(ctx.h, int(split)))


def htr_get_conv_split(ctx):
    v = C.c_int32()
    check(ctx.lib.htr_get_conv_split(ctx.h, C.byref(v)))
    return int(v.value)


def htr_batch_set_conv_split(b, split):
    check(b.lib.htr_batch_set_conv_split(b.h, int(split)))


def htr_batch_get_conv_split(b):
    v = C.c_int32()
    check(b.lib.htr_batch_get_conv_split(b.h, C.byref(v)))
    return int(v.value)


def htr_autotune(ctx, U, T_io, work, stream=None):
    """Times every candidate tile shape and persistent grid on one RHS and
    keeps the fastest; returns (shape, grid)."""
    sh, g = (C.c_int32 * 3)(), C.c_int32()
    check(ctx.lib.htr_autotune(ctx.h, _ptr(U), _ptr(T_io), _ptr(work), _stream(stream), sh, C.byref(g)))
    return tuple(sh), g.value


def htr_batch_set_tiling(b, member=-1, shape=None, grid=0):
    check(b.lib.htr_batch_set_tiling(b.h, int(member), _i3(shape) if shape is not None else None, int(grid)))


def htr_batch_get_tiling(b, member):
    sh, g = (C.c_int32 * 3)(), C.c_int32()
    check(b.lib.htr_batch_get_tiling(b.h, int(member), sh, C.byref(g)))
    return tuple(sh), g.value


def htr_batch_autotune(b, U, T_io, work, stream=None):
    """Tunes each equal-size member class's tile shape, then the persistent
    grid; returns the per-member shapes and the grid."""
    check(b.lib.htr_batch_autotune(b.h, _ptr(U), _ptr(T_io), _ptr(work), _stream(stream)))
    shapes = [htr_batch_get_tiling(b, m)[0] for m in range(b.nmem)]
    return shapes, htr_batch_get_tiling(b, 0)[1]


def htr_grid_metrics(ctx, mt, mf, stream=None):
    """Curvilinear context: node metric terms and J into mt [10][N], face
    metric terms into mf [9][N] (device tensors)."""
    check(ctx.lib.htr_grid_metrics(ctx.h, _ptr(mt), _ptr(mf), _stream(stream)))


def htr_check(ctx, stream=None):
    check(ctx.lib.htr_check(ctx.h, _stream(stream)))


# ------------------------------------------------------------ conveniences
def to_dev(a, device="cuda"):
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64), device=device)


def cons_from_case(ctx, case, device="cuda"):
    """U on the device from the case's primitive fields (GPU conversion)."""
    U = torch.empty((ctx.nv, ctx.N), dtype=torch.float64, device=device)
    htr_prim_to_cons(ctx, to_dev(case.Y, device), to_dev(case.T, device), to_dev(case.p, device),
                     to_dev(case.vel, device), U)
    return U


# ------------------------------------------------------------------ ensembles
class Batch:
    """Owns an htr_batch: members (grids with uniform spacing, lasers, ln A
    offsets) on a context's mechanism and scheme."""

    def __init__(self, ctx, grids, lasers, dlnA=None):
        lib = ctx.lib
        nmem = len(grids)
        descs = (htr_member_desc * nmem)()
        self._keep = []
        for m in range(nmem):
            g = grids[m]
            d = descs[m]
            for a in range(3):
                d.n[a] = int(g.n[a])
                d.dx[a] = float(1.0 / g.xin[a][0])
            L = make_laser(lasers[m]) if lasers[m] is not None else htr_laser()
            d.laser = L
            if dlnA is not None:
                arr = np.ascontiguousarray(np.asarray(dlnA[m], dtype=np.float64))
                self._keep.append(arr)
                d.dlnA = arr.ctypes.data_as(_lib._dp)
        h = C.c_void_p()
        check(lib.htr_batch_create(ctx.h, nmem, descs, C.byref(h)))
        self.h, self.lib, self.ctx = h, lib, ctx
        self.nmem = nmem
        offs = (C.c_int64 * (nmem + 1))()
        self.N = int(lib.htr_batch_cells(h, offs))
        self.offsets = [int(offs[m]) for m in range(nmem + 1)]
        self._keep = []

    @classmethod
    def from_cases(cls, ctx, cases, dlnA=None):
        return cls(ctx, [c.grid for c in cases], [c.laser if c.laser.on else None for c in cases], dlnA)

    def close(self):
        if getattr(self, "h", None):
            check(self.lib.htr_batch_destroy(self.h))
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def new_work(self, device="cuda"):
        return torch.empty(int(self.lib.htr_batch_work_bytes(self.h)) // 8, dtype=torch.float64, device=device)

    def pack(self, arrays, rows):
        """Packs per-member host arrays [rows][N_m] (or [N_m]) member-major."""
        parts = [np.asarray(a, dtype=np.float64).reshape(rows, -1) for a in arrays]
        return np.concatenate([p.ravel() for p in parts])

    def unpack(self, flat, rows, m):
        o0, o1 = self.offsets[m], self.offsets[m + 1]
        return np.asarray(flat)[rows * o0: rows * o1].reshape(rows, o1 - o0)


def htr_batch_prim_to_cons(b, Y, T, p, vel, U, stream=None):
    check(b.lib.htr_batch_prim_to_cons(b.h, _ptr(Y), _ptr(T), _ptr(p), _ptr(vel), _ptr(U), _stream(stream)))


def htr_rhs_batched(b, U, T_io, t_dev, dUdt, hrr=None, stream=None):
    check(b.lib.htr_rhs_batched(b.h, _ptr(U), _ptr(T_io), _ptr(t_dev), _ptr(dUdt), _ptr(hrr), _stream(stream)))


def htr_rk3_steps_batched(b, U, T_io, t_dev, dt_dev, compute_dt, nsteps, work, J_dev=None, use_graph=False,
                          stream=None):
    check(b.lib.htr_rk3_steps_batched(b.h, _ptr(U), _ptr(T_io), _ptr(t_dev), _ptr(dt_dev), int(compute_dt),
                                      int(nsteps), _ptr(work), _ptr(J_dev), int(bool(use_graph)),
                                      _stream(stream)))


def htr_batch_member_max(b, field, max_dev, accumulate=False, stream=None):
    check(b.lib.htr_batch_member_max(b.h, _ptr(field), _ptr(max_dev), int(bool(accumulate)), _stream(stream)))


def htr_batch_check(b, stream=None):
    check(b.lib.htr_batch_check(b.h, _stream(stream)))


def batch_state_from_cases(b, cases, device="cuda"):
    """Packed U (GPU conversion) and T for a list of member cases."""
    ns = b.ctx.ns
    Y = to_dev(b.pack([c.Y for c in cases], ns), device)
    T = to_dev(b.pack([c.T for c in cases], 1), device)
    p = to_dev(b.pack([c.p for c in cases], 1), device)
    vel = to_dev(b.pack([c.vel for c in cases], 3), device)
    U = torch.empty(b.N * (ns + 4), dtype=torch.float64, device=device)
    htr_batch_prim_to_cons(b, Y, T, p, vel, U)
    return U, T
