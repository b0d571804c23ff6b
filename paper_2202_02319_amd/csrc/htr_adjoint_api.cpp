// Host side of the discrete adjoint: one RHS vector-Jacobian product (a
// forward per-cell pass and sensor on the state, then the adjoint sweep and
// the adjoint per-cell kernel), and the reverse of one SSP-RK3 step.

#include <hip/hip_runtime.h>

#include <cmath>

#include "htr.h"
#include "htr_dev.h"
#include "htr_internal.h"

using namespace htr;

namespace {

struct AdjBufs {
  double* ubd;       // [nv][N] direct cotangent of the conserved variables
  double* pb;        // [8 + ns][N] cotangent of the per-cell fields
  double* B1;        // [nv][N]
  double* B2;        // [nv][N]
  double* thpart;    // [nblocks][4 + nr]
};

AdjBufs split(const htr_ctx* c, double* w) {
  const long long N = c->N;
  const int nv = c->ns + 4;
  AdjBufs b;
  b.ubd = w;
  b.pb = b.ubd + nv * N;
  b.B1 = b.pb + (8 + c->ns) * N;
  b.B2 = b.B1 + nv * N;
  b.thpart = b.B2 + nv * N;
  return b;
}

// With a tape view the stage's per-cell fields, temperature and sensor flags
// are taken from it; otherwise they are recomputed from U (T is the Newton
// guess cache).
htr_status rhs_adj(htr_ctx* c, const AdjBufs& b, const double* U, double* T, double tk, const htr_laser* laser,
                   const double* dlnA, const double* lam, double s, double h, double* out, double* pbar,
                   hipStream_t st, const TapeView* tv = nullptr) {
  Ctx C{};
  C.ns = c->ns;
  C.M = c->dM;
  C.mem = c->dmem;
  C.nmem = 1;
  C.nblocks = c->nblocks;
  C.scheme = c->scheme;
  CallArgs a{};
  a.t = tk;
  a.use_call_laser = 1;
  a.laser = make_laser(laser, c->n, c->L);
  a.dlnA = dlnA;
  a.flags = c->scheme.flags;
  const double* aux = c->ws.aux;
  const unsigned char* flag = c->ws.flag;
  const unsigned char* bits = nullptr;
  const double* Ts = T;
  if (tv) {
    aux = tv->aux;
    flag = tv->flag;
    bits = tv->bits;
    Ts = tv->T;
  } else {
    HIP_OK(launch_point(C.ns, C.M, C.mem, 1, C.nblocks, 0, a, U, T, c->ws.aux, c->ws.src, nullptr, nullptr, nullptr,
                        c->ws.status, 0, st));
    HIP_OK(launch_sensor(C.mem, 1, C.nblocks, 0, c->ws.aux, C.ns, c->ws.flag, c->ws.grad, C.scheme.theta_c,
                         nullptr, st));
  }
  const int nth = 4 + c->nr;
  HIP_OK(launch_adjoint(C.ns, C.M, C.mem, 1, C.nblocks, c->ntblocks, a, U, Ts, aux, flag, bits, lam, s, h, b.ubd, b.pb,
                        out, b.thpart, nth, C.scheme.psi_c, C.scheme.teno_CT, st));
  HIP_OK(launch_adj_theta(C.mem, 1, b.thpart, nth, pbar, st));
  return HTR_OK;
}

}  // namespace

extern "C" {

size_t htr_adjoint_work_bytes(const htr_ctx* c) {
  if (!c) return 0;
  const size_t nv = c->ns + 4;
  return sizeof(double) * ((3 * nv + 8 + c->ns) * (size_t)c->N + (size_t)c->nblocks * (4 + c->nr));
}

htr_status htr_rhs_adjoint(htr_ctx* c, const double* U, double* T_io, double t, const htr_laser* laser,
                           const double* dlnA_dev, const double* lam, double s, double h, double* Ubar_acc,
                           double* pbar_acc, double* adj_work, void* stream) {
  if (!c) return fail(HTR_EINVAL, "ctx is NULL");
  Marked mk_(&c->fence, stream);
  if (c->scheme.flags & HTR_WENO3Z)
    return fail(HTR_EUNSUPPORTED, "the discrete adjoint is built for the TENO6 scheme (HTR_WENO3Z is set)");
  if (c->curv) return fail(HTR_EUNSUPPORTED, "the discrete adjoint is built for rectilinear grids");
  if (c->host_mem.bounded) return fail(HTR_EUNSUPPORTED, "the discrete adjoint is built for periodic grids");
  if (!U || !T_io || !lam || !Ubar_acc || !pbar_acc || !adj_work) return fail(HTR_EINVAL, "NULL pointer");
  if (Ubar_acc == lam || Ubar_acc == U) return fail(HTR_EINVAL, "Ubar_acc must not alias U or lam");
  if (!std::isfinite(t) || !std::isfinite(s) || !std::isfinite(h)) return fail(HTR_EINVAL, "t, s, h must be finite");
  htr_status st = check_laser(laser);
  if (st) return st;
  htr_laser off{};
  return rhs_adj(c, split(c, adj_work), U, T_io, t, laser ? laser : &off, dlnA_dev, lam, s, h, Ubar_acc, pbar_acc,
                 (hipStream_t)stream);
}

htr_status htr_rk3_step_adjoint(htr_ctx* c, const double* Un, const double* stages, double* T_io, double t,
                                double dt, const htr_laser* laser, const double* dlnA_dev, double Jbar,
                                double* Ubar, double* pbar_acc, double* adj_work, const void* tape, void* stream) {
  if (!c) return fail(HTR_EINVAL, "ctx is NULL");
  Marked mk_(&c->fence, stream);
  if (c->scheme.flags & HTR_WENO3Z)
    return fail(HTR_EUNSUPPORTED, "the discrete adjoint is built for the TENO6 scheme (HTR_WENO3Z is set)");
  if (c->curv) return fail(HTR_EUNSUPPORTED, "the discrete adjoint is built for rectilinear grids");
  if (c->host_mem.bounded) return fail(HTR_EUNSUPPORTED, "the discrete adjoint is built for periodic grids");
  if (!Un || !stages || !T_io || !Ubar || !pbar_acc || !adj_work) return fail(HTR_EINVAL, "NULL pointer");
  if (!std::isfinite(t) || !(dt > 0) || !std::isfinite(Jbar)) return fail(HTR_EINVAL, "need finite t, Jbar and dt > 0");
  htr_status st = check_laser(laser);
  if (st) return st;
  htr_laser off{};
  if (!laser) laser = &off;
  const AdjBufs b = split(c, adj_work);
  const long long n = (long long)(c->ns + 4) * c->N;
  const double* U1 = stages;
  const double* U2 = stages + n;
  hipStream_t s = (hipStream_t)stream;
  const double bq[3] = {1.0 / 6.0, 1.0 / 6.0, 2.0 / 3.0};
  // stage 3: U^{n+1} = 1/3 U^n + 2/3 (U2 + dt L(U2, t + dt/2))
  HIP_OK(launch_axpby(n, 2.0 / 3.0, Ubar, 0.0, b.B2, s));
  TapeView tv[3];
  for (int k = 0; k < 3 && tape; ++k) tv[k] = tape_view(const_cast<void*>(tape), c->ns, c->N, k);
  st = rhs_adj(c, b, U2, T_io, t + 0.5 * dt, laser, dlnA_dev, Ubar, (2.0 / 3.0) * dt, dt * bq[2] * Jbar, b.B2,
               pbar_acc, s, tape ? &tv[2] : nullptr);
  if (st) return st;
  HIP_OK(launch_axpby(n, 1.0 / 3.0, Ubar, 0.0, Ubar, s));
  // stage 2: U2 = 3/4 U^n + 1/4 (U1 + dt L(U1, t + dt))
  HIP_OK(launch_axpby(n, 0.25, b.B2, 0.0, b.B1, s));
  st = rhs_adj(c, b, U1, T_io, t + dt, laser, dlnA_dev, b.B2, 0.25 * dt, dt * bq[1] * Jbar, b.B1, pbar_acc, s,
               tape ? &tv[1] : nullptr);
  if (st) return st;
  HIP_OK(launch_axpby(n, 0.75, b.B2, 1.0, Ubar, s));
  // stage 1: U1 = U^n + dt L(U^n, t)
  HIP_OK(launch_axpby(n, 1.0, b.B1, 1.0, Ubar, s));
  return rhs_adj(c, b, Un, T_io, t, laser, dlnA_dev, b.B1, dt, dt * bq[0] * Jbar, Ubar, pbar_acc, s,
                 tape ? &tv[0] : nullptr);
}

}  // extern "C"
