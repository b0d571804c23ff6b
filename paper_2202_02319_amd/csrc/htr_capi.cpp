// Host side of the C interface: argument validation, the context (device
// tables, member table, scratch), and the kernel sequences of one RHS
// evaluation, the stable step and one SSP-RK3 step.

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "htr.h"
#include "htr_dev.h"
#include "htr_internal.h"

using namespace htr;

static thread_local std::string g_last_error;

namespace htr {
htr_status fail(htr_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return st;
}
}  // namespace htr

namespace htr {

LaserDev make_laser(const htr_laser* L, const int n[3], const double Lp[3]) {
  LaserDev d{};
  if (!L || !L->on) {
    d.on = 0;
    d.st = 1.0;
    d.sr = 1.0;
    return d;
  }
  d.on = 1;
  d.E = L->E;
  for (int a = 0; a < 3; ++a) d.xc[a] = L->center[a];
  d.sr = L->sigma_r;
  d.t0 = L->t0;
  d.st = L->sigma_t;
  int dim = 0;
  for (int a = 0; a < 3; ++a) {
    if (n[a] > 1) ++dim;
    int M = (int)std::ceil(9.103 * L->sigma_r / Lp[a] - 0.5);
    d.M[a] = M < 0 ? 0 : M;
  }
  d.norm = 1.0 / (std::pow(2.0 * PI, 0.5 * (dim + 1)) * std::pow(L->sigma_r, dim) * L->sigma_t);
  return d;
}

htr_status check_laser(const htr_laser* L) {
  if (!L || !L->on) return HTR_OK;
  if (!(L->sigma_r > 0) || !(L->sigma_t > 0) || !std::isfinite(L->E) || !std::isfinite(L->t0))
    return fail(HTR_EINVAL, "laser: sigma_r and sigma_t must be > 0 and E, t0 finite");
  for (int a = 0; a < 3; ++a)
    if (!std::isfinite(L->center[a])) return fail(HTR_EINVAL, "laser: non-finite centre");
  return HTR_OK;
}

htr_status build_tables(const htr_mech_desc* m, MechTables* T) {
  if (!m) return fail(HTR_EINVAL, "mechanism descriptor is NULL");
  if (m->ns < 1) return fail(HTR_EINVAL, "ns must be >= 1 (got %d)", m->ns);
  if (m->ns > MAXNS) return fail(HTR_EUNSUPPORTED, "ns = %d exceeds HTR_MAX_NS = %d", m->ns, MAXNS);
  if (m->nr < 0) return fail(HTR_EINVAL, "nr must be >= 0");
  if (m->nr > MAXNR) return fail(HTR_EUNSUPPORTED, "nr = %d exceeds HTR_MAX_NR = %d", m->nr, MAXNR);
  if (!m->W || !m->nasa7 || !m->lj_sigma || !m->lj_epsk)
    return fail(HTR_EINVAL, "species tables must not be NULL");
  if (m->nr > 0 && (!m->lnA || !m->beta || !m->Ea || !m->nu_f || !m->nu_r))
    return fail(HTR_EINVAL, "reaction tables must not be NULL when nr > 0");
  if (!(m->Tmin > 0) || !(m->Tmax > m->Tmin)) return fail(HTR_EINVAL, "need 0 < Tmin < Tmax");
  std::memset(T, 0, sizeof(*T));
  const int ns = m->ns;
  T->ns = ns;
  T->nr = m->nr;
  T->Tmin = m->Tmin;
  T->Tmax = m->Tmax;
  for (int s = 0; s < ns; ++s) {
    const double W = m->W[s], sg = m->lj_sigma[s], ek = m->lj_epsk[s];
    if (!(W > 0) || !(sg > 0) || !(ek > 0)) return fail(HTR_EINVAL, "species %d: W, sigma, eps must be > 0", s);
    const double* a = m->nasa7 + 7 * s;
    for (int k = 0; k < 7; ++k)
      if (!std::isfinite(a[k])) return fail(HTR_EINVAL, "species %d: non-finite NASA coefficient", s);
    T->W[s] = W;
    T->iW[s] = 1.0 / W;
    T->RW[s] = RU / W;
    for (int k = 0; k < 5; ++k) T->cp[s][k] = a[k];
    T->hc[s][0] = a[0];
    T->hc[s][1] = a[1] / 2.0;
    T->hc[s][2] = a[2] / 3.0;
    T->hc[s][3] = a[3] / 4.0;
    T->hc[s][4] = a[4] / 5.0;
    T->hc[s][5] = a[5];
    T->sc[s][0] = a[0];
    T->sc[s][1] = a[1];
    T->sc[s][2] = a[2] / 2.0;
    T->sc[s][3] = a[3] / 3.0;
    T->sc[s][4] = a[4] / 4.0;
    T->sc[s][5] = a[6];
    const double mass = W / NAV;
    T->mu_pre[s] = (5.0 / 16.0) * std::sqrt(PI * mass * KB) / (PI * sg * sg);
    T->ieps[s] = 1.0 / ek;
    T->lneps[s] = std::log(ek);
    T->pw22[s] = std::pow(ek, 0.14874);
    T->euck[s] = 1.25 * RU / W;
  }
  for (int i = 0; i < ns; ++i)
    for (int j = 0; j < ns; ++j) {
      const double Wi = m->W[i], Wj = m->W[j];
      T->wq[i][j] = std::pow(Wj / Wi, 0.25);
      T->wp[i][j] = 1.0 / std::sqrt(8.0 * (1.0 + Wi / Wj));
      const double mij = 1.0 / (NAV * (1.0 / Wi + 1.0 / Wj));
      const double sg = 0.5 * (m->lj_sigma[i] + m->lj_sigma[j]);
      const double ek = std::sqrt(m->lj_epsk[i] * m->lj_epsk[j]);
      T->Dpre[i][j] = (3.0 / 16.0) * std::sqrt(2.0 * PI * KB * KB * KB / mij) / (PI * sg * sg);
      T->Dieps[i][j] = 1.0 / ek;
      T->Dlneps[i][j] = std::log(ek);
      T->pw11[i][j] = std::pow(ek, 0.15610);
      T->iDpre[i][j] = 1.0 / T->Dpre[i][j];
    }
  for (int j = 0; j < m->nr; ++j) {
    if (!std::isfinite(m->lnA[j]) || !std::isfinite(m->beta[j]) || !std::isfinite(m->Ea[j]))
      return fail(HTR_EINVAL, "reaction %d: non-finite Arrhenius parameter", j);
    T->lnA[j] = m->lnA[j];
    T->beta[j] = m->beta[j];
    T->EaR[j] = m->Ea[j] / RU;
    int dnu = 0, nre = 0, npr = 0;
    for (int s = 0; s < ns; ++s) {
      const int f = m->nu_f[j * ns + s], r = m->nu_r[j * ns + s];
      if (f < 0 || r < 0 || f > 3 || r > 3)
        return fail(HTR_EINVAL, "reaction %d: stoichiometric coefficients must be in 0..3", j);
      T->nunet[j][s] = (double)(r - f);
      dnu += r - f;
      if (f > 0) {
        if (nre == SIDE) return fail(HTR_EUNSUPPORTED, "reaction %d: more than %d reactant species", j, SIDE);
        T->ridx[j][nre] = s;
        T->rnu[j][nre++] = f;
      }
      if (r > 0) {
        if (npr == SIDE) return fail(HTR_EUNSUPPORTED, "reaction %d: more than %d product species", j, SIDE);
        T->pidx[j][npr] = s;
        T->pnu[j][npr++] = r;
      }
    }
    if (nre == 0 || npr == 0) return fail(HTR_EINVAL, "reaction %d: empty side", j);
    T->nre[j] = nre;
    T->npr[j] = npr;
    T->dnu[j] = (double)dnu;
  }
  return HTR_OK;
}

}  // namespace htr

namespace htr {

htr_status ws_alloc(Workspace& w, int ns, long long N, int nblocks, int nmem) {
  const int naux = 7 + ns;
  w.ns = ns;
  w.N = N;
  hipError_t e = hipSuccess;
  if ((e = hipMalloc(&w.aux, sizeof(double) * naux * N)) != hipSuccess ||
      (e = hipMalloc(&w.src, sizeof(double) * (ns + 1) * N)) != hipSuccess ||
      (e = hipMalloc(&w.flag, (size_t)N)) != hipSuccess ||
      (e = hipMalloc(&w.grad, sizeof(double) * 9 * N)) != hipSuccess ||
      (e = hipMalloc(&w.part, sizeof(double) * (ns + 4) * N)) != hipSuccess ||
      (e = hipMalloc(&w.tcls, (size_t)N)) != hipSuccess ||
      (e = hipMalloc(&w.blkred, sizeof(double) * 2 * (size_t)nblocks)) != hipSuccess ||
      (e = hipMalloc(&w.status, sizeof(unsigned))) != hipSuccess ||
      (e = hipMalloc(&w.scal, sizeof(double) * 2 * (size_t)nmem)) != hipSuccess)
    return fail(e == hipErrorOutOfMemory ? HTR_ENOMEM : HTR_EDEVICE, "workspace allocation: %s",
                hipGetErrorString(e));
  if ((e = hipMemset(w.status, 0, sizeof(unsigned))) != hipSuccess)
    return fail(HTR_EDEVICE, "hipMemset: %s", hipGetErrorString(e));
  return HTR_OK;
}

void ws_free(Workspace& w) {
  hipFree(w.aux);
  hipFree(w.src);
  hipFree(w.flag);
  hipFree(w.grad);
  hipFree(w.part);
  hipFree(w.tcls);
  hipFree(w.blkred);
  hipFree(w.status);
  hipFree(w.scal);
  w = Workspace{};
}

void Fence::mark(hipStream_t s) {
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(s, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone) return;
  for (auto& p : ev)
    if (p.first == s) {
      hipEventRecord(p.second, s);
      return;
    }
  hipEvent_t e = nullptr;
  if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) return;
  hipEventRecord(e, s);
  ev.emplace_back(s, e);
}
hipError_t Fence::wait() {
  hipError_t r = hipSuccess;
  for (auto& p : ev) {
    hipError_t e = hipEventSynchronize(p.second);
    if (e != hipSuccess && r == hipSuccess) r = e;
  }
  return r;
}
Fence::~Fence() {
  for (auto& p : ev) hipEventDestroy(p.second);
}

hipEvent_t Timer::get() {
  if (!pool.empty()) {
    hipEvent_t e = pool.back();
    pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}
void Timer::clear() {
  for (auto& r : recs) {
    hipEventSynchronize(r.b);   // the pair may still be pending on its stream
    pool.push_back(r.a);
    pool.push_back(r.b);
  }
  recs.clear();
}
Timer::~Timer() {
  clear();
  for (auto e : pool) hipEventDestroy(e);
}
TimedLaunch::TimedLaunch(Timer* t_, int cls_, hipStream_t s_) : t(t_), cls(cls_), s(s_) {
  if (t && t->on) {
    a = t->get();
    if (a) hipEventRecord(a, s);
  }
}
TimedLaunch::~TimedLaunch() {
  if (a) {
    hipEvent_t b = t->get();
    if (b) {
      hipEventRecord(b, s);
      t->recs.push_back({cls, a, b});
    } else {
      t->pool.push_back(a);
    }
  }
}

// One RHS evaluation at stage time t + tcoef*dt: point -> [reduce] -> sensor -> sweep.
// want_dt: the per-cell kernel also reduces the stable step and writes dt_dev.
htr_status stage(const Ctx& C, const Workspace& w, const CallArgs& a, const double* U, const double* Un,
                 double* T, double* out, double ca, double cb, int rhs_only, double* hrr, double* J_dev,
                 double jcoef, hipStream_t s, int want_dt, double* dt_out, unsigned char* teno_bits) {
  const bool need_red = J_dev != nullptr || want_dt;
  {
    TimedLaunch tl(C.timer, TC_POINT, s);
    HIP_OK(launch_point(C.ns, C.M, C.mem, C.nmem, C.nblocks, C.grid, a, U, T, w.aux, w.src, hrr,
                        need_red ? w.blkred : nullptr, nullptr, w.status, want_dt, s, C.curv));
  }
  if (need_red) {
    TimedLaunch tl(C.timer, TC_REDUCE, s);
    HIP_OK(launch_finalize(C.mem, C.nmem, w.blkred, C.scheme.cfl, dt_out, J_dev, a.dt_dev, jcoef, want_dt, s));
  }
  if (C.curv) {
    // curvilinear grid: mapped fluxes through per-face kernels, then the update
    if (teno_bits) return fail(HTR_EUNSUPPORTED, "no tape on curvilinear grids");
    {
      TimedLaunch tl(C.timer, TC_SENSOR, s);
      HIP_OK(launch_curv_igrad(C.ns, C.M, C.mem, C.nblocks, U, T, w.aux, C.cX, C.cdphi, s));
      HIP_OK(launch_curv_sensor(C.mem, C.nblocks, *C.curv, w.aux, C.ns, w.flag, C.scheme.theta_c, nullptr, s));
    }
    {
      TimedLaunch tl(C.timer, TC_CONV, s);
      HIP_OK(launch_curv_conv(C.ns, *C.host1, C.mem, *C.curv, a, U, w.aux, w.flag, C.cffc, C.scheme.psi_c,
                              C.scheme.teno_CT, s));
    }
    if (!(a.flags & HTR_VISC_OFF)) {
      TimedLaunch tl(C.timer, TC_DIFF, s);
      HIP_OK(launch_curv_diff(C.ns, C.M, C.mem, C.nblocks, *C.curv, U, T, w.aux, C.cX, C.cdphi, C.cffd, s));
    }
    {
      TimedLaunch tl(C.timer, TC_UPDATE, s);
      HIP_OK(launch_curv_update(C.ns, C.mem, C.nblocks, *C.curv, a, U, Un, w.src, C.cffc, C.cffd, out, ca, cb,
                                rhs_only, s));
    }
    return HTR_OK;
  }
  {
    TimedLaunch tl(C.timer, TC_SENSOR, s);
    HIP_OK(launch_sensor(C.mem, C.nmem, C.nblocks, C.grid, w.aux, C.ns, w.flag, w.grad, C.scheme.theta_c, nullptr,
                         s));
  }
  {
    TimedLaunch tl(C.timer, TC_CONV, s);
    HIP_OK(launch_conv(C.ns, C.M, C.mem, C.nmem, C.ntblocks, C.grid, a, U, w.aux, w.src, w.flag, w.part, teno_bits,
                       C.scheme.psi_c, C.scheme.teno_CT, C.conv_split ? w.tcls : nullptr, s));
  }
  if (C.bounded) {
    // the cells next to non-periodic boundaries: their whole right-hand side
    if (teno_bits) return fail(HTR_EUNSUPPORTED, "no tape on a grid with non-periodic boundaries");
    TimedLaunch tl(C.timer, TC_UPDATE, s);
    HIP_OK(launch_bnd(C.ns, C.M, C.mem, C.nblocks, a, U, T, w.aux, w.src, w.flag, w.grad, w.part, C.scheme.psi_c,
                      C.scheme.teno_CT, s));
  }
  {
    TimedLaunch tl(C.timer, TC_DIFF, s);
    HIP_OK(launch_diff(C.ns, C.M, C.mem, C.nmem, C.ndtblocks, C.grid, a, U, Un, T, w.aux, w.grad, w.part, out, ca,
                       cb,
                       rhs_only, s));
  }
  return HTR_OK;
}

htr_status rk3(const Ctx& C, const Workspace& w, double* U, double* T, double* t_dev, double* dt_dev,
               int compute_dt, const htr_laser* laser, const double* dlnA, double* work, double* J_dev,
               hipStream_t s, void* tape) {
  const long long tot = C.total_cells;
  double* U1 = work;
  double* U2 = work + (long long)(C.ns + 4) * tot;
  CallArgs a{};
  a.t = 0.0;
  a.t_dev = t_dev;
  a.dt_dev = dt_dev;
  a.use_call_laser = laser != nullptr;
  if (laser) a.laser = make_laser(laser, C.n1, C.L1);
  a.dlnA = dlnA;
  a.flags = C.scheme.flags;
  const double tc[3] = {0.0, 1.0, 0.5};
  const double bq[3] = {1.0 / 6.0, 1.0 / 6.0, 2.0 / 3.0};
  const double ca[3] = {0.0, 0.75, 1.0 / 3.0}, cb[3] = {1.0, 0.25, 2.0 / 3.0};
  const double* in[3] = {U, U1, U2};
  double* out[3] = {U1, U2, U};
  for (int k = 0; k < 3; ++k) {
    a.tcoef = tc[k];
    TapeView tv{};
    if (tape) tv = tape_view(tape, C.ns, tot, k);
    htr_status st = stage(C, w, a, in[k], U, T, out[k], ca[k], cb[k], 0, nullptr, J_dev, bq[k], s,
                          k == 0 && compute_dt, dt_dev, tape ? tv.bits : nullptr);
    if (st) return st;
    if (tape) {
      // the stage's per-cell fields, temperature and sensor flags, as its sweeps used them
      HIP_OK(hipMemcpyAsync(tv.aux, w.aux, sizeof(double) * (7 + C.ns) * tot, hipMemcpyDeviceToDevice, s));
      HIP_OK(hipMemcpyAsync(tv.T, T, sizeof(double) * tot, hipMemcpyDeviceToDevice, s));
      HIP_OK(hipMemcpyAsync(tv.flag, w.flag, tot, hipMemcpyDeviceToDevice, s));
    }
  }
  TimedLaunch tl(C.timer, TC_REDUCE, s);
  HIP_OK(launch_advance_time(C.nmem, t_dev, dt_dev, s));
  return HTR_OK;
}

}  // namespace htr

Ctx htr::view(const htr_ctx* c) {
  Ctx v{};
  v.ns = c->ns;
  v.M = c->dM;
  v.mem = c->dmem;
  v.nmem = 1;
  v.nblocks = c->nblocks;
  v.ntblocks = c->ntblocks;
  v.ndtblocks = c->ndtblocks;
  v.grid = c->grid;
  v.conv_split = c->conv_split;
  v.scheme = c->scheme;
  v.total_cells = c->N;
  for (int a = 0; a < 3; ++a) {
    v.n1[a] = c->n[a];
    v.L1[a] = c->L[a];
  }
  v.timer = const_cast<Timer*>(&c->timer);
  v.bounded = c->host_mem.bounded != 0;
  if (c->curv) {
    const long long N = c->N;
    v.curv = &c->cg;
    v.host1 = &c->host_mem;
    v.cX = c->dcw;
    v.cdphi = c->dcw + (long long)c->ns * N;
    v.cffc = v.cdphi + 3LL * (4 + c->ns) * N;
    v.cffd = v.cffc + 3LL * (c->ns + 4) * N;
  }
  return v;
}

extern "C" {

const char* htr_last_error(void) { return g_last_error.c_str(); }

int64_t htr_num_cells(const htr_ctx* ctx) { return ctx ? ctx->N : 0; }

htr_status htr_create(const htr_mech_desc* mech, const htr_grid_desc* grid, const htr_scheme* scheme,
                      htr_ctx** out) {
  if (!out) return fail(HTR_EINVAL, "out is NULL");
  *out = nullptr;
  if (!grid || !scheme) return fail(HTR_EINVAL, "grid or scheme descriptor is NULL");
  MechTables T;
  htr_status st = build_tables(mech, &T);
  if (st) return st;
  long long N = 1;
  for (int a = 0; a < 3; ++a) {
    if (grid->n[a] < 1) return fail(HTR_EINVAL, "grid n[%d] = %d must be >= 1", a, grid->n[a]);
    if (!grid->xnode[a] || !grid->xi_node[a] || !grid->xi_face[a])
      return fail(HTR_EINVAL, "grid arrays of axis %d must not be NULL", a);
    if (!(grid->L[a] > 0)) return fail(HTR_EINVAL, "grid period L[%d] must be > 0", a);
    for (int i = 0; i < grid->n[a]; ++i)
      if (!(grid->xi_node[a][i] > 0) || !(grid->xi_face[a][i] > 0) || !std::isfinite(grid->xnode[a][i]))
        return fail(HTR_EINVAL, "grid metric of axis %d must be positive and finite", a);
    N *= grid->n[a];
  }
  if (N > ((long long)1 << 31) * BLK) return fail(HTR_EUNSUPPORTED, "grid too large");
  if (!(scheme->cfl > 0) || !(scheme->teno_CT > 0) || !(scheme->teno_CT < 1) || !(scheme->theta_c >= 0) ||
      !(scheme->psi_c >= 0))
    return fail(HTR_EINVAL, "scheme: need cfl > 0, 0 < teno_CT < 1, theta_c >= 0, psi_c >= 0");
  if ((scheme->flags & HTR_FORCE_CENTRAL) && (scheme->flags & HTR_FORCE_TENO))
    return fail(HTR_EINVAL, "scheme: FORCE_CENTRAL and FORCE_TENO are exclusive");

  htr_ctx* c = new htr_ctx();
  HIP_OK(hipGetDevice(&c->device));
  c->ns = T.ns;
  c->nr = T.nr;
  c->scheme = *scheme;
  c->N = N;
  c->nblocks = (int)((N + BLK - 1) / BLK);
  for (int a = 0; a < 3; ++a) {
    c->n[a] = grid->n[a];
    c->L[a] = grid->L[a];
  }
  auto bail = [&](htr_status s2) {
    htr_destroy(c);
    return s2;
  };
  hipError_t e;
  if ((e = hipMalloc(&c->dM, sizeof(MechTables))) != hipSuccess)
    return bail(fail(HTR_ENOMEM, "hipMalloc tables: %s", hipGetErrorString(e)));
  if ((e = hipMemcpy(c->dM, &T, sizeof(MechTables), hipMemcpyHostToDevice)) != hipSuccess)
    return bail(fail(HTR_EDEVICE, "hipMemcpy tables: %s", hipGetErrorString(e)));
  const long long ng = 3LL * (grid->n[0] + grid->n[1] + grid->n[2]);
  if ((e = hipMalloc(&c->dgrid, sizeof(double) * ng)) != hipSuccess)
    return bail(fail(HTR_ENOMEM, "hipMalloc grid: %s", hipGetErrorString(e)));
  std::vector<double> hg;
  hg.reserve(ng);
  Member& M = c->host_mem;
  std::memset(&M, 0, sizeof(M));
  long long off = 0;
  for (int a = 0; a < 3; ++a) {
    const int na = grid->n[a];
    hg.insert(hg.end(), grid->xi_node[a], grid->xi_node[a] + na);
    hg.insert(hg.end(), grid->xi_face[a], grid->xi_face[a] + na);
    hg.insert(hg.end(), grid->xnode[a], grid->xnode[a] + na);
    M.xin[a] = c->dgrid + off;
    M.xif[a] = c->dgrid + off + na;
    M.xnode[a] = c->dgrid + off + 2 * na;
    off += 3 * na;
    M.n[a] = na;
    M.act[a] = na > 1;
    M.L[a] = grid->L[a];
  }
  if ((e = hipMemcpy(c->dgrid, hg.data(), sizeof(double) * ng, hipMemcpyHostToDevice)) != hipSuccess)
    return bail(fail(HTR_EDEVICE, "hipMemcpy grid: %s", hipGetErrorString(e)));
  M.N = N;
  M.off = 0;
  M.block_begin = 0;
  M.nblocks = c->nblocks;
  set_tiles(M, nullptr, &c->ntblocks, &c->ndtblocks);
  M.laser.on = 0;
  M.dlnA = nullptr;
  if ((e = hipMalloc(&c->dmem, sizeof(Member))) != hipSuccess)
    return bail(fail(HTR_ENOMEM, "hipMalloc member: %s", hipGetErrorString(e)));
  if ((e = hipMemcpy(c->dmem, &M, sizeof(Member), hipMemcpyHostToDevice)) != hipSuccess)
    return bail(fail(HTR_EDEVICE, "hipMemcpy member: %s", hipGetErrorString(e)));
  st = ws_alloc(c->ws, c->ns, N, c->nblocks, 1);
  if (st) return bail(st);
  st = noalloc_init(c->device);
  if (st) return bail(st);
  *out = c;
  return HTR_OK;
}

htr_status htr_create_curvilinear(const htr_mech_desc* mech, const htr_curv_grid_desc* grid,
                                  const htr_scheme* scheme, htr_ctx** out) {
  if (!out) return fail(HTR_EINVAL, "out is NULL");
  *out = nullptr;
  if (!grid || !grid->xyz) return fail(HTR_EINVAL, "grid descriptor or its coordinates are NULL");
  long long N = 1;
  for (int a = 0; a < 3; ++a) {
    if (grid->n[a] < 1) return fail(HTR_EINVAL, "grid n[%d] = %d must be >= 1", a, grid->n[a]);
    N *= grid->n[a];
  }
  for (long long q = 0; q < 3 * N; ++q)
    if (!std::isfinite(grid->xyz[q])) return fail(HTR_EINVAL, "grid coordinates must be finite");
  double P[3][3];
  for (int a = 0; a < 3; ++a)
    for (int c = 0; c < 3; ++c) {
      P[a][c] = grid->period[a][c];
      if (!std::isfinite(P[a][c])) return fail(HTR_EINVAL, "grid periods must be finite");
    }
  for (int a = 0; a < 3; ++a) {
    if (grid->n[a] > 1) continue;
    for (int c = 0; c < 3; ++c)
      if (c != a && P[a][c] != 0.0)
        return fail(HTR_EINVAL, "the period of inactive axis %d must lie along coordinate %d", a, a);
    for (int b = 0; b < 3; ++b)
      if (b != a && P[b][a] != 0.0)
        return fail(HTR_EINVAL, "period %d must have no component along inactive axis %d", b, a);
    if (!(P[a][a] != 0.0)) return fail(HTR_EINVAL, "the period of inactive axis %d is zero", a);
  }
  // B: columns P[a]; its inverse by cofactors
  double B[3][3];
  for (int r = 0; r < 3; ++r)
    for (int a = 0; a < 3; ++a) B[r][a] = P[a][r];
  const double det = B[0][0] * (B[1][1] * B[2][2] - B[1][2] * B[2][1]) -
                     B[0][1] * (B[1][0] * B[2][2] - B[1][2] * B[2][0]) +
                     B[0][2] * (B[1][0] * B[2][1] - B[1][1] * B[2][0]);
  if (!(std::fabs(det) > 0)) return fail(HTR_EINVAL, "the lattice periods are linearly dependent");
  CurvGeom g{};
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c) {
      const int r1 = (c + 1) % 3, r2 = (c + 2) % 3, c1 = (r + 1) % 3, c2 = (r + 2) % 3;
      g.Pinv[r][c] = (B[r1][c1] * B[r2][c2] - B[r1][c2] * B[r2][c1]) / det;
      g.P[r][c] = P[r][c];
    }
  // distances between lattice planes (laser image counts), the period itself on an inactive axis
  double h[3];
  for (int a = 0; a < 3; ++a) {
    const double* u = P[(a + 1) % 3];
    const double* w = P[(a + 2) % 3];
    const double cr[3] = {u[1] * w[2] - u[2] * w[1], u[2] * w[0] - u[0] * w[2], u[0] * w[1] - u[1] * w[0]};
    h[a] = grid->n[a] > 1 ? std::fabs(det) / std::sqrt(cr[0] * cr[0] + cr[1] * cr[1] + cr[2] * cr[2])
                          : std::fabs(P[a][a]);
  }
  // the rectilinear arrays of the context are placeholders (unused on this grid)
  std::vector<double> xn[3], one[3];
  htr_grid_desc rd{};
  for (int a = 0; a < 3; ++a) {
    xn[a].assign(grid->n[a], 0.0);
    one[a].assign(grid->n[a], 1.0);
    rd.n[a] = grid->n[a];
    rd.xnode[a] = xn[a].data();
    rd.xi_node[a] = one[a].data();
    rd.xi_face[a] = one[a].data();
    rd.L[a] = h[a];
  }
  htr_ctx* c = nullptr;
  htr_status st = htr_create(mech, &rd, scheme, &c);
  if (st) return st;
  auto bail = [&](htr_status s2) {
    htr_destroy(c);
    return s2;
  };
  hipError_t e;
  if ((e = hipMalloc(&c->dcurv, sizeof(double) * 22 * N)) != hipSuccess)
    return bail(fail(HTR_ENOMEM, "hipMalloc metrics: %s", hipGetErrorString(e)));
  const long long nw = (long long)c->ns + 3LL * (4 + c->ns) + 6LL * (c->ns + 4);
  if ((e = hipMalloc(&c->dcw, sizeof(double) * nw * N)) != hipSuccess)
    return bail(fail(HTR_ENOMEM, "hipMalloc curvilinear scratch: %s", hipGetErrorString(e)));
  double* mt = c->dcurv;
  double* mf = c->dcurv + 10 * N;
  double* xyz = c->dcurv + 19 * N;
  if ((e = hipMemcpy(xyz, grid->xyz, sizeof(double) * 3 * N, hipMemcpyHostToDevice)) != hipSuccess)
    return bail(fail(HTR_EDEVICE, "hipMemcpy coordinates: %s", hipGetErrorString(e)));
  g.mt = mt;
  g.mf = mf;
  g.xyz = xyz;
  if ((e = launch_curv_metrics(c->dmem, c->host_mem, g, mt, mf, nullptr)) != hipSuccess)
    return bail(fail(HTR_EDEVICE, "metric kernels: %s", hipGetErrorString(e)));
  std::vector<double> J(N);
  if ((e = hipMemcpy(J.data(), mt + 9 * N, sizeof(double) * N, hipMemcpyDeviceToHost)) != hipSuccess)
    return bail(fail(HTR_EDEVICE, "hipMemcpy J: %s", hipGetErrorString(e)));
  for (long long q = 0; q < N; ++q)
    if (!(J[q] > 0) || !std::isfinite(J[q]))
      return bail(fail(HTR_EINVAL, "det(d x / d xi) is not positive at node %lld", q));
  c->curv = true;
  c->cg = g;
  *out = c;
  return HTR_OK;
}

htr_status htr_grid_metrics(htr_ctx* c, double* mt, double* mf, void* stream) {
  if (!c) return fail(HTR_EINVAL, "ctx is NULL");
  Marked mk_(&c->fence, stream);
  if (!c->curv) return fail(HTR_EINVAL, "not a curvilinear context");
  if (!mt || !mf) return fail(HTR_EINVAL, "NULL pointer");
  hipStream_t s = (hipStream_t)stream;
  HIP_OK(hipMemcpyAsync(mt, c->cg.mt, sizeof(double) * 10 * c->N, hipMemcpyDeviceToDevice, s));
  HIP_OK(hipMemcpyAsync(mf, c->cg.mf, sizeof(double) * 9 * c->N, hipMemcpyDeviceToDevice, s));
  return HTR_OK;
}

htr_status htr_destroy(htr_ctx* c) {
  if (!c) return fail(HTR_EINVAL, "ctx is NULL");
  c->fence.wait();   // this context's own work, on every stream it was given
  hipFree(c->dM);
  hipFree(c->dgrid);
  hipFree(c->dmem);
  hipFree(c->dcurv);
  hipFree(c->dcw);
  ws_free(c->ws);
  delete c;
  return HTR_OK;
}

htr_status htr_set_boundaries(htr_ctx* c, const int32_t bc[3][2], const double pinf[3][2],
                              const double relax[3][2]) {
  if (!c || !bc || !pinf || !relax) return fail(HTR_EINVAL, "NULL argument");
  if (c->curv) return fail(HTR_EUNSUPPORTED, "non-periodic boundaries are for rectilinear grids");
  Member M = c->host_mem;
  M.bounded = 0;
  for (int a = 0; a < 3; ++a) {
    const int lo = bc[a][0], hi = bc[a][1];
    if (lo < HTR_BC_PERIODIC || lo > HTR_BC_OUTFLOW || hi < HTR_BC_PERIODIC || hi > HTR_BC_OUTFLOW)
      return fail(HTR_EINVAL, "axis %d: unknown boundary type", a);
    if ((lo == HTR_BC_PERIODIC) != (hi == HTR_BC_PERIODIC))
      return fail(HTR_EINVAL, "axis %d: periodic on one side only", a);
    if (lo != HTR_BC_PERIODIC && c->n[a] < 8) return fail(HTR_EINVAL, "axis %d: a bounded axis needs n >= 8", a);
    for (int side = 0; side < 2; ++side) {
      if (bc[a][side] == HTR_BC_OUTFLOW && !(pinf[a][side] > 0 && relax[a][side] >= 0 && std::isfinite(relax[a][side])))
        return fail(HTR_EINVAL, "axis %d side %d: outflow needs p_inf > 0 and relax >= 0", a, side);
      M.bc[a][side] = bc[a][side];
      M.pinf[a][side] = pinf[a][side];
      M.relax[a][side] = relax[a][side];
    }
    if (lo != HTR_BC_PERIODIC) M.bounded = 1;
  }
  Marked mk_(&c->fence, nullptr);
  HIP_OK(hipMemcpy(c->dmem, &M, sizeof(Member), hipMemcpyHostToDevice));
  c->host_mem = M;
  return HTR_OK;
}

htr_status htr_set_flags(htr_ctx* c, uint32_t flags) {
  if (!c) return fail(HTR_EINVAL, "ctx is NULL");
  if ((flags & HTR_FORCE_CENTRAL) && (flags & HTR_FORCE_TENO))
    return fail(HTR_EINVAL, "FORCE_CENTRAL and FORCE_TENO are exclusive");
  c->scheme.flags = flags;
  return HTR_OK;
}

htr_status htr_prim_to_cons(htr_ctx* c, const double* Y, const double* T, const double* p, const double* vel,
                            double* U, void* stream) {
  if (!c) return fail(HTR_EINVAL, "ctx is NULL");
  Marked mk_(&c->fence, stream);
  if (!Y || !T || !p || !vel || !U) return fail(HTR_EINVAL, "NULL field pointer");
  Ctx C = view(c);
  HIP_OK(launch_prim_to_cons(C.ns, C.M, C.mem, C.nmem, C.nblocks, Y, T, p, vel, U, (hipStream_t)stream));
  return HTR_OK;
}

htr_status htr_rhs(htr_ctx* c, const double* U, double* T_io, double t, const htr_laser* laser, double* dUdt,
                   double* hrr, void* stream) {
  if (!c) return fail(HTR_EINVAL, "ctx is NULL");
  Marked mk_(&c->fence, stream);
  if (!U || !T_io || !dUdt) return fail(HTR_EINVAL, "NULL field pointer");
  if (U == dUdt) return fail(HTR_EINVAL, "dUdt must not alias U");
  if (!std::isfinite(t)) return fail(HTR_EINVAL, "t must be finite");
  htr_status st = check_laser(laser);
  if (st) return st;
  Ctx C = view(c);
  CallArgs a{};
  a.t = t;
  a.use_call_laser = 1;
  a.laser = make_laser(laser, C.n1, C.L1);
  a.flags = c->scheme.flags;
  return stage(C, c->ws, a, U, U, T_io, dUdt, 0.0, 1.0, 1, hrr, nullptr, 0.0, (hipStream_t)stream, 0, nullptr);
}

htr_status htr_cells(htr_ctx* c, const double* U, double* T_io, double t, const htr_laser* laser, double* out,
                     void* stream) {
  if (!c) return fail(HTR_EINVAL, "ctx is NULL");
  Marked mk_(&c->fence, stream);
  if (!U || !T_io || !out) return fail(HTR_EINVAL, "NULL field pointer");
  htr_status st = check_laser(laser);
  if (st) return st;
  Ctx C = view(c);
  CallArgs a{};
  a.t = t;
  a.use_call_laser = 1;
  a.laser = make_laser(laser, C.n1, C.L1);
  a.flags = c->scheme.flags;
  hipStream_t s = (hipStream_t)stream;
  HIP_OK(launch_point(C.ns, C.M, C.mem, 1, C.nblocks, 0, a, U, T_io, c->ws.aux, c->ws.src, nullptr, nullptr, out,
                      c->ws.status, 0, s, C.curv));
  if (C.curv)
    HIP_OK(launch_curv_sensor(C.mem, C.nblocks, *C.curv, c->ws.aux, C.ns, c->ws.flag, C.scheme.theta_c, out, s));
  else
    HIP_OK(launch_sensor(C.mem, 1, C.nblocks, 0, c->ws.aux, C.ns, c->ws.flag, c->ws.grad, C.scheme.theta_c, out, s));
  return HTR_OK;
}

htr_status htr_stable_dt(htr_ctx* c, const double* U, double* T_io, double* dt_dev, void* stream) {
  if (!c) return fail(HTR_EINVAL, "ctx is NULL");
  Marked mk_(&c->fence, stream);
  if (!U || !T_io || !dt_dev) return fail(HTR_EINVAL, "NULL pointer");
  Ctx C = view(c);
  CallArgs a{};
  a.flags = c->scheme.flags | HTR_CHEM_OFF;   // the step limit needs no chemistry
  hipStream_t s = (hipStream_t)stream;
  HIP_OK(launch_point(C.ns, C.M, C.mem, 1, C.nblocks, 0, a, U, T_io, c->ws.aux, c->ws.src, nullptr, c->ws.blkred,
                      nullptr, c->ws.status, 1, s, C.curv));
  HIP_OK(launch_finalize(C.mem, 1, c->ws.blkred, c->scheme.cfl, dt_dev, nullptr, nullptr, 0.0, 1, s));
  return HTR_OK;
}

size_t htr_work_bytes(const htr_ctx* c) { return c ? sizeof(double) * 2 * (size_t)(c->ns + 4) * c->N : 0; }

htr_status htr_rk3_step(htr_ctx* c, double* U, double* T_io, double* t_dev, double* dt_dev, int compute_dt,
                        const htr_laser* laser, const double* dlnA_dev, double* work, double* J_dev,
                        void* stream) {
  if (!c) return fail(HTR_EINVAL, "ctx is NULL");
  Marked mk_(&c->fence, stream);
  if (!U || !T_io || !t_dev || !dt_dev || !work) return fail(HTR_EINVAL, "NULL pointer");
  if (work == U || work == T_io) return fail(HTR_EINVAL, "work must not alias U or T_io");
  htr_status st = check_laser(laser);
  if (st) return st;
  Ctx C = view(c);
  htr_laser off{};
  return rk3(C, c->ws, U, T_io, t_dev, dt_dev, compute_dt, laser ? laser : &off, dlnA_dev, work, J_dev,
             (hipStream_t)stream, nullptr);
}

size_t htr_tape_bytes(const htr_ctx* c) {
  if (!c) return 0;
  return tape_bytes(c->ns, c->N);
}

htr_status htr_rk3_step_taped(htr_ctx* c, double* U, double* T_io, double* t_dev, double* dt_dev, int compute_dt,
                              const htr_laser* laser, const double* dlnA_dev, double* work, double* J_dev,
                              void* tape, void* stream) {
  if (!c) return fail(HTR_EINVAL, "ctx is NULL");
  Marked mk_(&c->fence, stream);
  if (!U || !T_io || !t_dev || !dt_dev || !work || !tape) return fail(HTR_EINVAL, "NULL pointer");
  if (work == U || work == T_io) return fail(HTR_EINVAL, "work must not alias U or T_io");
  if (c->curv) return fail(HTR_EUNSUPPORTED, "the taped step (adjoint) is for rectilinear grids");
  if (c->host_mem.bounded) return fail(HTR_EUNSUPPORTED, "the taped step (adjoint) is for periodic grids");
  if (c->N >= (1LL << 31)) return fail(HTR_EUNSUPPORTED, "the tape indexes cells with 32 bits: N must be < 2^31");
  htr_status st = check_laser(laser);
  if (st) return st;
  Ctx C = view(c);
  htr_laser off{};
  return rk3(C, c->ws, U, T_io, t_dev, dt_dev, compute_dt, laser ? laser : &off, dlnA_dev, work, J_dev,
             (hipStream_t)stream, tape);
}

htr_status htr_timing(htr_ctx* c, int enable) {
  if (!c) return fail(HTR_EINVAL, "ctx is NULL");
  c->timer.clear();   // waits for each recorded launch's closing event
  c->timer.on = enable != 0;
  return HTR_OK;
}

htr_status htr_timing_read(htr_ctx* c, double* ms, int64_t* launches) {
  if (!c || !ms || !launches) return fail(HTR_EINVAL, "NULL pointer");
  for (int k = 0; k < HTR_TIMING_CLASSES; ++k) {
    ms[k] = 0.0;
    launches[k] = 0;
  }
  for (auto& r : c->timer.recs) {
    HIP_OK(hipEventSynchronize(r.b));
    float e = 0.0f;
    HIP_OK(hipEventElapsedTime(&e, r.a, r.b));
    ms[r.cls] += e;
    launches[r.cls] += 1;
  }
  return HTR_OK;
}

htr_status htr_check(htr_ctx* c, void* stream) {
  if (!c) return fail(HTR_EINVAL, "ctx is NULL");
  HIP_OK(hipStreamSynchronize((hipStream_t)stream));
  unsigned st = 0;
  HIP_OK(hipMemcpy(&st, c->ws.status, sizeof st, hipMemcpyDeviceToHost));
  HIP_OK(hipMemset(c->ws.status, 0, sizeof(unsigned)));
  if (st & ST_NONFINITE) return fail(HTR_ENONFINITE, "non-finite state or rho <= 0 met on the device");
  if (st & ST_NEWTON) return fail(HTR_ENEWTON, "temperature Newton iteration did not converge");
  if (st & ST_TRANGE) return fail(HTR_ETRANGE, "temperature outside [Tmin, Tmax]");
  return HTR_OK;
}

}  // extern "C"
