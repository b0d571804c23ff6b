// Ensembles: many independent member grids advanced together.  Every kernel
// of a batched call is one launch over the tiles of all members (each block
// finds its member in the device member table); the members' cells are
// packed member-major.  Many steps can be captured into one HIP graph.

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <vector>

#include "htr.h"
#include "htr_dev.h"
#include "htr_internal.h"

using namespace htr;

Ctx htr::bview(const htr_batch* b) {
  Ctx v{};
  v.ns = b->ctx->ns;
  v.M = b->ctx->dM;
  v.mem = b->dmem;
  v.nmem = b->nmem;
  v.nblocks = b->nblocks;
  v.ntblocks = b->ntblocks;
  v.ndtblocks = b->ndtblocks;
  v.grid = b->grid;
  v.conv_split = b->conv_split;
  v.scheme = b->ctx->scheme;
  v.total_cells = b->Ntot;
  v.timer = const_cast<Timer*>(&b->timer);
  return v;
}

void htr::drop_graph(htr_batch* b) {
  if (b->exec) hipGraphExecDestroy(b->exec);
  if (b->graph) hipGraphDestroy(b->graph);
  b->exec = nullptr;
  b->graph = nullptr;
  b->key_steps = -1;
}

extern "C" {

htr_status htr_batch_create(htr_ctx* ctx, int32_t nmem, const htr_member_desc* mds, htr_batch** out) {
  if (!out) return fail(HTR_EINVAL, "out is NULL");
  *out = nullptr;
  if (!ctx || !mds) return fail(HTR_EINVAL, "ctx or members is NULL");
  if (nmem < 1) return fail(HTR_EINVAL, "nmem must be >= 1");
  if (ctx->host_mem.bounded) return fail(HTR_EUNSUPPORTED, "ensembles are built on periodic grids");
  const int nr = ctx->nr;
  htr_batch* b = new htr_batch();
  b->ctx = ctx;
  b->nmem = nmem;
  b->host.resize(nmem);
  b->offs.resize(nmem + 1);
  long long off = 0, ng = 0;
  int blocks = 0;
  for (int m = 0; m < nmem; ++m) {
    const htr_member_desc& d = mds[m];
    long long N = 1;
    for (int a = 0; a < 3; ++a) {
      if (d.n[a] < 1 || !(d.dx[a] > 0) || !std::isfinite(d.dx[a])) {
        delete b;
        return fail(HTR_EINVAL, "member %d: n >= 1 and dx > 0 required on every axis", m);
      }
      N *= d.n[a];
      ng += 3LL * d.n[a];
    }
    if (check_laser(&d.laser)) {
      delete b;
      return HTR_EINVAL;
    }
    Member& M = b->host[m];
    std::memset(&M, 0, sizeof(M));
    M.N = N;
    M.off = off;
    M.block_begin = blocks;
    M.nblocks = (int)((N + BLK - 1) / BLK);
    for (int a = 0; a < 3; ++a) {
      M.n[a] = d.n[a];
      M.act[a] = d.n[a] > 1;
    }
    set_tiles(M, nullptr, &b->ntblocks, &b->ndtblocks);
    b->offs[m] = off;
    off += N;
    blocks += M.nblocks;
  }
  b->offs[nmem] = off;
  b->Ntot = off;
  b->nblocks = blocks;
  auto bail = [&](htr_status s2) {
    htr_batch_destroy(b);
    return s2;
  };
  hipError_t e;
  if ((e = hipMalloc(&b->dgrid, sizeof(double) * ng)) != hipSuccess ||
      (e = hipMalloc(&b->ddlnA, sizeof(double) * (size_t)nmem * (nr > 0 ? nr : 1))) != hipSuccess ||
      (e = hipMalloc(&b->dmem, sizeof(Member) * nmem)) != hipSuccess)
    return bail(fail(HTR_ENOMEM, "batch allocation: %s", hipGetErrorString(e)));
  std::vector<double> hg;
  hg.reserve(ng);
  std::vector<double> hd((size_t)nmem * (nr > 0 ? nr : 1), 0.0);
  long long go = 0;
  for (int m = 0; m < nmem; ++m) {
    const htr_member_desc& d = mds[m];
    Member& M = b->host[m];
    double L[3];
    for (int a = 0; a < 3; ++a) {
      const int na = d.n[a];
      L[a] = na * d.dx[a];
      for (int i = 0; i < na; ++i) hg.push_back(1.0 / d.dx[a]);
      for (int i = 0; i < na; ++i) hg.push_back(1.0 / d.dx[a]);
      for (int i = 0; i < na; ++i) hg.push_back((i + 0.5) * d.dx[a]);
      M.xin[a] = b->dgrid + go;
      M.xif[a] = b->dgrid + go + na;
      M.xnode[a] = b->dgrid + go + 2 * na;
      go += 3 * na;
      M.n[a] = na;
      M.act[a] = na > 1;
      M.L[a] = L[a];
    }
    M.laser = make_laser(&d.laser, d.n, L);
    if (d.dlnA && nr > 0) {
      for (int j = 0; j < nr; ++j) {
        if (!std::isfinite(d.dlnA[j])) return bail(fail(HTR_EINVAL, "member %d: non-finite dlnA", m));
        hd[(size_t)m * nr + j] = d.dlnA[j];
      }
      M.dlnA = b->ddlnA + (size_t)m * nr;
    } else {
      M.dlnA = nullptr;
    }
  }
  if ((e = hipMemcpy(b->dgrid, hg.data(), sizeof(double) * ng, hipMemcpyHostToDevice)) != hipSuccess ||
      (e = hipMemcpy(b->ddlnA, hd.data(), sizeof(double) * hd.size(), hipMemcpyHostToDevice)) != hipSuccess ||
      (e = hipMemcpy(b->dmem, b->host.data(), sizeof(Member) * nmem, hipMemcpyHostToDevice)) != hipSuccess)
    return bail(fail(HTR_EDEVICE, "batch upload: %s", hipGetErrorString(e)));
  htr_status st = ws_alloc(b->ws, ctx->ns, b->Ntot, b->nblocks, nmem);
  if (st) return bail(st);
  if ((e = hipStreamCreateWithFlags(&b->gstream, hipStreamNonBlocking)) != hipSuccess ||
      (e = hipEventCreateWithFlags(&b->ev_in, hipEventDisableTiming)) != hipSuccess ||
      (e = hipEventCreateWithFlags(&b->ev_out, hipEventDisableTiming)) != hipSuccess)
    return bail(fail(HTR_EDEVICE, "batch stream: %s", hipGetErrorString(e)));
  *out = b;
  return HTR_OK;
}

htr_status htr_batch_destroy(htr_batch* b) {
  if (!b) return fail(HTR_EINVAL, "batch is NULL");
  b->fence.wait();                      // this ensemble's work on the callers' streams
  if (b->gstream) hipStreamSynchronize(b->gstream);   // and its graph replays
  drop_graph(b);
  if (b->gstream) hipStreamDestroy(b->gstream);
  if (b->ev_in) hipEventDestroy(b->ev_in);
  if (b->ev_out) hipEventDestroy(b->ev_out);
  hipFree(b->dgrid);
  hipFree(b->ddlnA);
  hipFree(b->dmem);
  ws_free(b->ws);
  delete b;
  return HTR_OK;
}

htr_status htr_batch_member_max(htr_batch* b, const double* field, double* max_dev, int accumulate,
                                void* stream) {
  if (!b || !field || !max_dev) return fail(HTR_EINVAL, "NULL pointer");
  Marked mk_(&b->fence, stream);
  HIP_OK(launch_member_max(b->dmem, b->nmem, field, max_dev, accumulate, (hipStream_t)stream));
  return HTR_OK;
}

int64_t htr_batch_cells(const htr_batch* b, int64_t* offsets) {
  if (!b) return 0;
  if (offsets)
    for (int m = 0; m <= b->nmem; ++m) offsets[m] = b->offs[m];
  return b->Ntot;
}

size_t htr_batch_work_bytes(const htr_batch* b) {
  return b ? sizeof(double) * 2 * (size_t)(b->ctx->ns + 4) * b->Ntot : 0;
}

htr_status htr_batch_prim_to_cons(htr_batch* b, const double* Y, const double* T, const double* p,
                                  const double* vel, double* U, void* stream) {
  if (!b) return fail(HTR_EINVAL, "batch is NULL");
  Marked mk_(&b->fence, stream);
  if (!Y || !T || !p || !vel || !U) return fail(HTR_EINVAL, "NULL field pointer");
  Ctx C = bview(b);
  HIP_OK(launch_prim_to_cons(C.ns, C.M, C.mem, C.nmem, C.nblocks, Y, T, p, vel, U, (hipStream_t)stream));
  return HTR_OK;
}

htr_status htr_rhs_batched(htr_batch* b, const double* U, double* T_io, const double* t_dev, double* dUdt,
                           double* hrr, void* stream) {
  if (!b) return fail(HTR_EINVAL, "batch is NULL");
  Marked mk_(&b->fence, stream);
  if (!U || !T_io || !t_dev || !dUdt) return fail(HTR_EINVAL, "NULL pointer");
  if (U == dUdt) return fail(HTR_EINVAL, "dUdt must not alias U");
  Ctx C = bview(b);
  CallArgs a{};
  a.t_dev = t_dev;
  a.use_call_laser = 0;
  a.flags = C.scheme.flags;
  return stage(C, b->ws, a, U, U, T_io, dUdt, 0.0, 1.0, 1, hrr, nullptr, 0.0, (hipStream_t)stream, 0, nullptr);
}

htr_status htr_rk3_steps_batched(htr_batch* b, double* U, double* T_io, double* t_dev, double* dt_dev,
                                 int compute_dt, int nsteps, double* work, double* J_dev, int use_graph,
                                 void* stream) {
  if (!b) return fail(HTR_EINVAL, "batch is NULL");
  Marked mk_(&b->fence, stream);
  if (!U || !T_io || !t_dev || !dt_dev || !work) return fail(HTR_EINVAL, "NULL pointer");
  if (nsteps < 0) return fail(HTR_EINVAL, "nsteps must be >= 0");
  if (work == U || work == T_io) return fail(HTR_EINVAL, "work must not alias U or T_io");
  Ctx C = bview(b);
  hipStream_t s = (hipStream_t)stream;
  if (!use_graph) {
    for (int k = 0; k < nsteps; ++k) {
      htr_status st = rk3(C, b->ws, U, T_io, t_dev, dt_dev, compute_dt, nullptr, nullptr, work, J_dev, s, nullptr);
      if (st) return st;
    }
    return HTR_OK;
  }
  const void* key[7] = {U, T_io, t_dev, dt_dev, work, J_dev, b->ctx->dM};
  // the scheme (flags, thresholds) is baked into the captured kernel arguments
  const htr_scheme& sc = b->ctx->scheme;
  const bool same_scheme = sc.flags == b->key_scheme.flags && sc.cfl == b->key_scheme.cfl &&
                           sc.theta_c == b->key_scheme.theta_c && sc.psi_c == b->key_scheme.psi_c &&
                           sc.teno_CT == b->key_scheme.teno_CT;
  bool same = b->exec && b->key_steps == nsteps && b->key_cdt == compute_dt && same_scheme &&
              std::memcmp(key, b->key, sizeof key) == 0;
  if (!same) {
    drop_graph(b);
    C.timer = nullptr;   // no timing events inside a captured graph
    HIP_OK(hipStreamBeginCapture(b->gstream, hipStreamCaptureModeThreadLocal));
    htr_status st = HTR_OK;
    for (int k = 0; k < nsteps && !st; ++k)
      st = rk3(C, b->ws, U, T_io, t_dev, dt_dev, compute_dt, nullptr, nullptr, work, J_dev, b->gstream,
               nullptr);
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(b->gstream, &g);
    if (st) {
      if (g) hipGraphDestroy(g);
      return st;
    }
    if (e != hipSuccess) return fail(HTR_EDEVICE, "hipStreamEndCapture: %s", hipGetErrorString(e));
    b->graph = g;
    e = hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0);
    if (e != hipSuccess) {
      drop_graph(b);
      return fail(HTR_EDEVICE, "hipGraphInstantiate: %s", hipGetErrorString(e));
    }
    std::memcpy(b->key, key, sizeof key);
    b->key_steps = nsteps;
    b->key_cdt = compute_dt;
    b->key_scheme = sc;
  }
  // order the replay after the caller's stream and the caller's stream after it
  HIP_OK(hipEventRecord(b->ev_in, s));
  HIP_OK(hipStreamWaitEvent(b->gstream, b->ev_in, 0));
  {
    TimedLaunch tl(&b->timer, TC_REDUCE, b->gstream);
    HIP_OK(hipGraphLaunch(b->exec, b->gstream));
  }
  HIP_OK(hipEventRecord(b->ev_out, b->gstream));
  HIP_OK(hipStreamWaitEvent(s, b->ev_out, 0));
  return HTR_OK;
}

htr_status htr_batch_check(htr_batch* b, void* stream) {
  if (!b) return fail(HTR_EINVAL, "batch is NULL");
  HIP_OK(hipStreamSynchronize((hipStream_t)stream));
  HIP_OK(hipStreamSynchronize(b->gstream));
  unsigned st = 0;
  HIP_OK(hipMemcpy(&st, b->ws.status, sizeof st, hipMemcpyDeviceToHost));
  HIP_OK(hipMemset(b->ws.status, 0, sizeof(unsigned)));
  if (st & ST_NONFINITE) return fail(HTR_ENONFINITE, "non-finite state or rho <= 0 met on the device");
  if (st & ST_NEWTON) return fail(HTR_ENEWTON, "temperature Newton iteration did not converge");
  if (st & ST_TRANGE) return fail(HTR_ETRANGE, "temperature outside [Tmin, Tmax]");
  return HTR_OK;
}

}  // extern "C"
