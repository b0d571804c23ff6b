// Tile shapes, persistent launches and the autotuner of the forward kernels.
//
// The tiled sweeps accept any 256-cell tile shape that their staging
// buffers hold (tile_shape_ok), and every forward kernel can run as a
// persistent grid that strides over its logical blocks.  The autotuner times
// one RK3 stage (point, sensor, convective and diffusive sweeps with the
// stage update) for every candidate (shape, grid) and keeps the fastest; for an
// ensemble it tunes each class of equal-size members on a member table that
// holds only that class, then the persistent grid of the whole batch.
// Results do not depend on the choice: every face is evaluated once with
// the same arithmetic whatever the tile.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <map>
#include <vector>

#include "htr.h"
#include "htr_dev.h"
#include "htr_internal.h"

using namespace htr;

namespace {

// Candidate shapes for the active axes (each checked by tile_shape_ok).
std::vector<std::array<int, 3>> shape_candidates(const int act[3]) {
  std::vector<std::array<int, 3>> out;
  const int na = act[0] + act[1] + act[2];
  std::vector<std::array<int, 3>> raw;
  if (na == 3) {
    raw = {{16, 4, 4}, {8, 8, 4}, {8, 4, 8}, {32, 4, 2}, {16, 8, 2}, {4, 8, 8}};
  } else if (na == 2) {
    int a = -1, b = -1;
    for (int d = 0; d < 3; ++d)
      if (act[d]) (a < 0 ? a : b) = d;
    const int pairs[4][2] = {{16, 16}, {32, 8}, {64, 4}, {8, 32}};
    for (auto& p : pairs) {
      std::array<int, 3> t = {1, 1, 1};
      t[a] = p[0];
      t[b] = p[1];
      raw.push_back(t);
    }
  } else {
    int t[3];
    default_tile_shape(act, t);
    raw.push_back({t[0], t[1], t[2]});
  }
  for (auto& t : raw)
    if (tile_shape_ok(act, t.data(), nullptr)) out.push_back(t);
  return out;
}

// Persistent grid candidates: off, and 2 and 4 blocks per compute unit.
std::vector<int> grid_candidates() {
  int dev = 0, ncu = 0;
  hipGetDevice(&dev);
  if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || ncu < 1) ncu = 256;
  return {0, 2 * ncu, 4 * ncu};
}

// Milliseconds of one RK3 stage (right-hand side and stage update, written
// to out) on stream s: median of reps after one warm-up.  The stage's dt is
// read from the workspace scratch scalars: its value only scales the
// discarded output.
htr_status time_rhs(const Ctx& C, const Workspace& w, const double* U, double* T, double* out, hipStream_t s,
                    int reps, float* ms) {
  CallArgs a{};
  a.flags = C.scheme.flags;
  a.dt_dev = w.scal;
  hipEvent_t e0, e1;
  HIP_OK(hipEventCreate(&e0));
  HIP_OK(hipEventCreate(&e1));
  std::vector<float> v;
  htr_status st = HTR_OK;
  for (int r = 0; r <= reps && !st; ++r) {
    hipEventRecord(e0, s);
    st = stage(C, w, a, U, U, T, out, 0.75, 0.25, 0, nullptr, nullptr, 0.0, s, 0, nullptr);
    hipEventRecord(e1, s);
    if (st) break;
    if (hipEventSynchronize(e1) != hipSuccess) {
      st = fail(HTR_EDEVICE, "timing event failed");
      break;
    }
    float t = 0.0f;
    hipEventElapsedTime(&t, e0, e1);
    if (r > 0) v.push_back(t);
  }
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  if (st) return st;
  std::sort(v.begin(), v.end());
  *ms = v[v.size() / 2];
  return HTR_OK;
}

htr_status upload_ctx_member(htr_ctx* c) {
  HIP_OK(hipDeviceSynchronize());   // kernels in flight may still read the table
  HIP_OK(hipMemcpy(c->dmem, &c->host_mem, sizeof(Member), hipMemcpyHostToDevice));
  return HTR_OK;
}

// Re-derives every member's tiled-block range from its shape, uploads the table.
htr_status relayout_batch(htr_batch* b) {
  b->ntblocks = 0;
  b->ndtblocks = 0;
  for (auto& M : b->host) {
    const int t[3] = {M.tdim[0], M.tdim[1], M.tdim[2]};
    set_tiles(M, t, &b->ntblocks, &b->ndtblocks);
  }
  HIP_OK(hipDeviceSynchronize());
  HIP_OK(hipMemcpy(b->dmem, b->host.data(), sizeof(Member) * b->nmem, hipMemcpyHostToDevice));
  drop_graph(b);
  return HTR_OK;
}

htr_status check_shape(const Member& M, const int32_t* shape) {
  const int act[3] = {M.act[0], M.act[1], M.act[2]};
  const int t[3] = {shape[0], shape[1], shape[2]};
  const char* why = nullptr;
  if (!tile_shape_ok(act, t, &why))
    return fail(HTR_EINVAL, "tile %dx%dx%d: %s", shape[0], shape[1], shape[2], why);
  return HTR_OK;
}

}  // namespace

extern "C" {

htr_status htr_tile_shape_check(const int32_t n[3], const int32_t shape[3]) {
  if (!n || !shape) return fail(HTR_EINVAL, "NULL pointer");
  Member M{};
  for (int a = 0; a < 3; ++a) {
    if (n[a] < 1) return fail(HTR_EINVAL, "n must be >= 1 on every axis");
    M.act[a] = n[a] > 1;
  }
  return check_shape(M, shape);
}

htr_status htr_set_tiling(htr_ctx* c, const int32_t shape[3], int32_t grid) {
  if (!c) return fail(HTR_EINVAL, "ctx is NULL");
  if (c->curv) return fail(HTR_EUNSUPPORTED, "tiles and persistent grids apply to rectilinear grids");
  if (grid < 0) return fail(HTR_EINVAL, "grid must be >= 0");
  if (shape) {
    htr_status st = check_shape(c->host_mem, shape);
    if (st) return st;
  }
  int t[3];
  if (shape) {
    for (int a = 0; a < 3; ++a) t[a] = shape[a];
  } else {
    const int act[3] = {c->host_mem.act[0], c->host_mem.act[1], c->host_mem.act[2]};
    default_tile_shape(act, t);
  }
  c->ntblocks = 0;
  c->ndtblocks = 0;
  set_tiles(c->host_mem, t, &c->ntblocks, &c->ndtblocks);
  c->grid = grid;
  return upload_ctx_member(c);
}

htr_status htr_get_tiling(const htr_ctx* c, int32_t shape[3], int32_t* grid) {
  if (!c || !shape || !grid) return fail(HTR_EINVAL, "NULL pointer");
  for (int a = 0; a < 3; ++a) shape[a] = c->host_mem.tdim[a];
  *grid = c->grid;
  return HTR_OK;
}

htr_status htr_autotune(htr_ctx* c, const double* U, double* T_io, double* work, void* stream, int32_t shape_out[3],
                        int32_t* grid_out) {
  if (!c || !U || !T_io || !work) return fail(HTR_EINVAL, "NULL pointer");
  if (c->curv) return fail(HTR_EUNSUPPORTED, "tiles and persistent grids apply to rectilinear grids");
  hipStream_t s = (hipStream_t)stream;
  const int act[3] = {c->host_mem.act[0], c->host_mem.act[1], c->host_mem.act[2]};
  std::array<int, 3> best_t = {c->host_mem.tdim[0], c->host_mem.tdim[1], c->host_mem.tdim[2]};
  int best_g = c->grid, best_split = c->conv_split;
  // two passes over the candidates (shape, grid, split of the convective
  // sweep at grid 0); each candidate keeps its faster median
  struct Cand { std::array<int, 3> t; int g, split; };
  std::vector<Cand> cand;
  for (auto& t : shape_candidates(act))
    for (int g : grid_candidates()) {
      cand.push_back({t, g, 1});
      if (g == 0) cand.push_back({t, g, 0});
    }
  std::vector<float> tm(cand.size(), 1e30f);
  for (int pass = 0; pass < 2; ++pass) {
    for (size_t i = 0; i < cand.size(); ++i) {
      htr_status st = htr_set_tiling(c, cand[i].t.data(), cand[i].g);
      if (st) return st;
      c->conv_split = cand[i].split;
      float ms = 0.0f;
      st = time_rhs(view(c), c->ws, U, T_io, work, s, 5, &ms);
      if (st) return st;
      tm[i] = std::min(tm[i], ms);
    }
  }
  float best = 1e30f;
  for (size_t i = 0; i < cand.size(); ++i) {
    if (tm[i] < best) {
      best = tm[i];
      best_t = cand[i].t;
      best_g = cand[i].g;
      best_split = cand[i].split;
    }
  }
  c->conv_split = best_split;
  htr_status st = htr_set_tiling(c, best_t.data(), best_g);
  if (st) return st;
  if (shape_out)
    for (int a = 0; a < 3; ++a) shape_out[a] = best_t[a];
  if (grid_out) *grid_out = best_g;
  return HTR_OK;
}

htr_status htr_batch_set_tiling(htr_batch* b, int32_t member, const int32_t shape[3], int32_t grid) {
  if (!b) return fail(HTR_EINVAL, "batch is NULL");
  if (grid < 0) return fail(HTR_EINVAL, "grid must be >= 0");
  if (member < -1 || member >= b->nmem) return fail(HTR_EINVAL, "member %d out of range", member);
  const int m0 = member < 0 ? 0 : member, m1 = member < 0 ? b->nmem : member + 1;
  for (int m = m0; m < m1; ++m) {
    Member& M = b->host[m];
    const int act[3] = {M.act[0], M.act[1], M.act[2]};
    int t[3];
    if (shape) {
      htr_status st = check_shape(M, shape);
      if (st) return st;
      for (int a = 0; a < 3; ++a) t[a] = shape[a];
    } else {
      default_tile_shape(act, t);
    }
    for (int a = 0; a < 3; ++a) M.tdim[a] = t[a];
  }
  b->grid = grid;
  return relayout_batch(b);
}

htr_status htr_batch_get_tiling(const htr_batch* b, int32_t member, int32_t shape[3], int32_t* grid) {
  if (!b || !shape || !grid) return fail(HTR_EINVAL, "NULL pointer");
  if (member < 0 || member >= b->nmem) return fail(HTR_EINVAL, "member %d out of range", member);
  for (int a = 0; a < 3; ++a) shape[a] = b->host[member].tdim[a];
  *grid = b->grid;
  return HTR_OK;
}

htr_status htr_batch_autotune(htr_batch* b, const double* U, double* T_io, double* work, void* stream) {
  if (!b || !U || !T_io || !work) return fail(HTR_EINVAL, "NULL pointer");
  hipStream_t s = (hipStream_t)stream;
  // classes of equal-size members, largest total first
  std::map<std::array<int, 3>, std::vector<int>> cls;
  for (int m = 0; m < b->nmem; ++m) cls[{b->host[m].n[0], b->host[m].n[1], b->host[m].n[2]}].push_back(m);
  std::vector<std::vector<int>> order;
  for (auto& kv : cls) order.push_back(kv.second);
  std::sort(order.begin(), order.end(), [&](const std::vector<int>& x, const std::vector<int>& y) {
    return (long long)x.size() * b->host[x[0]].N > (long long)y.size() * b->host[y[0]].N;
  });
  Member* dsub = nullptr;
  HIP_OK(hipMalloc(&dsub, sizeof(Member) * b->nmem));
  htr_status st = HTR_OK;
  for (auto& members : order) {
    const Member& R = b->host[members[0]];
    const int act[3] = {R.act[0], R.act[1], R.act[2]};
    std::array<int, 3> best_t = {R.tdim[0], R.tdim[1], R.tdim[2]};
    float best = 1e30f;
    for (auto& t : shape_candidates(act)) {
      // a member table with only this class, its block ranges renumbered
      std::vector<Member> sub;
      int nb = 0, ntb = 0, ndtb = 0;
      long long cells = 0;
      for (int m : members) {
        Member M = b->host[m];
        M.block_begin = nb;
        nb += M.nblocks;
        set_tiles(M, t.data(), &ntb, &ndtb);
        cells += M.N;
        sub.push_back(M);
      }
      if ((st = (hipMemcpy(dsub, sub.data(), sizeof(Member) * sub.size(), hipMemcpyHostToDevice) == hipSuccess
                     ? HTR_OK
                     : fail(HTR_EDEVICE, "hipMemcpy member table"))))
        break;
      Ctx C = bview(b);
      C.mem = dsub;
      C.nmem = (int)sub.size();
      C.nblocks = nb;
      C.ntblocks = ntb;
      C.ndtblocks = ndtb;
      C.grid = 0;
      C.timer = nullptr;
      C.total_cells = cells;
      float ms = 0.0f;
      if ((st = time_rhs(C, b->ws, U, T_io, work, s, 5, &ms))) break;
      if (ms < best) {
        best = ms;
        best_t = t;
      }
    }
    if (st) break;
    for (int m : members)
      for (int a = 0; a < 3; ++a) b->host[m].tdim[a] = best_t[a];
  }
  hipDeviceSynchronize();
  hipFree(dsub);
  if (st) return st;
  if ((st = relayout_batch(b))) return st;
  // persistent grid of the whole batch (and, at grid 0, the convective
  // sweep's split)
  int best_g = 0, best_split = 1;
  float best = 1e30f;
  for (int g : grid_candidates()) {
    for (int split = 1; split >= (g == 0 ? 0 : 1); --split) {
      b->grid = g;
      b->conv_split = split;
      float ms = 0.0f;
      Ctx C = bview(b);
      C.timer = nullptr;
      if ((st = time_rhs(C, b->ws, U, T_io, work, s, 5, &ms))) return st;
      if (ms < best) {
        best = ms;
        best_g = g;
        best_split = split;
      }
    }
  }
  b->grid = best_g;
  b->conv_split = best_split;
  drop_graph(b);
  return HTR_OK;
}

htr_status htr_set_conv_split(htr_ctx* c, int32_t split) {
  if (!c) return fail(HTR_EINVAL, "ctx is NULL");
  if (split != 0 && split != 1) return fail(HTR_EINVAL, "split must be 0 or 1");
  if (c->curv) return fail(HTR_EUNSUPPORTED, "the convective sweep's split applies to rectilinear grids");
  c->conv_split = split;
  return HTR_OK;
}

htr_status htr_get_conv_split(const htr_ctx* c, int32_t* split) {
  if (!c || !split) return fail(HTR_EINVAL, "NULL pointer");
  *split = c->conv_split;
  return HTR_OK;
}

htr_status htr_batch_set_conv_split(htr_batch* b, int32_t split) {
  if (!b) return fail(HTR_EINVAL, "batch is NULL");
  if (split != 0 && split != 1) return fail(HTR_EINVAL, "split must be 0 or 1");
  HIP_OK(hipDeviceSynchronize());   // a replay in flight may still use the captured graph
  b->conv_split = split;
  drop_graph(b);
  return HTR_OK;
}

htr_status htr_batch_get_conv_split(const htr_batch* b, int32_t* split) {
  if (!b || !split) return fail(HTR_EINVAL, "NULL pointer");
  *split = b->conv_split;
  return HTR_OK;
}

}  // extern "C"
