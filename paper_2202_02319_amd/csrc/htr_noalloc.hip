// One SSP-RK3 step that allocates nothing: the two stage states and the
// per-cell scratch of the step (derived fields, sources, sensor flags,
// velocity gradients, partial right-hand side, block partials) live in a
// file-scope device array instead of caller work memory and the context's
// workspace.  For callers that cannot allocate device memory.
//
// The array's host-side name is not a device address.  Its address on each
// device is looked up once, with that device current, when a context is
// created there (htr_create calls noalloc_init), and kept per device; host
// code uses only that address.

#include <hip/hip_runtime.h>

#include <mutex>

#include "htr.h"
#include "htr_dev.h"
#include "htr_internal.h"

namespace {

constexpr size_t kScratchBytes = HTR_NOALLOC_MAX_BYTES;
constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_mu;
void* g_ptr[kMaxDevices] = {};

constexpr size_t kAlign = 256;
size_t up(size_t b) { return (b + kAlign - 1) / kAlign * kAlign; }

// Byte layout of the step's scratch for ns species and N cells in nblocks
// per-cell blocks; returns the total.
struct Layout {
  size_t work, aux, src, grad, part, blkred, scal, flag, tcls, total;
};
Layout layout(int ns, long long N, int nblocks) {
  const size_t d = sizeof(double), n = (size_t)N, nv = (size_t)ns + 4;
  Layout L{};
  size_t o = 0;
  L.work = o;   o += up(d * 2 * nv * n);
  L.aux = o;    o += up(d * (7 + (size_t)ns) * n);
  L.src = o;    o += up(d * ((size_t)ns + 1) * n);
  L.grad = o;   o += up(d * 9 * n);
  L.part = o;   o += up(d * nv * n);
  L.blkred = o; o += up(d * 2 * (size_t)nblocks);
  L.scal = o;   o += up(d * 2);
  L.flag = o;   o += up(n);
  L.tcls = o;   o += up(n);
  L.total = o;
  return L;
}

}  // namespace

namespace htr {

htr_status noalloc_init(int device) {
  if (device < 0 || device >= kMaxDevices) return fail(HTR_EUNSUPPORTED, "device index %d >= %d", device, kMaxDevices);
  std::lock_guard<std::mutex> g(g_mu);
  if (g_ptr[device]) return HTR_OK;
  void* p = nullptr;
  hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !p)
    return fail(HTR_EDEVICE, "hipGetSymbolAddress(scratch) on device %d: %s", device, hipGetErrorString(e));
  g_ptr[device] = p;
  return HTR_OK;
}

}  // namespace htr

extern "C" htr_status htr_rk3_step_noalloc(htr_ctx* c, double* U, double* T_io, double* t_dev, double* dt_dev,
                                           int compute_dt, const htr_laser* laser, const double* dlnA_dev,
                                           double* J_dev, void* stream) {
  using namespace htr;
  if (!c) return fail(HTR_EINVAL, "ctx is NULL");
  Marked mk_(&c->fence, stream);
  if (!U || !T_io || !t_dev || !dt_dev) return fail(HTR_EINVAL, "NULL pointer");
  htr_status st = check_laser(laser);
  if (st) return st;
  const Layout L = layout(c->ns, c->N, c->nblocks);
  if (L.total > kScratchBytes)
    return fail(HTR_EINVAL, "htr_rk3_step_noalloc: %lld cells with %d species need %zu bytes of scratch, "
                "more than the fixed %zu (HTR_NOALLOC_MAX_BYTES)", (long long)c->N, c->ns, L.total, kScratchBytes);
  int dev = -1;
  HIP_OK(hipGetDevice(&dev));
  if (dev != c->device) return fail(HTR_EINVAL, "the current device %d is not the context's device %d", dev, c->device);
  unsigned char* base = nullptr;
  {
    std::lock_guard<std::mutex> g(g_mu);
    if (dev >= 0 && dev < kMaxDevices) base = static_cast<unsigned char*>(g_ptr[dev]);
  }
  if (!base) return fail(HTR_EDEVICE, "no scratch address for device %d (no context was created on it)", dev);
  // Every region below is written in full before it is read within the
  // step, so nothing needs clearing; the status word stays the context's.
  Workspace w{};
  w.ns = c->ns;
  w.N = c->N;
  w.aux = reinterpret_cast<double*>(base + L.aux);
  w.src = reinterpret_cast<double*>(base + L.src);
  w.grad = reinterpret_cast<double*>(base + L.grad);
  w.part = reinterpret_cast<double*>(base + L.part);
  w.blkred = reinterpret_cast<double*>(base + L.blkred);
  w.scal = reinterpret_cast<double*>(base + L.scal);
  w.flag = base + L.flag;
  w.tcls = base + L.tcls;
  w.status = c->ws.status;
  double* work = reinterpret_cast<double*>(base + L.work);
  Ctx C = view(c);
  htr_laser off{};
  return rk3(C, w, U, T_io, t_dev, dt_dev, compute_dt, laser ? laser : &off, dlnA_dev, work, J_dev,
             (hipStream_t)stream, nullptr);
}
