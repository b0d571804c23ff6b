// Host-side internals shared by the C interface files.
#pragma once

#include <cstdarg>
#include <utility>
#include <vector>

#include "htr.h"
#include "htr_dev.h"

namespace htr {

// Sets the calling thread's last-error message and returns st.
htr_status fail(htr_status st, const char* fmt, ...) __attribute__((format(printf, 2, 3)));

#define HIP_OK(expr)                                                                              \
  do {                                                                                            \
    hipError_t e_ = (expr);                                                                       \
    if (e_ != hipSuccess) return ::htr::fail(HTR_EDEVICE, "%s: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

// Scratch owned by a context or an ensemble: per-cell derived fields,
// sources, sensor flags, block partials, status word.
struct Workspace {
  int ns = 0;
  long long N = 0;
  double* aux = nullptr;          // [7 + ns][N]
  double* src = nullptr;          // [ns + 1][N]
  unsigned char* flag = nullptr;  // [N]
  double* grad = nullptr;         // [9][N] nodal velocity gradient d u_m / d x_a (row 3a + m)
  double* part = nullptr;         // [nv][N] sources + convective flux differences of a stage
  unsigned char* tcls = nullptr;  // [N] (>= the tile count) tiles with TENO faces, marked by the lean sweep
  double* blkred = nullptr;       // [2][nblocks]
  unsigned* status = nullptr;
  double* scal = nullptr;         // [2][nmem] scratch scalars
};

// The streams a context or an ensemble has enqueued work on, each with an
// event recorded after the last such work.  Destroying the object waits on
// these events only, not on the whole device.  Work enqueued under stream
// capture is not tracked (the caller owns the graph and its launches).
struct Fence {
  std::vector<std::pair<hipStream_t, hipEvent_t>> ev;
  void mark(hipStream_t s);
  hipError_t wait();
  ~Fence();
};

// Marks the fence when an entry point returns, after it has enqueued its work.
struct Marked {
  Fence* f;
  hipStream_t s;
  Marked(Fence* f_, void* s_) : f(f_), s((hipStream_t)s_) {}
  ~Marked() { f->mark(s); }
};

// Timing classes (the order of htr_timing_read's arrays).
enum { TC_POINT = 0, TC_SENSOR = 1, TC_CONV = 2, TC_DIFF = 3, TC_REDUCE = 4, TC_UPDATE = 5 };

// HIP-event kernel timer (diagnostics).
struct Timer {
  bool on = false;
  struct Rec { int cls; hipEvent_t a, b; };
  std::vector<Rec> recs;
  std::vector<hipEvent_t> pool;
  hipEvent_t get();
  void clear();
  ~Timer();
};

// Brackets one launch with events when the timer is on.
struct TimedLaunch {
  Timer* t;
  int cls;
  hipStream_t s;
  hipEvent_t a = nullptr;
  TimedLaunch(Timer* t_, int cls_, hipStream_t s_);
  ~TimedLaunch();
};

// What a kernel sequence needs to know about the grids it runs on.
struct Ctx {
  int ns = 0;
  const MechTables* M = nullptr;
  const Member* mem = nullptr;
  int nmem = 1;
  int nblocks = 0;
  int ntblocks = 0;               // tiled launches (convective sweep)
  int ndtblocks = 0;              // diffusive-sweep launches
  int grid = 0;                   // persistent grid of the forward kernels (0: one block per logical block)
  int conv_split = 1;             // grid 0: central tiles in the lean convective sweep
  htr_scheme scheme{};
  long long total_cells = 0;
  int n1[3] = {1, 1, 1};          // grid of the single-member case (laser normalisation)
  double L1[3] = {1, 1, 1};
  Timer* timer = nullptr;
  bool bounded = false;           // single grid with non-periodic boundaries (boundary kernel)
  // curvilinear single grid (null: rectilinear sweeps)
  const CurvGeom* curv = nullptr;
  const Member* host1 = nullptr;  // host copy of the single member (curvilinear launch shapes)
  double* cX = nullptr;           // [ns][N] mole fractions
  double* cdphi = nullptr;        // [3][4 + ns][N] index-space central differences
  double* cffc = nullptr;         // [3][ns + 4][N] mapped convective face fluxes
  double* cffd = nullptr;         // [3][ns + 4][N] mapped diffusive face fluxes
};

LaserDev make_laser(const htr_laser* L, const int n[3], const double Lp[3]);
htr_status check_laser(const htr_laser* L);
htr_status build_tables(const htr_mech_desc* m, MechTables* T);
htr_status ws_alloc(Workspace& w, int ns, long long N, int nblocks, int nmem);
void ws_free(Workspace& w);
htr_status stage(const Ctx& C, const Workspace& w, const CallArgs& a, const double* U, const double* Un, double* T,
                 double* out, double ca, double cb, int rhs_only, double* hrr, double* J_dev, double jcoef,
                 hipStream_t s, int want_dt, double* dt_out, unsigned char* teno_bits = nullptr);
// Looks up, once per device and with that device current, the device
// address of the no-allocation step's scratch array (htr_noalloc.hip).
htr_status noalloc_init(int device);
htr_status rk3(const Ctx& C, const Workspace& w, double* U, double* T, double* t_dev, double* dt_dev,
               int compute_dt, const htr_laser* laser, const double* dlnA, double* work, double* J_dev,
               hipStream_t s, void* tape);

// Forward tape of one RK3 step: per stage k the per-cell fields [7 + ns][N],
// the temperature [N], the sensor flags [N] and the TENO cut-off patterns
// [3][nv][N] that the stage's sweeps used (doubles first, then the bytes).
struct TapeView {
  double* aux;
  double* T;
  unsigned char* flag;
  unsigned char* bits;
};
inline size_t tape_bytes(int ns, long long N) {
  return 3 * (sizeof(double) * (size_t)(8 + ns) * (size_t)N) + 3 * (size_t)N + 9 * (size_t)(ns + 4) * (size_t)N;
}
inline TapeView tape_view(void* tape, int ns, long long N, int k) {
  double* d = static_cast<double*>(tape);
  TapeView v;
  v.aux = d + (long long)k * (8 + ns) * N;
  v.T = v.aux + (long long)(7 + ns) * N;
  unsigned char* bytes = reinterpret_cast<unsigned char*>(d + 3LL * (8 + ns) * N);
  v.flag = bytes + (long long)k * N;
  v.bits = bytes + 3LL * N + (long long)k * 3 * (ns + 4) * N;
  return v;
}

}  // namespace htr

struct htr_ctx {
  int device = 0;
  int ns = 0, nr = 0;
  htr_scheme scheme{};
  htr::MechTables* dM = nullptr;   // device tables
  htr::Member host_mem{};          // single member (host copy)
  htr::Member* dmem = nullptr;     // device member table (one entry)
  double* dgrid = nullptr;         // device metric/coordinate arrays
  int n[3] = {1, 1, 1};
  double L[3] = {0, 0, 0};
  long long N = 0;
  int nblocks = 0;
  int ntblocks = 0;
  int ndtblocks = 0;
  int grid = 0;                    // persistent grid (0: off)
  int conv_split = 1;              // grid 0: lean convective sweep for the central tiles
  htr::Workspace ws;
  htr::Timer timer;
  htr::Fence fence;
  // curvilinear grid (htr_create_curvilinear); L above then holds the
  // distances between lattice planes (laser image counts)
  bool curv = false;
  htr::CurvGeom cg{};
  double* dcurv = nullptr;         // mt [10][N], mf [9][N], xyz [3][N]
  double* dcw = nullptr;           // X [ns][N], dphi [3][4 + ns][N], ffc and ffd [3][ns + 4][N]
};

// An ensemble (the opaque htr_batch of the C interface).
struct htr_batch {
  htr_ctx* ctx = nullptr;
  int nmem = 0;
  std::vector<htr::Member> host;
  std::vector<long long> offs;   // nmem + 1
  htr::Member* dmem = nullptr;
  double* dgrid = nullptr;
  double* ddlnA = nullptr;
  long long Ntot = 0;
  int nblocks = 0;
  int ntblocks = 0;
  int ndtblocks = 0;
  int grid = 0;                    // persistent grid (0: off)
  int conv_split = 1;              // grid 0: lean convective sweep for the central tiles
  htr::Workspace ws;
  htr::Timer timer;
  htr::Fence fence;
  hipStream_t gstream = nullptr;   // capture/replay stream (default priority)
  hipEvent_t ev_in = nullptr, ev_out = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  const void* key[7] = {};
  int key_steps = -1, key_cdt = -1;
  htr_scheme key_scheme{};         // scheme (flags, thresholds) baked into the captured kernels
};


namespace htr {
Ctx view(const htr_ctx* c);
Ctx bview(const htr_batch* b);
void drop_graph(htr_batch* b);   // the captured graph no longer matches the member table
}  // namespace htr
