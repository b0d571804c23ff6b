// Device-side data structures shared by the HIP kernels and the C interface.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "htr.h"

namespace htr {

constexpr int MAXNS = HTR_MAX_NS;
constexpr int MAXNR = HTR_MAX_NR;
constexpr int SIDE = HTR_MAX_SIDE;
constexpr int BLK = 256;            // threads per block of the per-cell kernels

// exact SI constants
constexpr double KB = 1.380649e-23;
constexpr double NAV = 6.02214076e23;
constexpr double RU = 8.31446261815324;
constexpr double PREF = 101325.0;   // standard-state pressure of K_c
constexpr double PI = 3.14159265358979323846;

// device status bits (first error wins by priority in htr_check)
constexpr unsigned ST_NONFINITE = 1u, ST_NEWTON = 2u, ST_TRANGE = 4u;

// Mechanism tables, precomputed on the host in the forms the kernels use.
struct MechTables {
  int ns, nr;
  double Tmin, Tmax;
  double W[MAXNS], iW[MAXNS], RW[MAXNS];   // W, 1/W, R_u/W
  double cp[MAXNS][5];                     // c_p/R = sum_k cp[k] T^k
  double hc[MAXNS][6];                     // h/(RT) = sum_{k<5} hc[k] T^k + hc[5]/T
  double sc[MAXNS][6];                     // s/R = sc[0] ln T + sum_{k=1..4} sc[k] T^k + sc[5]
  double mu_pre[MAXNS];                    // mu_s = mu_pre sqrt(T) / Omega22(T/eps)
  double ieps[MAXNS], lneps[MAXNS];        // 1/(eps/k), ln(eps/k)
  double euck[MAXNS];                      // (5/4) R_u / W
  double wq[MAXNS][MAXNS];                 // (W_j / W_i)^(1/4)
  double wp[MAXNS][MAXNS];                 // 1 / sqrt(8 (1 + W_i / W_j))
  double Dpre[MAXNS][MAXNS];               // D_ij = Dpre T^(3/2) / (p Omega11(T/eps_ij))
  double Dieps[MAXNS][MAXNS], Dlneps[MAXNS][MAXNS];
  double pw22[MAXNS];                      // (eps/k)^0.14874: T*^-0.14874 = T^-0.14874 pw22
  double pw11[MAXNS][MAXNS];               // eps_ij^0.15610
  double iDpre[MAXNS][MAXNS];              // 1 / Dpre
  double lnA[MAXNR], beta[MAXNR], EaR[MAXNR], dnu[MAXNR];
  double nunet[MAXNR][MAXNS];              // nu'' - nu'
  int nre[MAXNR], npr[MAXNR];              // distinct reactant / product species
  int ridx[MAXNR][SIDE], rnu[MAXNR][SIDE];
  int pidx[MAXNR][SIDE], pnu[MAXNR][SIDE];
};

struct LaserDev {
  double E, xc[3], sr, t0, st;
  double norm;     // 1 / ((2 pi)^((d+1)/2) sr^d st)
  int M[3];        // periodic images summed per axis
  int on;
};

// One grid (an ensemble member, or the single grid of a context).  Field
// arrays of all members are packed: member m's block of a [rows][N_m] field
// starts at base + rows * off.
struct Member {
  int n[3];
  int act[3];                 // n[a] > 1
  long long N;
  long long off;              // cell offset in packed arrays
  int block_begin;            // first block of this member in per-cell launches
  int nblocks;
  int tdim[3];                // tile of the convective sweep (256 cells)
  int ntile[3];               // tiles per axis
  int tblock_begin;           // first block of this member in tiled launches
  int ntblocks;
  int dtdim[3];               // tile of the diffusive sweep (DTILE cells)
  int dntile[3];
  int dtblock_begin;          // first block of this member in diffusive-sweep launches
  int ndtblocks;
  const double* xin[3];       // d(xi)/dx at nodes
  const double* xif[3];       // d(xi)/dx at faces i+1/2
  const double* xnode[3];     // node coordinates
  double L[3];
  LaserDev laser;
  const double* dlnA;         // nullable [nr]
  // non-periodic boundaries of a single-grid context (htr_set_boundaries):
  // per axis and side the boundary type (HTR_BC_*; 0 periodic), the
  // outflow's far-field pressure and relaxation coefficient
  int bc[3][2];
  double pinf[3][2];
  double relax[3][2];
  int bounded;                // any axis bounded
};

// Whether cell coordinate c lies within three nodes of a bounded boundary:
// the cells whose right-hand side the boundary kernel writes.
__device__ __forceinline__ bool in_boundary_slab(const Member& G, const int c[3]) {
  if (!G.bounded) return false;
  bool s = false;
#pragma unroll
  for (int a = 0; a < 3; ++a) s = s || (G.bc[a][0] != 0 && (c[a] < 3 || c[a] > G.n[a] - 4));
  return s;
}

// General curvilinear grid of a single-grid context (Methods › Numerical method, the mapped
// equations): metric terms at nodes and faces, node coordinates, lattice.
struct CurvGeom {
  const double* mt;    // [10][N]: (d xi_d / d x_c) / J at row 3d + c; J at row 9
  const double* mf;    // [9][N]: the same at face i+1/2 along d
  const double* xyz;   // [3][N] node coordinates
  double P[3][3];      // P[a]: lattice displacement when index a advances by n[a]
  double Pinv[3][3];   // inverse of the matrix whose columns are P[a]
};

// Per-call overrides used by the single-grid entry points.
struct CallArgs {
  double t;                   // time of stage 0 (when t_dev is null)
  const double* t_dev;        // nullable [nmem]: per-member time
  const double* dt_dev;       // nullable [nmem]: per-member step
  double tcoef;               // stage time = t + tcoef * dt
  LaserDev laser;             // used when use_call_laser
  int use_call_laser;
  const double* dlnA;         // nullable: overrides member dlnA
  unsigned flags;
};

__device__ __forceinline__ int find_member(const Member* __restrict__ mem, int nmem, int b) {
  int lo = 0, hi = nmem - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (mem[mid].block_begin <= b) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// Member of a block in the tiled launches.
__device__ __forceinline__ int find_member_tiled(const Member* __restrict__ mem, int nmem, int b) {
  int lo = 0, hi = nmem - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (mem[mid].tblock_begin <= b) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// Tile origin of local tiled block bl of a tiling (tile dims td, tiles per
// axis nt, nb tiles).  Blocks are dealt to the eight XCDs round-robin; the
// first 8*(nb/8) blocks are remapped so that each XCD works on one
// contiguous run of tiles and neighbouring tiles share its L2.
constexpr int TILE_ZGROUP = 4;
__device__ __forceinline__ void tile_origin_of(const int td[3], const int nt[3], int nb, int bl, int o[3]) {
  const int per = nb >> 3;
  const int lb = bl < 8 * per ? (bl & 7) * per + (bl >> 3) : bl;
  // lb -> tile: x fastest, then z within groups of TILE_ZGROUP tile layers, then
  // y, then the z group, so that tiles adjacent in y and z are processed
  // close together in time (only the last group may be thinner)
  const int ntx = nt[0], nty = nt[1], ntz = nt[2];
  const int gz = ntz < TILE_ZGROUP ? ntz : TILE_ZGROUP;
  const int per_group = ntx * nty * gz;
  const int grp = lb / per_group;
  const int gsz = ntz - grp * gz < gz ? ntz - grp * gz : gz;
  const int r = lb - grp * per_group;
  const int tx = r % ntx, r2 = r / ntx;
  const int tz = grp * gz + r2 % gsz, ty = r2 / gsz;
  o[0] = tx * td[0];
  o[1] = ty * td[1];
  o[2] = tz * td[2];
}
// The convective sweep's tiles (and the adjoint's).
__device__ __forceinline__ void tile_origin(const Member& G, int bl, int o[3]) {
  tile_origin_of(G.tdim, G.ntile, G.ntblocks, bl, o);
}
// Member of a block of the diffusive sweep.
__device__ __forceinline__ int find_member_dtiled(const Member* __restrict__ mem, int nmem, int b) {
  int lo = 0, hi = nmem - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (mem[mid].dtblock_begin <= b) lo = mid; else hi = mid - 1;
  }
  return lo;
}

__device__ __forceinline__ int wrapi(int i, int n) {
  i = i % n;
  return i < 0 ? i + n : i;
}

// Staging limits of the tiled kernels; a tile shape is accepted only if it
// fits all of them (tile_shape_ok).
// The diffusive sweep: DTILE-cell tiles in blocks of BLKF threads, one face
// per thread along each axis (a tile has at most BLKF faces along any axis):
// three 4-wave blocks per CU at its register count.
constexpr int DTILE = 192;
constexpr int BLKF = 256;
constexpr int XBOX_MAX = 2208;   // convective cross staging: the three direction boxes (22*4*4 + 16*10*4 + 16*4*10)
constexpr int XARM_MAX = 864;    // its halo cells: 6 per line along every axis
constexpr int XFACE_MAX = 912;   // faces over all axes (17*4*4 + 16*5*4 + 16*4*5)
constexpr int EXTA = 896;        // convective adjoint: tile extended by 5 + 5 along one axis
constexpr int FACEA = 640;       // faces touching a tile along one axis

// Dispatch on the species count (the kernels are templated on it).
#define HTR_NS_SWITCH(ns, CALL)                                                        \
  switch (ns) {                                                                        \
    case 1: return CALL(1); case 2: return CALL(2); case 3: return CALL(3);            \
    case 4: return CALL(4); case 5: return CALL(5); case 6: return CALL(6);            \
    case 7: return CALL(7); case 8: return CALL(8); case 9: return CALL(9);            \
    case 10: return CALL(10); case 11: return CALL(11); case 12: return CALL(12);      \
    default: return hipErrorInvalidValue;                                              \
  }

// host-side launchers (defined in the .hip files)
struct Workspace;
hipError_t launch_prim_to_cons(int ns, const MechTables* M, const Member* mem, int nmem, int nblocks,
                               const double* Y, const double* T, const double* p, const double* vel, double* U,
                               hipStream_t s);
// cg (nullable): the curvilinear geometry of a single-grid context (laser
// over lattice images, contravariant dt limit, volume 1/J)
hipError_t launch_point(int ns, const MechTables* M, const Member* mem, int nmem, int nblocks, int grid,
                        const CallArgs& a,
                        const double* U, double* T, double* aux, double* src, double* hrr, double* blkred,
                        double* cells_out, unsigned* status, int want_dt, hipStream_t s,
                        const CurvGeom* cg = nullptr);
hipError_t launch_sensor(const Member* mem, int nmem, int nblocks, int grid, const double* aux, int ns,
                         unsigned char* flag,
                         double* grad, double theta_c, double* theta_out, hipStream_t s);
// bits (nullable): TENO cut-off patterns [3][nv][N] bytes, per axis, variable
// and face (indexed by the face's upper cell); written for TENO faces only.
// tcls: one byte per tile (at least ntblocks), the lean sweep's tile marks;
// null: every tile in the full sweep (no lean launch).
hipError_t launch_conv(int ns, const MechTables* M, const Member* mem, int nmem, int ntblocks, int grid,
                       const CallArgs& a,
                       const double* U, const double* aux, const double* src, const unsigned char* flag, double* part,
                       unsigned char* bits, double psi_c, double CT, unsigned char* tcls, hipStream_t s);
// Right-hand side of the cells next to non-periodic boundaries (single
// grid), written over the convective sweep's part[] for those cells.
hipError_t launch_bnd(int ns, const MechTables* M, const Member* mem, int nblocks, const CallArgs& a, const double* U,
                      const double* T, const double* aux, const double* src, const unsigned char* flag,
                      const double* grad, double* part, double psi_c, double CT, hipStream_t s);
hipError_t launch_diff(int ns, const MechTables* M, const Member* mem, int nmem, int ntblocks, int grid,
                       const CallArgs& a,
                       const double* U, const double* Un, const double* T, const double* aux, const double* grad,
                       const double* part, double* out, double ca, double cb, int rhs_only, hipStream_t s);
// Tile shape of member M's convective sweep (shape == nullptr: the default
// for its active axes), appending its tiles to the running count *tblocks;
// and its diffusive sweep's tiles (a fixed shape for its active axes),
// appended to *dtblocks.
void set_tiles(Member& M, const int* shape, int* tblocks, int* dtblocks);
// Whether a tile shape suits a member with active axes act (message on failure).
bool tile_shape_ok(const int act[3], const int shape[3], const char** why);
// Default tile shape for the active axes.
void default_tile_shape(const int act[3], int shape[3]);
hipError_t launch_finalize(const Member* mem, int nmem, const double* blkred, double cfl, double* dt_dev,
                           double* J_dev, const double* dt_in, double jcoef, int want_dt, hipStream_t s);
hipError_t launch_advance_time(int nmem, double* t_dev, const double* dt_dev, hipStream_t s);
hipError_t launch_member_max(const Member* mem, int nmem, const double* field, double* out, int accumulate,
                             hipStream_t s);
// bits (nullable): the forward's TENO cut-off patterns (as launch_conv wrote them).
hipError_t launch_adjoint(int ns, const MechTables* M, const Member* mem, int nmem, int nblocks, int ntblocks,
                          const CallArgs& a,
                          const double* U, const double* T, const double* aux, const unsigned char* flag,
                          const unsigned char* bits,
                          const double* lam, double s, double h, double* ubd, double* pbv, double* out,
                          double* thpart, int nth, double psi_c, double CT, hipStream_t st);
hipError_t launch_adj_theta(const Member* mem, int nmem, const double* thpart, int nth, double* pbar,
                            hipStream_t st);
hipError_t launch_axpby(long long n, double a, const double* x, double b, double* y, hipStream_t st);

// Curvilinear grids (htr_curv.hip).  Metric terms of the node lattice
// (xyz, P) into mt rows 0..8, J into row 9 (0 where det(d x / d xi) is not
// positive and finite), face values into mf.
hipError_t launch_curv_metrics(const Member* mem, const Member& host, const CurvGeom& g, double* mt, double* mf,
                               hipStream_t s);
// Sensor flags (and theta into theta_out row nq - 1 when non-null) by the chain rule.
hipError_t launch_curv_sensor(const Member* mem, int nblocks, const CurvGeom& g, const double* aux, int ns,
                              unsigned char* flag, double theta_c, double* theta_out, hipStream_t s);
// Mole fractions X [ns][N] and index-space central differences of
// (u, v, w, T, X_s) along each active axis, dphi [3][4 + ns][N].
hipError_t launch_curv_igrad(int ns, const MechTables* M, const Member* mem, int nblocks, const double* U,
                             const double* T, const double* aux, double* X, double* dphi, hipStream_t s);
// Mapped face fluxes [3][ns + 4][N], face i+1/2 along d stored at node i:
// convective (the hybrid scheme on the metric-projected flux) and diffusive.
hipError_t launch_curv_conv(int ns, const Member& host, const Member* mem, const CurvGeom& g, const CallArgs& a,
                            const double* U, const double* aux, const unsigned char* flag, double* ffc, double psi_c,
                            double teno_CT, hipStream_t s);
hipError_t launch_curv_diff(int ns, const MechTables* M, const Member* mem, int nblocks, const CurvGeom& g,
                            const double* U, const double* T, const double* aux, const double* X,
                            const double* dphi, double* ffd, hipStream_t s);
// dU/dt = src + J sum_d ((ffd_d(i) - ffd_d(i - e_d)) - (ffc_d(i) - ffc_d(i - e_d)))
// (ffd not read when HTR_VISC_OFF), then the stage combination as the
// rectilinear sweep (or dU/dt itself when rhs_only).
hipError_t launch_curv_update(int ns, const Member* mem, int nblocks, const CurvGeom& g,
                              const CallArgs& a, const double* U, const double* Un, const double* src,
                              const double* ffc, const double* ffd, double* out, double ca, double cb, int rhs_only,
                              hipStream_t s);

}  // namespace htr
