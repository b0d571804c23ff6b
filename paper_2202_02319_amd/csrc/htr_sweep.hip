// Flux sweep: for every cell, the flux differences along every active
// direction of the hybrid TENO6/central convective flux and of the
// second-order diffusive flux, plus the chemistry and laser sources, fused
// with the SSP-RK3 stage combination (or written as dU/dt).
//
// Paper (arXiv 2202.02319) Sec. 5.2: conservative finite differences of the
// mapped equations (rectilinear metrics), TENO6 for the inviscid fluxes,
// second-order central differences for the diffusive fluxes; Sec. 5.1 eqs.
// (1)-(3), (5), (6) for the flux vectors.
//
// Two tiled kernels per stage, one block per 256-cell tile: k_conv (sources
// and convective flux differences, with the tile and its halo staged in
// LDS) and k_diff (diffusive flux differences and the stage update).  Every
// face is evaluated once, so the scheme is exactly conservative.

#include <math.h>

#include "htr_dev.h"
#include "htr_flux.h"

namespace htr {


// Tile shape of the tiled kernels: 256 cells, 16 x 4 x 4 on 3-D grids,
// 16 x 16 over the two active axes of 2-D grids, 256 along a 1-D grid.
void set_tiles(Member& M, int* tblocks) {
  int act[3] = {M.act[0], M.act[1], M.act[2]};
  const int na = act[0] + act[1] + act[2];
  int t[3] = {1, 1, 1};
  if (na == 3) {
    t[0] = 16; t[1] = 4; t[2] = 4;
  } else if (na == 2) {
    for (int a = 0; a < 3; ++a) t[a] = act[a] ? 16 : 1;
  } else if (na == 1) {
    for (int a = 0; a < 3; ++a) t[a] = act[a] ? 256 : 1;
  } else {
    t[0] = 256;
  }
  int nb = 1;
  for (int a = 0; a < 3; ++a) {
    M.tdim[a] = t[a];
    M.ntile[a] = (M.n[a] + t[a] - 1) / t[a];
    nb *= M.ntile[a];
  }
  M.tblock_begin = *tblocks;
  M.ntblocks = nb;
  *tblocks += nb;
}

// TENO6 face flux on the local Lax-Friedrichs split, kept out of line so the
// (far more common) central faces do not carry its register footprint.
__device__ __attribute__((noinline)) double teno_face(double f0, double f1, double f2, double f3, double f4,
                                                     double f5, double u0, double u1, double u2, double u3,
                                                     double u4, double u5, double al, double CT) {
  const double f6[6] = {f0, f1, f2, f3, f4, f5}, u6[6] = {u0, u1, u2, u3, u4, u5};
  double fp[6], fm[6];
#pragma unroll
  for (int mm = 0; mm < 6; ++mm) {
    fp[mm] = 0.5 * (f6[mm] + al * u6[mm]);
    fm[5 - mm] = 0.5 * (f6[mm] - al * u6[mm]);
  }
  return teno6(fp, CT) + teno6(fm, CT);
}

constexpr int BLKF = 320;        // threads of the diffusive sweep: one per face of a tile along an axis
constexpr int EXT_MAX = 640;     // tile extended by 3 + 3 cells along one axis
constexpr int FACE_MAX = 320;    // faces of a tile along one axis
constexpr int STG = (EXT_MAX + BLK - 1) / BLK;
constexpr int FPT = (FACE_MAX + BLK - 1) / BLK;

__device__ __forceinline__ long long lin(const Member& G, const int g[3]) {
  return ((long long)g[2] * G.n[1] + g[1]) * G.n[0] + g[0];
}

// Sources plus convective flux differences of every active direction, per
// cell, into part[nv][N].  Per direction the tile and a 3-cell halo along
// that direction are staged in LDS (velocity, pressure, sound speed, sensor
// flag, then one conserved variable at a time); every face is evaluated
// once: its hybrid decision and Lax-Friedrichs speed once for all
// variables, then its flux for each variable.
template <int NS>
__global__ __launch_bounds__(BLK, 3) void k_conv(const MechTables* __restrict__ M, const Member* __restrict__ mem,
                                              int nmem, CallArgs A, const double* __restrict__ Ub,
                                              const double* __restrict__ auxb, const double* __restrict__ srcb,
                                              const unsigned char* __restrict__ flagb, double* __restrict__ partb,
                                              double psi_c, double CT) {
  constexpr int NV = NS + 4, NAUX = 7 + NS;
  // staged arrays padded to STG * BLK so the staging loop needs no bounds
  // branch (entries past the box are written and never read)
  __shared__ double s_ud[STG * BLK], s_p[STG * BLK], s_c[STG * BLK], s_U[2][STG * BLK], s_F[2][FACE_MAX];
  __shared__ unsigned char s_fl[STG * BLK];
  const int m = find_member_tiled(mem, nmem, blockIdx.x);
  const Member& G = mem[m];
  const int t = threadIdx.x;
  int o[3];
  tile_origin(G, blockIdx.x - G.tblock_begin, o);
  const int T0 = G.tdim[0], T1 = G.tdim[1], T2 = G.tdim[2];
  const int l[3] = {t % T0, (t / T0) % T1, t / (T0 * T1)};
  const int gc[3] = {o[0] + l[0], o[1] + l[1], o[2] + l[2]};
  const bool valid = gc[0] < G.n[0] && gc[1] < G.n[1] && gc[2] < G.n[2];
  const long long N = G.N;
  const double* U = Ub + NV * G.off;
  const double* aux = auxb + NAUX * G.off;
  const unsigned char* flag = flagb + G.off;
  const long long q = valid ? lin(G, gc) : 0;
  double acc[NV];
  const double* src = srcb + (NS + 1) * G.off;
#pragma unroll
  for (int v = 0; v < NV; ++v) acc[v] = 0.0;
  if (valid) {
#pragma unroll
    for (int v = 0; v < NS; ++v) acc[v] = src[v * N + q];
    acc[NS + 3] = src[NS * N + q];
  }
  const unsigned flags = A.flags;
  for (int d = 0; d < 3; ++d) {
    if (!G.act[d]) continue;
    int B[3] = {T0, T1, T2};
    B[d] += 6;
    const int E = B[0] * B[1] * B[2];
    int FB[3] = {T0, T1, T2};
    FB[d] += 1;
    const int F = FB[0] * FB[1] * FB[2];
    const int bstride = d == 0 ? 1 : (d == 1 ? B[0] : B[0] * B[1]);
    // stage per-cell fields of the extended box; keep the global indices
    // (slots past the box load the box's last cell: in bounds, never read)
    long long qe[STG];
#pragma unroll
    for (int k = 0; k < STG; ++k) {
      const int e = t + k * BLK, ec = e < E ? e : E - 1;
      const int b[3] = {ec % B[0], (ec / B[0]) % B[1], ec / (B[0] * B[1])};
      int g[3];
#pragma unroll
      for (int a = 0; a < 3; ++a) g[a] = wrapi(o[a] + b[a] - (a == d ? 3 : 0), G.n[a]);
      qe[k] = lin(G, g);
      s_ud[e] = aux[(4 + d) * N + qe[k]];
      s_p[e] = aux[qe[k]];
      s_c[e] = aux[N + qe[k]];
      s_fl[e] = flag[qe[k]];
    }
    __syncthreads();
    // this thread's faces: hybrid decision and LF speed
    int fe0[FPT];
    bool fte[FPT];
    double fal[FPT];
#pragma unroll
    for (int k = 0; k < FPT; ++k) {
      const int f = t + k * BLK;
      fe0[k] = -1;
      fte[k] = false;
      fal[k] = 0.0;
      if (f < F) {
        const int fb[3] = {f % FB[0], (f / FB[0]) % FB[1], f / (FB[0] * FB[1])};
        // stencil positions j-3..j+2 of the tile = box positions j..j+5 along d
        fe0[k] = fb[0] + B[0] * (fb[1] + B[1] * fb[2]);
        const int e0 = fe0[k];
        bool te;
        if (flags & HTR_FORCE_TENO) te = true;
        else if (flags & HTR_FORCE_CENTRAL) te = false;
        else {
          int any = 0;
#pragma unroll
          for (int mm = 0; mm < 6; ++mm) any |= s_fl[e0 + mm * bstride];
          const double pa = s_p[e0 + 2 * bstride], pb = s_p[e0 + 3 * bstride];
          const double psi = fabs(pb - pa) / fmin(pa, pb);
          te = any != 0 || psi > psi_c;
        }
        fte[k] = te;
        if (te) {
          double al = fabs(s_ud[e0]) + s_c[e0];
#pragma unroll
          for (int mm = 1; mm < 6; ++mm) al = fmax(al, fabs(s_ud[e0 + mm * bstride]) + s_c[e0 + mm * bstride]);
          fal[k] = al;
        }
      }
    }
    int lf[3] = {l[0], l[1], l[2]};
    const int fL = lf[0] + FB[0] * (lf[1] + FB[1] * lf[2]);
    lf[d] += 1;
    const int fR = lf[0] + FB[0] * (lf[1] + FB[1] * lf[2]);
    const double xi = valid ? G.xin[d][gc[d]] : 0.0;
    // software pipeline: the next variable's staging loads are in flight
    // while the current variable's faces are evaluated (double-buffered LDS)
    double nxt[STG];
#pragma unroll
    for (int k = 0; k < STG; ++k) nxt[k] = U[qe[k]];
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      double* sU = s_U[v & 1];
      double* sF = s_F[v & 1];
#pragma unroll
      for (int k = 0; k < STG; ++k) sU[t + k * BLK] = nxt[k];
      if (v + 1 < NV) {
#pragma unroll
        for (int k = 0; k < STG; ++k) nxt[k] = U[(v + 1) * N + qe[k]];
      }
      __syncthreads();
#pragma unroll
      for (int k = 0; k < FPT; ++k) {
        if (fe0[k] < 0) continue;
        const int e0 = fe0[k];
        double f6[6], u6[6];
#pragma unroll
        for (int mm = 0; mm < 6; ++mm) {
          const int e = e0 + mm * bstride;
          u6[mm] = sU[e];
          f6[mm] = node_flux<NS>(v, d, u6[mm], s_ud[e], s_p[e]);
        }
        double Fh;
        if (!fte[k]) {
          // the face value goes through LDS before it is differenced, so its
          // last rounding cannot be fused into the difference
          Fh = (f6[0] - 8.0 * f6[1] + 37.0 * f6[2] + 37.0 * f6[3] - 8.0 * f6[4] + f6[5]) * (1.0 / 60.0);
        } else {
          Fh = teno_face(f6[0], f6[1], f6[2], f6[3], f6[4], f6[5], u6[0], u6[1], u6[2], u6[3], u6[4], u6[5],
                         fal[k], CT);
        }
        sF[t + k * BLK] = Fh;
      }
      __syncthreads();
      if (valid) acc[v] -= xi * (sF[fR] - sF[fL]);
    }
    __syncthreads();
  }
  if (valid) {
    double* part = partb + NV * G.off;
#pragma unroll
    for (int v = 0; v < NV; ++v) part[v * N + q] = acc[v];
  }
}

// Diffusive flux at the face between nodes qA and qB = A + e_d, in the sign
// with which it enters the right-hand side.  Tangential velocity derivatives
// at the face are the mean of the nodal central differences (grad).  Every
// input is loaded before any arithmetic so that all of the face's loads are
// in flight together (the kernel is bound by their latency).
template <int NS, int d>
__device__ __forceinline__ void diff_face(const MechTables* __restrict__ M, const Member& G, int cAd, long long qA,
                                          long long qB, long long N, const double* __restrict__ U,
                                          const double* __restrict__ T, const double* __restrict__ aux,
                                          const double* __restrict__ grad, double* Fd) {
  constexpr int t1 = (d + 1) % 3, t2 = (d + 2) % 3;
  const bool a1 = G.act[t1], a2 = G.act[t2];
  double uA[3], uB[3], g1A[3], g1B[3], g2A[3], g2B[3], rsA[NS], rsB[NS], DA[NS], DB[NS];
#pragma unroll
  for (int mm = 0; mm < 3; ++mm) {
    uA[mm] = aux[(4 + mm) * N + qA];
    uB[mm] = aux[(4 + mm) * N + qB];
    g1A[mm] = a1 ? grad[(3 * t1 + mm) * N + qA] : 0.0;
    g1B[mm] = a1 ? grad[(3 * t1 + mm) * N + qB] : 0.0;
    g2A[mm] = a2 ? grad[(3 * t2 + mm) * N + qA] : 0.0;
    g2B[mm] = a2 ? grad[(3 * t2 + mm) * N + qB] : 0.0;
  }
  const double muA = aux[2 * N + qA], muB = aux[2 * N + qB];
  const double laA = aux[3 * N + qA], laB = aux[3 * N + qB];
  const double TA = T[qA], TB = T[qB];
#pragma unroll
  for (int s = 0; s < NS; ++s) {
    rsA[s] = U[s * N + qA];
    rsB[s] = U[s * N + qB];
    DA[s] = aux[(7 + s) * N + qA];
    DB[s] = aux[(7 + s) * N + qB];
  }
  const double xf = G.xif[d][cAd];
  // velocity gradient at the face, g[a][mm] = d u_mm / d x_a
  double g[3][3];
#pragma unroll
  for (int mm = 0; mm < 3; ++mm) {
    g[d][mm] = xf * (uB[mm] - uA[mm]);
    g[t1][mm] = a1 ? 0.5 * (g1A[mm] + g1B[mm]) : 0.0;
    g[t2][mm] = a2 ? 0.5 * (g2A[mm] + g2B[mm]) : 0.0;
  }
  const double muf = 0.5 * (muA + muB);
  const double lamf = 0.5 * (laA + laB);
  const double divu = g[0][0] + g[1][1] + g[2][2];
  double tau[3];
#pragma unroll
  for (int mm = 0; mm < 3; ++mm) {
    tau[mm] = muf * (g[d][mm] + g[mm][d]);
    if (mm == d) tau[mm] -= (2.0 / 3.0) * muf * divu;
  }
  // species: mixture quantities at both nodes
  double rA = 0.0, rB = 0.0, nA = 0.0, nB = 0.0;
#pragma unroll
  for (int s = 0; s < NS; ++s) {
    rA += rsA[s];
    rB += rsB[s];
    nA += rsA[s] * M->iW[s];
    nB += rsB[s] * M->iW[s];
  }
  const double rhof = 0.5 * (rA + rB);
  const double inA = 1.0 / nA, inB = 1.0 / nB, irA = 1.0 / rA, irB = 1.0 / rB;
  const double iWf = 1.0 / (0.5 * (rA * inA + rB * inB));
  double term[NS];
  double corr = 0.0;
#pragma unroll
  for (int s = 0; s < NS; ++s) {
    const double Df = 0.5 * (DA[s] + DB[s]);
    // both mole fractions rounded before differencing (no FMA across the
    // difference), so a uniform composition gives exactly zero flux
    double XA, XB;
    {
#pragma clang fp contract(off)
      XA = rsA[s] * M->iW[s] * inA;
      XB = rsB[s] * M->iW[s] * inB;
    }
    const double dX = xf * (XB - XA);
    term[s] = rhof * Df * (M->W[s] * iWf) * dX;
    corr += term[s];
  }
  const double iTA = 1.0 / TA, iTB = 1.0 / TB;
  double qn = -lamf * xf * (TB - TA);
#pragma unroll
  for (int s = 0; s < NS; ++s) {
    const double Yf = 0.5 * (rsA[s] * irA + rsB[s] * irB);
    const double J = -term[s] + Yf * corr;
    const double hf = 0.5 * (M->RW[s] * TA * hRTi(M, s, TA, iTA) + M->RW[s] * TB * hRTi(M, s, TB, iTB));
    qn += J * hf;
    Fd[s] = -J;
  }
  double work = 0.0;
#pragma unroll
  for (int mm = 0; mm < 3; ++mm) {
    Fd[NS + mm] = tau[mm];
    work += tau[mm] * (0.5 * (uA[mm] + uB[mm]));
  }
  Fd[NS + 3] = work - qn;
}

// One direction of the diffusive sweep: every face of the tile (one per
// thread) into LDS, then each node adds its flux difference.
template <int NS, int d>
__device__ __forceinline__ void diff_dir(const MechTables* __restrict__ M, const Member& G, const int o[3],
                                         const int l[3], const int gc[3], bool valid, long long N,
                                         const double* __restrict__ U, const double* __restrict__ T,
                                         const double* __restrict__ aux, const double* __restrict__ grad,
                                         double (*s_Fd)[BLKF], double* acc) {
  constexpr int NV = NS + 4;
  const int t = threadIdx.x;
  int FB[3] = {G.tdim[0], G.tdim[1], G.tdim[2]};
  FB[d] += 1;
  const int F = FB[0] * FB[1] * FB[2];
  if (t < F) {
    const int fb[3] = {t % FB[0], (t / FB[0]) % FB[1], t / (FB[0] * FB[1])};
    int gA[3], gB[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const int c0 = o[a] + fb[a] - (a == d ? 1 : 0);
      gA[a] = wrapi(c0, G.n[a]);
      gB[a] = a == d ? wrapi(c0 + 1, G.n[a]) : gA[a];
    }
    double Fd[NV];
    diff_face<NS, d>(M, G, gA[d], lin(G, gA), lin(G, gB), N, U, T, aux, grad, Fd);
#pragma unroll
    for (int v = 0; v < NV; ++v) s_Fd[v][t] = Fd[v];
  }
  __syncthreads();
  if (valid) {
    int lf[3] = {l[0], l[1], l[2]};
    const int fL = lf[0] + FB[0] * (lf[1] + FB[1] * lf[2]);
    lf[d] += 1;
    const int fR = lf[0] + FB[0] * (lf[1] + FB[1] * lf[2]);
    const double xi = G.xin[d][gc[d]];
#pragma unroll
    for (int v = 0; v < NV; ++v) acc[v] += xi * (s_Fd[v][fR] - s_Fd[v][fL]);
  }
  __syncthreads();
}

// Diffusive flux differences (each face once, exchanged through LDS) added
// to part, then the SSP-RK3 stage combination (or dU/dt when rhs_only).
// BLKF threads: the first BLK own the tile's cells; every thread owns one
// face per direction (a tile has at most BLKF faces along any axis).
template <int NS>
__global__ __launch_bounds__(BLKF, 3) void k_diff(const MechTables* __restrict__ M,
                                                       const Member* __restrict__ mem, int nmem, CallArgs A,
                                                       const double* __restrict__ Ub, const double* Unb,
                                                       const double* __restrict__ Tb, const double* __restrict__ auxb,
                                                       const double* __restrict__ gradb,
                                                       const double* __restrict__ partb, double* outb, double ca,
                                                       double cb, int rhs_only) {
  constexpr int NV = NS + 4, NAUX = 7 + NS;
  __shared__ double s_Fd[NV][BLKF];
  const int m = find_member_tiled(mem, nmem, blockIdx.x);
  const Member& G = mem[m];
  const int t = threadIdx.x;
  int o[3];
  tile_origin(G, blockIdx.x - G.tblock_begin, o);
  const int T0 = G.tdim[0], T1 = G.tdim[1];
  const int l[3] = {t % T0, (t / T0) % T1, t / (T0 * T1)};
  const int gc[3] = {o[0] + l[0], o[1] + l[1], o[2] + l[2]};
  const bool valid = t < BLK && gc[0] < G.n[0] && gc[1] < G.n[1] && gc[2] < G.n[2];
  const long long N = G.N;
  const double* U = Ub + NV * G.off;
  const double* T = Tb + G.off;
  const double* aux = auxb + NAUX * G.off;
  const double* grad = gradb + 9 * G.off;
  const long long q = valid ? lin(G, gc) : 0;
  double acc[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) acc[v] = 0.0;
  if (!(A.flags & HTR_VISC_OFF)) {
    if (G.act[0]) diff_dir<NS, 0>(M, G, o, l, gc, valid, N, U, T, aux, grad, s_Fd, acc);
    if (G.act[1]) diff_dir<NS, 1>(M, G, o, l, gc, valid, N, U, T, aux, grad, s_Fd, acc);
    if (G.act[2]) diff_dir<NS, 2>(M, G, o, l, gc, valid, N, U, T, aux, grad, s_Fd, acc);
  }
  if (!valid) return;
  // every load before the first store: out may be the same array as U^n, so
  // the compiler could not otherwise move a later variable's loads above an
  // earlier variable's store, and each variable would cost a memory round trip
  const double* part = partb + NV * G.off;
  double* out = outb + NV * G.off;
  double pv[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) pv[v] = part[v * N + q];
  if (rhs_only) {
#pragma unroll
    for (int v = 0; v < NV; ++v) out[v * N + q] = pv[v] + acc[v];
  } else {
    const double dt = A.dt_dev[m];
    const double* Un = Unb + NV * G.off;
    double uv[NV], unv[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      uv[v] = U[v * N + q];
      unv[v] = ca != 0.0 ? Un[v * N + q] : 0.0;
    }
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      const double base = uv[v] + dt * (pv[v] + acc[v]);
      out[v * N + q] = ca != 0.0 ? ca * unv[v] + cb * base : cb * base;
    }
  }
}

template <int NS>
static hipError_t conv_t(const MechTables* M, const Member* mem, int nmem, int ntblocks, const CallArgs& a,
                         const double* U, const double* aux, const double* src, const unsigned char* flag,
                         double* part, double psi_c, double CT, hipStream_t s) {
  hipLaunchKernelGGL(k_conv<NS>, dim3(ntblocks), dim3(BLK), 0, s, M, mem, nmem, a, U, aux, src, flag, part, psi_c,
                     CT);
  return hipGetLastError();
}

template <int NS>
static hipError_t diff_t(const MechTables* M, const Member* mem, int nmem, int ntblocks, const CallArgs& a,
                         const double* U, const double* Un, const double* T, const double* aux, const double* grad,
                         const double* part, double* out, double ca, double cb, int rhs_only, hipStream_t s) {
  hipLaunchKernelGGL(k_diff<NS>, dim3(ntblocks), dim3(BLKF), 0, s, M, mem, nmem, a, U, Un, T, aux, grad, part, out,
                     ca, cb, rhs_only);
  return hipGetLastError();
}

hipError_t launch_conv(int ns, const MechTables* M, const Member* mem, int nmem, int ntblocks, const CallArgs& a,
                       const double* U, const double* aux, const double* src, const unsigned char* flag, double* part,
                       double psi_c, double CT, hipStream_t s) {
#define C_(NS) conv_t<NS>(M, mem, nmem, ntblocks, a, U, aux, src, flag, part, psi_c, CT, s)
  HTR_NS_SWITCH(ns, C_);
#undef C_
}

hipError_t launch_diff(int ns, const MechTables* M, const Member* mem, int nmem, int ntblocks, const CallArgs& a,
                       const double* U, const double* Un, const double* T, const double* aux, const double* grad,
                       const double* part, double* out, double ca, double cb, int rhs_only, hipStream_t s) {
#define C_(NS) diff_t<NS>(M, mem, nmem, ntblocks, a, U, Un, T, aux, grad, part, out, ca, cb, rhs_only, s)
  HTR_NS_SWITCH(ns, C_);
#undef C_
}

}  // namespace htr
