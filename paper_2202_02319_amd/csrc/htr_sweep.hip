// Flux sweep: for every cell, the flux differences along every active
// direction of the hybrid TENO6/central convective flux and of the
// second-order diffusive flux, plus the chemistry and laser sources, fused
// with the SSP-RK3 stage combination (or written as dU/dt).
//
// Paper (arXiv 2202.02319) Methods › Numerical method: conservative finite differences of the
// mapped equations (rectilinear metrics), TENO6 for the inviscid fluxes,
// second-order central differences for the diffusive fluxes; Methods › Solver eqs.
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


// Tile shapes of the tiled kernels: 256 cells.  Default 16 x 4 x 4 on 3-D
// grids, 16 x 16 over the two active axes of 2-D grids, 256 along a 1-D
// grid; other shapes are accepted if every staging buffer holds them.
void default_tile_shape(const int act[3], int t[3]) {
  const int na = act[0] + act[1] + act[2];
  t[0] = t[1] = t[2] = 1;
  if (na == 3) {
    t[0] = 16; t[1] = 4; t[2] = 4;
  } else if (na == 2) {
    for (int a = 0; a < 3; ++a) t[a] = act[a] ? 16 : 1;
  } else if (na == 1) {
    for (int a = 0; a < 3; ++a) t[a] = act[a] ? 256 : 1;
  } else {
    t[0] = 256;
  }
}

bool tile_shape_ok(const int act[3], const int t[3], const char** why) {
  const char* w = nullptr;
  const int na = act[0] + act[1] + act[2];
  if (t[0] < 1 || t[1] < 1 || t[2] < 1 || t[0] * t[1] * t[2] != BLK) w = "tile must have 256 cells";
  for (int a = 0; a < 3 && !w; ++a)
    if (na > 0 && !act[a] && t[a] != 1) w = "tile extends along an inactive axis";
  if (!w) {
    long box = 0, arms = 0, faces = 0;
    for (int d = 0; d < 3; ++d) {
      if (!act[d]) continue;
      const long cs = BLK / t[d];   // cross-section of the tile normal to d
      box += cs * (t[d] + 6);
      arms += 6 * cs;
      faces += cs * (t[d] + 1);
      if (!w && cs * (t[d] + 1) > BLKF) w = "too many faces along one axis for the diffusive sweep";
      if (!w && (cs * (t[d] + 10) > EXTA || cs * (t[d] + 5) > FACEA))
        w = "halo box too large for the convective adjoint";
    }
    if (!w && (box > XBOX_MAX || arms > XARM_MAX || faces > XFACE_MAX))
      w = "cross staging too large for the convective sweep";
  }
  if (why) *why = w;
  return w == nullptr;
}

void set_tiles(Member& M, const int* shape, int* tblocks) {
  const int act[3] = {M.act[0], M.act[1], M.act[2]};
  int t[3];
  if (shape) {
    t[0] = shape[0]; t[1] = shape[1]; t[2] = shape[2];
  } else {
    default_tile_shape(act, t);
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

__device__ __forceinline__ long long lin(const Member& G, const int g[3]) {
  return ((long long)g[2] * G.n[1] + g[1]) * G.n[0] + g[0];
}

// Cross staging of the convective sweep: the tile plus a 3-cell halo on both
// sides along every active axis.  Each staged value is loaded once and
// written into the line-contiguous box of every direction that uses it (the
// tile's own cells into all of them).
constexpr int APT = (XARM_MAX + BLK - 1) / BLK;
constexpr int XFPT = (XFACE_MAX + BLK - 1) / BLK;

// Sources plus convective flux differences of every active direction, per
// cell, into part[nv][N] (TENO6, or WENO3-Z with HTR_WENO3Z, at the faces the
// hybrid switch marks).  The sensor flag, pressure and LF node speed of the
// cross are staged once and every face of the tile takes its hybrid decision
// and Lax-Friedrichs speed once for all variables.  Then, per conserved
// variable, each staged cell's value and its node flux along each axis are
// written once (the loading thread keeps that cell's velocity and pressure
// in registers), and every face flux is evaluated once from them, all
// directions together.
template <int NS, bool TAPE>
__device__ __forceinline__ void conv_tile(int bl, const Member* __restrict__ mem, int nmem, const CallArgs& A,
                                          const double* __restrict__ Ub, const double* __restrict__ auxb,
                                          const double* __restrict__ srcb, const unsigned char* __restrict__ flagb,
                                          double* __restrict__ partb, unsigned char* __restrict__ bitsb, double psi_c,
                                          double CT) {
  constexpr int NV = NS + 4, NAUX = 7 + NS;
  // one spare slot past every box: a write target for threads without a halo cell
  __shared__ double s_U[XBOX_MAX + 1], s_Fn[XBOX_MAX + 1], s_F[2][XFACE_MAX];
  __shared__ double s_al[XFACE_MAX];   // LF speed of the TENO faces
  __shared__ short s_tl[XFACE_MAX];    // the tile's TENO faces
  __shared__ int s_nt;
  // before the variable loop the same memory holds the LF node speed, the
  // pressure and the sensor flags
  double* s_spd = s_U;
  double* s_p = s_Fn;
  unsigned char* s_fl = reinterpret_cast<unsigned char*>(&s_F[0][0]);
  const int m = find_member_tiled(mem, nmem, bl);
  const Member& G = mem[m];
  const int t = threadIdx.x;
  int o[3];
  tile_origin(G, bl - G.tblock_begin, o);
  const int T[3] = {G.tdim[0], G.tdim[1], G.tdim[2]};
  const int TT = T[0] * T[1] * T[2];
  const bool act[3] = {G.act[0] != 0, G.act[1] != 0, G.act[2] != 0};
  // layout of the boxes, the halo cells and the faces
  int boff[3], foff[3], aoff[3];
  int Ftot, Atot;
  {
    int eo = 0, fo = 0, ao = 0;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      boff[d] = eo;
      foff[d] = fo;
      aoff[d] = ao;
      if (act[d]) {
        eo += TT / T[d] * (T[d] + 6);
        fo += TT / T[d] * (T[d] + 1);
        ao += 6 * (TT / T[d]);
      }
    }
    Ftot = fo;
    Atot = ao;
  }
  // slot of box position b in box d
  auto bslot = [&](int d, int b0, int b1, int b2) {
    const int B0 = T[0] + (d == 0 ? 6 : 0), B1 = T[1] + (d == 1 ? 6 : 0);
    return boff[d] + b0 + B0 * (b1 + B1 * b2);
  };
  // this thread's cell
  const int l[3] = {t % T[0], (t / T[0]) % T[1], t / (T[0] * T[1])};
  const int gc[3] = {o[0] + l[0], o[1] + l[1], o[2] + l[2]};
  const bool valid = gc[0] < G.n[0] && gc[1] < G.n[1] && gc[2] < G.n[2];
  const long long N = G.N;
  const double* U = Ub + NV * G.off;
  const double* aux = auxb + NAUX * G.off;
  const unsigned char* flag = flagb + G.off;
  const double* src = srcb + (NS + 1) * G.off;
  // TENO cut-off patterns per axis, variable and face (indexed by the face's
  // upper cell), when a forward tape asks for them
  unsigned char* bits = TAPE ? bitsb + 3LL * NV * G.off : nullptr;
  long long qc;
  {
    int g[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) g[a] = wrapi(gc[a], G.n[a]);
    qc = lin(G, g);
  }
  int cs[3];
#pragma unroll
  for (int d = 0; d < 3; ++d)
    cs[d] = act[d] ? bslot(d, l[0] + (d == 0 ? 3 : 0), l[1] + (d == 1 ? 3 : 0), l[2] + (d == 2 ? 3 : 0))
                   : XBOX_MAX;
  // this thread's halo cells (box slot, global index, axis)
  int as[APT], ax[APT];
  long long aq[APT];
#pragma unroll
  for (int k = 0; k < APT; ++k) {
    const int a = t + k * BLK;
    as[k] = XBOX_MAX;
    aq[k] = qc;
    ax[k] = 0;
    if (a < Atot) {
      const int d = a < aoff[1] ? 0 : (a < aoff[2] ? 1 : 2);
      const int r = a - aoff[d], S = TT / T[d];
      const int j6 = r / S, cidx = r % S;
      const int side = j6 / 3, j = j6 - 3 * side;
      int lc[3];
      lc[d] = side == 0 ? j - 3 : T[d] + j;
      const int e1 = d == 0 ? 1 : 0, e2 = d == 2 ? 1 : 2;   // the two other axes, in order
      lc[e1] = cidx % T[e1];
      lc[e2] = cidx / T[e1];
      int g[3];
#pragma unroll
      for (int c = 0; c < 3; ++c) g[c] = wrapi(o[c] + lc[c], G.n[c]);
      aq[k] = lin(G, g);
      ax[k] = d;
      int b[3] = {lc[0], lc[1], lc[2]};
      b[d] += 3;
      as[k] = bslot(d, b[0], b[1], b[2]);
    }
  }
  // velocity along the box axis and pressure of every staged cell, kept in
  // registers by the thread that stages it
  double cu[3], cp, hu[APT], hp[APT];
  {
    cp = aux[qc];
    const double cc = aux[N + qc];
    const unsigned char fc = flag[qc];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      cu[d] = aux[(4 + d) * N + qc];
      s_spd[cs[d]] = fabs(cu[d]) + cc;
      s_p[cs[d]] = cp;
      s_fl[cs[d]] = fc;
    }
#pragma unroll
    for (int k = 0; k < APT; ++k) {
      hu[k] = aux[(4 + ax[k]) * N + aq[k]];
      hp[k] = aux[aq[k]];
      s_spd[as[k]] = fabs(hu[k]) + aux[N + aq[k]];
      s_p[as[k]] = hp[k];
      s_fl[as[k]] = flag[aq[k]];
    }
  }
  if (t == 0) s_nt = 0;
  __syncthreads();
  // face f of the list: axis, stencil start slot (stencil positions j-3..j+2
  // of the tile = box positions j..j+5 along d), stride along the axis, and
  // tile position of the face's upper cell
  auto face = [&](int f, int& d, int& e0, int& bs, int fb[3]) {
    d = f < foff[1] ? 0 : (f < foff[2] ? 1 : 2);
    const int r = f - foff[d];
    const int F0 = T[0] + (d == 0 ? 1 : 0), F1 = T[1] + (d == 1 ? 1 : 0);
    fb[0] = r % F0;
    fb[1] = (r / F0) % F1;
    fb[2] = r / (F0 * F1);
    e0 = bslot(d, fb[0], fb[1], fb[2]);
    const int B0 = T[0] + (d == 0 ? 6 : 0), B1 = T[1] + (d == 1 ? 6 : 0);
    bs = d == 0 ? 1 : (d == 1 ? B0 : B0 * B1);
  };
  // this thread's faces: stencil start slot, stride, hybrid decision; TENO
  // faces are also listed (with their Lax-Friedrichs speed) so that each
  // variable's TENO work is spread evenly over the block
  int fe0[XFPT], fst[XFPT];
  unsigned fte = 0;
  const unsigned flags = A.flags;
#pragma unroll
  for (int k = 0; k < XFPT; ++k) {
    const int f = t + k * BLK;
    fe0[k] = -1;
    fst[k] = 1;
    if (f < Ftot) {
      int d, e0, bs, fb[3];
      face(f, d, e0, bs, fb);
      fe0[k] = e0;
      fst[k] = bs;
      bool te;
      if (flags & HTR_FORCE_TENO) te = true;
      else if (flags & HTR_FORCE_CENTRAL) te = false;
      else {
        int any = 0;
#pragma unroll
        for (int mm = 0; mm < 6; ++mm) any |= s_fl[e0 + mm * bs];
        const double pa = s_p[e0 + 2 * bs], pb = s_p[e0 + 3 * bs];
        const double psi = fabs(pb - pa) / fmin(pa, pb);
        te = any != 0 || psi > psi_c;
      }
      if (te) {
        fte |= 1u << k;
        double al = s_spd[e0];
#pragma unroll
        for (int mm = 1; mm < 6; ++mm) al = fmax(al, s_spd[e0 + mm * bs]);
        s_al[f] = al;
        s_tl[atomicAdd(&s_nt, 1)] = (short)f;
      }
    }
  }
  // this cell's two faces per axis in the face list, and the metric
  int fL[3], fR[3];
  double xi[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    int lf[3] = {l[0], l[1], l[2]};
    const int F0 = T[0] + (d == 0 ? 1 : 0), F1 = T[1] + (d == 1 ? 1 : 0);
    fL[d] = foff[d] + lf[0] + F0 * (lf[1] + F1 * lf[2]);
    lf[d] += 1;
    fR[d] = foff[d] + lf[0] + F0 * (lf[1] + F1 * lf[2]);
    xi[d] = (valid && act[d]) ? G.xin[d][gc[d]] : 0.0;
  }
  const long long q = valid ? qc : 0;
  // software pipeline: the next variable's staging loads (and source) are in
  // flight while the current variable's faces are evaluated
  double ncore = U[qc], narm[APT];
#pragma unroll
  for (int k = 0; k < APT; ++k) narm[k] = U[aq[k]];
  double nsrc = valid ? src[q] : 0.0;
  double* part = partb + NV * G.off;
  __syncthreads();   // the decisions have read the node speeds, pressures and flags
  const int nteno = s_nt;
#pragma unroll 1
  for (int v = 0; v < NV; ++v) {
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      s_U[cs[d]] = ncore;
      s_Fn[cs[d]] = node_flux<NS>(v, d, ncore, cu[d], cp);
    }
#pragma unroll
    for (int k = 0; k < APT; ++k) {
      s_U[as[k]] = narm[k];
      s_Fn[as[k]] = node_flux<NS>(v, ax[k], narm[k], hu[k], hp[k]);
    }
    const double acc0 = nsrc;
    if (v + 1 < NV) {
      ncore = U[(v + 1) * N + qc];
#pragma unroll
      for (int k = 0; k < APT; ++k) narm[k] = U[(v + 1) * N + aq[k]];
      const int sv = v + 1 < NS ? v + 1 : (v + 1 == NS + 3 ? NS : -1);
      nsrc = (valid && sv >= 0) ? src[sv * N + q] : 0.0;
    }
    __syncthreads();
    double* sF = s_F[v & 1];
    // central faces: this thread's own
#pragma unroll
    for (int k = 0; k < XFPT; ++k) {
      if (fe0[k] < 0 || ((fte >> k) & 1u)) continue;
      const int e0 = fe0[k], bs = fst[k];
      double f6[6];
#pragma unroll
      for (int mm = 0; mm < 6; ++mm) f6[mm] = s_Fn[e0 + mm * bs];
      // the face value goes through LDS before it is differenced, so its
      // last rounding cannot be fused into the difference
      sF[t + k * BLK] =
          (f6[0] - 8.0 * f6[1] + 37.0 * f6[2] + 37.0 * f6[3] - 8.0 * f6[4] + f6[5]) * (1.0 / 60.0);
    }
    // TENO faces: the tile's list, dealt round-robin over the block
    for (int i = t; i < nteno; i += BLK) {
      const int f = s_tl[i];
      int d, e0, bs, fb[3];
      face(f, d, e0, bs, fb);
      const double al = s_al[f];
      double fp[6], fm[6];
#pragma unroll
      for (int mm = 0; mm < 6; ++mm) {
        const double f6 = s_Fn[e0 + mm * bs], u6 = s_U[e0 + mm * bs];
        fp[mm] = 0.5 * (f6 + al * u6);
        fm[5 - mm] = 0.5 * (f6 - al * u6);
      }
      if (flags & HTR_WENO3Z) {
        sF[f] = weno3z(fp) + weno3z(fm);
        continue;
      }
      double wp[4], qp[4], wm[4], qm[4];
      teno6_core(fp, CT, wp, qp);
      teno6_core(fm, CT, wm, qm);
      sF[f] = (wp[0] * qp[0] + wp[1] * qp[1] + wp[2] * qp[2] + wp[3] * qp[3]) +
              (wm[0] * qm[0] + wm[1] * qm[1] + wm[2] * qm[2] + wm[3] * qm[3]);
      if (TAPE) {
        // the cut-off pattern: bits 0-3 the + side's kept candidates, 4-7 the - side's
        unsigned pat = 0;
#pragma unroll
        for (int k = 0; k < 4; ++k) pat |= (wp[k] > 0.0 ? 1u : 0u) << k | (wm[k] > 0.0 ? 1u : 0u) << (k + 4);
        int g[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) g[c] = wrapi(o[c] + fb[c], G.n[c]);
        bits[(long long)(d * NV + v) * N + lin(G, g)] = (unsigned char)pat;
      }
    }
    __syncthreads();
    if (valid) {
      double acc = acc0;
#pragma unroll
      for (int d = 0; d < 3; ++d)
        if (act[d]) acc -= xi[d] * (sF[fR[d]] - sF[fL[d]]);
      part[v * N + q] = acc;
    }
  }
}

// MODE 0: one block per tile; 1: persistent blocks striding over the nlog
// tiles; 2: one block per tile, also writing the TENO cut-off patterns.
template <int NS, int MODE>
__global__ __launch_bounds__(BLK, 2) void k_conv(const MechTables* __restrict__ M, const Member* __restrict__ mem,
                                              int nmem, int nlog, CallArgs A, const double* __restrict__ Ub,
                                              const double* __restrict__ auxb, const double* __restrict__ srcb,
                                              const unsigned char* __restrict__ flagb, double* __restrict__ partb,
                                              unsigned char* __restrict__ bitsb, double psi_c, double CT) {
  if (MODE != 1) {
    conv_tile<NS, MODE == 2>(blockIdx.x, mem, nmem, A, Ub, auxb, srcb, flagb, partb, bitsb, psi_c, CT);
    return;
  }
  for (int bl = blockIdx.x; bl < nlog; bl += gridDim.x) {
    conv_tile<NS, false>(bl, mem, nmem, A, Ub, auxb, srcb, flagb, partb, bitsb, psi_c, CT);
    __syncthreads();   // the next tile reuses the LDS
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
  double uA[3], uB[3], g1A[3], g1B[3], g2A[3], g2B[3];
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
    const double ra = U[s * N + qA], rb = U[s * N + qB];
    rA += ra;
    rB += rb;
    nA += ra * M->iW[s];
    nB += rb * M->iW[s];
  }
  const double rhof = 0.5 * (rA + rB);
  const double inA = 1.0 / nA, inB = 1.0 / nB, irA = 1.0 / rA, irB = 1.0 / rB;
  const double iWf = 1.0 / (0.5 * (rA * inA + rB * inB));
  // two passes over the species (the correction flux, then each flux),
  // reloading per-species inputs rather than holding them in registers
  auto term = [&](int s) -> double {
    const double Df = 0.5 * (aux[(7 + s) * N + qA] + aux[(7 + s) * N + qB]);
    // both mole fractions rounded before differencing (no FMA across the
    // difference), so a uniform composition gives exactly zero flux
    double XA, XB;
    {
#pragma clang fp contract(off)
      XA = U[s * N + qA] * M->iW[s] * inA;
      XB = U[s * N + qB] * M->iW[s] * inB;
    }
    const double dX = xf * (XB - XA);
    return rhof * Df * (M->W[s] * iWf) * dX;
  };
  double corr = 0.0;
#pragma unroll
  for (int s = 0; s < NS; ++s) corr += term(s);
  const double iTA = 1.0 / TA, iTB = 1.0 / TB;
  double qn = -lamf * xf * (TB - TA);
#pragma unroll
  for (int s = 0; s < NS; ++s) {
    const double Yf = 0.5 * (U[s * N + qA] * irA + U[s * N + qB] * irB);
    const double J = -term(s) + Yf * corr;
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
__device__ __forceinline__ void diff_tile(int bl, const MechTables* __restrict__ M, const Member* __restrict__ mem,
                                          int nmem, const CallArgs& A, const double* __restrict__ Ub,
                                          const double* Unb, const double* __restrict__ Tb,
                                          const double* __restrict__ auxb, const double* __restrict__ gradb,
                                          const double* __restrict__ partb, double* outb, double ca, double cb,
                                          int rhs_only) {
  constexpr int NV = NS + 4, NAUX = 7 + NS;
  __shared__ double s_Fd[NV][BLKF];
  const int m = find_member_tiled(mem, nmem, bl);
  const Member& G = mem[m];
  const int t = threadIdx.x;
  int o[3];
  tile_origin(G, bl - G.tblock_begin, o);
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

template <int NS, bool PERSIST>
__global__ __launch_bounds__(BLKF, 3) void k_diff(const MechTables* __restrict__ M, const Member* __restrict__ mem,
                                                  int nmem, int nlog, CallArgs A, const double* __restrict__ Ub,
                                                  const double* Unb, const double* __restrict__ Tb,
                                                  const double* __restrict__ auxb, const double* __restrict__ gradb,
                                                  const double* __restrict__ partb, double* outb, double ca,
                                                  double cb, int rhs_only) {
  if (!PERSIST) {
    diff_tile<NS>(blockIdx.x, M, mem, nmem, A, Ub, Unb, Tb, auxb, gradb, partb, outb, ca, cb, rhs_only);
    return;
  }
  for (int bl = blockIdx.x; bl < nlog; bl += gridDim.x) {
    diff_tile<NS>(bl, M, mem, nmem, A, Ub, Unb, Tb, auxb, gradb, partb, outb, ca, cb, rhs_only);
    __syncthreads();   // the next tile reuses the LDS
  }
}

static int grid_of(int nblocks, int grid) { return (grid <= 0 || grid > nblocks) ? nblocks : grid; }

template <int NS>
static hipError_t conv_t(const MechTables* M, const Member* mem, int nmem, int ntblocks, int grid, const CallArgs& a,
                         const double* U, const double* aux, const double* src, const unsigned char* flag,
                         double* part, unsigned char* bits, double psi_c, double CT, hipStream_t s) {
  if (bits)   // taped: one block per tile
    hipLaunchKernelGGL((k_conv<NS, 2>), dim3(ntblocks), dim3(BLK), 0, s, M, mem, nmem, ntblocks, a, U, aux, src, flag,
                       part, bits, psi_c, CT);
  else if (grid < ntblocks)
    hipLaunchKernelGGL((k_conv<NS, 1>), dim3(grid), dim3(BLK), 0, s, M, mem, nmem, ntblocks, a, U, aux, src, flag,
                       part, bits, psi_c, CT);
  else
    hipLaunchKernelGGL((k_conv<NS, 0>), dim3(grid), dim3(BLK), 0, s, M, mem, nmem, ntblocks, a, U, aux, src, flag,
                       part, bits, psi_c, CT);
  return hipGetLastError();
}

template <int NS>
static hipError_t diff_t(const MechTables* M, const Member* mem, int nmem, int ntblocks, int grid, const CallArgs& a,
                         const double* U, const double* Un, const double* T, const double* aux, const double* grad,
                         const double* part, double* out, double ca, double cb, int rhs_only, hipStream_t s) {
  if (grid < ntblocks)
    hipLaunchKernelGGL((k_diff<NS, true>), dim3(grid), dim3(BLKF), 0, s, M, mem, nmem, ntblocks, a, U, Un, T, aux,
                       grad, part, out, ca, cb, rhs_only);
  else
    hipLaunchKernelGGL((k_diff<NS, false>), dim3(grid), dim3(BLKF), 0, s, M, mem, nmem, ntblocks, a, U, Un, T, aux,
                       grad, part, out, ca, cb, rhs_only);
  return hipGetLastError();
}

hipError_t launch_conv(int ns, const MechTables* M, const Member* mem, int nmem, int ntblocks, int grid,
                       const CallArgs& a, const double* U, const double* aux, const double* src,
                       const unsigned char* flag, double* part, unsigned char* bits, double psi_c, double CT,
                       hipStream_t s) {
  grid = grid_of(ntblocks, grid);
#define C_(NS) conv_t<NS>(M, mem, nmem, ntblocks, grid, a, U, aux, src, flag, part, bits, psi_c, CT, s)
  HTR_NS_SWITCH(ns, C_);
#undef C_
}

hipError_t launch_diff(int ns, const MechTables* M, const Member* mem, int nmem, int ntblocks, int grid,
                       const CallArgs& a, const double* U, const double* Un, const double* T, const double* aux,
                       const double* grad, const double* part, double* out, double ca, double cb, int rhs_only,
                       hipStream_t s) {
  grid = grid_of(ntblocks, grid);
#define C_(NS) diff_t<NS>(M, mem, nmem, ntblocks, grid, a, U, Un, T, aux, grad, part, out, ca, cb, rhs_only, s)
  HTR_NS_SWITCH(ns, C_);
#undef C_
}

}  // namespace htr
