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
// Two tiled kernels per stage: k_conv (sources and convective flux
// differences, one block per 256-cell tile with the tile and its halo staged
// in LDS) and k_diff (diffusive flux differences and the stage update, one
// block per 192-cell tile of its own).  Every face is evaluated once, so the
// scheme is exactly conservative.

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
      if (!w && (cs * (t[d] + 10) > EXTA || cs * (t[d] + 5) > FACEA))
        w = "halo box too large for the convective adjoint";
    }
    if (!w && (box > XBOX_MAX || arms > XARM_MAX || faces > XFACE_MAX))
      w = "cross staging too large for the convective sweep";
  }
  if (why) *why = w;
  return w == nullptr;
}

// The diffusive sweep's tile for the active axes: 16 x 4 x 3 in 3-D (204,
// 240 and 256 faces), 16 x 12 over the two active axes of 2-D grids (204 and
// 208), 192 along a 1-D grid.
static void diff_tile_shape(const int act[3], int t[3]) {
  const int na = act[0] + act[1] + act[2];
  t[0] = t[1] = t[2] = 1;
  if (na == 3) {
    t[0] = 16; t[1] = 4; t[2] = 3;
  } else if (na == 2) {
    int k = 0;
    for (int a = 0; a < 3; ++a)
      if (act[a]) t[a] = k++ == 0 ? 16 : 12;
  } else if (na == 1) {
    for (int a = 0; a < 3; ++a) t[a] = act[a] ? DTILE : 1;
  } else {
    t[0] = DTILE;
  }
}

void set_tiles(Member& M, const int* shape, int* tblocks, int* dtblocks) {
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
  int dt[3];
  diff_tile_shape(act, dt);
  int nd = 1;
  for (int a = 0; a < 3; ++a) {
    M.dtdim[a] = dt[a];
    M.dntile[a] = (M.n[a] + dt[a] - 1) / dt[a];
    nd *= M.dntile[a];
  }
  M.dtblock_begin = *dtblocks;
  M.ndtblocks = nd;
  *dtblocks += nd;
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
//
// KIND 0: every tile.  KIND 1 (the lean variant): a tile none of whose faces
// takes the TENO path is done here with the central faces alone (no staged
// conserved values, no TENO state, so fewer registers and more waves per
// SIMD); a tile with any TENO face is only marked in tcls[bl].  KIND 2: the
// marked tiles, in full; the others return at once.
template <int NS, bool TAPE, int KIND>
__device__ __forceinline__ void conv_tile(int bl, const Member* __restrict__ mem, int nmem, const CallArgs& A,
                                          const double* __restrict__ Ub, const double* __restrict__ auxb,
                                          const double* __restrict__ srcb, const unsigned char* __restrict__ flagb,
                                          double* __restrict__ partb, unsigned char* __restrict__ bitsb, double psi_c,
                                          double CT, unsigned char* __restrict__ tcls) {
  constexpr int NV = NS + 4, NAUX = 7 + NS;
  constexpr bool LEAN = KIND == 1;
  static_assert(!(TAPE && KIND != 0), "the taped sweep runs every tile in full");
  if constexpr (KIND == 2) {
    if (tcls[bl] == 0) return;   // the lean variant has done this tile
  }
  // one spare slot past every box: a write target for threads without a halo cell
  __shared__ double s_U[XBOX_MAX + 1], s_Fn[XBOX_MAX + 1], s_F[2][XFACE_MAX];
  __shared__ double s_al[XFACE_MAX];   // LF speed of the TENO faces, in list order
  // the tile's TENO faces: stencil start slot (bits 0-11), face index
  // (12-21) and stencil stride in its box (22-31)
  __shared__ unsigned s_tl[XFACE_MAX];
  __shared__ int s_tq[TAPE ? XFACE_MAX : 1];             // taped: the face's tape index (upper cell)
  __shared__ unsigned char s_td[TAPE ? XFACE_MAX : 1];   // taped: the face's axis
  __shared__ int s_nt;
  __shared__ double s_w[16][4];        // TENO6 normalised weights of every cut-off pattern
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
  if constexpr (LEAN) {
    // every node of the cross lies in the stencil of one of the tile's faces,
    // so a flagged node means a TENO face: such tiles are left to the full
    // variant after one barrier (the pressure-jump test follows below)
    int any = (A.flags & HTR_FORCE_TENO) != 0;
    if (!(A.flags & (HTR_FORCE_TENO | HTR_FORCE_CENTRAL))) {
      any = flag[qc];
#pragma unroll
      for (int k = 0; k < APT; ++k) any |= flag[aq[k]];
    }
    if (__syncthreads_or(any)) {
      if (t == 0) tcls[bl] = 1;
      return;
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
      if constexpr (!LEAN) s_spd[cs[d]] = fabs(cu[d]) + cc;
      s_p[cs[d]] = cp;
      s_fl[cs[d]] = fc;
    }
#pragma unroll
    for (int k = 0; k < APT; ++k) {
      hu[k] = aux[(4 + ax[k]) * N + aq[k]];
      hp[k] = aux[aq[k]];
      if constexpr (!LEAN) s_spd[as[k]] = fabs(hu[k]) + aux[N + aq[k]];
      s_p[as[k]] = hp[k];
      s_fl[as[k]] = flag[aq[k]];
    }
    (void)cc;
  }
  if (t == 0) s_nt = 0;
  if constexpr (!LEAN) {
    if (t < 16) teno6_weights(t, s_w[t]);
  }
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
  // a stride is at most T[0] T[1] <= BLK cells
  static_assert(XBOX_MAX < (1 << 12) && XFACE_MAX < (1 << 10) && BLK < (1 << 10), "TENO list packing");
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
      if (LEAN && te) {
        atomicOr(&s_nt, 1);
      } else if (te) {
        fte |= 1u << k;
        double al = s_spd[e0];
#pragma unroll
        for (int mm = 1; mm < 6; ++mm) al = fmax(al, s_spd[e0 + mm * bs]);
        const int slot = atomicAdd(&s_nt, 1);
        s_al[slot] = al;
        s_tl[slot] = (unsigned)e0 | (unsigned)f << 12 | (unsigned)bs << 22;
        if (TAPE) {
          int g[3];
#pragma unroll
          for (int c = 0; c < 3; ++c) g[c] = wrapi(o[c] + fb[c], G.n[c]);
          s_tq[slot] = (int)lin(G, g);
          s_td[slot] = (unsigned char)d;
        }
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
  if constexpr (LEAN) {
    if (t == 0) tcls[bl] = nteno != 0;
    if (nteno != 0) return;   // uniform: the full variant does this tile
  }
#pragma unroll 1
  for (int v = 0; v < NV; ++v) {
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      if constexpr (!LEAN) s_U[cs[d]] = ncore;
      s_Fn[cs[d]] = node_flux<NS>(v, d, ncore, cu[d], cp);
    }
#pragma unroll
    for (int k = 0; k < APT; ++k) {
      if constexpr (!LEAN) s_U[as[k]] = narm[k];
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
    for (int i = t; i < (LEAN ? 0 : nteno); i += BLK) {
      const unsigned pk = s_tl[i];
      const int e0 = pk & 0xfffu, f = (pk >> 12) & 0x3ffu, bs = pk >> 22;
      const double al = s_al[i];
      // the two sides of the split, without their factor 1/2
      double hp[6], hm[6];
#pragma unroll
      for (int mm = 0; mm < 6; ++mm) {
        const double f6 = s_Fn[e0 + mm * bs], u6 = s_U[e0 + mm * bs];
        hp[mm] = fma(al, u6, f6);
        hm[5 - mm] = fma(-al, u6, f6);
      }
      if (flags & HTR_WENO3Z) {
        sF[f] = weno3z_h(hp) + weno3z_h(hm);
        continue;
      }
      double qp[4], qm[4];
      const unsigned pp = teno6_decide(hp, CT, qp), pm = teno6_decide(hm, CT, qm);
      const double* wp = s_w[pp];
      const double* wm = s_w[pm];
      sF[f] = (wp[0] * qp[0] + wp[1] * qp[1] + wp[2] * qp[2] + wp[3] * qp[3]) +
              (wm[0] * qm[0] + wm[1] * qm[1] + wm[2] * qm[2] + wm[3] * qm[3]);
      if (TAPE) {
        // the cut-off pattern: bits 0-3 the + side's kept candidates, 4-7 the - side's
        const unsigned pat = pp | pm << 4;
        bits[(long long)(s_td[i] * NV + v) * N + s_tq[i]] = (unsigned char)pat;
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
// tiles; 2: one block per tile, also writing the TENO cut-off patterns;
// 3: one block per tile, the tiles that k_conv_lean marked in tcls.
template <int NS, int MODE>
__global__ __launch_bounds__(BLK, 2) void k_conv(const MechTables* __restrict__ M, const Member* __restrict__ mem,
                                              int nmem, int nlog, CallArgs A, const double* __restrict__ Ub,
                                              const double* __restrict__ auxb, const double* __restrict__ srcb,
                                              const unsigned char* __restrict__ flagb, double* __restrict__ partb,
                                              unsigned char* __restrict__ bitsb, double psi_c, double CT,
                                              unsigned char* __restrict__ tcls) {
  if constexpr (MODE == 1) {
    for (int bl = blockIdx.x; bl < nlog; bl += gridDim.x) {
      conv_tile<NS, false, 0>(bl, mem, nmem, A, Ub, auxb, srcb, flagb, partb, bitsb, psi_c, CT, tcls);
      __syncthreads();   // the next tile reuses the LDS
    }
  } else if constexpr (MODE == 2) {
    conv_tile<NS, true, 0>(blockIdx.x, mem, nmem, A, Ub, auxb, srcb, flagb, partb, bitsb, psi_c, CT, tcls);
  } else if constexpr (MODE == 3) {
    conv_tile<NS, false, 2>(blockIdx.x, mem, nmem, A, Ub, auxb, srcb, flagb, partb, bitsb, psi_c, CT, tcls);
  } else {
    conv_tile<NS, false, 0>(blockIdx.x, mem, nmem, A, Ub, auxb, srcb, flagb, partb, bitsb, psi_c, CT, tcls);
  }
}

// The lean convective sweep: the tiles without TENO faces (central fluxes
// only), at up to four blocks per CU; marks the other tiles in tcls for
// k_conv<NS, 3>.
template <int NS>
__global__ __launch_bounds__(BLK, 4) void k_conv_lean(const MechTables* __restrict__ M,
                                                      const Member* __restrict__ mem, int nmem, CallArgs A,
                                                      const double* __restrict__ Ub, const double* __restrict__ auxb,
                                                      const double* __restrict__ srcb,
                                                      const unsigned char* __restrict__ flagb,
                                                      double* __restrict__ partb, double psi_c,
                                                      unsigned char* __restrict__ tcls) {
  conv_tile<NS, false, 1>(blockIdx.x, mem, nmem, A, Ub, auxb, srcb, flagb, partb, nullptr, psi_c, 0.0, tcls);
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
  int FB[3] = {G.dtdim[0], G.dtdim[1], G.dtdim[2]};
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
// The diffusive sweep's own tiles (dtdim, DTILE cells): BLKF threads, the
// first DTILE own the tile's cells, and every thread owns one face per
// direction (a tile has at most BLKF faces along any axis).
template <int NS>
__device__ __forceinline__ void diff_tile(int bl, const MechTables* __restrict__ M, const Member* __restrict__ mem,
                                          int nmem, const CallArgs& A, const double* __restrict__ Ub,
                                          const double* Unb, const double* __restrict__ Tb,
                                          const double* __restrict__ auxb, const double* __restrict__ gradb,
                                          const double* __restrict__ partb, double* outb, double ca, double cb,
                                          int rhs_only) {
  constexpr int NV = NS + 4, NAUX = 7 + NS;
  __shared__ double s_Fd[NV][BLKF];
  const int m = find_member_dtiled(mem, nmem, bl);
  const Member& G = mem[m];
  const int t = threadIdx.x;
  int o[3];
  tile_origin_of(G.dtdim, G.dntile, G.ndtblocks, bl - G.dtblock_begin, o);
  const int T0 = G.dtdim[0], T1 = G.dtdim[1];
  const int l[3] = {t % T0, (t / T0) % T1, t / (T0 * T1)};
  const int gc[3] = {o[0] + l[0], o[1] + l[1], o[2] + l[2]};
  const bool valid = t < DTILE && gc[0] < G.n[0] && gc[1] < G.n[1] && gc[2] < G.n[2];
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
  // next to a non-periodic boundary part[] holds the whole right-hand side
  // (the boundary kernel's): no diffusive term is added here
  if (in_boundary_slab(G, gc)) {
#pragma unroll
    for (int v = 0; v < NV; ++v) acc[v] = 0.0;
  }
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

// ----------------------------------------------------- non-periodic boundaries
// Cells within three nodes of a bounded boundary (in_boundary_slab) get
// their whole right-hand side here, one thread per cell, evaluating each of
// their faces on its own (the tiled sweeps assume periodic wrap).  On a
// bounded axis the first and last nodes lie on the boundary; a face whose
// six-point stencil does not fit takes the widest centred interpolation that
// does ((-1, 7, 7, -1)/12 or (1, 1)/2), or, where the hybrid switch marks
// it, the local Lax-Friedrichs (Rusanov) flux of its two nodes.  Boundary
// nodes take the locally one-dimensional characteristic treatment of
// Poinsot & Lele (the paper's NSCBC, Methods › Diffusion flame › Physical
// model and numerical setup): the normal convective terms as wave
// amplitudes from one-sided differences, entering waves prescribed
// (outflow: the acoustic one relaxes p to p_inf; walls and inflows hold u
// and T, inflows also Y, with the entering acoustic wave equal to the
// leaving one; Methods › Model rocket combustor › Numerical setup).

__device__ __forceinline__ double cpR_b(const MechTables* __restrict__ M, int s, double T) {
  const double* a = M->cp[s];
  return a[0] + T * (a[1] + T * (a[2] + T * (a[3] + T * a[4])));
}

// Linear index of node k along axis d of the stencil through cell c
// (periodic axes wrap).
__device__ __forceinline__ long long node_along(const Member& G, const int c[3], int d, int k) {
  int g[3] = {c[0], c[1], c[2]};
  g[d] = G.bc[d][0] != 0 ? k : wrapi(k, G.n[d]);
  return lin(G, g);
}

// Convective flux through face i+1/2 along d (i = c[d] with the other
// coordinates of c), every variable, into out[].
template <int NS>
__device__ void bnd_conv_face(const Member& G, int d, const int c[3], const double* __restrict__ U,
                              const double* __restrict__ aux, const unsigned char* __restrict__ flag, unsigned flags,
                              double psi_c, double CT, double* out) {
  constexpr int NV = NS + 4;
  const long long N = G.N;
  const int i = c[d], n = G.n[d];
  int m = 6, start = i - 2;
  if (G.bc[d][0] != 0 && (i < 2 || i > n - 4)) {
    m = (i == 0 || i == n - 2) ? 2 : 4;
    start = i - m / 2 + 1;
  }
  long long st[6];
  for (int k = 0; k < m; ++k) st[k] = node_along(G, c, d, start + k);
  const int fa = m / 2 - 1, fb = m / 2;   // the face's two nodes
  bool te;
  if (flags & HTR_FORCE_TENO) te = true;
  else if (flags & HTR_FORCE_CENTRAL) te = false;
  else {
    int any = 0;
    for (int k = 0; k < m; ++k) any |= flag[st[k]];
    const double pa = aux[st[fa]], pb = aux[st[fb]];
    te = any != 0 || fabs(pb - pa) / fmin(pa, pb) > psi_c;
  }
  double ud[6], p[6];
  for (int k = 0; k < m; ++k) {
    ud[k] = aux[(4 + d) * N + st[k]];
    p[k] = aux[st[k]];
  }
  double al = 0.0;
  if (te) {
    al = fabs(ud[0]) + aux[N + st[0]];
    for (int k = 1; k < m; ++k) al = fmax(al, fabs(ud[k]) + aux[N + st[k]]);
  }
  for (int v = 0; v < NV; ++v) {
    double u6[6], f6[6];
    for (int k = 0; k < m; ++k) {
      u6[k] = U[v * N + st[k]];
      f6[k] = node_flux<NS>(v, d, u6[k], ud[k], p[k]);
    }
    if (!te) {
      if (m == 6)
        out[v] = (f6[0] - 8.0 * f6[1] + 37.0 * f6[2] + 37.0 * f6[3] - 8.0 * f6[4] + f6[5]) * (1.0 / 60.0);
      else if (m == 4)
        out[v] = (-f6[0] + 7.0 * f6[1] + 7.0 * f6[2] - f6[3]) * (1.0 / 12.0);
      else
        out[v] = 0.5 * (f6[0] + f6[1]);
    } else if (m == 6) {
      double hp[6], hm[6];
      for (int k = 0; k < 6; ++k) {
        hp[k] = fma(al, u6[k], f6[k]);
        hm[5 - k] = fma(-al, u6[k], f6[k]);
      }
      out[v] = (flags & HTR_WENO3Z) ? weno3z_h(hp) + weno3z_h(hm) : teno6_h(hp, CT) + teno6_h(hm, CT);
    } else {
      out[v] = 0.5 * (f6[fa] + f6[fb]) - 0.5 * al * (u6[fb] - u6[fa]);
    }
  }
}

template <int NS>
__device__ __forceinline__ void bnd_diff_face(const MechTables* __restrict__ M, const Member& G, int d, const int c[3],
                                              const double* __restrict__ U, const double* __restrict__ T,
                                              const double* __restrict__ aux, const double* __restrict__ grad,
                                              double* out) {
  int cb[3] = {c[0], c[1], c[2]};
  cb[d] = G.bc[d][0] != 0 ? c[d] + 1 : wrapi(c[d] + 1, G.n[d]);
  const long long qA = lin(G, c), qB = lin(G, cb);
  if (d == 0) diff_face<NS, 0>(M, G, c[0], qA, qB, G.N, U, T, aux, grad, out);
  else if (d == 1) diff_face<NS, 1>(M, G, c[1], qA, qB, G.N, U, T, aux, grad, out);
  else diff_face<NS, 2>(M, G, c[2], qA, qB, G.N, U, T, aux, grad, out);
}

template <int NS>
__global__ __launch_bounds__(BLK) void k_bnd(const MechTables* __restrict__ M, const Member* __restrict__ mem,
                                             CallArgs A, const double* __restrict__ U, const double* __restrict__ T,
                                             const double* __restrict__ aux, const double* __restrict__ src,
                                             const unsigned char* __restrict__ flag,
                                             const double* __restrict__ grad, double* __restrict__ part,
                                             double psi_c, double CT) {
  constexpr int NV = NS + 4;
  const Member& G = mem[0];
  const long long q = (long long)blockIdx.x * BLK + threadIdx.x;
  if (q >= G.N) return;
  const long long N = G.N;
  const int c[3] = {(int)(q % G.n[0]), (int)((q / G.n[0]) % G.n[1]), (int)(q / ((long long)G.n[0] * G.n[1]))};
  if (!in_boundary_slab(G, c)) return;
  const unsigned flags = A.flags;
  double acc[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) acc[v] = v < NS ? src[v * N + q] : (v == NS + 3 ? src[NS * N + q] : 0.0);
  bool onb = false;
  double fdw[3][NS];   // diffusive species flux of the face next to a wall node, per axis
  for (int a = 0; a < 3; ++a) {
    if (!G.act[a]) continue;
    const bool bnd = G.bc[a][0] != 0;
    const bool edge = bnd && (c[a] == 0 || c[a] == G.n[a] - 1);
    onb = onb || edge;
    if (edge) {
      // the node's face inside the domain, for a wall's species diffusion
      if (!(flags & HTR_VISC_OFF) && (G.bc[a][c[a] == 0 ? 0 : 1] == HTR_BC_WALL)) {
        int cf[3] = {c[0], c[1], c[2]};
        if (c[a] != 0) cf[a] -= 1;
        double fd[NV];
        bnd_diff_face<NS>(M, G, a, cf, U, T, aux, grad, fd);
        for (int s = 0; s < NS; ++s) fdw[a][s] = fd[s];
      }
      continue;
    }
    int cm[3] = {c[0], c[1], c[2]};
    cm[a] = bnd ? c[a] - 1 : wrapi(c[a] - 1, G.n[a]);
    double fcp[NV], fcm[NV], fdp[NV], fdm[NV];
    bnd_conv_face<NS>(G, a, c, U, aux, flag, flags, psi_c, CT, fcp);
    bnd_conv_face<NS>(G, a, cm, U, aux, flag, flags, psi_c, CT, fcm);
    if (flags & HTR_VISC_OFF) {
      for (int v = 0; v < NV; ++v) fdp[v] = fdm[v] = 0.0;
    } else {
      bnd_diff_face<NS>(M, G, a, c, U, T, aux, grad, fdp);
      bnd_diff_face<NS>(M, G, a, cm, U, T, aux, grad, fdm);
    }
    const double xi = G.xin[a][c[a]];
    for (int v = 0; v < NV; ++v) acc[v] += xi * ((fdp[v] - fdm[v]) - (fcp[v] - fcm[v]));
  }
  if (onb) {
    // boundary node: characteristic treatment along every bounded axis it lies on
    double Y[NS], rho = 0.0;
    for (int s = 0; s < NS; ++s) rho += U[s * N + q];
    for (int s = 0; s < NS; ++s) Y[s] = U[s * N + q] / rho;
    const double Tq = T[q], pq = aux[q], cc = aux[N + q];
    const double uq[3] = {aux[4 * N + q], aux[5 * N + q], aux[6 * N + q]};
    double cpm = 0.0, iW = 0.0, hs[NS];
    const double iT = 1.0 / Tq;
    for (int s = 0; s < NS; ++s) {
      cpm += Y[s] * M->RW[s] * cpR_b(M, s, Tq);
      iW += Y[s] * M->iW[s];
      hs[s] = M->RW[s] * Tq * hRTi(M, s, Tq, iT);
    }
    const double W = 1.0 / iW;
    const double cv = cpm - RU * iW, gam = cpm / cv, cc2 = cc * cc;
    bool held = false, holdY = false;
    double add[NV];
    for (int v = 0; v < NV; ++v) add[v] = 0.0;
    const long long stride[3] = {1, G.n[0], (long long)G.n[0] * G.n[1]};
    for (int a = 0; a < 3; ++a) {
      if (!G.act[a] || G.bc[a][0] == 0 || !(c[a] == 0 || c[a] == G.n[a] - 1)) continue;
      const int side = c[a] == 0 ? 0 : 1;
      const int type = G.bc[a][side];
      const double sgn = side ? 1.0 : -1.0;
      const long long s1 = side ? -stride[a] : stride[a];
      const double xi = G.xin[a][c[a]];
      // one-sided second-order derivative along a (inward)
      auto D = [&](double f0, double f1, double f2) {
        return side ? xi * (3.0 * f0 - 4.0 * f1 + f2) / 2.0 : xi * (-3.0 * f0 + 4.0 * f1 - f2) / 2.0;
      };
      double r1 = 0.0, r2 = 0.0;
      for (int s = 0; s < NS; ++s) {
        r1 += U[s * N + q + s1];
        r2 += U[s * N + q + 2 * s1];
      }
      const double Dp = D(pq, aux[q + s1], aux[q + 2 * s1]);
      const double Dr = D(rho, r1, r2);
      double Du[3];
      for (int mm = 0; mm < 3; ++mm)
        Du[mm] = D(uq[mm], aux[(4 + mm) * N + q + s1], aux[(4 + mm) * N + q + 2 * s1]);
      const double un = uq[a];
      double L1 = (un - cc) * (Dp - rho * cc * Du[a]);
      double L5 = (un + cc) * (Dp + rho * cc * Du[a]);
      if (type == HTR_BC_WALL || type == HTR_BC_INFLOW) {
        held = true;
        if (type == HTR_BC_INFLOW) holdY = true;
        const double Lout = side ? L5 : L1;
        const double drho = (type == HTR_BC_INFLOW ? -(gam / cc2) : -(1.0 / cc2)) * Lout;
        for (int s = 0; s < NS; ++s) add[s] += Y[s] * drho;
        if (type == HTR_BC_WALL && !(flags & HTR_VISC_OFF)) {
          const double x2 = 2.0 * xi;
          for (int s = 0; s < NS; ++s) add[s] += (side ? -x2 : x2) * fdw[a][s];
        }
        continue;
      }
      // outflow
      double L2 = un * (cc2 * Dr - Dp);
      double L3 = un * Du[(a + 1) % 3], L4 = un * Du[(a + 2) % 3];
      const double Ld = fabs(G.xnode[a][G.n[a] - 1] - G.xnode[a][0]);
      const double Mn = fabs(un) / cc;
      const double K = G.relax[a][side] * cc * (1.0 - Mn * Mn) / Ld;
      const double relaxp = K * (pq - G.pinf[a][side]);
      if (sgn * (un - cc) < 0) L1 = relaxp;
      if (sgn * (un + cc) < 0) L5 = relaxp;
      const bool backflow = sgn * un < 0;
      if (backflow) { L2 = 0.0; L3 = 0.0; L4 = 0.0; }
      const double rho_t = -(L2 + 0.5 * (L5 + L1)) / cc2;
      const double p_t = -0.5 * (L5 + L1);
      double u_t[3];
      u_t[a] = -(L5 - L1) / (2.0 * rho * cc);
      u_t[(a + 1) % 3] = -L3;
      u_t[(a + 2) % 3] = -L4;
      double ke = 0.0, udu = 0.0;
      for (int mm = 0; mm < 3; ++mm) { ke += uq[mm] * uq[mm]; udu += uq[mm] * u_t[mm]; }
      double dE = (cpm * W / RU - 1.0) * p_t + 0.5 * ke * rho_t + rho * udu;
      for (int s = 0; s < NS; ++s) {
        const double LY = backflow ? 0.0 : un * D(Y[s], U[s * N + q + s1] / r1, U[s * N + q + 2 * s1] / r2);
        const double drs = Y[s] * rho_t - rho * LY;
        add[s] += drs;
        dE += (hs[s] - cpm * Tq * W * M->iW[s]) * drs;
      }
      for (int mm = 0; mm < 3; ++mm) add[NS + mm] += uq[mm] * rho_t + rho * u_t[mm];
      add[NS + 3] += dE;
    }
    if (!held) {
      for (int v = 0; v < NV; ++v) acc[v] += add[v];
    } else {
      double drs[NS], drho = 0.0;
      for (int s = 0; s < NS; ++s) {
        drs[s] = acc[s] + add[s];
        drho += drs[s];
      }
      if (holdY)
        for (int s = 0; s < NS; ++s) drs[s] = Y[s] * drho;
      double ke = 0.0;
      for (int mm = 0; mm < 3; ++mm) ke += uq[mm] * uq[mm];
      double dE = 0.0;
      for (int s = 0; s < NS; ++s) {
        acc[s] = drs[s];
        dE += (hs[s] - RU * Tq * M->iW[s] + 0.5 * ke) * drs[s];
      }
      for (int mm = 0; mm < 3; ++mm) acc[NS + mm] = uq[mm] * drho;
      acc[NS + 3] = dE;
    }
  }
  for (int v = 0; v < NV; ++v) part[v * N + q] = acc[v];
}

template <int NS>
static hipError_t bnd_t(const MechTables* M, const Member* mem, int nblocks, const CallArgs& a, const double* U,
                        const double* T, const double* aux, const double* src, const unsigned char* flag,
                        const double* grad, double* part, double psi_c, double CT, hipStream_t s) {
  hipLaunchKernelGGL(k_bnd<NS>, dim3(nblocks), dim3(BLK), 0, s, M, mem, a, U, T, aux, src, flag, grad, part, psi_c, CT);
  return hipGetLastError();
}

hipError_t launch_bnd(int ns, const MechTables* M, const Member* mem, int nblocks, const CallArgs& a, const double* U,
                      const double* T, const double* aux, const double* src, const unsigned char* flag,
                      const double* grad, double* part, double psi_c, double CT, hipStream_t s) {
#define C_(NS) bnd_t<NS>(M, mem, nblocks, a, U, T, aux, src, flag, grad, part, psi_c, CT, s)
  HTR_NS_SWITCH(ns, C_);
#undef C_
}

static int grid_of(int nblocks, int grid) { return (grid <= 0 || grid > nblocks) ? nblocks : grid; }

template <int NS>
static hipError_t conv_t(const MechTables* M, const Member* mem, int nmem, int ntblocks, int grid, const CallArgs& a,
                         const double* U, const double* aux, const double* src, const unsigned char* flag,
                         double* part, unsigned char* bits, double psi_c, double CT, unsigned char* tcls,
                         hipStream_t s) {
  if (bits) {   // taped: one block per tile, every tile in full
    hipLaunchKernelGGL((k_conv<NS, 2>), dim3(ntblocks), dim3(BLK), 0, s, M, mem, nmem, ntblocks, a, U, aux, src, flag,
                       part, bits, psi_c, CT, tcls);
  } else if (grid < ntblocks) {
    hipLaunchKernelGGL((k_conv<NS, 1>), dim3(grid), dim3(BLK), 0, s, M, mem, nmem, ntblocks, a, U, aux, src, flag,
                       part, bits, psi_c, CT, tcls);
  } else if (!tcls) {   // every tile in the full sweep
    hipLaunchKernelGGL((k_conv<NS, 0>), dim3(ntblocks), dim3(BLK), 0, s, M, mem, nmem, ntblocks, a, U, aux, src, flag,
                       part, bits, psi_c, CT, tcls);
  } else {
    // central tiles in the lean variant, then the tiles with TENO faces
    hipLaunchKernelGGL((k_conv_lean<NS>), dim3(ntblocks), dim3(BLK), 0, s, M, mem, nmem, a, U, aux, src, flag, part,
                       psi_c, tcls);
    hipLaunchKernelGGL((k_conv<NS, 3>), dim3(ntblocks), dim3(BLK), 0, s, M, mem, nmem, ntblocks, a, U, aux, src, flag,
                       part, bits, psi_c, CT, tcls);
  }
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
                       unsigned char* tcls, hipStream_t s) {
  grid = grid_of(ntblocks, grid);
#define C_(NS) conv_t<NS>(M, mem, nmem, ntblocks, grid, a, U, aux, src, flag, part, bits, psi_c, CT, tcls, s)
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
