// Discrete adjoint of one right-hand side evaluation and of its heat release.
//
// For a cotangent lam of dU/dt (scaled by s) and a seed h of the heat release
// H = sum_cells dV HRR, these kernels add  s (dL/dU)^T lam + h dH/dU  to an
// accumulator and s (dL/dtheta)^T lam + h dH/dtheta to the parameter
// cotangent, theta = (E, centre x, y, z, ln A_1..nr).  The discrete switches
// (hybrid sensor, TENO cut-offs, the argmax of the Lax-Friedrichs speed, the
// Newton iteration count) are frozen: they are re-evaluated from the same
// inputs with the same arithmetic as the forward sweep, and the derivative
// is that of the scheme with those switches fixed.  The Newton temperature is
// differentiated through its implicit definition e(T, Y) = e.
//
// Three kernels per evaluation, after a forward per-cell pass on the state.
// Each node gathers what it receives, so no atomics are used and the result
// is deterministic:
//   k_adj_conv_tiled  one 256-node tile per block: the six convective faces
//                     per direction whose stencil contains the node, from
//                     face decisions and TENO cut-off patterns evaluated once
//                     per face in LDS; writes the cotangents of the node's
//                     conserved variables (direct) and of its per-cell fields
//                     (T, p, c, mu, lambda, u, D_s).
//   k_adj_diff        one thread per node: the two diffusive faces per
//                     direction and four per tangential axis through the
//                     cross-derivatives; adds to those cotangents.
//   k_adj_point       one thread per cell: reverse of the per-cell physics
//                     (heat release, chemistry, Bird and Wilke transport,
//                     EOS, implicit Newton T), plus the laser's parameter
//                     derivatives; block partials of the parameter cotangent.

#include <math.h>

#include "htr_dev.h"
#include "htr_flux.h"

namespace htr {

// rows of the per-cell field cotangent array
constexpr int PB_T = 0, PB_P = 1, PB_C = 2, PB_MU = 3, PB_LAM = 4, PB_U = 5, PB_D = 8;

__device__ __forceinline__ double cpRa(const MechTables* __restrict__ M, int s, double T) {
  const double* a = M->cp[s];
  return a[0] + T * (a[1] + T * (a[2] + T * (a[3] + T * a[4])));
}
__device__ __forceinline__ double dcpRa(const MechTables* __restrict__ M, int s, double T) {
  const double* a = M->cp[s];
  return a[1] + T * (2.0 * a[2] + T * (3.0 * a[3] + T * 4.0 * a[4]));
}
__device__ __forceinline__ double hRTa(const MechTables* __restrict__ M, int s, double T, double iT) {
  const double* a = M->hc[s];
  return a[0] + T * (a[1] + T * (a[2] + T * (a[3] + T * a[4]))) + a[5] * iT;
}
__device__ __forceinline__ double sRa(const MechTables* __restrict__ M, int s, double T, double lnT) {
  const double* a = M->sc[s];
  return a[0] * lnT + T * (a[1] + T * (a[2] + T * (a[3] + T * a[4]))) + a[5];
}
// collision integrals and their temperature derivatives (x = ln T - ln eps, Ts = T/eps)
__device__ __forceinline__ double om22a(double x, double Ts, double iT, double ieps, double* dT) {
  const double e0 = 1.16145 * exp(-0.14874 * x), e1 = 0.52487 * exp(-0.77320 * Ts), e2 = 2.16178 * exp(-2.43787 * Ts);
  *dT = -0.14874 * e0 * iT - (0.77320 * e1 + 2.43787 * e2) * ieps;
  return e0 + e1 + e2;
}
__device__ __forceinline__ double om11a(double x, double Ts, double iT, double ieps, double* dT) {
  const double e0 = 1.06036 * exp(-0.15610 * x), e1 = 0.19300 * exp(-0.47635 * Ts);
  const double e2 = 1.03587 * exp(-1.52996 * Ts), e3 = 1.76474 * exp(-3.89411 * Ts);
  *dT = -0.15610 * e0 * iT - (0.47635 * e1 + 1.52996 * e2 + 3.89411 * e3) * ieps;
  return e0 + e1 + e2 + e3;
}

// ------------------------------------------------------------- diffusive
// Face (A, B = A + e_d): adds the cotangent contributions to node A
// (side = 0) or node B (side = 1).
template <int NS, int d>
__device__ __forceinline__ void adj_diff_face(const MechTables* __restrict__ M, const Member& G,
                                              const int cA[3], long long qA, long long qB, long long N,
                                              const double* __restrict__ U, const double* __restrict__ T,
                                              const double* __restrict__ aux, const double* __restrict__ lam,
                                              double s, int side, double* ubar, double* pb) {
  constexpr int NV = NS + 4;
  const double xf = G.xif[d][cA[d]];
  int cB[3] = {cA[0], cA[1], cA[2]};
  cB[d] = wrapi(cA[d] + 1, G.n[d]);
  const long long strides[3] = {1, G.n[0], (long long)G.n[0] * G.n[1]};
  const double xiA = G.xin[d][cA[d]], xiB = G.xin[d][cB[d]];
  double Gv[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) Gv[v] = s * (xiA * lam[v * N + qA] - xiB * lam[v * N + qB]);
  double uA[3], uB[3];
#pragma unroll
  for (int mm = 0; mm < 3; ++mm) {
    uA[mm] = aux[(4 + mm) * N + qA];
    uB[mm] = aux[(4 + mm) * N + qB];
  }
  double g[3][3];
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int mm = 0; mm < 3; ++mm) g[a][mm] = 0.0;
#pragma unroll
  for (int mm = 0; mm < 3; ++mm) g[d][mm] = xf * (uB[mm] - uA[mm]);
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    if (a == d || !G.act[a]) continue;
#pragma unroll
    for (int sd = 0; sd < 2; ++sd) {
      const int cca = sd ? cB[a] : cA[a];
      const long long qc = sd ? qB : qA;
      const long long qp = qc + (long long)(wrapi(cca + 1, G.n[a]) - cca) * strides[a];
      const long long qm = qc + (long long)(wrapi(cca - 1, G.n[a]) - cca) * strides[a];
      const double xa = 0.5 * G.xin[a][cca];
#pragma unroll
      for (int mm = 0; mm < 3; ++mm) g[a][mm] += 0.5 * (xa * (aux[(4 + mm) * N + qp] - aux[(4 + mm) * N + qm]));
    }
  }
  const double muf = 0.5 * (aux[2 * N + qA] + aux[2 * N + qB]);
  const double lamf = 0.5 * (aux[3 * N + qA] + aux[3 * N + qB]);
  const double divu = g[0][0] + g[1][1] + g[2][2];
  double tau[3], uf[3];
#pragma unroll
  for (int mm = 0; mm < 3; ++mm) {
    tau[mm] = muf * (g[d][mm] + g[mm][d]);
    if (mm == d) tau[mm] -= (2.0 / 3.0) * muf * divu;
    uf[mm] = 0.5 * (uA[mm] + uB[mm]);
  }
  double rA = 0.0, rB = 0.0, nA = 0.0, nB = 0.0;
#pragma unroll
  for (int k = 0; k < NS; ++k) {
    const double a = U[k * N + qA], b = U[k * N + qB];
    rA += a;
    rB += b;
    nA += a * M->iW[k];
    nB += b * M->iW[k];
  }
  const double rhof = 0.5 * (rA + rB);
  const double Wf = 0.5 * (rA / nA + rB / nB);
  const double TA = T[qA], TB = T[qB];
  // pass 1: corr = sum_k term_k (per-species values are recomputed from
  // cached loads in every pass instead of being held in registers)
  double corr = 0.0;
#pragma unroll
  for (int k = 0; k < NS; ++k) {
    const double a = U[k * N + qA], b = U[k * N + qB];
    const double Df = 0.5 * (aux[(7 + k) * N + qA] + aux[(7 + k) * N + qB]);
    const double dX = xf * (b * M->iW[k] / nB - a * M->iW[k] / nA);
    corr += rhof * Df * (M->W[k] / Wf) * dX;
  }
  // ---- reverse
  const double qnb = -Gv[NS + 3];
  double taub[3];
#pragma unroll
  for (int mm = 0; mm < 3; ++mm) taub[mm] = Gv[NS + mm] + Gv[NS + 3] * uf[mm];
  const double lamfb = -qnb * xf * (TB - TA);
  double TAb = qnb * lamf * xf, TBb = -qnb * lamf * xf;
  // pass 2: species flux cotangents
  double Jb[NS];
  double corrb = 0.0;
#pragma unroll
  for (int k = 0; k < NS; ++k) {
    const double a = U[k * N + qA], b = U[k * N + qB];
    const double Df = 0.5 * (aux[(7 + k) * N + qA] + aux[(7 + k) * N + qB]);
    const double dX = xf * (b * M->iW[k] / nB - a * M->iW[k] / nA);
    const double term = rhof * Df * (M->W[k] / Wf) * dX;
    const double Yf = 0.5 * (a / rA + b / rB);
    const double J = -term + Yf * corr;
    const double hA = M->RW[k] * TA * hRTs(M, k, TA), hB = M->RW[k] * TB * hRTs(M, k, TB);
    const double hfb = qnb * J;
    TAb += hfb * 0.5 * M->RW[k] * cpRa(M, k, TA);
    TBb += hfb * 0.5 * M->RW[k] * cpRa(M, k, TB);
    Jb[k] = -Gv[k] + qnb * 0.5 * (hA + hB);
    corrb += Jb[k] * Yf;
  }
  // pass 3: back to the node's partial densities and diffusivities
  const double sgn = side ? 1.0 : -1.0;          // d(dX)/dX_B = +xf, d(dX)/dX_A = -xf
  const double rn = side ? rB : rA, nn = side ? nB : nA;
  const long long qn = side ? qB : qA;
  double rhofb = 0.0, Wfb = 0.0, nbar = 0.0, rbar = 0.0;
#pragma unroll
  for (int k = 0; k < NS; ++k) {
    const double a = U[k * N + qA], b = U[k * N + qB], an = U[k * N + qn];
    const double Df = 0.5 * (aux[(7 + k) * N + qA] + aux[(7 + k) * N + qB]);
    const double dX = xf * (b * M->iW[k] / nB - a * M->iW[k] / nA);
    const double term = rhof * Df * (M->W[k] / Wf) * dX;
    const double termb = -Jb[k] + corrb;
    const double Yfb = Jb[k] * corr;
    rhofb += termb * Df * (M->W[k] / Wf) * dX;
    Wfb -= termb * term / Wf;
    pb[PB_D + k] += 0.5 * termb * rhof * (M->W[k] / Wf) * dX;
    const double Xb = sgn * termb * rhof * Df * M->W[k] / Wf * xf;
    const double Xn = an * M->iW[k] / nn;
    nbar -= Xb * Xn / nn;
    rbar -= 0.5 * Yfb * an / (rn * rn);
    ubar[k] += Xb * M->iW[k] / nn + 0.5 * Yfb / rn;
  }
  rbar += 0.5 * Wfb / nn + 0.5 * rhofb;
  nbar += -0.5 * Wfb * rn / (nn * nn);
#pragma unroll
  for (int k = 0; k < NS; ++k) ubar[k] += rbar + nbar * M->iW[k];
  double mufb = -(2.0 / 3.0) * taub[d] * divu;
#pragma unroll
  for (int mm = 0; mm < 3; ++mm) mufb += taub[mm] * (g[d][mm] + g[mm][d]);
  // velocity gradient cotangent, normal row only (tangential rows go to the tangential neighbours)
  double gdb[3];
#pragma unroll
  for (int mm = 0; mm < 3; ++mm) gdb[mm] = muf * taub[mm];
  gdb[d] = (4.0 / 3.0) * muf * taub[d];
  pb[PB_T] += side ? TBb : TAb;
  pb[PB_MU] += 0.5 * mufb;
  pb[PB_LAM] += 0.5 * lamfb;
#pragma unroll
  for (int mm = 0; mm < 3; ++mm) pb[PB_U + mm] += 0.5 * Gv[NS + 3] * tau[mm] + sgn * xf * gdb[mm];
}

// Tangential-neighbour contributions: node q is u(A +- e_t) or u(B +- e_t)
// of the d-face (A, A + e_d).
template <int NS, int d, int t>
__device__ __forceinline__ void adj_diff_tangential(const Member& G, const int c[3], long long q,
                                                    long long N, const double* __restrict__ aux,
                                                    const double* __restrict__ lam, double s, double* pb) {
  constexpr int NV = NS + 4;
  const long long strides[3] = {1, G.n[0], (long long)G.n[0] * G.n[1]};
  // (shift along t, shift along d of A, sign)
  const int cfg[4][3] = {{-1, 0, 1}, {1, 0, -1}, {-1, -1, 1}, {1, -1, -1}};
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    int cA[3] = {c[0], c[1], c[2]};
    cA[t] = wrapi(c[t] + cfg[k][0], G.n[t]);
    cA[d] = wrapi(c[d] + cfg[k][1], G.n[d]);
    int cB[3] = {cA[0], cA[1], cA[2]};
    cB[d] = wrapi(cA[d] + 1, G.n[d]);
    const long long qA = ((long long)cA[2] * G.n[1] + cA[1]) * G.n[0] + cA[0];
    const long long qB = ((long long)cB[2] * G.n[1] + cB[1]) * G.n[0] + cB[0];
    const double xiA = G.xin[d][cA[d]], xiB = G.xin[d][cB[d]];
    double Gm[3], GE;
#pragma unroll
    for (int mm = 0; mm < 3; ++mm) Gm[mm] = s * (xiA * lam[(NS + mm) * N + qA] - xiB * lam[(NS + mm) * N + qB]);
    GE = s * (xiA * lam[(NS + 3) * N + qA] - xiB * lam[(NS + 3) * N + qB]);
    double taub[3];
#pragma unroll
    for (int mm = 0; mm < 3; ++mm) taub[mm] = Gm[mm] + GE * 0.5 * (aux[(4 + mm) * N + qA] + aux[(4 + mm) * N + qB]);
    const double muf = 0.5 * (aux[2 * N + qA] + aux[2 * N + qB]);
    // g[t][b] += 0.25 xi_t (u_b(node + e_t) - u_b(node - e_t)) for node in {A, B}
    const double w = cfg[k][2] * 0.25 * G.xin[t][cA[t]];
    pb[PB_U + d] += w * muf * taub[t];
    pb[PB_U + t] += w * (-(2.0 / 3.0)) * muf * taub[d];
  }
  (void)strides;
  (void)NV;
}

// ------------------------------------------------ convective, tiled
// One 256-node tile per block.  Per direction the tile with a 5-node halo
// is staged in LDS; every face whose stencil touches the tile takes its
// hybrid decision and LF speed once, and for each variable its TENO cut-off
// pattern once (four bits per side, in LDS).  Each node then gathers from
// the six faces containing it: the face cotangent times the frozen linear
// coefficient of its stencil position.
constexpr int STGA = (EXTA + BLK - 1) / BLK;
constexpr int FPTA = (FACEA + BLK - 1) / BLK;

template <int NS, int d>
__device__ __forceinline__ void adj_conv_tiled_dir(const Member& G, const int o[3], const int l[3],
                                                   const int gc[3], bool valid, long long N,
                                                   const double* __restrict__ U, const double* __restrict__ aux,
                                                   const unsigned char* __restrict__ flag,
                                                   const double* __restrict__ lam, double s, unsigned flags,
                                                   double psi_c, double CT, double* s_ud, double* s_p, double* s_c,
                                                   double* s_U, double* s_L, double* s_al, unsigned char* s_fl,
                                                   unsigned char* s_te, unsigned char* s_db, double* s_ub,
                                                   double& pbu, double& pbp, double& pbc,
                                                   const unsigned char* __restrict__ tbits,
                                                   const double (*s_cf)[6]) {
  constexpr int NV = NS + 4;
  const int t = threadIdx.x;
  const int T[3] = {G.tdim[0], G.tdim[1], G.tdim[2]};
  int B[3] = {T[0], T[1], T[2]};
  B[d] += 10;
  const int E = B[0] * B[1] * B[2];
  int FB[3] = {T[0], T[1], T[2]};
  FB[d] += 5;
  const int F = FB[0] * FB[1] * FB[2];
  const int bs = d == 0 ? 1 : (d == 1 ? B[0] : B[0] * B[1]);
  const int nd = G.n[d];
  // stage the per-cell fields of the box (box position = tile position + 5 along d)
  long long qe[STGA];
#pragma unroll
  for (int k = 0; k < STGA; ++k) {
    const int e = t + k * BLK;
    qe[k] = 0;
    if (e < E) {
      const int b[3] = {e % B[0], (e / B[0]) % B[1], e / (B[0] * B[1])};
      int g[3];
#pragma unroll
      for (int a = 0; a < 3; ++a) g[a] = wrapi(o[a] + b[a] - (a == d ? 5 : 0), G.n[a]);
      qe[k] = ((long long)g[2] * G.n[1] + g[1]) * G.n[0] + g[0];
      s_ud[e] = aux[(4 + d) * N + qe[k]];
      s_p[e] = aux[qe[k]];
      s_c[e] = aux[N + qe[k]];
      s_fl[e] = flag[qe[k]];
    }
  }
  __syncthreads();
  // this thread's faces: slot fb_d = j + 2 (0 .. T_d + 4) for the face between tile positions
  // j-1 and j, whose stencil covers box positions fb_d .. fb_d + 5 along d
  int fe0[FPTA];
  long long fq[FPTA];   // the face's upper cell (index of the forward's taped cut-off patterns)
#pragma unroll
  for (int k = 0; k < FPTA; ++k) {
    const int f = t + k * BLK;
    fe0[k] = -1;
    fq[k] = 0;
    if (f < F) {
      const int fb[3] = {f % FB[0], (f / FB[0]) % FB[1], f / (FB[0] * FB[1])};
      fe0[k] = fb[0] + B[0] * (fb[1] + B[1] * fb[2]);
      if (tbits) {
        int g[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) g[a] = wrapi(o[a] + fb[a] - (a == d ? 2 : 0), G.n[a]);
        fq[k] = ((long long)g[2] * G.n[1] + g[1]) * G.n[0] + g[0];
      }
      const int e0 = fe0[k];
      bool te;
      if (flags & HTR_FORCE_TENO) te = true;
      else if (flags & HTR_FORCE_CENTRAL) te = false;
      else {
        int any = 0;
#pragma unroll
        for (int mm = 0; mm < 6; ++mm) any |= s_fl[e0 + mm * bs];
        const double pa = s_p[e0 + 2 * bs], pv = s_p[e0 + 3 * bs];
        te = any != 0 || fabs(pv - pa) / fmin(pa, pv) > psi_c;
      }
      int am = 0;
      double al = 0.0;
      if (te) {
        al = fabs(s_ud[e0]) + s_c[e0];
#pragma unroll
        for (int mm = 1; mm < 6; ++mm) {
          const double sp = fabs(s_ud[e0 + mm * bs]) + s_c[e0 + mm * bs];
          if (sp > al) { al = sp; am = mm; }
        }
      }
      s_te[f] = (unsigned char)((te ? 1 : 0) | (am << 1));
      s_al[f] = al;
    }
  }
  // node side: its box index, the six face slots containing it, the metric
  const int ln[3] = {l[0], l[1], l[2]};
  const int enode = ln[0] + (d == 0 ? 5 : 0) + B[0] * (ln[1] + (d == 1 ? 5 : 0) + B[1] * (ln[2] + (d == 2 ? 5 : 0)));
  // the node's faces are slots ln_d + k, k = 0..5 (stencil start ln_d + k - 5 in tile positions);
  // the node sits at stencil position 5 - k unless the axis is shorter than the stencil
  const int fs = d == 0 ? 1 : (d == 1 ? FB[0] : FB[0] * FB[1]);
  const int f0 = ln[0] + FB[0] * (ln[1] + FB[1] * ln[2]);
  const bool longax = nd >= 6;
  // short periodic axis: faces revisited (count each once) and several stencil positions per face
  unsigned use = 0x3f, pos[6];
#pragma unroll
  for (int k = 0; k < 6; ++k) {
    pos[k] = 1u << (5 - k);
    if (!longax) {
      const int gf = wrapi(o[d] + ln[d] + k - 2, nd);
#pragma unroll
      for (int k2 = 0; k2 < k; ++k2)
        if (wrapi(o[d] + ln[d] + k2 - 2, nd) == gf) use &= ~(1u << k);
      pos[k] = 0;
#pragma unroll
      for (int mm = 0; mm < 6; ++mm)
        if (wrapi(o[d] + ln[d] + k - 5 + mm, nd) == gc[d]) pos[k] |= 1u << mm;
    }
  }
  double xi7[7];
#pragma unroll
  for (int o7 = 0; o7 < 7; ++o7) xi7[o7] = G.xin[d][wrapi(gc[d] + o7 - 3, nd)];
  const double C6[6] = {1.0 / 60.0, -8.0 / 60.0, 37.0 / 60.0, 37.0 / 60.0, -8.0 / 60.0, 1.0 / 60.0};
  const double sg = s_ud[enode] < 0.0 ? -1.0 : 1.0;
  double abar = 0.0;
  __syncthreads();
#pragma unroll 1
  for (int v = 0; v < NV; ++v) {
#pragma unroll
    for (int k = 0; k < STGA; ++k) {
      const int e = t + k * BLK;
      if (e < E) {
        s_U[e] = U[v * N + qe[k]];
        s_L[e] = s * lam[v * N + qe[k]];
      }
    }
    __syncthreads();
    // faces: cut-off bits of the TENO faces
#pragma unroll
    for (int k = 0; k < FPTA; ++k) {
      if (fe0[k] < 0) continue;
      const int f = t + k * BLK;
      if (!(s_te[f] & 1)) continue;
      if (tbits) {
        s_db[f] = tbits[(long long)(d * NV + v) * N + fq[k]];
        continue;
      }
      const int e0 = fe0[k];
      const double al = s_al[f];
      double hp[6], hm[6], q4[4];
#pragma unroll
      for (int mm = 0; mm < 6; ++mm) {
        const int e = e0 + mm * bs;
        const double u6 = s_U[e], f6 = node_flux<NS>(v, d, u6, s_ud[e], s_p[e]);
        hp[mm] = fma(al, u6, f6);
        hm[5 - mm] = fma(-al, u6, f6);
      }
      s_db[f] = (unsigned char)(teno6_decide(hp, CT, q4) | (teno6_decide(hm, CT, q4) << 4));
    }
    __syncthreads();
    if (valid) {
      double Fb = 0.0, Ub = 0.0;
#pragma unroll
      for (int k = 0; k < 6; ++k) {
        if (!((use >> k) & 1u)) continue;
        // face between tile positions ln-3+k and ln-2+k: cotangent from its two cells
        const double g = -xi7[k] * s_L[enode + (k - 3) * bs] + xi7[k + 1] * s_L[enode + (k - 2) * bs];
        const int f = f0 + k * fs;
        const unsigned te = s_te[f];
        if (!(te & 1)) {
          if (longax) {
            Fb += g * C6[5 - k];
          } else {
#pragma unroll
            for (int mm = 0; mm < 6; ++mm)
              if ((pos[k] >> mm) & 1u) Fb += g * C6[mm];
          }
        } else {
          const unsigned bits = s_db[f];
          const double* cp = s_cf[bits & 15u];
          const double* cm = s_cf[bits >> 4];
          const double al = s_al[f];
          if (longax) {
            Fb += g * 0.5 * (cp[5 - k] + cm[k]);
            Ub += g * 0.5 * al * (cp[5 - k] - cm[k]);
          } else {
#pragma unroll
            for (int mm = 0; mm < 6; ++mm) {
              if ((pos[k] >> mm) & 1u) {
                Fb += g * 0.5 * (cp[mm] + cm[5 - mm]);
                Ub += g * 0.5 * al * (cp[mm] - cm[5 - mm]);
              }
            }
          }
          // the Lax-Friedrichs speed's frozen argmax node receives d(|u_d| + c)
          if ((pos[k] >> (te >> 1)) & 1u) {
            const int e0 = enode + (k - 5) * bs;   // the face's stencil start
            double da = 0.0;
#pragma unroll
            for (int mm = 0; mm < 6; ++mm) da += (cp[mm] - cm[5 - mm]) * s_U[e0 + mm * bs];
            abar += g * 0.5 * da;
          }
        }
      }
      const double un = s_ud[enode], un_u = s_U[enode], un_p = s_p[enode];
      Ub += Fb * un;
      if (v == NS + 3) {
        pbu += Fb * (un_u + un_p);
        pbp += Fb * un;
      } else {
        pbu += Fb * un_u;
        if (v == NS + d) pbp += Fb;
      }
      s_ub[v * BLK + t] += Ub;
    }
    __syncthreads();
  }
  if (valid) {
    pbu += abar * sg;
    pbc += abar;
  }
}

template <int NS>
__global__ __launch_bounds__(BLK, 2) void k_adj_conv_tiled(const Member* __restrict__ mem, int nmem, CallArgs A,
                                                           const double* __restrict__ Ub,
                                                           const double* __restrict__ auxb,
                                                           const unsigned char* __restrict__ flagb,
                                                           const double* __restrict__ lamb, double s,
                                                           double* __restrict__ ubdb, double* __restrict__ pbb,
                                                           const unsigned char* __restrict__ tbitsb, double psi_c,
                                                           double CT) {
  constexpr int NV = NS + 4, NAUX = 7 + NS, NPB = 8 + NS;
  __shared__ double s_ud[EXTA], s_p[EXTA], s_c[EXTA], s_U[EXTA], s_L[EXTA], s_al[FACEA];
  __shared__ unsigned char s_fl[EXTA], s_te[FACEA], s_db[FACEA];
  __shared__ double s_ub[NV * BLK];   // per-thread cotangent accumulators
  __shared__ double s_cf[16][6];      // frozen TENO6 coefficients of every cut-off pattern
  const int m = find_member_tiled(mem, nmem, blockIdx.x);
  const Member& G = mem[m];
  const int t = threadIdx.x;
  int o[3];
  tile_origin(G, blockIdx.x - G.tblock_begin, o);
  const int T0 = G.tdim[0], T1 = G.tdim[1];
  const int l[3] = {t % T0, (t / T0) % T1, t / (T0 * T1)};
  const int gc[3] = {o[0] + l[0], o[1] + l[1], o[2] + l[2]};
  const bool valid = gc[0] < G.n[0] && gc[1] < G.n[1] && gc[2] < G.n[2];
  const long long N = G.N;
  const double* U = Ub + NV * G.off;
  const double* aux = auxb + NAUX * G.off;
  const unsigned char* flag = flagb + G.off;
  const double* lam = lamb + NV * G.off;
  const unsigned char* tbits = tbitsb ? tbitsb + 3LL * NV * G.off : nullptr;
  for (int v = 0; v < NV; ++v) s_ub[v * BLK + t] = 0.0;
  if (t < 16) teno6_coeffs_bits(t, s_cf[t]);   // read after the first direction's staging barrier
  double pbu[3] = {0.0, 0.0, 0.0}, pbp = 0.0, pbc = 0.0;
  const unsigned flags = A.flags;
  if (G.act[0])
    adj_conv_tiled_dir<NS, 0>(G, o, l, gc, valid, N, U, aux, flag, lam, s, flags, psi_c, CT, s_ud, s_p, s_c, s_U, s_L,
                              s_al, s_fl, s_te, s_db, s_ub, pbu[0], pbp, pbc, tbits, s_cf);
  if (G.act[1])
    adj_conv_tiled_dir<NS, 1>(G, o, l, gc, valid, N, U, aux, flag, lam, s, flags, psi_c, CT, s_ud, s_p, s_c, s_U, s_L,
                              s_al, s_fl, s_te, s_db, s_ub, pbu[1], pbp, pbc, tbits, s_cf);
  if (G.act[2])
    adj_conv_tiled_dir<NS, 2>(G, o, l, gc, valid, N, U, aux, flag, lam, s, flags, psi_c, CT, s_ud, s_p, s_c, s_U, s_L,
                              s_al, s_fl, s_te, s_db, s_ub, pbu[2], pbp, pbc, tbits, s_cf);
  if (!valid) return;
  const long long q = ((long long)gc[2] * G.n[1] + gc[1]) * G.n[0] + gc[0];
  double* ubd = ubdb + NV * G.off;
  double* pbo = pbb + NPB * G.off;
  for (int v = 0; v < NV; ++v) ubd[v * N + q] = s_ub[v * BLK + t];
  for (int k = 0; k < NPB; ++k) {
    double x = 0.0;
    if (k == PB_P) x = pbp;
    else if (k == PB_C) x = pbc;
    else if (k >= PB_U && k < PB_U + 3) x = pbu[k - PB_U];
    pbo[k * N + q] = x;
  }
}

// All diffusive contributions of direction d to a node: the two faces of
// which it is a node, and the faces of which it is a tangential neighbour.
template <int NS, int d>
__device__ __forceinline__ void adj_diff_dir(const MechTables* __restrict__ M, const Member& G, const int c[3],
                                             long long q, long long N, const double* __restrict__ U,
                                             const double* __restrict__ T, const double* __restrict__ aux,
                                             const double* __restrict__ lam, double s, double* ubar, double* pb) {
  const long long stride = d == 0 ? 1 : (d == 1 ? (long long)G.n[0] : (long long)G.n[0] * G.n[1]);
  int cm[3] = {c[0], c[1], c[2]};
  cm[d] = wrapi(c[d] - 1, G.n[d]);
  const long long qm = q + (long long)(cm[d] - c[d]) * stride;
  const long long qp = q + (long long)(wrapi(c[d] + 1, G.n[d]) - c[d]) * stride;
  adj_diff_face<NS, d>(M, G, cm, qm, q, N, U, T, aux, lam, s, 1, ubar, pb);
  adj_diff_face<NS, d>(M, G, c, q, qp, N, U, T, aux, lam, s, 0, ubar, pb);
  constexpr int t1 = (d + 1) % 3, t2 = (d + 2) % 3;
  if (G.act[t1]) adj_diff_tangential<NS, d, t1>(G, c, q, N, aux, lam, s, pb);
  if (G.act[t2]) adj_diff_tangential<NS, d, t2>(G, c, q, N, aux, lam, s, pb);
}

// Diffusive faces: one thread per node, adds to the convective cotangents.
template <int NS>
__global__ __launch_bounds__(BLK) void k_adj_diff(const MechTables* __restrict__ M, const Member* __restrict__ mem,
                                                  int nmem, const double* __restrict__ Ub,
                                                  const double* __restrict__ Tb, const double* __restrict__ auxb,
                                                  const double* __restrict__ lamb, double s,
                                                  double* __restrict__ ubdb, double* __restrict__ pbb) {
  constexpr int NV = NS + 4, NAUX = 7 + NS, NPB = 8 + NS;
  const int m = find_member(mem, nmem, blockIdx.x);
  const Member& G = mem[m];
  const long long q = (long long)(blockIdx.x - G.block_begin) * BLK + threadIdx.x;
  if (q >= G.N) return;
  const long long N = G.N;
  const double* U = Ub + NV * G.off;
  const double* T = Tb + G.off;
  const double* aux = auxb + NAUX * G.off;
  const double* lam = lamb + NV * G.off;
  const int c[3] = {(int)(q % G.n[0]), (int)((q / G.n[0]) % G.n[1]), (int)(q / ((long long)G.n[0] * G.n[1]))};
  double ubar[NV], pb[NPB];
  double* ubd = ubdb + NV * G.off;
  double* pbo = pbb + NPB * G.off;
#pragma unroll
  for (int v = 0; v < NV; ++v) ubar[v] = ubd[v * N + q];
#pragma unroll
  for (int k = 0; k < NPB; ++k) pb[k] = pbo[k * N + q];
  if (G.act[0]) adj_diff_dir<NS, 0>(M, G, c, q, N, U, T, aux, lam, s, ubar, pb);
  if (G.act[1]) adj_diff_dir<NS, 1>(M, G, c, q, N, U, T, aux, lam, s, ubar, pb);
  if (G.act[2]) adj_diff_dir<NS, 2>(M, G, c, q, N, U, T, aux, lam, s, ubar, pb);
#pragma unroll
  for (int v = 0; v < NV; ++v) ubd[v * N + q] = ubar[v];
#pragma unroll
  for (int k = 0; k < NPB; ++k) pbo[k * N + q] = pb[k];
}

// ------------------------------------------------------------------ point
// Deterministic block sum of one value per thread; every thread of the block
// must call it (it contains barriers).
__device__ __forceinline__ void block_sum_to(double v, double* wred, double* dst) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  if ((threadIdx.x & 63) == 0) wred[threadIdx.x >> 6] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    double a = 0.0;
    for (int w = 0; w < BLK / 64; ++w) a += wred[w];
    *dst = a;
  }
  __syncthreads();
}

template <int NS>
__global__ __launch_bounds__(BLK, 2) void k_adj_point(const MechTables* __restrict__ M, const Member* __restrict__ mem,
                                                   int nmem, CallArgs A, const double* __restrict__ Ub,
                                                   const double* __restrict__ Tb, const double* __restrict__ pbb,
                                                   const double* __restrict__ ubdb, const double* __restrict__ lamb,
                                                   double s, double h, double* __restrict__ outb,
                                                   double* __restrict__ thpart, int nth) {
  constexpr int NV = NS + 4, NPB = 8 + NS;
  __shared__ double conc[NS][BLK];
  __shared__ double wred[BLK / 64];
  const int m = find_member(mem, nmem, blockIdx.x);
  const Member& G = mem[m];
  const int tid = threadIdx.x;
  const long long q = (long long)(blockIdx.x - G.block_begin) * BLK + tid;
  const bool live = q < G.N;
  const long long N = G.N;
  const unsigned flags = A.flags;
  const bool chem = !(flags & HTR_CHEM_OFF);
  const int nr = M->nr;
  const double* dlnA = A.dlnA ? A.dlnA : G.dlnA;
  const double* U = Ub + NV * G.off;
  const double* pbv = pbb + NPB * G.off;
  const double* ubd = ubdb + NV * G.off;
  const double* lam = lamb + NV * G.off;
  double r[NS], Y[NS], X[NS], rb[NS], Yb[NS], Xb[NS], Gs[NS], hRTv[NS], omb_mol[NS], cb[NS];
  double T = 1000.0, iT = 1e-3, lnT = 0.0, Tbar = 0.0, rho = 1.0, irho = 1.0, E = 0.0, lnP = 0.0;
  double u[3] = {0.0, 0.0, 0.0}, ub[3] = {0.0, 0.0, 0.0};
  int ix = 0, jx = 0, kx = 0;
#pragma unroll
  for (int k = 0; k < NS; ++k) {
    r[k] = Y[k] = X[k] = rb[k] = Yb[k] = Xb[k] = Gs[k] = hRTv[k] = omb_mol[k] = cb[k] = 0.0;
  }
  // ---- phase 1: state, forward quantities, seeds of the chemistry
  if (live) {
    rho = 0.0;
#pragma unroll
    for (int k = 0; k < NS; ++k) {
      r[k] = U[k * N + q];
      rho += r[k];
      rb[k] = ubd[k * N + q];
    }
    irho = 1.0 / rho;
#pragma unroll
    for (int k = 0; k < NS; ++k) Y[k] = r[k] * irho;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      u[a] = U[(NS + a) * N + q] * irho;
      ub[a] = pbv[(PB_U + a) * N + q];
    }
    E = U[(NS + 3) * N + q];
    T = Tb[G.off + q];
    iT = 1.0 / T;
    lnT = log(T);
    Tbar = pbv[PB_T * N + q];
    ix = (int)(q % G.n[0]);
    jx = (int)((q / G.n[0]) % G.n[1]);
    kx = (int)(q / ((long long)G.n[0] * G.n[1]));
    if (chem) {
      const double dV = 1.0 / (G.xin[0][ix] * G.xin[1][jx] * G.xin[2][kx]);
      const double Hb = h * dV;
#pragma unroll
      for (int k = 0; k < NS; ++k) {
        conc[k][tid] = r[k] * M->iW[k];
        hRTv[k] = hRTa(M, k, T, iT);
        Gs[k] = hRTv[k] - sRa(M, k, T, lnT);
      }
      lnP = log(PREF / (RU * T));
      double om[NS];
#pragma unroll
      for (int k = 0; k < NS; ++k) om[k] = 0.0;
      for (int j = 0; j < nr; ++j) {
        double lnkf = M->lnA[j] + M->beta[j] * lnT - M->EaR[j] * iT;
        if (dlnA) lnkf += dlnA[j];
        double lnKc = M->dnu[j] * lnP;
#pragma unroll
        for (int k = 0; k < NS; ++k) lnKc -= M->nunet[j][k] * Gs[k];
        double rf = exp(lnkf), rbk = exp(lnkf - lnKc);
        for (int e = 0; e < M->nre[j]; ++e) {
          const double cc = conc[M->ridx[j][e]][tid];
          for (int kk = 0; kk < M->rnu[j][e]; ++kk) rf *= cc;
        }
        for (int e = 0; e < M->npr[j]; ++e) {
          const double cc = conc[M->pidx[j][e]][tid];
          for (int kk = 0; kk < M->pnu[j][e]; ++kk) rbk *= cc;
        }
#pragma unroll
        for (int k = 0; k < NS; ++k) om[k] += M->nunet[j][k] * (rf - rbk);
      }
      // seeds: the source rows of lam, and the heat release -sum h_k wdot_k
#pragma unroll
      for (int k = 0; k < NS; ++k) {
        const double omk = M->W[k] * om[k];
        const double hk = M->RW[k] * T * hRTv[k];
        const double wb = s * lam[k * N + q] - Hb * hk;
        Tbar += -Hb * omk * M->RW[k] * cpRa(M, k, T);
        omb_mol[k] = M->W[k] * wb;
      }
    }
  }
  // ---- phase 2: reverse of the reactions (every thread reaches the block sums)
  if (chem) {
    for (int j = 0; j < nr; ++j) {
      double lnkfb = 0.0;
      if (live) {
        double qb = 0.0;
#pragma unroll
        for (int k = 0; k < NS; ++k) qb += M->nunet[j][k] * omb_mol[k];
        double lnkf = M->lnA[j] + M->beta[j] * lnT - M->EaR[j] * iT;
        if (dlnA) lnkf += dlnA[j];
        double lnKc = M->dnu[j] * lnP;
        double dlnKc = -M->dnu[j] * iT;                       // d lnKc / dT
#pragma unroll
        for (int k = 0; k < NS; ++k) {
          lnKc -= M->nunet[j][k] * Gs[k];
          dlnKc += M->nunet[j][k] * hRTv[k] * iT;             // d G_k / dT = -hRT_k / T
        }
        const double kf = exp(lnkf), kb = exp(lnkf - lnKc);
        double rf = kf, rbk = kb;
        for (int e = 0; e < M->nre[j]; ++e) {
          const double cc = conc[M->ridx[j][e]][tid];
          for (int kk = 0; kk < M->rnu[j][e]; ++kk) rf *= cc;
        }
        for (int e = 0; e < M->npr[j]; ++e) {
          const double cc = conc[M->pidx[j][e]][tid];
          for (int kk = 0; kk < M->pnu[j][e]; ++kk) rbk *= cc;
        }
        // d(k prod c^nu)/dc_e = k nu_e c_e^(nu_e - 1) prod_{others} c^nu
        for (int e = 0; e < M->nre[j]; ++e) {
          double dp = kf * M->rnu[j][e];
          for (int e2 = 0; e2 < M->nre[j]; ++e2) {
            const double cc = conc[M->ridx[j][e2]][tid];
            const int pw = M->rnu[j][e2] - (e2 == e ? 1 : 0);
            for (int kk = 0; kk < pw; ++kk) dp *= cc;
          }
          const int sp = M->ridx[j][e];
#pragma unroll
          for (int k = 0; k < NS; ++k)
            if (k == sp) cb[k] += qb * dp;
        }
        for (int e = 0; e < M->npr[j]; ++e) {
          double dp = kb * M->pnu[j][e];
          for (int e2 = 0; e2 < M->npr[j]; ++e2) {
            const double cc = conc[M->pidx[j][e2]][tid];
            const int pw = M->pnu[j][e2] - (e2 == e ? 1 : 0);
            for (int kk = 0; kk < pw; ++kk) dp *= cc;
          }
          const int sp = M->pidx[j][e];
#pragma unroll
          for (int k = 0; k < NS; ++k)
            if (k == sp) cb[k] -= qb * dp;
        }
        lnkfb = qb * (rf - rbk);
        const double lnKcb = qb * rbk;
        Tbar += lnkfb * (M->beta[j] * iT + M->EaR[j] * iT * iT) + lnKcb * dlnKc;
      }
      block_sum_to(lnkfb, wred, &thpart[(long long)blockIdx.x * nth + 4 + j]);
    }
  } else if (tid == 0) {
    for (int j = 0; j < nr; ++j) thpart[(long long)blockIdx.x * nth + 4 + j] = 0.0;
  }
  // ---- phase 3: transport, EOS, implicit Newton T, conserved variables
  double thE = 0.0, thx[3] = {0.0, 0.0, 0.0};
  if (live) {
#pragma unroll
    for (int k = 0; k < NS; ++k) rb[k] += cb[k] * M->iW[k];
    double pbar = pbv[PB_P * N + q];
    const double cbar = pbv[PB_C * N + q];
    const double mub = pbv[PB_MU * N + q], lamb_ = pbv[PB_LAM * N + q];
    double iWm = 0.0, cp = 0.0, dcp = 0.0;
#pragma unroll
    for (int k = 0; k < NS; ++k) {
      iWm += Y[k] * M->iW[k];
      cp += Y[k] * M->RW[k] * cpRa(M, k, T);
      dcp += Y[k] * M->RW[k] * dcpRa(M, k, T);
    }
    const double Wm = 1.0 / iWm;
    const double p = rho * RU * T * iWm;
    const double cv = cp - RU * iWm;
    const double z = cp / cv * p * irho;
    const double cs = sqrt(z);
#pragma unroll
    for (int k = 0; k < NS; ++k) X[k] = Y[k] * Wm * M->iW[k];
    const double sqT = sqrt(T), T15 = T * sqT;
    // Bird mixture diffusivities
    {
      double Dacc[NS];
#pragma unroll
      for (int k = 0; k < NS; ++k) Dacc[k] = 0.0;
#pragma unroll
      for (int i = 0; i < NS; ++i)
#pragma unroll
        for (int j = i + 1; j < NS; ++j) {
          double dd;
          const double om = om11a(lnT - M->Dlneps[i][j], T * M->Dieps[i][j], iT, M->Dieps[i][j], &dd);
          const double iD = p * om / (M->Dpre[i][j] * T15);
          Dacc[i] += fmax(X[j], 0.0) * iD;
          Dacc[j] += fmax(X[i], 0.0) * iD;
        }
      double Daccb[NS];
#pragma unroll
      for (int k = 0; k < NS; ++k) {
        const double Db = pbv[(PB_D + k) * N + q];
        if (Dacc[k] < 1e-300) {
          double dd;
          const double om = om11a(lnT - M->Dlneps[k][k], T * M->Dieps[k][k], iT, M->Dieps[k][k], &dd);
          const double Dk = M->Dpre[k][k] * T15 / (p * om);
          pbar += -Db * Dk / p;
          Tbar += Db * Dk * (1.5 * iT - dd / om);
          Daccb[k] = 0.0;
        } else {
          const double Dk = (1.0 - Y[k]) / Dacc[k];
          Yb[k] += -Db / Dacc[k];
          Daccb[k] = -Db * Dk / Dacc[k];
        }
      }
#pragma unroll
      for (int i = 0; i < NS; ++i)
#pragma unroll
        for (int j = i + 1; j < NS; ++j) {
          double dd;
          const double om = om11a(lnT - M->Dlneps[i][j], T * M->Dieps[i][j], iT, M->Dieps[i][j], &dd);
          const double iD = p * om / (M->Dpre[i][j] * T15);
          if (X[j] > 0.0) Xb[j] += Daccb[i] * iD;
          if (X[i] > 0.0) Xb[i] += Daccb[j] * iD;
          const double iDb = Daccb[i] * fmax(X[j], 0.0) + Daccb[j] * fmax(X[i], 0.0);
          pbar += iDb * iD / p;
          Tbar += iDb * iD * (dd / om - 1.5 * iT);
        }
    }
    // Wilke viscosity and conductivity
    {
      double mus[NS], lams[NS], smu[NS], ismu[NS], dlnom[NS], cpk[NS];
#pragma unroll
      for (int k = 0; k < NS; ++k) {
        double dd;
        const double om = om22a(lnT - M->lneps[k], T * M->ieps[k], iT, M->ieps[k], &dd);
        mus[k] = M->mu_pre[k] * sqT / om;
        dlnom[k] = dd / om;
        cpk[k] = M->RW[k] * cpRa(M, k, T) + M->euck[k];
        lams[k] = mus[k] * cpk[k];
        smu[k] = sqrt(mus[k]);
        ismu[k] = 1.0 / smu[k];
      }
      double musb[NS], smub[NS], ismub[NS];
#pragma unroll
      for (int k = 0; k < NS; ++k) musb[k] = smub[k] = ismub[k] = 0.0;
#pragma unroll
      for (int i = 0; i < NS; ++i) {
        double den = 0.0;
#pragma unroll
        for (int j = 0; j < NS; ++j) {
          const double t1 = 1.0 + smu[i] * ismu[j] * M->wq[i][j];
          den += X[j] * (t1 * t1 * M->wp[i][j]);
        }
        const double id = 1.0 / den;
        Xb[i] += mub * mus[i] * id + lamb_ * lams[i] * id;
        musb[i] += mub * X[i] * id;
        const double lsb = lamb_ * X[i] * id;
        musb[i] += lsb * cpk[i];
        Tbar += lsb * mus[i] * M->RW[i] * dcpRa(M, i, T);
        const double denb = -(mub * X[i] * mus[i] + lamb_ * X[i] * lams[i]) * id * id;
#pragma unroll
        for (int j = 0; j < NS; ++j) {
          const double t1 = 1.0 + smu[i] * ismu[j] * M->wq[i][j];
          Xb[j] += denb * t1 * t1 * M->wp[i][j];
          const double t1b = denb * X[j] * 2.0 * t1 * M->wp[i][j];
          smub[i] += t1b * ismu[j] * M->wq[i][j];
          ismub[j] += t1b * smu[i] * M->wq[i][j];
        }
      }
#pragma unroll
      for (int k = 0; k < NS; ++k) {
        smub[k] += -ismub[k] * ismu[k] * ismu[k];
        musb[k] += smub[k] * 0.5 * ismu[k];
        Tbar += musb[k] * mus[k] * (0.5 * iT - dlnom[k]);
      }
    }
    // EOS, sound speed, mole fractions
    double iWmb = 0.0, rhob = 0.0, cpb = 0.0, cvb = 0.0, Wmb = 0.0;
#pragma unroll
    for (int k = 0; k < NS; ++k) {
      Yb[k] += Xb[k] * Wm * M->iW[k];
      Wmb += Xb[k] * Y[k] * M->iW[k];
    }
    const double zb = cbar * 0.5 / cs;
    cpb += zb * p * irho / cv;
    cvb += -zb * z / cv;
    pbar += zb * z / p;
    rhob += -zb * z * irho;
    cpb += cvb;
    iWmb += -RU * cvb;
    rhob += pbar * RU * T * iWm;
    Tbar += pbar * p * iT;
    iWmb += pbar * rho * RU * T;
    iWmb += -Wmb * Wm * Wm;
    Tbar += cpb * dcp;
#pragma unroll
    for (int k = 0; k < NS; ++k) Yb[k] += cpb * M->RW[k] * cpRa(M, k, T) + iWmb * M->iW[k];
    // implicit Newton temperature: e(T, Y) = e with c_v = de/dT
    const double eb = Tbar / cv;
#pragma unroll
    for (int k = 0; k < NS; ++k) Yb[k] += -Tbar * M->RW[k] * T * (hRTa(M, k, T, iT) - 1.0) / cv;
    // e = E / rho - |u|^2 / 2, u = m / rho, Y = r / rho, rho = sum r
    const double Eb = eb * irho;
    rhob += -eb * E * irho * irho;
    double mb[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      ub[a] += -eb * u[a];
      mb[a] = ub[a] * irho;
      rhob += -ub[a] * u[a] * irho;
    }
#pragma unroll
    for (int k = 0; k < NS; ++k) {
      rb[k] += Yb[k] * irho;
      rhob += -Yb[k] * Y[k] * irho;
    }
    double* out = outb + NV * G.off;
#pragma unroll
    for (int k = 0; k < NS; ++k) out[k * N + q] += rb[k] + rhob;
#pragma unroll
    for (int a = 0; a < 3; ++a) out[(NS + a) * N + q] += ubd[(NS + a) * N + q] + mb[a];
    out[(NS + 3) * N + q] += ubd[(NS + 3) * N + q] + Eb;
    // laser parameters: q_L = E norm prod_a G_a exp(-((t - t0)/st)^2 / 2)
    const LaserDev& L = A.use_call_laser ? A.laser : G.laser;
    if (L.on) {
      const double tk = (A.t_dev ? A.t_dev[m] : A.t) + (A.dt_dev ? A.tcoef * A.dt_dev[m] : 0.0);
      const double tt = (tk - L.t0) / L.st;
      const double tf = exp(-0.5 * tt * tt);
      const int cidx[3] = {ix, jx, kx};
      double Ga[3], dGa[3];
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        Ga[a] = 1.0;
        dGa[a] = 0.0;
        if (!G.act[a]) continue;
        const double Lp = G.L[a];
        double rr = G.xnode[a][cidx[a]] - L.xc[a];
        rr -= Lp * rint(rr / Lp);
        double g = 0.0, dg = 0.0;
        for (int mm = -L.M[a]; mm <= L.M[a]; ++mm) {
          const double zz = (rr - mm * Lp) / L.sr;
          const double ex = exp(-0.5 * zz * zz);
          g += ex;
          dg += ex * zz / L.sr;          // d/d(centre) of exp(-zz^2/2)
        }
        Ga[a] = g;
        dGa[a] = dg;
      }
      const double qLb = s * lam[(NS + 3) * N + q];
      const double base = L.norm * tf;
      thE = qLb * base * Ga[0] * Ga[1] * Ga[2];
      thx[0] = qLb * L.E * base * dGa[0] * Ga[1] * Ga[2];
      thx[1] = qLb * L.E * base * Ga[0] * dGa[1] * Ga[2];
      thx[2] = qLb * L.E * base * Ga[0] * Ga[1] * dGa[2];
    }
  }
  // ---- phase 4: laser parameter partials (every thread)
  block_sum_to(thE, wred, &thpart[(long long)blockIdx.x * nth + 0]);
  block_sum_to(thx[0], wred, &thpart[(long long)blockIdx.x * nth + 1]);
  block_sum_to(thx[1], wred, &thpart[(long long)blockIdx.x * nth + 2]);
  block_sum_to(thx[2], wred, &thpart[(long long)blockIdx.x * nth + 3]);
}

// One block per member: fixed-order sums of the parameter partials.
__global__ __launch_bounds__(BLK) void k_adj_theta(const Member* __restrict__ mem, const double* __restrict__ thpart,
                                                   int nth, double* __restrict__ pbar) {
  __shared__ double sh[BLK];
  const Member& G = mem[blockIdx.x];
  const int tid = threadIdx.x;
  for (int i = 0; i < nth; ++i) {
    double a = 0.0;
    for (int k = tid; k < G.nblocks; k += BLK) a += thpart[(long long)(G.block_begin + k) * nth + i];
    sh[tid] = a;
    __syncthreads();
    for (int o = BLK / 2; o > 0; o >>= 1) {
      if (tid < o) sh[tid] += sh[tid + o];
      __syncthreads();
    }
    if (tid == 0) pbar[(long long)blockIdx.x * nth + i] += sh[0];
    __syncthreads();
  }
}

// y = a x + b y over n doubles (b = 0: y = a x)
__global__ void k_axpby(long long n, double a, const double* __restrict__ x, double b, double* __restrict__ y) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] = b == 0.0 ? a * x[i] : a * x[i] + b * y[i];
}

template <int NS>
static hipError_t adj_t(const MechTables* M, const Member* mem, int nmem, int nblocks, int ntblocks,
                        const CallArgs& a,
                        const double* U, const double* T, const double* aux, const unsigned char* flag,
                        const unsigned char* bits, const double* lam, double s, double h, double* ubd, double* pbv,
                        double* out, double* thpart, int nth, double psi_c, double CT, hipStream_t st) {
  hipLaunchKernelGGL((k_adj_conv_tiled<NS>), dim3(ntblocks), dim3(BLK), 0, st, mem, nmem, a, U, aux, flag, lam, s,
                     ubd, pbv, bits, psi_c, CT);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (!(a.flags & HTR_VISC_OFF)) {
    hipLaunchKernelGGL(k_adj_diff<NS>, dim3(nblocks), dim3(BLK), 0, st, M, mem, nmem, U, T, aux, lam, s, ubd, pbv);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_adj_point<NS>, dim3(nblocks), dim3(BLK), 0, st, M, mem, nmem, a, U, T, pbv, ubd, lam, s, h, out,
                     thpart, nth);
  return hipGetLastError();
}

hipError_t launch_adjoint(int ns, const MechTables* M, const Member* mem, int nmem, int nblocks, int ntblocks,
                          const CallArgs& a,
                          const double* U, const double* T, const double* aux, const unsigned char* flag,
                          const unsigned char* bits, const double* lam, double s, double h, double* ubd, double* pbv,
                          double* out, double* thpart, int nth, double psi_c, double CT, hipStream_t st) {
#define C_(NS)                                                                                                   \
  adj_t<NS>(M, mem, nmem, nblocks, ntblocks, a, U, T, aux, flag, bits, lam, s, h, ubd, pbv, out, thpart, nth, psi_c, \
            CT, st)
  switch (ns) {
    case 1: return C_(1); case 2: return C_(2); case 3: return C_(3);
    case 4: return C_(4); case 5: return C_(5); case 6: return C_(6);
    case 7: return C_(7); case 8: return C_(8); case 9: return C_(9);
    case 10: return C_(10); case 11: return C_(11); case 12: return C_(12);
    default: return hipErrorInvalidValue;
  }
#undef C_
}

hipError_t launch_adj_theta(const Member* mem, int nmem, const double* thpart, int nth, double* pbar,
                            hipStream_t st) {
  hipLaunchKernelGGL(k_adj_theta, dim3(nmem), dim3(BLK), 0, st, mem, thpart, nth, pbar);
  return hipGetLastError();
}

hipError_t launch_axpby(long long n, double a, const double* x, double b, double* y, hipStream_t st) {
  hipLaunchKernelGGL(k_axpby, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, n, a, x, b, y);
  return hipGetLastError();
}

}  // namespace htr
