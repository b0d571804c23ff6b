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
// One thread per cell; each thread evaluates the two faces of its cell in
// each direction (the same face is evaluated bit-identically by both of its
// cells, so the scheme stays exactly conservative).  Node data come through
// the L1/L2 caches.

#include <math.h>

#include "htr_dev.h"
#include "htr_flux.h"

namespace htr {


// Convective contribution of direction d to acc[] (minus the flux difference).
template <int NS>
__device__ __forceinline__ void conv_dir(const Member& G, int d, const int c[3], long long q, long long N,
                                         const double* __restrict__ U, const double* __restrict__ aux,
                                         const unsigned char* __restrict__ flag, unsigned flags, double psi_c,
                                         double CT, double* acc) {
  constexpr int NV = NS + 4;
  const int n = G.n[d];
  const long long stride = d == 0 ? 1 : (d == 1 ? (long long)G.n[0] : (long long)G.n[0] * G.n[1]);
  long long qo[7];
  double ud[7], pp[7], cc[7];
  int fl = 0;
#pragma unroll
  for (int o = 0; o < 7; ++o) {
    qo[o] = q + (long long)(wrapi(c[d] + o - 3, n) - c[d]) * stride;
    ud[o] = aux[(4 + d) * N + qo[o]];
    pp[o] = aux[qo[o]];
    cc[o] = aux[N + qo[o]];
    fl |= (int)flag[qo[o]] << o;
  }
  // face L = c-1/2 uses nodes o = 0..5, face R = c+1/2 uses o = 1..6
  bool tL, tR;
  if (flags & HTR_FORCE_TENO) {
    tL = tR = true;
  } else if (flags & HTR_FORCE_CENTRAL) {
    tL = tR = false;
  } else {
    const double psiL = fabs(pp[3] - pp[2]) / fmin(pp[2], pp[3]);
    const double psiR = fabs(pp[4] - pp[3]) / fmin(pp[3], pp[4]);
    tL = (fl & 0x3f) != 0 || psiL > psi_c;
    tR = (fl & 0x7e) != 0 || psiR > psi_c;
  }
  double aL = 0.0, aR = 0.0;
  if (tL || tR) {
    double sp[7];
#pragma unroll
    for (int o = 0; o < 7; ++o) sp[o] = fabs(ud[o]) + cc[o];
    aL = sp[0];
#pragma unroll
    for (int o = 1; o < 6; ++o) aL = fmax(aL, sp[o]);
    aR = sp[1];
#pragma unroll
    for (int o = 2; o < 7; ++o) aR = fmax(aR, sp[o]);
  }
  const double xi = G.xin[d][c[d]];
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    double uv[7], f[7];
#pragma unroll
    for (int o = 0; o < 7; ++o) {
      uv[o] = U[v * N + qo[o]];
      f[o] = node_flux<NS>(v, d, uv[o], ud[o], pp[o]);
    }
    double F[2];
#pragma unroll
    for (int side = 0; side < 2; ++side) {
      const bool te = side ? tR : tL;
      const double* fs = f + side;
      if (!te) {
        // divided (not multiplied by 1/60) so that the rounding cannot be
        // fused into the face difference below: equal faces cancel exactly
        F[side] = (fs[0] - 8.0 * fs[1] + 37.0 * fs[2] + 37.0 * fs[3] - 8.0 * fs[4] + fs[5]) / 60.0;
      } else {
        const double al = side ? aR : aL;
        const double* us = uv + side;
        double fp[6], fm[6];
#pragma unroll
        for (int mm = 0; mm < 6; ++mm) {
          fp[mm] = 0.5 * (fs[mm] + al * us[mm]);
          fm[5 - mm] = 0.5 * (fs[mm] - al * us[mm]);
        }
        F[side] = teno6(fp, CT) + teno6(fm, CT);
      }
    }
    acc[v] -= xi * (F[1] - F[0]);
  }
}

// Diffusive flux at the face between nodes qA and qB (B = A + 1 along d),
// in the sign with which it enters the right-hand side, written to Fd[NV].
template <int NS>
__device__ __forceinline__ void diff_face(const MechTables* __restrict__ M, const Member& G, int d,
                                          const int cA[3], long long qA, long long qB, long long N,
                                          const double* __restrict__ U, const double* __restrict__ T,
                                          const double* __restrict__ aux, double* Fd) {
  const double xf = G.xif[d][cA[d]];
  int cB[3] = {cA[0], cA[1], cA[2]};
  cB[d] = wrapi(cA[d] + 1, G.n[d]);
  const long long strides[3] = {1, G.n[0], (long long)G.n[0] * G.n[1]};
  double uA[3], uB[3];
#pragma unroll
  for (int mm = 0; mm < 3; ++mm) {
    uA[mm] = aux[(4 + mm) * N + qA];
    uB[mm] = aux[(4 + mm) * N + qB];
  }
  // velocity gradient at the face, g[a][mm] = d u_mm / d x_a
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
    for (int side = 0; side < 2; ++side) {
      const int* cc = side ? cB : cA;
      const long long qc = side ? qB : qA;
      const long long qp = qc + (long long)(wrapi(cc[a] + 1, G.n[a]) - cc[a]) * strides[a];
      const long long qm = qc + (long long)(wrapi(cc[a] - 1, G.n[a]) - cc[a]) * strides[a];
      const double xa = 0.5 * G.xin[a][cc[a]];
#pragma unroll
      for (int mm = 0; mm < 3; ++mm) g[a][mm] += 0.5 * (xa * (aux[(4 + mm) * N + qp] - aux[(4 + mm) * N + qm]));
    }
  }
  const double muf = 0.5 * (aux[2 * N + qA] + aux[2 * N + qB]);
  const double lamf = 0.5 * (aux[3 * N + qA] + aux[3 * N + qB]);
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
    const double a = U[s * N + qA], b = U[s * N + qB];
    rA += a;
    rB += b;
    nA += a * M->iW[s];
    nB += b * M->iW[s];
  }
  const double rhof = 0.5 * (rA + rB);
  const double Wf = 0.5 * (rA / nA + rB / nB);
  const double inA = 1.0 / nA, inB = 1.0 / nB, irA = 1.0 / rA, irB = 1.0 / rB;
  double term[NS];
  double corr = 0.0;
#pragma unroll
  for (int s = 0; s < NS; ++s) {
    const double a = U[s * N + qA], b = U[s * N + qB];
    const double Df = 0.5 * (aux[(7 + s) * N + qA] + aux[(7 + s) * N + qB]);
    // both mole fractions rounded before differencing (no FMA across the
    // difference), so a uniform composition gives exactly zero flux
    double XA, XB;
    {
#pragma clang fp contract(off)
      XA = a * M->iW[s] * inA;
      XB = b * M->iW[s] * inB;
    }
    const double dX = xf * (XB - XA);
    term[s] = rhof * Df * (M->W[s] / Wf) * dX;
    corr += term[s];
  }
  const double TA = T[qA], TB = T[qB];
  double qn = -lamf * xf * (TB - TA);
#pragma unroll
  for (int s = 0; s < NS; ++s) {
    const double a = U[s * N + qA], b = U[s * N + qB];
    const double Yf = 0.5 * (a * irA + b * irB);
    const double J = -term[s] + Yf * corr;
    const double hf = 0.5 * (M->RW[s] * TA * hRTs(M, s, TA) + M->RW[s] * TB * hRTs(M, s, TB));
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

template <int NS>
__global__ __launch_bounds__(BLK) void k_sweep(const MechTables* __restrict__ M, const Member* __restrict__ mem,
                                               int nmem, CallArgs A, const double* __restrict__ Ub,
                                               const double* __restrict__ Unb, const double* __restrict__ Tb,
                                               const double* __restrict__ auxb, const double* __restrict__ srcb,
                                               const unsigned char* __restrict__ flagb, double* __restrict__ outb,
                                               double ca, double cb, int rhs_only, double psi_c, double CT) {
  constexpr int NV = NS + 4, NAUX = 7 + NS;
  const int m = find_member(mem, nmem, blockIdx.x);
  const Member& G = mem[m];
  const long long q = (long long)(blockIdx.x - G.block_begin) * BLK + threadIdx.x;
  if (q >= G.N) return;
  const long long N = G.N;
  const double* U = Ub + NV * G.off;
  const double* T = Tb + G.off;
  const double* aux = auxb + NAUX * G.off;
  const double* src = srcb + (NS + 1) * G.off;
  const unsigned char* flag = flagb + G.off;
  const int c[3] = {(int)(q % G.n[0]), (int)((q / G.n[0]) % G.n[1]), (int)(q / ((long long)G.n[0] * G.n[1]))};
  const long long strides[3] = {1, G.n[0], (long long)G.n[0] * G.n[1]};
  double acc[NV];
#pragma unroll
  for (int v = 0; v < NS; ++v) acc[v] = src[v * N + q];
  acc[NS] = acc[NS + 1] = acc[NS + 2] = 0.0;
  acc[NS + 3] = src[NS * N + q];
  const unsigned flags = A.flags;
  for (int d = 0; d < 3; ++d) {
    if (!G.act[d]) continue;
    conv_dir<NS>(G, d, c, q, N, U, aux, flag, flags, psi_c, CT, acc);
    if (!(flags & HTR_VISC_OFF)) {
      const double xi = G.xin[d][c[d]];
      int cm[3] = {c[0], c[1], c[2]};
      cm[d] = wrapi(c[d] - 1, G.n[d]);
      const long long qm = q + (long long)(cm[d] - c[d]) * strides[d];
      const long long qp = q + (long long)(wrapi(c[d] + 1, G.n[d]) - c[d]) * strides[d];
      double FL[NV], FR[NV];
      diff_face<NS>(M, G, d, cm, qm, q, N, U, T, aux, FL);
      diff_face<NS>(M, G, d, c, q, qp, N, U, T, aux, FR);
#pragma unroll
      for (int v = 0; v < NV; ++v) acc[v] += xi * (FR[v] - FL[v]);
    }
  }
  double* out = outb + NV * G.off;
  if (rhs_only) {
#pragma unroll
    for (int v = 0; v < NV; ++v) out[v * N + q] = acc[v];
  } else {
    const double dt = A.dt_dev[m];
    const double* Un = Unb + NV * G.off;
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      const double base = U[v * N + q] + dt * acc[v];
      out[v * N + q] = ca != 0.0 ? ca * Un[v * N + q] + cb * base : cb * base;
    }
  }
}

template <int NS>
static hipError_t sweep_t(const MechTables* M, const Member* mem, int nmem, int nblocks, const CallArgs& a,
                          const double* U, const double* Un, const double* T, const double* aux, const double* src,
                          const unsigned char* flag, double* out, double ca, double cb, int rhs_only, double psi_c,
                          double CT, hipStream_t s) {
  hipLaunchKernelGGL(k_sweep<NS>, dim3(nblocks), dim3(BLK), 0, s, M, mem, nmem, a, U, Un, T, aux, src, flag, out,
                     ca, cb, rhs_only, psi_c, CT);
  return hipGetLastError();
}

hipError_t launch_sweep(int ns, const MechTables* M, const Member* mem, int nmem, int nblocks, const CallArgs& a,
                        const double* U, const double* Un, const double* T, const double* aux, const double* src,
                        const unsigned char* flag, double* out, double ca, double cb, int rhs_only, double psi_c,
                        double CT, hipStream_t s) {
#define C_(NS) sweep_t<NS>(M, mem, nmem, nblocks, a, U, Un, T, aux, src, flag, out, ca, cb, rhs_only, psi_c, CT, s)
  switch (ns) {
    case 1: return C_(1); case 2: return C_(2); case 3: return C_(3);
    case 4: return C_(4); case 5: return C_(5); case 6: return C_(6);
    case 7: return C_(7); case 8: return C_(8); case 9: return C_(9);
    case 10: return C_(10); case 11: return C_(11); case 12: return C_(12);
    default: return hipErrorInvalidValue;
  }
#undef C_
}

}  // namespace htr
