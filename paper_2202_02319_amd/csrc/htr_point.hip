// Per-cell kernels: conserved state from primitives, and the point kernel
// (primitives with Newton for T, mixture-averaged transport, finite-rate
// chemistry, laser source, heat release, stable-step limit), plus the
// dilatation sensor and the per-member reductions.
//
// Paper (arXiv 2202.02319) Methods › Solver: eqs. (1)-(4), Wilke viscosity, NASA
// thermodynamics, heat flux eq. (5), diffusion velocity eq. (6) with Bird
// mixture-averaged and Hirschfelder binary diffusivities, Arrhenius
// chemistry; Methods › Diffusion flame › Physical model and numerical setup eq. (laser-qs) for q_L.
//
// One thread per cell.  The species count is a compile-time parameter so
// that every per-species array lives in registers; species concentrations
// used by the mass-action products (indexed by a reaction's species list)
// are staged in LDS, one column per thread.

#include <math.h>

#include "htr_dev.h"

namespace htr {

__device__ __forceinline__ double cpR(const MechTables* __restrict__ M, int s, double T) {
  const double* a = M->cp[s];
  return a[0] + T * (a[1] + T * (a[2] + T * (a[3] + T * a[4])));
}
__device__ __forceinline__ double hRT(const MechTables* __restrict__ M, int s, double T, double iT) {
  const double* a = M->hc[s];
  return a[0] + T * (a[1] + T * (a[2] + T * (a[3] + T * a[4]))) + a[5] * iT;
}
__device__ __forceinline__ double sR(const MechTables* __restrict__ M, int s, double T, double lnT) {
  const double* a = M->sc[s];
  return a[0] * lnT + T * (a[1] + T * (a[2] + T * (a[3] + T * a[4]))) + a[5];
}

// Neufeld-Janzen-Aziz collision integrals; x = ln T - ln(eps/k), Ts = T/(eps/k).
__device__ __forceinline__ double om22(double x, double Ts) {
  return 1.16145 * exp(-0.14874 * x) + 0.52487 * exp(-0.77320 * Ts) + 2.16178 * exp(-2.43787 * Ts);
}
__device__ __forceinline__ double om11(double x, double Ts) {
  return 1.06036 * exp(-0.15610 * x) + 0.19300 * exp(-0.47635 * Ts) + 1.03587 * exp(-1.52996 * Ts) +
         1.76474 * exp(-3.89411 * Ts);
}

__device__ __forceinline__ double laser_axis(const LaserDev& L, const Member& G, int a, int i) {
  if (!G.act[a]) return 1.0;
  if (G.bc[a][0] != 0) {   // bounded axis: no periodic images
    const double z = (G.xnode[a][i] - L.xc[a]) / L.sr;
    return exp(-0.5 * z * z);
  }
  const double Lp = G.L[a];
  double r = G.xnode[a][i] - L.xc[a];
  r -= Lp * rint(r / Lp);
  double g = 0.0;
  for (int m = -L.M[a]; m <= L.M[a]; ++m) {
    const double z = (r - m * Lp) / L.sr;
    g += exp(-0.5 * z * z);
  }
  return g;
}

// Laser kernel on a curvilinear grid: the Gaussian of the distance to the
// centre summed over the lattice images (nearest image in lattice
// coordinates, then M[a] periods each way along the active axes; an
// inactive axis drops its coordinate).
__device__ __forceinline__ double laser_curv(const LaserDev& L, const Member& G, const CurvGeom& cg, long long q) {
  const long long N = G.N;
  double r[3], sl[3], rm[3];
#pragma unroll
  for (int c = 0; c < 3; ++c) r[c] = cg.xyz[c * N + q] - L.xc[c];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const double v = cg.Pinv[a][0] * r[0] + cg.Pinv[a][1] * r[1] + cg.Pinv[a][2] * r[2];
    sl[a] = G.act[a] ? v - rint(v) : 0.0;
  }
#pragma unroll
  for (int c = 0; c < 3; ++c) rm[c] = sl[0] * cg.P[0][c] + sl[1] * cg.P[1][c] + sl[2] * cg.P[2][c];
  const double h = -0.5 / (L.sr * L.sr);
  // no images along an inactive axis (its coordinate is dropped)
  const int M0 = G.act[0] ? L.M[0] : 0, M1 = G.act[1] ? L.M[1] : 0, M2 = G.act[2] ? L.M[2] : 0;
  double g = 0.0;
  for (int m0 = -M0; m0 <= M0; ++m0)
    for (int m1 = -M1; m1 <= M1; ++m1)
      for (int m2 = -M2; m2 <= M2; ++m2) {
        double r2 = 0.0;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          const double z = rm[c] - (m0 * cg.P[0][c] + m1 * cg.P[1][c] + m2 * cg.P[2][c]);
          r2 += z * z;
        }
        g += exp(h * r2);
      }
  return g;
}

// ----------------------------------------------------------- prim -> cons
template <int NS>
__global__ __launch_bounds__(BLK) void k_prim_to_cons(const MechTables* __restrict__ M, const Member* __restrict__ mem,
                                                      int nmem, const double* __restrict__ Yb,
                                                      const double* __restrict__ Tb, const double* __restrict__ pb,
                                                      const double* __restrict__ vb, double* __restrict__ Ub) {
  const int m = find_member(mem, nmem, blockIdx.x);
  const Member& G = mem[m];
  const long long q = (long long)(blockIdx.x - G.block_begin) * BLK + threadIdx.x;
  if (q >= G.N) return;
  const long long N = G.N;
  const double* Y = Yb + NS * G.off;
  const double* vel = vb + 3 * G.off;
  double* U = Ub + (NS + 4) * G.off;
  const double T = Tb[G.off + q], p = pb[G.off + q], iT = 1.0 / T;
  double iW = 0.0, hm = 0.0;
#pragma unroll
  for (int s = 0; s < NS; ++s) {
    const double y = Y[s * N + q];
    iW += y * M->iW[s];
    hm += y * M->RW[s] * T * hRT(M, s, T, iT);
  }
  const double rho = p / (RU * T * iW);
#pragma unroll
  for (int s = 0; s < NS; ++s) U[s * N + q] = rho * Y[s * N + q];
  double ke = 0.0;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const double v = vel[a * N + q];
    U[(NS + a) * N + q] = rho * v;
    ke += v * v;
  }
  U[(NS + 3) * N + q] = rho * hm - p + 0.5 * rho * ke;
}

// ------------------------------------------------------------------ point
// aux rows per cell: 0 p, 1 c, 2 mu, 3 lambda, 4..6 velocity, 7.. D_s.
// src rows: 0..NS-1 wdot_s, NS q_L.  blkred per block: {sum dV hrr, min dt limit}.
// One logical block bl of 256 cells.
// CURV: curvilinear single grid (laser over lattice images, contravariant
// dt limit, cell volume 1/J from the metric terms in cg).
template <int NS, bool CURV>
__device__ __forceinline__ void point_block(int bl, const MechTables* __restrict__ M,
                                            const Member* __restrict__ mem, int nmem, const CallArgs& A,
                                            const double* __restrict__ Ub, double* __restrict__ Tb,
                                            double* __restrict__ auxb, double* __restrict__ srcb,
                                            double* __restrict__ hrrb, double* __restrict__ blkred,
                                            double* __restrict__ cellsb, unsigned* __restrict__ status,
                                            int want_dt, const CurvGeom& cg) {
  constexpr int NV = NS + 4, NAUX = 7 + NS;
  __shared__ double conc[NS][BLK];
  __shared__ double wred[2][BLK / 64];
  const int m = find_member(mem, nmem, bl);
  const Member& G = mem[m];
  const int tid = threadIdx.x;
  const long long q = (long long)(bl - G.block_begin) * BLK + tid;
  const bool live = q < G.N;
  const long long N = G.N;
  const unsigned flags = A.flags;
  double hdv = 0.0, lim = INFINITY;
  if (live) {
    const double* U = Ub + NV * G.off;
    double* aux = auxb + NAUX * G.off;
    double* src = srcb + (NS + 1) * G.off;
    double r[NS], Y[NS];
    double rho = 0.0;
    bool finite = true;
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      r[s] = U[s * N + q];
      rho += r[s];
      finite = finite && isfinite(r[s]);
      // molar concentrations for the reaction products (per-thread LDS column)
      conc[s][tid] = r[s] * M->iW[s];
    }
    const double mx = U[NS * N + q], my = U[(NS + 1) * N + q], mz = U[(NS + 2) * N + q];
    const double E = U[(NS + 3) * N + q];
    finite = finite && isfinite(mx) && isfinite(my) && isfinite(mz) && isfinite(E);
    unsigned err = 0;
    if (!finite || !(rho > 0.0)) err = ST_NONFINITE;
    const double irho = 1.0 / rho;
#pragma unroll
    for (int s = 0; s < NS; ++s) Y[s] = r[s] * irho;
    const double u = mx * irho, v = my * irho, w = mz * irho;
    const double e = E * irho - 0.5 * (u * u + v * v + w * w);
    // temperature: Newton on e(T) = sum_s Y_s (h_s - R_u T / W_s); converge, then one more step
    double T = Tb[G.off + q];
    bool conv = false;
    if (!err) {
      for (int it = 0; it < 50; ++it) {
        const double iT = 1.0 / T;
        double eT = 0.0, cv = 0.0;
#pragma unroll
        for (int s = 0; s < NS; ++s) {
          const double yr = Y[s] * M->RW[s];
          eT += yr * T * (hRT(M, s, T, iT) - 1.0);
          cv += yr * (cpR(M, s, T) - 1.0);
        }
        const double dT = (eT - e) / cv;
        T -= dT;
        if (!isfinite(T) || !(T > 0.0)) break;
        if (fabs(dT) <= 1e-12 * fabs(T)) {
          const double iT2 = 1.0 / T;
          double eT2 = 0.0, cv2 = 0.0;
#pragma unroll
          for (int s = 0; s < NS; ++s) {
            const double yr = Y[s] * M->RW[s];
            eT2 += yr * T * (hRT(M, s, T, iT2) - 1.0);
            cv2 += yr * (cpR(M, s, T) - 1.0);
          }
          T -= (eT2 - e) / cv2;
          conv = true;
          break;
        }
      }
      if (!conv) err = ST_NEWTON;
      else if (T < M->Tmin || T > M->Tmax) err = ST_TRANGE;
    }
    if (err) {
      atomicOr(status, err);
      T = NAN;
    }
    Tb[G.off + q] = T;
    const double iT = 1.0 / T;
    double iWm = 0.0, cp = 0.0;
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      iWm += Y[s] * M->iW[s];
      cp += Y[s] * M->RW[s] * cpR(M, s, T);
    }
    const double Wm = 1.0 / iWm;
    const double p = rho * RU * T * iWm;
    const double c = sqrt(cp / (cp - RU * iWm) * p * irho);
    aux[0 * N + q] = p;
    aux[1 * N + q] = c;
    aux[4 * N + q] = u;
    aux[5 * N + q] = v;
    aux[6 * N + q] = w;
    double X[NS];
#pragma unroll
    for (int s = 0; s < NS; ++s) X[s] = Y[s] * Wm * M->iW[s];

    // ---- transport.  The power terms of the collision integrals factor:
    // (T/eps)^-b = T^-b eps^b, one exponential per cell for each fit.
    const double lnT = log(T), sqT = sqrt(T);
    const double Tb22 = exp(-0.14874 * lnT), Tb11 = exp(-0.15610 * lnT);
    // (lambda_s and sqrt(mu_s) are formed where they are used, so that only
    // mu_s and 1/sqrt(mu_s) are held for all species)
    double mus[NS], ismu[NS];
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      const double Ts = T * M->ieps[s];
      const double o22 = 1.16145 * (Tb22 * M->pw22[s]) + 0.52487 * exp(-0.77320 * Ts) + 2.16178 * exp(-2.43787 * Ts);
      mus[s] = M->mu_pre[s] * sqT / o22;
      ismu[s] = 1.0 / sqrt(mus[s]);
    }
    double mu = 0.0, lam = 0.0;
#pragma unroll
    for (int i = 0; i < NS; ++i) {
      const double smu = sqrt(mus[i]);
      double den = 0.0;
#pragma unroll
      for (int j = 0; j < NS; ++j) {
        const double t1 = 1.0 + smu * ismu[j] * M->wq[i][j];
        den += X[j] * (t1 * t1 * M->wp[i][j]);
      }
      const double id = 1.0 / den;
      const double lams = mus[i] * (M->RW[i] * cpR(M, i, T) + M->euck[i]);
      mu += X[i] * mus[i] * id;
      lam += X[i] * lams * id;
    }
    aux[2 * N + q] = mu;
    aux[3 * N + q] = lam;
    double Dacc[NS], Ds[NS];
#pragma unroll
    for (int s = 0; s < NS; ++s) Dacc[s] = 0.0;
    const double T15 = T * sqT, pT15 = p / T15;
#pragma unroll
    for (int i = 0; i < NS; ++i) {
#pragma unroll
      for (int j = i + 1; j < NS; ++j) {
        const double Ts = T * M->Dieps[i][j];
        const double o11 = 1.06036 * (Tb11 * M->pw11[i][j]) + 0.19300 * exp(-0.47635 * Ts) +
                           1.03587 * exp(-1.52996 * Ts) + 1.76474 * exp(-3.89411 * Ts);
        const double iD = pT15 * o11 * M->iDpre[i][j];
        Dacc[i] += fmax(X[j], 0.0) * iD;
        Dacc[j] += fmax(X[i], 0.0) * iD;
      }
    }
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      if (Dacc[s] < 1e-300) {
        const double Ts = T * M->Dieps[s][s];
        Ds[s] = M->Dpre[s][s] * T15 / (p * om11(lnT - M->Dlneps[s][s], Ts));
      } else {
        Ds[s] = (1.0 - Y[s]) / Dacc[s];
      }
    }
#pragma unroll
    for (int s = 0; s < NS; ++s) aux[(7 + s) * N + q] = Ds[s];

    // ---- chemistry
    double om[NS];
#pragma unroll
    for (int s = 0; s < NS; ++s) om[s] = 0.0;
    double hrr = 0.0;
    if (!(flags & HTR_CHEM_OFF)) {
      double Gs[NS];
#pragma unroll
      for (int s = 0; s < NS; ++s) Gs[s] = hRT(M, s, T, iT) - sR(M, s, T, lnT);
      const double lnP = log(PREF / (RU * T));
      const double* dlnA = A.dlnA ? A.dlnA : G.dlnA;
      const int nr = M->nr;
      for (int j = 0; j < nr; ++j) {
        double lnkf = M->lnA[j] + M->beta[j] * lnT - M->EaR[j] * iT;
        if (dlnA) lnkf += dlnA[j];
        double lnKc = M->dnu[j] * lnP;
#pragma unroll
        for (int s = 0; s < NS; ++s) lnKc -= M->nunet[j][s] * Gs[s];
        double rf = exp(lnkf), rb = exp(lnkf - lnKc);
        for (int e = 0; e < M->nre[j]; ++e) {
          const double cs = conc[M->ridx[j][e]][tid];
          for (int k = 0; k < M->rnu[j][e]; ++k) rf *= cs;
        }
        for (int e = 0; e < M->npr[j]; ++e) {
          const double cs = conc[M->pidx[j][e]][tid];
          for (int k = 0; k < M->pnu[j][e]; ++k) rb *= cs;
        }
        const double qj = rf - rb;
#pragma unroll
        for (int s = 0; s < NS; ++s) om[s] += M->nunet[j][s] * qj;
      }
#pragma unroll
      for (int s = 0; s < NS; ++s) {
        om[s] *= M->W[s];
        hrr -= M->RW[s] * T * hRT(M, s, T, iT) * om[s];
      }
    }
    // ---- laser
    const int i = (int)(q % G.n[0]), jj = (int)((q / G.n[0]) % G.n[1]), k = (int)(q / ((long long)G.n[0] * G.n[1]));
    const LaserDev& L = A.use_call_laser ? A.laser : G.laser;
    double qL = 0.0;
    if (L.on) {
      const double tk = (A.t_dev ? A.t_dev[m] : A.t) + (A.dt_dev ? A.tcoef * A.dt_dev[m] : 0.0);
      const double tt = (tk - L.t0) / L.st;
      const double gs = CURV ? laser_curv(L, G, cg, q)
                             : laser_axis(L, G, 0, i) * laser_axis(L, G, 1, jj) * laser_axis(L, G, 2, k);
      qL = L.E * L.norm * gs * exp(-0.5 * tt * tt);
    }
#pragma unroll
    for (int s = 0; s < NS; ++s) src[s * N + q] = om[s];
    src[NS * N + q] = qL;
    if (hrrb) hrrb[G.off + q] = hrr;
    if (CURV) {
      const double Jq = cg.mt[9 * N + q];
      hdv = hrr / Jq;
      if (want_dt) {
        // contravariant speeds |u . grad xi_a| + c |grad xi_a|, grad xi_a = J mt_a
        double sc = 0.0, sd = 0.0;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
          if (!G.act[a]) continue;
          const double g0 = Jq * cg.mt[(3 * a) * N + q], g1 = Jq * cg.mt[(3 * a + 1) * N + q],
                       g2 = Jq * cg.mt[(3 * a + 2) * N + q];
          const double gg = g0 * g0 + g1 * g1 + g2 * g2;
          sc += fabs(u * g0 + v * g1 + w * g2) + c * sqrt(gg);
          sd += gg;
        }
        double nu = fmax(mu * irho, lam / (rho * cp));
#pragma unroll
        for (int s = 0; s < NS; ++s) nu = fmax(nu, Ds[s]);
        if (sc > 0.0) lim = 1.0 / sc;
        if (!(flags & HTR_VISC_OFF) && sd > 0.0) lim = fmin(lim, 1.0 / (2.0 * sd * nu));
      }
    }
    const double xi0 = CURV ? 1.0 : G.xin[0][i], xi1 = CURV ? 1.0 : G.xin[1][jj], xi2 = CURV ? 1.0 : G.xin[2][k];
    if (!CURV) hdv = hrr / (xi0 * xi1 * xi2);
    if (!CURV && want_dt) {
      double sc = 0.0, sd = 0.0;
      const double uu[3] = {u, v, w}, xx[3] = {xi0, xi1, xi2};
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        if (!G.act[a]) continue;
        sc += (fabs(uu[a]) + c) * xx[a];
        sd += xx[a] * xx[a];
      }
      double nu = fmax(mu * irho, lam / (rho * cp));
#pragma unroll
      for (int s = 0; s < NS; ++s) nu = fmax(nu, Ds[s]);
      if (sc > 0.0) lim = 1.0 / sc;
      if (!(flags & HTR_VISC_OFF) && sd > 0.0) lim = fmin(lim, 1.0 / (2.0 * sd * nu));
    }
    if (cellsb) {
      double* out = cellsb + (5 + 2 * NS + 3) * G.off;
      int row = 0;
      out[(row++) * N + q] = T;
      out[(row++) * N + q] = p;
      out[(row++) * N + q] = c;
      out[(row++) * N + q] = mu;
      out[(row++) * N + q] = lam;
#pragma unroll
      for (int s = 0; s < NS; ++s) out[(row++) * N + q] = Ds[s];
#pragma unroll
      for (int s = 0; s < NS; ++s) out[(row++) * N + q] = om[s];
      out[(row++) * N + q] = hrr;
      out[(row++) * N + q] = qL;
    }
  }
  if (blkred) {
    // deterministic block reduction: butterfly within each wavefront, then in order
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      hdv += __shfl_xor(hdv, o, 64);
      lim = fmin(lim, __shfl_xor(lim, o, 64));
    }
    if ((tid & 63) == 0) {
      wred[0][tid >> 6] = hdv;
      wred[1][tid >> 6] = lim;
    }
    __syncthreads();
    if (tid == 0) {
      double sh = 0.0, sl = INFINITY;
      for (int k = 0; k < BLK / 64; ++k) {
        sh += wred[0][k];
        sl = fmin(sl, wred[1][k]);
      }
      blkred[2 * bl] = sh;
      blkred[2 * bl + 1] = sl;
    }
  }
}

// Grid-stride over the nlog logical blocks: one pass when the grid has one
// block per logical block, persistent blocks when it has fewer.
template <int NS, bool PERSIST, bool CURV>
__global__ __launch_bounds__(BLK, NS <= 9 ? 3 : 2) void k_point(const MechTables* __restrict__ M,
                                                                const Member* __restrict__ mem, int nmem, int nlog,
                                                                CallArgs A, const double* __restrict__ Ub,
                                                                double* __restrict__ Tb, double* __restrict__ auxb,
                                                                double* __restrict__ srcb, double* __restrict__ hrrb,
                                                                double* __restrict__ blkred,
                                                                double* __restrict__ cellsb,
                                                                unsigned* __restrict__ status, int want_dt,
                                                                CurvGeom cg) {
  if (!PERSIST) {
    point_block<NS, CURV>(blockIdx.x, M, mem, nmem, A, Ub, Tb, auxb, srcb, hrrb, blkred, cellsb, status, want_dt,
                          cg);
    return;
  }
  for (int bl = blockIdx.x; bl < nlog; bl += gridDim.x) {
    point_block<NS, CURV>(bl, M, mem, nmem, A, Ub, Tb, auxb, srcb, hrrb, blkred, cellsb, status, want_dt, cg);
    __syncthreads();   // the next logical block reuses the LDS
  }
}

// ----------------------------------------------------------------- sensor
// theta = (div u)^2 / ((div u)^2 + |curl u|^2 + 1e-300) with second-order
// central differences; flag = theta > theta_c.  Also stores the nodal
// velocity gradient (the tangential derivatives of the diffusive fluxes).
__device__ __forceinline__ void sensor_block(int bl, const Member* __restrict__ mem, int nmem,
                                             const double* __restrict__ auxb, int naux,
                                             unsigned char* __restrict__ flagb, double* __restrict__ gradb,
                                             double theta_c, double* __restrict__ theta_out, int nq) {
  const int m = find_member(mem, nmem, bl);
  const Member& G = mem[m];
  const long long q = (long long)(bl - G.block_begin) * BLK + threadIdx.x;
  if (q >= G.N) return;
  const long long N = G.N;
  const double* vel = auxb + naux * G.off + 4 * N;
  const int c[3] = {(int)(q % G.n[0]), (int)((q / G.n[0]) % G.n[1]), (int)(q / ((long long)G.n[0] * G.n[1]))};
  const long long stride[3] = {1, G.n[0], (long long)G.n[0] * G.n[1]};
  double g[3][3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
#pragma unroll
    for (int mm = 0; mm < 3; ++mm) g[a][mm] = 0.0;
    if (!G.act[a]) continue;
    const double xi = G.xin[a][c[a]];
    if (G.bc[a][0] != 0 && (c[a] == 0 || c[a] == G.n[a] - 1)) {
      // boundary node of a bounded axis: one-sided second order, inward
      const long long s1 = c[a] == 0 ? stride[a] : -stride[a];
#pragma unroll
      for (int mm = 0; mm < 3; ++mm) {
        const double v0 = vel[mm * N + q], v1 = vel[mm * N + q + s1], v2 = vel[mm * N + q + 2 * s1];
        g[a][mm] = c[a] == 0 ? xi * (-3.0 * v0 + 4.0 * v1 - v2) / 2.0 : xi * (3.0 * v0 - 4.0 * v1 + v2) / 2.0;
      }
      continue;
    }
    const long long qp = q + (wrapi(c[a] + 1, G.n[a]) - c[a]) * stride[a];
    const long long qm = q + (wrapi(c[a] - 1, G.n[a]) - c[a]) * stride[a];
#pragma unroll
    for (int mm = 0; mm < 3; ++mm) g[a][mm] = xi * (vel[mm * N + qp] - vel[mm * N + qm]) / 2.0;
  }
  if (gradb) {
    double* grad = gradb + 9 * G.off;
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int mm = 0; mm < 3; ++mm) grad[(3 * a + mm) * N + q] = g[a][mm];
  }
  const double div = g[0][0] + g[1][1] + g[2][2];
  const double wx = g[1][2] - g[2][1], wy = g[2][0] - g[0][2], wz = g[0][1] - g[1][0];
  const double d2 = div * div;
  const double th = d2 / (d2 + wx * wx + wy * wy + wz * wz + 1e-300);
  flagb[G.off + q] = th > theta_c ? 1 : 0;
  if (theta_out) theta_out[(nq - 1) * N + nq * G.off + q] = th;
}

template <bool PERSIST>
__global__ __launch_bounds__(BLK) void k_sensor(const Member* __restrict__ mem, int nmem, int nlog,
                                                const double* __restrict__ auxb, int naux,
                                                unsigned char* __restrict__ flagb, double* __restrict__ gradb,
                                                double theta_c, double* __restrict__ theta_out, int nq) {
  if (!PERSIST) {
    sensor_block(blockIdx.x, mem, nmem, auxb, naux, flagb, gradb, theta_c, theta_out, nq);
    return;
  }
  for (int bl = blockIdx.x; bl < nlog; bl += gridDim.x)
    sensor_block(bl, mem, nmem, auxb, naux, flagb, gradb, theta_c, theta_out, nq);
}

// ------------------------------------------------------------- reductions
// One block per member: fixed-order sums of that member's block partials.
__global__ __launch_bounds__(BLK) void k_finalize(const Member* __restrict__ mem, const double* __restrict__ blkred,
                                                  double cfl, double* __restrict__ dt_dev, double* __restrict__ J_dev,
                                                  const double* __restrict__ dt_in, double jcoef, int want_dt) {
  __shared__ double sh[BLK], sl[BLK];
  const Member& G = mem[blockIdx.x];
  const int tid = threadIdx.x;
  double a = 0.0, b = INFINITY;
  for (int k = tid; k < G.nblocks; k += BLK) {
    a += blkred[2 * (G.block_begin + k)];
    b = fmin(b, blkred[2 * (G.block_begin + k) + 1]);
  }
  sh[tid] = a;
  sl[tid] = b;
  __syncthreads();
  for (int o = BLK / 2; o > 0; o >>= 1) {
    if (tid < o) {
      sh[tid] += sh[tid + o];
      sl[tid] = fmin(sl[tid], sl[tid + o]);
    }
    __syncthreads();
  }
  if (tid == 0) {
    double dt = 0.0;
    if (want_dt) {
      dt = cfl * sl[0];
      dt_dev[blockIdx.x] = dt;
    } else if (dt_in) {
      dt = dt_in[blockIdx.x];
    }
    if (J_dev) J_dev[blockIdx.x] += jcoef * dt * sh[0];
  }
}

// One block per member: the largest value of a packed per-cell field over the
// member's cells (out[m] = that, or max(out[m], that) when accumulating).
__global__ __launch_bounds__(BLK) void k_member_max(const Member* __restrict__ mem,
                                                   const double* __restrict__ field, double* __restrict__ out,
                                                   int accumulate) {
  __shared__ double red[BLK / 64];
  const Member& G = mem[blockIdx.x];
  double mx = -INFINITY;
  for (long long q = threadIdx.x; q < G.N; q += BLK) mx = fmax(mx, field[G.off + q]);
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) mx = fmax(mx, __shfl_xor(mx, o, 64));
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = mx;
  __syncthreads();
  if (threadIdx.x == 0) {
    double r = red[0];
    for (int w = 1; w < BLK / 64; ++w) r = fmax(r, red[w]);
    out[blockIdx.x] = accumulate ? fmax(out[blockIdx.x], r) : r;
  }
}

__global__ void k_advance_time(int nmem, double* __restrict__ t_dev, const double* __restrict__ dt_dev) {
  const int m = blockIdx.x * blockDim.x + threadIdx.x;
  if (m < nmem) t_dev[m] += dt_dev[m];
}

// ---------------------------------------------------------------- launchers
template <int NS>
static hipError_t prim_to_cons_t(const MechTables* M, const Member* mem, int nmem, int nblocks, const double* Y,
                                 const double* T, const double* p, const double* vel, double* U, hipStream_t s) {
  hipLaunchKernelGGL(k_prim_to_cons<NS>, dim3(nblocks), dim3(BLK), 0, s, M, mem, nmem, Y, T, p, vel, U);
  return hipGetLastError();
}

template <int NS>
static hipError_t point_t(const MechTables* M, const Member* mem, int nmem, int nblocks, int grid,
                          const CallArgs& a, const double* U, double* T, double* aux, double* src, double* hrr,
                          double* blkred, double* cells, unsigned* status, int want_dt, hipStream_t s,
                          const CurvGeom* cg) {
  const CurvGeom none{};
  if (cg)   // curvilinear single grid: one block per logical block
    hipLaunchKernelGGL((k_point<NS, false, true>), dim3(nblocks), dim3(BLK), 0, s, M, mem, nmem, nblocks, a, U, T,
                       aux, src, hrr, blkred, cells, status, want_dt, *cg);
  else if (grid < nblocks)
    hipLaunchKernelGGL((k_point<NS, true, false>), dim3(grid), dim3(BLK), 0, s, M, mem, nmem, nblocks, a, U, T, aux,
                       src, hrr, blkred, cells, status, want_dt, none);
  else
    hipLaunchKernelGGL((k_point<NS, false, false>), dim3(grid), dim3(BLK), 0, s, M, mem, nmem, nblocks, a, U, T, aux,
                       src, hrr, blkred, cells, status, want_dt, none);
  return hipGetLastError();
}

// grid <= 0 or >= nblocks: one block per logical block
static int grid_of(int nblocks, int grid) { return (grid <= 0 || grid > nblocks) ? nblocks : grid; }

hipError_t launch_prim_to_cons(int ns, const MechTables* M, const Member* mem, int nmem, int nblocks,
                               const double* Y, const double* T, const double* p, const double* vel, double* U,
                               hipStream_t s) {
#define C_(NS) prim_to_cons_t<NS>(M, mem, nmem, nblocks, Y, T, p, vel, U, s)
  HTR_NS_SWITCH(ns, C_)
#undef C_
}

hipError_t launch_point(int ns, const MechTables* M, const Member* mem, int nmem, int nblocks, int grid,
                        const CallArgs& a, const double* U, double* T, double* aux, double* src, double* hrr,
                        double* blkred, double* cells, unsigned* status, int want_dt, hipStream_t s,
                        const CurvGeom* cg) {
  grid = grid_of(nblocks, grid);
#define C_(NS) point_t<NS>(M, mem, nmem, nblocks, grid, a, U, T, aux, src, hrr, blkred, cells, status, want_dt, s, cg)
  HTR_NS_SWITCH(ns, C_)
#undef C_
}

hipError_t launch_sensor(const Member* mem, int nmem, int nblocks, int grid, const double* aux, int ns,
                         unsigned char* flag, double* grad, double theta_c, double* theta_out, hipStream_t s) {
  grid = grid_of(nblocks, grid);
  if (grid < nblocks)
    hipLaunchKernelGGL(k_sensor<true>, dim3(grid), dim3(BLK), 0, s, mem, nmem, nblocks, aux, 7 + ns, flag, grad,
                       theta_c, theta_out, 5 + 2 * ns + 3);
  else
    hipLaunchKernelGGL(k_sensor<false>, dim3(grid), dim3(BLK), 0, s, mem, nmem, nblocks, aux, 7 + ns, flag, grad,
                       theta_c, theta_out, 5 + 2 * ns + 3);
  return hipGetLastError();
}

hipError_t launch_member_max(const Member* mem, int nmem, const double* field, double* out, int accumulate,
                             hipStream_t s) {
  hipLaunchKernelGGL(k_member_max, dim3(nmem), dim3(BLK), 0, s, mem, field, out, accumulate);
  return hipGetLastError();
}

hipError_t launch_advance_time(int nmem, double* t_dev, const double* dt_dev, hipStream_t s) {
  hipLaunchKernelGGL(k_advance_time, dim3((nmem + 63) / 64), dim3(64), 0, s, nmem, t_dev, dt_dev);
  return hipGetLastError();
}

hipError_t launch_finalize(const Member* mem, int nmem, const double* blkred, double cfl, double* dt_dev,
                           double* J_dev, const double* dt_in, double jcoef, int want_dt, hipStream_t s) {
  hipLaunchKernelGGL(k_finalize, dim3(nmem), dim3(BLK), 0, s, mem, blkred, cfl, dt_dev, J_dev, dt_in, jcoef, want_dt);
  return hipGetLastError();
}

}  // namespace htr
