// General curvilinear grids (Methods › Numerical method, the mapped equations): metric terms,
// sensor, mapped face fluxes and the stage update of a single-grid context.
//
// The equations are mapped to a uniform index space with U~ = U/J and
// F~_d = (d xi_d / d x) . (F, G, H) / J along each index direction,
// J = det(d xi / d x), index spacing 1.  Metric terms are evaluated in the
// conservative form of Thomas & Lombard,
//   (d xi_d / d x_c) / J = D_f[(D_e x_c1) x_c2] - D_e[(D_f x_c1) x_c2],
// (d, e, f) and (c, c1, c2) cyclic, D the sixth-order central difference,
// with the face values at i+1/2 the six-point interpolation whose face
// difference is D: the sum over directions of face-metric differences is a
// sum of commuting second differences, so a uniform flow stays uniform.
//
// Per stage: k_point (CURV variant: laser over lattice images, contravariant
// dt limit, volume 1/J) -> mole fractions and index-space central
// differences -> sensor -> convective and diffusive face kernels (all
// directions in one launch each: the hybrid scheme on the metric-projected
// flux; the diffusive flux by the chain rule) -> update.  These kernels are plain per-node/per-face
// launches through L1/L2; the tiled LDS sweeps serve rectilinear grids.
#include <hip/hip_runtime.h>

#include "htr_dev.h"
#include "htr_flux.h"

namespace htr {

__device__ __forceinline__ long long lin(const Member& G, int i, int j, int k) {
  return ((long long)k * G.n[1] + j) * G.n[0] + i;
}

// Coordinate c of lattice node (i, j, k), any integers (a node n[a] cells
// further along a is displaced by P[a]), minus x0.
__device__ __forceinline__ double lat(const Member& G, const CurvGeom& g, int c, int i, int j, int k, double x0) {
  const int id[3] = {i, j, k};
  int w[3];
  double sh = 0.0;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    w[a] = wrapi(id[a], G.n[a]);
    sh += (double)((id[a] - w[a]) / G.n[a]) * g.P[a][c];
  }
  return (g.xyz[c * G.N + lin(G, w[0], w[1], w[2])] + sh) - x0;
}

__device__ __forceinline__ void step(int p[3], const int b[3], int e, int m) {
  p[0] = b[0];
  p[1] = b[1];
  p[2] = b[2];
  p[e] += m;
}

// D6 along e of coordinate c (relative to x0) at lattice point b.
__device__ double d6x(const Member& G, const CurvGeom& g, int c, const int b[3], int e, double x0) {
  const double w[3] = {45.0, -9.0, 1.0};
  double s = 0.0;
  for (int m = 1; m <= 3; ++m) {
    int pp[3], pm[3];
    step(pp, b, e, m);
    step(pm, b, e, -m);
    s += w[m - 1] * (lat(G, g, c, pp[0], pp[1], pp[2], x0) - lat(G, g, c, pm[0], pm[1], pm[2], x0));
  }
  return s / 60.0;
}

// D6 along o of the product (D6_e x_c1) x_c2 at lattice point b.
__device__ double d6prod(const Member& G, const CurvGeom& g, int c1, int c2, const int b[3], int e, int o,
                         const double x0[3]) {
  const double w[3] = {45.0, -9.0, 1.0};
  double s = 0.0;
  for (int m = 1; m <= 3; ++m) {
    int pp[3], pm[3];
    step(pp, b, o, m);
    step(pm, b, o, -m);
    const double fp = d6x(G, g, c1, pp, e, x0[c1]) * lat(G, g, c2, pp[0], pp[1], pp[2], x0[c2]);
    const double fm = d6x(G, g, c1, pm, e, x0[c1]) * lat(G, g, c2, pm[0], pm[1], pm[2], x0[c2]);
    s += w[m - 1] * (fp - fm);
  }
  return s / 60.0;
}

// J = 1 / det(d x / d xi) at row 9, or 0 where the determinant is not
// positive and finite (the host checks every node before accepting the grid).
__global__ __launch_bounds__(BLK) void k_curv_metrics(const Member* __restrict__ mem, CurvGeom g,
                                                      double* __restrict__ mt) {
  const Member& G = mem[0];
  const long long q = (long long)blockIdx.x * BLK + threadIdx.x;
  if (q >= G.N) return;
  const long long N = G.N;
  const int b[3] = {(int)(q % G.n[0]), (int)((q / G.n[0]) % G.n[1]), (int)(q / ((long long)G.n[0] * G.n[1]))};
  double x0[3];
#pragma unroll
  for (int c = 0; c < 3; ++c) x0[c] = g.xyz[c * N + q];
  for (int d = 0; d < 3; ++d) {
    const int e = (d + 1) % 3, f = (d + 2) % 3;
    for (int c = 0; c < 3; ++c) {
      const int c1 = (c + 1) % 3, c2 = (c + 2) % 3;
      mt[(3 * d + c) * N + q] = d6prod(G, g, c1, c2, b, e, f, x0) - d6prod(G, g, c1, c2, b, f, e, x0);
    }
  }
  double A[3][3];
  for (int c = 0; c < 3; ++c)
    for (int e = 0; e < 3; ++e) A[c][e] = d6x(G, g, c, b, e, x0[c]);
  const double det = A[0][0] * (A[1][1] * A[2][2] - A[1][2] * A[2][1]) -
                     A[0][1] * (A[1][0] * A[2][2] - A[1][2] * A[2][0]) +
                     A[0][2] * (A[1][0] * A[2][1] - A[1][1] * A[2][0]);
  mt[9 * N + q] = (det > 0.0 && isfinite(det)) ? 1.0 / det : 0.0;
}

__global__ __launch_bounds__(BLK) void k_curv_face_metrics(const Member* __restrict__ mem,
                                                           const double* __restrict__ mt, double* __restrict__ mf) {
  const Member& G = mem[0];
  const long long q = (long long)blockIdx.x * BLK + threadIdx.x;
  if (q >= G.N) return;
  const long long N = G.N;
  const int b[3] = {(int)(q % G.n[0]), (int)((q / G.n[0]) % G.n[1]), (int)(q / ((long long)G.n[0] * G.n[1]))};
  const double cw[6] = {1.0, -8.0, 37.0, 37.0, -8.0, 1.0};
  for (int d = 0; d < 3; ++d) {
    long long st[6];
    for (int m = 0; m < 6; ++m) {
      int p[3] = {b[0], b[1], b[2]};
      p[d] = wrapi(b[d] - 2 + m, G.n[d]);
      st[m] = lin(G, p[0], p[1], p[2]);
    }
    for (int c = 0; c < 3; ++c) {
      double s = 0.0;
      for (int m = 0; m < 6; ++m) s += cw[m] * mt[(3 * d + c) * N + st[m]];
      mf[(3 * d + c) * N + q] = s / 60.0;
    }
  }
}

// theta = (div u)^2 / ((div u)^2 + |curl u|^2 + 1e-300), second-order central
// differences through the chain rule d/dx_b = sum_a J mt[3a + b] d/d xi_a.
__global__ __launch_bounds__(BLK) void k_curv_sensor(const Member* __restrict__ mem, CurvGeom g,
                                                     const double* __restrict__ aux,
                                                     unsigned char* __restrict__ flag, double theta_c,
                                                     double* __restrict__ theta_out, int nq) {
  const Member& G = mem[0];
  const long long q = (long long)blockIdx.x * BLK + threadIdx.x;
  if (q >= G.N) return;
  const long long N = G.N;
  const double* vel = aux + 4 * N;
  const int c[3] = {(int)(q % G.n[0]), (int)((q / G.n[0]) % G.n[1]), (int)(q / ((long long)G.n[0] * G.n[1]))};
  const long long stride[3] = {1, G.n[0], (long long)G.n[0] * G.n[1]};
  const double Jq = g.mt[9 * N + q];
  double gr[3][3];
#pragma unroll
  for (int b = 0; b < 3; ++b)
#pragma unroll
    for (int m = 0; m < 3; ++m) gr[b][m] = 0.0;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    if (!G.act[a]) continue;
    const long long qp = q + (wrapi(c[a] + 1, G.n[a]) - c[a]) * stride[a];
    const long long qm = q + (wrapi(c[a] - 1, G.n[a]) - c[a]) * stride[a];
    double du[3];
#pragma unroll
    for (int m = 0; m < 3; ++m) du[m] = vel[m * N + qp] - vel[m * N + qm];
#pragma unroll
    for (int b = 0; b < 3; ++b) {
      const double mab = Jq * g.mt[(3 * a + b) * N + q];
#pragma unroll
      for (int m = 0; m < 3; ++m) gr[b][m] += mab * du[m] / 2.0;
    }
  }
  const double div = gr[0][0] + gr[1][1] + gr[2][2];
  const double wx = gr[1][2] - gr[2][1], wy = gr[2][0] - gr[0][2], wz = gr[0][1] - gr[1][0];
  const double d2 = div * div;
  const double th = d2 / (d2 + wx * wx + wy * wy + wz * wz + 1e-300);
  flag[q] = th > theta_c ? 1 : 0;
  if (theta_out) theta_out[(nq - 1) * N + q] = th;
}

// Mole fractions X_s = Y_s W / W_s.
template <int NS>
__global__ __launch_bounds__(BLK) void k_curv_molefrac(const MechTables* __restrict__ M,
                                                       const Member* __restrict__ mem, const double* __restrict__ U,
                                                       double* __restrict__ X) {
  const Member& G = mem[0];
  const long long q = (long long)blockIdx.x * BLK + threadIdx.x;
  if (q >= G.N) return;
  const long long N = G.N;
  double r[NS], rho = 0.0;
#pragma unroll
  for (int s = 0; s < NS; ++s) {
    r[s] = U[s * N + q];
    rho += r[s];
  }
  const double irho = 1.0 / rho;
  double iW = 0.0;
#pragma unroll
  for (int s = 0; s < NS; ++s) iW += r[s] * irho * M->iW[s];
  const double W = 1.0 / iW;
#pragma unroll
  for (int s = 0; s < NS; ++s) X[s * N + q] = r[s] * irho * W * M->iW[s];
}

// Index-space central differences (phi(i+1) - phi(i-1)) / 2 of
// phi = (u, v, w, T, X_s) along each axis (zero along an inactive axis).
template <int NS>
__global__ __launch_bounds__(BLK) void k_curv_igrad(const Member* __restrict__ mem, const double* __restrict__ T,
                                                    const double* __restrict__ aux, const double* __restrict__ X,
                                                    double* __restrict__ dphi) {
  constexpr int NP = 4 + NS;
  const Member& G = mem[0];
  const long long q = (long long)blockIdx.x * BLK + threadIdx.x;
  if (q >= G.N) return;
  const long long N = G.N;
  const int c[3] = {(int)(q % G.n[0]), (int)((q / G.n[0]) % G.n[1]), (int)(q / ((long long)G.n[0] * G.n[1]))};
  const long long stride[3] = {1, G.n[0], (long long)G.n[0] * G.n[1]};
  for (int a = 0; a < 3; ++a) {
    double* out = dphi + (long long)a * NP * N;
    if (!G.act[a]) {
      for (int k = 0; k < NP; ++k) out[k * N + q] = 0.0;
      continue;
    }
    const long long qp = q + (wrapi(c[a] + 1, G.n[a]) - c[a]) * stride[a];
    const long long qm = q + (wrapi(c[a] - 1, G.n[a]) - c[a]) * stride[a];
#pragma unroll
    for (int m = 0; m < 3; ++m) out[m * N + q] = (aux[(4 + m) * N + qp] - aux[(4 + m) * N + qm]) / 2.0;
    out[3 * N + q] = (T[qp] - T[qm]) / 2.0;
#pragma unroll
    for (int s = 0; s < NS; ++s) out[(4 + s) * N + q] = (X[s * N + qp] - X[s * N + qm]) / 2.0;
  }
}

// Mapped convective flux through face i+1/2 along d, stored at node i: the
// hybrid switch of the rectilinear sweep (TENO where a stencil node's sensor
// is set or the pressure jump across the face is large), central six-point
// flux or TENO6 / WENO3-Z on the local Lax-Friedrichs split with
// alpha = max |u . n| + c |n| over the stencil, of the physical flux
// projected on the face metric vector n (held fixed on the stencil).
//
// One block per tile of faces: CA faces along d by CB along the companion
// axis o (x, or y when d is x), one plane r of the remaining axis.  The
// tile's nodes and a 2 + 3 node halo along d are staged in LDS in one pass,
// the conserved variables with velocity, p, c and the sensor flags, behind
// a single barrier (staging the variables one at a time through a double
// buffer, one barrier each, took 1.05 against 0.78 ms at 128^3: the block
// waited on each variable's loads in turn).  Each face then keeps u . n, p,
// the switch and alpha in registers and works through the variables from
// LDS.  Every node value is loaded once per block, coalesced along x.
template <int NS, int CA, int CB, bool DX>
__global__ __launch_bounds__(BLK) void k_curv_conv(const Member* __restrict__ mem, CurvGeom g, int d, unsigned flags,
                                                   const double* __restrict__ U, const double* __restrict__ aux,
                                                   const unsigned char* __restrict__ flg, double* __restrict__ ffc,
                                                   double psi_c, double CT) {
  static_assert(CA * CB == BLK, "one face per thread");
  constexpr int NV = NS + 4;
  constexpr int NA = CA + 5;   // staged nodes along d
  constexpr int NB = NA * CB;  // staged nodes
  __shared__ double s_un[3][NB];   // velocity
  __shared__ double s_p[NB], s_c[NB];
  __shared__ unsigned char s_f[NB];
  __shared__ double s_U[NS + 4][NB];
  const Member& G = mem[0];
  const long long N = G.N;
  // axes: d (faces), o (companion), r (plane)
  const int o = DX ? 1 : 0;
  const int r = 3 - d - o;
  const int nto = (G.n[o] + CB - 1) / CB;
  const int nta = (G.n[d] + CA - 1) / CA;
  int b = blockIdx.x;
  const int to = b % nto;
  b /= nto;
  const int ta = b % nta;
  const int pr = b / nta;
  const int a0 = ta * CA, o0 = to * CB;
  const long long stride[3] = {1, G.n[0], (long long)G.n[0] * G.n[1]};
  // staged slot of node (k along d, j along o): x-consecutive threads read
  // consecutive slots (DX: k is along x; otherwise j is)
  auto slot = [](int k, int j) { return DX ? j * NA + k : k * CB + j; };
  auto node = [&](int k, int j) -> long long {
    const int ad = wrapi(a0 - 2 + k, G.n[d]);
    const int ao = wrapi(o0 + j, G.n[o]);
    return (long long)ad * stride[d] + (long long)ao * stride[o] + (long long)pr * stride[r];
  };
  for (int e = threadIdx.x; e < NB; e += BLK) {
    const int k = DX ? e % NA : e / CB, j = DX ? e / NA : e % CB;
    const long long q = node(k, j);
    const int sl = slot(k, j);
#pragma unroll
    for (int v = 0; v < NV; ++v) s_U[v][sl] = U[v * N + q];
    s_un[0][sl] = aux[4 * N + q];
    s_un[1][sl] = aux[5 * N + q];
    s_un[2][sl] = aux[6 * N + q];
    s_p[sl] = aux[q];
    s_c[sl] = aux[N + q];
    s_f[sl] = flg[q];
  }
  // this thread's face
  const int fa = DX ? threadIdx.x % CA : threadIdx.x / CB;
  const int fo = DX ? threadIdx.x / CA : threadIdx.x % CB;
  const bool live = a0 + fa < G.n[d] && o0 + fo < G.n[o];
  const long long qf = (long long)(a0 + fa) * stride[d] + (long long)(o0 + fo) * stride[o] + (long long)pr * stride[r];
  double n0 = 0.0, n1 = 0.0, n2 = 0.0;
  if (live) {
    n0 = g.mf[(3 * d) * N + qf];
    n1 = g.mf[(3 * d + 1) * N + qf];
    n2 = g.mf[(3 * d + 2) * N + qf];
  }
  __syncthreads();
  double un[6], pm[6];
  bool anyflag = false;
  double alpha = -1.0;
  const double nn = sqrt(n0 * n0 + n1 * n1 + n2 * n2);
#pragma unroll
  for (int m = 0; m < 6; ++m) {
    const int sl = slot(fa + m, fo);
    un[m] = s_un[0][sl] * n0 + s_un[1][sl] * n1 + s_un[2][sl] * n2;
    pm[m] = s_p[sl];
    anyflag = anyflag || s_f[sl] != 0;
    alpha = fmax(alpha, fabs(un[m]) + s_c[sl] * nn);
  }
  bool teno;
  if (flags & HTR_FORCE_TENO) teno = true;
  else if (flags & HTR_FORCE_CENTRAL) teno = false;
  else teno = anyflag || (fabs(pm[3] - pm[2]) / fmin(pm[2], pm[3]) > psi_c);
  const bool weno = (flags & HTR_WENO3Z) != 0;
  double* out = ffc + (long long)d * NV * N;
#pragma unroll 1
  for (int v = 0; v < NV; ++v) {
    if (live) {
      double f[6], Uv[6];
#pragma unroll
      for (int m = 0; m < 6; ++m) {
        Uv[m] = s_U[v][slot(fa + m, fo)];
        if (v < NS) f[m] = Uv[m] * un[m];
        else if (v < NS + 3) f[m] = Uv[m] * un[m] + pm[m] * (v == NS ? n0 : (v == NS + 1 ? n1 : n2));
        else f[m] = (Uv[m] + pm[m]) * un[m];
      }
      double res;
      if (!teno) {
        const double cc[6] = {1.0, -8.0, 37.0, 37.0, -8.0, 1.0};
        double sacc = 0.0;
#pragma unroll
        for (int m = 0; m < 6; ++m) sacc += cc[m] * f[m];
        res = sacc / 60.0;
      } else {
        double hp[6], hmr[6];
#pragma unroll
        for (int m = 0; m < 6; ++m) {
          hp[m] = fma(alpha, Uv[m], f[m]);
          hmr[5 - m] = fma(-alpha, Uv[m], f[m]);
        }
        res = weno ? weno3z_h(hp) + weno3z_h(hmr) : teno6_h(hp, CT) + teno6_h(hmr, CT);
      }
      out[v * N + qf] = res;
    }
  }
}

// Mapped diffusive flux through face i+1/2 along d = blockIdx.y, stored at
// node i: index-space derivatives at the face (normal from the two nodes,
// tangential the mean of the two nodal central differences), physical
// gradients by the chain rule with the face mean of d xi_e / d x, the flux
// vector projected on the face metric vector n; arithmetic-mean face
// coefficients.
template <int NS>
__global__ __launch_bounds__(BLK) void k_curv_diff(const MechTables* __restrict__ M, const Member* __restrict__ mem,
                                                   CurvGeom g, const double* __restrict__ U,
                                                   const double* __restrict__ T, const double* __restrict__ aux,
                                                   const double* __restrict__ X, const double* __restrict__ dphi,
                                                   double* __restrict__ ffd) {
  constexpr int NV = NS + 4, NP = 4 + NS;
  const Member& G = mem[0];
  const int d = blockIdx.y;
  if (!G.act[d]) return;
  const long long q = (long long)blockIdx.x * BLK + threadIdx.x;
  if (q >= G.N) return;
  const long long N = G.N;
  const int c0[3] = {(int)(q % G.n[0]), (int)((q / G.n[0]) % G.n[1]), (int)(q / ((long long)G.n[0] * G.n[1]))};
  int pb[3] = {c0[0], c0[1], c0[2]};
  pb[d] = wrapi(c0[d] + 1, G.n[d]);
  const long long qa = q, qb = lin(G, pb[0], pb[1], pb[2]);
  const double n0 = g.mf[(3 * d) * N + q], n1 = g.mf[(3 * d + 1) * N + q], n2 = g.mf[(3 * d + 2) * N + q];
  double* out = ffd + (long long)d * NV * N;
  // ---- diffusive flux
  const double nv3[3] = {n0, n1, n2};
  double Gf[3][3];   // d xi_e / d x_b at the face
  const double Ja = g.mt[9 * N + qa], Jb = g.mt[9 * N + qb];
#pragma unroll
  for (int e = 0; e < 3; ++e)
#pragma unroll
    for (int b = 0; b < 3; ++b)
      Gf[e][b] = 0.5 * (Ja * g.mt[(3 * e + b) * N + qa] + Jb * g.mt[(3 * e + b) * N + qb]);
  const double* dpa = dphi + qa;
  const double* dpb = dphi + qb;
  // derivative along index axis e at the face of phi row k (values va, vb at the two nodes)
  auto dxi = [&](int k, int e, double va, double vb) -> double {
    if (e == d) return vb - va;
    if (!G.act[e]) return 0.0;
    return 0.5 * (dpa[((long long)e * NP + k) * N] + dpb[((long long)e * NP + k) * N]);
  };
  double gu[3][3];   // gu[b][m] = d u_m / d x_b
#pragma unroll
  for (int m = 0; m < 3; ++m) {
    const double va = aux[(4 + m) * N + qa], vb = aux[(4 + m) * N + qb];
    double de[3];
#pragma unroll
    for (int e = 0; e < 3; ++e) de[e] = dxi(m, e, va, vb);
#pragma unroll
    for (int b = 0; b < 3; ++b) gu[b][m] = Gf[0][b] * de[0] + Gf[1][b] * de[1] + Gf[2][b] * de[2];
  }
  double rhoA = 0.0, rhoB = 0.0;
#pragma unroll
  for (int s = 0; s < NS; ++s) {
    rhoA += U[s * N + qa];
    rhoB += U[s * N + qb];
  }
  const double irA = 1.0 / rhoA, irB = 1.0 / rhoB;
  double iWA = 0.0, iWB = 0.0;
#pragma unroll
  for (int s = 0; s < NS; ++s) {
    iWA += U[s * N + qa] * irA * M->iW[s];
    iWB += U[s * N + qb] * irB * M->iW[s];
  }
  const double TA = T[qa], TB = T[qb];
  const double mu = 0.5 * (aux[2 * N + qa] + aux[2 * N + qb]);
  const double lam = 0.5 * (aux[3 * N + qa] + aux[3 * N + qb]);
  const double rho = 0.5 * (rhoA + rhoB);
  const double W = 0.5 * (1.0 / iWA + 1.0 / iWB);
  const double divu = gu[0][0] + gu[1][1] + gu[2][2];
  double tn[3];
#pragma unroll
  for (int m = 0; m < 3; ++m) {
    tn[m] = 0.0;
#pragma unroll
    for (int b = 0; b < 3; ++b) {
      double tau = mu * (gu[b][m] + gu[m][b]);
      if (b == m) tau -= (2.0 / 3.0) * mu * divu;
      tn[m] += nv3[b] * tau;
    }
  }
  // species: two passes (the correction flux first, then each species),
  // recomputing the face normal derivative rather than holding per-species
  // arrays, which keeps the kernel's register footprint small
  auto rhoDW_dXn = [&](int s) -> double {
    const double va = X[s * N + qa], vb = X[s * N + qb];
    double de[3];
#pragma unroll
    for (int e = 0; e < 3; ++e) de[e] = dxi(4 + s, e, va, vb);
    double dXn = 0.0;
#pragma unroll
    for (int b = 0; b < 3; ++b) dXn += (Gf[0][b] * de[0] + Gf[1][b] * de[1] + Gf[2][b] * de[2]) * nv3[b];
    const double Df = 0.5 * (aux[(7 + s) * N + qa] + aux[(7 + s) * N + qb]);
    return rho * Df * (M->W[s] / W) * dXn;
  };
  double corr = 0.0;
#pragma unroll 1
  for (int s = 0; s < NS; ++s) corr += rhoDW_dXn(s);
  double gT[3];
  {
    double de[3];
#pragma unroll
    for (int e = 0; e < 3; ++e) de[e] = dxi(3, e, TA, TB);
#pragma unroll
    for (int b = 0; b < 3; ++b) gT[b] = Gf[0][b] * de[0] + Gf[1][b] * de[1] + Gf[2][b] * de[2];
  }
  double qn = -lam * (gT[0] * n0 + gT[1] * n1 + gT[2] * n2);
#pragma unroll 1
  for (int s = 0; s < NS; ++s) {
    const double Yf = 0.5 * (U[s * N + qa] * irA + U[s * N + qb] * irB);
    const double hf = 0.5 * (M->RW[s] * TA * hRTs(M, s, TA) + M->RW[s] * TB * hRTs(M, s, TB));
    const double Jn = -rhoDW_dXn(s) + Yf * corr;
    qn += Jn * hf;
    out[s * N + q] = -Jn;
  }
  double work = 0.0;
#pragma unroll
  for (int m = 0; m < 3; ++m) work += tn[m] * 0.5 * (aux[(4 + m) * N + qa] + aux[(4 + m) * N + qb]);
#pragma unroll
  for (int m = 0; m < 3; ++m) out[(NS + m) * N + q] = tn[m];
  out[(NS + 3) * N + q] = work - qn;
}

// dU/dt = src + sum_d J ((Fd_d(i) - Fd_d(i - e_d)) - (Fc_d(i) - Fc_d(i - e_d)));
// out = dU/dt (rhs_only) or the stage combination ca U^n + cb (U + dt dU/dt).
template <int NS>
__global__ __launch_bounds__(BLK) void k_curv_update(const Member* __restrict__ mem, CurvGeom g, CallArgs A,
                                                     const double* __restrict__ U, const double* __restrict__ Un,
                                                     const double* __restrict__ src, const double* __restrict__ ffc,
                                                     const double* __restrict__ ffd, double* __restrict__ out,
                                                     double ca, double cb, int rhs_only) {
  constexpr int NV = NS + 4;
  const Member& G = mem[0];
  const long long q = (long long)blockIdx.x * BLK + threadIdx.x;
  if (q >= G.N) return;
  const long long N = G.N;
  const int c[3] = {(int)(q % G.n[0]), (int)((q / G.n[0]) % G.n[1]), (int)(q / ((long long)G.n[0] * G.n[1]))};
  const long long stride[3] = {1, G.n[0], (long long)G.n[0] * G.n[1]};
  const double Jq = g.mt[9 * N + q];
  double L[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) L[v] = v < NS ? src[v * N + q] : (v == NS + 3 ? src[NS * N + q] : 0.0);
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    if (!G.act[d]) continue;
    const long long qm = q + (wrapi(c[d] - 1, G.n[d]) - c[d]) * stride[d];
    const double* fc = ffc + (long long)d * NV * N;
    const double* fd = ffd + (long long)d * NV * N;
    if (A.flags & HTR_VISC_OFF) {
#pragma unroll
      for (int v = 0; v < NV; ++v) L[v] += Jq * (0.0 - (fc[v * N + q] - fc[v * N + qm]));
    } else {
#pragma unroll
      for (int v = 0; v < NV; ++v)
        L[v] += Jq * ((fd[v * N + q] - fd[v * N + qm]) - (fc[v * N + q] - fc[v * N + qm]));
    }
  }
  if (rhs_only) {
#pragma unroll
    for (int v = 0; v < NV; ++v) out[v * N + q] = L[v];
    return;
  }
  const double dt = A.dt_dev[0];
  double uv[NV], unv[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    uv[v] = U[v * N + q];
    unv[v] = ca != 0.0 ? Un[v * N + q] : 0.0;
  }
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    const double base = uv[v] + dt * L[v];
    out[v * N + q] = ca != 0.0 ? ca * unv[v] + cb * base : cb * base;
  }
}

// ---------------------------------------------------------------- launchers
static inline int blocks_of(long long N) { return (int)((N + BLK - 1) / BLK); }

hipError_t launch_curv_metrics(const Member* mem, const Member& host, const CurvGeom& g, double* mt, double* mf,
                               hipStream_t s) {
  const int nb = blocks_of(host.N);
  hipLaunchKernelGGL(k_curv_metrics, dim3(nb), dim3(BLK), 0, s, mem, g, mt);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_curv_face_metrics, dim3(nb), dim3(BLK), 0, s, mem, mt, mf);
  return hipGetLastError();
}

hipError_t launch_curv_sensor(const Member* mem, int nblocks, const CurvGeom& g, const double* aux, int ns,
                              unsigned char* flag, double theta_c, double* theta_out, hipStream_t s) {
  hipLaunchKernelGGL(k_curv_sensor, dim3(nblocks), dim3(BLK), 0, s, mem, g, aux, flag, theta_c, theta_out,
                     5 + 2 * ns + 3);
  return hipGetLastError();
}

template <int NS>
static hipError_t igrad_t(const MechTables* M, const Member* mem, int nblocks, const double* U, const double* T,
                          const double* aux, double* X, double* dphi, hipStream_t s) {
  hipLaunchKernelGGL(k_curv_molefrac<NS>, dim3(nblocks), dim3(BLK), 0, s, M, mem, U, X);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_curv_igrad<NS>, dim3(nblocks), dim3(BLK), 0, s, mem, T, aux, X, dphi);
  return hipGetLastError();
}

hipError_t launch_curv_igrad(int ns, const MechTables* M, const Member* mem, int nblocks, const double* U,
                             const double* T, const double* aux, double* X, double* dphi, hipStream_t s) {
#define C_(NS) igrad_t<NS>(M, mem, nblocks, U, T, aux, X, dphi, s)
  HTR_NS_SWITCH(ns, C_)
#undef C_
}

// Tiles of the convective face kernel: 64 x 4 faces in (x, y) when d is x,
// 16 along d by 16 along x otherwise.
template <int NS>
static hipError_t conv_t(const Member& host, const Member* mem, const CurvGeom& g, unsigned flags, const double* U,
                         const double* aux, const unsigned char* flag, double* ffc, double psi_c, double CT,
                         hipStream_t s) {
  for (int d = 0; d < 3; ++d) {
    if (!host.act[d]) continue;
    if (d == 0) {
      const int o = 1, r = 2;
      const int nb = ((host.n[0] + 63) / 64) * ((host.n[o] + 3) / 4) * host.n[r];
      hipLaunchKernelGGL((k_curv_conv<NS, 64, 4, true>), dim3(nb), dim3(BLK), 0, s, mem, g, d, flags, U, aux, flag,
                         ffc, psi_c, CT);
    } else {
      const int o = 0, r = 3 - d;
      const int nb = ((host.n[d] + 15) / 16) * ((host.n[o] + 15) / 16) * host.n[r];
      hipLaunchKernelGGL((k_curv_conv<NS, 16, 16, false>), dim3(nb), dim3(BLK), 0, s, mem, g, d, flags, U, aux,
                         flag, ffc, psi_c, CT);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_curv_conv(int ns, const Member& host, const Member* mem, const CurvGeom& g, const CallArgs& a,
                            const double* U, const double* aux, const unsigned char* flag, double* ffc, double psi_c,
                            double teno_CT, hipStream_t s) {
#define C_(NS) conv_t<NS>(host, mem, g, a.flags, U, aux, flag, ffc, psi_c, teno_CT, s)
  HTR_NS_SWITCH(ns, C_)
#undef C_
}

template <int NS>
static hipError_t diff_t(const MechTables* M, const Member* mem, int nblocks, const CurvGeom& g, const double* U,
                         const double* T, const double* aux, const double* X, const double* dphi, double* ffd,
                         hipStream_t s) {
  hipLaunchKernelGGL(k_curv_diff<NS>, dim3(nblocks, 3), dim3(BLK), 0, s, M, mem, g, U, T, aux, X, dphi, ffd);
  return hipGetLastError();
}

hipError_t launch_curv_diff(int ns, const MechTables* M, const Member* mem, int nblocks, const CurvGeom& g,
                            const double* U, const double* T, const double* aux, const double* X,
                            const double* dphi, double* ffd, hipStream_t s) {
#define C_(NS) diff_t<NS>(M, mem, nblocks, g, U, T, aux, X, dphi, ffd, s)
  HTR_NS_SWITCH(ns, C_)
#undef C_
}

template <int NS>
static hipError_t update_t(const Member* mem, int nblocks, const CurvGeom& g, const CallArgs& a, const double* U,
                           const double* Un, const double* src, const double* ffc, const double* ffd, double* out,
                           double ca, double cb, int rhs_only, hipStream_t s) {
  hipLaunchKernelGGL(k_curv_update<NS>, dim3(nblocks), dim3(BLK), 0, s, mem, g, a, U, Un, src, ffc, ffd, out, ca, cb,
                     rhs_only);
  return hipGetLastError();
}

hipError_t launch_curv_update(int ns, const Member* mem, int nblocks, const CurvGeom& g,
                              const CallArgs& a, const double* U, const double* Un, const double* src,
                              const double* ffc, const double* ffd, double* out, double ca, double cb, int rhs_only,
                              hipStream_t s) {
#define C_(NS) update_t<NS>(mem, nblocks, g, a, U, Un, src, ffc, ffd, out, ca, cb, rhs_only, s)
  HTR_NS_SWITCH(ns, C_)
#undef C_
}

}  // namespace htr
