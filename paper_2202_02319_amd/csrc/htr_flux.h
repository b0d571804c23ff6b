// Device functions shared by the forward flux sweep and its adjoint, so that
// both take the same discrete decisions from the same arithmetic.
#pragma once

#include <math.h>

#include "htr_dev.h"

namespace htr {

// TENO6 cut-off decisions from the four smoothness indicators b_k and the
// global one tau: candidate k is kept when its scale-separated weight
// gamma_k = (1 + tau / (b_k + 1e-40))^6, normalised by the sum over the
// four candidates, reaches C_T.  This is the reference arithmetic (every
// quotient correctly rounded, gamma scaled by the largest r before the
// sixth power); the result is four bits, bit k set when candidate k is kept.
__device__ __forceinline__ unsigned teno6_pattern_exact(double b0, double b1, double b2, double b3, double tau,
                                                        double CT) {
  const double r0 = 1.0 + tau / (b0 + 1e-40), r1 = 1.0 + tau / (b1 + 1e-40);
  const double r2 = 1.0 + tau / (b2 + 1e-40), r3 = 1.0 + tau / (b3 + 1e-40);
  const double irm = 1.0 / fmax(fmax(r0, r1), fmax(r2, r3));
  double g0 = r0 * irm, g1 = r1 * irm, g2 = r2 * irm, g3 = r3 * irm;
  g0 = g0 * g0 * g0; g0 *= g0;
  g1 = g1 * g1 * g1; g1 *= g1;
  g2 = g2 * g2 * g2; g2 *= g2;
  g3 = g3 * g3 * g3; g3 *= g3;
  const double igs = 1.0 / (g0 + g1 + g2 + g3);
  return (g0 * igs >= CT ? 1u : 0u) | (g1 * igs >= CT ? 2u : 0u) | (g2 * igs >= CT ? 4u : 0u) |
         (g3 * igs >= CT ? 8u : 0u);
}

// The same decisions without a correctly rounded quotient.  The test
// gamma_k / sum(gamma) >= C_T is the same as x_k >= C_T sum(x) for x_k =
// (s r_k)^6 with any scale s > 0, here s = 1, so:
//  - the four 1 / (b_k + 1e-40) come from one hardware reciprocal of their
//    product (refined by two Newton steps) and three products each
//    (Montgomery's simultaneous inversion);
//  - each x_k = r_k^6 (r_k >= 1) is then within about 1e-14 (relative) of
//    its exact value, and the reference arithmetic is within about the same
//    distance, so where every x_k lies further than 1e-12 C_T sum(x) from
//    C_T sum(x) both take the same decision.  Otherwise (and for a product of
//    the b_k outside [1e-290, 1e290], a sum of the x_k beyond 1e300, or any
//    non-finite value) the reference arithmetic decides.
__device__ __forceinline__ unsigned teno6_pattern(double b0, double b1, double b2, double b3, double tau,
                                                  double CT) {
  const double D0 = b0 + 1e-40, D1 = b1 + 1e-40, D2 = b2 + 1e-40, D3 = b3 + 1e-40;
  const double P01 = D0 * D1, P23 = D2 * D3, P = P01 * P23;
  double inv = __builtin_amdgcn_rcp(P);
  inv = fma(fma(-P, inv, 1.0), inv, inv);
  inv = fma(fma(-P, inv, 1.0), inv, inv);
  const double i01 = inv * P23, i23 = inv * P01;
  double x0 = fma(tau, i01 * D1, 1.0), x1 = fma(tau, i01 * D0, 1.0);
  double x2 = fma(tau, i23 * D3, 1.0), x3 = fma(tau, i23 * D2, 1.0);
  x0 = x0 * x0 * x0; x0 *= x0;
  x1 = x1 * x1 * x1; x1 *= x1;
  x2 = x2 * x2 * x2; x2 *= x2;
  x3 = x3 * x3 * x3; x3 *= x3;
  const double sx = x0 + x1 + x2 + x3, th = CT * sx, m = 1e-12 * th;
  const bool sure = P > 1e-290 && P < 1e290 && sx < 1e300 && fabs(x0 - th) > m && fabs(x1 - th) > m &&
                    fabs(x2 - th) > m && fabs(x3 - th) > m;
  if (!sure) return teno6_pattern_exact(b0, b1, b2, b3, tau, CT);
  return (x0 >= th ? 1u : 0u) | (x1 >= th ? 2u : 0u) | (x2 >= th ? 4u : 0u) | (x3 >= th ? 8u : 0u);
}

// TENO6 at x_{i+1/2} for one side of the Lax-Friedrichs flux splitting,
// from h[0..5] = 2 f_{i-2..i+3}: the splitting's factor 1/2 is folded into
// the constants, which are those of the formulas for f divided by powers of
// two, so the same operations on h round exactly as they do on f (away from
// underflow).  The smoothness indicators stay in the expanded form of the
// definitions' sums: an evaluation that rounds differently (from the
// stencil's differences, say) takes another cut-off wherever rounding
// decides one.  The candidate values in q[4] (those of f); returns the
// cut-off pattern (bit k: candidate k kept).
__device__ __forceinline__ unsigned teno6_decide(const double h[6], double CT, double q[4]) {
  q[0] = (-h[1] + 5.0 * h[2] + 2.0 * h[3]) * (1.0 / 12.0);
  q[1] = (2.0 * h[2] + 5.0 * h[3] - h[4]) * (1.0 / 12.0);
  q[2] = (2.0 * h[0] - 7.0 * h[1] + 11.0 * h[2]) * (1.0 / 12.0);
  q[3] = (3.0 * h[2] + 13.0 * h[3] - 5.0 * h[4] + h[5]) * (1.0 / 24.0);
  const double s0a = h[1] - 2.0 * h[2] + h[3], s0b = h[1] - h[3];
  const double s1a = h[2] - 2.0 * h[3] + h[4], s1b = 3.0 * h[2] - 4.0 * h[3] + h[4];
  const double s2a = h[0] - 2.0 * h[1] + h[2], s2b = h[0] - 4.0 * h[1] + 3.0 * h[2];
  const double s3a = -11.0 * h[2] + 18.0 * h[3] - 9.0 * h[4] + 2.0 * h[5];
  const double s3b = 2.0 * h[2] - 5.0 * h[3] + 4.0 * h[4] - h[5];
  const double s3c = -h[2] + 3.0 * h[3] - 3.0 * h[4] + h[5];
  const double b0 = (13.0 / 48.0) * s0a * s0a + (1.0 / 16.0) * s0b * s0b;
  const double b1 = (13.0 / 48.0) * s1a * s1a + (1.0 / 16.0) * s1b * s1b;
  const double b2 = (13.0 / 48.0) * s2a * s2a + (1.0 / 16.0) * s2b * s2b;
  const double b3 = (1.0 / 144.0) * s3a * s3a + (13.0 / 48.0) * s3b * s3b + (781.0 / 2880.0) * s3c * s3c;
  // six-point polynomial coefficients (origin at the centre of cell i)
  const double a1 = (341.0 * h[0] - 2785.0 * h[1] - 2590.0 * h[2] + 6670.0 * h[3] - 1895.0 * h[4] + 259.0 * h[5]) *
                    (1.0 / 11520.0);
  const double a2 = -(h[0] - 12.0 * h[1] + 22.0 * h[2] - 12.0 * h[3] + h[4]) * (1.0 / 32.0);
  const double a3 = -(5.0 * h[0] + 11.0 * h[1] - 70.0 * h[2] + 94.0 * h[3] - 47.0 * h[4] + 7.0 * h[5]) *
                    (1.0 / 288.0);
  const double a4 = (h[0] - 4.0 * h[1] + 6.0 * h[2] - 4.0 * h[3] + h[4]) * (1.0 / 48.0);
  const double a5 = -(h[0] - 5.0 * h[1] + 10.0 * h[2] - 10.0 * h[3] + 5.0 * h[4] - h[5]) * (1.0 / 240.0);
  const double b6 = a1 * (a1 + 0.5 * a3 + 0.125 * a5) + a2 * ((13.0 / 3.0) * a2 + (21.0 / 5.0) * a4) +
                    a3 * ((3129.0 / 80.0) * a3 + (14127.0 / 224.0) * a5) + (87617.0 / 140.0) * a4 * a4 +
                    (252337135.0 / 16128.0) * a5 * a5;
  const double tau = fabs(b6 - (b1 + b2 + 4.0 * b0) * (1.0 / 6.0));
  return teno6_pattern(b0, b1, b2, b3, tau, CT);
}

// Normalised weights of the kept candidates of a cut-off pattern: d_k
// delta_k / sum d delta with d = (9/20, 3/10, 1/20, 1/5).
__device__ __forceinline__ void teno6_weights(unsigned pat, double w[4]) {
  w[0] = (pat & 1u) ? 9.0 / 20.0 : 0.0;
  w[1] = (pat & 2u) ? 3.0 / 10.0 : 0.0;
  w[2] = (pat & 4u) ? 1.0 / 20.0 : 0.0;
  w[3] = (pat & 8u) ? 1.0 / 5.0 : 0.0;
  const double iw = 1.0 / (w[0] + w[1] + w[2] + w[3]);
  w[0] *= iw; w[1] *= iw; w[2] *= iw; w[3] *= iw;
}

// TENO6 reconstruction at x_{i+1/2} of one side of the split, from
// h = 2 f_{i-2..i+3}.
__device__ __forceinline__ double teno6_h(const double h[6], double CT) {
  double q[4], w[4];
  teno6_weights(teno6_decide(h, CT, q), w);
  return w[0] * q[0] + w[1] * q[1] + w[2] * q[2] + w[3] * q[3];
}

// Third-order WENO-Z reconstruction at x_{i+1/2} (Don & Borges) from f_{i-1},
// f_i, f_{i+1} = f[1..3] of the six-point face stencil: candidates on
// {i-1, i} and {i, i+1} with optimal weights 1/3 and 2/3, smoothness the
// squared first differences, global indicator |beta_0 - beta_1|.
__device__ __forceinline__ double weno3z(const double f[6]) {
  const double q0 = (-f[1] + 3.0 * f[2]) / 2.0;
  const double q1 = (f[2] + f[3]) / 2.0;
  const double b0 = (f[2] - f[1]) * (f[2] - f[1]);
  const double b1 = (f[3] - f[2]) * (f[3] - f[2]);
  const double tau = fabs(b0 - b1);
  const double a0 = (1.0 / 3.0) * (1.0 + tau / (b0 + 1e-40));
  const double a1 = (2.0 / 3.0) * (1.0 + tau / (b1 + 1e-40));
  return (a0 * q0 + a1 * q1) / (a0 + a1);
}

// WENO3-Z of one side of the split from h = 2 f (the stencil values halved
// first, as the scheme takes them).
__device__ __forceinline__ double weno3z_h(const double h[6]) {
  double f[6];
#pragma unroll
  for (int m = 0; m < 6; ++m) f[m] = 0.5 * h[m];
  return weno3z(f);
}

// Linear coefficients of the frozen reconstruction from its cut-off bits
// (the normalised weights of that pattern; coefficients of f, not of h).
__device__ __forceinline__ void teno6_coeffs_bits(unsigned b, double c[6]) {
  double w0 = (b & 1u) ? 9.0 / 20.0 : 0.0, w1 = (b & 2u) ? 3.0 / 10.0 : 0.0;
  double w2 = (b & 4u) ? 1.0 / 20.0 : 0.0, w3 = (b & 8u) ? 1.0 / 5.0 : 0.0;
  const double iw = 1.0 / (w0 + w1 + w2 + w3);
  w0 *= iw; w1 *= iw; w2 *= iw; w3 *= iw;
  c[0] = w2 * (2.0 / 6.0);
  c[1] = w0 * (-1.0 / 6.0) + w2 * (-7.0 / 6.0);
  c[2] = w0 * (5.0 / 6.0) + w1 * (2.0 / 6.0) + w2 * (11.0 / 6.0) + w3 * (3.0 / 12.0);
  c[3] = w0 * (2.0 / 6.0) + w1 * (5.0 / 6.0) + w3 * (13.0 / 12.0);
  c[4] = w1 * (-1.0 / 6.0) + w3 * (-5.0 / 12.0);
  c[5] = w3 * (1.0 / 12.0);
}

// Node convective flux of variable v along d (u_d normal velocity, p pressure).
template <int NS>
__device__ __forceinline__ double node_flux(int v, int d, double U, double ud, double p) {
  if (v == NS + 3) return (U + p) * ud;
  if (v == NS + d) return U * ud + p;
  return U * ud;
}

__device__ __forceinline__ double hRTi(const MechTables* __restrict__ M, int s, double T, double iT) {
  const double* a = M->hc[s];
  return a[0] + T * (a[1] + T * (a[2] + T * (a[3] + T * a[4]))) + a[5] * iT;
}

__device__ __forceinline__ double hRTs(const MechTables* __restrict__ M, int s, double T) {
  const double* a = M->hc[s];
  return a[0] + T * (a[1] + T * (a[2] + T * (a[3] + T * a[4]))) + a[5] / T;
}

}  // namespace htr
