// Reference (oracle) implementation of the reacting-flow right-hand side.
//
// TEST INFRASTRUCTURE ONLY.  This file is the slow, plain, FP64 CPU statement
// of what the GPU library computes.  Only the test suite, the smoke check and
// the CPU-baseline leg of the benchmark may load it; the product path never
// does.  It shares no code, header, table or constant generator with the HIP
// library: every formula below is written out here on its own.
//
// Paper: Maeda et al., "An integrated heterogeneous computing framework for
// ensemble simulations of laser-induced ignition" (arXiv 2202.02319).
//   governing equations            Methods › Solver, eqs. (1)-(3)
//   ideal-gas closure              eq. (4)
//   Wilke viscosity, NASA c_p      Methods › Solver, text after eq. (4)
//   heat flux                      eq. (5)
//   diffusion velocity             eq. (6), Bird mixture-averaged D_s with
//                                  Hirschfelder binary D_ij
//   finite-rate Arrhenius chem.    Methods › Solver (chemistry)
//   conservative FD, TENO6, 2nd-order central diffusion, SSP-RK3
//                                  Methods › Numerical method
//   laser source q_L               Methods › Diffusion flame › Physical model and numerical setup, eq. (laser-qs)
//
// Structure: every step is its own loop, in the order the method defines it:
//   1. per cell: primitives (Newton for T), transport, chemistry, laser;
//   2. per node: the Ducros-type sensor;
//   3. per direction and per face: convective flux (central or TENO6 on a
//      local Lax-Friedrichs split) and diffusive flux;
//   4. per cell: flux differences plus sources.
// No blocking, no fusion.  Everything is templated on the scalar type so the
// same code, run on Dual numbers, gives the forward-mode tangent with all
// discrete switches (TENO cut-off, sensor, argmax of the LF speed, Newton
// iteration count) taken on the real part.
//
// Parity status of each part is listed in the test suite; the whole RHS has
// no printed worked example in the paper, so its absolute values are pinned
// only through closed forms, invariants and textbook special cases.

#include <cmath>
#include <cstdint>
#include <cstring>
#include <vector>
#include <algorithm>

namespace orc {

// ---------------------------------------------------------------- constants
// Exact SI values (2019 SI): k_B, N_A; R_u = N_A k_B.
static const double kB = 1.380649e-23;
static const double NA = 6.02214076e23;
static const double Ru = 8.31446261815324;
static const double P0 = 101325.0;   // reference pressure of the standard state
static const double PI = 3.14159265358979323846;

enum { OK = 0, EINVAL = 1, ENONFINITE = 4, ENEWTON = 5, ETRANGE = 6 };
enum { CHEM_OFF = 1u, VISC_OFF = 2u, FORCE_CENTRAL = 4u, FORCE_TENO = 8u, WENO3Z = 16u };
// boundary types of a bounded axis side
enum { BC_PERIODIC = 0, BC_WALL = 1, BC_INFLOW = 2, BC_OUTFLOW = 3 };

// ------------------------------------------------------------- dual numbers
struct Dual {
  double v, d;
  Dual() : v(0), d(0) {}
  Dual(double a) : v(a), d(0) {}
  Dual(double a, double b) : v(a), d(b) {}
};
static inline Dual operator+(Dual a, Dual b) { return Dual(a.v + b.v, a.d + b.d); }
static inline Dual operator-(Dual a, Dual b) { return Dual(a.v - b.v, a.d - b.d); }
static inline Dual operator-(Dual a) { return Dual(-a.v, -a.d); }
static inline Dual operator*(Dual a, Dual b) { return Dual(a.v * b.v, a.d * b.v + a.v * b.d); }
static inline Dual operator/(Dual a, Dual b) {
  double q = a.v / b.v;
  return Dual(q, (a.d - q * b.d) / b.v);
}
static inline Dual& operator+=(Dual& a, Dual b) { a = a + b; return a; }
static inline Dual& operator-=(Dual& a, Dual b) { a = a - b; return a; }
static inline Dual& operator*=(Dual& a, Dual b) { a = a * b; return a; }
static inline Dual exp(Dual a) { double e = std::exp(a.v); return Dual(e, e * a.d); }
static inline Dual log(Dual a) { return Dual(std::log(a.v), a.d / a.v); }
static inline Dual sqrt(Dual a) { double s = std::sqrt(a.v); return Dual(s, a.d / (2.0 * s)); }
static inline Dual pow(Dual a, double b) {
  double p = std::pow(a.v, b);
  return Dual(p, b * std::pow(a.v, b - 1.0) * a.d);
}
static inline Dual fabs(Dual a) { return a.v < 0 ? -a : a; }
static inline double val(double a) { return a; }
static inline double val(const Dual& a) { return a.v; }
using std::exp; using std::log; using std::sqrt; using std::pow; using std::fabs;

// ------------------------------------------------------------------- tables
struct Case {
  int ns, nr;
  std::vector<double> W, a7, sig, epsk, lnA, beta, Ea;   // a7: [ns][7]
  std::vector<int> nuf, nur;                             // [nr][ns]
  double Tmin, Tmax;
  int n[3];
  std::vector<double> xnode[3], xin[3], xif[3];          // coordinate, node & face metric
  double L[3];
  double theta_c, psi_c, CT, cfl;
  unsigned flags;
  // general curvilinear grid (Methods › Numerical method, mapped equations): node coordinates,
  // the lattice periods, and the metric terms derived from them
  bool curv = false;
  std::vector<double> X[3];          // X[c][q]: coordinate c of node q
  double Pv[3][3];                   // Pv[a]: displacement of the lattice when index a advances by n[a]
  double Pinv[3][3];                 // inverse of the matrix with columns Pv[a]
  std::vector<double> mt[9];         // node metric terms (d xi_d / d x_c) / J at mt[3d + c]
  std::vector<double> mf[9];         // the same at face i+1/2 along d
  std::vector<double> Jac;           // J = det(d xi / d x) at nodes (1 / index-space cell volume)
  // Non-periodic boundaries (Methods › Diffusion flame › Physical model and
  // numerical setup; Methods › Model rocket combustor › Numerical setup):
  // per axis and side (0: low, 1: high) a boundary type; an axis is either
  // periodic on both sides or bounded on both.  On a bounded axis the first
  // and last nodes lie on the boundaries.
  int bc[3][2] = {{0, 0}, {0, 0}, {0, 0}};
  double pinf[3][2] = {{0, 0}, {0, 0}, {0, 0}};    // outflow: far-field pressure
  double relax[3][2] = {{0, 0}, {0, 0}, {0, 0}};   // outflow: relaxation coefficient sigma
  bool bounded(int a) const { return bc[a][0] != 0; }
  long long N() const { return (long long)n[0] * n[1] * n[2]; }
  long long idx(int i, int j, int k) const { return ((long long)k * n[1] + j) * n[0] + i; }
};

template <class S> struct Params {   // differentiable parameters
  std::vector<S> lnA;                // per reaction
  S E;                               // deposited energy
  S xc[3];                           // kernel centre
  double sr, t0, st;                 // kernel radius, delay, duration
  bool on;
};

static inline int wrap(int i, int n) { int r = i % n; return r < 0 ? r + n : r; }

// ------------------------------------------------------------ NASA-7 thermo
// c_p/R, h/(RT), s/R of one species from the 7-coefficient polynomial
// (McBride et al.).  The paper names the 9-coefficient variant; its tables
// are not available, so the seeded 7-coefficient form is used.
template <class S> static inline S cp_R(const double* a, S T) {
  return a[0] + T * (a[1] + T * (a[2] + T * (a[3] + T * a[4])));
}
template <class S> static inline S h_RT(const double* a, S T) {
  return a[0] + T * (a[1] / 2.0 + T * (a[2] / 3.0 + T * (a[3] / 4.0 + T * (a[4] / 5.0)))) + a[5] / T;
}
template <class S> static inline S s_R(const double* a, S T) {
  return a[0] * log(T) + T * (a[1] + T * (a[2] / 2.0 + T * (a[3] / 3.0 + T * (a[4] / 4.0)))) + a[6];
}

// ------------------------------------------------------ per-cell quantities
template <class S> struct Cell {
  S rho, u[3], T, p, c, W, cp, mu, lam;
  std::vector<S> Y, X, h, D, wdot;     // h: J/kg; D: mixture-averaged diffusivity
  S hrr, qL;
};

// Collision-integral fits of Neufeld, Janzen & Aziz (1972).
template <class S> static inline S omega22(S Ts) {
  return 1.16145 * pow(Ts, -0.14874) + 0.52487 * exp(-0.77320 * Ts) + 2.16178 * exp(-2.43787 * Ts);
}
template <class S> static inline S omega11(S Ts) {
  return 1.06036 * pow(Ts, -0.15610) + 0.19300 * exp(-0.47635 * Ts) + 1.03587 * exp(-1.52996 * Ts) +
         1.76474 * exp(-3.89411 * Ts);
}

// Species viscosity, Chapman-Enskog.
template <class S> static S mu_species(const Case& C, int s, S T) {
  double m = C.W[s] / NA;
  double sg = C.sig[s];
  return (5.0 / 16.0) * sqrt(PI * m * kB * T) / (PI * sg * sg * omega22(T / C.epsk[s]));
}
// Binary diffusion coefficient (Hirschfelder, Curtiss & Bird).
template <class S> static S D_binary(const Case& C, int i, int j, S T, S p) {
  double mij = 1.0 / (NA * (1.0 / C.W[i] + 1.0 / C.W[j]));
  double sg = 0.5 * (C.sig[i] + C.sig[j]);
  double ek = std::sqrt(C.epsk[i] * C.epsk[j]);
  S kT = kB * T;
  return (3.0 / 16.0) * sqrt(2.0 * PI * kT * kT * kT / mij) / (p * PI * sg * sg * omega11(T / ek));
}

// Step 1: primitives and thermodynamics (eqs. 1-4).  Returns an error code.
template <class S>
static int primitives(const Case& C, const S* Uc, double Tguess, Cell<S>& z) {
  const int ns = C.ns;
  z.Y.assign(ns, S(0)); z.X.assign(ns, S(0)); z.h.assign(ns, S(0));
  z.D.assign(ns, S(0)); z.wdot.assign(ns, S(0));
  for (int v = 0; v < ns + 4; ++v)
    if (!std::isfinite(val(Uc[v]))) return ENONFINITE;
  S rho = 0;
  for (int s = 0; s < ns; ++s) rho += Uc[s];
  if (!(val(rho) > 0)) return ENONFINITE;
  z.rho = rho;
  for (int s = 0; s < ns; ++s) z.Y[s] = Uc[s] / rho;
  for (int m = 0; m < 3; ++m) z.u[m] = Uc[ns + m] / rho;
  S ke = 0.5 * (z.u[0] * z.u[0] + z.u[1] * z.u[1] + z.u[2] * z.u[2]);
  S e = Uc[ns + 3] / rho - ke;
  // Newton on e(T) = sum_s Y_s (h_s(T) - R_u T / W_s); converge, then one more step.
  S T = Tguess;
  bool conv = false;
  for (int it = 0; it < 50; ++it) {
    S eT = 0, cv = 0;
    for (int s = 0; s < ns; ++s) {
      const double* a = &C.a7[7 * s];
      double RW = Ru / C.W[s];
      eT += z.Y[s] * RW * T * (h_RT(a, T) - 1.0);
      cv += z.Y[s] * RW * (cp_R(a, T) - 1.0);
    }
    S dT = (eT - e) / cv;
    T = T - dT;
    if (!std::isfinite(val(T)) || !(val(T) > 0)) return ENEWTON;
    if (std::fabs(val(dT)) <= 1e-12 * std::fabs(val(T))) {
      S eT2 = 0, cv2 = 0;
      for (int s = 0; s < ns; ++s) {
        const double* a = &C.a7[7 * s];
        double RW = Ru / C.W[s];
        eT2 += z.Y[s] * RW * T * (h_RT(a, T) - 1.0);
        cv2 += z.Y[s] * RW * (cp_R(a, T) - 1.0);
      }
      T = T - (eT2 - e) / cv2;
      conv = true;
      break;
    }
  }
  if (!conv) return ENEWTON;
  if (val(T) < C.Tmin || val(T) > C.Tmax) return ETRANGE;
  z.T = T;
  S iW = 0;
  for (int s = 0; s < ns; ++s) iW += z.Y[s] / C.W[s];
  z.W = 1.0 / iW;
  z.p = rho * Ru * T / z.W;                          // eq. (4)
  S cp = 0;
  for (int s = 0; s < ns; ++s) {
    const double* a = &C.a7[7 * s];
    double RW = Ru / C.W[s];
    z.X[s] = z.Y[s] * z.W / C.W[s];
    z.h[s] = RW * T * h_RT(a, T);
    cp += z.Y[s] * RW * cp_R(a, T);
  }
  z.cp = cp;
  S cv = cp - Ru / z.W;
  z.c = sqrt(cp / cv * z.p / rho);
  return OK;
}

// Step 1b: mixture-averaged transport: Wilke mu, Wilke-form lambda with
// Eucken species conductivities, Bird mixture diffusivities.
template <class S> static void transport(const Case& C, Cell<S>& z) {
  const int ns = C.ns;
  std::vector<S> mus(ns), lams(ns);
  for (int s = 0; s < ns; ++s) {
    const double* a = &C.a7[7 * s];
    double RW = Ru / C.W[s];
    mus[s] = mu_species(C, s, z.T);
    S cps = RW * cp_R(a, z.T);
    lams[s] = mus[s] * (cps + 1.25 * RW);             // Eucken
  }
  S mu = 0, lam = 0;
  for (int i = 0; i < ns; ++i) {
    S den = 0;
    for (int j = 0; j < ns; ++j) {
      S r = 1.0 + sqrt(mus[i] / mus[j]) * std::pow(C.W[j] / C.W[i], 0.25);
      S phi = r * r / std::sqrt(8.0 * (1.0 + C.W[i] / C.W[j]));
      den += z.X[j] * phi;
    }
    mu += z.X[i] * mus[i] / den;
    lam += z.X[i] * lams[i] / den;
  }
  z.mu = mu;
  z.lam = lam;
  for (int s = 0; s < ns; ++s) {
    S den = 0;
    for (int j = 0; j < ns; ++j) {
      if (j == s) continue;
      S xj = val(z.X[j]) > 0 ? z.X[j] : S(0);
      den += xj / D_binary(C, s, j, z.T, z.p);
    }
    if (val(den) < 1e-300) z.D[s] = D_binary(C, s, s, z.T, z.p);
    else z.D[s] = (1.0 - z.Y[s]) / den;
  }
}

// Step 1c: finite-rate chemistry with reverse rates from equilibrium constants.
template <class S>
static void chemistry(const Case& C, const Params<S>& P, const S* Uc, Cell<S>& z, double* rates = nullptr) {
  const int ns = C.ns;
  std::vector<S> G(ns), conc(ns);
  S lnT = log(z.T);
  for (int s = 0; s < ns; ++s) {
    const double* a = &C.a7[7 * s];
    G[s] = h_RT(a, z.T) - s_R(a, z.T);               // g_s/(R_u T)
    conc[s] = Uc[s] / C.W[s];
  }
  S lnP = log(P0 / (Ru * z.T));
  for (int s = 0; s < ns; ++s) z.wdot[s] = 0;
  for (int j = 0; j < C.nr; ++j) {
    S lnkf = P.lnA[j] + C.beta[j] * lnT - C.Ea[j] / (Ru * z.T);
    S lnKc = 0;
    int dnu = 0;
    for (int s = 0; s < ns; ++s) {
      int nu = C.nur[j * ns + s] - C.nuf[j * ns + s];
      lnKc -= (double)nu * G[s];
      dnu += nu;
    }
    lnKc += (double)dnu * lnP;
    S kf = exp(lnkf);
    S kb = exp(lnkf - lnKc);
    S rf = kf, rb = kb;
    for (int s = 0; s < ns; ++s) {
      for (int m = 0; m < C.nuf[j * ns + s]; ++m) rf *= conc[s];
      for (int m = 0; m < C.nur[j * ns + s]; ++m) rb *= conc[s];
    }
    S q = rf - rb;
    if (rates) { rates[2 * j] = val(rf); rates[2 * j + 1] = val(rb); }
    for (int s = 0; s < ns; ++s) {
      int nu = C.nur[j * ns + s] - C.nuf[j * ns + s];
      if (nu) z.wdot[s] += C.W[s] * (double)nu * q;
    }
  }
  S hrr = 0;
  for (int s = 0; s < ns; ++s) hrr -= z.h[s] * z.wdot[s];
  z.hrr = hrr;
}

// Step 1d: laser deposition, a Gaussian in space (wrapped over the periodic
// images) and time, normalised so that its space-time integral equals E.
template <class S>
static S laser_axis(const Case& C, const Params<S>& P, int a, int i) {
  if (C.n[a] == 1) return S(1);
  if (C.bounded(a)) {   // no periodic images across a boundary
    S z = (C.xnode[a][i] - P.xc[a]) / P.sr;
    return exp(-0.5 * z * z);
  }
  double Lp = C.L[a];
  S r = C.xnode[a][i] - P.xc[a];
  double shift = Lp * std::nearbyint(val(r) / Lp);   // minimum image (a discrete choice)
  r = r - shift;
  int M = (int)std::ceil(9.103 * P.sr / Lp - 0.5);
  if (M < 0) M = 0;
  S g = 0;
  for (int m = -M; m <= M; ++m) {
    S z = (r - (double)m * Lp) / P.sr;
    g += exp(-0.5 * z * z);
  }
  return g;
}
template <class S>
static S laser_q(const Case& C, const Params<S>& P, int i, int j, int k, double t) {
  if (!P.on) return S(0);
  int d = (C.n[0] > 1) + (C.n[1] > 1) + (C.n[2] > 1);
  double norm = std::pow(2.0 * PI, 0.5 * (d + 1)) * std::pow(P.sr, d) * P.st;
  double tt = (t - P.t0) / P.st;
  return P.E / norm * laser_axis(C, P, 0, i) * laser_axis(C, P, 1, j) * laser_axis(C, P, 2, k) *
         std::exp(-0.5 * tt * tt);
}

// ------------------------------------------------------ curvilinear grids
// Methods › Numerical method: the equations are mapped from (x, y, z) to a uniform index space
// (xi, eta, zeta), with U~ = U/J and F~ = (xi_x F + xi_y G + xi_z H)/J along
// each index direction, J = det(d xi / d x).  The index spacing is 1.
//
// Metric terms.  The paper asks for a free-stream-preserving evaluation; it
// is taken here in the conservative form of Thomas & Lombard (1979):
//   (d xi_d / d x_c) / J = D_f[(D_e x_{c1}) x_{c2}] - D_e[(D_f x_{c1}) x_{c2}]
// with (d, e, f) and (c, c1, c2) cyclic permutations of (0, 1, 2) and D the
// sixth-order central difference along an index direction (the derivative
// the six-point central flux implies).  Face values at i+1/2 use the
// six-point interpolation whose face difference is that same D, so the sum
// over directions of the face-metric differences is a sum of commuting second
// differences and vanishes: a uniform flow stays uniform to rounding.
// Coordinates are taken on the unbounded lattice (a node's image n[a] cells
// further along a is displaced by Pv[a]) and relative to the node at which
// the metric is evaluated (the form is invariant under translation).
static long long floordiv(int i, int n) { return (long long)((i - wrap(i, n)) / n); }

static double lattice_coord(const Case& C, int c, int i, int j, int k) {
  const int id[3] = {i, j, k};
  double x = C.X[c][C.idx(wrap(i, C.n[0]), wrap(j, C.n[1]), wrap(k, C.n[2]))];
  for (int a = 0; a < 3; ++a) x += (double)floordiv(id[a], C.n[a]) * C.Pv[a][c];
  return x;
}

// Sixth-order central difference along axis e of f at lattice point p.
template <class Fn> static double d6(Fn f, const int* p, int e) {
  const double w[3] = {45.0, -9.0, 1.0};
  double s = 0;
  for (int m = 1; m <= 3; ++m) {
    int pp[3] = {p[0], p[1], p[2]}, pm[3] = {p[0], p[1], p[2]};
    pp[e] += m;
    pm[e] -= m;
    s += w[m - 1] * (f(pp) - f(pm));
  }
  return s / 60.0;
}

static int set_metrics(Case& C) {
  const long long N = C.N();
  for (int r = 0; r < 9; ++r) { C.mt[r].assign(N, 0.0); C.mf[r].assign(N, 0.0); }
  C.Jac.assign(N, 0.0);
  int bad = 0;
#pragma omp parallel for schedule(static) reduction(+ : bad)
  for (long long q = 0; q < N; ++q) {
    const int p0[3] = {(int)(q % C.n[0]), (int)((q / C.n[0]) % C.n[1]), (int)(q / ((long long)C.n[0] * C.n[1]))};
    double x0[3];
    for (int c = 0; c < 3; ++c) x0[c] = C.X[c][q];
    auto xr = [&](int c) { return [&, c](const int* p) { return lattice_coord(C, c, p[0], p[1], p[2]) - x0[c]; }; };
    for (int d = 0; d < 3; ++d) {
      const int e = (d + 1) % 3, f = (d + 2) % 3;
      for (int c = 0; c < 3; ++c) {
        const int c1 = (c + 1) % 3, c2 = (c + 2) % 3;
        auto xc1 = xr(c1), xc2 = xr(c2);
        auto ge = [&](const int* p) { return d6(xc1, p, e) * xc2(p); };   // (D_e x_c1) x_c2
        auto gf = [&](const int* p) { return d6(xc1, p, f) * xc2(p); };   // (D_f x_c1) x_c2
        C.mt[3 * d + c][q] = d6(ge, p0, f) - d6(gf, p0, e);
      }
    }
    // 1/J = det(d x / d xi): columns D_e x
    double A[3][3];
    for (int c = 0; c < 3; ++c)
      for (int e = 0; e < 3; ++e) A[c][e] = d6(xr(c), p0, e);
    const double det = A[0][0] * (A[1][1] * A[2][2] - A[1][2] * A[2][1]) -
                       A[0][1] * (A[1][0] * A[2][2] - A[1][2] * A[2][0]) +
                       A[0][2] * (A[1][0] * A[2][1] - A[1][1] * A[2][0]);
    if (!(det > 0) || !std::isfinite(det)) { bad += 1; continue; }
    C.Jac[q] = 1.0 / det;
  }
  if (bad) return EINVAL;
  // face values: six-point interpolation along d of the node values
  const double cw[6] = {1.0, -8.0, 37.0, 37.0, -8.0, 1.0};
  for (int d = 0; d < 3; ++d)
    for (long long q = 0; q < N; ++q) {
      int c0[3] = {(int)(q % C.n[0]), (int)((q / C.n[0]) % C.n[1]), (int)(q / ((long long)C.n[0] * C.n[1]))};
      for (int c = 0; c < 3; ++c) {
        double s = 0;
        for (int m = 0; m < 6; ++m) {
          int cc[3] = {c0[0], c0[1], c0[2]};
          cc[d] = wrap(c0[d] - 2 + m, C.n[d]);
          s += cw[m] * C.mt[3 * d + c][C.idx(cc[0], cc[1], cc[2])];
        }
        C.mf[3 * d + c][q] = s / 60.0;
      }
    }
  return OK;
}

// Laser kernel on a curvilinear grid: the same Gaussian of the distance to
// the centre, summed over the lattice images.  The offset is first reduced
// to the nearest image in lattice coordinates (a discrete choice); images
// up to M_a periods away along each active axis are summed, with M_a such
// that every omitted image lies beyond 9.103 sigma_r (the distance between
// lattice planes along a is det / |Pv[b] x Pv[c]|).  An inactive axis drops
// its coordinate, as on rectilinear grids.
template <class S>
static S laser_q_curv(const Case& C, const Params<S>& P, long long q, double t) {
  if (!P.on) return S(0);
  int d = 0, act[3];
  for (int a = 0; a < 3; ++a) { act[a] = C.n[a] > 1; d += act[a]; }
  S r[3], sl[3];
  for (int c = 0; c < 3; ++c) r[c] = C.X[c][q] - P.xc[c];
  for (int a = 0; a < 3; ++a) {
    sl[a] = C.Pinv[a][0] * r[0] + C.Pinv[a][1] * r[1] + C.Pinv[a][2] * r[2];
    if (act[a]) sl[a] = sl[a] - std::nearbyint(val(sl[a]));
    else sl[a] = S(0);
  }
  S rm[3];
  for (int c = 0; c < 3; ++c) rm[c] = sl[0] * C.Pv[0][c] + sl[1] * C.Pv[1][c] + sl[2] * C.Pv[2][c];
  double vol = std::fabs(C.Pv[0][0] * (C.Pv[1][1] * C.Pv[2][2] - C.Pv[1][2] * C.Pv[2][1]) -
                         C.Pv[0][1] * (C.Pv[1][0] * C.Pv[2][2] - C.Pv[1][2] * C.Pv[2][0]) +
                         C.Pv[0][2] * (C.Pv[1][0] * C.Pv[2][1] - C.Pv[1][1] * C.Pv[2][0]));
  int M[3] = {0, 0, 0};
  for (int a = 0; a < 3; ++a) {
    if (!act[a]) continue;
    const double* u = C.Pv[(a + 1) % 3];
    const double* w = C.Pv[(a + 2) % 3];
    double cr[3] = {u[1] * w[2] - u[2] * w[1], u[2] * w[0] - u[0] * w[2], u[0] * w[1] - u[1] * w[0]};
    double h = vol / std::sqrt(cr[0] * cr[0] + cr[1] * cr[1] + cr[2] * cr[2]);
    M[a] = std::max(0, (int)std::ceil(9.103 * P.sr / h - 0.5));
  }
  S g = 0;
  for (int m0 = -M[0]; m0 <= M[0]; ++m0)
    for (int m1 = -M[1]; m1 <= M[1]; ++m1)
      for (int m2 = -M[2]; m2 <= M[2]; ++m2) {
        S r2 = 0;
        for (int c = 0; c < 3; ++c) {
          S z = rm[c] - (m0 * C.Pv[0][c] + m1 * C.Pv[1][c] + m2 * C.Pv[2][c]);
          r2 += z * z;
        }
        g += exp(-0.5 * r2 / (P.sr * P.sr));
      }
  double norm = std::pow(2.0 * PI, 0.5 * (d + 1)) * std::pow(P.sr, d) * P.st;
  double tt = (t - P.t0) / P.st;
  return P.E / norm * g * std::exp(-0.5 * tt * tt);
}

// ----------------------------------------------------------------- WENO3-Z
// Third-order WENO-Z reconstruction at x_{i+1/2} (Don & Borges 2013), the
// paper's alternative shock-capturing scheme (Methods › Numerical method), from f_{i-1}, f_i,
// f_{i+1} = f[1..3] of the six-point face stencil: candidates on {i-1, i} and
// {i, i+1} with optimal weights 1/3 and 2/3, smoothness indicators the
// squared first differences, global indicator tau = |beta_0 - beta_1|,
// alpha_k = d_k (1 + tau / (beta_k + eps)).
template <class S> static S weno3z(const S* f) {
  S q0 = (-f[1] + 3.0 * f[2]) / 2.0;
  S q1 = (f[2] + f[3]) / 2.0;
  S b0 = (f[2] - f[1]) * (f[2] - f[1]);
  S b1 = (f[3] - f[2]) * (f[3] - f[2]);
  S tau = fabs(b0 - b1);
  S a0 = (1.0 / 3.0) * (1.0 + tau / (b0 + 1e-40));
  S a1 = (2.0 / 3.0) * (1.0 + tau / (b1 + 1e-40));
  return (a0 * q0 + a1 * q1) / (a0 + a1);
}

// ------------------------------------------------------------------- TENO6
// Reconstruction at x_{i+1/2} from f[0..5] = f_{i-2..i+3} (Fu et al. 2016):
// four candidate stencils, Jiang-Shu smoothness of each, sixth-order global
// measure tau, sharp cut-off delta_k = [chi_k >= C_T], optimal weights d_k.
template <class S> static S teno6(const S* f, double CT, double* detail = nullptr) {
  double g[6];
  for (int k = 0; k < 6; ++k) g[k] = val(f[k]);
  // candidate reconstructions
  S q0 = (-f[1] + 5.0 * f[2] + 2.0 * f[3]) / 6.0;               // {i-1,i,i+1}
  S q1 = (2.0 * f[2] + 5.0 * f[3] - f[4]) / 6.0;                // {i,i+1,i+2}
  S q2 = (2.0 * f[0] - 7.0 * f[1] + 11.0 * f[2]) / 6.0;         // {i-2,i-1,i}
  S q3 = (3.0 * f[2] + 13.0 * f[3] - 5.0 * f[4] + f[5]) / 12.0; // {i..i+3}
  // smoothness indicators: sum over derivative orders of the cell-i integral
  // of the squared derivatives of each candidate polynomial.  Those
  // derivatives are combinations of the undivided differences of the stencil
  // values (first d, second D, third T, fourth Q, fifth P), so the
  // indicators and the six-point polynomial's coefficients are written with
  // the differences taken first: no cancellation between the stencil values
  // themselves enters them.
  double d[5], D[4], T[3], Q[2];
  for (int k = 0; k < 5; ++k) d[k] = g[k + 1] - g[k];
  for (int k = 0; k < 4; ++k) D[k] = d[k + 1] - d[k];
  for (int k = 0; k < 3; ++k) T[k] = D[k + 1] - D[k];
  for (int k = 0; k < 2; ++k) Q[k] = T[k + 1] - T[k];
  const double P = Q[1] - Q[0];
  // three-point candidates: the second difference (a) and the first
  // derivative at the centre of cell i (b), up to sign
  const double c0a = D[1], c0b = d[1] + d[2];               // {i-1,i,i+1}
  const double c1a = D[2], c1b = 3 * d[2] - d[3];           // {i,i+1,i+2}
  const double c2a = D[0], c2b = 3 * d[1] - d[0];           // {i-2,i-1,i}
  // four-point candidate: its first, second and third derivative terms
  const double c3a = 11 * d[2] - 7 * d[3] + 2 * d[4];
  const double c3b = D[2] - T[2];
  const double c3c = T[2];
  double b0 = 13.0 / 12.0 * c0a * c0a + 0.25 * c0b * c0b;
  double b1 = 13.0 / 12.0 * c1a * c1a + 0.25 * c1b * c1b;
  double b2 = 13.0 / 12.0 * c2a * c2a + 0.25 * c2b * c2b;
  double b3 = 1.0 / 36.0 * c3a * c3a + 13.0 / 12.0 * c3b * c3b + 781.0 / 720.0 * c3c * c3c;
  // six-point polynomial p(x) = sum a_k x^k with cell averages f (x in cell
  // widths, origin at the centre of cell i); beta6 as a quadratic form in a_1..a_5.
  double a1 = (-341 * d[0] + 2444 * d[1] + 5034 * d[2] - 1636 * d[3] + 259 * d[4]) / 5760.0;
  double a2 = (8 * D[1] - Q[0]) / 16.0;
  double a3 = (5 * T[0] + 26 * T[1] - 7 * T[2]) / 144.0;
  double a4 = Q[0] / 24.0;
  double a5 = P / 120.0;
  double b6 = a1 * a1 + 0.5 * a1 * a3 + 0.125 * a1 * a5 + 13.0 / 3.0 * a2 * a2 + 21.0 / 5.0 * a2 * a4 +
              3129.0 / 80.0 * a3 * a3 + 14127.0 / 224.0 * a3 * a5 + 87617.0 / 140.0 * a4 * a4 +
              252337135.0 / 16128.0 * a5 * a5;
  double tau = std::fabs(b6 - (b1 + b2 + 4.0 * b0) / 6.0);
  const double eps = 1e-40;
  double r[4] = {1.0 + tau / (b0 + eps), 1.0 + tau / (b1 + eps), 1.0 + tau / (b2 + eps), 1.0 + tau / (b3 + eps)};
  // gamma_k = r_k^6 and chi_k = gamma_k / sum gamma; evaluated relative to the
  // largest r so that the sixth power cannot overflow (same ratios).
  double rm = std::max(std::max(r[0], r[1]), std::max(r[2], r[3]));
  double gsum = 0, gam[4];
  for (int k = 0; k < 4; ++k) { double s = r[k] / rm; gam[k] = s * s * s * s * s * s; gsum += gam[k]; }
  const double dk[4] = {9.0 / 20.0, 3.0 / 10.0, 1.0 / 20.0, 1.0 / 5.0};
  double wsum = 0, w[4];
  for (int k = 0; k < 4; ++k) { w[k] = (gam[k] / gsum >= CT) ? dk[k] : 0.0; wsum += w[k]; }
  if (detail) {
    const double d[15] = {b0, b1, b2, b3, b6, tau, gam[0] / gsum, gam[1] / gsum, gam[2] / gsum, gam[3] / gsum,
                          w[0] / wsum, w[1] / wsum, w[2] / wsum, w[3] / wsum, 0.0};
    for (int k = 0; k < 15; ++k) detail[k] = d[k];
  }
  return (w[0] * q0 + w[1] * q1 + w[2] * q2 + w[3] * q3) / wsum;
}

// ----------------------------------------------------------------- the RHS
// d phi / d x_a at node c of a rectilinear grid: the second-order central
// difference, on a bounded axis one-sided second order at the boundary nodes
// (-3, 4, -1)/2 inward.  get(q) returns phi at linear index q.
template <class S, class Get>
static S nodal_diff(const Case& C, int a, const int* c, Get get) {
  const int n = C.n[a];
  auto at = [&](int i) {
    int cc[3] = {c[0], c[1], c[2]};
    cc[a] = C.bounded(a) ? i : wrap(i, n);
    return get(C.idx(cc[0], cc[1], cc[2]));
  };
  const double xi = C.xin[a][c[a]];
  const int i = c[a];
  if (C.bounded(a) && i == 0) return xi * (-3.0 * at(0) + 4.0 * at(1) - at(2)) / 2.0;
  if (C.bounded(a) && i == n - 1) return xi * (3.0 * at(n - 1) - 4.0 * at(n - 2) + at(n - 3)) / 2.0;
  return xi * (at(i + 1) - at(i - 1)) / 2.0;
}

template <class S> struct Fields {
  std::vector<Cell<S>> cell;
  std::vector<double> theta;   // sensor per node
};

template <class S>
static int eval_cells(const Case& C, const Params<S>& P, const S* U, double* T_io, double t,
                      Fields<S>& F) {
  const long long N = C.N();
  const int nv = C.ns + 4;
  F.cell.assign(N, Cell<S>());
  int err = OK;
#pragma omp parallel for schedule(static) reduction(max : err)
  for (long long q = 0; q < N; ++q) {
    std::vector<S> Uc(nv);
    for (int v = 0; v < nv; ++v) Uc[v] = U[v * N + q];
    Cell<S>& z = F.cell[q];
    int e = primitives(C, Uc.data(), T_io[q], z);
    if (e) { err = std::max(err, e); continue; }
    transport(C, z);
    if (!(C.flags & CHEM_OFF)) chemistry(C, P, Uc.data(), z);
    else z.hrr = 0;
    int i = q % C.n[0], j = (q / C.n[0]) % C.n[1], k = q / ((long long)C.n[0] * C.n[1]);
    z.qL = C.curv ? laser_q_curv(C, P, q, t) : laser_q(C, P, i, j, k, t);
  }
  if (err) return err;
  for (long long q = 0; q < N; ++q) T_io[q] = val(F.cell[q].T);
  // Step 2: dilatation/vorticity sensor at every node (second-order central).
  F.theta.assign(N, 0.0);
#pragma omp parallel for schedule(static)
  for (long long q = 0; q < N; ++q) {
    int i = q % C.n[0], j = (q / C.n[0]) % C.n[1], k = q / ((long long)C.n[0] * C.n[1]);
    int c[3] = {i, j, k};
    double g[3][3] = {{0}};   // g[a][m] = d u_m / d x_a
    for (int a = 0; a < 3; ++a) {
      if (C.n[a] == 1) continue;
      int cp[3] = {c[0], c[1], c[2]}, cm[3] = {c[0], c[1], c[2]};
      cp[a] = wrap(c[a] + 1, C.n[a]);
      cm[a] = wrap(c[a] - 1, C.n[a]);
      const Cell<S>& zp = F.cell[C.idx(cp[0], cp[1], cp[2])];
      const Cell<S>& zm = F.cell[C.idx(cm[0], cm[1], cm[2])];
      if (C.curv) {
        // chain rule: d/dx_b = sum_a (d xi_a / d x_b) d/d xi_a, with d xi_a / d x_b = J mt[3a + b]
        for (int b = 0; b < 3; ++b)
          for (int m = 0; m < 3; ++m)
            g[b][m] += C.Jac[q] * C.mt[3 * a + b][q] * (val(zp.u[m]) - val(zm.u[m])) / 2.0;
        continue;
      }
      for (int m = 0; m < 3; ++m)
        g[a][m] = nodal_diff<double>(C, a, c, [&](long long qq) { return val(F.cell[qq].u[m]); });
    }
    double div = g[0][0] + g[1][1] + g[2][2];
    double wx = g[1][2] - g[2][1], wy = g[2][0] - g[0][2], wz = g[0][1] - g[1][0];
    double d2 = div * div;
    F.theta[q] = d2 / (d2 + wx * wx + wy * wy + wz * wz + 1e-300);
  }
  return OK;
}

// Convective flux of variable v at a node along direction d.
template <class S> static S node_flux(const Case& C, const S* Uc, const Cell<S>& z, int v, int d) {
  const int ns = C.ns;
  S un = z.u[d];
  if (v < ns) return Uc[v] * un;
  if (v < ns + 3) return Uc[v] * un + ((v - ns) == d ? z.p : S(0));
  return (Uc[v] + z.p) * un;
}

// Step 3a: hybrid switch at face i+1/2: TENO where the sensor exceeds its
// threshold anywhere on the six-point stencil or the pressure jump across the
// face is large; the central flux elsewhere.  Decisions use the real part.
template <class S>
static bool use_teno(const Case& C, const Fields<S>& F, const long long* st) {
  if (C.flags & FORCE_TENO) return true;
  if (C.flags & FORCE_CENTRAL) return false;
  double th = 0;
  for (int m = 0; m < 6; ++m) th = std::max(th, F.theta[st[m]]);
  double pa = val(F.cell[st[2]].p), pb = val(F.cell[st[3]].p);
  double psi = std::fabs(pb - pa) / std::min(pa, pb);
  return (th > C.theta_c) || (psi > C.psi_c);
}

// Step 3b: convective numerical flux at face i+1/2 along d (all variables);
// st[0..5] are the linear indices of nodes i-2..i+3.  Returns 1 for TENO.
template <class S>
static int conv_flux(const Case& C, const S* U, const Fields<S>& F, int d, const long long* st, S* out) {
  const long long N = C.N();
  const int nv = C.ns + 4;
  bool teno = use_teno(C, F, st);
  std::vector<S> Uk(nv * 6);
  for (int m = 0; m < 6; ++m)
    for (int v = 0; v < nv; ++v) Uk[m * nv + v] = U[v * N + st[m]];
  if (!teno) {
    const double cc[6] = {1.0, -8.0, 37.0, 37.0, -8.0, 1.0};
    for (int v = 0; v < nv; ++v) {
      S s = 0;
      for (int m = 0; m < 6; ++m) s += cc[m] * node_flux(C, &Uk[m * nv], F.cell[st[m]], v, d);
      out[v] = s / 60.0;
    }
    return 0;
  }
  // local Lax-Friedrichs speed: largest |u_n| + c over the stencil (argmax frozen)
  int am = 0;
  double best = -1;
  for (int m = 0; m < 6; ++m) {
    double sp = std::fabs(val(F.cell[st[m]].u[d])) + val(F.cell[st[m]].c);
    if (sp > best) { best = sp; am = m; }
  }
  S alpha = fabs(F.cell[st[am]].u[d]) + F.cell[st[am]].c;
  for (int v = 0; v < nv; ++v) {
    S fp[6], fm[6];
    for (int m = 0; m < 6; ++m) {
      S fl = node_flux(C, &Uk[m * nv], F.cell[st[m]], v, d);
      fp[m] = 0.5 * (fl + alpha * Uk[m * nv + v]);
      fm[5 - m] = 0.5 * (fl - alpha * Uk[m * nv + v]);   // mirrored: i+3..i-2
    }
    out[v] = (C.flags & WENO3Z) ? weno3z(fp) + weno3z(fm) : teno6(fp, C.CT) + teno6(fm, C.CT);
  }
  return 1;
}

// Step 3b near a boundary of a bounded axis, where the six-point stencil
// does not fit: the face i+1/2 between nodes st[k-1] and st[k] (k = m/2) of
// an m-point stencil (m = 4: nodes i-1..i+2; m = 2: nodes i, i+1).  Central
// faces take the widest centred interpolation that fits, (-1, 7, 7, -1)/12
// or (1, 1)/2; faces the hybrid switch marks (sensor over the m nodes, or
// the pressure jump) take the first-order local Lax-Friedrichs (Rusanov)
// flux of the two face nodes, alpha = max over the m nodes of |u_n| + c.
template <class S>
static int conv_flux_reduced(const Case& C, const S* U, const Fields<S>& F, int d, const long long* st, int m,
                             S* out) {
  const long long N = C.N();
  const int nv = C.ns + 4;
  const int a = m / 2 - 1, b = m / 2;   // the face's two nodes within st
  bool flag;
  if (C.flags & FORCE_TENO) flag = true;
  else if (C.flags & FORCE_CENTRAL) flag = false;
  else {
    double th = 0;
    for (int k = 0; k < m; ++k) th = std::max(th, F.theta[st[k]]);
    double pa = val(F.cell[st[a]].p), pb = val(F.cell[st[b]].p);
    double psi = std::fabs(pb - pa) / std::min(pa, pb);
    flag = (th > C.theta_c) || (psi > C.psi_c);
  }
  std::vector<S> Uk(nv * m);
  for (int k = 0; k < m; ++k)
    for (int v = 0; v < nv; ++v) Uk[k * nv + v] = U[v * N + st[k]];
  if (!flag) {
    for (int v = 0; v < nv; ++v) {
      if (m == 4) {
        S s = -node_flux(C, &Uk[0], F.cell[st[0]], v, d) + 7.0 * node_flux(C, &Uk[nv], F.cell[st[1]], v, d) +
              7.0 * node_flux(C, &Uk[2 * nv], F.cell[st[2]], v, d) - node_flux(C, &Uk[3 * nv], F.cell[st[3]], v, d);
        out[v] = s / 12.0;
      } else {
        out[v] = (node_flux(C, &Uk[0], F.cell[st[0]], v, d) + node_flux(C, &Uk[nv], F.cell[st[1]], v, d)) / 2.0;
      }
    }
    return 0;
  }
  int am = 0;
  double best = -1;
  for (int k = 0; k < m; ++k) {
    double sp = std::fabs(val(F.cell[st[k]].u[d])) + val(F.cell[st[k]].c);
    if (sp > best) { best = sp; am = k; }
  }
  S alpha = fabs(F.cell[st[am]].u[d]) + F.cell[st[am]].c;
  for (int v = 0; v < nv; ++v) {
    S fa = node_flux(C, &Uk[a * nv], F.cell[st[a]], v, d);
    S fb = node_flux(C, &Uk[b * nv], F.cell[st[b]], v, d);
    out[v] = (fa + fb) / 2.0 - alpha * (Uk[b * nv + v] - Uk[a * nv + v]) / 2.0;
  }
  return 1;
}

// Step 3c: diffusive flux at face i+1/2 along d (eqs. 1-3, 5, 6), sign as it
// enters the right-hand side.  A second-order compact face form: normal
// derivatives from the two adjacent nodes, tangential derivatives as the mean
// of the nodal central differences, face coefficients as arithmetic means.
template <class S>
static void diff_flux(const Case& C, const Fields<S>& F, int d, int i, int j, int k, S* out) {
  const int ns = C.ns;
  int c0[3] = {i, j, k}, c1[3] = {i, j, k};
  c1[d] = wrap(c0[d] + 1, C.n[d]);
  const Cell<S>& A = F.cell[C.idx(c0[0], c0[1], c0[2])];
  const Cell<S>& B = F.cell[C.idx(c1[0], c1[1], c1[2])];
  double xf = C.xif[d][c0[d]];
  // velocity gradient at the face: grad[a][m] = d u_m / d x_a
  S grad[3][3];
  for (int a = 0; a < 3; ++a)
    for (int m = 0; m < 3; ++m) grad[a][m] = 0;
  for (int m = 0; m < 3; ++m) grad[d][m] = xf * (B.u[m] - A.u[m]);
  for (int a = 0; a < 3; ++a) {
    if (a == d || C.n[a] == 1) continue;
    for (int side = 0; side < 2; ++side) {
      const int* c = side ? c1 : c0;
      for (int m = 0; m < 3; ++m)
        grad[a][m] += 0.5 * nodal_diff<S>(C, a, c, [&](long long qq) { return F.cell[qq].u[m]; });
    }
  }
  S mu = 0.5 * (A.mu + B.mu), lam = 0.5 * (A.lam + B.lam), rho = 0.5 * (A.rho + B.rho);
  S W = 0.5 * (A.W + B.W);
  S divu = grad[0][0] + grad[1][1] + grad[2][2];
  // viscous stress row tau_{d m} (Stokes hypothesis)
  S tau[3];
  for (int m = 0; m < 3; ++m) {
    tau[m] = mu * (grad[d][m] + grad[m][d]);
    if (m == d) tau[m] -= (2.0 / 3.0) * mu * divu;
  }
  // species fluxes J_s = rho Y_s V_s with the correction velocity (sum J_s = 0)
  std::vector<S> Js(ns), Yf(ns), hf(ns);
  S corr = 0;
  for (int s = 0; s < ns; ++s) {
    S Df = 0.5 * (A.D[s] + B.D[s]);
    S dX = xf * (B.X[s] - A.X[s]);
    Js[s] = -rho * Df * (C.W[s] / W) * dX;
    corr += rho * Df * (C.W[s] / W) * dX;
    Yf[s] = 0.5 * (A.Y[s] + B.Y[s]);
    hf[s] = 0.5 * (A.h[s] + B.h[s]);
  }
  S qn = -lam * xf * (B.T - A.T);
  for (int s = 0; s < ns; ++s) {
    Js[s] += Yf[s] * corr;
    qn += Js[s] * hf[s];
  }
  for (int s = 0; s < ns; ++s) out[s] = -Js[s];
  S work = 0;
  for (int m = 0; m < 3; ++m) {
    out[ns + m] = tau[m];
    work += tau[m] * 0.5 * (A.u[m] + B.u[m]);
  }
  out[ns + 3] = work - qn;
}

// Mapped convective flux of variable v at a node through a face with metric
// vector n = (d xi_d / d x) / J: the physical flux projected on n.
template <class S>
static S node_flux_mapped(const Case& C, const S* Uc, const Cell<S>& z, int v, const double* n) {
  const int ns = C.ns;
  S un = z.u[0] * n[0] + z.u[1] * n[1] + z.u[2] * n[2];
  if (v < ns) return Uc[v] * un;
  if (v < ns + 3) return Uc[v] * un + z.p * n[v - ns];
  return (Uc[v] + z.p) * un;
}

// Step 3b on a curvilinear grid: the same hybrid switch, central flux and
// TENO6 (or WENO3-Z) on the local Lax-Friedrichs split, applied to the mapped
// flux with the face's metric vector held fixed across the stencil; the LF
// speed is the largest |u . n| + c |n| over the stencil.
template <class S>
static int conv_flux_curv(const Case& C, const S* U, const Fields<S>& F, int d, long long qf, const long long* st,
                          S* out) {
  const long long N = C.N();
  const int nv = C.ns + 4;
  double n[3] = {C.mf[3 * d][qf], C.mf[3 * d + 1][qf], C.mf[3 * d + 2][qf]};
  double nn = std::sqrt(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
  bool teno = use_teno(C, F, st);
  std::vector<S> Uk(nv * 6);
  for (int m = 0; m < 6; ++m)
    for (int v = 0; v < nv; ++v) Uk[m * nv + v] = U[v * N + st[m]];
  if (!teno) {
    const double cc[6] = {1.0, -8.0, 37.0, 37.0, -8.0, 1.0};
    for (int v = 0; v < nv; ++v) {
      S s = 0;
      for (int m = 0; m < 6; ++m) s += cc[m] * node_flux_mapped(C, &Uk[m * nv], F.cell[st[m]], v, n);
      out[v] = s / 60.0;
    }
    return 0;
  }
  int am = 0;
  double best = -1;
  for (int m = 0; m < 6; ++m) {
    const Cell<S>& z = F.cell[st[m]];
    double sp = std::fabs(val(z.u[0]) * n[0] + val(z.u[1]) * n[1] + val(z.u[2]) * n[2]) + val(z.c) * nn;
    if (sp > best) { best = sp; am = m; }
  }
  const Cell<S>& za = F.cell[st[am]];
  S alpha = fabs(za.u[0] * n[0] + za.u[1] * n[1] + za.u[2] * n[2]) + za.c * nn;
  for (int v = 0; v < nv; ++v) {
    S fp[6], fm[6];
    for (int m = 0; m < 6; ++m) {
      S fl = node_flux_mapped(C, &Uk[m * nv], F.cell[st[m]], v, n);
      fp[m] = 0.5 * (fl + alpha * Uk[m * nv + v]);
      fm[5 - m] = 0.5 * (fl - alpha * Uk[m * nv + v]);
    }
    out[v] = (C.flags & WENO3Z) ? weno3z(fp) + weno3z(fm) : teno6(fp, C.CT) + teno6(fm, C.CT);
  }
  return 1;
}

// Step 3c on a curvilinear grid: the mapped diffusive flux through face
// i+1/2 along d.  Index-space derivatives at the face: along d from the two
// adjacent nodes, along the other active axes the mean of the two nodes'
// central differences (the second-order compact face form of the rectilinear
// case).  Physical gradients by the chain rule with the face value of
// d xi_e / d x (mean of the two nodes); the flux vector is then projected on
// the face metric vector, as the convective flux.  Face coefficients are
// arithmetic means.
template <class S>
static void diff_flux_curv(const Case& C, const Fields<S>& F, int d, int i, int j, int k, S* out) {
  const int ns = C.ns;
  int c0[3] = {i, j, k}, c1[3] = {i, j, k};
  c1[d] = wrap(c0[d] + 1, C.n[d]);
  const long long qa = C.idx(c0[0], c0[1], c0[2]), qb = C.idx(c1[0], c1[1], c1[2]);
  const Cell<S>& A = F.cell[qa];
  const Cell<S>& B = F.cell[qb];
  const double n[3] = {C.mf[3 * d][qa], C.mf[3 * d + 1][qa], C.mf[3 * d + 2][qa]};
  // G[e][b] = d xi_e / d x_b at the face
  double G[3][3];
  for (int e = 0; e < 3; ++e)
    for (int b = 0; b < 3; ++b)
      G[e][b] = 0.5 * (C.Jac[qa] * C.mt[3 * e + b][qa] + C.Jac[qb] * C.mt[3 * e + b][qb]);
  // index-space derivative along e at the face of a per-cell quantity
  auto dxi = [&](auto get, int e) -> S {
    if (e == d) return get(B) - get(A);
    if (C.n[e] == 1) return S(0);
    S s = 0;
    for (int side = 0; side < 2; ++side) {
      const int* c = side ? c1 : c0;
      int cp[3] = {c[0], c[1], c[2]}, cm[3] = {c[0], c[1], c[2]};
      cp[e] = wrap(c[e] + 1, C.n[e]);
      cm[e] = wrap(c[e] - 1, C.n[e]);
      s += 0.5 * (get(F.cell[C.idx(cp[0], cp[1], cp[2])]) - get(F.cell[C.idx(cm[0], cm[1], cm[2])])) / 2.0;
    }
    return s;
  };
  // physical gradient at the face
  auto grad = [&](auto get, S* g) {
    S de[3];
    for (int e = 0; e < 3; ++e) de[e] = dxi(get, e);
    for (int b = 0; b < 3; ++b) g[b] = G[0][b] * de[0] + G[1][b] * de[1] + G[2][b] * de[2];
  };
  S gu[3][3];   // gu[b][m] = d u_m / d x_b
  for (int m = 0; m < 3; ++m) {
    S g[3];
    grad([m](const Cell<S>& z) { return z.u[m]; }, g);
    for (int b = 0; b < 3; ++b) gu[b][m] = g[b];
  }
  S mu = 0.5 * (A.mu + B.mu), lam = 0.5 * (A.lam + B.lam), rho = 0.5 * (A.rho + B.rho);
  S W = 0.5 * (A.W + B.W);
  S divu = gu[0][0] + gu[1][1] + gu[2][2];
  // (tau . n)_m = sum_b n_b tau_{b m}, Stokes hypothesis
  S tn[3];
  for (int m = 0; m < 3; ++m) {
    tn[m] = 0;
    for (int b = 0; b < 3; ++b) {
      S tau = mu * (gu[b][m] + gu[m][b]);
      if (b == m) tau -= (2.0 / 3.0) * mu * divu;
      tn[m] += n[b] * tau;
    }
  }
  std::vector<S> Jn(ns), Yf(ns), hf(ns);
  S corr = 0;
  for (int s = 0; s < ns; ++s) {
    S g[3];
    grad([s](const Cell<S>& z) { return z.X[s]; }, g);
    S dXn = g[0] * n[0] + g[1] * n[1] + g[2] * n[2];
    S Df = 0.5 * (A.D[s] + B.D[s]);
    Jn[s] = -rho * Df * (C.W[s] / W) * dXn;
    corr += rho * Df * (C.W[s] / W) * dXn;
    Yf[s] = 0.5 * (A.Y[s] + B.Y[s]);
    hf[s] = 0.5 * (A.h[s] + B.h[s]);
  }
  S gT[3];
  grad([](const Cell<S>& z) { return z.T; }, gT);
  S qn = -lam * (gT[0] * n[0] + gT[1] * n[1] + gT[2] * n[2]);
  for (int s = 0; s < ns; ++s) {
    Jn[s] += Yf[s] * corr;
    qn += Jn[s] * hf[s];
  }
  for (int s = 0; s < ns; ++s) out[s] = -Jn[s];
  S work = 0;
  for (int m = 0; m < 3; ++m) {
    out[ns + m] = tn[m];
    work += tn[m] * 0.5 * (A.u[m] + B.u[m]);
  }
  out[ns + 3] = work - qn;
}

// Step 5, boundary nodes of bounded axes (Poinsot & Lele's characteristic
// boundary conditions, cited by the paper as NSCBC).  The normal convective
// terms at a boundary node are written as the locally one-dimensional wave
// amplitudes along the axis (one-sided derivatives at the node, u_n the
// velocity along the axis, c the frozen sound speed):
//   L1 = (u_n - c)(dp - rho c du_n),  L5 = (u_n + c)(dp + rho c du_n),
//   L2 = u_n (c^2 drho - dp),  L3, L4 = u_n du_t,  LY_s = u_n dY_s,
// whose primitive rates are
//   rho_t = -(L2 + (L5 + L1)/2) / c^2,  p_t = -(L5 + L1)/2,
//   un_t = -(L5 - L1)/(2 rho c),  ut_t = -L3, -L4,  Y_t = -LY.
// Waves entering the domain are replaced:
// - outflow: the entering acoustic wave relaxes p to p_inf,
//   L = K (p - p_inf) with K = sigma c (1 - M^2) / L_axis; entering
//   entropy, shear and species waves (backflow) are zero; the normal
//   gradients of the diffusive fluxes are taken as zero;
// - wall (no-slip, isothermal) and inflow (velocity, temperature and, for
//   the inflow, composition imposed): these are held at the node's values
//   and the entering acoustic wave equals the leaving one.  At a wall
//   (u_n = 0) there is no entropy wave, L2 = 0, so rho_t = -L_out / c^2 (the
//   continuity equation; the held T stands for the heat the wall takes); at
//   an inflow the entropy wave holds T, L2 = (gamma - 1)(L5 + L1)/2, so
//   rho_t = -(gamma / c^2) L_out.  At a wall the species diffuse with zero
//   flux through the wall (half control volume); momentum and energy follow
//   from the held u and T.
// Tangential fluxes and sources at the node are those of any other node.
template <class S>
static void boundary_nodes(const Case& C, const Fields<S>& F, const std::vector<S>* Fd, S* dUdt) {
  const long long N = C.N();
  const int ns = C.ns, nv = ns + 4;
#pragma omp parallel for schedule(static)
  for (long long q = 0; q < N; ++q) {
    int c[3] = {(int)(q % C.n[0]), (int)((q / C.n[0]) % C.n[1]), (int)(q / ((long long)C.n[0] * C.n[1]))};
    bool onb = false;
    for (int a = 0; a < 3; ++a)
      if (C.bounded(a) && (c[a] == 0 || c[a] == C.n[a] - 1)) onb = true;
    if (!onb) continue;
    const Cell<S>& z = F.cell[q];
    const S cv = z.cp - Ru / z.W, gam = z.cp / cv, cc = z.c, cc2 = z.c * z.c;
    bool held = false, holdY = false;
    std::vector<S> add(nv, S(0));   // outflow sides: conserved rates; held sides: species terms
    for (int a = 0; a < 3; ++a) {
      if (!C.bounded(a)) continue;
      for (int side = 0; side < 2; ++side) {
        if (c[a] != (side ? C.n[a] - 1 : 0)) continue;
        const int type = C.bc[a][side];
        const double sgn = side ? 1.0 : -1.0;   // outward normal along a
        auto D = [&](auto get) { return nodal_diff<S>(C, a, c, get); };
        S Dp = D([&](long long qq) { return F.cell[qq].p; });
        S Dr = D([&](long long qq) { return F.cell[qq].rho; });
        S Du[3];
        for (int m = 0; m < 3; ++m) Du[m] = D([&](long long qq) { return F.cell[qq].u[m]; });
        const S un = z.u[a];
        S L1 = (un - cc) * (Dp - z.rho * cc * Du[a]);
        S L5 = (un + cc) * (Dp + z.rho * cc * Du[a]);
        if (type == BC_WALL || type == BC_INFLOW) {
          held = true;
          if (type == BC_INFLOW) holdY = true;
          // the entering acoustic wave equals the leaving one; at a wall
          // u_n = 0 carries no entropy wave, at an inflow the entropy wave
          // holds T: L2 = (gamma - 1)(L5 + L1)/2
          const S Lout = side ? L5 : L1;
          const S drho = (type == BC_INFLOW ? -(gam / cc2) : -(1.0 / cc2)) * Lout;
          for (int s = 0; s < ns; ++s) add[s] += z.Y[s] * drho;
          if (type == BC_WALL && !(C.flags & VISC_OFF)) {
            // zero species flux through the wall: half control volume at the node
            const long long qf = side ? q - (long long)(a == 0 ? 1 : (a == 1 ? C.n[0] : C.n[0] * C.n[1])) : q;
            const double x2 = 2.0 * C.xin[a][c[a]];
            for (int s = 0; s < ns; ++s) add[s] += (side ? -x2 : x2) * Fd[a][(size_t)qf * nv + s];
          }
          continue;
        }
        // outflow
        S L2 = un * (cc2 * Dr - Dp);
        S L3 = un * Du[(a + 1) % 3], L4 = un * Du[(a + 2) % 3];
        std::vector<S> LY(ns);
        for (int s = 0; s < ns; ++s) LY[s] = un * D([&](long long qq) { return F.cell[qq].Y[s]; });
        const double Ld = std::fabs(C.xnode[a][C.n[a] - 1] - C.xnode[a][0]);
        const S M = fabs(un) / cc;
        const S K = C.relax[a][side] * cc * (1.0 - M * M) / Ld;
        const S relaxp = K * (z.p - C.pinf[a][side]);
        if (sgn * val(un - cc) < 0) L1 = relaxp;
        if (sgn * val(un + cc) < 0) L5 = relaxp;
        if (sgn * val(un) < 0) {
          L2 = 0; L3 = 0; L4 = 0;
          for (int s = 0; s < ns; ++s) LY[s] = 0;
        }
        const S rho_t = -(L2 + 0.5 * (L5 + L1)) / cc2;
        const S p_t = -0.5 * (L5 + L1);
        S u_t[3];
        u_t[a] = -(L5 - L1) / (2.0 * z.rho * cc);
        u_t[(a + 1) % 3] = -L3;
        u_t[(a + 2) % 3] = -L4;
        S ke = 0, udu = 0;
        for (int m = 0; m < 3; ++m) { ke += z.u[m] * z.u[m]; udu += z.u[m] * u_t[m]; }
        S dE = (z.cp * z.W / Ru - 1.0) * p_t + 0.5 * ke * rho_t + z.rho * udu;
        for (int s = 0; s < ns; ++s) {
          S drs = z.Y[s] * rho_t - z.rho * LY[s];
          add[s] += drs;
          dE += (z.h[s] - z.cp * z.T * z.W / C.W[s]) * drs;
        }
        for (int m = 0; m < 3; ++m) add[ns + m] += z.u[m] * rho_t + z.rho * u_t[m];
        add[ns + 3] += dE;
      }
    }
    if (!held) {
      for (int v = 0; v < nv; ++v) dUdt[v * N + q] += add[v];
      continue;
    }
    // held node: species rates from every term, then u and T (and Y) held
    std::vector<S> drs(ns);
    S drho = 0;
    for (int s = 0; s < ns; ++s) { drs[s] = dUdt[s * N + q] + add[s]; drho += drs[s]; }
    if (holdY)
      for (int s = 0; s < ns; ++s) drs[s] = z.Y[s] * drho;
    S ke = 0;
    for (int m = 0; m < 3; ++m) ke += z.u[m] * z.u[m];
    S dE = 0;
    for (int s = 0; s < ns; ++s) {
      dUdt[s * N + q] = drs[s];
      dE += (z.h[s] - Ru * z.T / C.W[s] + 0.5 * ke) * drs[s];
    }
    for (int m = 0; m < 3; ++m) dUdt[(ns + m) * N + q] = z.u[m] * drho;
    dUdt[(ns + 3) * N + q] = dE;
  }
}

template <class S>
static int rhs(const Case& C, const Params<S>& P, const S* U, double* T_io, double t, S* dUdt,
               S* hrr_out, unsigned char* mask, Fields<S>* keep) {
  const long long N = C.N();
  const int ns = C.ns, nv = ns + 4;
  Fields<S> Floc;
  Fields<S>& F = keep ? *keep : Floc;
  int err = eval_cells(C, P, U, T_io, t, F);
  if (err) return err;
  for (long long q = 0; q < N * nv; ++q) dUdt[q] = 0;
  // Step 4 (sources): chemistry into the species equations, laser into energy.
  for (long long q = 0; q < N; ++q) {
    if (!(C.flags & CHEM_OFF))
      for (int s = 0; s < ns; ++s) dUdt[s * N + q] = F.cell[q].wdot[s];
    dUdt[(ns + 3) * N + q] = F.cell[q].qL;
    if (hrr_out) hrr_out[q] = F.cell[q].hrr;
  }
  std::vector<S> FdKeep[3];
  bool anyb = false;
  for (int d = 0; d < 3; ++d) {
    if (C.n[d] == 1) continue;
    const bool bnd = C.bounded(d);
    anyb = anyb || bnd;
    const int n = C.n[d];
    // face fluxes, face f = i+1/2 stored at the index of node i (on a bounded
    // axis faces i = 0 .. n-2 only)
    std::vector<S> Fc((size_t)N * nv), Fd((size_t)N * nv);
#pragma omp parallel for schedule(static)
    for (long long q = 0; q < N; ++q) {
      int c[3] = {(int)(q % C.n[0]), (int)((q / C.n[0]) % C.n[1]), (int)(q / ((long long)C.n[0] * C.n[1]))};
      if (bnd && c[d] == n - 1) {
        if (mask) mask[(size_t)d * N + q] = 0;
        continue;
      }
      // stencil: six points i-2..i+3, or near a boundary the reduced m points
      int m = 6, start = c[d] - 2;
      if (bnd && (c[d] < 2 || c[d] > n - 4)) {
        m = (c[d] == 0 || c[d] == n - 2) ? 2 : 4;
        start = c[d] - m / 2 + 1;
      }
      long long st[6];
      for (int k = 0; k < m; ++k) {
        int cc[3] = {c[0], c[1], c[2]};
        cc[d] = bnd ? start + k : wrap(start + k, n);
        st[k] = C.idx(cc[0], cc[1], cc[2]);
      }
      std::vector<S> fc(nv), fd(nv);
      int te = C.curv ? conv_flux_curv(C, U, F, d, q, st, fc.data())
                      : (m == 6 ? conv_flux(C, U, F, d, st, fc.data()) : conv_flux_reduced(C, U, F, d, st, m, fc.data()));
      if (mask) mask[(size_t)d * N + q] = (unsigned char)te;
      if (C.flags & VISC_OFF) for (int v = 0; v < nv; ++v) fd[v] = 0;
      else if (C.curv) diff_flux_curv(C, F, d, c[0], c[1], c[2], fd.data());
      else diff_flux(C, F, d, c[0], c[1], c[2], fd.data());
      for (int v = 0; v < nv; ++v) { Fc[(size_t)q * nv + v] = fc[v]; Fd[(size_t)q * nv + v] = fd[v]; }
    }
    // flux differences: dU/dt += xi_d (-(Fc_{i+1/2} - Fc_{i-1/2}) + (Fd_{i+1/2} - Fd_{i-1/2})),
    // on a curvilinear grid J times the mapped flux difference (index spacing 1);
    // on a bounded axis at the interior nodes only
    for (long long q = 0; q < N; ++q) {
      int c[3] = {(int)(q % C.n[0]), (int)((q / C.n[0]) % C.n[1]), (int)(q / ((long long)C.n[0] * C.n[1]))};
      if (bnd && (c[d] == 0 || c[d] == n - 1)) continue;
      int cm[3] = {c[0], c[1], c[2]};
      cm[d] = wrap(c[d] - 1, n);
      long long qm = C.idx(cm[0], cm[1], cm[2]);
      double xi = C.curv ? C.Jac[q] : C.xin[d][c[d]];
      for (int v = 0; v < nv; ++v) {
        S conv = Fc[(size_t)q * nv + v] - Fc[(size_t)qm * nv + v];
        S dif = Fd[(size_t)q * nv + v] - Fd[(size_t)qm * nv + v];
        dUdt[v * N + q] += xi * (dif - conv);
      }
    }
    if (bnd) FdKeep[d] = std::move(Fd);
  }
  if (anyb) boundary_nodes(C, F, FdKeep, dUdt);
  return OK;
}

// Cell volume (product of widths along all three axes).
static double cell_volume(const Case& C, long long q) {
  if (C.curv) return 1.0 / C.Jac[q];
  int c[3] = {(int)(q % C.n[0]), (int)((q / C.n[0]) % C.n[1]), (int)(q / ((long long)C.n[0] * C.n[1]))};
  return 1.0 / (C.xin[0][c[0]] * C.xin[1][c[1]] * C.xin[2][c[2]]);
}

// Largest stable step: convective and diffusive limits, times the CFL number.
static int stable_dt(const Case& C, const double* U, double* T_io, double* dt) {
  Params<double> P;
  P.lnA.assign(C.lnA.begin(), C.lnA.end());
  P.E = 0; P.xc[0] = P.xc[1] = P.xc[2] = 0; P.sr = 1; P.t0 = 0; P.st = 1; P.on = false;
  Fields<double> F;
  int err = eval_cells(C, P, U, T_io, 0.0, F);
  if (err) return err;
  double best = INFINITY;
  for (long long q = 0; q < C.N(); ++q) {
    const Cell<double>& z = F.cell[q];
    int c[3] = {(int)(q % C.n[0]), (int)((q / C.n[0]) % C.n[1]), (int)(q / ((long long)C.n[0] * C.n[1]))};
    double sc = 0, sd = 0;
    for (int a = 0; a < 3; ++a) {
      if (C.n[a] == 1) continue;
      if (C.curv) {
        // contravariant speed |u . grad xi_a| + c |grad xi_a|, grad xi_a = J mt_a
        double g[3], un = 0, g2 = 0;
        for (int b = 0; b < 3; ++b) {
          g[b] = C.Jac[q] * C.mt[3 * a + b][q];
          un += z.u[b] * g[b];
          g2 += g[b] * g[b];
        }
        sc += std::fabs(un) + z.c * std::sqrt(g2);
        sd += g2;
        continue;
      }
      double xi = C.xin[a][c[a]];
      sc += (std::fabs(z.u[a]) + z.c) * xi;
      sd += xi * xi;
    }
    double nu = std::max(z.mu / z.rho, z.lam / (z.rho * z.cp));
    for (int s = 0; s < C.ns; ++s) nu = std::max(nu, z.D[s]);
    double lim = sc > 0 ? 1.0 / sc : INFINITY;
    if (!(C.flags & VISC_OFF) && sd > 0) lim = std::min(lim, 1.0 / (2.0 * sd * nu));
    best = std::min(best, lim);
  }
  *dt = C.cfl * best;
  return OK;
}

// One SSP-RK3 step (Shu-Osher form) and the step's contribution to the
// time-integrated heat release, using the scheme's own quadrature weights.
template <class S>
static int rk3(const Case& C, const Params<S>& P, S* U, double* T_io, double t, double dt, S* J) {
  const long long N = C.N();
  const long long M = N * (C.ns + 4);
  std::vector<S> U1(M), U2(M), L(M), h(N);
  const double b[3] = {1.0 / 6.0, 1.0 / 6.0, 2.0 / 3.0};
  const double tk[3] = {t, t + dt, t + 0.5 * dt};
  S jstep = 0;
  for (int stage = 0; stage < 3; ++stage) {
    const S* Uk = stage == 0 ? U : (stage == 1 ? U1.data() : U2.data());
    int err = rhs(C, P, Uk, T_io, tk[stage], L.data(), h.data(), (unsigned char*)nullptr, (Fields<S>*)nullptr);
    if (err) return err;
    S js = 0;
    for (long long q = 0; q < N; ++q) js += cell_volume(C, q) * h[q];
    jstep += b[stage] * js;
    for (long long q = 0; q < M; ++q) {
      if (stage == 0) U1[q] = U[q] + dt * L[q];
      else if (stage == 1) U2[q] = 0.75 * U[q] + 0.25 * (U1[q] + dt * L[q]);
      else U[q] = (1.0 / 3.0) * U[q] + (2.0 / 3.0) * (U2[q] + dt * L[q]);
    }
  }
  if (J) *J += dt * jstep;
  return OK;
}

}  // namespace orc

using namespace orc;

// ---------------------------------------------------------------- C entry points
extern "C" {

void* orc_case_new(int ns, int nr, const double* W, const double* a7, const double* sig, const double* epsk,
                   const double* lnA, const double* beta, const double* Ea, const int* nuf, const int* nur,
                   double Tmin, double Tmax, const int* n, const double* xnode, const double* xin,
                   const double* xif, const double* L, double theta_c, double psi_c, double CT, double cfl,
                   unsigned flags) {
  Case* C = new Case();
  C->ns = ns; C->nr = nr;
  C->W.assign(W, W + ns);
  C->a7.assign(a7, a7 + 7 * ns);
  C->sig.assign(sig, sig + ns);
  C->epsk.assign(epsk, epsk + ns);
  C->lnA.assign(lnA, lnA + nr);
  C->beta.assign(beta, beta + nr);
  C->Ea.assign(Ea, Ea + nr);
  C->nuf.assign(nuf, nuf + nr * ns);
  C->nur.assign(nur, nur + nr * ns);
  C->Tmin = Tmin; C->Tmax = Tmax;
  long long off = 0;
  for (int a = 0; a < 3; ++a) {
    C->n[a] = n[a];
    C->xnode[a].assign(xnode + off, xnode + off + n[a]);
    C->xin[a].assign(xin + off, xin + off + n[a]);
    C->xif[a].assign(xif + off, xif + off + n[a]);
    C->L[a] = L[a];
    off += n[a];
  }
  C->theta_c = theta_c; C->psi_c = psi_c; C->CT = CT; C->cfl = cfl; C->flags = flags;
  return C;
}

void orc_case_free(void* h) { delete (Case*)h; }

// Boundary conditions: bc[3][2] per axis and side (0 periodic, 1 no-slip
// isothermal wall, 2 inflow, 3 outflow; an axis periodic on both sides or
// bounded on both), pinf[3][2] and relax[3][2] the outflow's far-field
// pressure and relaxation coefficient.  A bounded axis needs at least 8
// nodes; curvilinear grids stay periodic.  Returns 1 (EINVAL) otherwise.
int orc_case_set_boundaries(void* h, const int* bc, const double* pinf, const double* relax) {
  Case& C = *(Case*)h;
  if (C.curv) return EINVAL;
  for (int a = 0; a < 3; ++a) {
    const int lo = bc[2 * a], hi = bc[2 * a + 1];
    if ((lo == BC_PERIODIC) != (hi == BC_PERIODIC)) return EINVAL;
    if (lo < 0 || lo > 3 || hi < 0 || hi > 3) return EINVAL;
    if (lo != BC_PERIODIC && C.n[a] < 8) return EINVAL;
    for (int side = 0; side < 2; ++side) {
      if (bc[2 * a + side] == BC_OUTFLOW && !(pinf[2 * a + side] > 0 && relax[2 * a + side] >= 0)) return EINVAL;
      C.bc[a][side] = bc[2 * a + side];
      C.pinf[a][side] = pinf[2 * a + side];
      C.relax[a][side] = relax[2 * a + side];
    }
  }
  return OK;
}

// Makes the case curvilinear: node coordinates xyz[3][N] and lattice periods
// P[3][3] (row a: the displacement along index a over n[a] cells).  An
// inactive axis must have its period along its own coordinate axis, and the
// other periods no component along it.  Returns 1 for an invalid lattice or
// a node with det(d x / d xi) <= 0.
int orc_case_set_curvilinear(void* h, const double* xyz, const double* P) {
  Case& C = *(Case*)h;
  for (int a = 0; a < 3; ++a)
    if (C.bounded(a)) return EINVAL;
  const long long N = C.N();
  for (int c = 0; c < 3; ++c) C.X[c].assign(xyz + c * N, xyz + (c + 1) * N);
  for (int a = 0; a < 3; ++a)
    for (int c = 0; c < 3; ++c) C.Pv[a][c] = P[3 * a + c];
  for (int a = 0; a < 3; ++a) {
    if (C.n[a] > 1) continue;
    for (int c = 0; c < 3; ++c)
      if (c != a && C.Pv[a][c] != 0.0) return EINVAL;
    for (int b = 0; b < 3; ++b)
      if (b != a && C.Pv[b][a] != 0.0) return EINVAL;
    if (!(C.Pv[a][a] != 0.0)) return EINVAL;
  }
  // inverse of the matrix whose columns are the periods (cofactors / det)
  double B[3][3];
  for (int r = 0; r < 3; ++r)
    for (int a = 0; a < 3; ++a) B[r][a] = C.Pv[a][r];
  double det = B[0][0] * (B[1][1] * B[2][2] - B[1][2] * B[2][1]) - B[0][1] * (B[1][0] * B[2][2] - B[1][2] * B[2][0]) +
               B[0][2] * (B[1][0] * B[2][1] - B[1][1] * B[2][0]);
  if (!(std::fabs(det) > 0)) return EINVAL;
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c) {
      const int r1 = (c + 1) % 3, r2 = (c + 2) % 3, c1 = (r + 1) % 3, c2 = (r + 2) % 3;
      C.Pinv[r][c] = (B[r1][c1] * B[r2][c2] - B[r1][c2] * B[r2][c1]) / det;
    }
  C.curv = true;
  return set_metrics(C);
}

// Node metric terms [9][N] ((d xi_d / d x_c) / J at row 3d + c), face metric
// terms [9][N], and J [N] of a curvilinear case.
void orc_metrics(void* h, double* mt, double* mf, double* jac) {
  const Case& C = *(Case*)h;
  const long long N = C.N();
  for (int r = 0; r < 9; ++r)
    for (long long q = 0; q < N; ++q) {
      mt[r * N + q] = C.mt[r][q];
      mf[r * N + q] = C.mf[r][q];
    }
  for (long long q = 0; q < N; ++q) jac[q] = C.Jac[q];
}

void orc_set_flags(void* h, unsigned flags) { ((Case*)h)->flags = flags; }

static Params<double> make_params(const Case& C, const double* las, const double* lnA) {
  Params<double> P;
  P.lnA.assign(lnA ? lnA : C.lnA.data(), (lnA ? lnA : C.lnA.data()) + C.nr);
  P.E = las[0]; P.xc[0] = las[1]; P.xc[1] = las[2]; P.xc[2] = las[3];
  P.sr = las[4]; P.t0 = las[5]; P.st = las[6]; P.on = las[7] != 0.0;
  return P;
}

// Conserved state from primitives (Y_s, T, p, u): rho from eq. (4); total
// energy includes the species enthalpies of formation.
int orc_prim_to_cons(void* h, const double* Y, const double* T, const double* p, const double* vel, double* U) {
  const Case& C = *(Case*)h;
  const long long N = C.N();
  const int ns = C.ns;
  for (long long q = 0; q < N; ++q) {
    double iW = 0;
    for (int s = 0; s < ns; ++s) iW += Y[s * N + q] / C.W[s];
    double rho = p[q] / (Ru * T[q] * iW);
    double hm = 0;
    for (int s = 0; s < ns; ++s) hm += Y[s * N + q] * (Ru / C.W[s]) * T[q] * h_RT(&C.a7[7 * s], T[q]);
    double ke = 0;
    for (int m = 0; m < 3; ++m) {
      U[(ns + m) * N + q] = rho * vel[m * N + q];
      ke += vel[m * N + q] * vel[m * N + q];
    }
    for (int s = 0; s < ns; ++s) U[s * N + q] = rho * Y[s * N + q];
    U[(ns + 3) * N + q] = rho * hm - p[q] + 0.5 * rho * ke;
  }
  return OK;
}

// Per-cell quantities, for per-step comparisons.  out layout [nq][N] with
// rows: T, p, c, mu, lambda, D_s (ns), wdot_s (ns), hrr, q_L, theta.
int orc_cells(void* h, const double* U, double* T_io, double t, const double* las, double* out) {
  const Case& C = *(Case*)h;
  Params<double> P = make_params(C, las, nullptr);
  Fields<double> F;
  int err = eval_cells(C, P, U, T_io, t, F);
  if (err) return err;
  const long long N = C.N();
  const int ns = C.ns;
  for (long long q = 0; q < N; ++q) {
    const Cell<double>& z = F.cell[q];
    int r = 0;
    out[(r++) * N + q] = z.T;
    out[(r++) * N + q] = z.p;
    out[(r++) * N + q] = z.c;
    out[(r++) * N + q] = z.mu;
    out[(r++) * N + q] = z.lam;
    for (int s = 0; s < ns; ++s) out[(r++) * N + q] = z.D[s];
    for (int s = 0; s < ns; ++s) out[(r++) * N + q] = (C.flags & CHEM_OFF) ? 0.0 : z.wdot[s];
    out[(r++) * N + q] = z.hrr;
    out[(r++) * N + q] = z.qL;
    out[(r++) * N + q] = F.theta[q];
  }
  return OK;
}

int orc_rhs(void* h, const double* U, double* T_io, double t, const double* las, double* dUdt, double* hrr,
            unsigned char* mask) {
  const Case& C = *(Case*)h;
  Params<double> P = make_params(C, las, nullptr);
  return rhs(C, P, U, T_io, t, dUdt, hrr, mask, (Fields<double>*)nullptr);
}

int orc_stable_dt(void* h, const double* U, double* T_io, double* dt) {
  return stable_dt(*(Case*)h, U, T_io, dt);
}

int orc_rk3_step(void* h, double* U, double* T_io, double t, double dt, const double* las, const double* lnA,
                 double* J) {
  const Case& C = *(Case*)h;
  Params<double> P = make_params(C, las, lnA);
  return rk3(C, P, U, T_io, t, dt, J);
}

// Forward-mode tangent of one RK3 step: (U, dU) -> (U', dU'), and (J, dJ),
// for parameter tangents dlas = (dE, dxc, dyc, dzc) and dlnA.
int orc_rk3_tangent(void* h, double* U, double* dU, double* T_io, double t, double dt, const double* las,
                    const double* dlas, const double* lnA, const double* dlnA, double* J, double* dJ) {
  const Case& C = *(Case*)h;
  const long long M = C.N() * (C.ns + 4);
  Params<Dual> P;
  P.lnA.resize(C.nr);
  for (int j = 0; j < C.nr; ++j) P.lnA[j] = Dual(lnA ? lnA[j] : C.lnA[j], dlnA ? dlnA[j] : 0.0);
  P.E = Dual(las[0], dlas[0]);
  for (int a = 0; a < 3; ++a) P.xc[a] = Dual(las[1 + a], dlas[1 + a]);
  P.sr = las[4]; P.t0 = las[5]; P.st = las[6]; P.on = las[7] != 0.0;
  std::vector<Dual> Ud(M);
  for (long long q = 0; q < M; ++q) Ud[q] = Dual(U[q], dU[q]);
  Dual Jd(J ? *J : 0.0, dJ ? *dJ : 0.0);
  int err = rk3(C, P, Ud.data(), T_io, t, dt, &Jd);
  if (err) return err;
  for (long long q = 0; q < M; ++q) { U[q] = Ud[q].v; dU[q] = Ud[q].d; }
  if (J) *J = Jd.v;
  if (dJ) *dJ = Jd.d;
  return OK;
}

// Tangent of one RHS evaluation (state and parameter directions).
int orc_rhs_tangent(void* h, const double* U, const double* dU, double* T_io, double t, const double* las,
                    const double* dlas, const double* dlnA, double* dUdt, double* ddUdt, double* hrr,
                    double* dhrr) {
  const Case& C = *(Case*)h;
  const long long N = C.N();
  const long long M = N * (C.ns + 4);
  Params<Dual> P;
  P.lnA.resize(C.nr);
  for (int j = 0; j < C.nr; ++j) P.lnA[j] = Dual(C.lnA[j], dlnA ? dlnA[j] : 0.0);
  P.E = Dual(las[0], dlas[0]);
  for (int a = 0; a < 3; ++a) P.xc[a] = Dual(las[1 + a], dlas[1 + a]);
  P.sr = las[4]; P.t0 = las[5]; P.st = las[6]; P.on = las[7] != 0.0;
  std::vector<Dual> Ud(M), L(M), hd(N);
  for (long long q = 0; q < M; ++q) Ud[q] = Dual(U[q], dU[q]);
  int err = rhs(C, P, Ud.data(), T_io, t, L.data(), hd.data(), (unsigned char*)nullptr, (Fields<Dual>*)nullptr);
  if (err) return err;
  for (long long q = 0; q < M; ++q) { dUdt[q] = L[q].v; ddUdt[q] = L[q].d; }
  for (long long q = 0; q < N; ++q) {
    if (hrr) hrr[q] = hd[q].v;
    if (dhrr) dhrr[q] = hd[q].d;
  }
  return OK;
}

// Building blocks exposed for the pins.
double orc_teno6(const double* f, double CT) { return teno6(f, CT); }
double orc_weno3z(const double* f) { return weno3z(f); }
// beta0..beta3, beta6, tau, chi0..chi3, omega0..omega3
double orc_teno6_detail(const double* f, double CT, double* detail) { return teno6(f, CT, detail); }
// c_p/R, h/(RT), s/R of species s at temperature T
void orc_thermo(void* h, int s, double T, double* out) {
  const Case& C = *(Case*)h;
  const double* a = &C.a7[7 * s];
  out[0] = cp_R(a, T);
  out[1] = h_RT(a, T);
  out[2] = s_R(a, T);
}
double orc_omega22(double Ts) { return omega22(Ts); }
double orc_omega11(double Ts) { return omega11(Ts); }
double orc_mu_species(void* h, int s, double T) { return mu_species(*(Case*)h, s, T); }
double orc_D_binary(void* h, int i, int j, double T, double p) { return D_binary(*(Case*)h, i, j, T, p); }
double orc_cell_volume(void* h, long long q) { return cell_volume(*(Case*)h, q); }

// Forward and backward rates of progress (mol m^-3 s^-1) of every reaction
// in every cell: out[(2 j + {0,1}) N + q].
int orc_rates(void* h, const double* U, double* T_io, double* out) {
  const Case& C = *(Case*)h;
  const long long N = C.N();
  const int nv = C.ns + 4;
  Params<double> P;
  P.lnA.assign(C.lnA.begin(), C.lnA.end());
  P.E = 0; P.xc[0] = P.xc[1] = P.xc[2] = 0; P.sr = 1; P.t0 = 0; P.st = 1; P.on = false;
  std::vector<double> r(2 * C.nr + 2);
  for (long long q = 0; q < N; ++q) {
    std::vector<double> Uc(nv);
    for (int v = 0; v < nv; ++v) Uc[v] = U[v * N + q];
    Cell<double> z;
    int e = primitives(C, Uc.data(), T_io[q], z);
    if (e) return e;
    T_io[q] = z.T;
    chemistry(C, P, Uc.data(), z, r.data());
    for (int k = 0; k < 2 * C.nr; ++k) out[k * N + q] = r[k];
  }
  return OK;
}

}  // extern "C"
