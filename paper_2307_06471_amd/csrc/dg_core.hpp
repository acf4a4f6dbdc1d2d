// dg_core.hpp -- device-side building blocks of the cRKDG step on gfx950.
//
// Discretisation (Chen, Sun, Xing, arXiv 2307.06471, Section 2): per cell a
// tensor Legendre basis phi_mn = P_m(xi) P_n(eta) (mode m + Q n, Q = K+1);
// the volume and face integrals of the DG operator (equation (DG operator))
// and of the local operator (equation (dxl)) use a Q-point Gauss rule per
// direction.  The Legendre mass matrix is diagonal, |K| / ((2m+1)(2n+1)), so
// every operator is an explicit per-cell contraction.
//
// Everything here is register resident and fully unrolled: the Gauss nodes
// and Legendre values are compile-time constants, so the contractions are
// FMA chains against immediate/SGPR constants with no table loads.  The
// contractions are sum-factorised one direction at a time ("per line of
// quadrature points"), which keeps the live register set at one line of
// nodal values instead of the whole cell.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace crk {

// keep the scheduler from interleaving independent quadrature lines: the
// work is one line of points at a time, which bounds the live registers
#ifndef CRK_NO_SCHED_FENCE
#define CRK_FENCE() __builtin_amdgcn_sched_barrier(0)
#else
#define CRK_FENCE()
#endif

// ---------------------------------------------------------------------------
// Gauss--Legendre rules on [-1, 1] (closed forms for n <= 5, tabulated for
// n = 6, computed at compile time for n >= 7)
// ---------------------------------------------------------------------------
// Legendre polynomials by Bonnet's recursion and derivatives by
// P'_{m+1} = (m+1) P_m + x P'_m
constexpr double leg(int m, double x) {
  double p0 = 1.0, p1 = x;
  if (m == 0) return p0;
  for (int j = 1; j < m; ++j) {
    double p2 = ((2 * j + 1) * x * p1 - j * p0) / (j + 1);
    p0 = p1;
    p1 = p2;
  }
  return p1;
}
constexpr double dleg(int m, double x) {
  double d = 0.0;
  for (int j = 0; j < m; ++j) d = (j + 1) * leg(j, x) + x * d;
  return d;
}

// a-th root (ascending) of P_n for n >= 7: the roots are simple and at least
// 2/n^2 apart, so a grid of 8 n^2 intervals brackets each one; bisection then
// halves the bracket until it holds no double between its ends
constexpr double gl_root(int n, int a) {
  const int cells = 8 * n * n;
  int seen = 0;
  double lo = -1.0, flo = leg(n, -1.0);
  for (int c = 1; c <= cells; ++c) {
    const double hi = -1.0 + 2.0 * c / cells, fhi = leg(n, hi);
    if ((flo < 0.0) != (fhi < 0.0)) {
      if (seen == a) {
        double l = lo, h = hi, fl = flo;
        for (int it = 0; it < 80; ++it) {
          const double m = 0.5 * (l + h);
          if (m <= l || m >= h) break;
          const double fm = leg(n, m);
          if ((fm < 0.0) == (fl < 0.0)) {
            l = m;
            fl = fm;
          } else {
            h = m;
          }
        }
        return 0.5 * (l + h);
      }
      ++seen;
    }
    lo = hi;
    flo = fhi;
  }
  return 0.0;
}
constexpr double gl_x(int n, int a) {
  switch (n) {
    case 1: return 0.0;
    case 2: { constexpr double r = 0.57735026918962576450914878050196; return a == 0 ? -r : r; }
    case 3: { constexpr double r = 0.77459666924148337703585307995648;
              return a == 0 ? -r : (a == 1 ? 0.0 : r); }
    case 4: { constexpr double r1 = 0.33998104358485626480266575910324,
                               r2 = 0.86113631159405257522394648889281;
              return a == 0 ? -r2 : a == 1 ? -r1 : a == 2 ? r1 : r2; }
    case 5: { constexpr double r1 = 0.53846931010568309103631442070021,
                               r2 = 0.90617984593866399279762687829939;
              return a == 0 ? -r2 : a == 1 ? -r1 : a == 2 ? 0.0 : a == 3 ? r1 : r2; }
    case 6: { constexpr double r1 = 0.23861918608319690863050172168071,
                               r2 = 0.66120938646626451366139959501991,
                               r3 = 0.93246951420315202781230155449399;
              return a == 0 ? -r3 : a == 1 ? -r2 : a == 2 ? -r1 : a == 3 ? r1 : a == 4 ? r2 : r3; }
    default: return gl_root(n, a);
  }
}
constexpr double gl_w(int n, int a) {
  switch (n) {
    case 1: return 2.0;
    case 2: return 1.0;
    case 3: return a == 1 ? 8.0 / 9.0 : 5.0 / 9.0;
    case 4: { constexpr double w1 = 0.65214515486254614262693605077800,
                               w2 = 0.34785484513745385737306394922200;
              return (a == 1 || a == 2) ? w1 : w2; }
    case 5: { constexpr double w0 = 0.56888888888888888888888888888889,
                               w1 = 0.47862867049936646804129151483564,
                               w2 = 0.23692688505618908751426404071992;
              return a == 2 ? w0 : (a == 1 || a == 3) ? w1 : w2; }
    case 6: { constexpr double w1 = 0.46791393457269104738987034398955,
                               w2 = 0.36076157304813860756983351383772,
                               w3 = 0.17132449237917034504029614217273;
              return (a == 2 || a == 3) ? w1 : (a == 1 || a == 4) ? w2 : w3; }
    default: {
      // w_a = 2 / ((1 - x_a^2) P_n'(x_a)^2)
      const double x = gl_root(n, a), d = dleg(n, x);
      return 2.0 / ((1.0 - x * x) * d * d);
    }
  }
}

// tables for one degree: P[m][a] = P_m(x_a), D[m][a] = P'_m(x_a), W[a]
template <int Q>
struct GTab {
  double P[Q][Q];
  double D[Q][Q];
  double W[Q];
  double X[Q];
};
template <int Q>
constexpr GTab<Q> make_tab() {
  GTab<Q> t{};
  for (int a = 0; a < Q; ++a) {
    t.X[a] = gl_x(Q, a);
    t.W[a] = gl_w(Q, a);
    for (int m = 0; m < Q; ++m) {
      t.P[m][a] = leg(m, t.X[a]);
      t.D[m][a] = dleg(m, t.X[a]);
    }
  }
  return t;
}
template <int Q>
struct Tab {
  static constexpr GTab<Q> t = make_tab<Q>();
};

constexpr double sgn_pow(int m) { return (m % 2) ? -1.0 : 1.0; }  // (-1)^m

// ---------------------------------------------------------------------------
// Equations (Section 2.1 conservation law; Euler fluxes of Section 4.1.2)
// ---------------------------------------------------------------------------
// reciprocal and square root in the compute precision: IEEE-rounded in FP64
// (the FP64 method), the hardware instructions (within 1 ulp) in the FP32-bulk
// form
__device__ __forceinline__ double rcp_r(double x) { return 1.0 / x; }
__device__ __forceinline__ float rcp_r(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double sqrt_r(double x) { return sqrt(x); }
__device__ __forceinline__ float sqrt_r(float x) { return __builtin_amdgcn_sqrtf(x); }

template <class R>
struct Euler2 {
  using Real = R;
  static constexpr int NC = 4, DIM = 2;
  static constexpr bool EULER = true, BURGERS = false;
  R gm1, gam;

  __device__ __forceinline__ void flux2(const R (&q)[4], R (&f)[4], R (&g)[4]) const {
    const R ir = rcp_r(q[0]);
    const R u = q[1] * ir, v = q[2] * ir;
    const R p = gm1 * (q[3] - R(0.5) * (q[1] * u + q[2] * v));
    const R e = q[3] + p;
    f[0] = q[1]; f[1] = q[1] * u + p; f[2] = q[1] * v; f[3] = e * u;
    g[0] = q[2]; g[1] = q[2] * u;     g[2] = q[2] * v + p; g[3] = e * v;
  }
  // normal flux f.e_D and spectral radius |u_D| + c
  template <int D>
  __device__ __forceinline__ void nflux(const R (&q)[4], R (&f)[4], R& lam) const {
    const R ir = rcp_r(q[0]);
    const R u = q[1] * ir, v = q[2] * ir;
    const R p = gm1 * (q[3] - R(0.5) * (q[1] * u + q[2] * v));
    const R un = D == 0 ? u : v;
    const R mn = D == 0 ? q[1] : q[2];
    f[0] = mn;
    f[1] = q[1] * un + (D == 0 ? p : R(0));
    f[2] = q[2] * un + (D == 1 ? p : R(0));
    f[3] = (q[3] + p) * un;
    lam = fabs(un) + sqrt_r(gam * p * ir);
  }
  template <int D>
  __device__ __forceinline__ void nflux_only(const R (&q)[4], R (&f)[4]) const {
    R lam;
    nflux<D>(q, f, lam);
  }
  // Lax--Friedrichs flux through a face in the +e_D direction; qL is the
  // trace of the cell on the negative side (Section 2.1), alpha = the larger
  // of the two traces' spectral radii at this point
  template <int D>
  __device__ __forceinline__ void num_flux(const R (&qL)[4], const R (&qR)[4], R (&F)[4]) const {
    R fL[4], fR[4], lL, lR;
    nflux<D>(qL, fL, lL);
    nflux<D>(qR, fR, lR);
    const R a = lL > lR ? lL : lR;
#pragma unroll
    for (int c = 0; c < 4; ++c) F[c] = R(0.5) * (fL[c] + fR[c] - a * (qR[c] - qL[c]));
  }
  // the same with the direction chosen at run time (d = 0: x, 1: y), no branch
  __device__ __forceinline__ void nflux_d(const R (&q)[4], bool dy, R (&f)[4], R& lam) const {
    const R ir = rcp_r(q[0]);
    const R u = q[1] * ir, v = q[2] * ir;
    const R p = gm1 * (q[3] - R(0.5) * (q[1] * u + q[2] * v));
    const R un = dy ? v : u;
    const R px = dy ? R(0) : p, py = dy ? p : R(0);
    f[0] = dy ? q[2] : q[1];
    f[1] = q[1] * un + px;
    f[2] = q[2] * un + py;
    f[3] = (q[3] + p) * un;
    lam = fabs(un) + sqrt_r(gam * p * ir);
  }
  __device__ __forceinline__ void num_flux_d(const R (&qL)[4], const R (&qR)[4], bool dy,
                                             R (&F)[4]) const {
    R fL[4], fR[4], lL, lR;
    nflux_d(qL, dy, fL, lL);
    nflux_d(qR, dy, fR, lR);
    const R a = lL > lR ? lL : lR;
#pragma unroll
    for (int c = 0; c < 4; ++c) F[c] = R(0.5) * (fL[c] + fR[c] - a * (qR[c] - qL[c]));
  }
};

template <class R, int DIM_>
struct Adv {
  using Real = R;
  static constexpr int NC = 1, DIM = DIM_;
  static constexpr bool EULER = false, BURGERS = false;
  R ax, ay;
  int upwind;

  __device__ __forceinline__ void flux2(const R (&q)[1], R (&f)[1], R (&g)[1]) const {
    f[0] = ax * q[0];
    g[0] = ay * q[0];
  }
  template <int D>
  __device__ __forceinline__ void nflux_only(const R (&q)[1], R (&f)[1]) const {
    f[0] = (D == 0 ? ax : ay) * q[0];
  }
  template <int D>
  __device__ __forceinline__ void num_flux(const R (&qL)[1], const R (&qR)[1], R (&F)[1]) const {
    const R a = D == 0 ? ax : ay;
    if (upwind)
      F[0] = a >= R(0) ? a * qL[0] : a * qR[0];
    else
      F[0] = R(0.5) * (a * qL[0] + a * qR[0] - fabs(a) * (qR[0] - qL[0]));
  }
  __device__ __forceinline__ void num_flux_d(const R (&qL)[1], const R (&qR)[1], bool dy,
                                             R (&F)[1]) const {
    const R a = dy ? ay : ax;
    if (upwind)
      F[0] = a >= R(0) ? a * qL[0] : a * qR[0];
    else
      F[0] = R(0.5) * (a * qL[0] + a * qR[0] - fabs(a) * (qR[0] - qL[0]));
  }
};

// Burgers' equation u_t + (u^2/2)_x = 0 in 1D (Section 4.1.1, example
// 'ex:1dburgers') with the Godunov flux: the flux of the exact Riemann
// solution at the face.  For the convex f(u) = u^2/2 and left/right traces
// a, b: a <= b (rarefaction, or a contact at a = b) gives f at the point of
// [a, b] closest to the sonic point 0; a > b (shock) gives the larger of
// f(a) and f(b), the upwind side of the shock.
template <class R>
struct Burgers1 {
  using Real = R;
  static constexpr int NC = 1, DIM = 1;
  static constexpr bool EULER = false, BURGERS = true;

  __device__ __forceinline__ static R godunov(R a, R b) {
    if (a <= b) {
      const R u = fmin(fmax(a, R(0)), b);
      return R(0.5) * u * u;
    }
    return R(0.5) * fmax(a * a, b * b);
  }
  __device__ __forceinline__ void flux2(const R (&q)[1], R (&f)[1], R (&g)[1]) const {
    f[0] = R(0.5) * q[0] * q[0];
    g[0] = R(0);
  }
  template <int D>
  __device__ __forceinline__ void nflux_only(const R (&q)[1], R (&f)[1]) const {
    f[0] = R(0.5) * q[0] * q[0];
  }
  template <int D>
  __device__ __forceinline__ void num_flux(const R (&qL)[1], const R (&qR)[1], R (&F)[1]) const {
    F[0] = godunov(qL[0], qR[0]);
  }
  __device__ __forceinline__ void num_flux_d(const R (&qL)[1], const R (&qR)[1], bool,
                                             R (&F)[1]) const {
    F[0] = godunov(qL[0], qR[0]);
  }
};

// ---------------------------------------------------------------------------
// Per-cell contractions.  U is a cell's modal state U[c][mode].
// ---------------------------------------------------------------------------
template <int K, int DIM>
struct Sizes {
  static constexpr int Q = K + 1;
  static constexpr int NB = DIM == 2 ? Q * Q : Q;
};

// acc += sx * Vx(U) + sy * Vy(U), the volume part of the operators:
//   Vx_mn = (2m+1)(2n+1) sum_ab w_a w_b f(U_ab) P'_m(x_a) P_n(x_b)
//   Vy_mn = (2m+1)(2n+1) sum_ab w_a w_b g(U_ab) P_m(x_a) P'_n(x_b)
// The operator's volume term is -Vx/(2dx) - Vy/(2dy) (2D), -Vx/dx (1D).
template <class EQ, int K, class R>
__device__ __forceinline__ void volume_acc(const EQ& eq,
                                           const R (&U)[EQ::NC][Sizes<K, EQ::DIM>::NB],
                                           R sx, R sy,
                                           R (&acc)[EQ::NC][Sizes<K, EQ::DIM>::NB]) {
  constexpr int Q = K + 1, NC = EQ::NC;
  constexpr GTab<Q> T = Tab<Q>::t;
  if constexpr (EQ::DIM == 1) {
#pragma unroll
    for (int a = 0; a < Q; ++a) {
      R q[NC];
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        R s = U[c][0];
#pragma unroll
        for (int m = 1; m < Q; ++m)
          if (T.P[m][a] != 0.0) s = s + U[c][m] * R(T.P[m][a]);
        q[c] = s;
      }
      R f[NC];
      eq.template nflux_only<0>(q, f);
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        const R fs = sx * f[c];
#pragma unroll
        for (int m = 1; m < Q; ++m) {
          const double cf = (2 * m + 1) * T.W[a] * T.D[m][a];
          if (cf != 0.0) acc[c][m] = acc[c][m] + R(cf) * fs;
        }
      }
    }
  } else {
#pragma unroll
    for (int a = 0; a < Q; ++a) {
      // t[c][n] = sum_m U[c][m + Q n] P_m(x_a)
      R t[NC][Q];
#pragma unroll
      for (int c = 0; c < NC; ++c)
#pragma unroll
        for (int n = 0; n < Q; ++n) {
          R s = U[c][Q * n];
#pragma unroll
          for (int m = 1; m < Q; ++m)
            if (T.P[m][a] != 0.0) s = s + U[c][m + Q * n] * R(T.P[m][a]);
          t[c][n] = s;
        }
      R rf[NC][Q], rg[NC][Q];
#pragma unroll
      for (int b = 0; b < Q; ++b) {
        R q[NC];
#pragma unroll
        for (int c = 0; c < NC; ++c) {
          R s = t[c][0];
#pragma unroll
          for (int n = 1; n < Q; ++n)
            if (T.P[n][b] != 0.0) s = s + t[c][n] * R(T.P[n][b]);
          q[c] = s;
        }
        R f[NC], g[NC];
        eq.flux2(q, f, g);
#pragma unroll
        for (int c = 0; c < NC; ++c)
#pragma unroll
          for (int n = 0; n < Q; ++n) {
            const double cf = T.W[b] * T.P[n][b];
            const double cg = T.W[b] * T.D[n][b];
            if (b == 0) {
              rf[c][n] = R(cf) * f[c];
              rg[c][n] = R(cg) * g[c];
            } else {
              if (cf != 0.0) rf[c][n] = rf[c][n] + R(cf) * f[c];
              if (cg != 0.0) rg[c][n] = rg[c][n] + R(cg) * g[c];
            }
          }
      }
#pragma unroll
      for (int c = 0; c < NC; ++c)
#pragma unroll
        for (int n = 0; n < Q; ++n) {
          const R rfs = sx * rf[c][n];
          const R rgs = sy * rg[c][n];
#pragma unroll
          for (int m = 0; m < Q; ++m) {
            const double c1 = (2 * m + 1) * (2 * n + 1) * T.W[a] * T.D[m][a];
            const double c2 = (2 * m + 1) * (2 * n + 1) * T.W[a] * T.P[m][a];
            R v = acc[c][m + Q * n];
            if (c1 != 0.0) v = v + R(c1) * rfs;
            if (c2 != 0.0 && n > 0) v = v + R(c2) * rgs;
            acc[c][m + Q * n] = v;
          }
        }
      CRK_FENCE();
    }
  }
}

// Face traces.  x-faces (xi = S, S = +1 right, -1 left) at the Q eta-points;
// y-faces (eta = S) at the Q xi-points.  1D: one value per component.
template <int S, class EQ, int K, class R>
__device__ __forceinline__ void trace_x(const R (&U)[EQ::NC][Sizes<K, EQ::DIM>::NB],
                                        R (&tr)[EQ::NC][EQ::DIM == 2 ? K + 1 : 1]) {
  constexpr int Q = K + 1, NC = EQ::NC;
  constexpr GTab<Q> T = Tab<Q>::t;
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    if constexpr (EQ::DIM == 1) {
      R s = U[c][0];
#pragma unroll
      for (int m = 1; m < Q; ++m) s = (S > 0 || m % 2 == 0) ? s + U[c][m] : s - U[c][m];
      tr[c][0] = s;
    } else {
      R e[Q];
#pragma unroll
      for (int n = 0; n < Q; ++n) {
        R s = U[c][Q * n];
#pragma unroll
        for (int m = 1; m < Q; ++m)
          s = (S > 0 || m % 2 == 0) ? s + U[c][m + Q * n] : s - U[c][m + Q * n];
        e[n] = s;
      }
#pragma unroll
      for (int b = 0; b < Q; ++b) {
        R s = e[0];
#pragma unroll
        for (int n = 1; n < Q; ++n)
          if (T.P[n][b] != 0.0) s = s + e[n] * R(T.P[n][b]);
        tr[c][b] = s;
      }
    }
  }
}

template <int S, class EQ, int K, class R>
__device__ __forceinline__ void trace_y(const R (&U)[EQ::NC][Sizes<K, 2>::NB],
                                        R (&tr)[EQ::NC][K + 1]) {
  constexpr int Q = K + 1, NC = EQ::NC;
  constexpr GTab<Q> T = Tab<Q>::t;
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    R e[Q];
#pragma unroll
    for (int m = 0; m < Q; ++m) {
      R s = U[c][m];
#pragma unroll
      for (int n = 1; n < Q; ++n)
        s = (S > 0 || n % 2 == 0) ? s + U[c][m + Q * n] : s - U[c][m + Q * n];
      e[m] = s;
    }
#pragma unroll
    for (int a = 0; a < Q; ++a) {
      R s = e[0];
#pragma unroll
      for (int m = 1; m < Q; ++m)
        if (T.P[m][a] != 0.0) s = s + e[m] * R(T.P[m][a]);
      tr[c][a] = s;
    }
  }
}

// acc += lx * Lx(FR, FL) with
//   Lx_mn = (2m+1)(2n+1) sum_b w_b P_n(x_b) (FR_b - (-1)^m FL_b)       (2D)
//   Lx_m  = (2m+1) (FR - (-1)^m FL)                                    (1D)
// FR/FL: flux through the right/left face in the +x direction.  The
// operator's face term is Lx/(2dx) (2D) or Lx/dx (1D).
template <class EQ, int K, class R>
__device__ __forceinline__ void lift_x(const R (&FR)[EQ::NC][EQ::DIM == 2 ? K + 1 : 1],
                                       const R (&FL)[EQ::NC][EQ::DIM == 2 ? K + 1 : 1], R lx,
                                       R (&acc)[EQ::NC][Sizes<K, EQ::DIM>::NB]) {
  constexpr int Q = K + 1, NC = EQ::NC;
  constexpr GTab<Q> T = Tab<Q>::t;
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    if constexpr (EQ::DIM == 1) {
      const R ar = lx * FR[c][0], al = lx * FL[c][0];
#pragma unroll
      for (int m = 0; m < Q; ++m)
        acc[c][m] = acc[c][m] + R(2 * m + 1) * (m % 2 ? ar + al : ar - al);
    } else {
#pragma unroll
      for (int n = 0; n < Q; ++n) {
        R ar = R(T.W[0] * T.P[n][0]) * FR[c][0];
        R al = R(T.W[0] * T.P[n][0]) * FL[c][0];
#pragma unroll
        for (int b = 1; b < Q; ++b) {
          const double cw = T.W[b] * T.P[n][b];
          if (cw != 0.0) {
            ar = ar + R(cw) * FR[c][b];
            al = al + R(cw) * FL[c][b];
          }
        }
        ar = lx * ar;
        al = lx * al;
        const R sp = ar - al, sm = ar + al;
#pragma unroll
        for (int m = 0; m < Q; ++m)
          acc[c][m + Q * n] = acc[c][m + Q * n] + R((2 * m + 1) * (2 * n + 1)) * (m % 2 ? sm : sp);
      }
    }
  }
}

// acc += ly * Ly(GT, GB), Ly_mn = (2m+1)(2n+1) sum_a w_a P_m(x_a)(GT_a - (-1)^n GB_a)
template <class EQ, int K, class R>
__device__ __forceinline__ void lift_y(const R (&GT)[EQ::NC][K + 1], const R (&GB)[EQ::NC][K + 1],
                                       R ly, R (&acc)[EQ::NC][Sizes<K, 2>::NB]) {
  constexpr int Q = K + 1, NC = EQ::NC;
  constexpr GTab<Q> T = Tab<Q>::t;
#pragma unroll
  for (int c = 0; c < NC; ++c)
#pragma unroll
    for (int m = 0; m < Q; ++m) {
      R at = R(T.W[0] * T.P[m][0]) * GT[c][0];
      R ab = R(T.W[0] * T.P[m][0]) * GB[c][0];
#pragma unroll
      for (int a = 1; a < Q; ++a) {
        const double cw = T.W[a] * T.P[m][a];
        if (cw != 0.0) {
          at = at + R(cw) * GT[c][a];
          ab = ab + R(cw) * GB[c][a];
        }
      }
      at = ly * at;
      ab = ly * ab;
      const R sp = at - ab, sm = at + ab;
#pragma unroll
      for (int n = 0; n < Q; ++n)
        acc[c][m + Q * n] = acc[c][m + Q * n] + R((2 * m + 1) * (2 * n + 1)) * (n % 2 ? sm : sp);
    }
}

// normal flux of the interior trace at every face point (local operator)
template <int D, class EQ, int NP, class R>
__device__ __forceinline__ void trace_flux(const EQ& eq, const R (&tr)[EQ::NC][NP],
                                           R (&F)[EQ::NC][NP]) {
#pragma unroll
  for (int p = 0; p < NP; ++p) {
    R q[EQ::NC], f[EQ::NC];
#pragma unroll
    for (int c = 0; c < EQ::NC; ++c) q[c] = tr[c][p];
    eq.template nflux_only<D>(q, f);
#pragma unroll
    for (int c = 0; c < EQ::NC; ++c) F[c][p] = f[c];
  }
}

// acc += scale * (the face part of loc(U)) in 2D: the cell's own traces'
// physical flux on its four faces, lifted (equation (dxl))
template <class EQ, int K, class R>
__device__ __forceinline__ void loc_face_acc2(const EQ& eq, const R (&U)[EQ::NC][Sizes<K, 2>::NB],
                                              R scale, R inv_dx, R inv_dy,
                                              R (&acc)[EQ::NC][Sizes<K, 2>::NB]) {
  constexpr int NP = K + 1;
  const R hx = R(0.5) * scale * inv_dx, hy = R(0.5) * scale * inv_dy;
  R t0[EQ::NC][NP], t1[EQ::NC][NP], F0[EQ::NC][NP], F1[EQ::NC][NP];
  trace_x<+1, EQ, K, R>(U, t0);
  trace_x<-1, EQ, K, R>(U, t1);
  trace_flux<0, EQ, NP, R>(eq, t0, F0);
  trace_flux<0, EQ, NP, R>(eq, t1, F1);
  lift_x<EQ, K, R>(F0, F1, hx, acc);
  CRK_FENCE();
  trace_y<+1, EQ, K, R>(U, t0);
  trace_y<-1, EQ, K, R>(U, t1);
  trace_flux<1, EQ, NP, R>(eq, t0, F0);
  trace_flux<1, EQ, NP, R>(eq, t1, F1);
  lift_y<EQ, K, R>(F0, F1, hy, acc);
  CRK_FENCE();
}

// acc += scale * loc(U), the local operator of equation (dxl):
// volume term plus the cell's own traces' physical flux on its faces.
template <class EQ, int K, class R>
__device__ __forceinline__ void loc_acc(const EQ& eq, const R (&U)[EQ::NC][Sizes<K, EQ::DIM>::NB],
                                        R scale, R inv_dx, R inv_dy,
                                        R (&acc)[EQ::NC][Sizes<K, EQ::DIM>::NB]) {
  constexpr int NP = EQ::DIM == 2 ? K + 1 : 1;
  if constexpr (EQ::DIM == 2) {
    const R hx = R(0.5) * scale * inv_dx, hy = R(0.5) * scale * inv_dy;
    volume_acc<EQ, K, R>(eq, U, -hx, -hy, acc);
    loc_face_acc2<EQ, K, R>(eq, U, scale, inv_dx, inv_dy, acc);
  } else {
    const R hx = scale * inv_dx;
    volume_acc<EQ, K, R>(eq, U, -hx, R(0), acc);
    R t0[EQ::NC][1], t1[EQ::NC][1], F0[EQ::NC][1], F1[EQ::NC][1];
    trace_x<+1, EQ, K, R>(U, t0);
    trace_x<-1, EQ, K, R>(U, t1);
    trace_flux<0, EQ, 1, R>(eq, t0, F0);
    trace_flux<0, EQ, 1, R>(eq, t1, F1);
    lift_x<EQ, K, R>(F0, F1, hx, acc);
  }
}

}  // namespace crk
