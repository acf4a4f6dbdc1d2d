/*
 * crkdg_oracle.c -- serial FP64 CPU oracle of the compact RKDG method
 * (Chen, Sun, Xing, arXiv 2307.06471).
 *
 * TEST INFRASTRUCTURE ONLY: loaded by the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark, never by the product path.  Shares no
 * code with the HIP library.  Plain loops, FP64, no sum factorisation, built
 * with -ffp-contract=off.  See crkdg_oracle.h for the layout.
 */
#include "crkdg_oracle.h"

#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_MAXQ 8      /* largest Gauss rule used (k+3 with k <= 5) */
#define OR_MAXC 4      /* components */
#define OR_MAXB 36     /* modes: (k+1)^2 with k <= 5 */

/* ------------------------------------------------------------------ */
/* Tables                                                               */
/* ------------------------------------------------------------------ */

/* Legendre polynomial by the three-term recurrence
 * (m+1) P_{m+1} = (2m+1) x P_m - m P_{m-1}. */
double or_legendre(int m, double x) {
  if (m == 0) return 1.0;
  double pm1 = 1.0, p = x;
  for (int j = 1; j < m; ++j) {
    double pn = ((2.0 * j + 1.0) * x * p - j * pm1) / (j + 1.0);
    pm1 = p;
    p = pn;
  }
  return p;
}

/* derivative via P'_{m} = m P_{m-1} + x P'_{m-1} */
double or_dlegendre(int m, double x) {
  double d = 0.0;
  for (int j = 1; j <= m; ++j) d = j * or_legendre(j - 1, x) + x * d;
  return d;
}

/* n-point Gauss--Legendre rule on [-1,1] by Newton iteration on P_n,
 * weights 2 / ((1 - x^2) P_n'(x)^2).  Nodes returned in increasing order. */
int or_gauss(int n, double* x, double* w) {
  if (n < 1 || n > 16) return -1;
  for (int i = 0; i < n; ++i) {
    double z = cos(M_PI * (i + 0.75) / (n + 0.5));
    for (int it = 0; it < 100; ++it) {
      double dz = or_legendre(n, z) / or_dlegendre(n, z);
      z -= dz;
      if (fabs(dz) < 1e-16) break;
    }
    double d = or_dlegendre(n, z);
    x[n - 1 - i] = z;
    w[n - 1 - i] = 2.0 / ((1.0 - z * z) * d * d);
  }
  return 0;
}

int or_ncomp(const or_mesh* m) {
  if (m->equation == OR_EQ_ADVECTION || m->equation == OR_EQ_BURGERS) return 1;
  return m->dim + 2;
}

int or_nmodes(const or_mesh* m, int k) {
  return m->dim == 2 ? (k + 1) * (k + 1) : (k + 1);
}

static int ncells(const or_mesh* m) { return m->nx * (m->dim == 2 ? m->ny : 1); }
static double cdx(const or_mesh* m) { return (m->x1 - m->x0) / m->nx; }
static double cdy(const or_mesh* m) { return m->dim == 2 ? (m->y1 - m->y0) / m->ny : 1.0; }

/* basis function phi_mode(xi, eta) = P_m(xi) P_n(eta), mode = m + (k+1) n */
static double phi(const or_mesh* m, int k, int mode, double xi, double eta) {
  if (m->dim == 1) return or_legendre(mode, xi);
  int mm = mode % (k + 1), nn = mode / (k + 1);
  return or_legendre(mm, xi) * or_legendre(nn, eta);
}
static double dphi_dxi(const or_mesh* m, int k, int mode, double xi, double eta) {
  if (m->dim == 1) return or_dlegendre(mode, xi);
  int mm = mode % (k + 1), nn = mode / (k + 1);
  return or_dlegendre(mm, xi) * or_legendre(nn, eta);
}
static double dphi_deta(const or_mesh* m, int k, int mode, double xi, double eta) {
  int mm = mode % (k + 1), nn = mode / (k + 1);
  return or_legendre(mm, xi) * or_dlegendre(nn, eta);
}
/* diagonal Legendre mass: int_K phi^2 = |K| / prod (2 m_d + 1) */
static double mass(const or_mesh* m, int k, int mode) {
  double area = cdx(m) * cdy(m);
  if (m->dim == 1) return area / (2.0 * mode + 1.0);
  int mm = mode % (k + 1), nn = mode / (k + 1);
  return area / ((2.0 * mm + 1.0) * (2.0 * nn + 1.0));
}

/* state value of one cell at reference point (xi, eta) */
static void eval_state(const or_mesh* m, int k, const double* u, int cell, double xi,
                       double eta, double* q) {
  int nc = or_ncomp(m), nb = or_nmodes(m, k), N = ncells(m);
  for (int c = 0; c < nc; ++c) {
    double s = 0.0;
    for (int b = 0; b < nb; ++b) s += u[(c * nb + b) * N + cell] * phi(m, k, b, xi, eta);
    q[c] = s;
  }
}

/* ------------------------------------------------------------------ */
/* Physics: conservation law (Section 2.1) and 1D/2D Euler fluxes      */
/* (Sections 4.1.1 and 4.1.2)                                           */
/* ------------------------------------------------------------------ */

static double pressure(const or_mesh* m, const double* q) {
  double g = m->gamma;
  if (m->dim == 1) return (g - 1.0) * (q[2] - 0.5 * q[1] * q[1] / q[0]);
  return (g - 1.0) * (q[3] - 0.5 * (q[1] * q[1] + q[2] * q[2]) / q[0]);
}

/* physical flux in direction d (0: x, 1: y) */
static void phys_flux(const or_mesh* m, const double* q, int d, double* f) {
  if (m->equation == OR_EQ_ADVECTION) {
    f[0] = m->adv[d] * q[0];
    return;
  }
  if (m->equation == OR_EQ_BURGERS) { /* Section 4.1.1, example 'ex:1dburgers' */
    f[0] = 0.5 * q[0] * q[0];
    return;
  }
  double p = pressure(m, q);
  if (m->dim == 1) {
    double w = q[1] / q[0];
    f[0] = q[1];
    f[1] = q[1] * w + p;
    f[2] = w * (q[2] + p);
    return;
  }
  double u = q[1] / q[0], v = q[2] / q[0];
  if (d == 0) {
    f[0] = q[1];
    f[1] = q[1] * u + p;
    f[2] = q[1] * v;
    f[3] = u * (q[3] + p);
  } else {
    f[0] = q[2];
    f[1] = q[2] * u;
    f[2] = q[2] * v + p;
    f[3] = v * (q[3] + p);
  }
}

/* largest |eigenvalue| of d f_d / d u */
static double spectral_radius(const or_mesh* m, const double* q, int d) {
  if (m->equation == OR_EQ_ADVECTION) return fabs(m->adv[d]);
  if (m->equation == OR_EQ_BURGERS) return fabs(q[0]);
  double p = pressure(m, q);
  double c = sqrt(m->gamma * p / q[0]);
  return fabs(q[1 + d] / q[0]) + c;
}

/* Godunov flux of Burgers' equation (Section 4.1.1, example 'ex:1dburgers')
 * between the left trace a and the right trace b: the exact Riemann solution
 * at the face.  For the convex flux f(u) = u^2/2 that is the minimum of f over
 * [a, b] when a <= b, the maximum of f(a), f(b) when a > b. */
static double godunov_burgers(double a, double b) {
  double fa = 0.5 * a * a, fb = 0.5 * b * b;
  if (a <= b) {
    if (a >= 0.0) return fa;
    if (b <= 0.0) return fb;
    return 0.0; /* the sonic point u = 0 lies in [a, b] */
  }
  return fa > fb ? fa : fb;
}

/* numerical flux f^ . nu on a face with outward normal nu = s e_d (s = +-1),
 * interior trace qi, exterior trace qe.  Lax--Friedrichs (Section 2.1) with
 * alpha the pointwise larger spectral radius of the two traces; the upwind
 * flux for linear advection; the Godunov flux for Burgers' equation. */
static void num_flux(const or_mesh* m, const double* qi, const double* qe, int d, double s,
                     double* F) {
  int nc = or_ncomp(m);
  if (m->flux == OR_FLUX_UPWIND && m->equation == OR_EQ_ADVECTION) {
    double an = s * m->adv[d];
    F[0] = an >= 0.0 ? an * qi[0] : an * qe[0];
    return;
  }
  if (m->flux == OR_FLUX_GODUNOV) {
    /* the left state of the face (in +x) is the interior one when nu = +e_x */
    F[0] = s > 0.0 ? godunov_burgers(qi[0], qe[0]) : -godunov_burgers(qe[0], qi[0]);
    return;
  }
  double fi[OR_MAXC], fe[OR_MAXC];
  phys_flux(m, qi, d, fi);
  phys_flux(m, qe, d, fe);
  double ai = spectral_radius(m, qi, d), ae = spectral_radius(m, qe, d);
  double alpha = ai > ae ? ai : ae;
  for (int c = 0; c < nc; ++c) F[c] = 0.5 * (s * fi[c] + s * fe[c] - alpha * (qe[c] - qi[c]));
}

/* ------------------------------------------------------------------ */
/* Initial conditions / exact solutions (Section 4 examples and the     */
/* synthetic shock workloads)                                            */
/* ------------------------------------------------------------------ */

static void prim_to_cons(const or_mesh* m, double rho, double u, double v, double p,
                         double* q) {
  double g = m->gamma;
  if (m->dim == 1) {
    q[0] = rho;
    q[1] = rho * u;
    q[2] = p / (g - 1.0) + 0.5 * rho * u * u;
  } else {
    q[0] = rho;
    q[1] = rho * u;
    q[2] = rho * v;
    q[3] = p / (g - 1.0) + 0.5 * rho * (u * u + v * v);
  }
}

static double wrap_centered(double d, double period) {
  /* map d into [-period/2, period/2) */
  double r = fmod(d + 0.5 * period, period);
  if (r < 0) r += period;
  return r - 0.5 * period;
}

/* Double Mach reflection (Section 4, example "Double Mach reflection"): a
 * Mach 10 shock moving to the right into gas at rest, (rho, p) = (1.4, 1),
 * through (1/6, 0) at 60 degrees to the x-axis; the reflecting wall occupies
 * the bottom side from x = 1/6 on.  The paper fixes these settings and
 * leaves the states to the classical test (Woodward--Colella); the
 * post-shock state follows from the Rankine--Hugoniot conditions. */
#define DMR_XWALL (1.0 / 6.0)
#define DMR_MACH 10.0
#define DMR_ANGLE (M_PI / 3.0)

/* pre- and post-shock conserved states and the shock speed.  In the frame
 * of the shock the gas enters with speed w1 = S and leaves with w2:
 * mass rho1 w1 = rho2 w2, momentum p1 + rho1 w1^2 = p2 + rho2 w2^2, energy
 * h1 + w1^2/2 = h2 + w2^2/2 with h = gamma p / ((gamma - 1) rho).  For a
 * shock of Mach number M = S / c1 these give the density ratio
 * (gamma + 1) M^2 / ((gamma - 1) M^2 + 2); the momentum balance then gives
 * p2, and the gas behind the shock moves with S - w2 along the normal. */
void or_dmr_states(double gamma, double pre[4], double post[4], double* shock_speed) {
  double rho1 = 1.4, p1 = 1.0;
  double c1 = sqrt(gamma * p1 / rho1);
  double S = DMR_MACH * c1;
  double ratio = (gamma + 1.0) * DMR_MACH * DMR_MACH /
                 ((gamma - 1.0) * DMR_MACH * DMR_MACH + 2.0);
  double rho2 = rho1 * ratio;
  double w1 = S, w2 = S / ratio;
  double p2 = p1 + rho1 * w1 * w1 - rho2 * w2 * w2;
  double un = S - w2;
  /* the shock normal points into the gas at rest: (sin 60, -cos 60) */
  double nx = sin(DMR_ANGLE), ny = -cos(DMR_ANGLE);
  double u2 = un * nx, v2 = un * ny;
  pre[0] = rho1; pre[1] = 0.0; pre[2] = 0.0; pre[3] = p1 / (gamma - 1.0);
  post[0] = rho2; post[1] = rho2 * u2; post[2] = rho2 * v2;
  post[3] = p2 / (gamma - 1.0) + 0.5 * rho2 * (u2 * u2 + v2 * v2);
  if (shock_speed) *shock_speed = S;
}

static void exact_state(const or_mesh* m, int ic, const double* P, const double* aux,
                        double x, double y, double t, double* q) {
  int nc = or_ncomp(m);
  switch (ic) {
    case OR_IC_CONST:
      for (int c = 0; c < nc; ++c) q[c] = P[c];
      return;
    case OR_IC_ADV_SIN:
    case OR_IC_ADV_SIN_1D_SHIFT:
      if (m->dim == 1)
        q[0] = sin(x - m->adv[0] * t);
      else
        q[0] = sin(M_PI * (x - m->adv[0] * t)) * sin(M_PI * (y - m->adv[1] * t));
      return;
    case OR_IC_EULER_WAVE: {
      double u = P[0], v = P[1], p = P[2];
      if (m->dim == 1) {
        double rho = 1.0 + 0.2 * sin(M_PI * (x - u * t));
        prim_to_cons(m, rho, u, 0.0, p, q);
      } else {
        double rho = 1.0 + 0.2 * sin(M_PI * (x + y - (u + v) * t));
        prim_to_cons(m, rho, u, v, p, q);
      }
      return;
    }
    case OR_IC_VORTEX: {
      /* isentropic vortex on a uniform (1,1,1,1) flow, translated by (t, t) */
      double eps = P[0], xc = P[1], yc = P[2], Lx = P[3], Ly = P[4];
      double g = m->gamma;
      double xb = wrap_centered(x - xc - t, Lx), yb = wrap_centered(y - yc - t, Ly);
      double r2 = xb * xb + yb * yb;
      double e = exp(0.5 * (1.0 - r2));
      double du = -eps / (2.0 * M_PI) * e * yb, dv = eps / (2.0 * M_PI) * e * xb;
      double T = 1.0 - (g - 1.0) * eps * eps / (8.0 * g * M_PI * M_PI) * exp(1.0 - r2);
      double rho = pow(T, 1.0 / (g - 1.0));
      prim_to_cons(m, rho, 1.0 + du, 1.0 + dv, rho * T, q);
      return;
    }
    case OR_IC_QUADRANT: {
      double xs = P[0], ys = P[1];
      int quad = (x >= xs) ? ((y >= ys) ? 0 : 3) : ((y >= ys) ? 1 : 2); /* NE NW SW SE */
      const double* s = P + 2 + 4 * quad;
      prim_to_cons(m, s[0], s[1], s[2], s[3], q);
      return;
    }
    case OR_IC_SHOCK: {
      double th = P[0], rs = P[1], uns = P[2], ps = P[3], xs = P[4], ys = P[5];
      double rfloor = P[6], amp = P[7];
      double nxv = cos(th), nyv = sin(th);
      if (nxv * (x - xs) + nyv * (y - ys) < 0.0) {
        prim_to_cons(m, rs, uns * nxv, uns * nyv, ps, q);
        return;
      }
      /* bilinear interpolation of a cell-centre field given on an na x ma
       * grid over the domain (P[8], P[9]; 0 means the mesh's cells),
       * periodic wrap */
      int na = P[8] > 0.0 ? (int)P[8] : m->nx, ma = P[9] > 0.0 ? (int)P[9] : m->ny;
      double hx = (m->x1 - m->x0) / na, hy = (m->y1 - m->y0) / ma;
      double sx = (x - m->x0) / hx - 0.5, sy = (y - m->y0) / hy - 0.5;
      double fx = floor(sx), fy = floor(sy);
      double ax = sx - fx, ay = sy - fy;
      int i0 = ((int)fx % na + na) % na, j0 = ((int)fy % ma + ma) % ma;
      int i1 = (i0 + 1) % na, j1 = (j0 + 1) % ma;
      double xi = (1 - ax) * (1 - ay) * aux[j0 * na + i0] + ax * (1 - ay) * aux[j0 * na + i1] +
                  (1 - ax) * ay * aux[j1 * na + i0] + ax * ay * aux[j1 * na + i1];
      double rho = 1.0 + amp * xi;
      if (rho < rfloor) rho = rfloor;
      prim_to_cons(m, rho, 0.0, 0.0, 1.0, q);
      return;
    }
    case OR_IC_DMR: {
      /* the planar shock at time t: it has moved S t along its normal */
      double pre[4], post[4], S;
      or_dmr_states(m->gamma, pre, post, &S);
      double nx = sin(DMR_ANGLE), ny = -cos(DMR_ANGLE);
      double behind = nx * (x - DMR_XWALL) + ny * y < S * t;
      for (int c = 0; c < nc; ++c) q[c] = behind ? post[c] : pre[c];
      return;
    }
    case OR_IC_BURGERS_SIN: {
      /* characteristics: u(x, t) = u0(x - u t) with u0 = sin.  g(u) = u -
       * sin(x - u t) has g' = 1 + t cos(x - u t) >= 1 - t > 0 for t < 1, so
       * Newton's method from u = sin(x) converges; iterate to a fixed point */
      double u = sin(x);
      for (int it = 0; it < 100; ++it) {
        double g = u - sin(x - u * t), dg = 1.0 + t * cos(x - u * t);
        double un = u - g / dg;
        if (un == u) break;
        u = un;
      }
      q[0] = u;
      return;
    }
    default:
      for (int c = 0; c < nc; ++c) q[c] = NAN;
  }
}

/* L2 projection with a (k+3)-point Gauss rule per direction */
int or_project(const or_mesh* m, int k, int ic, const double* params, const double* aux,
               double t, double* u) {
  int nc = or_ncomp(m), nb = or_nmodes(m, k), N = ncells(m);
  int Q = k + 3;
  double xg[OR_MAXQ], wg[OR_MAXQ];
  if (or_gauss(Q, xg, wg)) return -1;
  double hx = cdx(m), hy = cdy(m);
  int Qy = m->dim == 2 ? Q : 1;
  for (int cell = 0; cell < N; ++cell) {
    int i = cell % m->nx, j = cell / m->nx;
    double xc = m->x0 + (i + 0.5) * hx;
    double yc = m->dim == 2 ? m->y0 + (j + 0.5) * hy : 0.0;
    double acc[OR_MAXC][OR_MAXB];
    memset(acc, 0, sizeof acc);
    for (int a = 0; a < Q; ++a)
      for (int bq = 0; bq < Qy; ++bq) {
        double xi = xg[a], eta = m->dim == 2 ? xg[bq] : 0.0;
        double wq = wg[a] * (m->dim == 2 ? wg[bq] : 1.0) * (hx * hy) / (m->dim == 2 ? 4.0 : 2.0);
        double q[OR_MAXC];
        exact_state(m, ic, params, aux, xc + 0.5 * hx * xi, yc + 0.5 * hy * eta, t, q);
        for (int b = 0; b < nb; ++b)
          for (int c = 0; c < nc; ++c) acc[c][b] += wq * q[c] * phi(m, k, b, xi, eta);
      }
    for (int c = 0; c < nc; ++c)
      for (int b = 0; b < nb; ++b) u[(c * nb + b) * N + cell] = acc[c][b] / mass(m, k, b);
  }
  return 0;
}

/* ------------------------------------------------------------------ */
/* Spatial operators: (DG operator) of Section 2.1 and (dxl) of        */
/* Section 2.2.  Integrals by a (k+1)-point Gauss rule per direction in */
/* the volume and on each face.                                          */
/* ------------------------------------------------------------------ */

/* exterior trace at a face point: neighbour value, or the ghost rule of
 * the boundary condition on that side */
static void exterior_trace(const or_mesh* m, int k, const double* u, int i, int j, int d,
                           int s, double xi, double eta, double t_bc, const double* qi,
                           double* qe) {
  int nc = or_ncomp(m);
  int ni = i, nj = j;
  int side;
  if (d == 0) { ni += s; side = s < 0 ? 0 : 1; }
  else        { nj += s; side = s < 0 ? 2 : 3; }
  int nyc = m->dim == 2 ? m->ny : 1;
  int outside = (d == 0) ? (ni < 0 || ni >= m->nx) : (nj < 0 || nj >= nyc);
  if (outside) {
    int bc = m->bc[side];
    if (bc == OR_BC_PERIODIC) {
      if (d == 0) ni = (ni + m->nx) % m->nx;
      else nj = (nj + nyc) % nyc;
    } else if (bc == OR_BC_TRANSMISSIVE) {
      for (int c = 0; c < nc; ++c) qe[c] = qi[c];
      return;
    } else {
      if (m->bc_exact > 0) {
        double hx = cdx(m), hy = cdy(m);
        double x = m->x0 + (i + 0.5) * hx + 0.5 * hx * xi;
        double y = m->dim == 2 ? m->y0 + (j + 0.5) * hy + 0.5 * hy * eta : 0.0;
        if (m->bc_exact == OR_IC_DMR && side == 2 && x >= DMR_XWALL) {
          /* reflecting wall: the interior trace with its normal momentum
           * mirrored */
          for (int c = 0; c < nc; ++c) qe[c] = qi[c];
          qe[2] = -qi[2];
          return;
        }
        exact_state(m, m->bc_exact, m->ic_params, NULL, x, y, t_bc, qe);
      } else {
        for (int c = 0; c < nc; ++c) qe[c] = m->bc_state[side][c];
      }
      return;
    }
  }
  /* the neighbour's trace at the same physical point: its reference
   * coordinate along d is the mirror of ours */
  double nxi = d == 0 ? -xi : xi, neta = d == 1 ? -eta : eta;
  eval_state(m, k, u, nj * m->nx + ni, nxi, neta, qe);
}

/* basis values tabulated at the points one operator application uses */
typedef struct {
  int Q, nvol, nfp;
  double vphi[OR_MAXQ * OR_MAXQ][OR_MAXB];   /* phi at volume points */
  double vdx[OR_MAXQ * OR_MAXQ][OR_MAXB];    /* d phi / d xi */
  double vdy[OR_MAXQ * OR_MAXQ][OR_MAXB];    /* d phi / d eta */
  double vxi[OR_MAXQ * OR_MAXQ], veta[OR_MAXQ * OR_MAXQ], vw[OR_MAXQ * OR_MAXQ];
  double fphi[2][2][OR_MAXQ][OR_MAXB];       /* [d][side: 0 for -1, 1 for +1][point] */
  double fxi[2][2][OR_MAXQ], feta[2][2][OR_MAXQ], fw[OR_MAXQ];
} basis_tab;

static void tabulate(const or_mesh* m, int k, basis_tab* T) {
  int Q = k + 1, dim = m->dim, nb = or_nmodes(m, k);
  double xg[OR_MAXQ], wg[OR_MAXQ];
  or_gauss(Q, xg, wg);
  T->Q = Q;
  T->nvol = dim == 2 ? Q * Q : Q;
  T->nfp = dim == 2 ? Q : 1;
  for (int a = 0; a < Q; ++a)
    for (int bq = 0; bq < (dim == 2 ? Q : 1); ++bq) {
      int p = a + Q * bq;
      double xi = xg[a], eta = dim == 2 ? xg[bq] : 0.0;
      T->vxi[p] = xi;
      T->veta[p] = eta;
      T->vw[p] = wg[a] * (dim == 2 ? wg[bq] : 1.0);
      for (int b = 0; b < nb; ++b) {
        T->vphi[p][b] = phi(m, k, b, xi, eta);
        T->vdx[p][b] = dphi_dxi(m, k, b, xi, eta);
        T->vdy[p][b] = dim == 2 ? dphi_deta(m, k, b, xi, eta) : 0.0;
      }
    }
  for (int d = 0; d < dim; ++d)
    for (int si = 0; si < 2; ++si)
      for (int p = 0; p < T->nfp; ++p) {
        double s = si ? 1.0 : -1.0;
        double xi = dim == 1 ? s : (d == 0 ? s : xg[p]);
        double eta = dim == 1 ? 0.0 : (d == 0 ? xg[p] : s);
        T->fxi[d][si][p] = xi;
        T->feta[d][si][p] = eta;
        for (int b = 0; b < nb; ++b) T->fphi[d][si][p][b] = phi(m, k, b, xi, eta);
      }
  for (int p = 0; p < T->nfp; ++p) T->fw[p] = dim == 2 ? wg[p] : 1.0;
}

static void eval_tab(const or_mesh* m, int k, const double* u, int cell, const double* ph,
                     double* q) {
  int nc = or_ncomp(m), nb = or_nmodes(m, k), N = ncells(m);
  for (int c = 0; c < nc; ++c) {
    double s = 0.0;
    for (int b = 0; b < nb; ++b) s += u[(c * nb + b) * N + cell] * ph[b];
    q[c] = s;
  }
}

int or_apply(const or_mesh* m, int k, int op, double t_bc, const double* u, double* out) {
  int nc = or_ncomp(m), nb = or_nmodes(m, k), N = ncells(m);
  if (k < 0 || k > 5 || nb > OR_MAXB) return -1;
  if (m->equation == OR_EQ_EULER && m->flux == OR_FLUX_UPWIND) return -2;
  if ((m->flux == OR_FLUX_GODUNOV) != (m->equation == OR_EQ_BURGERS) ||
      (m->equation == OR_EQ_BURGERS && m->dim != 1))
    return -2;
  basis_tab* T = (basis_tab*)malloc(sizeof(basis_tab));
  if (!T) return -1;
  tabulate(m, k, T);
  double hx = cdx(m), hy = cdy(m);
  double area = hx * hy;
  int dim = m->dim;
  int nyc = dim == 2 ? m->ny : 1;
  for (int cell = 0; cell < N; ++cell) {
    int i = cell % m->nx, j = cell / m->nx;
    double acc[OR_MAXC][OR_MAXB];
    memset(acc, 0, sizeof acc);
    /* volume term: - int_K f(u) . grad(phi) */
    for (int p = 0; p < T->nvol; ++p) {
      double wq = T->vw[p] * area / (dim == 2 ? 4.0 : 2.0);
      double q[OR_MAXC], fx[OR_MAXC], fy[OR_MAXC];
      eval_tab(m, k, u, cell, T->vphi[p], q);
      phys_flux(m, q, 0, fx);
      if (dim == 2) phys_flux(m, q, 1, fy);
      for (int b = 0; b < nb; ++b) {
        double gx = T->vdx[p][b] * (2.0 / hx);
        double gy = dim == 2 ? T->vdy[p][b] * (2.0 / hy) : 0.0;
        for (int c = 0; c < nc; ++c)
          acc[c][b] -= wq * (fx[c] * gx + (dim == 2 ? fy[c] * gy : 0.0));
      }
    }
    /* face terms: + sum_e int_e (flux . nu) phi, outward normal nu = s e_d */
    for (int d = 0; d < dim; ++d)
      for (int si = 0; si < 2; ++si) {
        int s = si ? 1 : -1;
        for (int p = 0; p < T->nfp; ++p) {
          double wf = T->fw[p] * (dim == 1 ? 1.0 : 0.5 * (d == 0 ? hy : hx));
          double xi = T->fxi[d][si][p], eta = T->feta[d][si][p];
          double qi[OR_MAXC], F[OR_MAXC];
          eval_tab(m, k, u, cell, T->fphi[d][si][p], qi);
          if (op == OR_OP_LOC) {
            double f[OR_MAXC];
            phys_flux(m, qi, d, f);
            for (int c = 0; c < nc; ++c) F[c] = s * f[c];
          } else {
            double qe[OR_MAXC];
            int ni = i + (d == 0 ? s : 0), nj = j + (d == 1 ? s : 0);
            int inside = ni >= 0 && ni < m->nx && nj >= 0 && nj < nyc;
            int side = d == 0 ? si : 2 + si;
            if (inside || m->bc[side] == OR_BC_PERIODIC) {
              ni = (ni + m->nx) % m->nx;
              nj = (nj + nyc) % nyc;
              /* the neighbour's trace at the same physical point lies on its
               * opposite face, same tangential coordinate */
              eval_tab(m, k, u, nj * m->nx + ni, T->fphi[d][1 - si][p], qe);
            } else {
              exterior_trace(m, k, u, i, j, d, s, xi, eta, t_bc, qi, qe);
            }
            num_flux(m, qi, qe, d, (double)s, F);
          }
          for (int b = 0; b < nb; ++b) {
            double ph = T->fphi[d][si][p][b];
            for (int c = 0; c < nc; ++c) acc[c][b] += wf * F[c] * ph;
          }
        }
      }
    for (int c = 0; c < nc; ++c)
      for (int b = 0; b < nb; ++b) out[(c * nb + b) * N + cell] = acc[c][b] / mass(m, k, b);
  }
  free(T);
  return 0;
}

/* ------------------------------------------------------------------ */
/* Time stepping                                                         */
/* ------------------------------------------------------------------ */

static size_t state_len(const or_mesh* m, int k) {
  return (size_t)or_ncomp(m) * or_nmodes(m, k) * ncells(m);
}

/* stage states of the cRKDG scheme, equation (crkdg) of Section 2.2:
 * u^(1) = u^n, u^(i) = u^n - dt sum_{j<i} a_ij loc(u^(j)) */
int or_crkdg_stages(const or_mesh* m, int k, int s, const double* A, const double* b,
                    const double* c, double t, double dt, const double* u, double* stages) {
  (void)b; (void)c; (void)t;
  size_t n = state_len(m, k);
  double* L = (double*)malloc(sizeof(double) * n * (s > 1 ? s - 1 : 1));
  if (!L) return -1;
  memcpy(stages, u, sizeof(double) * n);
  for (int i = 1; i < s; ++i) {
    int rc = or_apply(m, k, OR_OP_LOC, 0.0, stages + (size_t)(i - 1) * n, L + (size_t)(i - 1) * n);
    if (rc) { free(L); return rc; }
    double* ui = stages + (size_t)i * n;
    for (size_t e = 0; e < n; ++e) {
      double acc = 0.0;
      for (int jj = 0; jj < i; ++jj) acc += A[i * s + jj] * L[(size_t)jj * n + e];
      ui[e] = u[e] - dt * acc;
    }
  }
  free(L);
  return 0;
}

/* one cRKDG step (Section 2.2, equation (crkdg)): inner stages with the local
 * operator, final stage u^{n+1} = u^n - dt sum_i b_i DG(u^(i)) with the
 * boundary data of stage i at time t + c_i dt (Section 3.4). */
int or_step_crkdg(const or_mesh* m, int k, int s, const double* A, const double* b,
                  const double* c, double t, double dt, double* u) {
  size_t n = state_len(m, k);
  double* st = (double*)malloc(sizeof(double) * n * s);
  double* D = (double*)malloc(sizeof(double) * n);
  double* un = (double*)malloc(sizeof(double) * n);
  if (!st || !D || !un) { free(st); free(D); free(un); return -1; }
  int rc = or_crkdg_stages(m, k, s, A, b, c, t, dt, u, st);
  memcpy(un, u, sizeof(double) * n);
  double* acc = (double*)calloc(n, sizeof(double));
  for (int i = 0; i < s && !rc; ++i) {
    if (b[i] == 0.0) continue;
    rc = or_apply(m, k, OR_OP_DG, t + c[i] * dt, st + (size_t)i * n, D);
    for (size_t e = 0; e < n; ++e) acc[e] += b[i] * D[e];
  }
  if (!rc)
    for (size_t e = 0; e < n; ++e) u[e] = un[e] - dt * acc[e];
  free(st); free(D); free(un); free(acc);
  return rc;
}

/* original RKDG in Butcher form, Section 2.1, equation (rkdg) */
int or_step_rkdg(const or_mesh* m, int k, int s, const double* A, const double* b,
                 const double* c, double t, double dt, double* u) {
  size_t n = state_len(m, k);
  double* Ls = (double*)malloc(sizeof(double) * n * s);
  double* ui = (double*)malloc(sizeof(double) * n);
  if (!Ls || !ui) { free(Ls); free(ui); return -1; }
  int rc = 0;
  for (int i = 0; i < s && !rc; ++i) {
    for (size_t e = 0; e < n; ++e) {
      double acc = 0.0;
      for (int jj = 0; jj < i; ++jj) acc += A[i * s + jj] * Ls[(size_t)jj * n + e];
      ui[e] = u[e] - dt * acc;
    }
    rc = or_apply(m, k, OR_OP_DG, t + c[i] * dt, ui, Ls + (size_t)i * n);
  }
  if (!rc)
    for (size_t e = 0; e < n; ++e) {
      double acc = 0.0;
      for (int i = 0; i < s; ++i) acc += b[i] * Ls[(size_t)i * n + e];
      u[e] -= dt * acc;
    }
  free(Ls); free(ui);
  return rc;
}

/* original RKDG with the SSP-RK2/3 Shu--Osher forms (convex combinations of
 * forward-Euler steps, Section 3.2.1), limiter after every stage if M >= 0 */
int or_step_rkdg_ssp(const or_mesh* m, int k, int order, double t, double dt, double M,
                     double* u) {
  size_t n = state_len(m, k);
  double* u0 = (double*)malloc(sizeof(double) * n);
  double* u1 = (double*)malloc(sizeof(double) * n);
  double* D = (double*)malloc(sizeof(double) * n);
  if (!u0 || !u1 || !D) { free(u0); free(u1); free(D); return -1; }
  memcpy(u0, u, sizeof(double) * n);
  /* each stage is limited with boundary data at the time it approximates:
   * t + dt, then (order 3) t + dt/2, then t + dt */
  int rc = or_apply(m, k, OR_OP_DG, t, u0, D);
  for (size_t e = 0; e < n; ++e) u1[e] = u0[e] - dt * D[e];
  if (M >= 0.0 && or_limit_tvb_at(m, k, M, t + dt, u1, NULL) < 0) rc = -3;
  if (order == 2) {
    rc = rc ? rc : or_apply(m, k, OR_OP_DG, t + dt, u1, D);
    for (size_t e = 0; e < n; ++e) u[e] = 0.5 * u0[e] + 0.5 * (u1[e] - dt * D[e]);
  } else {
    rc = rc ? rc : or_apply(m, k, OR_OP_DG, t + dt, u1, D);
    for (size_t e = 0; e < n; ++e) u1[e] = 0.75 * u0[e] + 0.25 * (u1[e] - dt * D[e]);
    if (M >= 0.0 && or_limit_tvb_at(m, k, M, t + 0.5 * dt, u1, NULL) < 0) rc = -3;
    rc = rc ? rc : or_apply(m, k, OR_OP_DG, t + 0.5 * dt, u1, D);
    for (size_t e = 0; e < n; ++e) u[e] = u0[e] / 3.0 + 2.0 / 3.0 * (u1[e] - dt * D[e]);
  }
  if (!rc && M >= 0.0 && or_limit_tvb_at(m, k, M, t + dt, u, NULL) < 0) rc = -3;
  free(u0); free(u1); free(D);
  return rc;
}

/* the Shu--Osher form with the local operator substituted for the DG
 * operator in the inner stages, equation (ssprk2) of Section 3.2.1 and its
 * third-order analogue (Section 4.1.1, Euler example) */
int or_step_wrong_ssp(const or_mesh* m, int k, int order, double t, double dt, double* u) {
  (void)t;
  size_t n = state_len(m, k);
  double* u0 = (double*)malloc(sizeof(double) * n);
  double* u1 = (double*)malloc(sizeof(double) * n);
  double* D = (double*)malloc(sizeof(double) * n);
  if (!u0 || !u1 || !D) { free(u0); free(u1); free(D); return -1; }
  memcpy(u0, u, sizeof(double) * n);
  int rc = or_apply(m, k, OR_OP_LOC, t, u0, D);
  for (size_t e = 0; e < n; ++e) u1[e] = u0[e] - dt * D[e];
  if (order == 2) {
    rc = rc ? rc : or_apply(m, k, OR_OP_DG, t + dt, u1, D);
    for (size_t e = 0; e < n; ++e) u[e] = 0.5 * u0[e] + 0.5 * (u1[e] - dt * D[e]);
  } else {
    rc = rc ? rc : or_apply(m, k, OR_OP_LOC, t + dt, u1, D);
    for (size_t e = 0; e < n; ++e) u1[e] = 0.75 * u0[e] + 0.25 * (u1[e] - dt * D[e]);
    rc = rc ? rc : or_apply(m, k, OR_OP_DG, t + 0.5 * dt, u1, D);
    for (size_t e = 0; e < n; ++e) u[e] = u0[e] / 3.0 + 2.0 / 3.0 * (u1[e] - dt * D[e]);
  }
  free(u0); free(u1); free(D);
  return rc;
}

/* ------------------------------------------------------------------ */
/* TVB minmod limiter, applied once per step after the final stage      */
/* (Section 2.2 remark on limiters; Section 4.2).  The paper defers the  */
/* details to its reference [rkdg5]; the reading used here:              */
/*  - per direction d, forward / backward trace-average jumps            */
/*    a = sum_{m>=1} u_{m0},  a~ = sum_{m>=1} (-1)^{m+1} u_{m0}           */
/*  - differences of neighbouring cell averages D+ and D-                */
/*  - Euler: characteristic variables with the left eigenvectors of the  */
/*    flux Jacobian in direction d at the cell average                   */
/*  - modified minmod: a if |a| <= M h_d^2, else minmod(a, D+, D-)         */
/*  - troubled if any modified minmod changes its first argument         */
/*  - troubled cells: limited P1 slopes, every other non-mean mode = 0    */
/* ------------------------------------------------------------------ */

static double minmod3(double a, double b, double c) {
  int sa = (a > 0) - (a < 0), sb = (b > 0) - (b < 0), sc = (c > 0) - (c < 0);
  if (sa != 0 && sa == sb && sa == sc) {
    double mn = fabs(a);
    if (fabs(b) < mn) mn = fabs(b);
    if (fabs(c) < mn) mn = fabs(c);
    return sa * mn;
  }
  return 0.0;
}

static double tvb_minmod(double a, double b, double c, double Mh2) {
  if (fabs(a) <= Mh2) return a;
  return minmod3(a, b, c);
}

/* distance of the modified-minmod decision from a tie: the TVB threshold,
 * a sign change of a nonzero argument, or |a| against |b|, |c|.  An argument
 * that is exactly zero is a difference of identical cell averages and stays
 * exactly zero under any rounding of the characteristic projection, so it
 * is not a tie. */
static double margin_of(double a, double b, double c, double Mh2) {
  double r = fabs(fabs(a) - Mh2);
  if (fabs(a) > Mh2) {
    double t[5] = {fabs(a), fabs(b), fabs(c), fabs(fabs(a) - fabs(b)), fabs(fabs(a) - fabs(c))};
    for (int i = 0; i < 5; ++i)
      if (t[i] != 0.0 && t[i] < r) r = t[i];
  }
  return r;
}

int or_euler_eig(const or_mesh* m, const double* q, int d, double* L, double* R) {
  double g = m->gamma;
  double rho = q[0];
  double p = pressure(m, q);
  double c = sqrt(g * p / rho);
  double b1 = (g - 1.0) / (c * c);
  if (m->dim == 1) {
    double w = q[1] / rho, H = (q[2] + p) / rho;
    double b2 = 0.5 * b1 * w * w;
    double Rm[9] = {1.0, 1.0, 1.0, w - c, w, w + c, H - w * c, 0.5 * w * w, H + w * c};
    double Lm[9] = {0.5 * (b2 + w / c), -0.5 * (b1 * w + 1.0 / c), 0.5 * b1,
                    1.0 - b2, b1 * w, -b1,
                    0.5 * (b2 - w / c), -0.5 * (b1 * w - 1.0 / c), 0.5 * b1};
    memcpy(R, Rm, sizeof Rm);
    memcpy(L, Lm, sizeof Lm);
    return 0;
  }
  double u = q[1] / rho, v = q[2] / rho, H = (q[3] + p) / rho;
  double q2 = u * u + v * v;
  double b2 = 0.5 * b1 * q2;
  if (d == 0) {
    /* R columns: u-c, u (entropy), u (shear), u+c ; stored row-major R[r*4+col] */
    double Rm[16] = {1.0, 1.0, 0.0, 1.0,
                     u - c, u, 0.0, u + c,
                     v, v, 1.0, v,
                     H - u * c, 0.5 * q2, v, H + u * c};
    double Lm[16] = {0.5 * (b2 + u / c), -0.5 * (b1 * u + 1.0 / c), -0.5 * b1 * v, 0.5 * b1,
                     1.0 - b2, b1 * u, b1 * v, -b1,
                     -v, 0.0, 1.0, 0.0,
                     0.5 * (b2 - u / c), -0.5 * (b1 * u - 1.0 / c), -0.5 * b1 * v, 0.5 * b1};
    memcpy(R, Rm, sizeof Rm);
    memcpy(L, Lm, sizeof Lm);
  } else {
    double Rm[16] = {1.0, 1.0, 0.0, 1.0,
                     u, u, 1.0, u,
                     v - c, v, 0.0, v + c,
                     H - v * c, 0.5 * q2, u, H + v * c};
    double Lm[16] = {0.5 * (b2 + v / c), -0.5 * b1 * u, -0.5 * (b1 * v + 1.0 / c), 0.5 * b1,
                     1.0 - b2, b1 * u, b1 * v, -b1,
                     -u, 1.0, 0.0, 0.0,
                     0.5 * (b2 - v / c), -0.5 * b1 * u, -0.5 * (b1 * v - 1.0 / c), 0.5 * b1};
    memcpy(R, Rm, sizeof Rm);
    memcpy(L, Lm, sizeof Lm);
  }
  return 0;
}

/* cell average of a neighbour across side (d, s), with the ghost rule; t is
 * the time of boundary data that depend on it (double Mach reflection) */
static void neighbour_avg(const or_mesh* m, int k, const double* u, int i, int j, int d, int s,
                          double t, double* qa) {
  int nc = or_ncomp(m), nb = or_nmodes(m, k), N = ncells(m);
  int nyc = m->dim == 2 ? m->ny : 1;
  int ni = i + (d == 0 ? s : 0), nj = j + (d == 1 ? s : 0);
  int side = d == 0 ? (s < 0 ? 0 : 1) : (s < 0 ? 2 : 3);
  int outside = (d == 0) ? (ni < 0 || ni >= m->nx) : (nj < 0 || nj >= nyc);
  if (outside) {
    int bc = m->bc[side];
    if (bc == OR_BC_PERIODIC) {
      ni = (ni + m->nx) % m->nx;
      nj = (nj + nyc) % nyc;
    } else if (bc == OR_BC_TRANSMISSIVE) {
      ni = i; nj = j;
    } else if (m->bc_exact == OR_IC_DMR) {
      /* the ghost cell's centre, mirrored across the boundary */
      double hx = cdx(m), hy = cdy(m);
      double xg = m->x0 + (ni + 0.5) * hx, yg = m->y0 + (nj + 0.5) * hy;
      if (side == 2 && m->x0 + (i + 0.5) * hx >= DMR_XWALL) {
        for (int c = 0; c < nc; ++c) qa[c] = u[(c * nb + 0) * N + j * m->nx + i];
        qa[2] = -qa[2];  /* reflecting wall: normal momentum mirrored */
      } else {
        exact_state(m, OR_IC_DMR, NULL, NULL, xg, yg, t, qa);
      }
      return;
    } else {
      for (int c = 0; c < nc; ++c) qa[c] = m->bc_state[side][c];
      return;
    }
  }
  for (int c = 0; c < nc; ++c) qa[c] = u[(c * nb + 0) * N + nj * m->nx + ni];
}

static int mode_index(const or_mesh* m, int k, int d, int deg) {
  if (m->dim == 1) return deg;
  return d == 0 ? deg : deg * (k + 1);
}

/* the troubled-cell test for one cell; returns 1 if troubled */
static int tvb_test(const or_mesh* m, int k, double M, double t, const double* u, int cell,
                    double* margin) {
  int nc = or_ncomp(m), nb = or_nmodes(m, k), N = ncells(m);
  int i = cell % m->nx, j = cell / m->nx;
  int troubled = 0;
  double mg = INFINITY;
  for (int d = 0; d < m->dim; ++d) {
    double h = d == 0 ? cdx(m) : cdy(m);
    double Mh2 = M * h * h;
    double a[OR_MAXC], at[OR_MAXC], dp[OR_MAXC], dm[OR_MAXC], qb[OR_MAXC], qn[OR_MAXC];
    for (int c = 0; c < nc; ++c) {
      qb[c] = u[(c * nb) * N + cell];
      a[c] = 0.0;
      at[c] = 0.0;
      for (int deg = 1; deg <= k; ++deg) {
        double v = u[(c * nb + mode_index(m, k, d, deg)) * N + cell];
        a[c] += v;
        at[c] += (deg % 2 == 1) ? v : -v;
      }
    }
    neighbour_avg(m, k, u, i, j, d, +1, t, qn);
    for (int c = 0; c < nc; ++c) dp[c] = qn[c] - qb[c];
    neighbour_avg(m, k, u, i, j, d, -1, t, qn);
    for (int c = 0; c < nc; ++c) dm[c] = qb[c] - qn[c];
    if (m->equation == OR_EQ_EULER) {
      double L[16], R[16], ca[OR_MAXC], cat[OR_MAXC], cp[OR_MAXC], cm[OR_MAXC];
      or_euler_eig(m, qb, d, L, R);
      for (int r = 0; r < nc; ++r) {
        ca[r] = cat[r] = cp[r] = cm[r] = 0.0;
        for (int c = 0; c < nc; ++c) {
          ca[r] += L[r * nc + c] * a[c];
          cat[r] += L[r * nc + c] * at[c];
          cp[r] += L[r * nc + c] * dp[c];
          cm[r] += L[r * nc + c] * dm[c];
        }
      }
      memcpy(a, ca, sizeof ca); memcpy(at, cat, sizeof cat);
      memcpy(dp, cp, sizeof cp); memcpy(dm, cm, sizeof cm);
    }
    for (int r = 0; r < nc; ++r) {
      if (tvb_minmod(a[r], dp[r], dm[r], Mh2) != a[r]) troubled = 1;
      if (tvb_minmod(at[r], dp[r], dm[r], Mh2) != at[r]) troubled = 1;
      double m1 = margin_of(a[r], dp[r], dm[r], Mh2), m2 = margin_of(at[r], dp[r], dm[r], Mh2);
      if (m1 < mg) mg = m1;
      if (m2 < mg) mg = m2;
    }
  }
  if (margin) *margin = mg;
  return troubled;
}

/* limited P1 reconstruction of one cell, reading u0 (pre-limiting) and
 * writing into u; keeps the mean */
static void tvb_reconstruct(const or_mesh* m, int k, double M, double t, const double* u0,
                            double* u, int cell) {
  int nc = or_ncomp(m), nb = or_nmodes(m, k), N = ncells(m);
  int i = cell % m->nx, j = cell / m->nx;
  double newslope[2][OR_MAXC];
  for (int d = 0; d < m->dim; ++d) {
    double h = d == 0 ? cdx(m) : cdy(m);
    double Mh2 = M * h * h;
    int sm = mode_index(m, k, d, 1);
    double sl[OR_MAXC], dp[OR_MAXC], dm[OR_MAXC], qb[OR_MAXC], qn[OR_MAXC];
    for (int c = 0; c < nc; ++c) {
      qb[c] = u0[(c * nb) * N + cell];
      sl[c] = u0[(c * nb + sm) * N + cell];
    }
    neighbour_avg(m, k, u0, i, j, d, +1, t, qn);
    for (int c = 0; c < nc; ++c) dp[c] = qn[c] - qb[c];
    neighbour_avg(m, k, u0, i, j, d, -1, t, qn);
    for (int c = 0; c < nc; ++c) dm[c] = qb[c] - qn[c];
    if (m->equation == OR_EQ_EULER) {
      double L[16], R[16], cs[OR_MAXC], lim[OR_MAXC];
      or_euler_eig(m, qb, d, L, R);
      for (int r = 0; r < nc; ++r) {
        double s1 = 0, s2 = 0, s3 = 0;
        for (int c = 0; c < nc; ++c) {
          s1 += L[r * nc + c] * sl[c];
          s2 += L[r * nc + c] * dp[c];
          s3 += L[r * nc + c] * dm[c];
        }
        cs[r] = s1;
        lim[r] = tvb_minmod(s1, s2, s3, Mh2);
      }
      (void)cs;
      for (int c = 0; c < nc; ++c) {
        double s = 0;
        for (int r = 0; r < nc; ++r) s += R[c * nc + r] * lim[r];
        newslope[d][c] = s;
      }
    } else {
      for (int c = 0; c < nc; ++c) newslope[d][c] = tvb_minmod(sl[c], dp[c], dm[c], Mh2);
    }
  }
  for (int c = 0; c < nc; ++c)
    for (int b = 1; b < nb; ++b) u[(c * nb + b) * N + cell] = 0.0;
  for (int d = 0; d < m->dim; ++d) {
    int sm = mode_index(m, k, d, 1);
    for (int c = 0; c < nc; ++c) u[(c * nb + sm) * N + cell] = newslope[d][c];
  }
}

/* positivity of density and pressure at the operator's volume and face
 * Gauss points (a safeguard, not part of the paper) */
static int physical_at_points(const or_mesh* m, int k, const double* u, int cell) {
  int Q = k + 1;
  double xg[OR_MAXQ], wg[OR_MAXQ];
  or_gauss(Q, xg, wg);
  int dim = m->dim;
  int Qy = dim == 2 ? Q : 1;
  double q[OR_MAXC];
  for (int a = 0; a < Q; ++a)
    for (int b = 0; b < Qy; ++b) {
      eval_state(m, k, u, cell, xg[a], dim == 2 ? xg[b] : 0.0, q);
      double p = pressure(m, q);
      if (!(q[0] > 0.0) || !(p > 0.0)) return 0;
    }
  for (int s = -1; s <= 1; s += 2)
    for (int p = 0; p < (dim == 2 ? Q : 1); ++p) {
      eval_state(m, k, u, cell, (double)s, dim == 2 ? xg[p] : 0.0, q);
      if (!(q[0] > 0.0) || !(pressure(m, q) > 0.0)) return 0;
      if (dim == 2) {
        eval_state(m, k, u, cell, xg[p], (double)s, q);
        if (!(q[0] > 0.0) || !(pressure(m, q) > 0.0)) return 0;
      }
    }
  return 1;
}

int64_t or_tvb_flags_at(const or_mesh* m, int k, double M, double t, const double* u,
                        uint8_t* flags, double* margin) {
  int N = ncells(m);
  int64_t n = 0;
  for (int cell = 0; cell < N; ++cell) {
    double mg = INFINITY;
    int tr = k >= 1 ? tvb_test(m, k, M, t, u, cell, &mg) : 0;
    if (flags) flags[cell] = (uint8_t)tr;
    if (margin) margin[cell] = mg;
    n += tr;
  }
  return n;
}

int64_t or_tvb_flags(const or_mesh* m, int k, double M, const double* u, uint8_t* flags,
                     double* margin) {
  return or_tvb_flags_at(m, k, M, 0.0, u, flags, margin);
}

int64_t or_limit_tvb(const or_mesh* m, int k, double M, double* u, uint8_t* flags) {
  return or_limit_tvb_at(m, k, M, 0.0, u, flags);
}

int64_t or_limit_tvb_at(const or_mesh* m, int k, double M, double t, double* u, uint8_t* flags) {
  int N = ncells(m), nc = or_ncomp(m), nb = or_nmodes(m, k);
  size_t n = state_len(m, k);
  double* u0 = (double*)malloc(sizeof(double) * n);
  if (!u0) return -1;
  memcpy(u0, u, sizeof(double) * n);
  int64_t count = 0;
  int bad = 0;
  for (int cell = 0; cell < N; ++cell) {
    uint8_t fl = 0;
    int cbad = 0;
    if (m->equation == OR_EQ_EULER) {
      double qb[OR_MAXC];
      for (int c = 0; c < nc; ++c) qb[c] = u0[(c * nb) * N + cell];
      cbad = !(qb[0] > 0.0) || !(pressure(m, qb) > 0.0);
      bad |= cbad;
    }
    if (k >= 1 && !cbad && tvb_test(m, k, M, t, u0, cell, NULL)) {
      tvb_reconstruct(m, k, M, t, u0, u, cell);
      fl |= 1;
    }
    if (m->equation == OR_EQ_EULER && !cbad && k >= 1 && !physical_at_points(m, k, u, cell)) {
      if (!(fl & 1)) tvb_reconstruct(m, k, M, t, u0, u, cell);
      fl |= 2;
      if (!physical_at_points(m, k, u, cell)) {
        for (int c = 0; c < nc; ++c)
          for (int b = 1; b < nb; ++b) u[(c * nb + b) * N + cell] = 0.0;
        fl |= 4;
      }
    }
    if (flags) flags[cell] = fl;
    count += fl != 0;
  }
  free(u0);
  return bad ? -1 : count;
}

/* ------------------------------------------------------------------ */
/* Diagnostics                                                           */
/* ------------------------------------------------------------------ */

double or_max_wavespeed(const or_mesh* m, int k, const double* u) {
  int nc = or_ncomp(m), nb = or_nmodes(m, k), N = ncells(m);
  double hx = cdx(m), hy = cdy(m), smax = 0.0;
  for (int cell = 0; cell < N; ++cell) {
    double q[OR_MAXC];
    for (int c = 0; c < nc; ++c) q[c] = u[(c * nb) * N + cell];
    double s = spectral_radius(m, q, 0) / hx;
    if (m->dim == 2) s += spectral_radius(m, q, 1) / hy;
    if (!(s <= smax)) smax = s; /* propagates NaN */
  }
  return smax;
}

/* L1, L2 (unnormalised integrals) and Linf errors of component comp against
 * an exact solution, with a (k+3)-point Gauss rule per direction */
int or_errors(const or_mesh* m, int k, const double* u, int ic, const double* params,
              const double* aux, double t, int comp, double out[3]) {
  int N = ncells(m), Q = k + 3, dim = m->dim;
  double xg[OR_MAXQ], wg[OR_MAXQ];
  or_gauss(Q, xg, wg);
  double hx = cdx(m), hy = cdy(m);
  double l1 = 0, l2 = 0, li = 0;
  int Qy = dim == 2 ? Q : 1;
  for (int cell = 0; cell < N; ++cell) {
    int i = cell % m->nx, j = cell / m->nx;
    double xc = m->x0 + (i + 0.5) * hx, yc = dim == 2 ? m->y0 + (j + 0.5) * hy : 0.0;
    for (int a = 0; a < Q; ++a)
      for (int b = 0; b < Qy; ++b) {
        double xi = xg[a], eta = dim == 2 ? xg[b] : 0.0;
        double wq = wg[a] * (dim == 2 ? wg[b] : 1.0) * hx * hy / (dim == 2 ? 4.0 : 2.0);
        double qh[OR_MAXC], qe[OR_MAXC];
        eval_state(m, k, u, cell, xi, eta, qh);
        exact_state(m, ic, params, aux, xc + 0.5 * hx * xi, yc + 0.5 * hy * eta, t, qe);
        double e = qh[comp] - qe[comp];
        l1 += wq * fabs(e);
        l2 += wq * e * e;
        if (fabs(e) > li) li = fabs(e);
      }
  }
  out[0] = l1;
  out[1] = sqrt(l2);
  out[2] = li;
  return 0;
}

int or_errors_vs_avg(const or_mesh* m, int k, const double* u, const double* ref, int comp,
                     double out[3]) {
  int N = ncells(m), nb = or_nmodes(m, k);
  double area = cdx(m) * cdy(m), l1 = 0, l2 = 0, li = 0;
  for (int cell = 0; cell < N; ++cell) {
    double e = u[(comp * nb) * N + cell] - ref[cell];
    l1 += area * fabs(e);
    l2 += area * e * e;
    if (fabs(e) > li) li = fabs(e);
  }
  out[0] = l1;
  out[1] = sqrt(l2);
  out[2] = li;
  return 0;
}

double or_total_mass(const or_mesh* m, int k, const double* u, int comp) {
  int N = ncells(m), nb = or_nmodes(m, k);
  double area = cdx(m) * cdy(m), s = 0.0;
  for (int cell = 0; cell < N; ++cell) s += area * u[(comp * nb) * N + cell];
  return s;
}

/* ------------------------------------------------------------------ */
/* Learned troubled-cell indicator (not in the paper)                   */
/* ------------------------------------------------------------------ */

int or_mlp_features(const or_mesh* m, int k, double M, const double* u, double* X) {
  int N = ncells(m), nb = or_nmodes(m, k), nc = or_ncomp(m);
  if (m->dim != 2 || m->equation != OR_EQ_EULER) return -1;
  int comps[2] = {0, nc - 1};
  for (int cell = 0; cell < N; ++cell) {
    int i = cell % m->nx, j = cell / m->nx;
    for (int qi = 0; qi < 2; ++qi) {
      int c = comps[qi];
      for (int d = 0; d < 2; ++d) {
        double h = d == 0 ? cdx(m) : cdy(m);
        double a = 0.0, at = 0.0;
        for (int deg = 1; deg <= k; ++deg) {
          double v = u[(c * nb + mode_index(m, k, d, deg)) * N + cell];
          a += v;
          at += (deg % 2 == 1) ? v : -v;
        }
        double qn[OR_MAXC], qb = u[(c * nb) * N + cell];
        neighbour_avg(m, k, u, i, j, d, +1, 0.0, qn);
        double dp = qn[c] - qb;
        neighbour_avg(m, k, u, i, j, d, -1, 0.0, qn);
        double dm = qb - qn[c];
        double s = fabs(dp) + fabs(dm) + M * h * h + 1e-300;
        double* x = X + (size_t)cell * 12 + (qi * 2 + d) * 3;
        x[0] = a / s;
        x[1] = at / s;
        x[2] = (dp - dm) / s;
      }
    }
  }
  return 0;
}

#define H1 32
#define H2 32
#define NF 12
/* parameter offsets */
#define OW1 0
#define OB1 (OW1 + H1 * NF)
#define OW2 (OB1 + H1)
#define OB2 (OW2 + H2 * H1)
#define OW3 (OB2 + H2)
#define OB3 (OW3 + H2)
#define NPAR (OB3 + 1)

static double relu(double v) { return v > 0.0 ? v : 0.0; }

static double mlp_one(const double* P, const double* x, double* h1, double* h2) {
  for (int o = 0; o < H1; ++o) {
    double s = P[OB1 + o];
    for (int i = 0; i < NF; ++i) s += P[OW1 + o * NF + i] * x[i];
    h1[o] = relu(s);
  }
  for (int o = 0; o < H2; ++o) {
    double s = P[OB2 + o];
    for (int i = 0; i < H1; ++i) s += P[OW2 + o * H1 + i] * h1[i];
    h2[o] = relu(s);
  }
  double z = P[OB3];
  for (int i = 0; i < H2; ++i) z += P[OW3 + i] * h2[i];
  return z;
}

int or_mlp_forward(const double* params, const double* X, int B, double* logits) {
  double h1[H1], h2[H2];
  for (int n = 0; n < B; ++n) logits[n] = mlp_one(params, X + (size_t)n * NF, h1, h2);
  return 0;
}

static double softplus(double x) { return (x > 0 ? x : 0.0) + log1p(exp(-fabs(x))); }
static double sigmoid(double x) { return 1.0 / (1.0 + exp(-x)); }

/* mean over the batch of the weighted binary cross-entropy with logits,
 * l = pw * y * softplus(-z) + (1 - y) * softplus(z); analytic gradient */
double or_mlp_loss_grad(const double* P, const double* X, const uint8_t* y, int B,
                        double pw, double* grad) {
  double h1[H1], h2[H2], d2[H2], d1[H1];
  double loss = 0.0;
  if (grad) memset(grad, 0, sizeof(double) * NPAR);
  for (int n = 0; n < B; ++n) {
    const double* x = X + (size_t)n * NF;
    double z = mlp_one(P, x, h1, h2);
    double yy = y[n] ? 1.0 : 0.0;
    loss += pw * yy * softplus(-z) + (1.0 - yy) * softplus(z);
    if (!grad) continue;
    double dz = (-pw * yy * (1.0 - sigmoid(z)) + (1.0 - yy) * sigmoid(z)) / B;
    grad[OB3] += dz;
    for (int i = 0; i < H2; ++i) {
      grad[OW3 + i] += dz * h2[i];
      d2[i] = h2[i] > 0.0 ? dz * P[OW3 + i] : 0.0;
    }
    for (int o = 0; o < H2; ++o) {
      grad[OB2 + o] += d2[o];
      for (int i = 0; i < H1; ++i) grad[OW2 + o * H1 + i] += d2[o] * h1[i];
    }
    for (int i = 0; i < H1; ++i) {
      double s = 0.0;
      for (int o = 0; o < H2; ++o) s += P[OW2 + o * H1 + i] * d2[o];
      d1[i] = h1[i] > 0.0 ? s : 0.0;
    }
    for (int o = 0; o < H1; ++o) {
      grad[OB1 + o] += d1[o];
      for (int i = 0; i < NF; ++i) grad[OW1 + o * NF + i] += d1[o] * x[i];
    }
  }
  return loss / B;
}

int or_adam(double* p, double* m1, double* m2, const double* g, int n, int step, double lr,
            double b1, double b2, double eps) {
  double c1 = 1.0 - pow(b1, step), c2 = 1.0 - pow(b2, step);
  for (int i = 0; i < n; ++i) {
    m1[i] = b1 * m1[i] + (1.0 - b1) * g[i];
    m2[i] = b2 * m2[i] + (1.0 - b2) * g[i] * g[i];
    p[i] -= lr * (m1[i] / c1) / (sqrt(m2[i] / c2) + eps);
  }
  return 0;
}
