/*
 * crkdg_oracle.h -- serial FP64 CPU oracle of the compact Runge--Kutta
 * discontinuous Galerkin (cRKDG) method of Chen, Sun and Xing (arXiv 2307.06471).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark load this library.  It shares no source with
 * the HIP library: its own Legendre/Gauss tables, its own flux functions, its
 * own initial conditions.  Plain per-cell loops, no sum factorisation, no
 * threads, no SIMD; built with -O2 -ffp-contract=off.
 *
 * Data layout (the exchange format, identical to the HIP library's canonical
 * host format): u[comp][mode][cell], cell = j*nx + i (x fastest), mode
 * index m + (k+1)*n for the tensor Legendre basis P_m(xi) P_n(eta) (1D: m).
 * Mode 0 is the cell average.
 *
 * Every function is a plain restatement of a definition in the paper:
 *   - DG operator, Section 2.1, equation (DG operator);
 *   - local operator, Section 2.2, equation (dxl);
 *   - cRKDG step, Section 2.2, equation (crkdg); RKDG, Section 2.1 (rkdg);
 *   - Shu--Osher substitution, Section 3.2.1, equations (ssprk2) and
 *     (ssprk2-wrong_scheme);
 *   - limiter applied once after the final stage, Section 2.2 remark on
 *     limiters and Section 4.2;
 *   - Burgers' equation with the Godunov flux and its exact solution by
 *     characteristics, Section 4.1.1 example 'ex:1dburgers' (pinned to the
 *     printed errors of Table 'table_burgers1d').
 * Readings of points the paper leaves open are listed in the design notes
 * (quadrature, Lax--Friedrichs alpha, TVB limiter details, error norms).
 *
 * Parity unpinned: the TVB limiter details (the paper defers to reference
 * [rkdg5]), the positivity safeguard and the MLP indicator are not in the
 * paper; they are pinned only by generic properties (truth tables, exact
 * mean preservation, finite-difference gradients).
 */
#ifndef CRKDG_ORACLE_H
#define CRKDG_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { OR_EQ_ADVECTION = 0, OR_EQ_EULER = 1, OR_EQ_BURGERS = 2 /* 1D only */ };
enum { OR_FLUX_UPWIND = 0, OR_FLUX_LLF = 1, OR_FLUX_GODUNOV = 2 /* Burgers only */ };
enum { OR_BC_PERIODIC = 0, OR_BC_TRANSMISSIVE = 1, OR_BC_DIRICHLET = 2 };
enum { OR_OP_LOC = 0, OR_OP_DG = 1 };

/* initial-condition / exact-solution identifiers */
enum {
  OR_IC_CONST = 0,          /* params: conserved state (ncomp values)                  */
  OR_IC_ADV_SIN = 1,        /* 1D: sin(x - a t); 2D: sin(pi(x-a t)) sin(pi(y-b t))       */
  OR_IC_EULER_WAVE = 2,     /* rho=1+0.2 sin(pi(x+y-(u+v)t)), (u,v,p) from params[0..2]  */
  OR_IC_VORTEX = 3,         /* isentropic vortex; params: eps, xc, yc, period_x, period_y */
  OR_IC_QUADRANT = 4,       /* params: xs, ys, then rho,u,v,p for NE, NW, SW, SE         */
  OR_IC_SHOCK = 5,          /* params: theta, rho_s, un_s, p_s, x0, y0, rho_floor, amp;
                               aux: cell-centre noise field xi[ny][nx]                    */
  OR_IC_ADV_SIN_1D_SHIFT = 6, /* 1D advection sin(x - a t) used as inflow data           */
  OR_IC_DMR = 7,            /* double Mach reflection: the planar Mach 10 shock through
                               (1/6, 0) at 60 degrees, moved to time t (no params).  As
                               bc_exact: Dirichlet sides take this solution at the face
                               point, except the bottom side from x = 1/6 on, which is a
                               reflecting wall (interior trace, normal momentum mirrored) */
  OR_IC_BURGERS_SIN = 8     /* 1D Burgers: u(x, 0) = sin(x); at time t (before the shock
                               forms at t = 1) the solution of u = sin(x - u t)        */
};

typedef struct {
  int dim;              /* 1 or 2 */
  int nx, ny;           /* cells (ny = 1 when dim == 1) */
  double x0, x1, y0, y1;
  int bc[4];            /* x-left, x-right, y-bottom, y-top */
  double bc_state[4][4];/* conserved ghost state on Dirichlet sides */
  int bc_exact;         /* if > 0: Dirichlet data from exact solution with this id */
  int equation;         /* OR_EQ_* */
  double adv[2];        /* advection velocity */
  double gamma;         /* ratio of specific heats */
  int flux;             /* OR_FLUX_* */
  const double* ic_params; /* parameters of the exact solution used by bc_exact */
} or_mesh;

int    or_ncomp(const or_mesh* m);
int    or_nmodes(const or_mesh* m, int k);

/* tables (Gauss--Legendre by Newton iteration, Legendre by three-term recurrence) */
int    or_gauss(int n, double* x, double* w);
double or_legendre(int m, double x);
double or_dlegendre(int m, double x);

/* L2 projection of an initial condition with (k+3)^dim Gauss points */
int    or_project(const or_mesh* m, int k, int ic, const double* params,
                  const double* aux, double t, double* u);

/* one application of the local operator (op=OR_OP_LOC) or the DG operator
 * (op=OR_OP_DG); out = nabla . f(u) in the modal basis.  t_bc is the time at
 * which time-dependent Dirichlet data are evaluated. */
int    or_apply(const or_mesh* m, int k, int op, double t_bc, const double* u, double* out);

/* time steps; u is updated in place.  Tableau A is s*s row-major, strictly
 * lower triangular. */
int    or_step_crkdg(const or_mesh* m, int k, int s, const double* A, const double* b,
                     const double* c, double t, double dt, double* u);
int    or_step_rkdg(const or_mesh* m, int k, int s, const double* A, const double* b,
                    const double* c, double t, double dt, double* u);
/* Shu--Osher SSP forms of the original RKDG (order 2 or 3), with the limiter
 * after every stage when M >= 0 */
int    or_step_rkdg_ssp(const or_mesh* m, int k, int order, double t, double dt,
                        double M, double* u);
/* Shu--Osher form with the local operator substituted in the inner stages
 * (the non-conservative, sub-optimal scheme); order 2 or 3 */
int    or_step_wrong_ssp(const or_mesh* m, int k, int order, double t, double dt, double* u);

/* stage states of one cRKDG step (u^(1..s)), for operator-level parity */
int    or_crkdg_stages(const or_mesh* m, int k, int s, const double* A, const double* b,
                       const double* c, double t, double dt, const double* u, double* stages);

/* TVB minmod limiter applied once (after the final stage).  flags[cell] is a
 * bit mask: 1 troubled (TVB test), 2 positivity check failed (limited P1),
 * 4 still non-physical (P0).  Returns the number of flagged cells, or -1 if
 * a cell average is non-physical. */
int64_t or_limit_tvb(const or_mesh* m, int k, double M, double* u, uint8_t* flags);
/* the same with time-dependent ghost data evaluated at time t (double Mach
 * reflection: ghost cell average = the exact solution at the ghost cell's
 * centre, or the cell's own average with the normal momentum mirrored at the
 * reflecting wall); or_limit_tvb is this at t = 0 */
int64_t or_limit_tvb_at(const or_mesh* m, int k, double M, double t, double* u, uint8_t* flags);
/* troubled-cell indicator only, with decision margins (see or_limit_tvb) */
int64_t or_tvb_flags(const or_mesh* m, int k, double M, const double* u, uint8_t* flags,
                     double* margin);
int64_t or_tvb_flags_at(const or_mesh* m, int k, double M, double t, const double* u,
                        uint8_t* flags, double* margin);
/* double Mach reflection: pre- and post-shock conserved states (Rankine--
 * Hugoniot) and the shock speed, for the given gamma */
void   or_dmr_states(double gamma, double pre[4], double post[4], double* shock_speed);
/* characteristic decomposition of the Euler Jacobian in direction d at a state */
int    or_euler_eig(const or_mesh* m, const double* ubar, int d, double* L, double* R);

/* diagnostics */
double or_max_wavespeed(const or_mesh* m, int k, const double* u);
int    or_errors(const or_mesh* m, int k, const double* u, int ic, const double* params,
                 const double* aux, double t, int comp, double out[3]);
int    or_errors_vs_avg(const or_mesh* m, int k, const double* u, const double* ref_avg,
                        int comp, double out[3]);
double or_total_mass(const or_mesh* m, int k, const double* u, int comp);

/* 12-feature troubled-cell descriptor (reading: q in {rho, E} x d in {x, y};
 * [forward trace jump, backward trace jump, second difference] / scale) */
int    or_mlp_features(const or_mesh* m, int k, double M, const double* u, double* X);
/* 12 -> 32 -> 32 -> 1 MLP, ReLU/ReLU/logit; parameters packed W1,b1,W2,b2,w3,b3.
 * or_mlp_forward: the network's definition, binary64 throughout; it is the
 * reference for training and for inference alike */
int    or_mlp_forward(const double* params, const double* X, int B, double* logits);
double or_mlp_loss_grad(const double* params, const double* X, const uint8_t* y, int B,
                        double pos_weight, double* grad);
int    or_adam(double* params, double* m1, double* m2, const double* grad, int n, int step,
               double lr, double beta1, double beta2, double eps);

#ifdef __cplusplus
}
#endif
#endif
