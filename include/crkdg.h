/*
 * crkdg.h -- C ABI of the MI355X (gfx950) compact Runge--Kutta discontinuous
 * Galerkin (cRKDG) step library.
 *
 * Method: Chen, Sun and Xing, "The Runge--Kutta discontinuous Galerkin method
 * with compact stencils for hyperbolic conservation laws" (arXiv 2307.06471).
 * One time step (Section 2.2, equation (crkdg)):
 *     u^(1) = u^n,
 *     u^(i) = u^n - dt sum_{j<i} a_ij  loc(u^(j)),      i = 2..s  (inner stages)
 *     u^{n+1} = u^n - dt sum_i b_i DG(u^(i))                    (final stage)
 * where loc is the element-local projected derivative of equation (dxl) and
 * DG the DG operator of equation (DG operator) with a Lax--Friedrichs (or, for
 * linear advection, upwind; for Burgers' equation, Godunov) face flux.  Boundary data enter only the final
 * stage (Section 3.4).  A limiter is applied once per step, after the final
 * stage (Section 2.2, remark on limiters; Section 4.2).
 *
 * Conventions
 *  - Ownership: all device memory (DOFs, workspace, flags, MLP parameters) is
 *    allocated by the caller (for instance PyTorch) and passed as raw device
 *    pointers; the library never allocates or frees device memory.  The
 *    handle owns host metadata only.
 *  - Streams: every call is ordered on the stream given to crkdg_bind.  Only
 *    calls that return a value on the host (marked "syncs") wait for it.
 *  - Canonical DOF layout (host exchange and the FP64 device layout):
 *    u[comp][mode][cell], cell = j*nx + i (x fastest), tensor Legendre basis
 *    phi_mode = P_m(xi) P_n(eta), mode = m + (k+1) n (1D: mode = m); mode 0 is
 *    the cell average.  Components: advection 1; 1D Euler (rho, rho w, E);
 *    2D Euler (rho, rho u, rho v, E), gamma from the mesh.
 *  - Precision forms (2D Euler, k >= 1):
 *    CRKDG_FP32_MIXED ("FP32 bulk"): inner and final stages compute in FP32;
 *    the cell averages, the face-flux sums of the final stage and the
 *    limiter's tests stay FP64.  The DOF buffer holds the cell averages
 *    avg[comp][cell] in FP64 followed by the higher modes
 *    hi[comp][mode-1][cell] in FP32; conversion happens in set/get_state.
 *    CRKDG_FP32_INNER: only the inner stages compute in FP32 (the
 *    increments u^(i) - u^n accumulate in FP32; a stored stage is formed as
 *    u^n + increment in FP64); the final stage and the limiter are FP64 and
 *    the DOF buffer has the FP64 layout.  Section 3.3 (the
 *    perturbed-RK theorem it cites): perturbing only the inner-stage
 *    operator evaluations by O(eps) perturbs a step by O(eps dt^2), so this
 *    form keeps the FP64 accuracy.
 *    CRKDG_FP32_INCREMENTS: the inner and the final stage compute in FP32
 *    on FP64 states: both accumulate the increment over u^n in FP32 and add
 *    it to u^n in FP64 (u^(i) as in CRKDG_FP32_INNER, u^{n+1} likewise; the
 *    cell averages and face-flux sums stay FP64).  FP32 rounding then enters
 *    a step only through increments of size O(dt), where the FP32-bulk form
 *    also rounds the stored higher modes themselves every step.  FP64 DOF
 *    layout; the limiter is the FP64 one.
 *  - Errors: every int-returning call returns CRKDG_OK (0) or a negative code;
 *    crkdg_strerror maps it to text.  Kernel launch failures return
 *    CRKDG_EHIP.  Invalid arguments never reach a kernel.
 */
#ifndef CRKDG_H
#define CRKDG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define CRKDG_OK 0
#define CRKDG_EINVAL (-1)        /* bad argument (k, tableau, dt, sizes, null) */
#define CRKDG_EUNSUPPORTED (-2)  /* valid but not built (e.g. upwind flux for Euler) */
#define CRKDG_ENONPHYSICAL (-3)  /* a cell average has rho <= 0 or p <= 0 or NaN */
#define CRKDG_EHIP (-4)          /* HIP runtime or launch failure */
#define CRKDG_EUNBOUND (-5)      /* state used before crkdg_bind */

/* CRKDG_EQ_BURGERS: u_t + (u^2/2)_x = 0 in 1D (Section 4.1.1, example
 * 'ex:1dburgers'), with CRKDG_FLUX_GODUNOV only (the exact Riemann solution's
 * flux at the face: min of u^2/2 over [uL, uR] if uL <= uR, else the larger
 * of uL^2/2, uR^2/2) */
enum { CRKDG_EQ_ADVECTION = 0, CRKDG_EQ_EULER = 1, CRKDG_EQ_BURGERS = 2 };
enum { CRKDG_FLUX_UPWIND = 0, CRKDG_FLUX_LLF = 1, CRKDG_FLUX_GODUNOV = 2 };
enum { CRKDG_BC_PERIODIC = 0, CRKDG_BC_TRANSMISSIVE = 1, CRKDG_BC_DIRICHLET = 2 };
enum { CRKDG_FP64 = 0, CRKDG_FP32_MIXED = 1, CRKDG_FP32_INNER = 2, CRKDG_FP32_INCREMENTS = 3 };
enum { CRKDG_OP_LOC = 0, CRKDG_OP_DG = 1 };

/* initial conditions / exact solutions known to the library */
enum {
  CRKDG_IC_CONST = 0,       /* params: conserved state                                   */
  CRKDG_IC_ADV_SIN = 1,     /* 1D sin(x - a t); 2D sin(pi(x - a t)) sin(pi(y - b t))       */
  CRKDG_IC_EULER_WAVE = 2,  /* rho = 1 + 0.2 sin(pi(x + y - (u+v) t)); params: u, v, p      */
  CRKDG_IC_VORTEX = 3,      /* isentropic vortex; params: eps, xc, yc, Lx, Ly (exact at t) */
  CRKDG_IC_QUADRANT = 4,    /* params: xs, ys, then (rho,u,v,p) for NE, NW, SW, SE        */
  CRKDG_IC_SHOCK = 5,       /* params: theta, rho_s, un_s, p_s, x0, y0, rho_floor, amp;
                               aux: cell-centre field xi[ny][nx] (device, FP64)          */
  CRKDG_IC_DMR = 6,         /* double Mach reflection (Section 4, example "Double Mach
                               reflection"): a Mach 10 shock moving right into gas at rest
                               (rho, p) = (1.4, 1), through (1/6, 0) at 60 degrees to the
                               x-axis at t = 0, post-shock state from the Rankine--Hugoniot
                               conditions; no params (2D Euler only).  As bc_exact (sides
                               x-left, y-bottom, y-top Dirichlet, x-right transmissive):
                               Dirichlet data are this moving shock at the face point and
                               stage time, except on the bottom from x = 1/6 on, a
                               reflecting wall (the cell's own trace with the normal
                               momentum mirrored).  The limiter's ghost averages there are
                               the same rules at the ghost cell's centre and the state's
                               time (crkdg_get_time).  The learned indicator
                               (crkdg_limit_mlp, crkdg_mlp_features, crkdg_limit_dt with
                               parameters) is CRKDG_EUNSUPPORTED on such a mesh. */
  CRKDG_IC_BURGERS_SIN = 7  /* 1D Burgers: u(x, 0) = sin x; at time t < 1 (before the shock
                               forms) the solution of u = sin(x - u t) (no params) */
};

typedef struct {
  int dim;                  /* 1 or 2 */
  int nx, ny;               /* cells; ny = 1 when dim == 1 */
  double x0, x1, y0, y1;    /* domain */
  int bc[4];                /* x-left, x-right, y-bottom, y-top: CRKDG_BC_* */
  double bc_state[4][4];    /* conserved ghost state on Dirichlet sides */
  int bc_exact;             /* > 0: Dirichlet data = exact solution with this CRKDG_IC_*
                               id (CRKDG_IC_ADV_SIN or CRKDG_IC_DMR), evaluated at the
                               stage time t^n + c_i dt */
  int equation;             /* CRKDG_EQ_* */
  double adv[2];            /* advection velocity */
  double gamma;             /* ratio of specific heats (Euler) */
  int precision;            /* CRKDG_FP64 | CRKDG_FP32_MIXED | CRKDG_FP32_INNER |
                               CRKDG_FP32_INCREMENTS */
} crkdg_mesh;

typedef struct crkdg_state crkdg_state;

/* Create a handle (host only; no device work).  k = 0..4 polynomial degree
 * (Q^k on rectangles, P^k in 1D; Section 2.1); k = 4 for the scalar
 * equations (advection, Burgers) only.  flux: CRKDG_FLUX_*.
 * rk_stages selects the paper's tableaus: 1 forward Euler, 2 scheme (eq:2),
 * 3 scheme (eq:3), 4 classical RK4, 5 the fifth-order Runge--Kutta--Fehlberg
 * method (six stages; Section 4 pairs it with k = 4).  RK4's tableau has
 * only a subdiagonal, so its inner stages run as one element-local pass;
 * Fehlberg's full tableau takes the materialised path (FP64 only: one pass
 * per inner stage writing loc(u^(j)), then a combination pass).
 * The workspace holds the stage states of max(4, stages) stages.
 * Returns CRKDG_EINVAL for bad sizes/arguments, including meshes whose
 * cells x max((k+1)^dim, 4) x 8 bytes reach 4 GiB (one component of one
 * state must stay below 4 GiB: 59.6 M cells for Q2, 33.5 M for Q3),
 * CRKDG_EUNSUPPORTED for an unsupported combination.
 * *out is set only on success. */
int crkdg_create(const crkdg_mesh* mesh, int k, int flux, int rk_stages, crkdg_state** out);

/* Replace the tableau by an explicit one (Section 2.1, equation (butcher)):
 * s <= 6 stages, A row-major s*s strictly lower triangular (a_ij = 0 for
 * j >= i), b and c of length s; host arrays, copied.  sum(b) need not be 1.
 * Before crkdg_bind any s is accepted and sizes the workspace
 * (crkdg_workspace_bytes); after it, s may not exceed what the bound
 * workspace holds (max(4, stages) at bind time): CRKDG_EINVAL. */
int crkdg_set_tableau(crkdg_state* st, int s, const double* c, const double* A, const double* b);

/* bytes of the DOF buffer and of the workspace for the chosen layout */
size_t crkdg_state_bytes(const crkdg_state* st);
size_t crkdg_workspace_bytes(const crkdg_state* st);

/* Bind caller-owned device memory: dofs (crkdg_state_bytes, 256-byte aligned)
 * holds u^n; work (crkdg_workspace_bytes, 256-byte aligned) holds the second
 * state buffer, the stage states and reduction scratch.  stream is a
 * hipStream_t (NULL = default stream).  The current state may afterwards
 * live in either buffer (double buffering); crkdg_current_dofs tells which. */
int crkdg_bind(crkdg_state* st, void* dofs_dev, void* work_dev, void* stream);
void* crkdg_current_dofs(const crkdg_state* st);

/* host <-> device state in the canonical FP64 layout; set/get are
 * stream-ordered; get_state syncs */
int crkdg_set_state(crkdg_state* st, const double* host_dofs);
int crkdg_get_state(const crkdg_state* st, double* host_dofs);
/* time t^n used for time-dependent boundary data; crkdg_get_time reads the
 * device copy back (and syncs) after crkdg_step_dev on such a mesh */
int crkdg_set_time(crkdg_state* st, double t);
double crkdg_get_time(const crkdg_state* st);

/* L2 projection of an initial condition with (k+3) Gauss points per
 * direction into the current state (device kernel; aux: device FP64 or NULL) */
int crkdg_project(crkdg_state* st, int ic, const double* params, int nparams,
                  const double* aux_dev);

/* One cRKDG step of size dt (> 0, finite), Section 2.2 equation (crkdg); no
 * limiter.  Advances the internal time by dt. */
int crkdg_step(crkdg_state* st, double dt);
/* Same, with dt read from device memory (written by crkdg_compute_dt or
 * crkdg_limit_dt); no host synchronisation.  Without time-dependent boundary
 * data the internal time is not advanced.  With them (bc_exact), the time is
 * kept in device memory (the library's workspace): the stages take their
 * boundary data at t + c_i * (*dt_dev), the limiter's ghost averages at the
 * advanced time, and crkdg_get_time reads it back (syncs).
 * crkdg_step_dev and crkdg_limit_dt only launch kernels on the bound stream
 * (no allocation, memset, copy or synchronisation), so a run of them can be
 * captured in a HIP graph and replayed; the handle alternates between two
 * state buffers on the host side, so a captured run must hold an even
 * number of steps. */
int crkdg_step_dev(crkdg_state* st, const double* dt_dev);

/* Schedule of crkdg_step / crkdg_step_dev.  The compact stencil of Section
 * 3.1 (a step reaches only the face neighbours of a cell, for any number of
 * stages, because the inner stages are element local) lets one kernel do
 * the whole step on a strip of cells plus a one-cell ring: read u^n once,
 * recompute the ring's inner stages, evaluate the strip's faces, write
 * u^{n+1}; no stage state goes through memory.
 *   CRKDG_SCHED_SPLIT  inner-stage pass, then final-stage pass (any case);
 *   CRKDG_SCHED_FUSED  the one-pass step, for 2D Euler in the FP32-bulk
 *                      or the FP64 form with k = 1 or 2, constant boundary
 *                      data
 *                      (periodic, transmissive, time-independent Dirichlet)
 *                      and a subdiagonal tableau whose weights are nonzero
 *                      only on the first and last stages (schemes (eq:2),
 *                      (eq:3), forward Euler).
 * The results of the two schedules agree to the rounding of the form's
 * arithmetic (in the FP32-bulk form the fused step sums the stage-weighted
 * face fluxes in FP32, the split final stage in FP64; both convert each
 * face's sum exactly into the FP64 cell-average update, so both conserve).
 * crkdg_set_schedule returns CRKDG_EUNSUPPORTED for CRKDG_SCHED_FUSED on a
 * handle that does not meet these conditions, CRKDG_EINVAL for an unknown
 * value.  crkdg_get_schedule returns the schedule the next step takes (a
 * later crkdg_set_tableau can make a fused handle fall back to the split
 * schedule).  New handles start with CRKDG_SCHED_FUSED: every step that the
 * one-pass kernel can take runs there (on the 4096 x 1024 Q2 shock workload
 * it takes 0.65 ms against 0.92 ms for the two split passes in the FP32-bulk
 * form, 1.66 ms against 2.26 ms in FP64). */
#define CRKDG_SCHED_SPLIT 0
#define CRKDG_SCHED_FUSED 1
int crkdg_set_schedule(crkdg_state* st, int sched);
int crkdg_get_schedule(const crkdg_state* st);

/* One step of the original RKDG method that the paper compares against
 * (Section 2.1, equation (rkdg)), in the Shu--Osher SSP form of order 2 or 3
 * (Section 3.2.1 gives the order-2 form): every stage applies the DG
 * operator with face fluxes and boundary data at its stage time and, when
 * M >= 0, the TVB limiter of crkdg_limit (no flags); M < 0 skips the limiter.
 * order 0: the Butcher form of equation (rkdg) with the state's own tableau
 * (crkdg_create's rk_stages or crkdg_set_tableau; Section 4 runs RKDG with
 * classical RK4 at k = 3 and the fifth-order Runge--Kutta--Fehlberg method at
 * k = 4), without limiter (M must be < 0, else CRKDG_EINVAL); it uses the
 * workspace's operator slots and first two stage slots.
 * FP64 state only (CRKDG_EUNSUPPORTED otherwise).  dt_dev (device double,
 * nullable) overrides dt, as in crkdg_step_dev (with time-dependent boundary
 * data the time is kept and advanced in device memory, the stages' data and
 * limiter ghosts read it there); otherwise dt must be finite and > 0 and the
 * time advances by dt.  Uses the workspace's first stage slot; stream-ordered,
 * no sync. */
int crkdg_step_rkdg(crkdg_state* st, int order, double M, double dt, const double* dt_dev);

/* dt = cfl / max_K [ (|u|+c)/dx + (|v|+c)/dy ] from the FP64 cell averages
 * (advection: |a|/dx + |b|/dy), written to device memory (one double).
 * Stream-ordered, no sync.  The paper gives CFL numbers only (Section 4);
 * this wave-speed formula is the build's reading. */
int crkdg_compute_dt(crkdg_state* st, double cfl, double* dt_dev);
/* s_max of the formula above, returned on the host (syncs) */
int crkdg_max_wavespeed(crkdg_state* st, double* s_max_host);

/* TVB minmod limiter applied once after the final stage (Section 2.2 remark
 * on limiters; Section 4.2): troubled-cell test in characteristic variables
 * with constant M (threshold M h^2), limited P1 reconstruction of troubled
 * cells with every other non-mean mode zeroed, cell averages unchanged, then
 * an FP64 positivity check of rho and p at the operator's quadrature points
 * (demotion to P1, then P0).  flags_dev (uint8 per cell, may be NULL) is a
 * bit mask: 1 troubled, 2 positivity failure (limited P1), 4 demoted to P0,
 * 8 decided by the TVB fallback (learned-indicator mode).  If
 * n_flagged_host is not NULL the call syncs and returns the count there.
 * Returns CRKDG_ENONPHYSICAL (after syncing) only when n_flagged_host is
 * given and a cell average is non-physical. */
int crkdg_limit(crkdg_state* st, double M, uint8_t* flags_dev, int64_t* n_flagged_host);

/* Learned troubled-cell indicator (not part of the paper's method): the
 * same final-stage limiter, with the TVB troubled-cell test replaced by a
 * 12 -> 32 -> 32 -> 1 perceptron (ReLU, ReLU, logistic output; parameters
 * packed W1[32][12], b1[32], W2[32][32], b2[32], w3[32], b3 as 1505 device
 * floats) on 12 stencil features (computed in FP64, rounded to FP32),
 * evaluated in FP32: both hidden layers on the FP32 matrix cores, the output
 * layer on the vector units.
 * p = sigmoid(logit): p >= tau_hi troubled, p <= tau_lo smooth, otherwise
 * the FP64 TVB test decides (flag bit 8); tau_lo <= tau_hi.
 * Reconstruction and positivity check as in crkdg_limit.  counts_host
 * (nullable, syncs): [0] flagged cells, [1] cells decided by the fallback.
 * 2D Euler only (CRKDG_EUNSUPPORTED otherwise). */
int crkdg_limit_mlp(crkdg_state* st, double M, const float* params_dev, float tau_lo,
                    float tau_hi, uint8_t* flags_dev, int64_t* counts_host);
/* The final-stage limiter followed by the next step's dt: crkdg_limit
 * (params_dev == NULL) or crkdg_limit_mlp (params_dev set, with the band
 * tau_lo <= tau_hi), and dt = cfl / s_max of the limited state written to
 * dt_dev (1 device double), with s_max as in crkdg_compute_dt.  The limiter
 * never changes a cell average, so s_max comes from the averages the limiter
 * has already read: this saves the separate pass of crkdg_compute_dt.
 * Stream-ordered, no sync, no counts; flags_dev nullable. */
int crkdg_limit_dt(crkdg_state* st, double M, const float* params_dev, float tau_lo,
                   float tau_hi, uint8_t* flags_dev, double cfl, double* dt_dev);
/* The 12 features of every cell of the current state, X[cell][12] FP32
 * (computed in FP64): for q in {rho, E} and d in {x, y}, with a / at the
 * forward / backward face-average jumps of q, dp / dm the neighbouring
 * cell-average differences and s = |dp| + |dm| + M h_d^2 + 1e-300:
 * a/s, at/s, (dp - dm)/s.  2D Euler only. */
int crkdg_mlp_features(crkdg_state* st, double M, float* X_dev);
/* MLP kernels on device arrays (stream = hipStream_t or NULL):
 * forward logits of B samples X[B][12] by the limiter's FP32 inference;
 * the batch-mean weighted BCE loss (FP32 forward and backward)
 * pos_weight*y*softplus(-z) + (1-y)*softplus(z) and its gradient (1505
 * floats; loss: 1 device float or NULL) with a deterministic two-level
 * reduction in caller-owned work memory of crkdg_mlp_work_bytes(B); one
 * Adam update with bias correction (step >= 1). */
size_t crkdg_mlp_work_bytes(int B);
int crkdg_mlp_forward(const float* params, const float* X, int B, float* logits, void* stream);
int crkdg_mlp_grad(const float* params, const float* X, const uint8_t* y, int B,
                   float pos_weight, float* grad, float* loss, void* work, size_t work_bytes,
                   void* stream);
int crkdg_mlp_adam(float* params, float* m1, float* m2, const float* grad, int step, float lr,
                   float beta1, float beta2, float eps, void* stream);
/* For callers that cannot allocate device memory (code under HIP graph
 * capture, serving loops, harnesses that forbid hipMalloc): crkdg_mlp_grad
 * without the work argument.  The same kernels and reduction order, so the
 * result is bit-identical to crkdg_mlp_grad's.  The workgroup partials live
 * in a library-owned device array of CRKDG_MLP_NOALLOC_MAX_B / 64 x 1506
 * floats (1.5 MB), one per GPU, held until the process ends; this call
 * allocates nothing (no hipMalloc, no allocating library routine).  The
 * first call on a device looks up that device's copy of the array.  Every
 * call on one GPU shares its array: calls that overlap on one GPU (other
 * streams or threads) race and must be serialised by the caller.
 * CRKDG_EINVAL for B < 1, B > CRKDG_MLP_NOALLOC_MAX_B, a null pointer or a
 * non-positive pos_weight; CRKDG_EHIP if the device lookup fails. */
#define CRKDG_MLP_NOALLOC_MAX_B 16384
int crkdg_mlp_grad_noalloc(const float* params, const float* X, const uint8_t* y, int B,
                           float pos_weight, float* grad, float* loss, void* stream);

/* L1, L2 (unnormalised integrals over the domain) and Linf errors of
 * component comp against exact solution ic at time t, (k+3)^dim Gauss points
 * per cell; out on host (syncs).  Deterministic two-pass reduction.  The
 * error tables of Section 4 (Tables 'table:boundary_treatment',
 * 'table:euler accuracy', 'table:2deuler-periodic-rectangle') report these
 * norms; the paper does not define them, and the unnormalised integral is
 * the reading under which its printed L2 exceeds its Linf on (0, 4 pi).
 * params: the initial-condition parameters of ic (nparams of them, as for
 * crkdg_project).  CRKDG_EINVAL for an unknown ic or a component out of
 * range, CRKDG_EUNBOUND before crkdg_bind. */
int crkdg_error(crkdg_state* st, int ic, const double* params, int nparams, double t,
                int comp, double out_l1_l2_linf[3]);
/* L1, L2 (unnormalised, |K|-weighted sums) and Linf errors of the cell
 * averages of component comp against a finer reference state `ref` restricted
 * to this mesh: each coarse cell is compared with the mean of the r x ry fine
 * cell averages covering it (r = ref nx / nx, ry = ref ny / ny; the error
 * tables of Section 4 measure against a refined solution where no exact one
 * exists).  Both states must be bound, have the same equation and domain, and
 * the fine cell counts must be integer multiples of the coarse ones; ref may
 * have any degree and precision.  out on host (syncs both streams).
 * Deterministic two-pass reduction.  CRKDG_EINVAL on mismatched meshes. */
int crkdg_error_ref(crkdg_state* st, crkdg_state* ref, int comp, double out_l1_l2_linf[3]);
/* sum over cells of |K| * cell average of component comp (syncs) */
int crkdg_total(crkdg_state* st, int comp, double* out_host);

/* Operator-level entry points (materialised path; general tableaus):
 * out = loc(in) or DG(in) at boundary-data time t_bc (device arrays in the
 * state's layout, FP64 layout only). */
int crkdg_apply_op(crkdg_state* st, int op, const void* in_dev, void* out_dev, double t_bc);
/* RK stage combination out = base + sum_j coef_j X_j, j < n <= 6 (device
 * arrays of crkdg_state_bytes each, FP64 layout only). */
int crkdg_combine(crkdg_state* st, void* out_dev, const void* base_dev, int n,
                  const double* coef, const void* const* X_dev);

/* Measurement: record a HIP event pair on the bound stream around every
 * kernel launch (at most max_launches) until crkdg_profile_end, which syncs
 * and returns the summed milliseconds and launch counts per kernel class:
 * 0 inner stages, 1 final stage, 2 local operator, 3 stage combination,
 * 4 dt reduction, 5 limiter, 6 other, 7 fused step.  Host-side events only;
 * no device memory is allocated. */
int crkdg_profile_begin(crkdg_state* st, int max_launches);
int crkdg_profile_end(crkdg_state* st, double ms[8], int64_t counts[8]);

/* Host-only: the library's own n-point Gauss--Legendre rule (n = 1..8). */
int crkdg_gauss_rule(int n, double* x, double* w);

void crkdg_destroy(crkdg_state* st);
const char* crkdg_strerror(int code);

#ifdef __cplusplus
}
#endif
#endif
