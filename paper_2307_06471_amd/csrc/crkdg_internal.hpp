// crkdg_internal.hpp -- types shared by the host API and the kernel launchers
// of the cRKDG library (not part of the public C ABI).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/crkdg.h"

namespace crk {

constexpr int MAXS = 6;        // stages of the largest tableau (Fehlberg's)
constexpr int NPARAM = 24;     // initial-condition parameters passed to kernels

// device layouts of a state
//  L64:  double u[comp][mode][cell]                      (canonical)
//  LMIX: double avg[comp][cell], then float hi[comp][mode-1][cell]
//  L32:  float u[comp][mode][cell]                       (FP32 stage states)
enum Layout { L64 = 0, LMIX = 1, L32 = 2 };

struct Geo {
  int nx, ny;
  long long N;
  double x0, y0, dx, dy, inv_dx, inv_dy;
};

struct BCDev {
  int type[4];           // x-left, x-right, y-bottom, y-top
  double state[4][4];    // Dirichlet conserved states
  int exact;             // > 0: time-dependent Dirichlet data from this IC id
  double params[NPARAM]; // its parameters
  double t;              // limiter: time of the time-dependent ghost averages
  const double* t_ptr;   // if set: that time is *t_ptr (+ dt_fac * *dt_ptr if
  const double* dt_ptr;  // dt_ptr is set), read from device memory
  double dt_fac;
};

// double Mach reflection data in BCDev::params / projection parameters:
// [0] x of the wall's start, [1..2] unit shock normal (into the gas at rest),
// [3] shock speed, [4..7] post-shock and [8..11] pre-shock conserved states
constexpr int DMR_NPARAM = 12;

struct PhysDev {
  double gamma, ax, ay;
  int upwind;
};

// one equation/dimension/degree selection
enum EqId { EQ_ADV1 = 0, EQ_ADV2 = 1, EQ_EULER2 = 2, EQ_BURGERS1 = 3 };

// compute precision of a state's step
//  P64:    FP64 throughout (the plain method)
//  PBULK:  FP32 inner and final stages, FP64 cell averages and face sums
//  PINNER: FP32 inner stages (increments over u^n accumulated in FP32, each
//          stored stage formed as u^n + increment in FP64), FP64 final stage
//          (Section 3.3: perturbing only the inner-stage operator evaluations
//          by O(eps) perturbs a step by O(eps dt^2))
//  PINC:   FP32 arithmetic in the inner and the final stage on FP64 states:
//          both accumulate increments over u^n in FP32 and add them to u^n
//          in FP64 (cell averages and face sums FP64), so FP32 rounding
//          enters a step through dt-sized increments only
enum Prec { P64 = 0, PBULK = 1, PINNER = 2, PINC = 3 };

struct InnerArgs {
  const void* un;
  int lay_in;            // layout of u^n
  void* stage[MAXS];     // stage[i] receives u^(i+1) (i >= 1) when bit i of store_mask is set
  int lay_stage;         // layout of the stored stage states
  int s;
  int store_mask;
  double a_sub[MAXS];    // a_{i, i-1}
  double dt;
  const double* dt_ptr;  // if set, dt = *dt_ptr
};

struct FinalArgs {
  const void* base;      // u^n (NULL: zero), layout lay_base
  int lay_base;
  // optional second base: the update starts from bw1 * base + bw2 * base2
  // (Shu--Osher stages of the original RKDG); base2 must be st[0], and in 2D
  // the FP64 layout
  const void* base2;
  double bw1, bw2;
  void* out;             // u^{n+1}, layout lay_base
  int ns;
  const void* st[MAXS];
  int lay[MAXS];         // layout of each final-stage state
  double w[MAXS];        // b_i
  double tst[MAXS];      // boundary-data time of each stage
  double dt;
  const double* dt_ptr;
  // if set: the step's start time is in device memory and stage s's
  // boundary data are taken at *t_ptr + cst[s] * dt (instead of tst[s])
  const double* t_ptr;
  double cst[MAXS];
};

// the whole step in one pass (2D, FP32-bulk, subdiagonal tableaus whose
// weights are nonzero only on the first and last stages, constant boundary
// data): u^n in, u^{n+1} out
struct FusedArgs {
  const void* un;
  void* out;
  int s;
  double a_sub[MAXS];    // a_{i, i-1}
  double w_first, w_last;  // b_1 and b_s (s = 1: w_first only)
  double dt;
  const double* dt_ptr;
  int strip;             // rows a workgroup marches over (set by the launcher)
};

// one inner stage of a full tableau (FP64 layout): L_{i-1} = loc(in), stored
// to L_out if set; out = un + sum_j coef_j X_j (+ coef_last L_{i-1} if
// use_last), every coefficient times *dt_ptr if set
struct LocCombineArgs {
  const double* in;       // u^(i-1)
  const double* un;       // u^n
  double* L_out;          // NULL: L_{i-1} is not needed by a later stage
  double* out;            // u^(i)
  const double* X[MAXS];  // L_j (j < i - 1) with a_ij != 0, ascending j
  double coef[MAXS];
  int nx;
  int use_last;           // a_{i,i-1} != 0
  double coef_last;
  const double* dt_ptr;
};

// launchers (crkdg_kernels.hip); each returns hipSuccess or the launch error.
// prec: one of Prec (layouts and compute types follow from it).
// device time of time-dependent boundary data: *t = v, or *t += *dt
hipError_t launch_time_set(double* t, double v, hipStream_t s);
hipError_t launch_time_add(double* t, const double* dt, hipStream_t s);
hipError_t launch_inner(int eq, int k, int prec, const PhysDev& ph, const Geo& g,
                        const InnerArgs& a, hipStream_t s);
hipError_t launch_final(int eq, int k, int prec, const PhysDev& ph, const Geo& g,
                        const BCDev& bc, const FinalArgs& a, hipStream_t s);
// whether launch_fused supports this step (equation, degree, precision,
// boundary data); the tableau condition is the caller's
bool fused_supported(int eq, int k, int prec, const BCDev& bc);
hipError_t launch_fused(int eq, int k, int prec, const PhysDev& ph, const Geo& g,
                        const BCDev& bc, const FusedArgs& a, hipStream_t s);
hipError_t launch_loc(int eq, int k, const PhysDev& ph, const Geo& g, const double* in,
                      double* out, hipStream_t s);
hipError_t launch_loc_combine(int eq, int k, const PhysDev& ph, const Geo& g,
                              const LocCombineArgs& a, hipStream_t s);
hipError_t launch_combine(long long n, double* out, const double* base, int nx,
                          const double* coef, const double* const* X, const double* dt_ptr,
                          hipStream_t s);
hipError_t launch_wavespeed(int eq, int k, int lay, const PhysDev& ph, const Geo& g,
                            const void* u, double* partial, int nblocks, double cfl,
                            double* smax_out, double* dt_out, hipStream_t s);
hipError_t launch_error(int eq, int k, int lay, const PhysDev& ph, const Geo& g, const void* u,
                        int ic, const double* params, const double* aux, double t, int comp,
                        double* partial, int nblocks, double* out3, hipStream_t s);
hipError_t launch_total(int eq, int k, int lay, const Geo& g, const void* u, int comp,
                        double* partial, int nblocks, double* out, hipStream_t s);
// errors of cell averages ac[cell] against the r x ry restriction of the
// finer averages af (row length nxf)
hipError_t launch_error_ref(const Geo& g, const double* ac, const double* af, int r, int ry,
                            long long nxf, double area, double* partial, int nb, double* out3,
                            hipStream_t s);
hipError_t launch_project(int eq, int k, int lay, const PhysDev& ph, const Geo& g, int ic,
                          const double* params, const double* aux, double t, void* u,
                          hipStream_t s);
// mlp_params == NULL: TVB test; else learned indicator with the TVB fallback band
// wave_partial (nullable): per-block max wave speed of the (limited) state,
// one double per 256 cells
hipError_t launch_limit(int eq, int k, int lay, const PhysDev& ph, const Geo& g,
                        const BCDev& bc, double M, const float* mlp_params, float tau_lo,
                        float tau_hi, void* u, uint8_t* flags, unsigned long long* counters,
                        double* wave_partial, hipStream_t s);
// dt = cfl / max(partial[0..n)) (and/or the max itself), one block
hipError_t launch_wave_final(const double* partial, int n, double cfl, double* smax, double* dt,
                             hipStream_t s);
hipError_t launch_mlp_features(int k, int lay, const Geo& g, const BCDev& bc, double M,
                               const void* u, float* X, hipStream_t s);
// MLP training kernels (crkdg_mlp.hip)
hipError_t launch_mlp_forward(const float* P, const float* X, int B, float* logits, hipStream_t s);
hipError_t launch_mlp_grad(const float* P, const float* X, const uint8_t* y, int B,
                           float pos_weight, float* grad, float* loss, float* work, hipStream_t s);
hipError_t launch_mlp_adam(float* P, float* m1, float* m2, const float* grad, int step, float lr,
                           float b1, float b2, float eps, hipStream_t s);
size_t mlp_work_floats(int B);
hipError_t launch_mlp_grad_noalloc(const float* P, const float* X, const uint8_t* y, int B,
                                   float pw, float* grad, float* loss, hipStream_t s);
int mlp_noalloc_max_batch();

constexpr int RED_BLOCKS = 1024;  // blocks of the first reduction pass

}  // namespace crk
