// crkdg_kernels.hip -- HIP kernels of the cRKDG step for gfx950.
//
//   k_inner    all inner stages of one step, element local (Section 2.2,
//              equation (crkdg), first line): one lane per cell, the whole
//              stage chain in registers, no neighbour data, no boundary data.
//   k_final2   final stage (equation (crkdg), second line): a 64x4 tile of
//              cells per workgroup; stage traces are exchanged through LDS,
//              every face flux is computed once per tile in canonical (+x/+y)
//              orientation and the stage-weighted sum G = sum_i b_i F^(i)
//              (equation (g)) is accumulated in FP64 and lifted into both
//              neighbours with opposite signs, so the cell-average update
//              (equation (avg)) is conservative and done in FP64.
//   k_final1   the same for 1D meshes.
//   k_fused2   the whole step in one pass (Section 3.1's compact stencil):
//              a workgroup walks a strip of 62 columns, recomputes its
//              one-cell ring's inner stages, evaluates the strip's faces and
//              writes u^{n+1}; 2D Euler, FP32 bulk or FP64, k = 1, 2.
//   k_loc      one application of the local operator (materialised path).
//   k_combine  RK stage combination, out = base + sum_j coef_j X_j (streaming).
//   k_wave*    dt selection from the cell averages (max reduction).
//   k_error*   L1/L2/Linf errors, deterministic two-pass reduction.
//   k_project  L2 projection of an initial condition, (k+3)-point rule.
//   k_limit    TVB minmod troubled-cell test and limited P1 reconstruction
//              in FP64, in place (only a cell's own non-mean modes change).
//
// Precision: the step kernels are templated on the compute type R.  R =
// double is the plain FP64 method; R = float is the FP32-bulk form, in which
// the cell averages stay FP64 in memory and in the final update and the
// stage states of the inner stages are FP32; the face-flux sums G are FP64
// in k_final2 and FP32 in k_fused2, each converted exactly into the FP64
// average update.
#include <math.h>

#include "crkdg_internal.hpp"
#include "dg_core.hpp"
#include "mlp_core.hpp"

// Tuning (measured on the 4096 x 1024 Q2 shock workload): occupancy targets
// in wavefronts per SIMD for __launch_bounds__, and whether the FP64 inner
// kernel keeps u^n in registers (off: at one wavefront per SIMD it loses
// what it saves in re-reads).
#ifndef LIMIT_OCC_TVB
#define LIMIT_OCC_TVB 3
#endif
#ifndef LIMIT_OCC_MLP
#define LIMIT_OCC_MLP 4
#endif
#ifndef INNER_KEEP_F64
#define INNER_KEEP_F64 0
#endif
#ifndef INNER_OCC_F32
#define INNER_OCC_F32 2
#endif
#ifndef INNER_OCC_F64
#define INNER_OCC_F64 1
#endif
#ifndef FINAL_OCC_F32
#define FINAL_OCC_F32 2
#endif
#ifndef FINAL_OCC_F64
#define FINAL_OCC_F64 1
#endif
#ifndef FINAL_TX_F32
#define FINAL_TX_F32 64
#endif
#ifndef FINAL_TY_F32
#define FINAL_TY_F32 4
#endif
#ifndef FINAL_TX_F64
#define FINAL_TX_F64 64
#endif
#ifndef FINAL_TY_F64
#define FINAL_TY_F64 4
#endif

namespace crk {

// ---------------------------------------------------------------------------
// state access (layouts in crkdg_internal.hpp)
// ---------------------------------------------------------------------------
// State arrays are read and written with buffer instructions: a resource
// descriptor (scalar registers) per component slab, the array's start within
// the slab as a scalar offset, and one 32-bit per-lane byte offset shared by
// every array.  No per-load 64-bit address arithmetic, and the compiler keeps
// a single offset register live instead of a 64-bit address per array.
// crkdg_create caps the mesh so that every component slab (and the block of
// FP64 averages) stays below 4 GiB.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t rsrc(const void* base) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, (int)0xffffffff,
                                           0x00020000);
}
__device__ __forceinline__ const void* byte_add(const void* p, long long bytes) {
  return (const char*)p + bytes;
}
template <class T>
__device__ __forceinline__ T bload(__amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff) {
  if constexpr (sizeof(T) == 8)
    return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b64(r, (int)voff, (int)soff, 0));
  else
    return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b32(r, (int)voff, (int)soff, 0));
}
template <class T>
__device__ __forceinline__ void bstore(T v, __amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff) {
  if constexpr (sizeof(T) == 8)
    __builtin_amdgcn_raw_buffer_store_b64(
        __builtin_bit_cast(decltype(__builtin_amdgcn_raw_buffer_load_b64(r, 0, 0, 0)), v), r,
        (int)voff, (int)soff, 0);
  else
    __builtin_amdgcn_raw_buffer_store_b32(
        __builtin_bit_cast(decltype(__builtin_amdgcn_raw_buffer_load_b32(r, 0, 0, 0)), v), r,
        (int)voff, (int)soff, 0);
}

template <class T, int NC, int NB, int LAY>
__device__ __forceinline__ void load_state(const void* __restrict__ p, long long N, long long cell,
                                           T (&u)[NC][NB]) {
  const unsigned o8 = (unsigned)cell * 8u, o4 = (unsigned)cell * 4u;
  if constexpr (LAY == L64) {
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      const auto r = rsrc(byte_add(p, (long long)c * NB * N * 8));
#pragma unroll
      for (int b = 0; b < NB; ++b) u[c][b] = (T)bload<double>(r, o8, (unsigned)(b * N * 8));
    }
  } else if constexpr (LAY == LMIX) {
    const auto ra = rsrc(p);
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      u[c][0] = (T)bload<double>(ra, o8, (unsigned)(c * N * 8));
      const auto rh = rsrc(byte_add(p, (long long)NC * N * 8 + (long long)c * (NB - 1) * N * 4));
#pragma unroll
      for (int b = 1; b < NB; ++b) u[c][b] = (T)bload<float>(rh, o4, (unsigned)((b - 1) * N * 4));
    }
  } else {
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      const auto r = rsrc(byte_add(p, (long long)c * NB * N * 4));
#pragma unroll
      for (int b = 0; b < NB; ++b) u[c][b] = (T)bload<float>(r, o4, (unsigned)(b * N * 4));
    }
  }
}

// store; the averages come from a0 (FP64) when given, else from u
template <class T, int NC, int NB, int LAY>
__device__ __forceinline__ void store_state(void* __restrict__ p, long long N, long long cell,
                                            const T (&u)[NC][NB], const double* a0 = nullptr) {
  const unsigned o8 = (unsigned)cell * 8u, o4 = (unsigned)cell * 4u;
  if constexpr (LAY == L64) {
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      const auto r = rsrc(byte_add(p, (long long)c * NB * N * 8));
      bstore<double>(a0 ? a0[c] : (double)u[c][0], r, o8, 0u);
#pragma unroll
      for (int b = 1; b < NB; ++b) bstore<double>((double)u[c][b], r, o8, (unsigned)(b * N * 8));
    }
  } else if constexpr (LAY == LMIX) {
    const auto ra = rsrc(p);
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      bstore<double>(a0 ? a0[c] : (double)u[c][0], ra, o8, (unsigned)(c * N * 8));
      const auto rh = rsrc(byte_add(p, (long long)NC * N * 8 + (long long)c * (NB - 1) * N * 4));
#pragma unroll
      for (int b = 1; b < NB; ++b) bstore<float>((float)u[c][b], rh, o4, (unsigned)((b - 1) * N * 4));
    }
  } else {
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      const auto r = rsrc(byte_add(p, (long long)c * NB * N * 4));
#pragma unroll
      for (int b = 0; b < NB; ++b) bstore<float>((float)u[c][b], r, o4, (unsigned)(b * N * 4));
    }
  }
}

// the higher modes only (the limiter never changes a cell average)
template <class T, int NC, int NB, int LAY>
__device__ __forceinline__ void store_higher_modes(void* __restrict__ p, long long N, long long cell,
                                                   const T (&u)[NC][NB]) {
  const unsigned o8 = (unsigned)cell * 8u, o4 = (unsigned)cell * 4u;
  if constexpr (LAY == L64) {
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      const auto r = rsrc(byte_add(p, (long long)c * NB * N * 8));
#pragma unroll
      for (int b = 1; b < NB; ++b) bstore<double>((double)u[c][b], r, o8, (unsigned)(b * N * 8));
    }
  } else if constexpr (LAY == LMIX) {
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      const auto rh = rsrc(byte_add(p, (long long)NC * N * 8 + (long long)c * (NB - 1) * N * 4));
#pragma unroll
      for (int b = 1; b < NB; ++b) bstore<float>((float)u[c][b], rh, o4, (unsigned)((b - 1) * N * 4));
    }
  } else {
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      const auto r = rsrc(byte_add(p, (long long)c * NB * N * 4));
#pragma unroll
      for (int b = 1; b < NB; ++b) bstore<float>((float)u[c][b], r, o4, (unsigned)(b * N * 4));
    }
  }
}

// cell average of component c (mode 0), as double
template <int NC, int NB, int LAY>
__device__ __forceinline__ double load_avg(const void* __restrict__ p, long long N, int c,
                                           long long cell) {
  if constexpr (LAY == L64)
    return bload<double>(rsrc(byte_add(p, (long long)c * NB * N * 8)), (unsigned)cell * 8u, 0u);
  else if constexpr (LAY == LMIX)
    return bload<double>(rsrc(p), (unsigned)cell * 8u, (unsigned)(c * N * 8));
  else
    return (double)bload<float>(rsrc(byte_add(p, (long long)c * NB * N * 4)), (unsigned)cell * 4u, 0u);
}

// the step kernels' layout follows the compute type: FP64 layout for the
// FP64 method, mixed layout (FP64 averages, FP32 higher modes) for FP32 bulk
template <class EQ>
struct StepLayout {
  static constexpr int value = sizeof(typename EQ::Real) == 4 ? LMIX : L64;
};

template <class EQ>
struct MakeEq;
template <class R>
struct MakeEq<Euler2<R>> {
  __device__ static Euler2<R> make(const PhysDev& ph) {
    Euler2<R> e;
    e.gam = (R)ph.gamma;
    e.gm1 = (R)(ph.gamma - 1.0);
    return e;
  }
};
template <class R, int D>
struct MakeEq<Adv<R, D>> {
  __device__ static Adv<R, D> make(const PhysDev& ph) {
    Adv<R, D> e;
    e.ax = (R)ph.ax;
    e.ay = D == 2 ? (R)ph.ay : R(0);
    e.upwind = ph.upwind;
    return e;
  }
};
template <class R>
struct MakeEq<Burgers1<R>> {
  __device__ static Burgers1<R> make(const PhysDev&) { return Burgers1<R>{}; }
};
template <class EQ>
__device__ __forceinline__ EQ make_eq(const PhysDev& ph) {
  return MakeEq<EQ>::make(ph);
}

// ---------------------------------------------------------------------------
// exact solutions / initial data (device side; used by projection, error
// norms and time-dependent Dirichlet data)
// ---------------------------------------------------------------------------
__device__ __forceinline__ void prim2cons(int dim, double gamma, double rho, double u, double v,
                                          double p, double* q) {
  if (dim == 1) {
    q[0] = rho;
    q[1] = rho * u;
    q[2] = p / (gamma - 1.0) + 0.5 * rho * u * u;
  } else {
    q[0] = rho;
    q[1] = rho * u;
    q[2] = rho * v;
    q[3] = p / (gamma - 1.0) + 0.5 * rho * (u * u + v * v);
  }
}

__device__ __forceinline__ double periodic_offset(double d, double L) {
  // representative of d modulo L in [-L/2, L/2)
  double r = d - L * floor(d / L + 0.5);
  return r;
}

// double Mach reflection: the planar shock moved along its normal to time t
// (P as in DMR_NPARAM)
__device__ __forceinline__ void dmr_state(const double* P, double x, double y, double t,
                                          double* q) {
  const double* st = P[1] * (x - P[0]) + P[2] * y < P[3] * t ? P + 4 : P + 8;
  for (int c = 0; c < 4; ++c) q[c] = st[c];
}

template <class EQ>
__device__ void exact_state(int ic, const double* P, const double* aux, const Geo& g,
                            const PhysDev& ph, double x, double y, double t, double* q) {
  constexpr int dim = EQ::DIM;
  switch (ic) {
    case CRKDG_IC_CONST:
      for (int c = 0; c < EQ::NC; ++c) q[c] = P[c];
      return;
    case CRKDG_IC_ADV_SIN:
      if (dim == 1)
        q[0] = sin(x - ph.ax * t);
      else
        q[0] = sin(M_PI * (x - ph.ax * t)) * sin(M_PI * (y - ph.ay * t));
      return;
    case CRKDG_IC_BURGERS_SIN: {
      // u = u0(x - u t), u0 = sin (characteristics, before the shock at t = 1):
      // Newton's method on h(v) = v - sin(x - v t), h' = 1 + t cos(x - v t) >= 1 - t
      double v = sin(x);
      for (int it = 0; it < 50; ++it) {
        const double ph_ = x - v * t;
        const double dv = (v - sin(ph_)) / (1.0 + t * cos(ph_));
        v -= dv;
        if (fabs(dv) <= 1e-17) break;
      }
      q[0] = v;
      return;
    }
    case CRKDG_IC_EULER_WAVE: {
      const double u = P[0], v = P[1], p = P[2];
      const double rho = dim == 1 ? 1.0 + 0.2 * sin(M_PI * (x - u * t))
                                  : 1.0 + 0.2 * sin(M_PI * (x + y - (u + v) * t));
      prim2cons(dim, ph.gamma, rho, u, v, p, q);
      return;
    }
    case CRKDG_IC_VORTEX: {
      const double eps = P[0], gm = ph.gamma;
      const double xr = periodic_offset(x - P[1] - t, P[3]);
      const double yr = periodic_offset(y - P[2] - t, P[4]);
      const double r2 = xr * xr + yr * yr;
      const double amp = eps / (2.0 * M_PI) * exp(0.5 * (1.0 - r2));
      const double T = 1.0 - (gm - 1.0) * eps * eps / (8.0 * gm * M_PI * M_PI) * exp(1.0 - r2);
      const double rho = pow(T, 1.0 / (gm - 1.0));
      prim2cons(dim, gm, rho, 1.0 - amp * yr, 1.0 + amp * xr, rho * T, q);
      return;
    }
    case CRKDG_IC_QUADRANT: {
      const bool east = x >= P[0], north = y >= P[1];
      const int quad = east ? (north ? 0 : 3) : (north ? 1 : 2);  // NE NW SW SE
      const double* s = P + 2 + 4 * quad;
      prim2cons(dim, ph.gamma, s[0], s[1], s[2], s[3], q);
      return;
    }
    case CRKDG_IC_SHOCK: {
      const double cth = cos(P[0]), sth = sin(P[0]);
      if (cth * (x - P[4]) + sth * (y - P[5]) < 0.0) {
        prim2cons(dim, ph.gamma, P[1], P[2] * cth, P[2] * sth, P[3], q);
        return;
      }
      // bilinear interpolation of a cell-centre field on an na x ma grid over
      // the domain (P[8], P[9]; 0: the mesh's own cells), periodic wrap
      const int na = P[8] > 0.0 ? (int)P[8] : g.nx, ma = P[9] > 0.0 ? (int)P[9] : g.ny;
      const double hxa = g.dx * g.nx / na, hya = g.dy * g.ny / ma;
      const double fx = (x - g.x0) / hxa - 0.5, fy = (y - g.y0) / hya - 0.5;
      const double bx = floor(fx), by = floor(fy);
      const double wx = fx - bx, wy = fy - by;
      int i0 = (int)bx % na; if (i0 < 0) i0 += na;
      int j0 = (int)by % ma; if (j0 < 0) j0 += ma;
      const int i1 = i0 + 1 == na ? 0 : i0 + 1, j1 = j0 + 1 == ma ? 0 : j0 + 1;
      const double a00 = aux[(long long)j0 * na + i0], a10 = aux[(long long)j0 * na + i1];
      const double a01 = aux[(long long)j1 * na + i0], a11 = aux[(long long)j1 * na + i1];
      const double xi = (1.0 - wy) * ((1.0 - wx) * a00 + wx * a10) + wy * ((1.0 - wx) * a01 + wx * a11);
      double rho = 1.0 + P[7] * xi;
      if (rho < P[6]) rho = P[6];
      prim2cons(dim, ph.gamma, rho, 0.0, 0.0, 1.0, q);
      return;
    }
    case CRKDG_IC_DMR:
      dmr_state(P, x, y, t, q);
      return;
    default:
      for (int c = 0; c < EQ::NC; ++c) q[c] = __builtin_nan("");
  }
}

// ---------------------------------------------------------------------------
// K1: inner stages (local operator only)
// ---------------------------------------------------------------------------
// occupancy targets (waves per SIMD) for the register-resident step kernels
template <class EQ, int K>
struct Occ {
  static constexpr bool F32 = sizeof(typename EQ::Real) == 4;
  static constexpr int inner = F32 ? INNER_OCC_F32 : INNER_OCC_F64;
  static constexpr int final_ = F32 ? FINAL_OCC_F32 : FINAL_OCC_F64;
};

// LIN: layout of u^n; LOUT: layout of the stored stages; INC: accumulate
// the increments u^(i) - u^n in the compute precision and store u^n + the
// increment in FP64 (the FP32-inner form)
template <class EQ, int K, int LIN, int LOUT, bool INC>
__global__ __launch_bounds__(256, (Occ<EQ, K>::inner)) void k_inner(PhysDev ph, Geo g, InnerArgs a) {
  using R = typename EQ::Real;
  constexpr int NC = EQ::NC, NB = Sizes<K, EQ::DIM>::NB;
  const long long cell = (long long)blockIdx.x * 256 + threadIdx.x;
  if (cell >= g.N) return;
  const EQ eq = make_eq<EQ>(ph);
  const double dt = a.dt_ptr ? *a.dt_ptr : a.dt;
  R u[NC][NB];
  load_state<R, NC, NB, LIN>(a.un, g.N, cell, u);
  // u^n in the compute precision stays in registers when KEEP (every stage
  // starts from it; re-reading it after a stage's arithmetic mostly misses
  // the L2 and doubles the kernel's HBM reads); the FP64 form re-reads it,
  // since another 72 registers would halve its occupancy
  constexpr bool KEEP = INC || sizeof(R) == 4 || INNER_KEEP_F64;
  R un[KEEP ? NC : 1][KEEP ? NB : 1];
  if constexpr (KEEP) {
#pragma unroll
    for (int c = 0; c < NC; ++c)
#pragma unroll
      for (int b = 0; b < NB; ++b) un[c][b] = u[c][b];
  }
#pragma unroll 1
  for (int i = 1; i < a.s; ++i) {
    R acc[NC][NB];
    if constexpr (INC) {
#pragma unroll
      for (int c = 0; c < NC; ++c)
#pragma unroll
        for (int b = 0; b < NB; ++b) acc[c][b] = R(0);
    } else if constexpr (KEEP) {
#pragma unroll
      for (int c = 0; c < NC; ++c)
#pragma unroll
        for (int b = 0; b < NB; ++b) acc[c][b] = un[c][b];
    } else {
      load_state<R, NC, NB, LIN>(a.un, g.N, cell, acc);
    }
    loc_acc<EQ, K, R>(eq, u, R(-dt * a.a_sub[i]), R(g.inv_dx), R(g.inv_dy), acc);
    if constexpr (INC) {
      // acc is the increment; the next stage is evaluated at u^n + acc, and a
      // stored stage is u^n + acc formed in FP64 (one rounding)
#pragma unroll
      for (int c = 0; c < NC; ++c)
#pragma unroll
        for (int b = 0; b < NB; ++b) u[c][b] = un[c][b] + acc[c][b];
      if ((a.store_mask >> i) & 1) {
        static_assert(LIN == L64 && LOUT == L64, "FP64 state and stages");
        const unsigned o8 = (unsigned)cell * 8u;
#pragma unroll
        for (int c = 0; c < NC; ++c) {
          const auto rin = rsrc(byte_add(a.un, (long long)c * NB * g.N * 8));
          const auto rout = rsrc(byte_add(a.stage[i], (long long)c * NB * g.N * 8));
#pragma unroll
          for (int b = 0; b < NB; ++b) {
            const unsigned so = (unsigned)(b * g.N * 8);
            bstore<double>(bload<double>(rin, o8, so) + (double)acc[c][b], rout, o8, so);
          }
        }
      }
    } else {
#pragma unroll
      for (int c = 0; c < NC; ++c)
#pragma unroll
        for (int b = 0; b < NB; ++b) u[c][b] = acc[c][b];
      if ((a.store_mask >> i) & 1) store_state<R, NC, NB, LOUT>(a.stage[i], g.N, cell, u);
    }
  }
}

// ---------------------------------------------------------------------------
// neighbour traces and boundary ghosts for the final stage
// ---------------------------------------------------------------------------
// side: 0 left (want the neighbour's xi=+1 trace), 1 right (its xi=-1 trace),
//       2 bottom (its eta=+1 trace), 3 top (its eta=-1 trace).
// own: this cell's trace on the shared face (used by the transmissive rule).
template <class EQ, int K, int SIDE>
__device__ __forceinline__ void neighbour_trace(const Geo& g, const PhysDev& ph, const BCDev& bc,
                                                const void* __restrict__ S, int i, int j,
                                                double tb,
                                                const typename EQ::Real (&own)[EQ::NC][EQ::DIM == 2 ? K + 1 : 1],
                                                typename EQ::Real (&out)[EQ::NC][EQ::DIM == 2 ? K + 1 : 1]) {
  using R = typename EQ::Real;
  constexpr int NC = EQ::NC, NB = Sizes<K, EQ::DIM>::NB, NP = EQ::DIM == 2 ? K + 1 : 1;
  int ni = i + (SIDE == 0 ? -1 : SIDE == 1 ? 1 : 0);
  int nj = j + (SIDE == 2 ? -1 : SIDE == 3 ? 1 : 0);
  const bool outside = ni < 0 || ni >= g.nx || nj < 0 || nj >= g.ny;
  if (outside) {
    const int type = bc.type[SIDE];
    if (type == CRKDG_BC_TRANSMISSIVE) {
#pragma unroll
      for (int c = 0; c < NC; ++c)
#pragma unroll
        for (int p = 0; p < NP; ++p) out[c][p] = own[c][p];
      return;
    }
    if (type == CRKDG_BC_DIRICHLET) {
      constexpr GTab<K + 1> T = Tab<K + 1>::t;
#pragma unroll
      for (int p = 0; p < NP; ++p) {
        double q[4];
#pragma unroll
        for (int c = 0; c < NC; ++c) q[c] = bc.state[SIDE][c];
        if constexpr (!EQ::EULER) {
          // time-dependent inflow data (advection only): the exact solution
          // sin(x - a t) (1D) / sin(pi(x - a t)) sin(pi(y - b t)) (2D) at the
          // stage time
          if (bc.exact == CRKDG_IC_ADV_SIN) {
            const double xc = g.x0 + (i + 0.5) * g.dx, yc = g.y0 + (j + 0.5) * g.dy;
            double x, y;
            if (SIDE < 2) {
              x = xc + (SIDE == 0 ? -0.5 : 0.5) * g.dx;
              y = EQ::DIM == 2 ? yc + 0.5 * g.dy * T.X[p] : 0.0;
            } else {
              x = xc + 0.5 * g.dx * T.X[p];
              y = yc + (SIDE == 2 ? -0.5 : 0.5) * g.dy;
            }
            q[0] = EQ::DIM == 1 ? sin(x - ph.ax * tb)
                                : sin(M_PI * (x - ph.ax * tb)) * sin(M_PI * (y - ph.ay * tb));
          }
        }
#pragma unroll
        for (int c = 0; c < NC; ++c) out[c][p] = (R)q[c];
      }
      return;
    }
    if (ni < 0) ni += g.nx;
    if (ni >= g.nx) ni -= g.nx;
    if (nj < 0) nj += g.ny;
    if (nj >= g.ny) nj -= g.ny;
  }
  R U[NC][NB];
  load_state<R, NC, NB, StepLayout<EQ>::value>(S, g.N, (long long)nj * g.nx + ni, U);
  if constexpr (SIDE == 0) trace_x<+1, EQ, K, R>(U, out);
  if constexpr (SIDE == 1) trace_x<-1, EQ, K, R>(U, out);
  if constexpr (SIDE == 2) trace_y<+1, EQ, K, R>(U, out);
  if constexpr (SIDE == 3) trace_y<-1, EQ, K, R>(U, out);
}

// ---------------------------------------------------------------------------
// K2 (2D): final stage on a tile of TX x TY cells
// ---------------------------------------------------------------------------
// Tile shape per compute type (measured on the 4096 x 1024 Q2 shock workload:
// 64 x 4 beats 32 x 8 and 16 x 16, whose shorter rows coalesce worse).
template <class R>
struct FinalTile {
  static constexpr int TX = sizeof(R) == 4 ? FINAL_TX_F32 : FINAL_TX_F64;
  static constexpr int TY = sizeof(R) == 4 ? FINAL_TY_F32 : FINAL_TY_F64;
};

// the exterior trace across side `side` (0 left, 1 right, 2 bottom, 3 top) of
// cell (ci, cj): the neighbour's facing trace, or the boundary ghost (Section
// 3.4: boundary data enter only here).  Uses the same trace functions as the
// owner of the neighbour cell, so both tiles sharing a face see identical
// traces and compute identical fluxes.
template <class EQ, int K, int LAY, bool DMRB = false>
__device__ __forceinline__ void halo_trace(const Geo& g, const PhysDev& ph, const BCDev& bc,
                                           const void* __restrict__ S, int side, int ci, int cj,
                                           double tb, typename EQ::Real (&out)[EQ::NC][K + 1]) {
  using R = typename EQ::Real;
  constexpr int NC = EQ::NC, Q = K + 1, NB = Q * Q;
  int ni = ci + (side == 0 ? -1 : side == 1 ? 1 : 0);
  int nj = cj + (side == 2 ? -1 : side == 3 ? 1 : 0);
  int face = side ^ 1;  // the neighbour's face: left side <- its right trace, ...
  // double Mach reflection, bottom side: the reflecting wall takes the cell's
  // own trace (below) with the normal momentum mirrored
  constexpr bool dmr = DMRB && EQ::EULER && EQ::DIM == 2;
  bool wall = false;
  if (ni < 0 || ni >= g.nx || nj < 0 || nj >= g.ny) {
    const int type = bc.type[side];
    if (type == CRKDG_BC_DIRICHLET && !(dmr && side == 2)) {
      constexpr GTab<Q> T = Tab<Q>::t;
#pragma unroll
      for (int p = 0; p < Q; ++p) {
        double q[4];
#pragma unroll
        for (int c = 0; c < NC; ++c) q[c] = bc.state[side][c];
        if constexpr (dmr) {  // the moving shock at the face point and stage time
          const double xc = g.x0 + (ci + 0.5) * g.dx, yc = g.y0 + (cj + 0.5) * g.dy;
          const double x = side < 2 ? xc + (side == 0 ? -0.5 : 0.5) * g.dx : xc + 0.5 * g.dx * T.X[p];
          const double y = side < 2 ? yc + 0.5 * g.dy * T.X[p] : yc + (side == 2 ? -0.5 : 0.5) * g.dy;
          dmr_state(bc.params, x, y, tb, q);
        }
        if constexpr (!EQ::EULER) {
          // time-dependent inflow data (advection): sin(pi(x - a t)) sin(pi(y - b t))
          // at the stage time
          if (bc.exact == CRKDG_IC_ADV_SIN) {
            const double xc = g.x0 + (ci + 0.5) * g.dx, yc = g.y0 + (cj + 0.5) * g.dy;
            const double x = side < 2 ? xc + (side == 0 ? -0.5 : 0.5) * g.dx : xc + 0.5 * g.dx * T.X[p];
            const double y = side < 2 ? yc + 0.5 * g.dy * T.X[p] : yc + (side == 2 ? -0.5 : 0.5) * g.dy;
            q[0] = sin(M_PI * (x - ph.ax * tb)) * sin(M_PI * (y - ph.ay * tb));
          }
        }
#pragma unroll
        for (int c = 0; c < NC; ++c) out[c][p] = (R)q[c];
      }
      return;
    }
    if (type == CRKDG_BC_TRANSMISSIVE || type == CRKDG_BC_DIRICHLET) {
      ni = ci;  // the exterior trace is the cell's own trace on this face
      nj = cj;
      face = side;
      wall = type == CRKDG_BC_DIRICHLET;  // the DMR bottom side
    } else {  // periodic
      if (ni < 0) ni += g.nx;
      if (ni >= g.nx) ni -= g.nx;
      if (nj < 0) nj += g.ny;
      if (nj >= g.ny) nj -= g.ny;
    }
  }
  R U[NC][NB];
  load_state<R, NC, NB, LAY>(S, g.N, (long long)nj * g.nx + ni, U);
  switch (face) {
    case 0: trace_x<-1, EQ, K, R>(U, out); break;
    case 1: trace_x<+1, EQ, K, R>(U, out); break;
    case 2: trace_y<-1, EQ, K, R>(U, out); break;
    default: trace_y<+1, EQ, K, R>(U, out); break;
  }
  if constexpr (dmr) {
    if (wall) {  // before the wall's start the bottom takes the shock data
      constexpr GTab<Q> T = Tab<Q>::t;
      const double xc = g.x0 + (ci + 0.5) * g.dx, yb = g.y0 + cj * g.dy;
#pragma unroll
      for (int p = 0; p < Q; ++p) {
        const double x = xc + 0.5 * g.dx * T.X[p];
        if (x >= bc.params[0]) {
          out[2][p] = -out[2][p];
        } else {
          double q[4];
          dmr_state(bc.params, x, yb, tb, q);
#pragma unroll
          for (int c = 0; c < NC; ++c) out[c][p] = (R)q[c];
        }
      }
    }
  }
}

// face point f of a TX x TY tile: x faces first (TX + 1 per row, TY rows, Q
// points each), then y faces (TX per row, TY + 1 rows); column index fastest,
// quadrature point slowest.  Returns true for a y face.
template <int TX, int TY>
__device__ __forceinline__ bool face_point(int f, int nxp, int& fx, int& fy, int& p) {
  const bool dy = f >= nxp;
  const int e = dy ? f - nxp : f;
  const int w = dy ? TX : TX + 1, h = dy ? TY + 1 : TY;
  fx = e % w;
  const int r = e / w;
  fy = r % h;
  p = r / h;
  return dy;
}

template <class R, int NV, int TX, int TY>
struct FinalSmem {
  // traces of the current stage (R), per face row/column of the tile:
  //   tR[v][y][x]: right trace of cell x-1 (x = 0: the left halo cell's)
  //   tL[v][y][x]: left trace of cell x   (x = nx_tile: the right halo's)
  //   tT[v][y][x]: top trace of cell row y-1 (y = 0: the bottom halo's)
  //   tB[v][y][x]: bottom trace of row y   (y = ny_tile: the top halo's)
  static constexpr int NXF = NV * TY * (TX + 1), NYF = NV * (TY + 1) * TX;
  static constexpr size_t TRACE_BYTES = sizeof(R) * 2 * (NXF + NYF);
  // after the stage loop the same bytes hold the face sums G (FP64)
  static constexpr size_t G_BYTES = sizeof(double) * (NXF + NYF);
  static constexpr size_t BYTES = TRACE_BYTES > G_BYTES ? TRACE_BYTES : G_BYTES;
};

// LAY: layout of u^n, of the stored stages and of u^{n+1}
// B2: the update starts from bw1 base + bw2 st[0] (stages of the original
// RKDG; FinalArgs::base2 is st[0]), folded into the first stage's load.
// DMRB: double Mach reflection boundary data (bc.exact == CRKDG_IC_DMR)
template <class EQ, int K, int LAY, bool B2, bool DMRB>
__global__ __launch_bounds__(FinalTile<typename EQ::Real>::TX * FinalTile<typename EQ::Real>::TY,
                             (Occ<EQ, K>::final_)) void k_final2(PhysDev ph, Geo g, BCDev bc,
                                                                 FinalArgs a) {
  using R = typename EQ::Real;
  constexpr int TX = FinalTile<R>::TX, TY = FinalTile<R>::TY, NT = TX * TY;
  constexpr int Q = K + 1, NC = EQ::NC, NB = Q * Q, NV = NC * Q;
  using SM = FinalSmem<R, NV, TX, TY>;
  // face points of the tile: x faces (TX + 1 per row, TY rows), then y faces
  constexpr int NXP = Q * (TX + 1) * TY, NFP = NXP + Q * TX * (TY + 1);
  constexpr int NPASS = (NFP + NT - 1) / NT;
  constexpr int NHALO = 2 * TY + 2 * TX;
  static_assert(NHALO <= NT, "one lane per halo cell");
  __shared__ __attribute__((aligned(16))) char smem[SM::BYTES];
  R(*tR)[TY][TX + 1] = reinterpret_cast<R(*)[TY][TX + 1]>(smem);
  R(*tL)[TY][TX + 1] = reinterpret_cast<R(*)[TY][TX + 1]>(smem + sizeof(R) * SM::NXF);
  R(*tT)[TY + 1][TX] = reinterpret_cast<R(*)[TY + 1][TX]>(smem + sizeof(R) * 2 * SM::NXF);
  R(*tB)[TY + 1][TX] = reinterpret_cast<R(*)[TY + 1][TX]>(smem + sizeof(R) * (2 * SM::NXF + SM::NYF));
  double(*gx)[TY][TX + 1] = reinterpret_cast<double(*)[TY][TX + 1]>(smem);
  double(*gy)[TY + 1][TX] = reinterpret_cast<double(*)[TY + 1][TX]>(smem + sizeof(double) * SM::NXF);
  // flat views: component c of face point e at c * CSX + e (x) / c * CSY + e (y)
  constexpr int CSX = Q * TY * (TX + 1), CSY = Q * (TY + 1) * TX;
  const R* tRf = &tR[0][0][0];
  const R* tLf = &tL[0][0][0];
  const R* tTf = &tT[0][0][0];
  const R* tBf = &tB[0][0][0];
  double* gxf = &gx[0][0][0];
  double* gyf = &gy[0][0][0];

  const int tid = threadIdx.x, tx = tid % TX, ty = tid / TX;
  const int i0 = blockIdx.x * TX, j0 = blockIdx.y * TY;
  const int nax = min(TX, g.nx - i0), nay = min(TY, g.ny - j0);
  const int i = i0 + tx, j = j0 + ty;
  const bool active = tx < nax && ty < nay;
  const bool full = nax == TX && nay == TY;
  const long long cell = (long long)j * g.nx + i;
  const EQ eq = make_eq<EQ>(ph);
  const double dt = a.dt_ptr ? *a.dt_ptr : a.dt;

  // this lane's halo cell: bottom row, top row, then the left and right
  // columns, so that with TX = 64 each halo wave runs one trace variant
  int hside = -1, hci = 0, hcj = 0, hslot = 0;
  if (tid < TX) {
    hside = tid < nax ? 2 : -1; hci = i0 + tid; hcj = j0; hslot = tid;
  } else if (tid < 2 * TX) {
    hside = tid - TX < nax ? 3 : -1; hci = i0 + tid - TX; hcj = j0 + nay - 1; hslot = tid - TX;
  } else if (tid < 2 * TX + TY) {
    hside = tid - 2 * TX < nay ? 0 : -1; hci = i0; hcj = j0 + tid - 2 * TX; hslot = tid - 2 * TX;
  } else if (tid < NHALO) {
    hside = tid - 2 * TX - TY < nay ? 1 : -1; hci = i0 + nax - 1; hcj = j0 + tid - 2 * TX - TY;
    hslot = tid - 2 * TX - TY;
  }

  // FP32 arithmetic on the FP64 layout: acc holds the increment over u^n
  // (FP32), added to u^n in FP64 at the store (the FP32-increments form)
  constexpr bool INC = LAY == L64 && sizeof(R) == 4;
  static_assert(!(INC && B2), "the original RKDG runs in FP64");
  R acc[NC][NB];
  double a0[NC];  // cell averages, FP64
#pragma unroll
  for (int c = 0; c < NC; ++c) {
#pragma unroll
    for (int b = 0; b < NB; ++b) acc[c][b] = R(0);
    a0[c] = 0.0;
  }
  // u^n is usually also the first final-stage state (u^(1) = u^n): then it is
  // read once, in the stage loop
  const bool base_is_st0 = !INC && a.base != nullptr && a.ns > 0 && a.base == a.st[0];
  if (active && a.base) {
    if (!INC && !base_is_st0) load_state<R, NC, NB, LAY>(a.base, g.N, cell, acc);
#pragma unroll
    for (int c = 0; c < NC; ++c) a0[c] = load_avg<NC, NB, LAY>(a.base, g.N, c, cell);
  }
  // FP64 stage-weighted face flux sums G = sum_i b_i F^(i) (equation (g)) of
  // the face points this lane evaluates
  double Gp[NPASS][NC];
#pragma unroll
  for (int k = 0; k < NPASS; ++k)
#pragma unroll
    for (int c = 0; c < NC; ++c) Gp[k][c] = 0.0;

#pragma unroll 1
  for (int s = 0; s < a.ns; ++s) {
    const void* __restrict__ S = a.st[s];
    const double w = a.w[s];
    if (active) {
      R U[NC][NB];
      load_state<R, NC, NB, LAY>(S, g.N, cell, U);
      if (s == 0 && base_is_st0) {
#pragma unroll
        for (int c = 0; c < NC; ++c)
#pragma unroll
          for (int b = 0; b < NB; ++b) acc[c][b] = U[c][b];
      }
      if constexpr (B2) {  // the update starts from bw1 base + bw2 st[0]
        if (s == 0) {
          const R w1 = R(a.bw1), w2 = R(a.bw2);
#pragma unroll
          for (int c = 0; c < NC; ++c) {
#pragma unroll
            for (int b = 0; b < NB; ++b) acc[c][b] = w1 * acc[c][b] + w2 * U[c][b];
            a0[c] = a.bw1 * a0[c] + a.bw2 * load_avg<NC, NB, LAY>(S, g.N, c, cell);
          }
        }
      }
      const R vs = R(0.5 * dt * w);
      volume_acc<EQ, K, R>(eq, U, vs * R(g.inv_dx), vs * R(g.inv_dy), acc);
      R t[NC][Q];
      trace_x<+1, EQ, K, R>(U, t);
#pragma unroll
      for (int c = 0; c < NC; ++c)
#pragma unroll
        for (int p = 0; p < Q; ++p) tR[c * Q + p][ty][tx + 1] = t[c][p];
      trace_x<-1, EQ, K, R>(U, t);
#pragma unroll
      for (int c = 0; c < NC; ++c)
#pragma unroll
        for (int p = 0; p < Q; ++p) tL[c * Q + p][ty][tx] = t[c][p];
      trace_y<+1, EQ, K, R>(U, t);
#pragma unroll
      for (int c = 0; c < NC; ++c)
#pragma unroll
        for (int p = 0; p < Q; ++p) tT[c * Q + p][ty + 1][tx] = t[c][p];
      trace_y<-1, EQ, K, R>(U, t);
#pragma unroll
      for (int c = 0; c < NC; ++c)
#pragma unroll
        for (int p = 0; p < Q; ++p) tB[c * Q + p][ty][tx] = t[c][p];
    }
    if (hside >= 0) {
      R h[NC][Q];
      const double tb = a.t_ptr ? *a.t_ptr + a.cst[s] * dt : a.tst[s];
      halo_trace<EQ, K, LAY, DMRB>(g, ph, bc, S, hside, hci, hcj, tb, h);
#pragma unroll
      for (int c = 0; c < NC; ++c)
#pragma unroll
        for (int p = 0; p < Q; ++p) {
          const int v = c * Q + p;
          if (hside == 0) tR[v][hslot][0] = h[c][p];
          else if (hside == 1) tL[v][hslot][nax] = h[c][p];
          else if (hside == 2) tT[v][0][hslot] = h[c][p];
          else tB[v][nay][hslot] = h[c][p];
        }
    }
    __syncthreads();
    // every face point of the tile once: qL from the cell below / to the
    // left, qR from the cell above / to the right.  With the column index
    // fastest, the face point's index is its offset in the trace arrays, and
    // consecutive lanes read consecutive LDS words (no bank conflicts).
#pragma unroll
    for (int k = 0; k < NPASS; ++k) {
      const int f = tid + k * NT;
      if (f >= NFP) break;
      const bool dy = f >= NXP;
      const int e = dy ? f - NXP : f;
      bool valid = full;
      if (!full) {
        int fx, fy, p;
        face_point<TX, TY>(f, NXP, fx, fy, p);
        valid = dy ? (fx < nax && fy <= nay) : (fx <= nax && fy < nay);
      }
      if (valid) {
        const R* A = dy ? tTf : tRf;
        const R* B = dy ? tBf : tLf;
        const int cs = dy ? CSY : CSX;
        R qa[NC], qb[NC], F[NC];
#pragma unroll
        for (int c = 0; c < NC; ++c) {
          qa[c] = A[c * cs + e];
          qb[c] = B[c * cs + e];
        }
        eq.num_flux_d(qa, qb, dy, F);
#pragma unroll
        for (int c = 0; c < NC; ++c) Gp[k][c] += w * (double)F[c];
      }
    }
    __syncthreads();
  }
  // face sums to LDS (over the traces), then each cell reads its four faces
#pragma unroll
  for (int k = 0; k < NPASS; ++k) {
    const int f = tid + k * NT;
    if (f >= NFP) break;
    const bool dy = f >= NXP;
    const int e = dy ? f - NXP : f;
    double* G = dy ? gyf : gxf;
    const int cs = dy ? CSY : CSX;
#pragma unroll
    for (int c = 0; c < NC; ++c) G[c * cs + e] = Gp[k][c];
  }
  __syncthreads();
  if (!active) return;
  double GL[NC][Q], GR[NC][Q], GB[NC][Q], GT[NC][Q];
#pragma unroll
  for (int c = 0; c < NC; ++c)
#pragma unroll
    for (int p = 0; p < Q; ++p) {
      GL[c][p] = gx[c * Q + p][ty][tx];
      GR[c][p] = gx[c * Q + p][ty][tx + 1];
      GB[c][p] = gy[c * Q + p][ty][tx];
      GT[c][p] = gy[c * Q + p][ty + 1][tx];
    }
  // cell averages: FP64 update from the FP64 face sums (equation (avg))
  {
    constexpr GTab<Q> T = Tab<Q>::t;
    const double lx = -0.5 * dt * g.inv_dx, ly = -0.5 * dt * g.inv_dy;
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      double sx = 0.0, sy = 0.0;
#pragma unroll
      for (int p = 0; p < Q; ++p) {
        sx += T.W[p] * (GR[c][p] - GL[c][p]);
        sy += T.W[p] * (GT[c][p] - GB[c][p]);
      }
      a0[c] += lx * sx + ly * sy;
    }
  }
  // higher modes in the compute precision
  {
    R gr[NC][Q], gl[NC][Q];
#pragma unroll
    for (int c = 0; c < NC; ++c)
#pragma unroll
      for (int p = 0; p < Q; ++p) {
        gr[c][p] = (R)GR[c][p];
        gl[c][p] = (R)GL[c][p];
      }
    lift_x<EQ, K, R>(gr, gl, R(-0.5 * dt * g.inv_dx), acc);
#pragma unroll
    for (int c = 0; c < NC; ++c)
#pragma unroll
      for (int p = 0; p < Q; ++p) {
        gr[c][p] = (R)GT[c][p];
        gl[c][p] = (R)GB[c][p];
      }
    lift_y<EQ, K, R>(gr, gl, R(-0.5 * dt * g.inv_dy), acc);
  }
  if constexpr (INC) {
    // u^{n+1} = u^n + increment, formed in FP64 (one rounding per mode)
    const unsigned o8 = (unsigned)cell * 8u;
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      const auto rin = rsrc(byte_add(a.base, (long long)c * NB * g.N * 8));
      const auto rout = rsrc(byte_add(a.out, (long long)c * NB * g.N * 8));
      bstore<double>(a0[c], rout, o8, 0u);
#pragma unroll
      for (int b = 1; b < NB; ++b) {
        const unsigned so = (unsigned)(b * g.N * 8);
        bstore<double>(bload<double>(rin, o8, so) + (double)acc[c][b], rout, o8, so);
      }
    }
  } else {
    store_state<R, NC, NB, LAY>(a.out, g.N, cell, acc, a0);
  }
}

// ---------------------------------------------------------------------------
// K14: the whole step in one pass (the compact stencil of Section 3.1)
// ---------------------------------------------------------------------------
// A cRKDG step reaches only the face neighbours of a cell, whatever the
// number of stages: the inner stages are element local and only the final
// stage couples neighbours (Section 3.1).  So a workgroup can read u^n of
// its cells plus a one-cell ring, compute every inner stage of the ring cells
// itself, evaluate the shared faces, and write u^{n+1}: one read of u^n and
// one write of u^{n+1} per step, no stage state in memory.
//
// A workgroup of four wavefronts walks up a strip of 62 columns: wavefront w
// holds row 4t + w in iteration t, one lane per cell of a 64-cell row (the 62
// owned cells and the two ring cells).  Walking reuses each row's traces for
// the face above it, so only the strip's two end rows and the two ring
// columns are recomputed ((H + 2) / H x 64 / 62 of the work for a strip of H
// rows).  A ring cell outside the mesh has no lane work: across a
// non-periodic side the boundary face takes the boundary rule (transmissive:
// the owned cell's own trace; Dirichlet: the boundary state).  Every face is
// evaluated in canonical (+x / +y) orientation; a face shared with another
// strip is evaluated by both with the same code on the same traces (a ring
// cell's inner stages are computed by the same instructions as by its
// owner), so both see the same bits and the FP64 cell averages stay
// conservative (equation (avg)).  Per iteration:
//   P1  (no barrier) u^n and the inner stages (register chain); the first
//       inner stage and the first final-stage term share u^n's volume
//       integral; the volume terms of u^n and u^(s); the x faces of the row:
//       right traces pass to the next lane by a lane shift, a lane evaluates
//       its left face and passes the stage-weighted flux G = sum_i b_i F^(i)
//       (equation (g)) back for its left neighbour's right face; the row's
//       top traces (of u^n and u^(s)) go to the row's LDS slot, its bottom
//       traces stay in registers;
//   P2  (after a barrier) the face below each row: the row's own bottom
//       traces against the top traces of the row below; G lifts into the
//       row's own update as its bottom face and goes to LDS, over the traces
//       it has read, for the row below as its top face;
//   P3  (after a barrier) rows 4t .. 4t + 2 take their top face and are
//       stored; row 4t + 3 waits in LDS for the face the next iteration's
//       first wavefront evaluates, and is stored then.
// Slots: wavefronts 0 - 2 own slots 0 - 2; wavefront 3 alternates between
// slots 3 and 4, so that its row's traces survive into the next iteration's
// P2 while the next iteration's wavefront 3 writes its own.  While the inner
// stages run, a wavefront's own next slot holds the update's share of the
// volume integral.  The tableau must have nonzero weights b_i only on the
// first and last stages (scheme (eq:2), scheme (eq:3), forward Euler), so
// that at most u^n and u^(s) are live; the split kernels take the others.
// Tuning (measured on the 4096 x 1024 Q2 shock workload): strips of 30 rows
// (46 the same; 14 and 62 slower: more recomputed rows, or too few
// workgroups for an even last wave), and two wavefronts per SIMD: the kernel
// needs 221 registers, and forcing three (168 registers) spills 53 values and
// ran 1.8x slower.  The FP64 form (Real = double, the same code) needs 419
// registers (256 VGPRs and 163 AGPRs) and 104 KB of LDS: one wavefront per
// SIMD, and still 27% faster than the split FP64 kernels.
// Strip order: workgroups reach the eight XCDs in turn, so in launch order
// neighbouring strips land in different L2s and each fetches the 128-byte
// lines at their shared edge (a 64-cell row of FP32 modes starts one cell
// before a line): u^n was read 1.63 times.  Runs of 16 neighbouring strips
// per XCD read it 1.12 times and run 1% faster; one contiguous block per XCD
// read it 1.09 times but ran 4% slower.
#ifndef MARCH_H
#define MARCH_H 30
#endif
#ifndef MARCH_OCC
#define MARCH_OCC 2
#endif
#ifndef MARCH_XCD
#define MARCH_XCD 16
#endif

template <class R, int NC, int Q>
struct MarchSmem {
  static constexpr int NB = Q * Q;
  static constexpr int TRACES = 2 * NC * Q * 64;    // top traces of both states, [s][c][p][lane]
  static constexpr int SHARE = NC * (NB - 1) * 64;  // the update's volume share, [c][mode][lane]
  static constexpr int SLOTF = TRACES > SHARE ? TRACES : SHARE;
  static constexpr int NSLOT = 5;
  // the parked row: FP64 averages [c][lane], higher modes [c][mode][lane],
  // the bottom-face G [c][p][lane]
  static constexpr size_t PARK_BYTES = sizeof(double) * NC * 64 + sizeof(R) * (NC * (NB - 1) + NC * Q) * 64;
  static constexpr size_t BYTES = PARK_BYTES + sizeof(R) * NSLOT * SLOTF;
};

__device__ __forceinline__ int march_slot(int ry) {
  return (ry & 3) == 3 ? 3 + ((ry >> 2) & 1) : (ry & 3);
}

template <class EQ, int K>
__global__ __launch_bounds__(256, sizeof(typename EQ::Real) == 8 ? 1 : MARCH_OCC) void k_fused2(
    PhysDev ph, Geo g, BCDev bc, FusedArgs a) {
  using R = typename EQ::Real;
  constexpr int LAY = StepLayout<EQ>::value;
  constexpr int Q = K + 1, NC = EQ::NC, NB = Q * Q;
  using SM = MarchSmem<R, NC, Q>;
  constexpr GTab<Q> T = Tab<Q>::t;
  __shared__ __attribute__((aligned(16))) char smem[SM::BYTES];
  double* pa0 = reinterpret_cast<double*>(smem);                  // [NC][64]
  R* pfin = reinterpret_cast<R*>(smem + sizeof(double) * NC * 64);  // [NC * (NB - 1)][64]
  R* pgb = pfin + NC * (NB - 1) * 64;                               // [NC * Q][64]
  R* slots = reinterpret_cast<R*>(smem + SM::PARK_BYTES);           // [NSLOT][SLOTF]

  const int lx = threadIdx.x & 63, w = threadIdx.x >> 6;
#if MARCH_XCD
  // workgroups go to the eight XCDs in turn; give each XCD runs of
  // MARCH_XCD neighbouring strips, so that the lines at their shared edges
  // and ring columns meet in the same L2
  int bxs, bys;
  {
    const unsigned gx = gridDim.x, tot = gx * gridDim.y;
    const unsigned w = blockIdx.x + blockIdx.y * gx;
    constexpr unsigned L = MARCH_XCD, BLK = 8u * L;
    const unsigned lg = w < (tot / BLK) * BLK ? (w / BLK) * BLK + (w & 7u) * L + (w >> 3) % L : w;
    bxs = (int)(lg % gx);
    bys = (int)(lg / gx);
  }
  const int i0 = bxs * 62, j0 = bys * a.strip;
#else
  const int i0 = blockIdx.x * 62, j0 = blockIdx.y * a.strip;
#endif
  const int nax = min(62, g.nx - i0), nh = min(a.strip, g.ny - j0);
  const int nrows = nh + 2, niter = (nrows + 3) / 4;
  const EQ eq = make_eq<EQ>(ph);
  const double dt = a.dt_ptr ? *a.dt_ptr : a.dt;
  const bool share_vol = a.s > 1 && a.w_first != 0.0;
  const R wf = R(a.w_first), wl = R(a.w_last);
  const double lxs = -0.5 * dt * g.inv_dx, lys = -0.5 * dt * g.inv_dy;
  const bool perx = bc.type[0] == CRKDG_BC_PERIODIC, pery = bc.type[2] == CRKDG_BC_PERIODIC;
  // the lane's column: owned (1 .. nax), ring (0, nax + 1) or unused
  const bool colown = lx >= 1 && lx <= nax;
  int i = i0 - 1 + lx;
  bool colhas = colown;  // a ring column holds cells inside the mesh or across a periodic side
  if (lx == 0 || lx == nax + 1) {
    colhas = (i >= 0 && i < g.nx) || perx;
    if (i < 0) i += g.nx;
    if (i >= g.nx) i -= g.nx;
  }
  // the left neighbour lane's column (for the lane's left face)
  const bool lefthas = lx >= 2 ? true : (lx == 1 ? ((i0 - 1 >= 0) || perx) : false);
  const bool bl = colown && i == 0 && !perx, br = colown && i == g.nx - 1 && !perx;

#pragma unroll 1
  for (int t = 0; t < niter; ++t) {
    const int ry = 4 * t + w;
    const bool rowvalid = ry < nrows;
    const bool rowown = ry >= 1 && ry <= nh;
    int j = j0 - 1 + ry;
    bool rowhas = rowown;
    if (rowvalid && !rowown) {
      rowhas = (j >= 0 && j < g.ny) || pery;
      if (j < 0) j += g.ny;
      if (j >= g.ny) j -= g.ny;
    }
    // ring rows hold only the owned columns; ring columns only owned rows
    const bool has = rowvalid && ((rowown && colhas && (colown || lx == 0 || lx == nax + 1)) ||
                                  (!rowown && rowhas && colown));
    const bool owned = rowown && colown;
    const long long cell = (long long)j * g.nx + i;
    const bool bb = owned && j == 0 && !pery, bt = owned && j == g.ny - 1 && !pery;
    R* slot = slots + march_slot(ry) * SM::SLOTF;

    // ---- P1: inner stages, x faces, traces ----
    R un[NC][NB], u[NC][NB];
#pragma unroll
    for (int c = 0; c < NC; ++c)
#pragma unroll
      for (int b = 0; b < NB; ++b) u[c][b] = R(0);
    if (has) load_state<R, NC, NB, LAY>(a.un, g.N, cell, un);
    else {
#pragma unroll
      for (int c = 0; c < NC; ++c)
#pragma unroll
        for (int b = 0; b < NB; ++b) un[c][b] = R(0);
    }
    if (has && a.s > 1) {
      R acc[NC][NB];
      if (share_vol) {
        R Z[NC][NB];
#pragma unroll
        for (int c = 0; c < NC; ++c)
#pragma unroll
          for (int b = 0; b < NB; ++b) Z[c][b] = R(0);
        volume_acc<EQ, K, R>(eq, un, R(g.inv_dx), R(g.inv_dy), Z);
        const R ci = R(0.5 * dt * a.a_sub[1]), cf = R(0.5 * dt * a.w_first);
#pragma unroll
        for (int c = 0; c < NC; ++c)
#pragma unroll
          for (int b = 0; b < NB; ++b) {
            acc[c][b] = un[c][b] + ci * Z[c][b];
            if (b > 0) slot[(c * (NB - 1) + b - 1) * 64 + lx] = un[c][b] + cf * Z[c][b];
          }
        loc_face_acc2<EQ, K, R>(eq, un, R(-dt * a.a_sub[1]), R(g.inv_dx), R(g.inv_dy), acc);
      } else {
#pragma unroll
        for (int c = 0; c < NC; ++c)
#pragma unroll
          for (int b = 0; b < NB; ++b) acc[c][b] = un[c][b];
        loc_acc<EQ, K, R>(eq, un, R(-dt * a.a_sub[1]), R(g.inv_dx), R(g.inv_dy), acc);
      }
#pragma unroll
      for (int c = 0; c < NC; ++c)
#pragma unroll
        for (int b = 0; b < NB; ++b) u[c][b] = acc[c][b];
#pragma unroll 1
      for (int st = 2; st < a.s; ++st) {
#pragma unroll
        for (int c = 0; c < NC; ++c)
#pragma unroll
          for (int b = 0; b < NB; ++b) acc[c][b] = un[c][b];
        loc_acc<EQ, K, R>(eq, u, R(-dt * a.a_sub[st]), R(g.inv_dx), R(g.inv_dy), acc);
#pragma unroll
        for (int c = 0; c < NC; ++c)
#pragma unroll
          for (int b = 0; b < NB; ++b) u[c][b] = acc[c][b];
      }
    }
    // the update of an owned cell (higher modes in FP32, averages in FP64)
    R fin[NC][NB];
    double a0[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) {
#pragma unroll
      for (int b = 0; b < NB; ++b)
        fin[c][b] = share_vol && has && b > 0 ? slot[(c * (NB - 1) + b - 1) * 64 + lx] : un[c][b];
      a0[c] = owned ? load_avg<NC, NB, LAY>(a.un, g.N, c, cell) : 0.0;
    }
    if (owned) {
      if (!share_vol && a.w_first != 0.0) {
        const R vs = R(0.5 * dt * a.w_first);
        volume_acc<EQ, K, R>(eq, un, vs * R(g.inv_dx), vs * R(g.inv_dy), fin);
      }
      if (a.w_last != 0.0) {
        const R vs = R(0.5 * dt * a.w_last);
        volume_acc<EQ, K, R>(eq, u, vs * R(g.inv_dx), vs * R(g.inv_dy), fin);
      }
    }
    // x faces of an owned row: lane L evaluates the face between lanes L - 1
    // and L (L = 1 .. nax + 1), both final-stage states
    R Gx[NC][Q];
#pragma unroll
    for (int c = 0; c < NC; ++c)
#pragma unroll
      for (int p = 0; p < Q; ++p) Gx[c][p] = R(0);
    if (rowown) {
      auto xface = [&](const R(&U)[NC][NB], const R wgt) {
        R tr[NC][Q], tl[NC][Q];
        trace_x<+1, EQ, K, R>(U, tr);
        trace_x<-1, EQ, K, R>(U, tl);
#pragma unroll
        for (int p = 0; p < Q; ++p) {
          R A[NC], B[NC], F[NC];
#pragma unroll
          for (int c = 0; c < NC; ++c) A[c] = __shfl_up(tr[c][p], 1);
          if (lx >= 1 && lx <= nax + 1) {
#pragma unroll
            for (int c = 0; c < NC; ++c) {
              if (!lefthas) A[c] = bc.type[0] == CRKDG_BC_TRANSMISSIVE ? tl[c][p] : (R)bc.state[0][c];
              B[c] = has ? tl[c][p] : (bc.type[1] == CRKDG_BC_TRANSMISSIVE ? A[c] : (R)bc.state[1][c]);
            }
            eq.num_flux_d(A, B, false, F);
#pragma unroll
            for (int c = 0; c < NC; ++c) Gx[c][p] = Gx[c][p] + wgt * F[c];
          }
        }
      };
      if (a.w_first != 0.0) xface(un, wf);
      if (a.w_last != 0.0) xface(u, wl);
    }
    {
      // the right face's G is the right neighbour lane's left-face G
      R GR[NC][Q];
#pragma unroll
      for (int c = 0; c < NC; ++c)
#pragma unroll
        for (int p = 0; p < Q; ++p) GR[c][p] = __shfl_down(Gx[c][p], 1);
      if (owned) {
#pragma unroll
        for (int c = 0; c < NC; ++c) {
          double sx = 0.0;
#pragma unroll
          for (int p = 0; p < Q; ++p) sx += T.W[p] * ((double)GR[c][p] - (double)Gx[c][p]);
          a0[c] += lxs * sx;
        }
        lift_x<EQ, K, R>(GR, Gx, R(lxs), fin);
      }
    }
    // top traces to the row's slot (the share read back above), bottom
    // traces kept for P2
    R tb[2][NC][Q];
#pragma unroll
    for (int s2 = 0; s2 < 2; ++s2)
#pragma unroll
      for (int c = 0; c < NC; ++c)
#pragma unroll
        for (int p = 0; p < Q; ++p) tb[s2][c][p] = R(0);
    if (has && colown) {
      R tt[NC][Q];
      trace_y<+1, EQ, K, R>(un, tt);
#pragma unroll
      for (int c = 0; c < NC; ++c)
#pragma unroll
        for (int p = 0; p < Q; ++p) slot[((0 * NC + c) * Q + p) * 64 + lx] = tt[c][p];
      trace_y<+1, EQ, K, R>(u, tt);
#pragma unroll
      for (int c = 0; c < NC; ++c)
#pragma unroll
        for (int p = 0; p < Q; ++p) slot[((1 * NC + c) * Q + p) * 64 + lx] = tt[c][p];
      trace_y<-1, EQ, K, R>(un, tb[0]);
      trace_y<-1, EQ, K, R>(u, tb[1]);
    }
    __syncthreads();  // B1: every row's top traces are in its slot

    // ---- P2: the face below each row ----
    R GB[NC][Q];
#pragma unroll
    for (int c = 0; c < NC; ++c)
#pragma unroll
      for (int p = 0; p < Q; ++p) GB[c][p] = R(0);
    if (rowvalid && ry >= 1 && colown) {
      R* below = slots + march_slot(ry - 1) * SM::SLOTF;
      const bool lowhas = ry - 1 >= 1 || ((j0 - 1 >= 0) || pery);  // row ry - 1 holds cells
      const bool uphas = has;
#pragma unroll
      for (int p = 0; p < Q; ++p) {
        R G[NC];
#pragma unroll
        for (int c = 0; c < NC; ++c) G[c] = R(0);
#pragma unroll
        for (int s2 = 0; s2 < 2; ++s2) {
          const R wgt = s2 == 0 ? wf : wl;
          if (wgt == R(0)) continue;
          R A[NC], B[NC], F[NC];
#pragma unroll
          for (int c = 0; c < NC; ++c) {
            A[c] = lowhas ? below[((s2 * NC + c) * Q + p) * 64 + lx]
                          : (bc.type[2] == CRKDG_BC_TRANSMISSIVE ? tb[s2][c][p] : (R)bc.state[2][c]);
            B[c] = uphas ? tb[s2][c][p]
                         : (bc.type[3] == CRKDG_BC_TRANSMISSIVE ? A[c] : (R)bc.state[3][c]);
          }
          eq.num_flux_d(A, B, true, F);
#pragma unroll
          for (int c = 0; c < NC; ++c) G[c] = G[c] + wgt * F[c];
        }
#pragma unroll
        for (int c = 0; c < NC; ++c) GB[c][p] = G[c];
      }
      // the lane has read the traces below; its G is the top face of that
      // row (same lane column of the same slot)
      if (ry - 1 >= 1) {
#pragma unroll
        for (int c = 0; c < NC; ++c)
#pragma unroll
          for (int p = 0; p < Q; ++p) below[(c * Q + p) * 64 + lx] = GB[c][p];
      }
    }
    __syncthreads();  // B2: every face's G is known

    // ---- P3: rows whose top face is known are stored ----
    auto finish = [&](R(&f)[NC][NB], double(&av)[NC], const R(&gb)[NC][Q], const R* gtop,
                      long long cl) {
      R GT[NC][Q];
#pragma unroll
      for (int c = 0; c < NC; ++c)
#pragma unroll
        for (int p = 0; p < Q; ++p) GT[c][p] = gtop[(c * Q + p) * 64 + lx];
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        double sy = 0.0;
#pragma unroll
        for (int p = 0; p < Q; ++p) sy += T.W[p] * ((double)GT[c][p] - (double)gb[c][p]);
        av[c] += lys * sy;
      }
      lift_y<EQ, K, R>(GT, gb, R(lys), f);
      store_state<R, NC, NB, LAY>(a.out, g.N, cl, f, av);
    };
    if (w == 3) {
      // the row parked by the previous iteration's wavefront 3: its top face
      // is the face this iteration's wavefront 0 evaluated
      if (t > 0) {
        const int rp = ry - 4;
        if (rp >= 1 && rp <= nh && colown) {
          R f[NC][NB], gb[NC][Q];
          double av[NC];
          int jp = j0 - 1 + rp;
#pragma unroll
          for (int c = 0; c < NC; ++c) {
            av[c] = pa0[c * 64 + lx];
            f[c][0] = R(0);
#pragma unroll
            for (int b = 1; b < NB; ++b) f[c][b] = pfin[(c * (NB - 1) + b - 1) * 64 + lx];
#pragma unroll
            for (int p = 0; p < Q; ++p) gb[c][p] = pgb[(c * Q + p) * 64 + lx];
          }
          finish(f, av, gb, slots + march_slot(rp) * SM::SLOTF, (long long)jp * g.nx + i);
        }
      }
      if (owned) {  // park this row until the next iteration
#pragma unroll
        for (int c = 0; c < NC; ++c) {
          pa0[c * 64 + lx] = a0[c];
#pragma unroll
          for (int b = 1; b < NB; ++b) pfin[(c * (NB - 1) + b - 1) * 64 + lx] = fin[c][b];
#pragma unroll
          for (int p = 0; p < Q; ++p) pgb[(c * Q + p) * 64 + lx] = GB[c][p];
        }
      }
    } else if (owned) {
      finish(fin, a0, GB, slot, cell);
    }
  }
}

// ---------------------------------------------------------------------------
// K2 (1D): final stage on a row of 256 cells (FP64 only)
// ---------------------------------------------------------------------------
constexpr int B1 = 256;

template <class EQ, int K>
__global__ __launch_bounds__(B1) void k_final1(PhysDev ph, Geo g, BCDev bc, FinalArgs a) {
  using R = typename EQ::Real;
  constexpr int NC = EQ::NC, NB = K + 1;
  __shared__ R sR[NC][B1 + 1];
  const int tx = threadIdx.x;
  const int i = blockIdx.x * B1 + tx;
  const bool active = i < g.nx;
  const bool last_col = active && (tx == B1 - 1 || i == g.nx - 1);
  const EQ eq = make_eq<EQ>(ph);
  const double dt = a.dt_ptr ? *a.dt_ptr : a.dt;
  R acc[NC][NB], GL[NC][1], GR[NC][1];
#pragma unroll
  for (int c = 0; c < NC; ++c) {
#pragma unroll
    for (int b = 0; b < NB; ++b) acc[c][b] = 0.0;
    GL[c][0] = GR[c][0] = 0.0;
  }
  if (active && a.base) load_state<R, NC, NB, L64>(a.base, g.N, i, acc);
  if (active && a.base && a.base2) {  // bw1 base + bw2 base2
    R U2[NC][NB];
    load_state<R, NC, NB, L64>(a.base2, g.N, i, U2);
#pragma unroll
    for (int c = 0; c < NC; ++c)
#pragma unroll
      for (int b = 0; b < NB; ++b) acc[c][b] = R(a.bw1) * acc[c][b] + R(a.bw2) * U2[c][b];
  }
#pragma unroll 1
  for (int s = 0; s < a.ns; ++s) {
    const void* __restrict__ S = a.st[s];
    const R w = a.w[s];
    const double tb = a.t_ptr ? *a.t_ptr + a.cst[s] * dt : a.tst[s];
    R tL[NC][1], tR[NC][1], tRn[NC][1];
    if (active) {
      R U[NC][NB];
      load_state<R, NC, NB, L64>(S, g.N, i, U);
      volume_acc<EQ, K, R>(eq, U, dt * w * R(g.inv_dx), R(0), acc);
      trace_x<+1, EQ, K, R>(U, tR);
      trace_x<-1, EQ, K, R>(U, tL);
#pragma unroll
      for (int c = 0; c < NC; ++c) sR[c][tx + 1] = tR[c][0];
      if (tx == 0) {
        R h[NC][1];
        neighbour_trace<EQ, K, 0>(g, ph, bc, S, i, 0, tb, tL, h);
#pragma unroll
        for (int c = 0; c < NC; ++c) sR[c][0] = h[c][0];
      }
      if (last_col) neighbour_trace<EQ, K, 1>(g, ph, bc, S, i, 0, tb, tR, tRn);
    }
    __syncthreads();
    if (active) {
      R qa[NC], qb[NC], F[NC];
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        qa[c] = sR[c][tx];
        qb[c] = tL[c][0];
      }
      eq.template num_flux<0>(qa, qb, F);
#pragma unroll
      for (int c = 0; c < NC; ++c) GL[c][0] = GL[c][0] + w * F[c];
      if (last_col) {
#pragma unroll
        for (int c = 0; c < NC; ++c) {
          qa[c] = tR[c][0];
          qb[c] = tRn[c][0];
        }
        eq.template num_flux<0>(qa, qb, F);
#pragma unroll
        for (int c = 0; c < NC; ++c) GR[c][0] = GR[c][0] + w * F[c];
      }
    }
    __syncthreads();
  }
  if (active) {
#pragma unroll
    for (int c = 0; c < NC; ++c) sR[c][tx] = GL[c][0];
  }
  __syncthreads();
  if (!active) return;
  if (!last_col) {
#pragma unroll
    for (int c = 0; c < NC; ++c) GR[c][0] = sR[c][tx + 1];
  }
  lift_x<EQ, K, R>(GR, GL, R(-dt) * R(g.inv_dx), acc);
  store_state<R, NC, NB, L64>(a.out, g.N, i, acc);
}

// ---------------------------------------------------------------------------
// local operator applied once: out = loc(in)   (FP64 layout)
// ---------------------------------------------------------------------------
template <class EQ, int K>
__global__ __launch_bounds__(256) void k_loc(PhysDev ph, Geo g, const double* __restrict__ in,
                                             double* __restrict__ out) {
  using R = typename EQ::Real;
  constexpr int NC = EQ::NC, NB = Sizes<K, EQ::DIM>::NB;
  const long long cell = (long long)blockIdx.x * 256 + threadIdx.x;
  if (cell >= g.N) return;
  const EQ eq = make_eq<EQ>(ph);
  R u[NC][NB], acc[NC][NB];
  load_state<R, NC, NB, L64>(in, g.N, cell, u);
#pragma unroll
  for (int c = 0; c < NC; ++c)
#pragma unroll
    for (int b = 0; b < NB; ++b) acc[c][b] = 0.0;
  loc_acc<EQ, K, R>(eq, u, R(1), R(g.inv_dx), R(g.inv_dy), acc);
  store_state<R, NC, NB, L64>(out, g.N, cell, acc);
}

// One inner stage of a tableau with a full lower triangle in one pass:
// L_{i-1} = loc(u^(i-1)) (equation (dxl)), stored only when a later stage
// needs it, and u^(i) = u^n + sum_{j<i} coef_j L_j (equation (crkdg), first
// line), the earlier L_j read back, L_{i-1} taken from registers and added
// last (the order of the two-pass k_loc + k_combine, so the bits agree).
template <class EQ, int K>
__global__ __launch_bounds__(256) void k_loc_combine(PhysDev ph, Geo g, LocCombineArgs a) {
  constexpr int NC = EQ::NC, NB = Sizes<K, EQ::DIM>::NB;
  const long long cell = (long long)blockIdx.x * 256 + threadIdx.x;
  if (cell >= g.N) return;
  const EQ eq = make_eq<EQ>(ph);
  double u[NC][NB], L[NC][NB];
  load_state<double, NC, NB, L64>(a.in, g.N, cell, u);
#pragma unroll
  for (int c = 0; c < NC; ++c)
#pragma unroll
    for (int b = 0; b < NB; ++b) L[c][b] = 0.0;
  loc_acc<EQ, K, double>(eq, u, 1.0, g.inv_dx, g.inv_dy, L);
  if (a.L_out) store_state<double, NC, NB, L64>(a.L_out, g.N, cell, L);
  // the accumulator starts from u^n (already in u when u^(i-1) is u^n)
  if (a.in != a.un) load_state<double, NC, NB, L64>(a.un, g.N, cell, u);
  const double scale = a.dt_ptr ? *a.dt_ptr : 1.0;
  const unsigned o8 = (unsigned)cell * 8u;
#pragma unroll 1
  for (int j = 0; j < a.nx; ++j) {
    const double cf = a.coef[j] * scale;
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      const auto r = rsrc(byte_add(a.X[j], (long long)c * NB * g.N * 8));
#pragma unroll
      for (int b = 0; b < NB; ++b) u[c][b] = u[c][b] + cf * bload<double>(r, o8, (unsigned)(b * g.N * 8));
    }
  }
  if (a.use_last) {
    const double cf = a.coef_last * scale;
#pragma unroll
    for (int c = 0; c < NC; ++c)
#pragma unroll
      for (int b = 0; b < NB; ++b) u[c][b] = u[c][b] + cf * L[c][b];
  }
  store_state<double, NC, NB, L64>(a.out, g.N, cell, u);
}

// ---------------------------------------------------------------------------
// RK stage combination: out = base + sum_j (coef_j * dtscale) X_j
// ---------------------------------------------------------------------------
struct CombineArgs {
  double* out;
  const double* base;
  const double* X[MAXS];
  double coef[MAXS];
  int n;
  const double* dt_ptr;  // if set, every coefficient is multiplied by *dt_ptr
};

// streaming tuning (measured on 1.2 GB FP64 arrays, 1/3/5 inputs): two
// 16-byte vectors per thread and iteration, non-temporal loads and stores,
// up to 65536 blocks: 5.9 / 5.8 / 5.6 TB/s, against 4.5 / 4.6 / 4.9 TB/s
// with one plain vector and 8192 blocks
#ifndef COMBINE_U
#define COMBINE_U 2
#endif
#ifndef COMBINE_NT
#define COMBINE_NT 1
#endif
typedef double dbl2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ dbl2 stream_load(const dbl2* p) {
#if COMBINE_NT
  return __builtin_nontemporal_load(p);
#else
  return *p;
#endif
}
__device__ __forceinline__ void stream_store(dbl2 v, dbl2* p) {
#if COMBINE_NT
  __builtin_nontemporal_store(v, p);
#else
  *p = v;
#endif
}
__global__ __launch_bounds__(256) void k_combine(long long n, CombineArgs a) {
  // n doubles; pairs are processed as 16-byte vectors, COMBINE_U of them per
  // thread and iteration (one grid stride apart, so each access stays
  // coalesced); the odd tail element by the first thread
  const double scale = a.dt_ptr ? *a.dt_ptr : 1.0;
  double cf[MAXS];
#pragma unroll
  for (int j = 0; j < MAXS; ++j) cf[j] = a.coef[j] * scale;
  const long long n2 = n / 2;
  const dbl2* __restrict__ base = reinterpret_cast<const dbl2*>(a.base);
  dbl2* __restrict__ out = reinterpret_cast<dbl2*>(a.out);
  const long long stride = (long long)gridDim.x * 256;
  for (long long e0 = (long long)blockIdx.x * 256 + threadIdx.x; e0 < n2; e0 += stride * COMBINE_U) {
    dbl2 v[COMBINE_U];
#pragma unroll
    for (int u = 0; u < COMBINE_U; ++u) {
      const long long e = e0 + u * stride;
      v[u] = (base && e < n2) ? stream_load(base + e) : dbl2{0.0, 0.0};
    }
#pragma unroll
    for (int j = 0; j < MAXS; ++j) {
      if (j < a.n) {
        const dbl2* __restrict__ X = reinterpret_cast<const dbl2*>(a.X[j]);
#pragma unroll
        for (int u = 0; u < COMBINE_U; ++u) {
          const long long e = e0 + u * stride;
          if (e < n2) {
            const dbl2 x = stream_load(X + e);
            v[u].x = v[u].x + cf[j] * x.x;
            v[u].y = v[u].y + cf[j] * x.y;
          }
        }
      }
    }
#pragma unroll
    for (int u = 0; u < COMBINE_U; ++u) {
      const long long e = e0 + u * stride;
      if (e < n2) stream_store(v[u], out + e);
    }
  }
  if ((n & 1) && blockIdx.x == 0 && threadIdx.x == 0) {
    const long long e = n - 1;
    double v = a.base ? a.base[e] : 0.0;
    for (int j = 0; j < a.n; ++j) v = v + cf[j] * a.X[j][e];
    a.out[e] = v;
  }
}

// ---------------------------------------------------------------------------
// reductions
// ---------------------------------------------------------------------------
// deterministic block sum / max: fixed tree in LDS
template <int NT>
__device__ __forceinline__ double block_sum(double v, double* sh) {
  const int t = threadIdx.x;
  sh[t] = v;
  __syncthreads();
#pragma unroll
  for (int o = NT / 2; o > 0; o >>= 1) {
    if (t < o) sh[t] = sh[t] + sh[t + o];
    __syncthreads();
  }
  const double r = sh[0];
  __syncthreads();
  return r;
}
// maximum over the block (a NaN anywhere gives NaN): lane exchanges within
// each wavefront, then the NT / 64 wavefront maxima through sh
template <int NT>
__device__ __forceinline__ double block_max(double v, double* sh) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    const double w = __shfl_xor(v, o);
    if (w > v || w != w) v = w;
  }
  const int t = threadIdx.x;
  if ((t & 63) == 0) sh[t >> 6] = v;
  __syncthreads();
  double r = sh[0];
#pragma unroll
  for (int k = 1; k < NT / 64; ++k) {
    const double w = sh[k];
    if (w > r || w != w) r = w;
  }
  __syncthreads();
  return r;
}

// primitive quantities of a cell average (FP64), computed once per cell and
// shared by the wave speed, the characteristic decomposition and the limited
// reconstruction
struct EulerPrim {
  double ir, u, v, q2, p, c, ic, H;
};
__device__ __forceinline__ EulerPrim euler_prim(double gamma, const double* q) {
  EulerPrim w;
  w.ir = 1.0 / q[0];
  w.u = q[1] * w.ir;
  w.v = q[2] * w.ir;
  w.q2 = w.u * w.u + w.v * w.v;
  w.p = (gamma - 1.0) * (q[3] - 0.5 * (q[1] * w.u + q[2] * w.v));
  w.c = sqrt(gamma * w.p * w.ir);
  w.ic = 1.0 / w.c;
  w.H = (q[3] + w.p) * w.ir;
  return w;
}
__device__ __forceinline__ double euler_speed(const Geo& g, const EulerPrim& w) {
  return (fabs(w.u) + w.c) * g.inv_dx + (fabs(w.v) + w.c) * g.inv_dy;
}

template <class EQ>
__device__ __forceinline__ double cell_speed(const PhysDev& ph, const Geo& g, const double* q) {
  if constexpr (EQ::EULER) {
    const double ir = 1.0 / q[0];
    const double u = q[1] * ir, v = q[2] * ir;
    const double p = (ph.gamma - 1.0) * (q[3] - 0.5 * (q[1] * u + q[2] * v));
    const double c = sqrt(ph.gamma * p * ir);
    return (fabs(u) + c) * g.inv_dx + (fabs(v) + c) * g.inv_dy;
  } else if constexpr (EQ::BURGERS) {
    return fabs(q[0]) * g.inv_dx;
  } else {
    return fabs(ph.ax) * g.inv_dx + (EQ::DIM == 2 ? fabs(ph.ay) * g.inv_dy : 0.0);
  }
}

template <class EQ, int K, int LAY>
__global__ __launch_bounds__(256) void k_wave_partial(PhysDev ph, Geo g, const void* __restrict__ u,
                                                      double* __restrict__ partial) {
  constexpr int NC = EQ::NC, NB = Sizes<K, EQ::DIM>::NB;
  __shared__ double sh[256];
  double m = 0.0;
  for (long long cell = (long long)blockIdx.x * 256 + threadIdx.x; cell < g.N;
       cell += (long long)gridDim.x * 256) {
    double q[4];
#pragma unroll
    for (int c = 0; c < NC; ++c) q[c] = load_avg<NC, NB, LAY>(u, g.N, c, cell);
    const double s = cell_speed<EQ>(ph, g, q);
    if (s > m || s != s) m = s;
  }
  m = block_max<256>(m, sh);
  if (threadIdx.x == 0) partial[blockIdx.x] = m;
}

__global__ __launch_bounds__(1024) void k_wave_final(const double* __restrict__ partial, int n, double cfl,
                                                     double* smax_out, double* dt_out) {
  __shared__ double sh[1024];
  double m = 0.0;
  // eight independent loads in flight per thread, then a fixed-order tree
  for (int e0 = threadIdx.x; e0 < n; e0 += 8 * 1024) {
    double w[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int e = e0 + q * 1024;
      w[q] = e < n ? partial[e] : 0.0;
    }
#pragma unroll
    for (int q = 0; q < 8; ++q)
      if (w[q] > m || w[q] != w[q]) m = w[q];
  }
  m = block_max<1024>(m, sh);
  if (threadIdx.x == 0) {
    if (smax_out) *smax_out = m;
    if (dt_out) *dt_out = cfl / m;
  }
}

template <class EQ, int K, int LAY>
__global__ __launch_bounds__(256) void k_error_partial(PhysDev ph, Geo g, const void* __restrict__ u,
                                                       int ic,
                                                       const double* __restrict__ params,
                                                       const double* __restrict__ aux, double t,
                                                       int comp, double* __restrict__ partial) {
  constexpr int NC = EQ::NC, NB = Sizes<K, EQ::DIM>::NB, Q = K + 1, QE = K + 3;
  constexpr int DIM = EQ::DIM;
  constexpr GTab<QE> E = Tab<QE>::t;
  __shared__ double sh[256];
  double P[NPARAM];
  for (int e = 0; e < NPARAM; ++e) P[e] = params[e];
  double l1 = 0.0, l2 = 0.0, li = 0.0;
  const double wscale = DIM == 2 ? 0.25 * g.dx * g.dy : 0.5 * g.dx;
  for (long long cell = (long long)blockIdx.x * 256 + threadIdx.x; cell < g.N;
       cell += (long long)gridDim.x * 256) {
    const int i = (int)(cell % g.nx), j = (int)(cell / g.nx);
    const double xc = g.x0 + (i + 0.5) * g.dx, yc = g.y0 + (j + 0.5) * g.dy;
    double Ua[NC][NB];
    load_state<double, NC, NB, LAY>(u, g.N, cell, Ua);
#pragma unroll
    for (int a = 0; a < QE; ++a)
#pragma unroll
      for (int bq = 0; bq < (DIM == 2 ? QE : 1); ++bq) {
        const double xi = E.X[a], eta = DIM == 2 ? E.X[bq] : 0.0;
        double v = 0.0;
#pragma unroll
        for (int b = 0; b < NB; ++b) {
          const int m = b % Q, n = b / Q;
          v += Ua[comp][b] * leg(m, xi) * (DIM == 2 ? leg(n, eta) : 1.0);
        }
        double q[4];
        exact_state<EQ>(ic, P, aux, g, ph, xc + 0.5 * g.dx * xi, yc + 0.5 * g.dy * eta, t, q);
        const double e = fabs(v - q[comp]);
        const double wq = wscale * E.W[a] * (DIM == 2 ? E.W[bq] : 1.0);
        l1 += wq * e;
        l2 += wq * e * e;
        if (e > li || e != e) li = e;
      }
  }
  l1 = block_sum<256>(l1, sh);
  l2 = block_sum<256>(l2, sh);
  li = block_max<256>(li, sh);
  if (threadIdx.x == 0) {
    partial[3 * blockIdx.x + 0] = l1;
    partial[3 * blockIdx.x + 1] = l2;
    partial[3 * blockIdx.x + 2] = li;
  }
}

template <class EQ, int K, int LAY>
__global__ __launch_bounds__(256) void k_total_partial(Geo g, const void* __restrict__ u,
                                                       int comp, double* __restrict__ partial) {
  constexpr int NC = EQ::NC, NB = Sizes<K, EQ::DIM>::NB;
  __shared__ double sh[256];
  double s = 0.0;
  for (long long cell = (long long)blockIdx.x * 256 + threadIdx.x; cell < g.N;
       cell += (long long)gridDim.x * 256)
    s += load_avg<NC, NB, LAY>(u, g.N, comp, cell);
  s = block_sum<256>(s, sh);
  if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

// errors of one component's cell averages against a finer reference mesh
// restricted to this one (mean of the r x ry fine averages covering a cell;
// each line of fine cells summed in x order, lines in y order)
__global__ __launch_bounds__(256) void k_error_ref_partial(Geo g, const double* __restrict__ ac,
                                                           const double* __restrict__ af, int r,
                                                           int ry, long long nxf, double area,
                                                           double* __restrict__ partial) {
  __shared__ double sh[256];
  const double inv = 1.0 / (double)(r * ry);
  double l1 = 0.0, l2 = 0.0, li = 0.0;
  for (long long cell = (long long)blockIdx.x * 256 + threadIdx.x; cell < g.N;
       cell += (long long)gridDim.x * 256) {
    const long long i = cell % g.nx, j = cell / g.nx;
    double s = 0.0;
    for (int jj = 0; jj < ry; ++jj) {
      const double* row = af + (j * ry + jj) * nxf + i * r;
      for (int ii = 0; ii < r; ++ii) s += row[ii];
    }
    const double e = fabs(ac[cell] - s * inv);
    l1 += area * e;
    l2 += area * e * e;
    if (e > li || e != e) li = e;
  }
  l1 = block_sum<256>(l1, sh);
  l2 = block_sum<256>(l2, sh);
  li = block_max<256>(li, sh);
  if (threadIdx.x == 0) {
    partial[3 * blockIdx.x + 0] = l1;
    partial[3 * blockIdx.x + 1] = l2;
    partial[3 * blockIdx.x + 2] = li;
  }
}

// sums (stride 3 groups: l1, l2 summed, linf max) in a fixed order
__global__ __launch_bounds__(256) void k_sum_final(const double* __restrict__ partial, int n, int width,
                                                   double scale, double* out) {
  __shared__ double sh[256];
  for (int q = 0; q < width; ++q) {
    double s = 0.0;
    const bool is_max = width == 3 && q == 2;
    for (int e = threadIdx.x; e < n; e += 256) {
      const double w = partial[width * e + q];
      if (is_max) {
        if (w > s || w != w) s = w;
      } else {
        s += w;
      }
    }
    s = is_max ? block_max<256>(s, sh) : block_sum<256>(s, sh);
    if (threadIdx.x == 0) {
      if (width == 3 && q == 1) s = sqrt(s);
      out[q] = (width == 1) ? s * scale : s;
    }
  }
}

// ---------------------------------------------------------------------------
// L2 projection of an initial condition with a (k+3)-point rule (FP64 math)
// ---------------------------------------------------------------------------
template <class EQ, int K, int LAY>
__global__ __launch_bounds__(256) void k_project(PhysDev ph, Geo g, int ic,
                                                 const double* __restrict__ params,
                                                 const double* __restrict__ aux, double t,
                                                 void* __restrict__ u) {
  constexpr int NC = EQ::NC, NB = Sizes<K, EQ::DIM>::NB, Q = K + 1, QE = K + 3;
  constexpr int DIM = EQ::DIM;
  constexpr GTab<QE> E = Tab<QE>::t;
  const long long cell = (long long)blockIdx.x * 256 + threadIdx.x;
  if (cell >= g.N) return;
  double P[NPARAM];
  for (int e = 0; e < NPARAM; ++e) P[e] = params[e];
  const int i = (int)(cell % g.nx), j = (int)(cell / g.nx);
  const double xc = g.x0 + (i + 0.5) * g.dx, yc = g.y0 + (j + 0.5) * g.dy;
  double acc[NC][NB];
  for (int c = 0; c < NC; ++c)
    for (int b = 0; b < NB; ++b) acc[c][b] = 0.0;
  for (int a = 0; a < QE; ++a)
    for (int bq = 0; bq < (DIM == 2 ? QE : 1); ++bq) {
      const double xi = E.X[a], eta = DIM == 2 ? E.X[bq] : 0.0;
      const double wq = E.W[a] * (DIM == 2 ? E.W[bq] : 1.0);
      double q[4];
      exact_state<EQ>(ic, P, aux, g, ph, xc + 0.5 * g.dx * xi, yc + 0.5 * g.dy * eta, t, q);
      for (int b = 0; b < NB; ++b) {
        const int m = b % Q, n = b / Q;
        const double ph_ = leg(m, xi) * (DIM == 2 ? leg(n, eta) : 1.0);
        for (int c = 0; c < NC; ++c) acc[c][b] += wq * q[c] * ph_;
      }
    }
  for (int c = 0; c < NC; ++c)
    for (int b = 0; b < NB; ++b) {
      const int m = b % Q, n = b / Q;
      const double norm = DIM == 2 ? (2 * m + 1) * (2 * n + 1) / 4.0 : (2 * m + 1) / 2.0;
      acc[c][b] *= norm;
    }
  store_state<double, NC, NB, LAY>(u, g.N, cell, acc);
}

// ---------------------------------------------------------------------------
// TVB minmod limiter, once per step after the final stage (in place, FP64)
// ---------------------------------------------------------------------------
__device__ __forceinline__ double minmod3(double a, double b, double c) {
  const bool pos = a > 0.0 && b > 0.0 && c > 0.0;
  const bool neg = a < 0.0 && b < 0.0 && c < 0.0;
  if (!(pos || neg)) return 0.0;
  double m = fabs(a);
  if (fabs(b) < m) m = fabs(b);
  if (fabs(c) < m) m = fabs(c);
  return pos ? m : -m;
}
__device__ __forceinline__ double tvb(double a, double b, double c, double Mh2) {
  return fabs(a) <= Mh2 ? a : minmod3(a, b, c);
}

// left/right eigenvectors of the 2D Euler flux Jacobian in direction d at q
// (L rows, R columns, row-major 4x4)
__device__ void euler_eigvec(double gamma, const EulerPrim& w, int d, double* L, double* Rm) {
  const double u = w.u, v = w.v, q2 = w.q2, c = w.c, ic = w.ic, H = w.H;
  const double b1 = (gamma - 1.0) * ic * ic, b2 = 0.5 * b1 * q2;
  const double un = d == 0 ? u : v, ut = d == 0 ? v : u;
  // in the rotated frame (normal, tangential); map back to (x, y) columns
  const int in = d == 0 ? 1 : 2, it = d == 0 ? 2 : 1;
  double Rl[4][4] = {};
  // columns: un - c, entropy, shear, un + c
  Rl[0][0] = 1.0; Rl[in][0] = un - c; Rl[it][0] = ut; Rl[3][0] = H - un * c;
  Rl[0][1] = 1.0; Rl[in][1] = un;     Rl[it][1] = ut; Rl[3][1] = 0.5 * q2;
  Rl[0][2] = 0.0; Rl[in][2] = 0.0;    Rl[it][2] = 1.0; Rl[3][2] = ut;
  Rl[0][3] = 1.0; Rl[in][3] = un + c; Rl[it][3] = ut; Rl[3][3] = H + un * c;
  double Ll[4][4] = {};
  Ll[0][0] = 0.5 * (b2 + un * ic); Ll[0][in] = -0.5 * (b1 * un + ic); Ll[0][it] = -0.5 * b1 * ut; Ll[0][3] = 0.5 * b1;
  Ll[1][0] = 1.0 - b2;             Ll[1][in] = b1 * un;               Ll[1][it] = b1 * ut;        Ll[1][3] = -b1;
  Ll[2][0] = -ut;                  Ll[2][in] = 0.0;                   Ll[2][it] = 1.0;            Ll[2][3] = 0.0;
  Ll[3][0] = 0.5 * (b2 - un * ic); Ll[3][in] = -0.5 * (b1 * un - ic); Ll[3][it] = -0.5 * b1 * ut; Ll[3][3] = 0.5 * b1;
  for (int r = 0; r < 4; ++r)
    for (int s = 0; s < 4; ++s) {
      L[r * 4 + s] = Ll[r][s];
      Rm[r * 4 + s] = Rl[r][s];
    }
}

// A sufficient condition for physical_points from the modal coefficients:
// every basis function is at most 1 in magnitude at the Gauss points, so
// rho_q >= avg - sum |modes| (likewise E), |m_q| <= |avg| + sum |modes|, and
// rho_q E_q - |m_q|^2 / 2 >= rho_lo E_lo - (mx_hi^2 + my_hi^2) / 2.  The
// relative margin keeps the rounding of these few operations from turning a
// failing cell into a passing one; cells that do not clear it take the exact
// test, so the decisions are those of physical_points.  avg: the cell
// averages; rabs[c]: the sum of |mode| over the higher modes of component c.
__device__ __forceinline__ bool surely_physical_sums(const double (&avg)[4], const double (&rabs)[4]) {
  const double rlo = avg[0] - rabs[0], elo = avg[3] - rabs[3];
  const double mx = fabs(avg[1]) + rabs[1], my = fabs(avg[2]) + rabs[2];
  const double lhs = rlo * elo, rhs = 0.5 * (mx * mx + my * my);
  return rlo > 0.0 && elo > 0.0 && lhs - rhs > 1e-10 * lhs;
}
template <int K>
__device__ __forceinline__ bool surely_physical(const double (&U)[4][(K + 1) * (K + 1)]) {
  constexpr int NB = (K + 1) * (K + 1);
  double avg[4], r[4];
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    double t = 0.0;
#pragma unroll
    for (int b = 1; b < NB; ++b) t += fabs(U[c][b]);
    avg[c] = U[c][0];
    r[c] = t;
  }
  return surely_physical_sums(avg, r);
}

// density and pressure positive at the operator's volume and face points
template <int K>
__device__ bool physical_points(double gamma, const double (&U)[4][(K + 1) * (K + 1)]) {
  // rho > 0 and p > 0 at every volume and face Gauss point.  With rho > 0 and
  // gamma > 1, p > 0 is the same as rho E - |m|^2 / 2 > 0, which needs no
  // division; the points are visited without early exit (no divergence).
  (void)gamma;
  constexpr int Q = K + 1;
  constexpr GTab<Q> T = Tab<Q>::t;
  bool ok = true;
  auto check = [&](double r, double mx, double my, double E) {
    ok = ok && (r > 0.0) && (r * E - 0.5 * (mx * mx + my * my) > 0.0);
  };
  // volume points, sum-factorised: first the eta lines, then the xi points
#pragma unroll
  for (int a = 0; a < Q; ++a) {
    double t[4][Q];
#pragma unroll
    for (int c = 0; c < 4; ++c)
#pragma unroll
      for (int n = 0; n < Q; ++n) {
        double v = U[c][Q * n];
#pragma unroll
        for (int m = 1; m < Q; ++m) v += U[c][m + Q * n] * T.P[m][a];
        t[c][n] = v;
      }
#pragma unroll
    for (int b = 0; b < Q; ++b) {
      double q[4];
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        double v = t[c][0];
#pragma unroll
        for (int n = 1; n < Q; ++n) v += t[c][n] * T.P[n][b];
        q[c] = v;
      }
      check(q[0], q[1], q[2], q[3]);
    }
  }
  double tr[4][Q];
  auto face = [&]() {
#pragma unroll
    for (int p = 0; p < Q; ++p) check(tr[0][p], tr[1][p], tr[2][p], tr[3][p]);
  };
  trace_x<+1, Euler2<double>, K, double>(U, tr);
  face();
  trace_x<-1, Euler2<double>, K, double>(U, tr);
  face();
  trace_y<+1, Euler2<double>, K, double>(U, tr);
  face();
  trace_y<-1, Euler2<double>, K, double>(U, tr);
  face();
  return ok;
}

struct LimitArgs {
  double M;
  const float* P;       // MLP parameters (device; learned-indicator mode)
  float z_lo, z_hi;     // logit thresholds: z <= z_lo smooth, z >= z_hi troubled,
                        // else the TVB test decides
  double* wave_partial; // if set: per-block max of the cell wave speeds (dt of the next step)
};

// one mode of component c of a cell, as double
template <int NC, int NB, int LAY>
__device__ __forceinline__ double load_mode(const void* __restrict__ p, long long N, int c, int b,
                                            unsigned cell) {
  if constexpr (LAY == L64) {
    return bload<double>(rsrc(byte_add(p, (long long)c * NB * N * 8)), cell * 8u,
                         (unsigned)(b * N * 8));
  } else if constexpr (LAY == LMIX) {
    if (b == 0) return bload<double>(rsrc(p), cell * 8u, (unsigned)(c * N * 8));
    return (double)bload<float>(
        rsrc(byte_add(p, (long long)NC * N * 8 + (long long)c * (NB - 1) * N * 4)), cell * 4u,
        (unsigned)((b - 1) * N * 4));
  } else {
    return (double)bload<float>(rsrc(byte_add(p, (long long)c * NB * N * 4)), cell * 4u,
                                (unsigned)(b * N * 4));
  }
}

// mode index of degree deg along direction d (mode m + (k+1) n)
template <int DIM, int Q>
__device__ __forceinline__ constexpr int dir_mode(int d, int deg) {
  return DIM == 1 ? deg : (d == 0 ? deg : deg * Q);
}

// cell averages of the two neighbours of cell (i, j) in direction d, with the
// ghost rule of a boundary they lie beyond; dp = right - own, dm = own - left
template <int NC, int NB, int LAY, bool DMRB = false>
__device__ __forceinline__ void limit_neighbours(const Geo& g, const BCDev& bc,
                                                 const void* __restrict__ u, int i, int j, int d,
                                                 const double (&avg)[NC], double (&dp)[NC],
                                                 double (&dm)[NC]) {
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    const int s = k ? -1 : 1;
    int ni = i + (d == 0 ? s : 0), nj = j + (d == 1 ? s : 0);
    const int side = d == 0 ? (s < 0 ? 0 : 1) : (s < 0 ? 2 : 3);
    double qa[NC];
    bool ghost = false;
    if (ni < 0 || ni >= g.nx || nj < 0 || nj >= g.ny) {
      const int type = bc.type[side];
      if (type == CRKDG_BC_TRANSMISSIVE) {
        ghost = true;
#pragma unroll
        for (int c = 0; c < NC; ++c) qa[c] = avg[c];
      } else if (DMRB && NC == 4 && type == CRKDG_BC_DIRICHLET) {
        // the ghost cell's centre at the limiter's time; the reflecting wall
        // mirrors the cell's own average
        ghost = true;
        const double xg = g.x0 + (ni + 0.5) * g.dx, yg = g.y0 + (nj + 0.5) * g.dy;
        if (side == 2 && g.x0 + (i + 0.5) * g.dx >= bc.params[0]) {
#pragma unroll
          for (int c = 0; c < NC; ++c) qa[c] = c == 2 ? -avg[c] : avg[c];
        } else {
          double q[4];
          const double tl =
              bc.t_ptr ? *bc.t_ptr + (bc.dt_ptr ? bc.dt_fac * *bc.dt_ptr : 0.0) : bc.t;
          dmr_state(bc.params, xg, yg, tl, q);
#pragma unroll
          for (int c = 0; c < NC; ++c) qa[c] = q[c];
        }
      } else if (type == CRKDG_BC_DIRICHLET) {
        ghost = true;
#pragma unroll
        for (int c = 0; c < NC; ++c) qa[c] = bc.state[side][c];
      } else {  // periodic: one step across the domain
        ni += ni < 0 ? g.nx : (ni >= g.nx ? -g.nx : 0);
        nj += nj < 0 ? g.ny : (nj >= g.ny ? -g.ny : 0);
      }
    }
    if (!ghost) {
#pragma unroll
      for (int c = 0; c < NC; ++c) qa[c] = load_avg<NC, NB, LAY>(u, g.N, c, (long long)nj * g.nx + ni);
    }
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      if (k == 0)
        dp[c] = qa[c] - avg[c];
      else
        dm[c] = avg[c] - qa[c];
    }
  }
}

// the TVB minmod troubled-cell test in direction d (characteristic variables
// for Euler): a / at are the cell's forward / backward trace-average jumps
template <class EQ>
__device__ __forceinline__ bool tvb_troubled_dir(const PhysDev& ph, double Mh2, const EulerPrim& wp,
                                                 int d, const double (&a)[EQ::NC],
                                                 const double (&at)[EQ::NC],
                                                 const double (&dp)[EQ::NC],
                                                 const double (&dm)[EQ::NC]) {
  constexpr int NC = EQ::NC;
  double ca[NC], cat[NC], cp[NC], cm[NC];
  if constexpr (EQ::EULER) {
    double L[16], Rm[16];
    euler_eigvec(ph.gamma, wp, d, L, Rm);
#pragma unroll
    for (int r = 0; r < NC; ++r) {
      ca[r] = cat[r] = cp[r] = cm[r] = 0.0;
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        ca[r] += L[r * 4 + c] * a[c];
        cat[r] += L[r * 4 + c] * at[c];
        cp[r] += L[r * 4 + c] * dp[c];
        cm[r] += L[r * 4 + c] * dm[c];
      }
    }
  } else {
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      ca[c] = a[c]; cat[c] = at[c]; cp[c] = dp[c]; cm[c] = dm[c];
    }
  }
  bool tr = false;
#pragma unroll
  for (int r = 0; r < NC; ++r)
    if (tvb(ca[r], cp[r], cm[r], Mh2) != ca[r] || tvb(cat[r], cp[r], cm[r], Mh2) != cat[r]) tr = true;
  return tr;
}

// limited P1 slope in direction d from the slope mode sl (characteristic
// minmod for Euler, mapped back with the right eigenvectors)
template <class EQ>
__device__ __forceinline__ void tvb_slope_dir(const PhysDev& ph, double Mh2, const EulerPrim& wp,
                                              int d, const double (&sl)[EQ::NC],
                                              const double (&dp)[EQ::NC],
                                              const double (&dm)[EQ::NC], double (&ns)[EQ::NC]) {
  constexpr int NC = EQ::NC;
  if constexpr (EQ::EULER) {
    double L[16], Rm[16], lim[NC];
    euler_eigvec(ph.gamma, wp, d, L, Rm);
#pragma unroll
    for (int r = 0; r < NC; ++r) {
      double s1 = 0.0, s2 = 0.0, s3 = 0.0;
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        s1 += L[r * 4 + c] * sl[c];
        s2 += L[r * 4 + c] * dp[c];
        s3 += L[r * 4 + c] * dm[c];
      }
      lim[r] = tvb(s1, s2, s3, Mh2);
    }
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      double s = 0.0;
#pragma unroll
      for (int r = 0; r < NC; ++r) s += Rm[c * 4 + r] * lim[r];
      ns[c] = s;
    }
  } else {
#pragma unroll
    for (int c = 0; c < NC; ++c) ns[c] = tvb(sl[c], dp[c], dm[c], Mh2);
  }
}

// The limiter in two passes over a block of 256 cells.  The first pass reads
// of each cell only what the troubled-cell decision needs (averages, the
// trace-average jumps, the sum of |higher modes| for the positivity bound,
// the neighbour averages) and decides: smooth cells that surely pass the
// positivity test are done.  The rest (troubled cells, cells inside the
// learned indicator's uncertainty band, cells whose positivity needs the
// point test) go into a queue in LDS, and the second pass gives them to the
// block's first lanes, so that the heavy work (the band's TVB test, the point
// positivity test, the limited reconstruction and the store) runs on as few
// wavefronts as there are such cells rather than on every wavefront that
// holds one.  Each queued cell is processed the same whichever lane takes it.
//
// MLP = false: the TVB minmod test decides for every cell.  MLP = true
// (2D Euler only): the learned indicator decides outside its uncertainty band
// and the FP64 TVB test inside it; the network runs once per wavefront on
// the matrix cores, so every lane takes part even past the last cell.
//
// Flags per cell: 1 troubled (limited), 2 positivity-limited, 4 reduced to
// its average, 8 decided by the TVB test inside the uncertainty band.
// DMRB: double Mach reflection ghost averages (bc.exact == CRKDG_IC_DMR)
template <class EQ, int K, int LAY, bool MLP, bool DMRB>
__global__ __launch_bounds__(256, MLP ? LIMIT_OCC_MLP : LIMIT_OCC_TVB) void k_limit(PhysDev ph, Geo g, BCDev bc, LimitArgs la,
                                               void* __restrict__ u,
                                               uint8_t* __restrict__ flags,
                                               unsigned long long* __restrict__ counters) {
  constexpr int NC = EQ::NC, DIM = EQ::DIM, Q = K + 1, NB = Sizes<K, DIM>::NB;
  constexpr bool EUL = EQ::EULER;
  constexpr bool USE_MLP = MLP && EUL && DIM == 2 && K >= 1;
  __shared__ unsigned int cnt[4];  // limited, non-physical averages, band; [3]: queue length
  __shared__ unsigned short queue[256];
  if (threadIdx.x < 4) cnt[threadIdx.x] = 0;
  __syncthreads();
  // crkdg_create keeps the cell count far below 2^32
  const unsigned cell = blockIdx.x * 256u + threadIdx.x;
  const bool in = cell < (unsigned)g.N;
  const double M = la.M;
  const double Mh2[2] = {M * g.dx * g.dx, M * g.dy * g.dy};
  bool bad = false, troubled = false, band = false, heavy = false;
  double spd = 0.0;
  {
    double avg[NC], a[2][NC], at[2][NC], rabs[NC], dp[2][NC], dm[2][NC];
    EulerPrim wp{};
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      avg[c] = 0.0;
      rabs[c] = 0.0;
#pragma unroll
      for (int d = 0; d < 2; ++d) a[d][c] = at[d][c] = dp[d][c] = dm[d][c] = 0.0;
    }
    int i = 0, j = 0;
    if (in) {
      i = (int)(cell % (unsigned)g.nx);
      j = (int)(cell / (unsigned)g.nx);
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        avg[c] = load_mode<NC, NB, LAY>(u, g.N, c, 0, cell);
#pragma unroll
        for (int b = 1; b < NB; ++b) {
          const double v = load_mode<NC, NB, LAY>(u, g.N, c, b, cell);
          rabs[c] += fabs(v);
        }
#pragma unroll
        for (int d = 0; d < DIM; ++d)
#pragma unroll
          for (int deg = 1; deg <= K; ++deg) {
            const double v = load_mode<NC, NB, LAY>(u, g.N, c, dir_mode<DIM, Q>(d, deg), cell);
            a[d][c] += v;
            at[d][c] += (deg % 2) ? v : -v;
          }
      }
      if constexpr (EUL) {
        wp = euler_prim(ph.gamma, avg);
        bad = !(avg[0] > 0.0) || !(wp.p > 0.0);
        spd = euler_speed(g, wp);
      } else {
        spd = cell_speed<EQ>(ph, g, avg);
      }
#pragma unroll
      for (int d = 0; d < DIM; ++d) limit_neighbours<NC, NB, LAY, DMRB>(g, bc, u, i, j, d, avg, dp[d], dm[d]);
    }
    if constexpr (USE_MLP) {
      __shared__ MlpWeightsSmem ws;
      mlp_stage_weights(la.P, ws);
      float x[MLP_IN];
#pragma unroll
      for (int e = 0; e < MLP_IN; ++e) x[e] = 0.0f;
      if (in && !bad) cell_features_jumps(a, at, dp, dm, Mh2[0], Mh2[1], x);
      __syncthreads();  // the staged weights
      const float z = mlp_infer_wave(la.P, ws, x);
      if (in && !bad) {
        if (z >= la.z_hi)
          troubled = true;
        else if (z > la.z_lo)
          band = true;
      }
    } else if constexpr (K >= 1) {
      if (in && !bad)
#pragma unroll
        for (int d = 0; d < DIM; ++d)
          troubled = tvb_troubled_dir<EQ>(ph, Mh2[d], wp, d, a[d], at[d], dp[d], dm[d]) || troubled;
    }
    if constexpr (K >= 1) {
      heavy = in && !bad && (troubled || band);
      if constexpr (EUL) heavy = heavy || (in && !bad && !surely_physical_sums(avg, rabs));
    }
  }
  // queue the heavy cells (one LDS atomic per wavefront)
  const unsigned long long hm = __ballot(heavy);
  if (hm) {
    const int lane = (int)(threadIdx.x & 63u);
    const int leader = __ffsll((long long)hm) - 1;
    unsigned base = 0;
    if (lane == leader) base = atomicAdd(&cnt[3], (unsigned)__popcll(hm));
    base = (unsigned)__shfl((int)base, leader);
    if (heavy) {
      const unsigned rank = (unsigned)__popcll(hm & ((1ull << lane) - 1ull));
      queue[base + rank] = (unsigned short)(threadIdx.x | (troubled ? 0x100u : 0u) | (band ? 0x200u : 0u));
    }
  }
  if (in && !heavy && flags) flags[cell] = 0;
  if (counters) {
    if (bad) atomicAdd(&cnt[1], 1u);
    if (band) atomicAdd(&cnt[2], 1u);
  }
  // the limiter never changes a cell average, so the wave speeds of the
  // limited state (the next step's dt) come from the averages already read;
  // the reduction's barriers also publish the queue
  if (la.wave_partial) {
    __shared__ double sh[4];
    const double m = block_max<256>(spd, sh);
    if (threadIdx.x == 0) la.wave_partial[blockIdx.x] = m;
  } else {
    __syncthreads();
  }
  // second pass: the queued cells on the block's first lanes
  if (K >= 1 && threadIdx.x < cnt[3]) {
    const unsigned e = queue[threadIdx.x];
    const unsigned qc = blockIdx.x * 256u + (e & 0xffu);
    const bool tr0 = (e & 0x100u) != 0, bnd = (e & 0x200u) != 0;
    const int i = (int)(qc % (unsigned)g.nx), j = (int)(qc / (unsigned)g.nx);
    double avg[NC], sl[2][NC], a[2][NC], at[2][NC];
    bool phys = true;  // the unlimited polynomial passes the point positivity test
    {
      double U[NC][NB];
      load_state<double, NC, NB, LAY>(u, g.N, qc, U);
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        avg[c] = U[c][0];
#pragma unroll
        for (int d = 0; d < 2; ++d) {
          sl[d][c] = d < DIM ? U[c][dir_mode<DIM, Q>(d, 1)] : 0.0;
          double s = 0.0, st = 0.0;
#pragma unroll
          for (int deg = 1; deg <= K; ++deg) {
            const double v = d < DIM ? U[c][dir_mode<DIM, Q>(d, deg)] : 0.0;
            s += v;
            st += (deg % 2) ? v : -v;
          }
          a[d][c] = s;
          at[d][c] = st;
        }
      }
      if constexpr (EUL)
        if (!tr0) phys = surely_physical<K>(U) || physical_points<K>(ph.gamma, U);
    }
    EulerPrim wp{};
    if constexpr (EUL) wp = euler_prim(ph.gamma, avg);
    double dp[2][NC], dm[2][NC];
#pragma unroll
    for (int d = 0; d < DIM; ++d) limit_neighbours<NC, NB, LAY, DMRB>(g, bc, u, i, j, d, avg, dp[d], dm[d]);
    bool tr = tr0;
    if (bnd) {
      tr = false;
#pragma unroll
      for (int d = 0; d < DIM; ++d)
        tr = tvb_troubled_dir<EQ>(ph, Mh2[d], wp, d, a[d], at[d], dp[d], dm[d]) || tr;
    }
    uint8_t f = bnd ? 8 : 0;
    if (tr)
      f |= 1;
    else if (!phys)
      f |= 2;
    if (tr || !phys) {
      double V[NC][NB];
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        V[c][0] = avg[c];
#pragma unroll
        for (int b = 1; b < NB; ++b) V[c][b] = 0.0;
      }
#pragma unroll
      for (int d = 0; d < DIM; ++d) {
        double ns[NC];
        tvb_slope_dir<EQ>(ph, Mh2[d], wp, d, sl[d], dp[d], dm[d], ns);
#pragma unroll
        for (int c = 0; c < NC; ++c) V[c][dir_mode<DIM, Q>(d, 1)] = ns[c];
      }
      if constexpr (EUL) {
        if (!surely_physical<K>(V) && !physical_points<K>(ph.gamma, V)) {
          f |= 2 | 4;
#pragma unroll
          for (int c = 0; c < NC; ++c)
#pragma unroll
            for (int b = 1; b < NB; ++b) V[c][b] = 0.0;
        }
      }
      store_higher_modes<double, NC, NB, LAY>(u, g.N, qc, V);
    }
    if (flags) flags[qc] = f;
    if (counters && (f & 7)) atomicAdd(&cnt[0], 1u);
  }
  if (counters) {
    __syncthreads();
    if (threadIdx.x == 0) {
      if (cnt[0]) atomicAdd(&counters[0], (unsigned long long)cnt[0]);
      if (cnt[1]) atomicAdd(&counters[1], (unsigned long long)cnt[1]);
      if (cnt[2]) atomicAdd(&counters[2], (unsigned long long)cnt[2]);
    }
  }
}

// 12 stencil features per cell for the learned indicator (training data)
template <int K, int LAY>
__global__ __launch_bounds__(256) void k_mlp_features(Geo g, BCDev bc, double M,
                                                      const void* __restrict__ u,
                                                      float* __restrict__ X) {
  constexpr int NC = 4, Q = K + 1, NB = Q * Q;
  const long long cell = (long long)blockIdx.x * 256 + threadIdx.x;
  if (cell >= g.N) return;
  const int i = (int)(cell % g.nx), j = (int)(cell / g.nx);
  double U[NC][NB];
  load_state<double, NC, NB, LAY>(u, g.N, cell, U);
  // the limiter's neighbour averages and ghost rules (time-dependent ghost
  // data at the time in bc.t)
  double avg[NC], dp[2][4], dm[2][4];
  for (int c = 0; c < NC; ++c) avg[c] = U[c][0];
  for (int d = 0; d < 2; ++d) limit_neighbours<NC, NB, LAY>(g, bc, u, i, j, d, avg, dp[d], dm[d]);
  float x[MLP_IN];
  cell_features<NB, Q>(U, dp, dm, M * g.dx * g.dx, M * g.dy * g.dy, x);
#pragma unroll
  for (int f = 0; f < MLP_IN; ++f) X[cell * MLP_IN + f] = x[f];
}

__global__ void k_zero_u64(unsigned long long* p, int n) {
  if ((int)threadIdx.x < n) p[threadIdx.x] = 0ull;
}

// ---------------------------------------------------------------------------
// dispatch
// ---------------------------------------------------------------------------
// k = 0..4 for the scalar equations, 0..3 for Euler
template <template <class, int> class F, class R, class... A>
hipError_t dispatch_r(int eq, int k, A&&... args) {
  switch (eq * 5 + k) {
    case EQ_ADV1 * 5 + 0: return F<Adv<R, 1>, 0>::run(args...);
    case EQ_ADV1 * 5 + 1: return F<Adv<R, 1>, 1>::run(args...);
    case EQ_ADV1 * 5 + 2: return F<Adv<R, 1>, 2>::run(args...);
    case EQ_ADV1 * 5 + 3: return F<Adv<R, 1>, 3>::run(args...);
    case EQ_ADV1 * 5 + 4: return F<Adv<R, 1>, 4>::run(args...);
    case EQ_ADV2 * 5 + 0: return F<Adv<R, 2>, 0>::run(args...);
    case EQ_ADV2 * 5 + 1: return F<Adv<R, 2>, 1>::run(args...);
    case EQ_ADV2 * 5 + 2: return F<Adv<R, 2>, 2>::run(args...);
    case EQ_ADV2 * 5 + 3: return F<Adv<R, 2>, 3>::run(args...);
    case EQ_ADV2 * 5 + 4: return F<Adv<R, 2>, 4>::run(args...);
    case EQ_EULER2 * 5 + 0: return F<Euler2<R>, 0>::run(args...);
    case EQ_EULER2 * 5 + 1: return F<Euler2<R>, 1>::run(args...);
    case EQ_EULER2 * 5 + 2: return F<Euler2<R>, 2>::run(args...);
    case EQ_EULER2 * 5 + 3: return F<Euler2<R>, 3>::run(args...);
    case EQ_BURGERS1 * 5 + 0: return F<Burgers1<R>, 0>::run(args...);
    case EQ_BURGERS1 * 5 + 1: return F<Burgers1<R>, 1>::run(args...);
    case EQ_BURGERS1 * 5 + 2: return F<Burgers1<R>, 2>::run(args...);
    case EQ_BURGERS1 * 5 + 3: return F<Burgers1<R>, 3>::run(args...);
    case EQ_BURGERS1 * 5 + 4: return F<Burgers1<R>, 4>::run(args...);
    default: return hipErrorInvalidValue;
  }
}
template <template <class, int> class F, class... A>
hipError_t dispatch(int eq, int k, A&&... args) {
  return dispatch_r<F, double>(eq, k, args...);
}
// the FP32 forms exist for 2D Euler, k = 1..3
template <template <class, int> class F, class R, class... A>
hipError_t dispatch_euler(int eq, int k, A&&... args) {
  if (eq != EQ_EULER2) return hipErrorInvalidValue;
  switch (k) {
    case 1: return F<Euler2<R>, 1>::run(args...);
    case 2: return F<Euler2<R>, 2>::run(args...);
    case 3: return F<Euler2<R>, 3>::run(args...);
    default: return hipErrorInvalidValue;
  }
}
template <template <class, int> class F, class... A>
hipError_t dispatch_mixed(int eq, int k, A&&... args) {
  return dispatch_euler<F, float>(eq, k, args...);
}

static unsigned nblk(long long n, int t) { return (unsigned)((n + t - 1) / t); }

template <int LIN, int LOUT, bool INC>
struct InnerL {
  template <class EQ, int K>
  struct Run {
    static hipError_t run(const PhysDev& ph, const Geo& g, const InnerArgs& a, hipStream_t s) {
      hipLaunchKernelGGL((k_inner<EQ, K, LIN, LOUT, INC>), dim3(nblk(g.N, 256)), dim3(256), 0, s,
                         ph, g, a);
      return hipGetLastError();
    }
  };
};
template <int LAY>
struct FinalL {
  template <class EQ, int K>
  struct Run {
    static hipError_t run(const PhysDev& ph, const Geo& g, const BCDev& bc, const FinalArgs& a,
                          hipStream_t s) {
      if constexpr (EQ::DIM == 2) {
        using T = FinalTile<typename EQ::Real>;
        dim3 grid(nblk(g.nx, T::TX), nblk(g.ny, T::TY));
        if (a.base2 && (a.ns < 1 || a.base2 != a.st[0])) return hipErrorInvalidValue;
        const dim3 blk(T::TX * T::TY);
        const bool dmr = bc.exact == CRKDG_IC_DMR;
        if constexpr (LAY == L64 && sizeof(typename EQ::Real) == 8) {
          if (a.base2) {
            if constexpr (EQ::EULER) {
              if (dmr) {
                hipLaunchKernelGGL((k_final2<EQ, K, LAY, true, true>), grid, blk, 0, s, ph, g, bc, a);
                return hipGetLastError();
              }
            }
            hipLaunchKernelGGL((k_final2<EQ, K, LAY, true, false>), grid, blk, 0, s, ph, g, bc, a);
            return hipGetLastError();
          }
        } else if (a.base2) {
          return hipErrorInvalidValue;  // the original RKDG runs on the FP64 layout only
        }
        if constexpr (EQ::EULER) {
          if (dmr) {
            hipLaunchKernelGGL((k_final2<EQ, K, LAY, false, true>), grid, blk, 0, s, ph, g, bc, a);
            return hipGetLastError();
          }
        }
        hipLaunchKernelGGL((k_final2<EQ, K, LAY, false, false>), grid, blk, 0, s, ph, g, bc, a);
      } else {
        hipLaunchKernelGGL((k_final1<EQ, K>), dim3(nblk(g.nx, B1)), dim3(B1), 0, s, ph, g, bc, a);
      }
      return hipGetLastError();
    }
  };
};

template <class EQ, int K>
struct RunLoc {
  static hipError_t run(const PhysDev& ph, const Geo& g, const double* in, double* out,
                        hipStream_t s) {
    hipLaunchKernelGGL((k_loc<EQ, K>), dim3(nblk(g.N, 256)), dim3(256), 0, s, ph, g, in, out);
    return hipGetLastError();
  }
};
template <class EQ, int K>
struct RunLocCombine {
  static hipError_t run(const PhysDev& ph, const Geo& g, const LocCombineArgs& a, hipStream_t s) {
    hipLaunchKernelGGL((k_loc_combine<EQ, K>), dim3(nblk(g.N, 256)), dim3(256), 0, s, ph, g, a);
    return hipGetLastError();
  }
};
template <class EQ, int K>
struct RunWave {
  static hipError_t run(const PhysDev& ph, const Geo& g, const void* u, int lay, double* partial,
                        int nb, double cfl, double* smax, double* dt, hipStream_t s) {
    if (lay == LMIX)
      hipLaunchKernelGGL((k_wave_partial<EQ, K, LMIX>), dim3(nb), dim3(256), 0, s, ph, g, u, partial);
    else
      hipLaunchKernelGGL((k_wave_partial<EQ, K, L64>), dim3(nb), dim3(256), 0, s, ph, g, u, partial);
    hipLaunchKernelGGL(k_wave_final, dim3(1), dim3(1024), 0, s, partial, nb, cfl, smax, dt);
    return hipGetLastError();
  }
};
template <class EQ, int K>
struct RunError {
  static hipError_t run(const PhysDev& ph, const Geo& g, const void* u, int lay, int ic,
                        const double* params, const double* aux, double t, int comp,
                        double* partial, int nb, double* out3, hipStream_t s) {
    if (lay == LMIX)
      hipLaunchKernelGGL((k_error_partial<EQ, K, LMIX>), dim3(nb), dim3(256), 0, s, ph, g, u, ic,
                         params, aux, t, comp, partial);
    else
      hipLaunchKernelGGL((k_error_partial<EQ, K, L64>), dim3(nb), dim3(256), 0, s, ph, g, u, ic,
                         params, aux, t, comp, partial);
    hipLaunchKernelGGL(k_sum_final, dim3(1), dim3(256), 0, s, partial, nb, 3, 1.0, out3);
    return hipGetLastError();
  }
};
template <class EQ, int K>
struct RunTotal {
  static hipError_t run(const Geo& g, const void* u, int lay, int comp, double* partial, int nb,
                        double* out, hipStream_t s) {
    if (lay == LMIX)
      hipLaunchKernelGGL((k_total_partial<EQ, K, LMIX>), dim3(nb), dim3(256), 0, s, g, u, comp, partial);
    else
      hipLaunchKernelGGL((k_total_partial<EQ, K, L64>), dim3(nb), dim3(256), 0, s, g, u, comp, partial);
    const double area = g.dx * (EQ::DIM == 2 ? g.dy : 1.0);
    hipLaunchKernelGGL(k_sum_final, dim3(1), dim3(256), 0, s, partial, nb, 1, area, out);
    return hipGetLastError();
  }
};
template <class EQ, int K>
struct RunProject {
  static hipError_t run(const PhysDev& ph, const Geo& g, int ic, const double* params,
                        const double* aux, double t, void* u, int lay, hipStream_t s) {
    if (lay == LMIX)
      hipLaunchKernelGGL((k_project<EQ, K, LMIX>), dim3(nblk(g.N, 256)), dim3(256), 0, s, ph, g, ic,
                         params, aux, t, u);
    else
      hipLaunchKernelGGL((k_project<EQ, K, L64>), dim3(nblk(g.N, 256)), dim3(256), 0, s, ph, g, ic,
                         params, aux, t, u);
    return hipGetLastError();
  }
};
template <class EQ, int K>
struct RunLimit {
  static hipError_t run(const PhysDev& ph, const Geo& g, const BCDev& bc, const LimitArgs& la,
                        bool mlp, void* u, int lay, uint8_t* flags, unsigned long long* counters,
                        hipStream_t s) {
    if (counters) hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(64), 0, s, counters, 3);
    const dim3 grid(nblk(g.N, 256));
    const bool dmr = EQ::EULER && bc.exact == CRKDG_IC_DMR;
    if (mlp && dmr) return hipErrorInvalidValue;  // the learned indicator has no DMR ghosts
    if (mlp) {
      if (lay == LMIX)
        hipLaunchKernelGGL((k_limit<EQ, K, LMIX, true, false>), grid, dim3(256), 0, s, ph, g, bc, la, u, flags, counters);
      else
        hipLaunchKernelGGL((k_limit<EQ, K, L64, true, false>), grid, dim3(256), 0, s, ph, g, bc, la, u, flags, counters);
    } else if (dmr) {
      if constexpr (EQ::EULER) {
        if (lay == LMIX)
          hipLaunchKernelGGL((k_limit<EQ, K, LMIX, false, true>), grid, dim3(256), 0, s, ph, g, bc, la, u, flags, counters);
        else
          hipLaunchKernelGGL((k_limit<EQ, K, L64, false, true>), grid, dim3(256), 0, s, ph, g, bc, la, u, flags, counters);
      }
    } else {
      if (lay == LMIX)
        hipLaunchKernelGGL((k_limit<EQ, K, LMIX, false, false>), grid, dim3(256), 0, s, ph, g, bc, la, u, flags, counters);
      else
        hipLaunchKernelGGL((k_limit<EQ, K, L64, false, false>), grid, dim3(256), 0, s, ph, g, bc, la, u, flags, counters);
    }
    return hipGetLastError();
  }
};

__global__ void k_time_set(double* t, double v) { *t = v; }
__global__ void k_time_add(double* t, const double* dt) { *t += *dt; }
hipError_t launch_time_set(double* t, double v, hipStream_t s) {
  hipLaunchKernelGGL(k_time_set, dim3(1), dim3(1), 0, s, t, v);
  return hipGetLastError();
}
hipError_t launch_time_add(double* t, const double* dt, hipStream_t s) {
  hipLaunchKernelGGL(k_time_add, dim3(1), dim3(1), 0, s, t, dt);
  return hipGetLastError();
}
hipError_t launch_inner(int eq, int k, int prec, const PhysDev& ph, const Geo& g,
                        const InnerArgs& a, hipStream_t s) {
  switch (prec) {
    case PBULK: return dispatch_mixed<InnerL<LMIX, LMIX, false>::template Run>(eq, k, ph, g, a, s);
    case PINNER:
    case PINC: return dispatch_mixed<InnerL<L64, L64, true>::template Run>(eq, k, ph, g, a, s);
    default: return dispatch<InnerL<L64, L64, false>::template Run>(eq, k, ph, g, a, s);
  }
}
hipError_t launch_final(int eq, int k, int prec, const PhysDev& ph, const Geo& g,
                        const BCDev& bc, const FinalArgs& a, hipStream_t s) {
  switch (prec) {
    case PBULK: return dispatch_mixed<FinalL<LMIX>::template Run>(eq, k, ph, g, bc, a, s);
    case PINC:  // FP32 increments over the FP64 u^n
      if (!a.base || a.base2) return hipErrorInvalidValue;
      return dispatch_mixed<FinalL<L64>::template Run>(eq, k, ph, g, bc, a, s);
    default: return dispatch<FinalL<L64>::template Run>(eq, k, ph, g, bc, a, s);  // FP64 final stage
  }
}
bool fused_supported(int eq, int k, int prec, const BCDev& bc) {
  return eq == EQ_EULER2 && (prec == PBULK || prec == P64) && (k == 1 || k == 2) &&
         bc.exact <= 0;
}
hipError_t launch_fused(int eq, int k, int prec, const PhysDev& ph, const Geo& g,
                        const BCDev& bc, const FusedArgs& a, hipStream_t s) {
  if (!fused_supported(eq, k, prec, bc) || a.s < 1 || a.s > MAXS) return hipErrorInvalidValue;
  FusedArgs am = a;
  am.strip = MARCH_H;
  const dim3 grid(nblk(g.nx, 62), nblk(g.ny, MARCH_H)), blk(256);
  if (prec == P64) {
    if (k == 1)
      hipLaunchKernelGGL((k_fused2<Euler2<double>, 1>), grid, blk, 0, s, ph, g, bc, am);
    else
      hipLaunchKernelGGL((k_fused2<Euler2<double>, 2>), grid, blk, 0, s, ph, g, bc, am);
  } else if (k == 1) {
    hipLaunchKernelGGL((k_fused2<Euler2<float>, 1>), grid, blk, 0, s, ph, g, bc, am);
  } else {
    hipLaunchKernelGGL((k_fused2<Euler2<float>, 2>), grid, blk, 0, s, ph, g, bc, am);
  }
  return hipGetLastError();
}
hipError_t launch_loc(int eq, int k, const PhysDev& ph, const Geo& g, const double* in,
                      double* out, hipStream_t s) {
  return dispatch<RunLoc>(eq, k, ph, g, in, out, s);
}
hipError_t launch_loc_combine(int eq, int k, const PhysDev& ph, const Geo& g,
                              const LocCombineArgs& a, hipStream_t s) {
  if (a.nx < 0 || a.nx > MAXS) return hipErrorInvalidValue;
  return dispatch<RunLocCombine>(eq, k, ph, g, a, s);
}
hipError_t launch_combine(long long n, double* out, const double* base, int nx,
                          const double* coef, const double* const* X, const double* dt_ptr,
                          hipStream_t s) {
  CombineArgs a{};
  a.out = out;
  a.base = base;
  a.n = nx;
  a.dt_ptr = dt_ptr;
  for (int j = 0; j < nx && j < MAXS; ++j) {
    a.X[j] = X[j];
    a.coef[j] = coef[j];
  }
#ifndef COMBINE_MAXBLK
#define COMBINE_MAXBLK 65536
#endif
  unsigned blocks = nblk(n / 2, 256);
  if (blocks > COMBINE_MAXBLK) blocks = COMBINE_MAXBLK;
  if (blocks == 0) blocks = 1;
  hipLaunchKernelGGL(k_combine, dim3(blocks), dim3(256), 0, s, n, a);
  return hipGetLastError();
}
hipError_t launch_wave_final(const double* partial, int n, double cfl, double* smax, double* dt,
                             hipStream_t s) {
  hipLaunchKernelGGL(k_wave_final, dim3(1), dim3(1024), 0, s, partial, n, cfl, smax, dt);
  return hipGetLastError();
}
hipError_t launch_wavespeed(int eq, int k, int lay, const PhysDev& ph, const Geo& g,
                            const void* u, double* partial, int nb, double cfl, double* smax,
                            double* dt, hipStream_t s) {
  return dispatch<RunWave>(eq, k, ph, g, u, lay, partial, nb, cfl, smax, dt, s);
}
hipError_t launch_error(int eq, int k, int lay, const PhysDev& ph, const Geo& g, const void* u,
                        int ic, const double* params, const double* aux, double t, int comp,
                        double* partial, int nb, double* out3, hipStream_t s) {
  return dispatch<RunError>(eq, k, ph, g, u, lay, ic, params, aux, t, comp, partial, nb, out3, s);
}
hipError_t launch_error_ref(const Geo& g, const double* ac, const double* af, int r, int ry,
                            long long nxf, double area, double* partial, int nb, double* out3,
                            hipStream_t s) {
  hipLaunchKernelGGL(k_error_ref_partial, dim3(nb), dim3(256), 0, s, g, ac, af, r, ry, nxf, area,
                     partial);
  hipLaunchKernelGGL(k_sum_final, dim3(1), dim3(256), 0, s, partial, nb, 3, 1.0, out3);
  return hipGetLastError();
}
hipError_t launch_total(int eq, int k, int lay, const Geo& g, const void* u, int comp,
                        double* partial, int nb, double* out, hipStream_t s) {
  return dispatch<RunTotal>(eq, k, g, u, lay, comp, partial, nb, out, s);
}
hipError_t launch_project(int eq, int k, int lay, const PhysDev& ph, const Geo& g, int ic,
                          const double* params, const double* aux, double t, void* u,
                          hipStream_t s) {
  return dispatch<RunProject>(eq, k, ph, g, ic, params, aux, t, u, lay, s);
}
hipError_t launch_limit(int eq, int k, int lay, const PhysDev& ph, const Geo& g,
                        const BCDev& bc, double M, const float* mlp_params, float tau_lo,
                        float tau_hi, void* u, uint8_t* flags, unsigned long long* counters,
                        double* wave_partial, hipStream_t s) {
  // probabilities to logit thresholds (monotone, so the decisions agree)
  auto logit = [](float p) -> float {
    if (!(p > 0.0f)) return -INFINITY;
    if (!(p < 1.0f)) return INFINITY;
    return (float)log((double)p / (1.0 - (double)p));
  };
  LimitArgs la{M, mlp_params, logit(tau_lo), logit(tau_hi), wave_partial};
  return dispatch<RunLimit>(eq, k, ph, g, bc, la, mlp_params != nullptr, u, lay, flags, counters, s);
}
hipError_t launch_mlp_features(int k, int lay, const Geo& g, const BCDev& bc, double M,
                               const void* u, float* X, hipStream_t s) {
  const dim3 grid(nblk(g.N, 256));
  switch (k * 4 + lay) {
    case 1 * 4 + L64: hipLaunchKernelGGL((k_mlp_features<1, L64>), grid, dim3(256), 0, s, g, bc, M, u, X); break;
    case 2 * 4 + L64: hipLaunchKernelGGL((k_mlp_features<2, L64>), grid, dim3(256), 0, s, g, bc, M, u, X); break;
    case 3 * 4 + L64: hipLaunchKernelGGL((k_mlp_features<3, L64>), grid, dim3(256), 0, s, g, bc, M, u, X); break;
    case 1 * 4 + LMIX: hipLaunchKernelGGL((k_mlp_features<1, LMIX>), grid, dim3(256), 0, s, g, bc, M, u, X); break;
    case 2 * 4 + LMIX: hipLaunchKernelGGL((k_mlp_features<2, LMIX>), grid, dim3(256), 0, s, g, bc, M, u, X); break;
    case 3 * 4 + LMIX: hipLaunchKernelGGL((k_mlp_features<3, LMIX>), grid, dim3(256), 0, s, g, bc, M, u, X); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace crk
