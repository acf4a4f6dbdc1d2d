// mlp_core.hpp -- the learned troubled-cell indicator (not part of the paper's
// method): a 12 -> 32 -> 32 -> 1 perceptron with ReLU hidden layers and a
// logistic output on per-cell stencil features.  Training runs in FP32 per
// lane; inference runs per wavefront on the bf16 matrix cores.
//
// Parameters are packed W1[32][12], b1[32], W2[32][32], b2[32], w3[32], b3.
// All lanes of a wave read the same weight at the same time, so the weights
// travel through the scalar cache into SGPR operands of the FMAs.
#pragma once
#include <hip/hip_runtime.h>

namespace crk {

constexpr int MLP_IN = 12, MLP_H1 = 32, MLP_H2 = 32;
constexpr int MLP_OW1 = 0;
constexpr int MLP_OB1 = MLP_OW1 + MLP_H1 * MLP_IN;
constexpr int MLP_OW2 = MLP_OB1 + MLP_H1;
constexpr int MLP_OB2 = MLP_OW2 + MLP_H2 * MLP_H1;
constexpr int MLP_OW3 = MLP_OB2 + MLP_H2;
constexpr int MLP_OB3 = MLP_OW3 + MLP_H2;
constexpr int MLP_NPAR = MLP_OB3 + 1;  // 1505

__device__ __forceinline__ float relu_f(float v) { return v > 0.0f ? v : 0.0f; }

// forward pass in FP32 (training semantics); optionally keeps the hidden
// activations
template <bool KEEP>
__device__ __forceinline__ float mlp_forward1(const float* __restrict__ P, const float (&x)[MLP_IN],
                                              float* h1o = nullptr, float* h2o = nullptr) {
  float h1[MLP_H1];
#pragma unroll
  for (int o = 0; o < MLP_H1; ++o) {
    float s = P[MLP_OB1 + o];
#pragma unroll
    for (int i = 0; i < MLP_IN; ++i) s = s + P[MLP_OW1 + o * MLP_IN + i] * x[i];
    h1[o] = relu_f(s);
  }
  float z = P[MLP_OB3];
#pragma unroll 4
  for (int o = 0; o < MLP_H2; ++o) {
    float s = P[MLP_OB2 + o];
#pragma unroll
    for (int i = 0; i < MLP_H1; ++i) s = s + P[MLP_OW2 + o * MLP_H1 + i] * h1[i];
    const float h2 = relu_f(s);
    if (KEEP) h2o[o] = h2;
    z = z + P[MLP_OW3 + o] * h2;
  }
  if (KEEP)
#pragma unroll
    for (int o = 0; o < MLP_H1; ++o) h1o[o] = h1[o];
  return z;
}

// ---------------------------------------------------------------------------
// Inference at bfloat16 on the matrix cores: one wavefront evaluates its 64
// lanes' feature vectors together.  Layers 1 and 2 are 32x32x16 bf16 MFMAs
// (features, W1, W2 and the first hidden layer rounded to bf16, round to
// nearest even; FP32 accumulation; biases added in FP32 afterwards); the
// second hidden layer and the output stay FP32.  Operand layouts of
// v_mfma_f32_32x32x16_bf16: lane l supplies row (A) / column (B) l % 32 and
// the 8 k-values (l / 32) * 8 ... + 7; accumulator element j of lane l is
// row (j / 4) * 8 + (l / 32) * 4 + j % 4, column l % 32.  The transposes
// between layers go through a per-wave LDS scratch.
// ---------------------------------------------------------------------------
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

struct MlpWaveSmem {
  union {
    struct {
      __bf16 x[64][16];   // features, padded 12 -> 16
      __bf16 h1[64][32];  // first hidden layer
    };
    float h2[32][36];     // second hidden layer, one half of the rows at a time,
                          // written once x and h1 are read (rows of 144 B:
                          // 16-byte aligned, consecutive rows 4 banks apart)
  };
};
// W1 and W2 in bf16, already in the matrix cores' B-operand order: lane l
// reads its 8 values of W1 and twice 8 of W2 with three 16-byte loads
struct MlpWeightsSmem {
  bf16x8 w1[64], w2a[64], w2b[64];
};

// the block stages the weights once (every thread calls this, then the
// block synchronises)
__device__ __forceinline__ void mlp_stage_weights(const float* __restrict__ P,
                                                  MlpWeightsSmem& ws) {
  for (int t = threadIdx.x; t < 3 * 64 * 8; t += blockDim.x) {
    const int which = t / 512, l = (t / 8) & 63, e = t & 7;
    const int n = l & 31, k = (l >> 5) * 8 + e;
    float v;
    if (which == 0) v = k < MLP_IN ? P[MLP_OW1 + n * MLP_IN + k] : 0.0f;
    else if (which == 1) v = P[MLP_OW2 + n * MLP_H1 + k];
    else v = P[MLP_OW2 + n * MLP_H1 + 16 + k];
    bf16x8* dst = which == 0 ? ws.w1 : which == 1 ? ws.w2a : ws.w2b;
    dst[l][e] = (__bf16)v;
  }
}

// order this wave's LDS accesses (they complete in issue order on the
// hardware; this keeps the compiler from moving them across)
__device__ __forceinline__ void wave_lds_fence() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// every lane of the wave must call this (uniform control flow), after the
// block has staged the weights
__device__ __forceinline__ float mlp_infer_wave(const float* __restrict__ P,
                                                const MlpWeightsSmem& ws,
                                                const float (&x)[MLP_IN], MlpWaveSmem& sm) {
  const int l = threadIdx.x & 63;
  const int n = l & 31, kb = (l >> 5) * 8;
  {
    bf16x8 lo, hi;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      lo[e] = (__bf16)x[e];
      hi[e] = (__bf16)(e + 8 < MLP_IN ? x[e + 8] : 0.0f);
    }
    *reinterpret_cast<bf16x8*>(&sm.x[l][0]) = lo;
    *reinterpret_cast<bf16x8*>(&sm.x[l][8]) = hi;
  }
  const bf16x8 w1 = ws.w1[l], w2a = ws.w2a[l], w2b = ws.w2b[l];
  const float b1 = P[MLP_OB1 + n], b2 = P[MLP_OB2 + n];
  wave_lds_fence();
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const bf16x8 a = *reinterpret_cast<const bf16x8*>(&sm.x[h * 32 + n][kb]);
    f32x16 c = {};
    c = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, w1, c, 0, 0, 0);
#pragma unroll
    for (int j = 0; j < 16; ++j) {
      const int r = (j >> 2) * 8 + (l >> 5) * 4 + (j & 3);
      sm.h1[h * 32 + r][n] = (__bf16)relu_f(c[j] + b1);
    }
  }
  wave_lds_fence();
  bf16x8 a0[2], a1[2];  // all of layer 2's inputs, before h2 overwrites them
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    a0[h] = *reinterpret_cast<const bf16x8*>(&sm.h1[h * 32 + n][kb]);
    a1[h] = *reinterpret_cast<const bf16x8*>(&sm.h1[h * 32 + n][16 + kb]);
  }
  wave_lds_fence();
  typedef float f32x4 __attribute__((ext_vector_type(4)));
  float z = 0.0f;
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    f32x16 c = {};
    c = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a0[h], w2a, c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a1[h], w2b, c, 0, 0, 0);
#pragma unroll
    for (int j = 0; j < 16; ++j) {
      const int r = (j >> 2) * 8 + (l >> 5) * 4 + (j & 3);
      sm.h2[r][n] = relu_f(c[j] + b2);
    }
    wave_lds_fence();
    // lane l's row is row l % 32 of half l / 32
    if ((l >> 5) == h) {
      z = P[MLP_OB3];
#pragma unroll
      for (int q = 0; q < MLP_H2 / 4; ++q) {
        const f32x4 v = *reinterpret_cast<const f32x4*>(&sm.h2[n][4 * q]);
#pragma unroll
        for (int e = 0; e < 4; ++e) z = z + P[MLP_OW3 + 4 * q + e] * v[e];
      }
    }
    wave_lds_fence();  // the half is read before the next one overwrites it
  }
  return z;
}

// 12 stencil features of one cell (computed in FP64, returned in FP32): for
// q in {density, energy} and direction d in {x, y}, with a / at the forward /
// backward trace-average jumps, dp / dm the differences of neighbouring cell
// averages and s = |dp| + |dm| + M h_d^2 + 1e-300:  a/s, at/s, (dp - dm)/s.
// a[d][c] and at[d][c] are the jumps of component c in direction d.
__device__ __forceinline__ void cell_features_jumps(const double (&a)[2][4], const double (&at)[2][4],
                                                    const double (&dp)[2][4], const double (&dm)[2][4],
                                                    double Mh2x, double Mh2y, float (&x)[MLP_IN]) {
#pragma unroll
  for (int qi = 0; qi < 2; ++qi) {
    const int c = qi ? 3 : 0;
#pragma unroll
    for (int d = 0; d < 2; ++d) {
      const double s = fabs(dp[d][c]) + fabs(dm[d][c]) + (d == 0 ? Mh2x : Mh2y) + 1e-300;
      const double is = 1.0 / s;  // one division; FP64 products, then rounded to FP32
      float* xo = x + (qi * 2 + d) * 3;
      xo[0] = (float)(a[d][c] * is);
      xo[1] = (float)(at[d][c] * is);
      xo[2] = (float)((dp[d][c] - dm[d][c]) * is);
    }
  }
}

// the jumps along the cell's centre lines from its modes (mode m + Q n):
// u(+1) - avg = sum of the modes of degree 1..Q-1 in that direction, and
// avg - u(-1) = the same sum with the even degrees negated
template <int NB, int Q>
__device__ __forceinline__ void trace_jumps(const double (&U)[4][NB], double (&a)[2][4],
                                            double (&at)[2][4]) {
#pragma unroll
  for (int c = 0; c < 4; ++c)
#pragma unroll
    for (int d = 0; d < 2; ++d) {
      double s = 0.0, st = 0.0;
#pragma unroll
      for (int deg = 1; deg < Q; ++deg) {
        const double v = U[c][d == 0 ? deg : deg * Q];
        s += v;
        st += (deg % 2) ? v : -v;
      }
      a[d][c] = s;
      at[d][c] = st;
    }
}

template <int NB, int Q>
__device__ __forceinline__ void cell_features(const double (&U)[4][NB], const double (&dp)[2][4],
                                              const double (&dm)[2][4], double Mh2x, double Mh2y,
                                              float (&x)[MLP_IN]) {
  double a[2][4], at[2][4];
  trace_jumps<NB, Q>(U, a, at);
  cell_features_jumps(a, at, dp, dm, Mh2x, Mh2y, x);
}

}  // namespace crk
