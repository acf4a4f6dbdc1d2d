// mlp_core.hpp -- the learned troubled-cell indicator (not part of the paper's
// method): a 12 -> 32 -> 32 -> 1 perceptron with tanh hidden layers and a
// logistic output, evaluated per cell in FP32 on stencil features.
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

// tanh from the hardware exponential: 1 - 2 / (exp(2x) + 1); absolute error
// ~1e-7, saturates correctly for large |x|
__device__ __forceinline__ float tanh_fast(float x) {
  const float e = __expf(2.0f * x);
  return 1.0f - __fdividef(2.0f, e + 1.0f);
}

// forward pass; optionally keeps the hidden activations
template <bool KEEP>
__device__ __forceinline__ float mlp_forward1(const float* __restrict__ P, const float (&x)[MLP_IN],
                                              float* h1o = nullptr, float* h2o = nullptr) {
  float h1[MLP_H1];
#pragma unroll
  for (int o = 0; o < MLP_H1; ++o) {
    float s = P[MLP_OB1 + o];
#pragma unroll
    for (int i = 0; i < MLP_IN; ++i) s = s + P[MLP_OW1 + o * MLP_IN + i] * x[i];
    h1[o] = tanh_fast(s);
  }
  float z = P[MLP_OB3];
#pragma unroll 4
  for (int o = 0; o < MLP_H2; ++o) {
    float s = P[MLP_OB2 + o];
#pragma unroll
    for (int i = 0; i < MLP_H1; ++i) s = s + P[MLP_OW2 + o * MLP_H1 + i] * h1[i];
    const float h2 = tanh_fast(s);
    if (KEEP) h2o[o] = h2;
    z = z + P[MLP_OW3 + o] * h2;
  }
  if (KEEP)
#pragma unroll
    for (int o = 0; o < MLP_H1; ++o) h1o[o] = h1[o];
  return z;
}

// 12 stencil features of one cell (computed in FP64, returned in FP32): for
// q in {density, energy} and direction d in {x, y}, with a / at the forward /
// backward trace-average jumps, dp / dm the differences of neighbouring cell
// averages and s = |dp| + |dm| + M h_d^2 + 1e-300:  a/s, at/s, (dp - dm)/s
template <int NB, int Q>
__device__ __forceinline__ void cell_features(const double (&U)[4][NB], const double (&dp)[2][4],
                                              const double (&dm)[2][4], double Mh2x, double Mh2y,
                                              float (&x)[MLP_IN]) {
#pragma unroll
  for (int qi = 0; qi < 2; ++qi) {
    const int c = qi ? 3 : 0;
#pragma unroll
    for (int d = 0; d < 2; ++d) {
      double a = 0.0, at = 0.0;
#pragma unroll
      for (int deg = 1; deg < Q; ++deg) {
        const double v = U[c][d == 0 ? deg : deg * Q];
        a += v;
        at += (deg % 2) ? v : -v;
      }
      const double s = fabs(dp[d][c]) + fabs(dm[d][c]) + (d == 0 ? Mh2x : Mh2y) + 1e-300;
      float* xo = x + (qi * 2 + d) * 3;
      xo[0] = (float)(a / s);
      xo[1] = (float)(at / s);
      xo[2] = (float)((dp[d][c] - dm[d][c]) / s);
    }
  }
}

}  // namespace crk
