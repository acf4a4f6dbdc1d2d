// mlp_core.hpp -- the learned troubled-cell indicator (not part of the paper's
// method): a 12 -> 32 -> 32 -> 1 perceptron with ReLU hidden layers and a
// logistic output on per-cell stencil features.  Training runs in FP32 per
// lane; inference runs per wavefront on the FP32 matrix cores.
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
// Inference in FP32 on the matrix cores: one wavefront evaluates its 64
// cells as two groups of 32 (group h: the cells of lanes 32h .. 32h + 31).
// v_mfma_f32_32x32x2_f32 computes D[32x32] += A[32x2] B[2x32] in FP32; lane l
// supplies A[l % 32][l / 32] and B[l / 32][l % 32], and accumulator element j
// of lane l is D[r(j, l)][l % 32] with r(j, l) = 8 (j / 4) + 4 (l / 32) + j % 4.
//   layer 1  D1 = [W1 | b1] [x; 1]: neurons are rows, cells columns, seven
//            steps over the 12 features and the bias row (padded to 14); a
//            lane holds features of its own cell, and one v_permlane32_swap
//            per feature pair gives both groups' B operands;
//   layer 2  D2 = [W2 | b2] [h1; 1]: step j (j < 16) contracts the two input
//            neurons r(j, 0) and r(j, 32), exactly the layer-1 accumulator
//            element j the lane already holds, so relu(D1) feeds layer 2 in
//            place; step 16 adds the bias;
//   output   each lane sums w3 relu(D2) over its 16 neurons, and the two
//            lanes of a cell (l and l ^ 32) add their halves after one more
//            permlane swap.
// No value is rounded below FP32 and no activation passes through LDS.
// ---------------------------------------------------------------------------
typedef float f32x16 __attribute__((ext_vector_type(16)));

constexpr int MLP_S1 = (MLP_IN + 2) / 2;  // layer-1 steps: 12 features + bias row
constexpr int MLP_S2 = MLP_H1 / 2 + 1;    // layer-2 steps: 32 inputs + bias row

__device__ __forceinline__ int mlp_acc_row(int j, int l) {
  return 8 * (j >> 2) + 4 * ((l >> 5) & 1) + (j & 3);
}

// the weights in the matrix cores' A-operand order per step and lane (and
// the output weights in accumulator order): each lane reads one float per
// step, consecutive lanes consecutive words
struct MlpWeightsSmem {
  float w1[MLP_S1][64];
  float w2[MLP_S2][64];
  float w3[16][64];
};

// the block stages the weights once (every thread calls this, then the
// block synchronises)
__device__ __forceinline__ void mlp_stage_weights(const float* __restrict__ P,
                                                  MlpWeightsSmem& ws) {
  constexpr int NS = MLP_S1 + MLP_S2 + 16;
  for (int t = threadIdx.x; t < NS * 64; t += blockDim.x) {
    const int step = t >> 6, l = t & 63, n = l & 31, hi = l >> 5;
    if (step < MLP_S1) {
      const int kk = 2 * step + hi;  // feature index; MLP_IN is the bias row
      ws.w1[step][l] = kk < MLP_IN ? P[MLP_OW1 + n * MLP_IN + kk]
                                   : (kk == MLP_IN ? P[MLP_OB1 + n] : 0.0f);
    } else if (step < MLP_S1 + MLP_S2) {
      const int j = step - MLP_S1;
      ws.w2[j][l] = j < MLP_S2 - 1 ? P[MLP_OW2 + n * MLP_H1 + mlp_acc_row(j, l)]
                                   : (hi ? 0.0f : P[MLP_OB2 + n]);
    } else {
      const int j = step - MLP_S1 - MLP_S2;
      ws.w3[j][l] = P[MLP_OW3 + mlp_acc_row(j, l)];
    }
  }
}

// swap lanes 32..63 of a with lanes 0..31 of b
__device__ __forceinline__ void lane_half_swap(float& a, float& b) {
  const auto r = __builtin_amdgcn_permlane32_swap(__builtin_bit_cast(unsigned, a),
                                                  __builtin_bit_cast(unsigned, b), false, false);
  a = __builtin_bit_cast(float, (unsigned)r[0]);
  b = __builtin_bit_cast(float, (unsigned)r[1]);
}

// logit of this lane's cell; every lane of the wave must call this (uniform
// control flow), after the block has staged the weights
__device__ __forceinline__ float mlp_infer_wave(const float* __restrict__ P,
                                                const MlpWeightsSmem& ws,
                                                const float (&x)[MLP_IN]) {
  const int l = threadIdx.x & 63;
  const float one = l < 32 ? 1.0f : 0.0f;  // B operand of a bias step
  f32x16 d0 = {}, d1 = {};
#pragma unroll
  for (int s = 0; s < MLP_S1; ++s) {
    float b0 = one, b1 = one;
    if (2 * s + 1 < MLP_IN) {
      b0 = x[2 * s];
      b1 = x[2 * s + 1];
      lane_half_swap(b0, b1);  // b0: group 0's operand, b1: group 1's
    }
    const float a = ws.w1[s][l];
    d0 = __builtin_amdgcn_mfma_f32_32x32x2f32(a, b0, d0, 0, 0, 0);
    d1 = __builtin_amdgcn_mfma_f32_32x32x2f32(a, b1, d1, 0, 0, 0);
  }
  float part[2];
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const f32x16& d = h ? d1 : d0;
    f32x16 e = {};
#pragma unroll
    for (int j = 0; j < MLP_S2 - 1; ++j)
      e = __builtin_amdgcn_mfma_f32_32x32x2f32(ws.w2[j][l], relu_f(d[j]), e, 0, 0, 0);
    e = __builtin_amdgcn_mfma_f32_32x32x2f32(ws.w2[MLP_S2 - 1][l], one, e, 0, 0, 0);
    float z = 0.0f;
#pragma unroll
    for (int j = 0; j < 16; ++j) z = z + ws.w3[j][l] * relu_f(e[j]);
    part[h] = z;
  }
  lane_half_swap(part[0], part[1]);
  return P[MLP_OB3] + (part[0] + part[1]);
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
