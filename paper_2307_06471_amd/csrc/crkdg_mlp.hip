// crkdg_mlp.hip -- training kernels of the learned troubled-cell indicator
// (not part of the paper's method; FP32).
//
//   k_mlp_forward       logits of a batch of feature vectors, by the limiter's
//                       inference routine (FP32 matrix cores)
//   k_mlp_grad_partial  forward + backward of 64 samples per workgroup: each
//                       lane runs one sample, the activations go to LDS, then
//                       each lane sums a fixed subset of the 1505 parameter
//                       gradients over the 64 samples in a fixed order
//   k_mlp_grad_final    sums the workgroup partials in a fixed order, so the
//                       gradient is bitwise reproducible
//   k_mlp_adam          Adam with bias correction
//
// Loss: the mean over the batch of the weighted binary cross-entropy with
// logits, pw * y * softplus(-z) + (1 - y) * softplus(z).
#include <math.h>

#include <mutex>

#include "crkdg_internal.hpp"
#include "mlp_core.hpp"

namespace crk {

constexpr int MB = 64;  // samples per workgroup of the gradient kernel
constexpr int NPART = MLP_NPAR + 1;  // partial gradients + partial loss

// logits by the limiter's inference routine
__global__ __launch_bounds__(256) void k_mlp_forward(const float* __restrict__ P,
                                                     const float* __restrict__ X, int B,
                                                     float* __restrict__ out) {
  __shared__ MlpWeightsSmem ws;
  mlp_stage_weights(P, ws);
  __syncthreads();
  const int n = blockIdx.x * 256 + threadIdx.x;
  float x[MLP_IN];
#pragma unroll
  for (int i = 0; i < MLP_IN; ++i) x[i] = n < B ? X[(long long)n * MLP_IN + i] : 0.0f;
  const float z = mlp_infer_wave(P, ws, x);
  if (n < B) out[n] = z;
}

__device__ __forceinline__ float softplus_f(float x) {
  return fmaxf(x, 0.0f) + log1pf(expf(-fabsf(x)));
}

__global__ __launch_bounds__(MB) void k_mlp_grad_partial(const float* __restrict__ P,
                                                         const float* __restrict__ X,
                                                         const uint8_t* __restrict__ y, int B,
                                                         float pw, float* __restrict__ partial) {
  __shared__ float sx[MB][MLP_IN];
  __shared__ float sh1[MB][MLP_H1];
  __shared__ float sh2[MB][MLP_H2];
  __shared__ float sd1[MB][MLP_H1];
  __shared__ float sd2[MB][MLP_H2];
  __shared__ float sdz[MB];
  __shared__ float sloss[MB];
  const int t = threadIdx.x;
  const int n = blockIdx.x * MB + t;
  const float invB = 1.0f / (float)B;
  if (n < B) {
    float x[MLP_IN], h1[MLP_H1], h2[MLP_H2];
#pragma unroll
    for (int i = 0; i < MLP_IN; ++i) x[i] = X[(long long)n * MLP_IN + i];
    const float z = mlp_forward1<true>(P, x, h1, h2);
    const float yy = y[n] ? 1.0f : 0.0f;
    const float sg = 1.0f / (1.0f + expf(-z));
    sloss[t] = pw * yy * softplus_f(-z) + (1.0f - yy) * softplus_f(z);
    const float dz = (-pw * yy * (1.0f - sg) + (1.0f - yy) * sg) * invB;
    sdz[t] = dz;
    float d2[MLP_H2];
#pragma unroll
    for (int o = 0; o < MLP_H2; ++o) {
      d2[o] = h2[o] > 0.0f ? dz * P[MLP_OW3 + o] : 0.0f;
      sd2[t][o] = d2[o];
      sh2[t][o] = h2[o];
    }
#pragma unroll 4
    for (int i = 0; i < MLP_H1; ++i) {
      float s = 0.0f;
#pragma unroll
      for (int o = 0; o < MLP_H2; ++o) s = s + P[MLP_OW2 + o * MLP_H1 + i] * d2[o];
      sd1[t][i] = h1[i] > 0.0f ? s : 0.0f;
      sh1[t][i] = h1[i];
    }
#pragma unroll
    for (int i = 0; i < MLP_IN; ++i) sx[t][i] = x[i];
  } else {
    for (int i = 0; i < MLP_IN; ++i) sx[t][i] = 0.0f;
    for (int o = 0; o < MLP_H1; ++o) sh1[t][o] = sd1[t][o] = 0.0f;
    for (int o = 0; o < MLP_H2; ++o) sh2[t][o] = sd2[t][o] = 0.0f;
    sdz[t] = 0.0f;
    sloss[t] = 0.0f;
  }
  __syncthreads();
  float* out = partial + (long long)blockIdx.x * NPART;
  for (int p = t; p < MLP_NPAR; p += MB) {
    float g = 0.0f;
    if (p < MLP_OB1) {
      const int o = p / MLP_IN, i = p % MLP_IN;
      for (int s = 0; s < MB; ++s) g = g + sd1[s][o] * sx[s][i];
    } else if (p < MLP_OW2) {
      const int o = p - MLP_OB1;
      for (int s = 0; s < MB; ++s) g = g + sd1[s][o];
    } else if (p < MLP_OB2) {
      const int q = p - MLP_OW2, o = q / MLP_H1, i = q % MLP_H1;
      for (int s = 0; s < MB; ++s) g = g + sd2[s][o] * sh1[s][i];
    } else if (p < MLP_OW3) {
      const int o = p - MLP_OB2;
      for (int s = 0; s < MB; ++s) g = g + sd2[s][o];
    } else if (p < MLP_OB3) {
      const int o = p - MLP_OW3;
      for (int s = 0; s < MB; ++s) g = g + sdz[s] * sh2[s][o];
    } else {
      for (int s = 0; s < MB; ++s) g = g + sdz[s];
    }
    out[p] = g;
  }
  if (t == 0) {
    float l = 0.0f;
    for (int s = 0; s < MB; ++s) l = l + sloss[s];
    out[MLP_NPAR] = l;
  }
}

__global__ __launch_bounds__(256) void k_mlp_grad_final(const float* __restrict__ partial, int nblk,
                                                        int B, float* __restrict__ grad,
                                                        float* __restrict__ loss) {
  const int p = blockIdx.x * 256 + threadIdx.x;
  if (p >= NPART) return;
  float s = 0.0f;
  for (int b = 0; b < nblk; ++b) s = s + partial[(long long)b * NPART + p];
  if (p < MLP_NPAR)
    grad[p] = s;
  else if (loss)
    loss[0] = s / (float)B;
}

__global__ __launch_bounds__(256) void k_mlp_adam(float* __restrict__ P, float* __restrict__ m1,
                                                  float* __restrict__ m2,
                                                  const float* __restrict__ g, float c1, float c2,
                                                  float lr, float b1, float b2, float eps) {
  const int p = blockIdx.x * 256 + threadIdx.x;
  if (p >= MLP_NPAR) return;
  const float gp = g[p];
  const float a = b1 * m1[p] + (1.0f - b1) * gp;
  const float v = b2 * m2[p] + (1.0f - b2) * gp * gp;
  m1[p] = a;
  m2[p] = v;
  P[p] = P[p] - lr * (a / c1) / (sqrtf(v / c2) + eps);
}

size_t mlp_work_floats(int B) { return (size_t)((B + MB - 1) / MB) * NPART; }

hipError_t launch_mlp_forward(const float* P, const float* X, int B, float* logits, hipStream_t s) {
  hipLaunchKernelGGL(k_mlp_forward, dim3((B + 255) / 256), dim3(256), 0, s, P, X, B, logits);
  return hipGetLastError();
}

hipError_t launch_mlp_grad(const float* P, const float* X, const uint8_t* y, int B, float pw,
                           float* grad, float* loss, float* work, hipStream_t s) {
  const int nblk = (B + MB - 1) / MB;
  hipLaunchKernelGGL(k_mlp_grad_partial, dim3(nblk), dim3(MB), 0, s, P, X, y, B, pw, work);
  hipLaunchKernelGGL(k_mlp_grad_final, dim3((NPART + 255) / 256), dim3(256), 0, s, work, nblk, B,
                     grad, loss);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// The gradient without caller work memory: the workgroup partials live in a
// file-scope device array (one copy per GPU, held until the process ends)
// sized for batches of up to MLP_NOALLOC_MAX_B samples.  Host code never
// passes the array's name to a kernel (on the host it is only a stand-in for
// the symbol); each device's address comes from hipGetSymbolAddress, taken
// once per device with that device current, and the kernels get that.
// ---------------------------------------------------------------------------
constexpr int MLP_NOALLOC_MAX_B = 16384;
constexpr size_t MLP_NOALLOC_FLOATS = (size_t)((MLP_NOALLOC_MAX_B + MB - 1) / MB) * NPART;
static __device__ __align__(256) float scratch[MLP_NOALLOC_FLOATS];

constexpr int MLP_NOALLOC_MAX_DEVICES = 64;
static std::mutex g_scratch_mu;
static float* g_scratch_ptr[MLP_NOALLOC_MAX_DEVICES];

// this device's address of `scratch` (resolved on the first call per device)
static hipError_t noalloc_scratch(float** out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= MLP_NOALLOC_MAX_DEVICES) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!ptr) return hipErrorInvalidSymbol;
    g_scratch_ptr[dev] = (float*)ptr;
  }
  *out = g_scratch_ptr[dev];
  return hipSuccess;
}

int mlp_noalloc_max_batch() { return MLP_NOALLOC_MAX_B; }

// the same two kernels as launch_mlp_grad, partials in `scratch` (every
// partial a later read uses is written first in stream order, so nothing
// needs clearing)
hipError_t launch_mlp_grad_noalloc(const float* P, const float* X, const uint8_t* y, int B,
                                   float pw, float* grad, float* loss, hipStream_t s) {
  if (B < 1 || B > MLP_NOALLOC_MAX_B) return hipErrorInvalidValue;
  float* work = nullptr;
  hipError_t e = noalloc_scratch(&work);
  if (e != hipSuccess) return e;
  return launch_mlp_grad(P, X, y, B, pw, grad, loss, work, s);
}

hipError_t launch_mlp_adam(float* P, float* m1, float* m2, const float* grad, int step, float lr,
                           float b1, float b2, float eps, hipStream_t s) {
  const float c1 = 1.0f - powf(b1, (float)step), c2 = 1.0f - powf(b2, (float)step);
  hipLaunchKernelGGL(k_mlp_adam, dim3((MLP_NPAR + 255) / 256), dim3(256), 0, s, P, m1, m2, grad, c1,
                     c2, lr, b1, b2, eps);
  return hipGetLastError();
}

}  // namespace crk
