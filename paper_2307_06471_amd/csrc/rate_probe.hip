// rate_probe.hip -- a stand-alone measurement (not part of the library): the
// FP32 rates one MI355X reaches with the vector and the matrix units, which
// the design of the step kernels rests on.
//
//  1. v_fma_f32 issue rate by wavefronts per SIMD (1, 2, 3, 4, 8) and by
//     independent FMA chains per lane (1, 2, 4, 8): how fast a kernel held
//     to a given occupancy by its registers can issue FP32 work.
//  2. FP32 matrix rate of v_mfma_f32_16x16x4_f32 and v_mfma_f32_32x32x2_f32
//     (independent accumulators) against the vector FMA rate.
//
// Build and run (gfx950):
//   hipcc --offload-arch=gfx950 -O3 -Xclang -target-feature -Xclang -packed-fp32-ops \
//     paper_2307_06471_amd/csrc/rate_probe.hip -o rate_probe && ./rate_probe
#include <hip/hip_runtime.h>

#include <cstdio>

typedef float v4f __attribute__((ext_vector_type(4)));
typedef float v16f __attribute__((ext_vector_type(16)));

#define CHECK(x)                                                              \
  do {                                                                        \
    hipError_t e_ = (x);                                                      \
    if (e_ != hipSuccess) {                                                   \
      std::fprintf(stderr, "%s: %s\n", #x, hipGetErrorString(e_));           \
      return 1;                                                               \
    }                                                                         \
  } while (0)

template <int CH>
__global__ __launch_bounds__(256) void k_fma(float* out, int iters, float x) {
  float r[CH];
  for (int i = 0; i < CH; ++i) r[i] = x + i + threadIdx.x;
  const float m = 0.999f, c = 1e-3f;
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int i = 0; i < CH; ++i) r[i] = fmaf(r[i], m, c);
  }
  float s = 0.f;
  for (int i = 0; i < CH; ++i) s += r[i];
  out[blockIdx.x * blockDim.x + threadIdx.x] = s;
}

__global__ __launch_bounds__(256) void k_mfma16(float* out, int iters, float x) {
  v4f acc[4];
  for (int i = 0; i < 4; ++i) acc[i] = v4f{0.f, 0.f, 0.f, 0.f};
  const float a = x + threadIdx.x, b = x - threadIdx.x;
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int i = 0; i < 4; ++i) acc[i] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc[i], 0, 0, 0);
  }
  float s = 0.f;
  for (int i = 0; i < 4; ++i) s += acc[i][0] + acc[i][1] + acc[i][2] + acc[i][3];
  out[blockIdx.x * blockDim.x + threadIdx.x] = s;
}

__global__ __launch_bounds__(256) void k_mfma32(float* out, int iters, float x) {
  v16f acc[2];
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 16; ++j) acc[i][j] = 0.f;
  const float a = x + threadIdx.x, b = x - threadIdx.x;
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int i = 0; i < 2; ++i) acc[i] = __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, acc[i], 0, 0, 0);
  }
  float s = 0.f;
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 16; ++j) s += acc[i][j];
  out[blockIdx.x * blockDim.x + threadIdx.x] = s;
}

// best of three launches, in ms
template <class F>
static int time_ms(F launch, float* best) {
  hipEvent_t e0, e1;
  CHECK(hipEventCreate(&e0));
  CHECK(hipEventCreate(&e1));
  *best = 1e30f;
  for (int rep = 0; rep < 3; ++rep) {
    CHECK(hipEventRecord(e0));
    launch();
    CHECK(hipGetLastError());
    CHECK(hipEventRecord(e1));
    CHECK(hipEventSynchronize(e1));
    float ms;
    CHECK(hipEventElapsedTime(&ms, e0, e1));
    if (ms < *best) *best = ms;
  }
  CHECK(hipEventDestroy(e0));
  CHECK(hipEventDestroy(e1));
  return 0;
}

template <int CH>
static int fma_row(float* out, int wps, int iters, double clock_ghz, int simds) {
  const int blocks = simds / 4 * wps;  // four wavefronts per block
  float ms;
  if (time_ms([&] { hipLaunchKernelGGL(k_fma<CH>, dim3(blocks), dim3(256), 0, 0, out, iters, 1.0f); },
              &ms))
    return 1;
  const double instr = (double)blocks * 4 * iters * CH;  // wave64 instructions
  std::printf("v_fma_f32  waves/SIMD %d  chains %d: %8.3f ms  %6.1f TFLOP/s  %5.2f cycles per "
              "wave64 instruction per SIMD\n",
              wps, CH, ms, instr * 64 * 2 / (ms * 1e-3) / 1e12,
              ms * 1e-3 * clock_ghz * 1e9 / (instr / simds));
  return 0;
}

int main() {
  hipDeviceProp_t prop;
  CHECK(hipGetDeviceProperties(&prop, 0));
  const int simds = prop.multiProcessorCount * 4;
  const double clock_ghz = prop.clockRate / 1e6;
  std::printf("%s: %d compute units, %d SIMDs, %.2f GHz peak engine clock\n", prop.gcnArchName,
              prop.multiProcessorCount, simds, clock_ghz);
  float* out;
  const size_t n = (size_t)simds / 4 * 8 * 256;
  CHECK(hipMalloc(&out, sizeof(float) * n));
  const int iters = 8192;
  for (int wps : {1, 2, 3, 4, 8}) {
    if (fma_row<1>(out, wps, iters, clock_ghz, simds) || fma_row<2>(out, wps, iters, clock_ghz, simds) ||
        fma_row<4>(out, wps, iters, clock_ghz, simds) || fma_row<8>(out, wps, iters, clock_ghz, simds))
      return 1;
  }
  const int blocks = simds / 4 * 4, miters = 4096;  // four wavefronts per SIMD
  const double waves = blocks * 4.0;
  float ms;
  if (time_ms([&] { hipLaunchKernelGGL(k_mfma16, dim3(blocks), dim3(256), 0, 0, out, miters, 1.0f); },
              &ms))
    return 1;
  std::printf("v_mfma_f32_16x16x4_f32 (4 waves/SIMD, 4 accumulators): %6.1f TFLOP/s\n",
              waves * miters * 4 * 16 * 16 * 4 * 2 / (ms * 1e-3) / 1e12);
  if (time_ms([&] { hipLaunchKernelGGL(k_mfma32, dim3(blocks), dim3(256), 0, 0, out, miters, 1.0f); },
              &ms))
    return 1;
  std::printf("v_mfma_f32_32x32x2_f32 (4 waves/SIMD, 2 accumulators): %6.1f TFLOP/s\n",
              waves * miters * 2 * 32 * 32 * 2 * 2 / (ms * 1e-3) / 1e12);
  CHECK(hipDeviceSynchronize());
  CHECK(hipFree(out));
  return 0;
}
