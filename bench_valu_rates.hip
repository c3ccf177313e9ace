// Issue-rate probe behind the benchmark's VALU slot weights: wave-instructions per cycle per
// compute unit for an FP32 FMA, an FP64 FMA, the FP32 log2 of the transcendental unit and the
// 32 x 32 -> 64-bit integer multiply-add of Philox, each in eight independent chains per lane
// so that issue, not latency, limits the loop.  Every thread writes one result to its own
// slot of the output buffer (grid = buffer size).
//
// Build and run on the device:
//   hipcc -O3 --offload-arch=gfx950 -Xclang -target-feature -Xclang -packed-fp32-ops \
//         -o bench_valu_rates bench_valu_rates.hip && ./bench_valu_rates
#include <hip/hip_runtime.h>
#include <cstdio>
#include <cstdint>
#include <chrono>

constexpr int ITERS = 4096;
constexpr int CH = 8;  // independent chains per lane

__global__ void k_mad64(uint32_t *out, uint32_t seed) {
  uint32_t a[CH];
  for (int c = 0; c < CH; ++c) a[c] = seed + threadIdx.x * 7 + c;
  for (int i = 0; i < ITERS; ++i)
#pragma unroll
    for (int c = 0; c < CH; ++c) {
      const uint64_t p = (uint64_t)0xD2511F53u * (uint64_t)a[c];
      a[c] = (uint32_t)(p >> 32) ^ (uint32_t)p;
    }
  uint32_t r = 0;
  for (int c = 0; c < CH; ++c) r ^= a[c];
  out[blockIdx.x * blockDim.x + threadIdx.x] = r;
}

__global__ void k_fma(float *out, float seed) {
  float a[CH];
  for (int c = 0; c < CH; ++c) a[c] = seed + threadIdx.x * 1e-3f + c;
  for (int i = 0; i < ITERS; ++i)
#pragma unroll
    for (int c = 0; c < CH; ++c) a[c] = __builtin_fmaf(a[c], 0.999f, 1e-3f);
  float r = 0;
  for (int c = 0; c < CH; ++c) r += a[c];
  out[blockIdx.x * blockDim.x + threadIdx.x] = r;
}

__global__ void k_log(float *out, float seed) {
  float a[CH];
  for (int c = 0; c < CH; ++c) a[c] = seed + threadIdx.x * 1e-3f + c;
  for (int i = 0; i < ITERS; ++i)
#pragma unroll
    for (int c = 0; c < CH; ++c) a[c] = __builtin_amdgcn_logf(a[c]) + 2.0f;
  float r = 0;
  for (int c = 0; c < CH; ++c) r += a[c];
  out[blockIdx.x * blockDim.x + threadIdx.x] = r;
}

__global__ void k_fma64(double *out, double seed) {
  double a[CH];
  for (int c = 0; c < CH; ++c) a[c] = seed + threadIdx.x * 1e-3 + c;
  for (int i = 0; i < ITERS; ++i)
#pragma unroll
    for (int c = 0; c < CH; ++c) a[c] = __builtin_fma(a[c], 0.999, 1e-3);
  double r = 0;
  for (int c = 0; c < CH; ++c) r += a[c];
  out[blockIdx.x * blockDim.x + threadIdx.x] = r;
}

#define CHECK(expr)                                                                  \
  do {                                                                               \
    const hipError_t e_ = (expr);                                                    \
    if (e_ != hipSuccess) {                                                          \
      fprintf(stderr, "%s: %s\n", #expr, hipGetErrorString(e_));                     \
      return 1;                                                                      \
    }                                                                                \
  } while (0)

int main() {
  int dev = 0;
  hipDeviceProp_t prop;
  CHECK(hipGetDeviceProperties(&prop, dev));
  const int cus = prop.multiProcessorCount;
  const int threads = 256, blocks = cus * 16;  // 16 waves per SIMD worth of work
  const size_t n = (size_t)threads * blocks;
  void *buf;
  CHECK(hipMalloc(&buf, n * 8));
  hipEvent_t a, b;
  CHECK(hipEventCreate(&a));
  CHECK(hipEventCreate(&b));
  const double clk = prop.clockRate * 1e3;  // Hz
  auto run = [&](const char *name, auto launch, int instr_per_iter) -> int {
    launch();
    CHECK(hipGetLastError());
    CHECK(hipDeviceSynchronize());
    CHECK(hipEventRecord(a));
    launch();
    CHECK(hipEventRecord(b));
    CHECK(hipEventSynchronize(b));
    float ms = 0;
    CHECK(hipEventElapsedTime(&ms, a, b));
    const double wave_instr = (double)n / 64 * ITERS * CH * instr_per_iter;
    const double per_cu_cycle = wave_instr / (ms * 1e-3 * clk) / cus;
    printf("%-8s %.3f ms  %.3f wave-instr per CU-cycle (clock %.0f MHz)\n", name, ms, per_cu_cycle,
           clk / 1e6);
    return 0;
  };
  int rc = 0;
  rc |= run("mad64", [&] { hipLaunchKernelGGL(k_mad64, dim3(blocks), dim3(threads), 0, 0, (uint32_t *)buf, 1u); }, 1);
  rc |= run("fma32", [&] { hipLaunchKernelGGL(k_fma, dim3(blocks), dim3(threads), 0, 0, (float *)buf, 1.0f); }, 1);
  rc |= run("log32", [&] { hipLaunchKernelGGL(k_log, dim3(blocks), dim3(threads), 0, 0, (float *)buf, 1.0f); }, 1);
  rc |= run("fma64", [&] { hipLaunchKernelGGL(k_fma64, dim3(blocks), dim3(threads), 0, 0, (double *)buf, 1.0); }, 1);
  CHECK(hipFree(buf));
  return rc;
}
