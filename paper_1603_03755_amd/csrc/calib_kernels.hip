// VALU issue-rate calibration for the roofline of the sweep kernels: a grid
// of eight waves per SIMD on every CU, each lane running eight independent
// chains of one instruction type, so the rate measured is the issue rate of
// that instruction, not its latency.  The instructions are the three kinds
// the Metropolis and Wolff loops are built from: a three-input XOR
// (v_bitop3_b32), a widening 32x32 -> 64-bit multiply-add (v_mad_u64_u32,
// Philox's multiply) and a packed 16-bit multiply-add (v_pk_mad_u16).
//
// Built on its own as libsqa_calib.so, a measurement tool of the benchmark and
// not part of the library's interface: one C entry point, loaded by ctypes.
#include <hip/hip_runtime.h>

#include "device_common.h"

namespace sqa {

constexpr int kCalibChains = 8;

__global__ __launch_bounds__(256) void calib_xor3_kernel(uint32_t *out, int iters, uint32_t seed) {
  uint32_t x[kCalibChains];
#pragma unroll
  for (int i = 0; i < kCalibChains; ++i) x[i] = seed + threadIdx.x * kCalibChains + i;
  const uint32_t b = seed ^ 0x5555u;
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int i = 0; i < kCalibChains; ++i) x[i] = __builtin_amdgcn_bitop3_b32(x[i], seed + 3u * i, b, 0x96);
  }
  uint32_t r = 0;
#pragma unroll
  for (int i = 0; i < kCalibChains; ++i) r ^= x[i];
  out[blockIdx.x * blockDim.x + threadIdx.x] = r;
}

__global__ __launch_bounds__(256) void calib_mad64_kernel(uint32_t *out, int iters, uint32_t seed) {
  uint32_t x[kCalibChains];
#pragma unroll
  for (int i = 0; i < kCalibChains; ++i) x[i] = seed + threadIdx.x * kCalibChains + i;
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int i = 0; i < kCalibChains; ++i) x[i] = x[i] * 0xD2511F53u + 1u;   // one v_mad_u64_u32 each
  }
  uint32_t r = 0;
#pragma unroll
  for (int i = 0; i < kCalibChains; ++i) r ^= x[i];
  out[blockIdx.x * blockDim.x + threadIdx.x] = r;
}

__global__ __launch_bounds__(256) void calib_pkmad_kernel(uint32_t *out, int iters, uint32_t seed) {
  u16x2 x[kCalibChains];
  const u16x2 w = {3, 5};
#pragma unroll
  for (int i = 0; i < kCalibChains; ++i) x[i] = as_u16x2(seed + threadIdx.x * kCalibChains + i);
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int i = 0; i < kCalibChains; ++i) x[i] = x[i] * w + x[(i + 1) % kCalibChains];
  }
  uint32_t r = 0;
#pragma unroll
  for (int i = 0; i < kCalibChains; ++i) r ^= as_u32(x[i]);
  out[blockIdx.x * blockDim.x + threadIdx.x] = r;
}

}  // namespace sqa

// op: 0 = three-input XOR, 1 = widening multiply-add, 2 = packed 16-bit
// multiply-add.  Launches eight waves per SIMD on every CU, each lane running
// `iters` iterations of eight independent chains; synchronous.  Returns 0 and
// the timed launch's duration (*ms_out) and its VALU wave-instructions of the
// chains (*wave_instructions_out); 1 for bad arguments (before any device
// call), 2 when a HIP call failed.
extern "C" __attribute__((visibility("default"))) int sqa_calib_valu_issue(int32_t op, int32_t iters, float *ms_out,
                                                                         double *wave_instructions_out) {
  using namespace sqa;
  if (op < 0 || op > 2 || iters <= 0 || !ms_out || !wave_instructions_out) return 1;
  int dev = 0, cus = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  if (e != hipSuccess) return 2;
  const int blocks = cus * 8;                  // 8 workgroups of 4 waves: 8 waves per SIMD
  uint32_t *out = nullptr;
  e = hipMalloc(&out, static_cast<size_t>(blocks) * 256 * sizeof(uint32_t));
  if (e != hipSuccess) return 2;
  hipEvent_t t0 = nullptr, t1 = nullptr;
  e = hipEventCreate(&t0);
  if (e == hipSuccess) e = hipEventCreate(&t1);
  auto launch = [&]() {
    if (op == 0) hipLaunchKernelGGL(calib_xor3_kernel, dim3(blocks), dim3(256), 0, nullptr, out, iters, 12345u);
    else if (op == 1) hipLaunchKernelGGL(calib_mad64_kernel, dim3(blocks), dim3(256), 0, nullptr, out, iters, 12345u);
    else hipLaunchKernelGGL(calib_pkmad_kernel, dim3(blocks), dim3(256), 0, nullptr, out, iters, 12345u);
    return hipGetLastError();
  };
  if (e == hipSuccess) e = launch();                    // warm-up
  if (e == hipSuccess) e = hipDeviceSynchronize();
  if (e == hipSuccess) e = hipEventRecord(t0, nullptr);
  if (e == hipSuccess) e = launch();
  if (e == hipSuccess) e = hipEventRecord(t1, nullptr);
  if (e == hipSuccess) e = hipEventSynchronize(t1);
  float ms = 0.0f;
  if (e == hipSuccess) e = hipEventElapsedTime(&ms, t0, t1);
  if (t0) (void)hipEventDestroy(t0);
  if (t1) (void)hipEventDestroy(t1);
  (void)hipFree(out);
  if (e != hipSuccess) return 2;
  *ms_out = ms;
  *wave_instructions_out = static_cast<double>(blocks) * 4.0 * iters * kCalibChains;
  return 0;
}
