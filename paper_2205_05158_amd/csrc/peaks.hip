// Throughput probes of the units the hot path is bounded by, measured on the GPU the
// benchmark runs on so the roofline can be stated against measured as well as published
// peaks: bf16 MFMA (16x16x32), fp32 FMA (non-packed, as every kernel here is built),
// the transcendental pair a tanh costs (exp2 and reciprocal), and an HBM stream copy.
// Separate library (libdpdpeaks.so): benchmarking only, not part of the C ABI of the path.
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// Each wave runs 4 independent accumulation chains of 16x16x32 MFMAs.
__global__ __launch_bounds__(256) void k_mfma_bf16(float* sink, int iters) {
  bf16x8 a, b;
  for (int e = 0; e < 8; ++e) {
    a[e] = (__bf16)(1e-3f * (float)(threadIdx.x % 7 + e));
    b[e] = (__bf16)(1e-3f * (float)(threadIdx.x % 5 + e));
  }
  f32x4 c0 = {0, 0, 0, 0}, c1 = c0, c2 = c0, c3 = c0;
  for (int i = 0; i < iters; ++i) {
    c0 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c0, 0, 0, 0);
    c1 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c1, 0, 0, 0);
    c2 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c2, 0, 0, 0);
    c3 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c3, 0, 0, 0);
  }
  const f32x4 s = c0 + c1 + c2 + c3;
  sink[blockIdx.x * blockDim.x + threadIdx.x] = s[0] + s[1] + s[2] + s[3];
}

// 8 independent fp32 FMA chains per thread.
__global__ __launch_bounds__(256) void k_fma_f32(float* sink, int iters) {
  float v[8];
  const float m = 0.999f, d = 1e-7f * (float)threadIdx.x;
  for (int j = 0; j < 8; ++j) v[j] = (float)j + d;
  for (int i = 0; i < iters; ++i) {
#pragma unroll
    for (int j = 0; j < 8; ++j) v[j] = fmaf(v[j], m, d);
  }
  float s = 0.f;
  for (int j = 0; j < 8; ++j) s += v[j];
  sink[blockIdx.x * blockDim.x + threadIdx.x] = s;
}

// 4 independent chains of (exp2, reciprocal) pairs per thread, the transcendental part
// of one tanh evaluation.
__global__ __launch_bounds__(256) void k_trans(float* sink, int iters) {
  float v[4];
  for (int j = 0; j < 4; ++j) v[j] = 0.25f + 1e-3f * (float)(threadIdx.x % 13 + j);
  for (int i = 0; i < iters; ++i) {
#pragma unroll
    for (int j = 0; j < 4; ++j) v[j] = __builtin_amdgcn_rcpf(__builtin_amdgcn_exp2f(v[j]) + 1.0f);
  }
  sink[blockIdx.x * blockDim.x + threadIdx.x] = v[0] + v[1] + v[2] + v[3];
}

__global__ __launch_bounds__(256) void k_copy(const float4* __restrict__ src, float4* __restrict__ dst,
                                              int64_t n4) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n4;
       i += (int64_t)gridDim.x * blockDim.x)
    dst[i] = src[i];
}

}  // namespace

// sink: device float[blocks * 256]; returns 0 or the HIP error code.
extern "C" int peak_mfma_bf16(float* sink, int blocks, int iters, hipStream_t s) {
  k_mfma_bf16<<<blocks, 256, 0, s>>>(sink, iters);
  return (int)hipGetLastError();
}
extern "C" int peak_fma_f32(float* sink, int blocks, int iters, hipStream_t s) {
  k_fma_f32<<<blocks, 256, 0, s>>>(sink, iters);
  return (int)hipGetLastError();
}
extern "C" int peak_trans(float* sink, int blocks, int iters, hipStream_t s) {
  k_trans<<<blocks, 256, 0, s>>>(sink, iters);
  return (int)hipGetLastError();
}
// src, dst: device buffers of n_bytes (a multiple of 16).
extern "C" int peak_copy(const void* src, void* dst, int64_t n_bytes, int blocks, hipStream_t s) {
  k_copy<<<blocks, 256, 0, s>>>(static_cast<const float4*>(src), static_cast<float4*>(dst), n_bytes / 16);
  return (int)hipGetLastError();
}
