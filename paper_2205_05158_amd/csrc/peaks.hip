// Throughput probes of the units the hot path is bounded by, measured on the GPU the
// benchmark runs on so the roofline can be stated against measured as well as published
// peaks: bf16 MFMA (16x16x32 and 32x32x16, with the shader clock they ran at), fp32 FMA
// (non-packed, as every kernel here is built), the transcendental pair a tanh costs
// (exp2 and reciprocal), and an HBM stream copy.
// Separate library (libdpdpeaks.so): benchmarking only, not part of the C ABI of the path.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

typedef float f32x16 __attribute__((ext_vector_type(16)));

// Each wave runs 4 independent accumulation chains of bf16 MFMAs, 16x16x32 (the TDNN
// layers' shape) or 32x32x16 (the dW shape).  Thread 0 of every workgroup records the
// shader-clock counter (s_memtime) and the 100 MHz real-time counter (s_memrealtime)
// around its loop, so the clock the matrix cores actually ran at can be stated.
template <bool BIG>
__global__ __launch_bounds__(256) void k_mfma_bf16(float* sink, long long* clk, int iters) {
  bf16x8 a, b;
  for (int e = 0; e < 8; ++e) {
    a[e] = (__bf16)(1e-3f * (float)(threadIdx.x % 7 + e));
    b[e] = (__bf16)(1e-3f * (float)(threadIdx.x % 5 + e));
  }
  using Acc = std::conditional_t<BIG, f32x16, f32x4>;
  constexpr int NV = BIG ? 16 : 4;
  Acc c[4];
  for (int j = 0; j < 4; ++j)
    for (int e = 0; e < NV; ++e) c[j][e] = 0.f;
  const long long t0 = __builtin_amdgcn_s_memtime(), r0 = __builtin_amdgcn_s_memrealtime();
  for (int i = 0; i < iters; ++i) {
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      if constexpr (BIG) c[j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c[j], 0, 0, 0);
      else c[j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c[j], 0, 0, 0);
    }
  }
  const long long t1 = __builtin_amdgcn_s_memtime(), r1 = __builtin_amdgcn_s_memrealtime();
  float s = 0.f;
  for (int j = 0; j < 4; ++j)
    for (int e = 0; e < NV; ++e) s += c[j][e];
  sink[blockIdx.x * blockDim.x + threadIdx.x] = s;
  if (threadIdx.x == 0) {
    clk[2 * blockIdx.x] = t1 - t0;
    clk[2 * blockIdx.x + 1] = r1 - r0;
  }
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

// Stream copy: four 16-byte non-temporal loads in flight per thread, then their stores.
typedef float fv4 __attribute__((ext_vector_type(4)));
__global__ __launch_bounds__(256) void k_copy(const fv4* __restrict__ src, fv4* __restrict__ dst, int64_t n4) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (; i + 3 * stride < n4; i += 4 * stride) {
    fv4 v[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) v[u] = __builtin_nontemporal_load(&src[i + u * stride]);
#pragma unroll
    for (int u = 0; u < 4; ++u) __builtin_nontemporal_store(v[u], &dst[i + u * stride]);
  }
  for (; i < n4; i += stride) dst[i] = src[i];
}

}  // namespace

// sink: device float[blocks * 256]; clk: device int64[2 * blocks] (per workgroup: shader
// clocks and 100 MHz ticks of its loop); big = 0: 16x16x32, 1: 32x32x16.  Returns 0 or the
// HIP error code.
extern "C" int peak_mfma_bf16(float* sink, long long* clk, int blocks, int iters, int big, hipStream_t s) {
  if (big) k_mfma_bf16<true><<<blocks, 256, 0, s>>>(sink, clk, iters);
  else k_mfma_bf16<false><<<blocks, 256, 0, s>>>(sink, clk, iters);
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
  k_copy<<<blocks, 256, 0, s>>>(static_cast<const fv4*>(src), static_cast<fv4*>(dst), n_bytes / 16);
  return (int)hipGetLastError();
}
