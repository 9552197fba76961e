// Device-side building blocks shared by the dpdmi kernels (gfx950 only).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "dpdmi.h"

namespace dpdmi {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kWave = 64;

__host__ __device__ constexpr int round_up(int a, int b) { return (a + b - 1) / b * b; }
__host__ __device__ constexpr int64_t ceil_div64(int64_t a, int64_t b) { return (a + b - 1) / b; }

// ---------------------------------------------------------------------------
// Stream table, passed to every kernel by value (no device metadata, nothing to
// copy or allocate).  Streams are cut into tiles of `tile` samples; stream s owns
// tiles [tile0[s], tile0[s+1]).  Its parameter set is s (per-stream) or 0.
// ---------------------------------------------------------------------------
struct StreamTable {
  int64_t off[DPD_MAX_STREAMS + 1];
  int32_t tile0[DPD_MAX_STREAMS + 1];
  // bf16 TDNN forward feeding the reverse mode: first stored-activation group (16 samples)
  // of each stream, 4 groups per 64-sample reverse-mode tile
  int32_t grp0[DPD_MAX_STREAMS + 1];
  int32_t n;            // number of streams
  int32_t per_stream;   // parameter set = stream index when 1, else 0
  int32_t tile;         // samples per tile
  int32_t n_tiles;      // tile0[n]
};

// Stream owning global tile t (binary search over the uniform table).
__device__ inline int stream_of_tile(const StreamTable& st, int t) {
  int lo = 0, hi = st.n - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (st.tile0[mid] <= t) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// Stream owning sample index i.
__device__ inline int stream_of_sample(const StreamTable& st, int64_t i) {
  int lo = 0, hi = st.n - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (st.off[mid] <= i) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// Contiguous split of n_tiles tiles over G workgroups: workgroup g owns
// [start(g), start(g+1)).  owner() is its inverse.  Every workgroup owns >= 1 tile
// when G <= n_tiles.
__host__ __device__ inline int wg_tile_start(int g, int G, int n_tiles) {
  return (int)(((int64_t)g * n_tiles) / G);
}
__host__ __device__ inline int wg_of_tile(int t, int G, int n_tiles) {
  return (int)((((int64_t)t + 1) * G - 1) / n_tiles);
}

// ---------------------------------------------------------------------------
// Arithmetic helpers
// ---------------------------------------------------------------------------
// tanh for float32: 1 - 2/(e^{2|x|} + 1) with the hardware base-2 exponential and
// reciprocal for |x| >= 1/4 (cancellation costs at most 2 bits there); below, the
// Maclaurin series of tanh through x^11 (coefficients 1, -1/3, 2/15, -17/315,
// 62/2835, -1382/155925; truncation error < 3e-10 relative for |x| < 1/4).  Sign
// restored; saturates to +-1 for |x| > 10 (tanh rounds to 1 in float32 beyond ~9.01).
// A NaN argument gives NaN (the clamp is a comparison, which keeps NaN, not fminf).
__device__ __forceinline__ float tanh_f32(float x) {
  float ax = fabsf(x);
  float e = __builtin_amdgcn_exp2f((ax > 10.0f ? 10.0f : ax) * 2.8853900817779268f);   // 2 log2(e)
  float big = 1.0f - 2.0f * __builtin_amdgcn_rcpf(e + 1.0f);
  float x2 = ax * ax;
  float p = -8.8632355299e-3f;                  // -1382/155925
  p = p * x2 + 2.1869488536e-2f;                // 62/2835
  p = p * x2 - 5.3968253968e-2f;                // -17/315
  p = p * x2 + 1.3333333333e-1f;                // 2/15
  p = p * x2 - 3.3333333333e-1f;                // -1/3
  float small = ax + ax * x2 * p;
  float t = ax < 0.25f ? small : big;
  return copysignf(t, x);
}

// tanh(y / (2 log2 e)) for a pre-activation already scaled by 2 log2 e (bf16 layers fold
// that factor into the bias and apply it with the bias add): 1 - 2/(2^y + 1).
constexpr float kTanhScale = 2.8853900817779268f;   // 2 log2(e)
__device__ __forceinline__ float tanh_bf16_scaled(float y) {
  return fmaf(-2.0f, __builtin_amdgcn_rcpf(__builtin_amdgcn_exp2f(y) + 1.0f), 1.0f);
}

// Compiler-level memory fence: keeps loads from being hoisted across it (e.g. the
// coefficient reads of a per-position loop, or the weight-operand loads of the next
// 32-row block), which bounds register pressure.  Emits no instruction.
#define DPD_KEEP_LOADS_LOCAL() asm volatile("" ::: "memory")

// Neumaier compensated accumulation in float32.
struct Comp {
  float s = 0.f, c = 0.f;
  __device__ __forceinline__ void add(float v) {
    float t = s + v;
    if (fabsf(s) >= fabsf(v)) c += (s - t) + v; else c += (v - t) + s;
    s = t;
  }
  __device__ __forceinline__ float value() const { return s + c; }
};

// ---------------------------------------------------------------------------
// MFMA 32x32 operand layout (wave64).  For C/D (32x32 fp32, 16 registers per lane):
// register j of lane l holds row rho(j, l/32) and column l%32 with
// rho(j, h) = 8*(j/4) + 4*h + j%4.  A (32 x K) and B (K x 32) operands: lane l
// holds row/column l%32 and the K-slice selected by h = l/32.
// ---------------------------------------------------------------------------
__host__ __device__ constexpr int mfma_row(int j, int h) { return 8 * (j >> 2) + 4 * h + (j & 3); }

__device__ __forceinline__ f32x16 mfma_bf16(bf16x8 a, bf16x8 b, f32x16 c) {
  return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f32x16 mfma_f32(float a, float b, f32x16 c) {
  return __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ float2 ld2(const float* p, int64_t i) {
  return reinterpret_cast<const float2*>(p)[i];
}
__device__ __forceinline__ void st2(float* p, int64_t i, float2 v) {
  reinterpret_cast<float2*>(p)[i] = v;
}

}  // namespace dpdmi
