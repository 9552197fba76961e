// Complex helpers and the radix-16 4096-point FFT shared by the OFDM kernels
// (ofdm.hip) and the Welch PSD (spectrum.hip).  Workgroups of kFftThreads = 256
// threads.
#pragma once

#include "kernels.hpp"

namespace dpdmi {

namespace {

constexpr int kFftThreads = 256;
constexpr int kFftMax = 4096;

// Half twiddle table tw[e] = exp(-2 pi i e / n), e < n/2; w^e = -tw[e - n/2] above.
__device__ inline void fft_twiddles(float2* tw, int n) {
  for (int e = threadIdx.x; e < n / 2; e += blockDim.x) {
    float s, c;
    sincospif(-2.0f * (float)e / (float)n, &s, &c);
    tw[e] = make_float2(c, s);
  }
}

template <bool INV>
__device__ __forceinline__ float2 twiddle(const float2* tw, int e, int n) {
  const int h = n >> 1;
  float2 v = e < h ? tw[e] : tw[e - h];
  if (e >= h) v = make_float2(-v.x, -v.y);
  if (INV) v.y = -v.y;
  return v;
}

__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }

// ---------------------------------------------------------------------------
// 4096-point path (the paper's OFDM symbol): three radix-16 Stockham passes, one
// butterfly per thread per pass (256 threads) with its sixteen values in registers;
// passes exchange through a padded LDS row (one float2 gap after every 16, so the
// stride-16 writes of the first pass spread over all 64 banks).  Global memory is read
// straight into the first pass and written straight from the last.  The inverse is the
// forward transform of the conjugate, conjugated.
// ---------------------------------------------------------------------------
constexpr int kF16Row = kFftMax + kFftMax / 16;
__device__ __forceinline__ int p16(int i) { return i + (i >> 4); }

__device__ __forceinline__ void dft4f(float2& a0, float2& a1, float2& a2, float2& a3) {
  const float2 t0 = cadd(a0, a2), t1 = csub(a0, a2), t2 = cadd(a1, a3), d = csub(a1, a3);
  const float2 t3 = make_float2(d.y, -d.x);     // (a1 - a3) (-i)
  a0 = cadd(t0, t2);
  a1 = cadd(t1, t3);
  a2 = csub(t0, t2);
  a3 = csub(t1, t3);
}

// Forward 16-point DFT in place as 4 x 4: X[k] ends in v[4 (k mod 4) + k / 4] (X16).
__device__ __forceinline__ void dft16f(float2 (&v)[16]) {
  constexpr float c1 = 0.92387953251128674f, s1 = 0.38268343236508978f, rh = 0.70710678118654752f;
  // exp(-2 pi i m / 16), m = 0..9 (the products q p of the middle twiddles)
  const float2 w[10] = {{1.f, 0.f}, {c1, -s1}, {rh, -rh}, {s1, -c1}, {0.f, -1.f},
                        {-s1, -c1}, {-rh, -rh}, {-c1, -s1}, {-1.f, 0.f}, {-c1, s1}};
#pragma unroll
  for (int q = 0; q < 4; ++q) dft4f(v[q], v[q + 4], v[q + 8], v[q + 12]);
#pragma unroll
  for (int q = 1; q < 4; ++q)
#pragma unroll
    for (int p = 1; p < 4; ++p) v[q + 4 * p] = cmul(v[q + 4 * p], w[q * p]);
#pragma unroll
  for (int p = 0; p < 4; ++p) dft4f(v[4 * p], v[4 * p + 1], v[4 * p + 2], v[4 * p + 3]);
}
#define X16(v, k) (v)[4 * ((k) & 3) + ((k) >> 2)]

// First pass (sub-transform length 1): v[r] = x[t + 256 r] on entry.
__device__ __forceinline__ void f16_pass1(float2* buf, float2 (&v)[16]) {
  const int t = threadIdx.x;
  dft16f(v);
#pragma unroll
  for (int r = 0; r < 16; ++r) buf[p16(t * 16 + r)] = X16(v, r);
}

// Second pass (length 16), in place; the caller's barrier precedes it and follows it.
__device__ __forceinline__ void f16_pass2(float2* buf, const float2* tw) {
  const int t = threadIdx.x, k = t & 15;
  float2 v[16];
#pragma unroll
  for (int r = 0; r < 16; ++r) v[r] = buf[p16(t + 256 * r)];
  __syncthreads();
#pragma unroll
  for (int r = 1; r < 16; ++r) v[r] = cmul(v[r], twiddle<false>(tw, 16 * r * k, kFftMax));
  dft16f(v);
#pragma unroll
  for (int r = 0; r < 16; ++r) buf[p16((t - k) * 16 + k + 16 * r)] = X16(v, r);
}

// Last pass (length 256): X16(v, r) is transform output t + 256 r on return.
__device__ __forceinline__ void f16_pass3(const float2* buf, const float2* tw, float2 (&v)[16]) {
  const int t = threadIdx.x;
#pragma unroll
  for (int r = 0; r < 16; ++r) v[r] = buf[p16(t + 256 * r)];
#pragma unroll
  for (int r = 1; r < 16; ++r) v[r] = cmul(v[r], twiddle<false>(tw, r * t, kFftMax));
  dft16f(v);
}

}  // namespace

}  // namespace dpdmi
