// Welch power spectral density of a PA output and its adjacent-channel power ratio
// (the out-of-band metric named in Sec. I).  Segments of nfft samples, hop nfft/2,
// periodic Hann window; each workgroup transforms a contiguous group of segments and
// accumulates |X_k|^2 per bin: 4096-point segments with the radix-16 transform of
// fft.hpp (samples windowed as they are loaded, each thread's 16 bins in registers),
// other sizes with an in-LDS radix-2 decimation-in-time FFT.  A single-workgroup pass
// sums the group spectra in a fixed order (Neumaier) and integrates the channel powers.
#include "fft.hpp"

namespace dpdmi {

namespace {

constexpr int kMaxFft = kFftMax;

// 4096-point segments: thread t holds the samples t + 256 r (r = 0..15) of a segment,
// whose Hann weights are fixed, and after the three radix-16 passes the bins t + 256 r.
__global__ __launch_bounds__(kFftThreads) void k_welch4096(const float* __restrict__ y, int nseg,
                                                           float* __restrict__ part) {
  __shared__ float2 buf[kF16Row];
  __shared__ float2 tw[kFftMax / 2];
  fft_twiddles(tw, kFftMax);
  const int t = threadIdx.x;
  const int G = gridDim.x, g = blockIdx.x;
  const int s0 = (int)(((int64_t)g * nseg) / G), s1 = (int)(((int64_t)(g + 1) * nseg) / G);
  float win[16], acc[16];
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    win[r] = 0.5f - 0.5f * cospif(2.0f * (float)(t + 256 * r) / (float)kFftMax);
    acc[r] = 0.f;
  }
  const float2* y2 = reinterpret_cast<const float2*>(y);
  for (int sg = s0; sg < s1; ++sg) {
    const int64_t base = (int64_t)sg * (kFftMax / 2);
    float2 v[16];
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const float2 a = y2[base + t + 256 * r];
      v[r] = make_float2(a.x * win[r], a.y * win[r]);
    }
    __syncthreads();                       // the previous segment's last-pass reads are done
    f16_pass1(buf, v);
    __syncthreads();
    f16_pass2(buf, tw);
    __syncthreads();
    f16_pass3(buf, tw, v);
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const float2 X = X16(v, r);
      acc[r] += X.x * X.x + X.y * X.y;
    }
  }
#pragma unroll
  for (int r = 0; r < 16; ++r) part[(int64_t)g * kFftMax + t + 256 * r] = acc[r];
}

__global__ __launch_bounds__(kFftThreads) void k_welch(const float* __restrict__ y, int64_t n,
                                                       int nfft, int log2n, int nseg,
                                                       float* __restrict__ part) {
  __shared__ float2 buf[kMaxFft];
  __shared__ float2 tw[kMaxFft / 2];
  const int tid = threadIdx.x;
  const int G = gridDim.x, g = blockIdx.x;
  const int s0 = (int)(((int64_t)g * nseg) / G), s1 = (int)(((int64_t)(g + 1) * nseg) / G);
  const int half = nfft / 2;
  // twiddles W^k = exp(-2 pi i k / nfft)
  for (int k = tid; k < half; k += kFftThreads) {
    float sv, cv;
    sincospif(-2.0f * (float)k / (float)nfft, &sv, &cv);
    tw[k] = make_float2(cv, sv);
  }
  constexpr int kBinsPerThread = kMaxFft / kFftThreads;
  float acc[kBinsPerThread];
#pragma unroll
  for (int q = 0; q < kBinsPerThread; ++q) acc[q] = 0.f;
  for (int sg = s0; sg < s1; ++sg) {
    __syncthreads();
    const int64_t base = (int64_t)sg * half;
    for (int i = tid; i < nfft; i += kFftThreads) {
      float2 v = ld2(y, base + i);
      float w = 0.5f - 0.5f * cospif(2.0f * (float)i / (float)nfft);
      int r = __brev((unsigned)i) >> (32 - log2n);
      buf[r] = make_float2(v.x * w, v.y * w);
    }
    __syncthreads();
    for (int st = 1; st <= log2n; ++st) {
      const int m = 1 << st, mh = m >> 1;
      for (int b = tid; b < half; b += kFftThreads) {
        int grp = b / mh, k = b % mh;
        int i0 = grp * m + k, i1 = i0 + mh;
        float2 wv = tw[k * (nfft / m)];
        float2 a = buf[i0], c = buf[i1];
        float2 t = make_float2(wv.x * c.x - wv.y * c.y, wv.x * c.y + wv.y * c.x);
        buf[i0] = make_float2(a.x + t.x, a.y + t.y);
        buf[i1] = make_float2(a.x - t.x, a.y - t.y);
      }
      __syncthreads();
    }
#pragma unroll
    for (int q = 0; q < kBinsPerThread; ++q) {
      int k = tid + q * kFftThreads;
      if (k < nfft) {
        float2 X = buf[k];
        acc[q] += X.x * X.x + X.y * X.y;
      }
    }
  }
#pragma unroll
  for (int q = 0; q < kBinsPerThread; ++q) {
    int k = tid + q * kFftThreads;
    if (k < nfft) part[(int64_t)g * nfft + k] = acc[q];
  }
}

// psd[k] = sum over groups (fixed order, Neumaier) / (nseg * sum of Hann^2); one
// thread per bin.
// Group partials summed in two fixed-order stages: k_welch_sum adds the groups of split
// blockIdx.y (compensated) into sums[split][k] (value and compensation), k_welch_sum2
// adds the splits in order and scales.
__global__ __launch_bounds__(kFftThreads) void k_welch_sum(const float* __restrict__ part, int G,
                                                           int nfft, int splits,
                                                           float2* __restrict__ sums) {
  const int k = blockIdx.x * kFftThreads + threadIdx.x;
  if (k >= nfft) return;
  const int sp = blockIdx.y;
  const int g0 = (int)((int64_t)sp * G / splits), g1 = (int)((int64_t)(sp + 1) * G / splits);
  Comp s;
  int g = g0;
  for (; g + 8 <= g1; g += 8) {          // eight loads ahead of their (ordered) adds
    float v[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) v[q] = part[(int64_t)(g + q) * nfft + k];
#pragma unroll
    for (int q = 0; q < 8; ++q) s.add(v[q]);
  }
  for (; g < g1; ++g) s.add(part[(int64_t)g * nfft + k]);
  sums[(int64_t)sp * nfft + k] = make_float2(s.s, s.c);
}

__global__ __launch_bounds__(kFftThreads) void k_welch_sum2(const float2* __restrict__ sums, int splits,
                                                            int nseg, int nfft, float* __restrict__ psd) {
  const int k = blockIdx.x * kFftThreads + threadIdx.x;
  if (k >= nfft) return;
  const float scale = 1.0f / ((float)nseg * 0.375f * (float)nfft);   // sum of Hann^2 = 3 nfft / 8
  Comp s;
  for (int sp = 0; sp < splits; ++sp) {
    const float2 v = sums[(int64_t)sp * nfft + k];
    s.add(v.x);
    s.add(v.y);
  }
  psd[k] = s.value() * scale;
}

// Channel powers of the PSD and the ACPR (one workgroup, fixed order).
__global__ __launch_bounds__(kFftThreads) void k_welch_final(const float* __restrict__ psd,
                                                             int nfft, int half_bins,
                                                             float* __restrict__ acpr) {
  __shared__ float sh[6 * kFftThreads];
  const int tid = threadIdx.x;
  Comp lo, mn, up;
  for (int k = tid; k < nfft; k += kFftThreads) {
    float v = psd[k];
    int ks = k < nfft / 2 ? k : k - nfft;
    int a = ks < 0 ? -ks : ks;
    if (a <= half_bins) mn.add(v);
    else if (ks > half_bins && ks <= 3 * half_bins) up.add(v);
    else if (ks < -half_bins && ks >= -3 * half_bins) lo.add(v);
  }
  // the three band sums over the threads, a fixed tree
  Comp* band[3] = {&lo, &mn, &up};
  for (int b = 0; b < 3; ++b) {
    sh[2 * b * kFftThreads + tid] = band[b]->s;
    sh[(2 * b + 1) * kFftThreads + tid] = band[b]->c;
  }
  __syncthreads();
  for (int w = kFftThreads / 2; w > 0; w >>= 1) {
    if (tid < w) {
#pragma unroll
      for (int b = 0; b < 3; ++b) {
        Comp x{sh[2 * b * kFftThreads + tid], sh[(2 * b + 1) * kFftThreads + tid]};
        x.add(sh[2 * b * kFftThreads + tid + w]);
        x.add(sh[(2 * b + 1) * kFftThreads + tid + w]);
        sh[2 * b * kFftThreads + tid] = x.s;
        sh[(2 * b + 1) * kFftThreads + tid] = x.c;
      }
    }
    __syncthreads();
  }
  if (tid == 0) {
    const Comp L{sh[0], sh[kFftThreads]}, Mn{sh[2 * kFftThreads], sh[3 * kFftThreads]},
        U{sh[4 * kFftThreads], sh[5 * kFftThreads]};
    float pm = Mn.value();
    float aL = 10.f * log10f(L.value() / pm), aU = 10.f * log10f(U.value() / pm);
    acpr[0] = aL;
    acpr[1] = aU;
    acpr[2] = fmaxf(aL, aU);
  }
}

}  // namespace

void launch_welch(const float* y, int64_t n, int nfft, float* seg_part, int n_groups,
                  hipStream_t s) {
  int log2n = 0;
  while ((1 << log2n) < nfft) ++log2n;
  int nseg = (int)((n - nfft) / (nfft / 2) + 1);
  if (nfft == kFftMax) k_welch4096<<<n_groups, kFftThreads, 0, s>>>(y, nseg, seg_part);
  else k_welch<<<n_groups, kFftThreads, 0, s>>>(y, n, nfft, log2n, nseg, seg_part);
}

void launch_welch_final(const float* seg_part, int n_groups, int nseg, int nfft, int half_bins,
                        float2* sums, float* psd, float* acpr, hipStream_t s) {
  const int nb = (nfft + kFftThreads - 1) / kFftThreads;
  k_welch_sum<<<dim3(nb, kWelchSplits), kFftThreads, 0, s>>>(seg_part, n_groups, nfft, kWelchSplits, sums);
  k_welch_sum2<<<nb, kFftThreads, 0, s>>>(sums, kWelchSplits, nseg, nfft, psd);
  k_welch_final<<<1, kFftThreads, 0, s>>>(psd, nfft, half_bins, acpr);
}

}  // namespace dpdmi
