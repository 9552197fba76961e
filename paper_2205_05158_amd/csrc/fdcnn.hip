// FD-CNN DPD (the paper's proposed frequency-domain CNN, Sec. IV-A; configuration of
// Sec. V-A) applied to a batch of UE symbol vectors: forward and reverse mode.
//
// Per item: the N_d data-subcarrier symbols fill a side x side grid row-major (zero
// padded); its Re and Im planes are convolved by n_conv kernels of size kc with zero
// padding keeping the plane size, biased, ReLU; the plane-major flattened vector h
// (F = n_conv side^2 values) feeds a linear output layer of 2 N_d neurons (Re parts,
// then Im parts).
//
// The output layer of the batch is a dense contraction (items x F) x (F x 2 N_d); it and
// its two reverse-mode products (dh = g W, dW = g^T h over the items) run on the fp32
// matrix cores (32x32x2) through one tiled kernel with problem-specific operand
// loaders and epilogues.  The convolution (2 x n_conv x kc^2 weights) is vector ALU work
// over LDS-staged planes.
#include "kernels.hpp"

namespace dpdmi {

namespace {

constexpr int kCnnThreads = 256;
constexpr int kCnnMaxSide = 32;
constexpr int kCnnMaxKc = 7;
constexpr int kCnnMaxConv = 4;
constexpr int kCnnPad = kCnnMaxSide + kCnnMaxKc - 1;

struct CnnGeom {
  int n_d, side, n_conv, kc, F, NO;   // F = n_conv side^2, NO = 2 n_d
  int64_t off_bc, off_wf, off_bf;     // packed parameter offsets (floats)
};

// Zero-padded Re and Im planes of item b into LDS: xp[2][W][W], W = side + kc - 1
// (synchronises the workgroup before and after filling).
__device__ void load_planes(const CnnGeom& g, const float* __restrict__ s, int64_t b, float* xp) {
  const int hp = g.kc / 2, W = g.side + 2 * hp;
  for (int i = threadIdx.x; i < 2 * W * W; i += kCnnThreads) xp[i] = 0.f;
  __syncthreads();
  for (int n = threadIdx.x; n < g.n_d; n += kCnnThreads) {
    const float2 v = ld2(s, b * g.n_d + n);
    const int r = n / g.side + hp, c = n % g.side + hp;
    xp[r * W + c] = v.x;
    xp[W * W + r * W + c] = v.y;
  }
  __syncthreads();
}

// Convolution + bias + ReLU, one item per workgroup iteration: h[b][F], plane-major.
__global__ __launch_bounds__(kCnnThreads) void k_cnn_conv(CnnGeom g, int64_t n_items,
                                                          const float* __restrict__ s,
                                                          const float* __restrict__ w,
                                                          float* __restrict__ h) {
  __shared__ float xp[2 * kCnnPad * kCnnPad];
  __shared__ float wc[kCnnMaxConv * 2 * kCnnMaxKc * kCnnMaxKc + kCnnMaxConv];
  const int nw = g.n_conv * 2 * g.kc * g.kc;
  for (int i = threadIdx.x; i < nw + g.n_conv; i += kCnnThreads) wc[i] = w[i];   // weights then biases
  const int hp = g.kc / 2, W = g.side + 2 * hp, S2 = g.side * g.side;
  for (int64_t b = blockIdx.x; b < n_items; b += gridDim.x) {
    __syncthreads();   // previous item done with xp (and wc visible)
    load_planes(g, s, b, xp);
    for (int f = threadIdx.x; f < g.F; f += kCnnThreads) {
      const int o = f / S2, i = (f % S2) / g.side, j = f % g.side;
      float acc = wc[nw + o];
      for (int c = 0; c < 2; ++c)
        for (int p = 0; p < g.kc; ++p)
          for (int q = 0; q < g.kc; ++q)
            acc = fmaf(wc[((o * 2 + c) * g.kc + p) * g.kc + q], xp[c * W * W + (i + p) * W + (j + q)], acc);
      h[b * g.F + f] = fmaxf(acc, 0.f);
    }
  }
}

// ---------------------------------------------------------------- fp32 MFMA GEMM
// C[m][n] = sum_k A(m, k) B(k, n) over a 64 x 64 tile per workgroup (4 waves, 32 x 32
// each, 32x32x2 f32 MFMAs), K in steps of 32 staged through LDS; the problem object
// supplies the operand reads (any layout, zero outside) and the epilogue.
constexpr int kGT = 64, kGK = 32;

template <class P>
__global__ __launch_bounds__(256) void k_cnn_gemm(P pr, int M, int N, int K, int k_splits) {
  __shared__ float As[kGK][kGT + 4];
  __shared__ float Bs[kGK][kGT + 4];
  const int tid = threadIdx.x, lane = tid % 64, wave = tid / 64;
  const int m0 = blockIdx.x * kGT, n0 = blockIdx.y * kGT;
  const int split = blockIdx.z;
  const int kb = (int)((int64_t)split * K / k_splits), ke = (int)((int64_t)(split + 1) * K / k_splits);
  const int wm = 32 * (wave % 2), wn = 32 * (wave / 2);
  constexpr int kPer = kGK * kGT / 256;   // operand elements per thread and K step
  // the next K step's operands are read into registers while this step's MFMAs run
  // element e of a tile: K index fastest when the operand is contiguous along K
  // (P::A_KFAST / P::B_KFAST), else the M / N index, so consecutive lanes read
  // consecutive addresses
  auto kk_of = [](int e, bool kfast) { return kfast ? e % kGK : e / kGT; };
  auto mm_of = [](int e, bool kfast) { return kfast ? e / kGK : e % kGT; };
  float ra[kPer], rb[kPer];
  auto fetch = [&](int k0) {
#pragma unroll
    for (int r = 0; r < kPer; ++r) {
      const int e = tid + 256 * r;
      const int ka = k0 + kk_of(e, P::A_KFAST), ma = mm_of(e, P::A_KFAST);
      const int kb2 = k0 + kk_of(e, P::B_KFAST), nb = mm_of(e, P::B_KFAST);
      ra[r] = (ka < ke && m0 + ma < M) ? pr.a(m0 + ma, ka) : 0.f;
      rb[r] = (kb2 < ke && n0 + nb < N) ? pr.b(kb2, n0 + nb) : 0.f;
    }
  };
  // two accumulation chains (even / odd K pairs) so consecutive MFMAs are independent
  f32x16 acc0, acc1;
#pragma unroll
  for (int j = 0; j < 16; ++j) acc0[j] = acc1[j] = 0.f;
  if (kb < ke) fetch(kb);
  for (int k0 = kb; k0 < ke; k0 += kGK) {
    __syncthreads();
#pragma unroll
    for (int r = 0; r < kPer; ++r) {
      const int e = tid + 256 * r;
      As[kk_of(e, P::A_KFAST)][mm_of(e, P::A_KFAST)] = ra[r];
      Bs[kk_of(e, P::B_KFAST)][mm_of(e, P::B_KFAST)] = rb[r];
    }
    __syncthreads();
    if (k0 + kGK < ke) fetch(k0 + kGK);
#pragma unroll
    for (int kk = 0; kk < kGK; kk += 4) {
      acc0 = __builtin_amdgcn_mfma_f32_32x32x2f32(As[kk + lane / 32][wm + lane % 32],
                                                   Bs[kk + lane / 32][wn + lane % 32], acc0, 0, 0, 0);
      acc1 = __builtin_amdgcn_mfma_f32_32x32x2f32(As[kk + 2 + lane / 32][wm + lane % 32],
                                                   Bs[kk + 2 + lane / 32][wn + lane % 32], acc1, 0, 0, 0);
    }
  }
  // D: register j of lane l = row 8 (j / 4) + 4 (l / 32) + j % 4, column l % 32
#pragma unroll
  for (int j = 0; j < 16; ++j) {
    const int m = m0 + wm + mfma_row(j, lane / 32), n = n0 + wn + lane % 32;
    if (m < M && n < N) pr.store(split, m, n, acc0[j] + acc1[j]);
  }
}

// forward output layer: y[b][o] = sum_f h[b][f] Wf[o][f] + bf[o] -> out[b][o % n_d].(re|im)
struct FwdOut {
  static constexpr bool A_KFAST = true, B_KFAST = true;
  const float* h; const float* wf; const float* bf; float* out; int F, n_d;
  __device__ float a(int m, int k) const { return h[(int64_t)m * F + k]; }
  __device__ float b(int k, int n) const { return wf[(int64_t)n * F + k]; }
  __device__ void store(int, int m, int n, float v) const {
    const int c = n / n_d, i = n % n_d;
    out[((int64_t)m * n_d + i) * 2 + c] = v + bf[n];
  }
};
// dpre[b][f] = (sum_o gy[b][o] Wf[o][f]) * (h[b][f] > 0); gy[b][o] = g_out[b][o % n_d].(re|im)
struct BwdH {
  static constexpr bool A_KFAST = true, B_KFAST = false;
  const float* g; const float* wf; const float* h; float* dpre; int F, n_d;
  __device__ float a(int m, int k) const { return g[((int64_t)m * n_d + k % n_d) * 2 + k / n_d]; }
  __device__ float b(int k, int n) const { return wf[(int64_t)k * F + n]; }
  __device__ void store(int, int m, int n, float v) const {
    dpre[(int64_t)m * F + n] = h[(int64_t)m * F + n] > 0.f ? v : 0.f;
  }
};
// [dWf | dbf] partial of split s: part[s][o][f] = sum_{b in split} gy[b][o] h1[b][f] with
// h1 = [h | 1] (column F of ones gives the bias gradient)
struct BwdW {
  static constexpr bool A_KFAST = false, B_KFAST = false;
  const float* g; const float* h; float* part; int F, n_d, NO;
  __device__ float a(int m, int k) const { return g[((int64_t)k * n_d + m % n_d) * 2 + m / n_d]; }
  __device__ float b(int k, int n) const { return n < F ? h[(int64_t)k * F + n] : 1.f; }
  __device__ void store(int s, int m, int n, float v) const {
    part[((int64_t)s * NO + m) * (F + 1) + n] = v;
  }
};

// [dWf | dbf] = sum of the split partials (fixed order)
__global__ void k_cnn_dwf_reduce(CnnGeom g, int k_splits, const float* __restrict__ part,
                                 float* __restrict__ dw) {
  const int64_t nW = (int64_t)g.NO * (g.F + 1);
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nW) return;
  float acc = 0.f;
  for (int s = 0; s < k_splits; ++s) acc += part[s * nW + i];
  const int o = (int)(i / (g.F + 1)), f = (int)(i % (g.F + 1));
  if (f < g.F) dw[g.off_wf + (int64_t)o * g.F + f] = acc;
  else dw[g.off_bf + o] = acc;
}

// Convolution weight and bias gradients.  Per iteration a workgroup stages IPW items
// (their output-gradient planes dpre and zero-padded input planes) in LDS; thread
// (slot, t), slot < IPW, t < nt, accumulates gradient entry t over all positions of the
// item in its slot, in one register, across the workgroup's items.  The slots are then
// added in LDS and the workgroup's partials written to cpart[wg][nt]; k_cnn_dwc_reduce
// adds the workgroups in order.
constexpr int kCnnDwcLds = 12288;   // floats of item staging (48 KB)

__global__ __launch_bounds__(kCnnThreads) void k_cnn_dwc(CnnGeom g, int64_t n_items,
                                                         const float* __restrict__ s,
                                                         const float* __restrict__ dpre,
                                                         float* __restrict__ cpart) {
  __shared__ float buf[kCnnDwcLds];
  __shared__ float red[kCnnThreads];
  const int nw = g.n_conv * 2 * g.kc * g.kc, nt = nw + g.n_conv;
  const int hp = g.kc / 2, W = g.side + 2 * hp, S2 = g.side * g.side;
  const int per_item = g.F + 2 * W * W;                     // dpre plane, then x planes
  const int ipw = min(kCnnThreads / nt, kCnnDwcLds / per_item);
  const int t = threadIdx.x % nt, slot = threadIdx.x / nt;
  const bool active = slot < ipw;
  // entry t: (o, c, p, q) of a weight, or the bias of kernel t - nw
  const bool is_bias = t >= nw;
  const int o = is_bias ? t - nw : t / (2 * g.kc * g.kc);
  const int c = is_bias ? 0 : (t / (g.kc * g.kc)) % 2;
  const int p = is_bias ? 0 : (t / g.kc) % g.kc, q = is_bias ? 0 : t % g.kc;
  float acc = 0.f;
  const int64_t stride = (int64_t)gridDim.x * ipw;
  for (int64_t b0 = (int64_t)blockIdx.x * ipw; b0 < n_items; b0 += stride) {
    __syncthreads();
    for (int e = threadIdx.x; e < ipw * per_item; e += kCnnThreads) buf[e] = 0.f;
    __syncthreads();
    for (int e = threadIdx.x; e < ipw * g.F; e += kCnnThreads) {
      const int k = e / g.F;
      if (b0 + k < n_items) buf[k * per_item + e % g.F] = dpre[(b0 + k) * g.F + e % g.F];
    }
    for (int e = threadIdx.x; e < ipw * g.n_d; e += kCnnThreads) {
      const int k = e / g.n_d, n = e % g.n_d;
      if (b0 + k < n_items) {
        const float2 v = ld2(s, (b0 + k) * g.n_d + n);
        float* xp = buf + k * per_item + g.F;
        const int r = n / g.side + hp, cc = n % g.side + hp;
        xp[r * W + cc] = v.x;
        xp[W * W + r * W + cc] = v.y;
      }
    }
    __syncthreads();
    if (active && b0 + slot < n_items) {
      const float* dl = buf + slot * per_item + o * S2;
      const float* xp = buf + slot * per_item + g.F + c * W * W;
      for (int i = 0; i < g.side; ++i)
        for (int j = 0; j < g.side; ++j) {
          const float d = dl[i * g.side + j];
          acc += is_bias ? d : d * xp[(i + p) * W + (j + q)];
        }
    }
  }
  __syncthreads();
  red[threadIdx.x] = active ? acc : 0.f;
  __syncthreads();
  if (threadIdx.x < nt) {
    float sum = 0.f;
    for (int k = 0; k < ipw; ++k) sum += red[k * nt + threadIdx.x];
    cpart[(int64_t)blockIdx.x * nt + threadIdx.x] = sum;
  }
}

// One workgroup per gradient entry t: thread i sums partials i, i + 256, ... in order,
// then a fixed tree over the threads (deterministic).
__global__ __launch_bounds__(256) void k_cnn_dwc_reduce(CnnGeom g, int n_wg, const float* __restrict__ cpart,
                                                        float* __restrict__ dw) {
  __shared__ float red[256];
  const int nt = g.n_conv * 2 * g.kc * g.kc + g.n_conv;
  const int t = blockIdx.x;
  float acc = 0.f;
  for (int i = threadIdx.x; i < n_wg; i += 256) acc += cpart[(int64_t)i * nt + t];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int w2 = 128; w2 > 0; w2 >>= 1) {
    if (threadIdx.x < w2) red[threadIdx.x] += red[threadIdx.x + w2];
    __syncthreads();
  }
  if (threadIdx.x == 0) dw[t] = red[0];   // conv weights then conv biases (contiguous from 0)
}

CnnGeom geom(const CnnDims& d) {
  CnnGeom g;
  g.n_d = d.n_d; g.side = d.side; g.n_conv = d.n_conv; g.kc = d.kc;
  g.F = d.F; g.NO = 2 * d.n_d;
  g.off_bc = (int64_t)d.n_conv * 2 * d.kc * d.kc;
  g.off_wf = g.off_bc + d.n_conv;
  g.off_bf = g.off_wf + (int64_t)g.NO * g.F;
  return g;
}

}  // namespace

CnnDims cnn_dims(int n_d, int side, int n_conv, int kc) {
  CnnDims d;
  d.n_d = n_d; d.side = side; d.n_conv = n_conv; d.kc = kc;
  d.F = n_conv * side * side;
  d.params = (int64_t)n_conv * 2 * kc * kc + n_conv + (int64_t)2 * n_d * d.F + 2 * n_d;
  return d;
}

bool cnn_supported(const CnnDims& d) {
  return d.n_d >= 1 && d.side >= 1 && d.side <= kCnnMaxSide && d.n_d <= d.side * d.side &&
         d.n_conv >= 1 && d.n_conv <= kCnnMaxConv && d.kc >= 1 && d.kc <= kCnnMaxKc && d.kc % 2 == 1 &&
         d.n_conv * 2 * d.kc * d.kc + d.n_conv <= kCnnThreads;
}

void launch_cnn_conv(const CnnDims& d, int64_t n_items, const float* s, const float* w, float* h,
                     int cus, hipStream_t st) {
  const int grid = (int)std::min<int64_t>(n_items, 8 * (int64_t)cus);
  k_cnn_conv<<<grid, kCnnThreads, 0, st>>>(geom(d), n_items, s, w, h);
}

void launch_cnn_out(const CnnDims& d, int64_t n_items, const float* h, const float* w, float* out,
                    hipStream_t st) {
  const CnnGeom g = geom(d);
  FwdOut pr{h, w + g.off_wf, w + g.off_bf, out, g.F, g.n_d};
  dim3 gg((unsigned)((n_items + kGT - 1) / kGT), (unsigned)((g.NO + kGT - 1) / kGT), 1);
  k_cnn_gemm<FwdOut><<<gg, 256, 0, st>>>(pr, (int)n_items, g.NO, g.F, 1);
}

void launch_cnn_dh(const CnnDims& d, int64_t n_items, const float* gout, const float* w, const float* h,
                   float* dpre, hipStream_t st) {
  const CnnGeom g = geom(d);
  BwdH ph{gout, w + g.off_wf, h, dpre, g.F, g.n_d};
  dim3 gh((unsigned)((n_items + kGT - 1) / kGT), (unsigned)((g.F + kGT - 1) / kGT), 1);
  k_cnn_gemm<BwdH><<<gh, 256, 0, st>>>(ph, (int)n_items, g.F, g.NO, 1);
}

void launch_cnn_dwout(const CnnDims& d, int64_t n_items, const float* gout, const float* h, float* wpart,
                      hipStream_t st) {
  const CnnGeom g = geom(d);
  BwdW pw{gout, h, wpart, g.F, g.n_d, g.NO};
  dim3 gw((unsigned)((g.NO + kGT - 1) / kGT), (unsigned)((g.F + 1 + kGT - 1) / kGT), kCnnSplits);
  k_cnn_gemm<BwdW><<<gw, 256, 0, st>>>(pw, g.NO, g.F + 1, (int)n_items, kCnnSplits);
}

void launch_cnn_dwout_reduce(const CnnDims& d, const float* wpart, float* dw, hipStream_t st) {
  const CnnGeom g = geom(d);
  const int64_t nr = (int64_t)g.NO * (g.F + 1);
  k_cnn_dwf_reduce<<<(unsigned)((nr + 255) / 256), 256, 0, st>>>(g, kCnnSplits, wpart, dw);
}

void launch_cnn_dwconv(const CnnDims& d, int64_t n_items, const float* s, const float* dpre, float* cpart,
                       float* dw, hipStream_t st) {
  const CnnGeom g = geom(d);
  const int cg = (int)std::min<int64_t>(n_items, kCnnConvWg);
  k_cnn_dwc<<<cg, kCnnThreads, 0, st>>>(g, n_items, s, dpre, cpart);
  k_cnn_dwc_reduce<<<g.n_conv * 2 * g.kc * g.kc + g.n_conv, 256, 0, st>>>(g, cg, cpart, dw);
}

}  // namespace dpdmi
