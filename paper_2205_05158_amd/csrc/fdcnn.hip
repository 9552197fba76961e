// FD-CNN DPD (the paper's proposed frequency-domain CNN, Sec. IV-C; configuration of
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
constexpr int kCnnMaxF = kCnnMaxConv * kCnnMaxSide * kCnnMaxSide;

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
  f32x16 acc;
#pragma unroll
  for (int j = 0; j < 16; ++j) acc[j] = 0.f;
  for (int k0 = kb; k0 < ke; k0 += kGK) {
    __syncthreads();
    for (int e = tid; e < kGK * kGT; e += 256) {
      const int kk = e / kGT, mm = e % kGT;
      const int k = k0 + kk;
      As[kk][mm] = (k < ke && m0 + mm < M) ? pr.a(m0 + mm, k) : 0.f;
      Bs[kk][mm] = (k < ke && n0 + mm < N) ? pr.b(k, n0 + mm) : 0.f;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < kGK; kk += 2) {
      const float a = As[kk + lane / 32][wm + lane % 32];
      const float bv = Bs[kk + lane / 32][wn + lane % 32];
      acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a, bv, acc, 0, 0, 0);
    }
  }
  // D: register j of lane l = row 8 (j / 4) + 4 (l / 32) + j % 4, column l % 32
#pragma unroll
  for (int j = 0; j < 16; ++j) {
    const int m = m0 + wm + mfma_row(j, lane / 32), n = n0 + wn + lane % 32;
    if (m < M && n < N) pr.store(split, m, n, acc[j]);
  }
}

// forward output layer: y[b][o] = sum_f h[b][f] Wf[o][f] + bf[o] -> out[b][o % n_d].(re|im)
struct FwdOut {
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

// Convolution weight and bias gradients: thread group k of the workgroup (entries t =
// 0..nt-1 per group, G = threads / nt groups) owns gradient entry t over the positions
// f = k, k + G, ... of every item of the workgroup, in one register; the groups are then
// added in LDS and the workgroup's partials written to cpart[wg][nt]; k_cnn_dwc_reduce
// adds the workgroups in order.
__global__ __launch_bounds__(kCnnThreads) void k_cnn_dwc(CnnGeom g, int64_t n_items,
                                                         const float* __restrict__ s,
                                                         const float* __restrict__ dpre,
                                                         float* __restrict__ cpart) {
  __shared__ float xp[2 * kCnnPad * kCnnPad];
  __shared__ float dl[kCnnMaxF];
  __shared__ float red[kCnnThreads];
  const int nw = g.n_conv * 2 * g.kc * g.kc, nt = nw + g.n_conv;
  const int hp = g.kc / 2, W = g.side + 2 * hp, S2 = g.side * g.side;
  const int G = kCnnThreads / nt;
  const int t = threadIdx.x % nt, grp = threadIdx.x / nt;
  const bool active = grp < G;
  // entry t: (o, c, p, q) of a weight, or the bias of kernel t - nw
  const bool is_bias = t >= nw;
  const int o = is_bias ? t - nw : t / (2 * g.kc * g.kc);
  const int c = is_bias ? 0 : (t / (g.kc * g.kc)) % 2;
  const int p = is_bias ? 0 : (t / g.kc) % g.kc, q = is_bias ? 0 : t % g.kc;
  float acc = 0.f;
  for (int64_t b = blockIdx.x; b < n_items; b += gridDim.x) {
    __syncthreads();
    for (int f = threadIdx.x; f < g.F; f += kCnnThreads) dl[f] = dpre[b * g.F + f];
    load_planes(g, s, b, xp);    // (synchronises)
    if (active) {
      for (int pos = grp; pos < S2; pos += G) {
        const int i = pos / g.side, j = pos % g.side;
        const float d = dl[o * S2 + pos];
        acc += is_bias ? d : d * xp[c * W * W + (i + p) * W + (j + q)];
      }
    }
  }
  __syncthreads();
  red[threadIdx.x] = active ? acc : 0.f;
  __syncthreads();
  if (threadIdx.x < nt) {
    float sum = 0.f;
    for (int k = 0; k < G; ++k) sum += red[k * nt + threadIdx.x];
    cpart[(int64_t)blockIdx.x * nt + threadIdx.x] = sum;
  }
}

__global__ void k_cnn_dwc_reduce(CnnGeom g, int n_wg, const float* __restrict__ cpart, float* __restrict__ dw) {
  const int nt = g.n_conv * 2 * g.kc * g.kc + g.n_conv;
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nt) return;
  float acc = 0.f;
  for (int i = 0; i < n_wg; ++i) acc += cpart[(int64_t)i * nt + t];
  dw[t] = acc;   // conv weights then conv biases (offsets 0 and off_bc are contiguous)
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
  k_cnn_dwc_reduce<<<1, 256, 0, st>>>(g, cg, cpart, dw);
}

}  // namespace dpdmi
