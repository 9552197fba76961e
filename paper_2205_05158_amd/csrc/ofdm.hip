// Multi-user OFDM downlink around the frequency-domain DPDs (Sec. II-A, Sec. III-C):
// batched unitary FFTs, the FD-NN wrapper (per-UE IDFT, a delay-line ReLU network over
// all UEs, per-UE DFT) forward and backward, ZF precoding, and the link of per-antenna
// PAs (optionally behind per-antenna TD-GMP DPDs), the multi-tap channel, AWGN and QAM
// decisions.
//
// Every delay inside an OFDM symbol is cyclic (a cyclic prefix longer than every memory
// is implied by the frequency-domain channel form), so a whole symbol row is one
// workgroup's problem: the FFT, the DPD and the PA of one antenna's symbol run in LDS
// between one HBM read and one HBM write.
#include "fft.hpp"

namespace dpdmi {

namespace {

constexpr int kFftPer = kFftMax / 4 / kFftThreads;   // radix-4 butterflies per thread

// ---------------------------------------------------------------------------
// LDS FFT: Stockham autosort, radix-4 passes and one radix-2 pass when log2 n is odd.
// Pass with sub-transform length ns: butterfly j (< n/R) reads buf[j + r n/R],
// multiplies element r by w^(r (j mod ns) n / (ns R)), w = exp(-2 pi i / n), takes the
// R-point DFT and writes buf[(j - j mod ns) R + j mod ns + r ns].  In place: all reads
// of a pass complete (barrier) before its writes.  Twiddles: half table
// tw[e] = exp(-2 pi i e / n), e < n/2, and w^e = -tw[e - n/2] above.  Unscaled.
// ---------------------------------------------------------------------------
// Whole workgroup (kFftThreads threads) transforms buf[0, n) in place; n = 2^log2n <= 4096.
// Starts and ends with a barrier-complete buffer.
template <bool INV>
__device__ void fft_lds(float2* buf, const float2* tw, int n, int log2n) {
  const int tid = threadIdx.x;
  int ns = 1, rem = log2n;
  while (rem >= 2) {
    const int q = n >> 2;
    const int step = n / (ns * 4);
    float2 y[kFftPer][4];
#pragma unroll
    for (int m = 0; m < kFftPer; ++m) {
      const int j = tid + m * kFftThreads;
      if (j < q) {
        const int k = j & (ns - 1);
        float2 a0 = buf[j], a1 = buf[j + q], a2 = buf[j + 2 * q], a3 = buf[j + 3 * q];
        if (ns > 1) {
          a1 = cmul(a1, twiddle<INV>(tw, k * step, n));
          a2 = cmul(a2, twiddle<INV>(tw, 2 * k * step, n));
          a3 = cmul(a3, twiddle<INV>(tw, 3 * k * step, n));
        }
        const float2 t0 = cadd(a0, a2), t1 = csub(a0, a2), t2 = cadd(a1, a3), d = csub(a1, a3);
        // forward: (a1 - a3) (-i); inverse: (a1 - a3) (+i)
        const float2 t3 = INV ? make_float2(-d.y, d.x) : make_float2(d.y, -d.x);
        y[m][0] = cadd(t0, t2);
        y[m][1] = cadd(t1, t3);
        y[m][2] = csub(t0, t2);
        y[m][3] = csub(t1, t3);
      }
    }
    __syncthreads();
#pragma unroll
    for (int m = 0; m < kFftPer; ++m) {
      const int j = tid + m * kFftThreads;
      if (j < q) {
        const int k = j & (ns - 1);
        const int base = (j - k) * 4 + k;
#pragma unroll
        for (int r = 0; r < 4; ++r) buf[base + r * ns] = y[m][r];
      }
    }
    __syncthreads();
    ns *= 4;
    rem -= 2;
  }
  if (rem == 1) {
    const int h = n >> 1;
    const int step = n / (ns * 2);
    float2 y[2 * kFftPer][2];
#pragma unroll
    for (int m = 0; m < 2 * kFftPer; ++m) {
      const int j = tid + m * kFftThreads;
      if (j < h) {
        const int k = j & (ns - 1);
        const float2 a0 = buf[j];
        const float2 a1 = ns > 1 ? cmul(buf[j + h], twiddle<INV>(tw, k * step, n)) : buf[j + h];
        y[m][0] = cadd(a0, a1);
        y[m][1] = csub(a0, a1);
      }
    }
    __syncthreads();
#pragma unroll
    for (int m = 0; m < 2 * kFftPer; ++m) {
      const int j = tid + m * kFftThreads;
      if (j < h) {
        const int k = j & (ns - 1);
        const int base = (j - k) * 2 + k;
        buf[base] = y[m][0];
        buf[base + ns] = y[m][1];
      }
    }
    __syncthreads();
  }
}

__device__ __forceinline__ float2 conjf2(float2 a) { return make_float2(a.x, -a.y); }

// 4096-point rows (in may equal out: each thread reads and writes the same indices).
template <bool INV>
__global__ __launch_bounds__(kFftThreads) void k_fft4096(const float2* in, float2* out, float scale, int64_t rows) {
  __shared__ float2 buf[kF16Row];
  __shared__ float2 tw[kFftMax / 2];
  fft_twiddles(tw, kFftMax);
  const int t = threadIdx.x;
  for (int64_t row = blockIdx.x; row < rows; row += gridDim.x) {
    const float2* src = in + row * kFftMax;
    float2* dst = out + row * kFftMax;
    float2 v[16];
#pragma unroll
    for (int r = 0; r < 16; ++r) v[r] = INV ? conjf2(src[t + 256 * r]) : src[t + 256 * r];
    __syncthreads();                       // the previous row's last-pass reads are done
    f16_pass1(buf, v);
    __syncthreads();
    f16_pass2(buf, tw);
    __syncthreads();
    f16_pass3(buf, tw, v);
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const float2 a = X16(v, r);
      dst[t + 256 * r] = make_float2(a.x * scale, (INV ? -a.y : a.y) * scale);
    }
  }
}

// Batched unitary transform of `rows` contiguous rows of n points (in may equal out).
// Persistent: workgroup g takes rows g, g + G, ...; the twiddle table is built once.
template <bool INV>
__global__ __launch_bounds__(kFftThreads) void k_fft(const float2* in, float2* out, int n,
                                                     int log2n, float scale, int64_t rows) {
  __shared__ float2 buf[kFftMax];
  __shared__ float2 tw[kFftMax / 2];
  fft_twiddles(tw, n);
  for (int64_t row = blockIdx.x; row < rows; row += gridDim.x) {
    const float2* src = in + row * n;
    float2* dst = out + row * n;
    __syncthreads();                       // previous row's stores read buf
    for (int i = threadIdx.x; i < n; i += kFftThreads) buf[i] = src[i];
    __syncthreads();
    fft_lds<INV>(buf, tw, n, log2n);
    for (int i = threadIdx.x; i < n; i += kFftThreads) {
      const float2 v = buf[i];
      dst[i] = make_float2(v.x * scale, v.y * scale);
    }
  }
}

// ---------------------------------------------------------------------------
// FD-NN network on time samples.  Weights live in LDS zero-padded to compile-time
// widths: inputs FM (>= 2 U (L4+1)), hidden DM (>= D), outputs 16 (>= 2 U); padded
// hidden units stay ReLU(0) = 0 and padded inputs are 0, so the padded network equals
// the real one.  LDS weight layout (floats): W1 transposed [FM][DM], b1[DM],
// (W2[DM][DM] b2[DM]), Wo[16][DM], bo[16]; row starts are 16-byte aligned so rows are
// read as broadcast float4 (every lane of a wave reads the same weights).
// ---------------------------------------------------------------------------
constexpr int kNnOut = 16;
constexpr int kNnFwdT = 256;     // forward: threads = samples per tile
constexpr int kNnBwdT = 128;     // backward: threads = samples per tile
constexpr int kNnMaxMem = 7;     // L4 <= 7

template <int FM, int DM, int NH>
struct NnLayout {
  static constexpr int w1 = 0, b1 = DM * FM;
  static constexpr int w2 = b1 + DM, b2 = w2 + (NH > 1 ? DM * DM : 0);
  static constexpr int wo = b2 + (NH > 1 ? DM : 0), bo = wo + kNnOut * DM;
  static constexpr int total = bo + kNnOut;
};

// Packed parameter index p of the real network -> padded LDS index (or -1 if none).
template <int FM, int DM, int NH>
__device__ inline int nn_padded_index(int p, int F, int D, int U) {
  using Ly = NnLayout<FM, DM, NH>;
  if (p < D * F) return Ly::w1 + (p % F) * DM + p / F;     // W1[i][j] -> W1T[j][i]
  p -= D * F;
  if (p < D) return Ly::b1 + p;
  p -= D;
  if (NH > 1) {
    if (p < D * D) return Ly::w2 + (p / D) * DM + p % D;
    p -= D * D;
    if (p < D) return Ly::b2 + p;
    p -= D;
  }
  if (p < 2 * U * D) return Ly::wo + (p / D) * DM + p % D;
  p -= 2 * U * D;
  if (p < 2 * U) return Ly::bo + p;
  return -1;
}

template <int FM, int DM, int NH>
__device__ void nn_load_weights(float* lw, const float* __restrict__ w, int F, int D, int U, int P) {
  using Ly = NnLayout<FM, DM, NH>;
  for (int i = threadIdx.x; i < Ly::total; i += blockDim.x) lw[i] = 0.f;
  __syncthreads();
  for (int p = threadIdx.x; p < P; p += blockDim.x) lw[nn_padded_index<FM, DM, NH>(p, F, D, U)] = w[p];
  __syncthreads();
}

// Tap window of one tile: win[u][m] = td[u][(n0 - L4 + m) mod N], m < S + L4.
template <int S>
__device__ void nn_load_window(float2 (*win)[S + kNnMaxMem], const float2* __restrict__ td_sym,
                               int n0, int N, int U, int L4) {
  const int W = S + L4;
  for (int e = threadIdx.x; e < U * W; e += blockDim.x) {
    const int u = e / W, m = e % W;
    int n = (n0 - L4 + m) % N;
    if (n < 0) n += N;
    win[u][m] = td_sym[(int64_t)u * N + n];
  }
}

// First layer for sample s of the tile: h[i] = ReLU(b1[i] + sum over feature pairs
// (u, t) of W1[i][2p] Re z + W1[i][2p+1] Im z), z = td[u][n - t], p = u (L4+1) + t.
template <int FM, int DM, int S>
__device__ __forceinline__ void nn_layer1(float (&h)[DM], const float* lw, const float2 (*win)[S + kNnMaxMem],
                                          int s, int U, int L4) {
  using V = const float4*;
#pragma unroll
  for (int i4 = 0; i4 < DM / 4; ++i4) {
    const float4 b = reinterpret_cast<V>(lw + DM * FM)[i4];
    h[4 * i4] = b.x;
    h[4 * i4 + 1] = b.y;
    h[4 * i4 + 2] = b.z;
    h[4 * i4 + 3] = b.w;
  }
  const int np = U * (L4 + 1);
  int u = 0, t = 0;
#pragma unroll 1
  for (int p = 0; p < np; ++p) {
    const float2 z = win[u][s + L4 - t];
    V wr = reinterpret_cast<V>(lw + 2 * p * DM);
    V wi = reinterpret_cast<V>(lw + (2 * p + 1) * DM);
#pragma unroll
    for (int i4 = 0; i4 < DM / 4; ++i4) {
      const float4 a = wr[i4], c = wi[i4];
      h[4 * i4] = fmaf(a.x, z.x, fmaf(c.x, z.y, h[4 * i4]));
      h[4 * i4 + 1] = fmaf(a.y, z.x, fmaf(c.y, z.y, h[4 * i4 + 1]));
      h[4 * i4 + 2] = fmaf(a.z, z.x, fmaf(c.z, z.y, h[4 * i4 + 2]));
      h[4 * i4 + 3] = fmaf(a.w, z.x, fmaf(c.w, z.y, h[4 * i4 + 3]));
    }
    if (++t > L4) {
      t = 0;
      ++u;
    }
  }
#pragma unroll
  for (int i = 0; i < DM; ++i) h[i] = fmaxf(h[i], 0.f);
}

// out[o] = b[o] + sum_i W[o][i] in[i] for o < NO (W rows of NI floats in LDS, broadcast
// reads), optional ReLU.
template <int NO, int NI, bool RELU>
__device__ __forceinline__ void nn_dense(float (&out)[NO], const float (&in)[NI], const float* W,
                                         const float* b) {
#pragma unroll
  for (int o = 0; o < NO; ++o) {
    DPD_KEEP_LOADS_LOCAL();   // one row of weights in flight at a time (register pressure)
    float acc = b[o];
    const float4* row = reinterpret_cast<const float4*>(W + o * NI);
#pragma unroll
    for (int i4 = 0; i4 < NI / 4; ++i4) {
      const float4 w4 = row[i4];
      acc = fmaf(w4.x, in[4 * i4], acc);
      acc = fmaf(w4.y, in[4 * i4 + 1], acc);
      acc = fmaf(w4.z, in[4 * i4 + 2], acc);
      acc = fmaf(w4.w, in[4 * i4 + 3], acc);
    }
    out[o] = RELU ? fmaxf(acc, 0.f) : acc;
  }
}

// g[j] = (sum_o W[o][j] d[o]) where act[j] > 0, else 0 (the delta one layer down through
// a ReLU): rows of W in LDS, NO x NI.
template <int NO, int NI>
__device__ __forceinline__ void nn_back(float (&g)[NI], const float (&d)[NO], const float (&act)[NI],
                                        const float* W) {
#pragma unroll
  for (int j = 0; j < NI; ++j) g[j] = 0.f;
#pragma unroll
  for (int o = 0; o < NO; ++o) {
    DPD_KEEP_LOADS_LOCAL();
    const float4* row = reinterpret_cast<const float4*>(W + o * NI);
#pragma unroll
    for (int j4 = 0; j4 < NI / 4; ++j4) {
      const float4 w4 = row[j4];
      g[4 * j4] = fmaf(w4.x, d[o], g[4 * j4]);
      g[4 * j4 + 1] = fmaf(w4.y, d[o], g[4 * j4 + 1]);
      g[4 * j4 + 2] = fmaf(w4.z, d[o], g[4 * j4 + 2]);
      g[4 * j4 + 3] = fmaf(w4.w, d[o], g[4 * j4 + 3]);
    }
  }
#pragma unroll
  for (int j = 0; j < NI; ++j) g[j] = act[j] > 0.f ? g[j] : 0.f;
}

template <int FM, int DM, int NH>
__global__ __launch_bounds__(kNnFwdT) void k_fdnn_fwd(const float2* __restrict__ td, const float* __restrict__ w,
                                                      float2* __restrict__ o_td, int N, int U, int L4, int D,
                                                      int P, int tiles_per_sym, int n_tiles) {
  using Ly = NnLayout<FM, DM, NH>;
  constexpr int S = kNnFwdT;
  __shared__ __align__(16) float lw[Ly::total];
  __shared__ float2 win[8][S + kNnMaxMem];
  __shared__ float2 so[S][kNnOut / 2 + 1];
  const int F = 2 * U * (L4 + 1);
  nn_load_weights<FM, DM, NH>(lw, w, F, D, U, P);
  const int t0 = wg_tile_start(blockIdx.x, gridDim.x, n_tiles);
  const int t1 = wg_tile_start(blockIdx.x + 1, gridDim.x, n_tiles);
  for (int tile = t0; tile < t1; ++tile) {
    const int sym = tile / tiles_per_sym;
    const int n0 = (tile % tiles_per_sym) * S;
    const float2* td_sym = td + (int64_t)sym * U * N;
    __syncthreads();
    nn_load_window<S>(win, td_sym, n0, N, U, L4);
    __syncthreads();
    const int n = n0 + threadIdx.x;
    if (n >= N) continue;
    float h1[DM];
    nn_layer1<FM, DM, S>(h1, lw, win, threadIdx.x, U, L4);
    float o[kNnOut];
    if constexpr (NH > 1) {
      float h2[DM];
      nn_dense<DM, DM, true>(h2, h1, lw + Ly::w2, lw + Ly::b2);
      nn_dense<kNnOut, DM, false>(o, h2, lw + Ly::wo, lw + Ly::bo);
    } else {
      nn_dense<kNnOut, DM, false>(o, h1, lw + Ly::wo, lw + Ly::bo);
    }
    // outputs go through this thread's own LDS row so that the per-UE stores are a
    // plain runtime loop (conditional stores of register values made the compiler
    // keep far more registers live)
    float2* dst = o_td + (int64_t)sym * U * N + n;
#pragma unroll
    for (int q = 0; q < kNnOut / 2; ++q) so[threadIdx.x][q] = make_float2(o[2 * q], o[2 * q + 1]);
    for (int u = 0; u < U; ++u) dst[(int64_t)u * N] = so[threadIdx.x][u];
  }
}

// acc[r] += delta[s][RB rg + r] a for r < RB (delta rows of RS floats in LDS, read as
// broadcast float4: all lanes of a wave share rg).
template <int RB, int RS>
__device__ __forceinline__ void nn_outer(float (&acc)[RB], const float* delta, int rg, int s, float a) {
  const float4* d4 = reinterpret_cast<const float4*>(delta + s * RS + RB * rg);
#pragma unroll
  for (int r4 = 0; r4 < RB / 4; ++r4) {
    const float4 v = d4[r4];
    acc[4 * r4] = fmaf(v.x, a, acc[4 * r4]);
    acc[4 * r4 + 1] = fmaf(v.y, a, acc[4 * r4 + 1]);
    acc[4 * r4 + 2] = fmaf(v.z, a, acc[4 * r4 + 2]);
    acc[4 * r4 + 3] = fmaf(v.w, a, acc[4 * r4 + 3]);
  }
}

// Backward of the network for time-sample gradients g_td (real convention: output 2u
// gets Re g_td[u][n], 2u + 1 Im).  Persistent over a contiguous tile range; per thread
// register accumulators of the padded dW, written once as this workgroup's partial
// part[blockIdx.x][Ly::total].  Ownership (128 threads): W1 column (feature) t % FM and
// rows [R1 (t / FM), +R1); W2 and Wo column t % 32 (< DM) and rows of group t / 32;
// biases: thread t < DM b1, 32 <= t < 32 + DM b2, 64 <= t < 80 bo.  Each layer's
// deltas and inputs are staged in LDS for the tile, then every owner sums its outer
// products over the tile's samples.
template <int FM, int DM, int NH>
__global__ __launch_bounds__(kNnBwdT) void k_fdnn_bwd(const float2* __restrict__ td, const float2* __restrict__ g_td,
                                                      const float* __restrict__ w, float* __restrict__ part,
                                                      int N, int U, int L4, int D, int P, int tiles_per_sym,
                                                      int n_tiles) {
  using Ly = NnLayout<FM, DM, NH>;
  constexpr int S = kNnBwdT;
  constexpr int R1 = DM * FM / kNnBwdT;        // W1 rows per thread (FM * (128 / FM) threads)
  constexpr int R2 = DM * 32 / kNnBwdT;        // W2 rows per thread
  constexpr int RO = kNnOut * 32 / kNnBwdT;    // Wo rows per thread
  static_assert(R1 % 4 == 0 && R2 % 4 == 0 && RO % 4 == 0, "row blocks are float4 reads");
  __shared__ __align__(16) float lw[Ly::total];
  __shared__ float2 win[8][S + kNnMaxMem];
  __shared__ __align__(16) float sd[S * DM];       // staged deltas of one layer
  __shared__ __align__(16) float sa[S * DM];       // staged input activations of one layer
  const int F = 2 * U * (L4 + 1);
  nn_load_weights<FM, DM, NH>(lw, w, F, D, U, P);
  const int tid = threadIdx.x;
  const int c1 = tid % FM, g1 = tid / FM;
  const int c2 = tid % 32, g2 = tid / 32;
  // feature of W1 column c1: UE fu, delay ft, Re (0) or Im (1)
  const int fu = (c1 / 2) / (L4 + 1), ft = (c1 / 2) % (L4 + 1), fim = c1 & 1;
  float a1[R1], a2[R2], ao[RO], ab = 0.f;
#pragma unroll
  for (int i = 0; i < R1; ++i) a1[i] = 0.f;
#pragma unroll
  for (int i = 0; i < R2; ++i) a2[i] = 0.f;
#pragma unroll
  for (int i = 0; i < RO; ++i) ao[i] = 0.f;
  const int t0 = wg_tile_start(blockIdx.x, gridDim.x, n_tiles);
  const int t1 = wg_tile_start(blockIdx.x + 1, gridDim.x, n_tiles);
  for (int tile = t0; tile < t1; ++tile) {
    const int sym = tile / tiles_per_sym;
    const int n0 = (tile % tiles_per_sym) * S;
    const int cnt = min(S, N - n0);
    const float2* td_sym = td + (int64_t)sym * U * N;
    __syncthreads();
    nn_load_window<S>(win, td_sym, n0, N, U, L4);
    __syncthreads();
    // per-sample forward and the output-layer delta (zero for samples past N)
    const bool live = tid < cnt;
    float h1[DM];
    nn_layer1<FM, DM, S>(h1, lw, win, tid, U, L4);
    float dout[kNnOut];
#pragma unroll
    for (int u = 0; u < kNnOut / 2; ++u) {
      float2 g = make_float2(0.f, 0.f);
      if (live && u < U) g = g_td[(int64_t)sym * U * N + (int64_t)u * N + n0 + tid];
      dout[2 * u] = g.x;
      dout[2 * u + 1] = g.y;
    }
    float dh[DM];
    if constexpr (NH > 1) {
      float h2[DM];
      nn_dense<DM, DM, true>(h2, h1, lw + Ly::w2, lw + Ly::b2);
      // ---- output layer: dWo[o][j] += dout[o] h2[j]
#pragma unroll
      for (int o = 0; o < kNnOut; ++o) sd[tid * kNnOut + o] = dout[o];
#pragma unroll
      for (int j = 0; j < DM; ++j) sa[tid * DM + j] = h2[j];
      __syncthreads();
      if (c2 < DM)
        for (int s = 0; s < cnt; ++s) nn_outer<RO, kNnOut>(ao, sd, g2, s, sa[s * DM + c2]);
      if (tid >= 64 && tid < 64 + kNnOut)
        for (int s = 0; s < cnt; ++s) ab += sd[s * kNnOut + tid - 64];
      nn_back<kNnOut, DM>(dh, dout, h2, lw + Ly::wo);
      __syncthreads();
      // ---- second hidden layer: dW2[i][j] += dh[i] h1[j]
#pragma unroll
      for (int j = 0; j < DM; ++j) {
        sd[tid * DM + j] = dh[j];
        sa[tid * DM + j] = h1[j];
      }
      __syncthreads();
      if (c2 < DM)
        for (int s = 0; s < cnt; ++s) nn_outer<R2, DM>(a2, sd, g2, s, sa[s * DM + c2]);
      if (tid >= 32 && tid < 32 + DM)
        for (int s = 0; s < cnt; ++s) ab += sd[s * DM + tid - 32];
      float d1[DM];
      nn_back<DM, DM>(d1, dh, h1, lw + Ly::w2);
#pragma unroll
      for (int j = 0; j < DM; ++j) dh[j] = d1[j];
      __syncthreads();
    } else {
      // ---- output layer: dWo[o][j] += dout[o] h1[j]
#pragma unroll
      for (int o = 0; o < kNnOut; ++o) sd[tid * kNnOut + o] = dout[o];
#pragma unroll
      for (int j = 0; j < DM; ++j) sa[tid * DM + j] = h1[j];
      __syncthreads();
      if (c2 < DM)
        for (int s = 0; s < cnt; ++s) nn_outer<RO, kNnOut>(ao, sd, g2, s, sa[s * DM + c2]);
      if (tid >= 64 && tid < 64 + kNnOut)
        for (int s = 0; s < cnt; ++s) ab += sd[s * kNnOut + tid - 64];
      nn_back<kNnOut, DM>(dh, dout, h1, lw + Ly::wo);
      __syncthreads();
    }
    // ---- first layer: dW1[i][c] += d1[i] f[c] (features re-read from the window)
#pragma unroll
    for (int j = 0; j < DM; ++j) sd[tid * DM + j] = dh[j];
    __syncthreads();
    if (c1 < F) {
      for (int s = 0; s < cnt; ++s) {
        const float2 z = win[fu][s + L4 - ft];
        nn_outer<R1, DM>(a1, sd, g1, s, fim ? z.y : z.x);
      }
    }
    if (tid < DM)
      for (int s = 0; s < cnt; ++s) ab += sd[s * DM + tid];
  }
  // write the partial (padded layout); untouched entries of the layout are written 0
  float* out = part + (int64_t)blockIdx.x * Ly::total;
  __syncthreads();
  for (int i = tid; i < Ly::total; i += kNnBwdT) out[i] = 0.f;
  __syncthreads();
#pragma unroll
  for (int r = 0; r < R1; ++r) out[Ly::w1 + c1 * DM + R1 * g1 + r] = a1[r];
  if (c2 < DM) {
    if constexpr (NH > 1) {
#pragma unroll
      for (int r = 0; r < R2; ++r) out[Ly::w2 + (R2 * g2 + r) * DM + c2] = a2[r];
    }
#pragma unroll
    for (int r = 0; r < RO; ++r) out[Ly::wo + (RO * g2 + r) * DM + c2] = ao[r];
  }
  if (tid < DM) out[Ly::b1 + tid] = ab;
  if (NH > 1 && tid >= 32 && tid < 32 + DM) out[Ly::b2 + tid - 32] = ab;
  if (tid >= 64 && tid < 64 + kNnOut) out[Ly::bo + tid - 64] = ab;
}

// Fixed-order sum of the workgroup partials in two stages: mid[sp][p] = sum over the
// partials g of split sp (in order) of part[g][padded(p)]; dw[p] = sum over the splits in
// order.
constexpr int kNnSplits = 32;
template <int FM, int DM, int NH>
__global__ __launch_bounds__(256) void k_fdnn_reduce1(const float* __restrict__ part, int G, int F, int D,
                                                      int U, int P, float* __restrict__ mid) {
  using Ly = NnLayout<FM, DM, NH>;
  const int p = blockIdx.x * 256 + threadIdx.x;
  if (p >= P) return;
  const int sp = blockIdx.y;
  const int g0 = (int)((int64_t)sp * G / kNnSplits), g1 = (int)((int64_t)(sp + 1) * G / kNnSplits);
  const int q = nn_padded_index<FM, DM, NH>(p, F, D, U);
  float acc = 0.f;
  for (int g = g0; g < g1; ++g) acc += part[(int64_t)g * Ly::total + q];
  mid[(int64_t)sp * P + p] = acc;
}

__global__ __launch_bounds__(256) void k_fdnn_reduce2(const float* __restrict__ mid, int P, float* __restrict__ dw) {
  const int p = blockIdx.x * 256 + threadIdx.x;
  if (p >= P) return;
  float acc = 0.f;
  for (int sp = 0; sp < kNnSplits; ++sp) acc += mid[(int64_t)sp * P + p];
  dw[p] = acc;
}

// ---------------------------------------------------------------------------
// ZF precoder: one single-wave workgroup per (channel, subcarrier); FP64 throughout.
// ---------------------------------------------------------------------------
constexpr int kZfMaxU = 8;
constexpr int kZfMaxB = 256;
constexpr int kZfMaxT = 64;
constexpr int kZfE = 2;     // H_k elements per lane and pass
constexpr int kZfTc = 8;    // taps per batch of loads

__device__ __forceinline__ double2 zmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

// Subcarrier of data symbol d: 1 + d for d < n_d / 2, else N - n_d + d.
__device__ __forceinline__ int data_bin(int d, int N, int n_d) {
  return d < n_d / 2 ? 1 + d : N - n_d + d;
}

// e^{-2 pi i (k t mod N) / N} in double.
__device__ __forceinline__ double2 unit_phase(int64_t k, int t, int N) {
  const int64_t e = (k * t) % N;
  double s, c;
  sincospi(-2.0 * (double)e / (double)N, &s, &c);
  return make_double2(c, s);
}

// (r, k) -> the (row, column) of the element 64 further on in a row-major array of C
// columns (q = 64 / C, m = 64 % C).
__device__ __forceinline__ void step64(int& r, int& k, int q, int m, int C) {
  r += q;
  k += m;
  if (k >= C) {
    k -= C;
    ++r;
  }
}

// Pt_k = H_k^H (H_k H_k^H)^-1 with H_k = sum_t H_t e^{-2 pi i k t / N}; tr(Pt^H Pt) -> trace.
// Subcarrier k = blockIdx.x (all_bins) or the data subcarrier blockIdx.x.  Dynamic LDS:
// the T phases and H_k [U][B] (sized to the problem, so small antenna counts keep many
// waves resident).
__global__ __launch_bounds__(64) void k_zf(const float2* __restrict__ h, int N, int n_d, int all_bins, int U,
                                           int B, int T, float2* __restrict__ pt, double* __restrict__ trace) {
  extern __shared__ double2 zf_dyn[];
  double2* ph = zf_dyn;
  double2* hk = zf_dyn + T;                 // H_k rows of B + 1 (the pad spreads rows over the banks)
  const int hs = B + 1;
  __shared__ double2 A[kZfMaxU][kZfMaxU + 1], I[kZfMaxU][kZfMaxU + 1];   // padded rows: column reads hit distinct banks
  __shared__ double red[64];
  const int lane = threadIdx.x;
  const int c = blockIdx.y;
  const int nbins = all_bins ? N : n_d;
  // element e = lane + 64 m of a row-major [R][C] array sits at (e / C, e % C); the lanes
  // step through m with a carry instead of integer divisions
  const int qB = 64 / B, rB = 64 % B, hu0 = lane / B, hb0 = lane % B;
  const int qU = 64 / U, rU = 64 % U, pb0 = lane / U, pu0 = lane % U;
  // one subcarrier per workgroup (grid-stride form; looping over several per workgroup
  // measured slower)
  for (int kb = blockIdx.x; kb < nbins; kb += gridDim.x) {
    const int k = all_bins ? kb : data_bin(kb, N, n_d);
    __syncthreads();                         // the previous subcarrier is done with the LDS
    for (int t = lane; t < T; t += 64) ph[t] = unit_phase(k, t, N);
    __syncthreads();
    const float2* hc = h + (int64_t)c * T * U * B;
    int hu = hu0, hb = hb0;                  // (row, column) of H_k element lane + 64 m
    for (int e0 = lane; e0 < U * B; e0 += 64 * kZfE) {
      double2 acc[kZfE];
#pragma unroll
      for (int q = 0; q < kZfE; ++q) acc[q] = make_double2(0.0, 0.0);
      for (int t0 = 0; t0 < T; t0 += kZfTc) {
        // the chunk's kZfE x kZfTc tap loads are issued together (one wait per chunk, not per tap)
        // (unconditional loads from clamped, in-bounds indices: a guarded load is a branch
        // that ends in its own wait; the taps past T are skipped below, lanes past U B unused)
        float2 v[kZfE][kZfTc];
#pragma unroll
        for (int q = 0; q < kZfE; ++q)
#pragma unroll
          for (int tt = 0; tt < kZfTc; ++tt)
            v[q][tt] = hc[(int64_t)min(t0 + tt, T - 1) * U * B + min(e0 + 64 * q, U * B - 1)];
#pragma unroll
        for (int tt = 0; tt < kZfTc; ++tt) {
          if (t0 + tt < T) {
            const double2 p = ph[t0 + tt];
#pragma unroll
            for (int q = 0; q < kZfE; ++q)
              acc[q] = make_double2(acc[q].x + (double)v[q][tt].x * p.x - (double)v[q][tt].y * p.y,
                                    acc[q].y + (double)v[q][tt].x * p.y + (double)v[q][tt].y * p.x);
          }
        }
      }
#pragma unroll
      for (int q = 0; q < kZfE; ++q) {
        if (e0 + 64 * q < U * B) hk[hu * hs + hb] = acc[q];
        step64(hu, hb, qB, rB, B);
      }
    }
    __syncthreads();
    const int i = lane / kZfMaxU, j = lane % kZfMaxU;
    const bool own = i < U && j < U;
    if (own) {
      double2 g = make_double2(0.0, 0.0);
      for (int b = 0; b < B; ++b) {          // G[i][j] = sum_b H[i][b] conj(H[j][b])
        const double2 x = hk[i * hs + b], y = hk[j * hs + b];
        g.x = fma(x.x, y.x, g.x);
        g.x = fma(x.y, y.y, g.x);
        g.y = fma(x.y, y.x, g.y);
        g.y = fma(-x.x, y.y, g.y);
      }
      A[i][j] = g;
      I[i][j] = make_double2(i == j ? 1.0 : 0.0, 0.0);
    }
    __syncthreads();
    // Gauss-Jordan on [A | I] without pivoting (A is Hermitian positive definite)
    for (int p = 0; p < U; ++p) {
      double2 na = make_double2(0.0, 0.0), ni = na;
      if (own) {
        const double2 piv = A[p][p];
        const double r2 = 1.0 / (piv.x * piv.x + piv.y * piv.y);   // one FP64 division per pivot
        const double2 inv = make_double2(piv.x * r2, -piv.y * r2);
        if (i == p) {
          na = zmul(A[p][j], inv);
          ni = zmul(I[p][j], inv);
        } else {
          const double2 fct = zmul(A[i][p], inv);
          const double2 x = zmul(fct, A[p][j]), y = zmul(fct, I[p][j]);
          na = make_double2(A[i][j].x - x.x, A[i][j].y - x.y);
          ni = make_double2(I[i][j].x - y.x, I[i][j].y - y.y);
        }
      }
      __syncthreads();
      if (own) {
        A[i][j] = na;
        I[i][j] = ni;
      }
      __syncthreads();
    }
    // Pt[b][u] = sum_j conj(H[j][b]) Ginv[j][u]
    double tr = 0.0;
    float2* dst = pt + ((int64_t)c * N + k) * B * U;
    int b = pb0, u = pu0;                    // (b, u) of element e of Pt_k [B][U]
    for (int e = lane; e < B * U; e += 64) {
      double2 acc = make_double2(0.0, 0.0);
      for (int jj = 0; jj < U; ++jj) {         // conj(H[jj][b]) Ginv[jj][u]
        const double2 hv = hk[jj * hs + b], q = I[jj][u];
        acc.x = fma(hv.x, q.x, acc.x);
        acc.x = fma(hv.y, q.y, acc.x);
        acc.y = fma(hv.x, q.y, acc.y);
        acc.y = fma(-hv.y, q.x, acc.y);
      }
      dst[e] = make_float2((float)acc.x, (float)acc.y);
      tr += acc.x * acc.x + acc.y * acc.y;
      step64(b, u, qU, rU, U);
    }
    red[lane] = tr;
    __syncthreads();
    for (int w = 32; w > 0; w >>= 1) {
      if (lane < w) red[lane] += red[lane + w];
      __syncthreads();
    }
    if (lane == 0) trace[(int64_t)c * N + k] = red[0];
  }
}

// alpha[c] = sqrt(P_T / mean over data subcarriers of trace[c][k]) (fixed-order tree).
__global__ __launch_bounds__(256) void k_zf_alpha(const double* __restrict__ trace, int N, int n_d,
                                                  float p_total, float* __restrict__ alpha) {
  __shared__ double red[256];
  const int c = blockIdx.x;
  double s = 0.0;
  for (int d = threadIdx.x; d < n_d; d += 256) s += trace[(int64_t)c * N + data_bin(d, N, n_d)];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) alpha[c] = (float)sqrt((double)p_total * (double)n_d / red[0]);
}

// x[i][b][k] = alpha_c sum_u Pt[c][k][b][u] s[i][u][k] on the precoded subcarriers, else 0.
// One workgroup per (tile of tw precoded subcarriers, symbol i); the guard subcarriers are
// zeroed beforehand by zero_complex.  Three phases: the tile's symbols into LDS; one thread per
// (subcarrier, antenna) with the antenna fastest, so a wave reads consecutive rows of Pt; the
// outputs leave through an LDS tile [B][tw+1] with the subcarrier fastest (contiguous
// tw-wide runs of each antenna row of x).
constexpr int kPcTile = 32;

// Tile width in subcarriers: kPcTile, halved for more than 128 antennas so that the LDS
// tiles stay within 64 KiB.
inline int precode_tile(int B) { return B <= 128 ? kPcTile : kPcTile / 2; }

template <bool VEC>
__global__ __launch_bounds__(256) void k_precode(const float2* __restrict__ pt, const float* __restrict__ alpha,
                                                 const float2* __restrict__ s, int N, int n_d, int U, int B,
                                                 int spc, int all_bins, int tw, float2* __restrict__ x) {
  extern __shared__ float2 pc_lds[];
  float2* st = pc_lds;                  // [kZfMaxU][tw]
  float2* xt = pc_lds + kZfMaxU * tw;   // [B][tw + 1]
  const int XS = tw + 1;
  const int i = blockIdx.y;
  const int c = i / spc;
  const int e0 = blockIdx.x * tw;
  const int nb = min(tw, (all_bins ? N : n_d) - e0);
  const float a = alpha[c];
  const float2* si = s + (int64_t)i * U * N;
  for (int j = threadIdx.x; j < U * tw; j += 256) {
    const int u = j / tw, el = j % tw;
    if (el < nb) st[j] = si[(int64_t)u * N + (all_bins ? e0 + el : data_bin(e0 + el, N, n_d))];
  }
  __syncthreads();
  if (VEC && U == kZfMaxU) {
    // eight UEs: four lanes per 64-byte row of Pt, one 16-byte piece each, so a wave's load
    // is 1 KB of consecutive rows; the four partial sums meet by two xor shuffles (the loop
    // bound is a multiple of 4, so a lane group is active or idle as a whole)
    for (int j = threadIdx.x; j < nb * B * 4; j += 256) {
      const int r = j >> 2, q = j & 3;
      const int el = r / B, b = r - el * B;
      const int k = all_bins ? e0 + el : data_bin(e0 + el, N, n_d);
      const float4 v = reinterpret_cast<const float4*>(pt + (((int64_t)c * N + k) * B + b) * kZfMaxU)[q];
      float2 acc = cmul(make_float2(v.x, v.y), st[(2 * q) * tw + el]);
      acc = cadd(acc, cmul(make_float2(v.z, v.w), st[(2 * q + 1) * tw + el]));
      acc.x += __shfl_xor(acc.x, 1);
      acc.y += __shfl_xor(acc.y, 1);
      acc.x += __shfl_xor(acc.x, 2);
      acc.y += __shfl_xor(acc.y, 2);
      if (q == 0) xt[b * XS + el] = make_float2(a * acc.x, a * acc.y);
    }
  } else {
    for (int j = threadIdx.x; j < nb * B; j += 256) {
      const int el = j / B, b = j - el * B;
      const int k = all_bins ? e0 + el : data_bin(e0 + el, N, n_d);
      const float2* row = pt + (((int64_t)c * N + k) * B + b) * U;
      float2 acc = make_float2(0.f, 0.f);
      if (VEC) {
        // even U and a 16-byte aligned pt: the row is U/2 aligned 16-byte pairs
        const float4* row4 = reinterpret_cast<const float4*>(row);
#pragma unroll
        for (int u2 = 0; u2 < kZfMaxU / 2; ++u2) {
          if (2 * u2 < U) {
            const float4 q = row4[u2];
            acc = cadd(acc, cmul(make_float2(q.x, q.y), st[(2 * u2) * tw + el]));
            acc = cadd(acc, cmul(make_float2(q.z, q.w), st[(2 * u2 + 1) * tw + el]));
          }
        }
      } else {
#pragma unroll
        for (int u = 0; u < kZfMaxU; ++u)
          if (u < U) acc = cadd(acc, cmul(row[u], st[u * tw + el]));
      }
      xt[b * XS + el] = make_float2(a * acc.x, a * acc.y);
    }
  }
  __syncthreads();
  float2* xi = x + (int64_t)i * B * N;
  for (int j = threadIdx.x; j < nb * B; j += 256) {
    const int b = j / nb, el = j - b * nb;
    xi[(int64_t)b * N + (all_bins ? e0 + el : data_bin(e0 + el, N, n_d))] = xt[b * XS + el];
  }
}

// ---------------------------------------------------------------------------
// Link
// ---------------------------------------------------------------------------
// True channel on the data subcarriers: hd[c][d][u][b] = sum_t H_t[u][b] e^{-2 pi i k_d t / N};
// one workgroup per (data subcarrier, realisation), the T phases shared through LDS.
__global__ __launch_bounds__(256) void k_chan_data(const float2* __restrict__ h, int N, int n_d, int U, int B,
                                                   int T, float2* __restrict__ hd) {
  __shared__ double2 ph[kZfMaxT];
  const int d = blockIdx.x, c = blockIdx.y;
  const int k = data_bin(d, N, n_d);
  for (int t = threadIdx.x; t < T; t += 256) ph[t] = unit_phase(k, t, N);
  __syncthreads();
  const float2* hc = h + (int64_t)c * T * U * B;
  float2* dst = hd + ((int64_t)c * n_d + d) * U * B;
  // (a plain loop over the taps: with four waves per workgroup and many workgroups resident,
  // batching the tap loads as in k_zf measured 15 % slower here)
  for (int e = threadIdx.x; e < U * B; e += 256) {
    double re = 0.0, im = 0.0;
    for (int t = 0; t < T; ++t) {
      const float2 v = hc[(int64_t)t * U * B + e];
      re += (double)v.x * ph[t].x - (double)v.y * ph[t].y;
      im += (double)v.x * ph[t].y + (double)v.y * ph[t].x;
    }
    dst[e] = make_float2((float)re, (float)im);
  }
}

// GMP of eq. (9) with cyclic delays on the LDS symbol buf (magnitudes in r), results to
// the registers y[m] for samples t + m kFftThreads.  coef: this antenna's [J] set.  N is a
// power of two, so every cyclic index is a mask.  Samples go in batches of Q with the
// coefficient loops outside: each (wave-uniform) coefficient is read once per batch, and
// the batch's Horner chains run side by side.
template <int Q>
__device__ __forceinline__ void gmp_cyclic_batch(const float2* buf, const float* r, int N,
                                                 const float2* __restrict__ coef, int K, int M, int L, int q0,
                                                 float2 (&y)[kFftMax / kFftThreads]) {
  const int na = K * (M + 1), nb = (K - 1) * (M + 1) * L, sb = (M + 1) * L;
  const int mask = N - 1;
  int nn[Q];
  float2 acc[Q];
#pragma unroll
  for (int j = 0; j < Q; ++j) {
    nn[j] = threadIdx.x + (q0 + j) * kFftThreads;
    acc[j] = make_float2(0.f, 0.f);
  }
  for (int l = 0; l <= M; ++l) {
    float rl[Q];
    float2 ul[Q], poly[Q];
    const float2 top = coef[(K - 1) * (M + 1) + l];
#pragma unroll
    for (int j = 0; j < Q; ++j) {
      const int nl = (nn[j] - l) & mask;
      rl[j] = r[nl];
      ul[j] = buf[nl];
      poly[j] = top;
    }
    for (int k = K - 2; k >= 0; --k) {                  // Horner over k of a_{k,l} r^k
      const float2 a = coef[k * (M + 1) + l];
#pragma unroll
      for (int j = 0; j < Q; ++j) poly[j] = make_float2(fmaf(poly[j].x, rl[j], a.x), fmaf(poly[j].y, rl[j], a.y));
    }
    for (int g = 1; K > 1 && g <= L; ++g) {
      const int ib = na + l * L + (g - 1), ic = ib + nb;
      const float2 tb = coef[ib + (K - 2) * sb], tc = coef[ic + (K - 2) * sb];
      float rb[Q], rc[Q];
      float2 pb[Q], pc[Q];
#pragma unroll
      for (int j = 0; j < Q; ++j) {
        rb[j] = r[(nn[j] - l - g) & mask];
        rc[j] = r[(nn[j] - l + g) & mask];
        pb[j] = tb;
        pc[j] = tc;
      }
      for (int k = K - 2; k >= 1; --k) {                // b_{k,l,g}, c_{k,l,g} at k - 1 of [K-1]
        const float2 bb = coef[ib + (k - 1) * sb], cc = coef[ic + (k - 1) * sb];
#pragma unroll
        for (int j = 0; j < Q; ++j) {
          pb[j] = make_float2(fmaf(pb[j].x, rb[j], bb.x), fmaf(pb[j].y, rb[j], bb.y));
          pc[j] = make_float2(fmaf(pc[j].x, rc[j], cc.x), fmaf(pc[j].y, rc[j], cc.y));
        }
      }
#pragma unroll
      for (int j = 0; j < Q; ++j)
        poly[j] = make_float2(fmaf(pb[j].x, rb[j], fmaf(pc[j].x, rc[j], poly[j].x)),
                              fmaf(pb[j].y, rb[j], fmaf(pc[j].y, rc[j], poly[j].y)));
    }
#pragma unroll
    for (int j = 0; j < Q; ++j) acc[j] = cadd(acc[j], cmul(ul[j], poly[j]));
  }
#pragma unroll
  for (int j = 0; j < Q; ++j) y[q0 + j] = acc[j];
}

__device__ void gmp_cyclic_lds(const float2* buf, const float* r, int N, const float2* __restrict__ coef,
                               int K, int M, int L, float2 (&y)[kFftMax / kFftThreads]) {
  constexpr int kQ = 8;
  constexpr int kMaxQ = kFftMax / kFftThreads;
  const int nq = (N + kFftThreads - 1) / kFftThreads;  // samples per thread (<= 16)
  // fully unrolled, so that y is indexed by constants only (a runtime index would put it
  // in scratch memory)
#pragma unroll
  for (int q0 = 0; q0 < kMaxQ; q0 += kQ) {
    if (q0 + kQ <= nq) {
      gmp_cyclic_batch<kQ>(buf, r, N, coef, K, M, L, q0, y);
    } else if (q0 < nq) {
      // short symbols: one sample at a time (thread t's samples t + 256 q below N only)
#pragma unroll
      for (int q = q0; q < q0 + kQ; ++q)
        if (q < nq && threadIdx.x + q * kFftThreads < N) gmp_cyclic_batch<1>(buf, r, N, coef, K, M, L, q, y);
    }
  }
}

// One workgroup per (symbol, antenna) row, persistent: x (precoded subcarriers) -> IDFT
// -> optional DPD -> PA -> DFT -> y_fd.  Both transforms unitary.  For 4096-point symbols
// the radix-16 passes run in registers; the PA's output samples (t + 256 m of thread t)
// are already the first pass's inputs.
__global__ __launch_bounds__(kFftThreads) void k_link_pa(const float2* __restrict__ x, int N, int log2n,
                                                         float scale, int B, int64_t rows,
                                                         const float2* __restrict__ dpd, int Kd, int Md, int Ld,
                                                         int Jd, const float2* __restrict__ pa, int Kp, int Mp,
                                                         int Lp, int Jp, float2* __restrict__ y_fd) {
  __shared__ float2 buf[kF16Row];
  __shared__ float2 tw[kFftMax / 2];
  __shared__ float r[kFftMax];
  fft_twiddles(tw, N);
  const int t = threadIdx.x;
  const bool f16 = N == kFftMax;
  for (int64_t row = blockIdx.x; row < rows; row += gridDim.x) {
    const int b = (int)(row % B);
    if (f16) {
      float2 v[16];
#pragma unroll
      for (int q = 0; q < 16; ++q) v[q] = conjf2(x[row * N + t + 256 * q]);
      __syncthreads();                     // the previous row is done with buf
      f16_pass1(buf, v);
      __syncthreads();
      f16_pass2(buf, tw);
      __syncthreads();
      f16_pass3(buf, tw, v);
      __syncthreads();                     // every last-pass read precedes the sample writes
#pragma unroll
      for (int q = 0; q < 16; ++q) {
        const float2 a = X16(v, q);
        const float2 u = make_float2(a.x * scale, -a.y * scale);
        buf[t + 256 * q] = u;
        r[t + 256 * q] = sqrtf(u.x * u.x + u.y * u.y);
      }
    } else {
      __syncthreads();
      for (int i = t; i < N; i += kFftThreads) buf[i] = x[row * N + i];
      __syncthreads();
      fft_lds<true>(buf, tw, N, log2n);
      for (int i = t; i < N; i += kFftThreads) {
        const float2 v = make_float2(buf[i].x * scale, buf[i].y * scale);
        buf[i] = v;
        r[i] = sqrtf(v.x * v.x + v.y * v.y);
      }
    }
    __syncthreads();
    float2 y[kFftMax / kFftThreads];
    if (dpd) {
      gmp_cyclic_lds(buf, r, N, dpd + (int64_t)b * Jd, Kd, Md, Ld, y);
      __syncthreads();
#pragma unroll
      for (int m = 0; m < kFftMax / kFftThreads; ++m) {
        const int n = t + m * kFftThreads;
        if (n < N) {
          buf[n] = y[m];
          r[n] = sqrtf(y[m].x * y[m].x + y[m].y * y[m].y);
        }
      }
      __syncthreads();
    }
    gmp_cyclic_lds(buf, r, N, pa + (int64_t)b * Jp, Kp, Mp, Lp, y);
    __syncthreads();                       // the GMP's neighbour reads precede the FFT writes
    if (f16) {
      f16_pass1(buf, y);                   // y[m] is sample t + 256 m
      __syncthreads();
      f16_pass2(buf, tw);
      __syncthreads();
      f16_pass3(buf, tw, y);
#pragma unroll
      for (int q = 0; q < 16; ++q) {
        const float2 a = X16(y, q);
        y_fd[row * N + t + 256 * q] = make_float2(a.x * scale, a.y * scale);
      }
    } else {
#pragma unroll
      for (int m = 0; m < kFftMax / kFftThreads; ++m) {
        const int n = t + m * kFftThreads;
        if (n < N) buf[n] = y[m];
      }
      __syncthreads();
      fft_lds<false>(buf, tw, N, log2n);
      for (int i = t; i < N; i += kFftThreads)
        y_fd[row * N + i] = make_float2(buf[i].x * scale, buf[i].y * scale);
    }
  }
}

// ---------------------------------------------------------------------------
// Reverse mode of the link (receiver-side training of the frequency-domain DPDs)
// ---------------------------------------------------------------------------
// Index of data symbol on subcarrier k, or -1 for a guard subcarrier.
__device__ __forceinline__ int data_index(int k, int N, int n_d) {
  const int h = n_d / 2;
  if (k >= 1 && k <= h) return k - 1;
  if (k >= N - h) return k - (N - n_d);
  return -1;
}

// g_y[i][b][k_d] = sum_u conj(H_k[u][b]) conj(1 / (alpha G)) g_r[i][u][d] for data symbol
// d (adjoint of channel and equalisation).  A workgroup holds kRxbD data symbols (fastest,
// so the g_y stores are contiguous) x 4 antenna groups, each thread the antennas b of its
// group; the guard subcarriers of g_y are zeroed beforehand by zero_complex.
constexpr int kRxbD = 64;

__global__ __launch_bounds__(256) void k_link_rx_bwd(const float2* __restrict__ hd, const float* __restrict__ alpha,
                                                     float g_re, float g_im, const float2* __restrict__ g_r, int N,
                                                     int n_d, int U, int B, int spc, float2* __restrict__ g_y) {
  const int d = blockIdx.x * kRxbD + threadIdx.x % kRxbD;
  const int bg = threadIdx.x / kRxbD;
  const int i = blockIdx.y;
  if (d >= n_d) return;
  const int k = data_bin(d, N, n_d);
  float2* gi = g_y + (int64_t)i * B * N + k;
  const int c = i / spc;
  // conj(1 / (alpha G)) = G / (alpha |G|^2)
  const float den = alpha[c] * (g_re * g_re + g_im * g_im);
  const float2 cj = make_float2(g_re / den, g_im / den);
  float2 gz[kZfMaxU];
#pragma unroll
  for (int u = 0; u < kZfMaxU; ++u)
    gz[u] = u < U ? cmul(cj, g_r[((int64_t)i * U + u) * n_d + d]) : make_float2(0.f, 0.f);
  const float2* hk = hd + ((int64_t)c * n_d + d) * U * B;   // hd[c][d][u][b]
  for (int b = bg; b < B; b += 256 / kRxbD) {
    float2 acc = make_float2(0.f, 0.f);
#pragma unroll
    for (int u = 0; u < kZfMaxU; ++u) {
      if (u < U) {
        const float2 h = hk[u * B + b];
        // conj(h) gz
        acc.x += h.x * gz[u].x + h.y * gz[u].y;
        acc.y += h.x * gz[u].y - h.y * gz[u].x;
      }
    }
    gi[(int64_t)b * N] = acc;
  }
}

// p[0, n) = 0 (grid-stride; V = float4 for 16-byte aligned buffers, else float2).
template <typename V>
__global__ __launch_bounds__(256) void k_zero(V* __restrict__ p, int64_t n) {
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < n; e += (int64_t)gridDim.x * 256) p[e] = V{};
}

// Zeroes n2 complex values (float2) at p: 16-byte stores when p is 16-byte aligned and n2 even.
static void zero_complex(float* p, int64_t n2, hipStream_t s) {
  if (n2 <= 0) return;
  if ((uintptr_t)p % 16 == 0 && n2 % 2 == 0) {
    const int64_t n4 = n2 / 2;
    k_zero<float4><<<(unsigned)std::min<int64_t>((n4 + 255) / 256, 8192), 256, 0, s>>>(reinterpret_cast<float4*>(p),
                                                                                       n4);
  } else {
    k_zero<float2><<<(unsigned)std::min<int64_t>((n2 + 255) / 256, 8192), 256, 0, s>>>(reinterpret_cast<float2*>(p),
                                                                                       n2);
  }
}

// Unitary IDFT of one global row into dst (LDS, natural order), through the scratch row.
// dst may alias scratch.  Ends with a barrier.
__device__ void row_idft(const float2* __restrict__ src, float2* scratch, const float2* tw, float2* dst, int N,
                         int log2n, float scale) {
  const int t = threadIdx.x;
  if (N == kFftMax) {
    float2 v[16];
#pragma unroll
    for (int q = 0; q < 16; ++q) v[q] = conjf2(src[t + 256 * q]);
    __syncthreads();
    f16_pass1(scratch, v);
    __syncthreads();
    f16_pass2(scratch, tw);
    __syncthreads();
    f16_pass3(scratch, tw, v);
    __syncthreads();
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      const float2 a = X16(v, q);
      dst[t + 256 * q] = make_float2(a.x * scale, -a.y * scale);
    }
  } else {
    __syncthreads();
    for (int i = t; i < N; i += kFftThreads) scratch[i] = src[i];
    __syncthreads();
    fft_lds<true>(scratch, tw, N, log2n);
    for (int i = t; i < N; i += kFftThreads) {
      const float2 v = scratch[i];
      dst[i] = make_float2(v.x * scale, v.y * scale);     // dst == scratch: same index
    }
  }
  __syncthreads();
}

// Cyclic GMP reverse mode, gather form, for samples m = t + 256 q (registers g[q]):
// g[m] = sum_l conj(Q_l(m)) gy[m + l]
//        + x[m] / |x[m]| sum over the monomials whose envelope sample is m of
//          k |x[m]|^(k-1) Re(conj(gy[n]) c x[n - l]),
// Q_l(p) = sum_k a_kl r[p]^k + sum_{g,k>=1} (b_klg r[p - g]^k + c_klg r[p + g]^k).
// Batches of Q samples with the coefficient loops outside (as gmp_cyclic_batch); N is a
// power of two.
template <int Q>
__device__ __forceinline__ void gmp_cyclic_bwd_batch(const float2* x, const float* r, const float2* gy, int N,
                                                     const float2* __restrict__ coef, int K, int M, int L, int q0,
                                                     float2 (&g)[kFftMax / kFftThreads]) {
  const int na = K * (M + 1), nb = (K - 1) * (M + 1) * L;
  const int sb = (M + 1) * L;                  // stride of k in the b / c blocks
  const int mask = N - 1;
  int nn[Q];
  float rm[Q], env[Q];
  float2 xm[Q], hol[Q];
#pragma unroll
  for (int j = 0; j < Q; ++j) {
    nn[j] = threadIdx.x + (q0 + j) * kFftThreads;
    rm[j] = r[nn[j]];
    xm[j] = x[nn[j]];
    hol[j] = make_float2(0.f, 0.f);
    env[j] = 0.f;
  }
  for (int l = 0; l <= M; ++l) {
    float2 gyl[Q], poly[Q], dpa[Q];
    const float2 top = coef[(K - 1) * (M + 1) + l];
#pragma unroll
    for (int j = 0; j < Q; ++j) {
      gyl[j] = gy[(nn[j] + l) & mask];
      poly[j] = top;
      dpa[j] = make_float2(0.f, 0.f);
    }
    // Q_l's a-part and its derivative in r[m], one pass over k
    for (int k = K - 1; k >= 0; --k) {
      const float2 a = coef[k * (M + 1) + l];
      const float fk = (float)k;
#pragma unroll
      for (int j = 0; j < Q; ++j) {
        if (k >= 1) dpa[j] = make_float2(fmaf(dpa[j].x, rm[j], fk * a.x), fmaf(dpa[j].y, rm[j], fk * a.y));
        if (k <= K - 2) poly[j] = make_float2(fmaf(poly[j].x, rm[j], a.x), fmaf(poly[j].y, rm[j], a.y));
      }
    }
    // envelope of the a-monomials at m: n = m + l, multiplied sample x[m]
#pragma unroll
    for (int j = 0; j < Q; ++j) {
      const float2 w = cmul(dpa[j], xm[j]);
      env[j] += gyl[j].x * w.x + gyl[j].y * w.y;     // Re(conj(gy) w)
    }
    for (int gg = 1; K > 1 && gg <= L; ++gg) {
      const int ib = na + l * L + (gg - 1), ic = ib + nb;
      const float2 tb = coef[ib + (K - 2) * sb], tc = coef[ic + (K - 2) * sb];
      const float fk1 = (float)(K - 1);
      float rb[Q], rc[Q];
      float2 pb[Q], pc[Q], db[Q], dc[Q];
#pragma unroll
      for (int j = 0; j < Q; ++j) {
        rb[j] = r[(nn[j] - gg) & mask];
        rc[j] = r[(nn[j] + gg) & mask];
        pb[j] = tb;
        pc[j] = tc;
        db[j] = make_float2(fk1 * tb.x, fk1 * tb.y);
        dc[j] = make_float2(fk1 * tc.x, fk1 * tc.y);
      }
      for (int k = K - 2; k >= 1; --k) {
        const float2 bb = coef[ib + (k - 1) * sb], cc = coef[ic + (k - 1) * sb];
        const float fk = (float)k;
#pragma unroll
        for (int j = 0; j < Q; ++j) {
          pb[j] = make_float2(fmaf(pb[j].x, rb[j], bb.x), fmaf(pb[j].y, rb[j], bb.y));
          pc[j] = make_float2(fmaf(pc[j].x, rc[j], cc.x), fmaf(pc[j].y, rc[j], cc.y));
          db[j] = make_float2(fmaf(db[j].x, rm[j], fk * bb.x), fmaf(db[j].y, rm[j], fk * bb.y));
          dc[j] = make_float2(fmaf(dc[j].x, rm[j], fk * cc.x), fmaf(dc[j].y, rm[j], fk * cc.y));
        }
      }
#pragma unroll
      for (int j = 0; j < Q; ++j) {
        poly[j] = make_float2(fmaf(pb[j].x, rb[j], fmaf(pc[j].x, rc[j], poly[j].x)),
                              fmaf(pb[j].y, rb[j], fmaf(pc[j].y, rc[j], poly[j].y)));
        // envelope sample m of b_{k,l,g}: n = m + l + g, multiplied sample x[m + g]
        const float2 gyb = gy[(nn[j] + l + gg) & mask];
        const float2 wb = cmul(db[j], x[(nn[j] + gg) & mask]);
        env[j] += gyb.x * wb.x + gyb.y * wb.y;
        // of c_{k,l,g}: n = m + l - g, multiplied sample x[m - g]
        const float2 gyc = gy[(nn[j] + l - gg) & mask];
        const float2 wc = cmul(dc[j], x[(nn[j] - gg) & mask]);
        env[j] += gyc.x * wc.x + gyc.y * wc.y;
      }
    }
    // conj(Q_l(m)) gy[m + l]
#pragma unroll
    for (int j = 0; j < Q; ++j) {
      hol[j].x += poly[j].x * gyl[j].x + poly[j].y * gyl[j].y;
      hol[j].y += poly[j].x * gyl[j].y - poly[j].y * gyl[j].x;
    }
  }
#pragma unroll
  for (int j = 0; j < Q; ++j) {
    const float2 unit = rm[j] > 0.f ? make_float2(xm[j].x / rm[j], xm[j].y / rm[j]) : make_float2(0.f, 0.f);
    g[q0 + j] = make_float2(fmaf(env[j], unit.x, hol[j].x), fmaf(env[j], unit.y, hol[j].y));
  }
}

__device__ void gmp_cyclic_bwd_lds(const float2* x, const float* r, const float2* gy, int N,
                                   const float2* __restrict__ coef, int K, int M, int L,
                                   float2 (&g)[kFftMax / kFftThreads]) {
  constexpr int kQ = 8;
  constexpr int kMaxQ = kFftMax / kFftThreads;
  const int nq = (N + kFftThreads - 1) / kFftThreads;
#pragma unroll
  for (int q0 = 0; q0 < kMaxQ; q0 += kQ) {
    if (q0 + kQ <= nq) {
      gmp_cyclic_bwd_batch<kQ>(x, r, gy, N, coef, K, M, L, q0, g);
    } else if (q0 < nq) {
#pragma unroll
      for (int q = q0; q < q0 + kQ; ++q)
        if (q < nq && threadIdx.x + q * kFftThreads < N) gmp_cyclic_bwd_batch<1>(x, r, gy, N, coef, K, M, L, q, g);
    }
  }
}

// One workgroup per (symbol, antenna) row, persistent: u = IDFT(x), gy = IDFT(g_y) (the
// adjoint of the DFT), g_u by the cyclic GMP reverse mode, g_x = DFT(g_u) (the adjoint of
// the IDFT).
__global__ __launch_bounds__(kFftThreads) void k_link_pa_bwd(const float2* __restrict__ x,
                                                             const float2* __restrict__ g_y, int N, int log2n,
                                                             float scale, int B, int64_t rows,
                                                             const float2* __restrict__ pa, int Kp, int Mp, int Lp,
                                                             int Jp, float2* __restrict__ g_x) {
  __shared__ float2 scratch[kF16Row];      // transforms; afterwards the gy row
  __shared__ float2 xs[kFftMax];
  __shared__ float2 tw[kFftMax / 2];
  __shared__ float r[kFftMax];
  fft_twiddles(tw, N);
  const int t = threadIdx.x;
  for (int64_t row = blockIdx.x; row < rows; row += gridDim.x) {
    const int b = (int)(row % B);
    row_idft(x + row * N, scratch, tw, xs, N, log2n, scale);
    for (int i = t; i < N; i += kFftThreads) r[i] = sqrtf(xs[i].x * xs[i].x + xs[i].y * xs[i].y);
    row_idft(g_y + row * N, scratch, tw, scratch, N, log2n, scale);
    float2 g[kFftMax / kFftThreads];
    gmp_cyclic_bwd_lds(xs, r, scratch, N, pa + (int64_t)b * Jp, Kp, Mp, Lp, g);
    __syncthreads();                       // gy (in scratch) and x are read before reuse
    if (N == kFftMax) {
      f16_pass1(scratch, g);
      __syncthreads();
      f16_pass2(scratch, tw);
      __syncthreads();
      f16_pass3(scratch, tw, g);
#pragma unroll
      for (int q = 0; q < 16; ++q) {
        const float2 a = X16(g, q);
        g_x[row * N + t + 256 * q] = make_float2(a.x * scale, a.y * scale);
      }
    } else {
#pragma unroll
      for (int q = 0; q < kFftMax / kFftThreads; ++q) {
        const int n = t + q * kFftThreads;
        if (n < N) scratch[n] = g[q];
      }
      __syncthreads();
      fft_lds<false>(scratch, tw, N, log2n);
      for (int i = t; i < N; i += kFftThreads)
        g_x[row * N + i] = make_float2(scratch[i].x * scale, scratch[i].y * scale);
    }
    __syncthreads();                       // this row is done with the LDS rows
  }
}

// g_s[i][u][k] = alpha_c sum_b conj(Pt[c][k][b][u]) g_x[i][b][k] on the precoded
// subcarriers, 0 elsewhere (adjoint of k_precode; the guard subcarriers are zeroed beforehand).
// Same tiling: the tile of g_x enters LDS with the subcarrier fastest, one thread per
// (subcarrier, UE) with the UE fastest accumulates over the antennas, the outputs leave through
// an LDS tile [U][tw+1].
__global__ __launch_bounds__(256) void k_precode_bwd(const float2* __restrict__ pt, const float* __restrict__ alpha,
                                                     const float2* __restrict__ g_x, int N, int n_d, int U, int B,
                                                     int spc, int all_bins, int tw, float2* __restrict__ g_s) {
  extern __shared__ float2 pc_lds[];
  const int XS = tw + 1;
  float2* gt = pc_lds;              // [B][tw + 1]
  float2* ot = pc_lds + B * XS;     // [kZfMaxU][tw + 1]
  const int i = blockIdx.y;
  const int c = i / spc;
  const int e0 = blockIdx.x * tw;
  const int nb = min(tw, (all_bins ? N : n_d) - e0);
  const float2* gi = g_x + (int64_t)i * B * N;
  for (int j = threadIdx.x; j < nb * B; j += 256) {
    const int b = j / nb, el = j - b * nb;
    gt[b * XS + el] = gi[(int64_t)b * N + (all_bins ? e0 + el : data_bin(e0 + el, N, n_d))];
  }
  __syncthreads();
  const float a = alpha[c];
  for (int j = threadIdx.x; j < nb * U; j += 256) {
    const int el = j / U, u = j - el * U;
    const int k = all_bins ? e0 + el : data_bin(e0 + el, N, n_d);
    const float2* col = pt + ((int64_t)c * N + k) * B * U + u;
    float2 acc = make_float2(0.f, 0.f);
#pragma unroll 8
    for (int b = 0; b < B; ++b) {
      const float2 p = col[(int64_t)b * U];
      const float2 v = gt[b * XS + el];
      acc.x += p.x * v.x + p.y * v.y;     // conj(p) v
      acc.y += p.x * v.y - p.y * v.x;
    }
    ot[u * XS + el] = make_float2(a * acc.x, a * acc.y);
  }
  __syncthreads();
  float2* gs = g_s + (int64_t)i * U * N;
  for (int j = threadIdx.x; j < nb * U; j += 256) {
    const int u = j / nb, el = j - u * nb;
    gs[(int64_t)u * N + (all_bins ? e0 + el : data_bin(e0 + el, N, n_d))] = ot[u * XS + el];
  }
}

// Receiver: thread per (symbol i, data symbol d, UE u): y = sum_b H_k[u][b] x_pa[b] + w,
// r = y / (alpha G), nearest QAM point; the workgroup's errors per UE into its partial.  A
// workgroup holds kRxD data symbols x kZfMaxU UE slots (UE fastest): eight times the threads
// of a thread-per-data-symbol receiver (which left most of the chip idle at 64 symbols), each
// thread summing one contiguous 256-byte row of H_k.
constexpr int kRxD = 256 / kZfMaxU;

__global__ __launch_bounds__(256) void k_link_rx(const float2* __restrict__ y_fd, const float2* __restrict__ hd,
                                                 const float* __restrict__ alpha, float g_re, float g_im,
                                                 const float2* __restrict__ noise, const int32_t* __restrict__ tx,
                                                 int N, int n_d, int U, int B, int spc, int qam_m,
                                                 float2* __restrict__ r_out, int32_t* __restrict__ err_part) {
  __shared__ int32_t cnt[256];
  const int dl = threadIdx.x / kZfMaxU, u = threadIdx.x % kZfMaxU;
  const int d = blockIdx.x * kRxD + dl;
  const int i = blockIdx.y;
  int e = 0;
  if (d < n_d && u < U) {
    const int c = i / spc;
    const int k = data_bin(d, N, n_d);
    const float2* hk = hd + (((int64_t)c * n_d + d) * U + u) * B;   // hd[c][d][u][b]
    const float2* yi = y_fd + (int64_t)i * B * N + k;
    float2 acc = make_float2(0.f, 0.f);
    for (int b = 0; b < B; ++b) acc = cadd(acc, cmul(hk[b], yi[(int64_t)b * N]));
    // 1 / (alpha G) = conj(G) / (alpha |G|^2)
    const float den = alpha[c] * (g_re * g_re + g_im * g_im);
    const float2 inv = make_float2(g_re / den, -g_im / den);
    const float qs = sqrtf(2.0f * (float)(qam_m * qam_m - 1) / 3.0f);   // unit-energy scale
    if (noise) acc = cadd(acc, noise[((int64_t)i * U + u) * N + k]);
    const float2 rv = cmul(acc, inv);
    if (r_out) r_out[((int64_t)i * U + u) * n_d + d] = rv;
    const int ire = min(max((int)floorf((rv.x * qs + (float)qam_m) * 0.5f), 0), qam_m - 1);
    const int iim = min(max((int)floorf((rv.y * qs + (float)qam_m) * 0.5f), 0), qam_m - 1);
    e = (ire * qam_m + iim) != tx[((int64_t)i * U + u) * n_d + d];
  }
  cnt[threadIdx.x] = e;
  __syncthreads();
  for (int w = kRxD / 2; w > 0; w >>= 1) {   // over the data symbols, per UE slot
    if (dl < w) cnt[threadIdx.x] += cnt[threadIdx.x + w * kZfMaxU];
    __syncthreads();
  }
  if (threadIdx.x < U)
    err_part[((int64_t)blockIdx.y * gridDim.x + blockIdx.x) * U + threadIdx.x] = cnt[threadIdx.x];
}

// errors[u] = sum over the partials in order (int64).
__global__ __launch_bounds__(256) void k_link_errors(const int32_t* __restrict__ part, int64_t n_part, int U,
                                                     int64_t* __restrict__ errors) {
  __shared__ long long red[256];
  for (int u = 0; u < U; ++u) {
    long long s = 0;
    for (int64_t p = threadIdx.x; p < n_part; p += 256) s += part[p * U + u];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
      if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
      __syncthreads();
    }
    if (threadIdx.x == 0) errors[u] = red[0];
    __syncthreads();
  }
}

int ilog2(int n) {
  int l = 0;
  while ((1 << l) < n) ++l;
  return l;
}

// mode 0: forward network; 1: backward kernel (partials); 2: reduction of the partials.
template <int FM, int DM, int NH>
void nn_launch(int mode, const NnDims& d, int64_t n_sym, const float2* td, const float2* g_td, const float* w,
               float2* o_td, float* part, float* dw, int cus, hipStream_t s) {
  const int F = 2 * d.users * (d.memory + 1);
  if (mode == 0) {
    const int tps = (d.n_fft + kNnFwdT - 1) / kNnFwdT;
    const int n_tiles = (int)(n_sym * tps);
    const int G = std::min(n_tiles, 4 * cus);
    k_fdnn_fwd<FM, DM, NH><<<G, kNnFwdT, 0, s>>>(td, w, o_td, d.n_fft, d.users, d.memory, d.hidden,
                                                  d.params, tps, n_tiles);
    return;
  }
  const int tps = (d.n_fft + kNnBwdT - 1) / kNnBwdT;
  const int n_tiles = (int)(n_sym * tps);
  const int G = std::min(n_tiles, fdnn_bwd_groups(cus));
  if (mode == 1) {
    k_fdnn_bwd<FM, DM, NH><<<G, kNnBwdT, 0, s>>>(td, g_td, w, part, d.n_fft, d.users, d.memory, d.hidden,
                                                  d.params, tps, n_tiles);
    return;
  }
  float* mid = part + (int64_t)kFdnnMaxGroups * d.part_floats;
  const int pb = (d.params + 255) / 256;
  k_fdnn_reduce1<FM, DM, NH><<<dim3(pb, kNnSplits), 256, 0, s>>>(part, G, F, d.hidden, d.users, d.params, mid);
  k_fdnn_reduce2<<<pb, 256, 0, s>>>(mid, d.params, dw);
}

template <int NH>
void nn_dispatch(int mode, const NnDims& d, int64_t n_sym, const float2* td, const float2* g_td, const float* w,
                 float2* o_td, float* part, float* dw, int cus, hipStream_t s) {
  const int F = 2 * d.users * (d.memory + 1);
  if (F <= 32) {
    if (d.hidden <= 16) nn_launch<32, 16, NH>(mode, d, n_sym, td, g_td, w, o_td, part, dw, cus, s);
    else nn_launch<32, 32, NH>(mode, d, n_sym, td, g_td, w, o_td, part, dw, cus, s);
  } else {
    if (d.hidden <= 16) nn_launch<64, 16, NH>(mode, d, n_sym, td, g_td, w, o_td, part, dw, cus, s);
    else nn_launch<64, 32, NH>(mode, d, n_sym, td, g_td, w, o_td, part, dw, cus, s);
  }
}

void nn_run(int mode, const NnDims& d, int64_t n_sym, const float* td, const float* g_td, const float* w,
            float* o_td, float* part, float* dw, int cus, hipStream_t s) {
  const float2* t2 = reinterpret_cast<const float2*>(td);
  const float2* g2 = reinterpret_cast<const float2*>(g_td);
  float2* o2 = reinterpret_cast<float2*>(o_td);
  if (d.n_hidden == 1) nn_dispatch<1>(mode, d, n_sym, t2, g2, w, o2, part, dw, cus, s);
  else nn_dispatch<2>(mode, d, n_sym, t2, g2, w, o2, part, dw, cus, s);
}

}  // namespace

NnDims nn_dims(int n_fft, int users, int memory, int hidden, int n_hidden) {
  NnDims d;
  d.n_fft = n_fft;
  d.users = users;
  d.memory = memory;
  d.hidden = hidden;
  d.n_hidden = n_hidden;
  const int F = 2 * users * (memory + 1);
  d.params = hidden * F + hidden + (n_hidden - 1) * (hidden * hidden + hidden) + 2 * users * hidden + 2 * users;
  // padded partial size of the widest instantiation; the reduction's split sums follow
  // the partials
  d.part_floats = 32 * 64 + 32 + 32 * 32 + 32 + kNnOut * 32 + kNnOut;
  d.mid_floats = kNnSplits * d.params;
  return d;
}

bool nn_supported(const NnDims& d) {
  const int F = 2 * d.users * (d.memory + 1);
  return fft_size_ok(d.n_fft) && d.users >= 1 && d.users <= 8 && d.memory >= 0 && d.memory <= kNnMaxMem &&
         F <= 64 && d.hidden >= 1 && d.hidden <= 32 && (d.n_hidden == 1 || d.n_hidden == 2);
}

// Backward grid: five workgroups (ten waves) per CU, as many as the LDS holds (30 KB
// each for the paper's network); each writes one partial.
int fdnn_bwd_groups(int cus) { return std::min(5 * cus, kFdnnMaxGroups); }

bool fft_size_ok(int n) { return n >= 2 && n <= kFftMax && (n & (n - 1)) == 0; }

void launch_fft(const float* in, float* out, int n, int64_t rows, bool inverse, int cus, hipStream_t s) {
  const int G = (int)std::min<int64_t>(rows, 4 * (int64_t)cus);
  const float scale = (float)(1.0 / sqrt((double)n));
  const float2* i2 = reinterpret_cast<const float2*>(in);
  float2* o2 = reinterpret_cast<float2*>(out);
  if (n == kFftMax) {
    if (inverse) k_fft4096<true><<<G, kFftThreads, 0, s>>>(i2, o2, scale, rows);
    else k_fft4096<false><<<G, kFftThreads, 0, s>>>(i2, o2, scale, rows);
    return;
  }
  if (inverse) k_fft<true><<<G, kFftThreads, 0, s>>>(i2, o2, n, ilog2(n), scale, rows);
  else k_fft<false><<<G, kFftThreads, 0, s>>>(i2, o2, n, ilog2(n), scale, rows);
}

void launch_fdnn_fwd(const NnDims& d, int64_t n_sym, const float* td, const float* w, float* o_td, int cus,
                     hipStream_t s) {
  nn_run(0, d, n_sym, td, nullptr, w, o_td, nullptr, nullptr, cus, s);
}

void launch_fdnn_bwd(const NnDims& d, int64_t n_sym, const float* td, const float* g_td, const float* w,
                     float* part, int cus, hipStream_t s) {
  nn_run(1, d, n_sym, td, g_td, w, nullptr, part, nullptr, cus, s);
}

void launch_fdnn_reduce(const NnDims& d, int64_t n_sym, float* part, float* dw, int cus, hipStream_t s) {
  nn_run(2, d, n_sym, nullptr, nullptr, nullptr, nullptr, part, dw, cus, s);
}

void launch_zf(const float* h_est, int N, int n_d, int all_bins, int U, int B, int T, int n_ch, float p_total,
               float* pt, double* trace, float* alpha, hipStream_t s) {
  const size_t lds = sizeof(double2) * (size_t)(T + U * (B + 1));
  const int nbins = all_bins ? N : n_d;
  k_zf<<<dim3(nbins, n_ch), 64, lds, s>>>(reinterpret_cast<const float2*>(h_est), N, n_d, all_bins, U, B, T,
                                           reinterpret_cast<float2*>(pt), trace);
  k_zf_alpha<<<n_ch, 256, 0, s>>>(trace, N, n_d, p_total, alpha);
}

void launch_precode(const float* pt, const float* alpha, const float* sym, int N, int n_d, int U, int B,
                    int n_sym, int spc, int all_bins, float* x, hipStream_t s) {
  if (!all_bins) zero_complex(x, (int64_t)n_sym * B * N, s);
  const int tw = precode_tile(B);
  const dim3 grid(((all_bins ? N : n_d) + tw - 1) / tw, n_sym);
  const size_t lds = sizeof(float2) * (size_t)(kZfMaxU * tw + B * (tw + 1));
  const auto* p2 = reinterpret_cast<const float2*>(pt);
  const auto* s2 = reinterpret_cast<const float2*>(sym);
  auto* x2 = reinterpret_cast<float2*>(x);
  if (U % 2 == 0 && (uintptr_t)pt % 16 == 0)
    k_precode<true><<<grid, 256, lds, s>>>(p2, alpha, s2, N, n_d, U, B, spc, all_bins, tw, x2);
  else
    k_precode<false><<<grid, 256, lds, s>>>(p2, alpha, s2, N, n_d, U, B, spc, all_bins, tw, x2);
}

void launch_chan_data(const float* h, int N, int n_d, int U, int B, int T, int n_ch, float* hd, hipStream_t s) {
  k_chan_data<<<dim3(n_d, n_ch), 256, 0, s>>>(reinterpret_cast<const float2*>(h), N, n_d, U, B, T,
                                               reinterpret_cast<float2*>(hd));
}

void launch_link_pa(const float* x, int N, int B, int64_t rows, const float* dpd, const dpd_gmp_desc* dd,
                    const float* pa, const dpd_gmp_desc& pd, float* y_fd, int cus, hipStream_t s) {
  const int G = (int)std::min<int64_t>(rows, 2 * (int64_t)cus);
  const float scale = (float)(1.0 / sqrt((double)N));
  const int Jp = pd.K * (pd.M + 1) + 2 * (pd.K - 1) * (pd.M + 1) * pd.L;
  const int Jd = dd ? dd->K * (dd->M + 1) + 2 * (dd->K - 1) * (dd->M + 1) * dd->L : 0;
  k_link_pa<<<G, kFftThreads, 0, s>>>(reinterpret_cast<const float2*>(x), N, ilog2(N), scale, B, rows,
                                      reinterpret_cast<const float2*>(dpd), dd ? dd->K : 0, dd ? dd->M : 0,
                                      dd ? dd->L : 0, Jd, reinterpret_cast<const float2*>(pa), pd.K, pd.M, pd.L,
                                      Jp, reinterpret_cast<float2*>(y_fd));
}

void launch_link_rx_bwd(const float* hd, const float* alpha, float g_re, float g_im, const float* g_r, int N, int n_d,
                        int U, int B, int n_sym, int spc, float* g_y, hipStream_t s) {
  zero_complex(g_y, (int64_t)n_sym * B * N, s);
  k_link_rx_bwd<<<dim3((n_d + kRxbD - 1) / kRxbD, n_sym), 256, 0, s>>>(reinterpret_cast<const float2*>(hd), alpha, g_re,
                                                               g_im, reinterpret_cast<const float2*>(g_r), N, n_d, U,
                                                               B, spc, reinterpret_cast<float2*>(g_y));
}

void launch_link_pa_bwd(const float* x, const float* g_y, int N, int B, int n_sym, const float* pa,
                        const dpd_gmp_desc& pd, float* g_x, int cus, hipStream_t s) {
  const int64_t rows = (int64_t)n_sym * B;
  const int G = (int)std::min<int64_t>(rows, 2 * (int64_t)cus);
  const float scale = (float)(1.0 / sqrt((double)N));
  const int Jp = pd.K * (pd.M + 1) + 2 * (pd.K - 1) * (pd.M + 1) * pd.L;
  k_link_pa_bwd<<<G, kFftThreads, 0, s>>>(reinterpret_cast<const float2*>(x), reinterpret_cast<const float2*>(g_y), N,
                                          ilog2(N), scale, B, rows, reinterpret_cast<const float2*>(pa), pd.K, pd.M,
                                          pd.L, Jp, reinterpret_cast<float2*>(g_x));
}

void launch_precode_bwd(const float* pt, const float* alpha, const float* g_x, int N, int n_d, int U, int B,
                        int n_sym, int spc, int all_bins, float* g_s, hipStream_t s) {
  if (!all_bins) zero_complex(g_s, (int64_t)n_sym * U * N, s);
  const int tw = precode_tile(B);
  const dim3 grid(((all_bins ? N : n_d) + tw - 1) / tw, n_sym);
  const size_t lds = sizeof(float2) * (size_t)((B + kZfMaxU) * (tw + 1));
  k_precode_bwd<<<grid, 256, lds, s>>>(reinterpret_cast<const float2*>(pt), alpha, reinterpret_cast<const float2*>(g_x),
                                       N, n_d, U, B, spc, all_bins, tw, reinterpret_cast<float2*>(g_s));
}

int64_t link_rx_parts(int n_d, int n_sym) { return (int64_t)((n_d + kRxD - 1) / kRxD) * n_sym; }

void launch_link_rx(const float* y_fd, const float* hd, const float* alpha, float g_re, float g_im,
                    const float* noise, const int32_t* tx, int N, int n_d, int U, int B, int n_sym, int spc,
                    int qam_m, float* r_out, int32_t* err_part, int64_t* errors, hipStream_t s) {
  k_link_rx<<<dim3((n_d + kRxD - 1) / kRxD, n_sym), 256, 0, s>>>(
      reinterpret_cast<const float2*>(y_fd), reinterpret_cast<const float2*>(hd), alpha, g_re, g_im,
      reinterpret_cast<const float2*>(noise), tx, N, n_d, U, B, spc, qam_m, reinterpret_cast<float2*>(r_out),
      err_part);
  k_link_errors<<<1, 256, 0, s>>>(err_part, link_rx_parts(n_d, n_sym), U, errors);
}

}  // namespace dpdmi
