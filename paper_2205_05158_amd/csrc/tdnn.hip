// Tuned TDNN DPD kernels for gfx950: the dense layers of the tapped-delay-line
// network (Sec. III-C core, eq. (8) slot) on MFMA, plus the fused
// direct-learning backward (Sec. V-A-2) through the GMP PA (eq. (9)).
//
// Formulation.  A layer h_i = tanh(W_i h_{i-1} + b_i) over 32 samples is computed
// transposed, h_i^T = W_i h_{i-1}^T, with the weights as the MFMA A operand
// (rows = output neurons) and the activations as the B operand (columns = samples).
// In the 32x32 accumulator layout a lane owns one sample column and 16 neuron rows
// rho(j, h); those rows are exactly a B-operand K-slice of the next layer once the
// next layer's weights are permuted the same way.  So activations never leave the
// registers between layers; the pack kernel writes every weight matrix in that
// per-lane operand order (one 16-byte bf16 or 4-byte fp32 load per lane per MFMA).
// The backward chain delta_{i-1}^T = W_i^T delta_i^T uses the same trick with a
// second, transposed pack.  dW_i = sum_s delta_i[s] h_{i-1}[s]^T contracts over
// samples, so delta and h are staged through LDS (rows = neurons, columns =
// samples) and each wave accumulates its share of 32x32 dW blocks over the
// workgroup's 128 samples into a per-(workgroup, stream) slot in global memory.
#include <algorithm>

#include "gmp.hpp"
#include "kernels.hpp"

namespace dpdmi {

namespace {

constexpr int kThreads = 256;        // 4 waves
constexpr int kTile = 128;           // samples per workgroup tile (32 per wave)

template <int PREC> struct Prec;
template <> struct Prec<DPD_BF16> {
  static constexpr int KS = 16;      // MFMA K per instruction
  using A = bf16x8;                  // one lane's A/B operand
  using E = __bf16;                  // LDS staging element
};
template <> struct Prec<DPD_FP32> {
  static constexpr int KS = 2;
  using A = float;
  using E = float;
};

constexpr int cmax(int a, int b) { return a > b ? a : b; }

template <int PREC, int T, int H, int NL>
struct Cfg {
  using P = Prec<PREC>;
  using A = typename P::A;
  using E = typename P::E;
  static constexpr int KS = P::KS;
  static constexpr int KIN = 5 * T;
  static constexpr int KIN_P = round_up(KIN, KS);
  static constexpr int NKS1 = KIN_P / KS;
  static constexpr int HP = round_up(H, 32);
  static constexpr int NB = HP / 32;
  static constexpr int NKSH = HP / KS;
  static constexpr int C1 = round_up(KIN_P, 32);     // dW columns of layer 1
  static constexpr int NN1 = C1 / 32;
  // packed parameter set (bytes)
  static constexpr int64_t ES = sizeof(A);
  static constexpr int64_t OFF_FWD1 = 0;
  static constexpr int64_t OFF_FWDH = OFF_FWD1 + (int64_t)NB * NKS1 * 64 * ES;
  static constexpr int64_t OFF_BWDH = OFF_FWDH + (int64_t)(NL - 1) * NB * NKSH * 64 * ES;
  static constexpr int64_t OFF_VEC = OFF_BWDH + (int64_t)(NL - 1) * NB * NKSH * 64 * ES;
  // float vector block: bias [NL][NB][2][16], wo [2][NB][2][16], bo[2] (+2 pad)
  static constexpr int NVEC = NL * HP + 2 * HP + 4;
  static constexpr int64_t PACK = OFF_VEC + (int64_t)NVEC * 4;
  // natural dW slot (floats): per layer W block [rows][cols] then bias [rows]
  static constexpr int64_t DW_L1 = (int64_t)HP * C1 + HP;
  static constexpr int64_t DW_H = (int64_t)HP * HP + HP;
  static constexpr int64_t DW_O = 32LL * HP + 32;
  static constexpr int64_t SLOT = DW_L1 + (NL - 1) * DW_H + DW_O;
  __host__ __device__ static constexpr int64_t dw_off(int li) {   // li = 0..NL (NL = output)
    return li == 0 ? 0 : DW_L1 + (int64_t)(li - 1) * DW_H;
  }
};

// Supported TDNN shapes of the tuned kernels.
template <class F>
bool tdnn_dispatch(int prec, int T, int H, int NL, F&& f) {
#define DPD_CASE(P_, T_, H_, NL_) \
  if (prec == P_ && T == T_ && H == H_ && NL == NL_) { f.template operator()<P_, T_, H_, NL_>(); return true; }
  DPD_CASE(DPD_FP32, 4, 20, 2)
  DPD_CASE(DPD_FP32, 10, 64, 3)
  DPD_CASE(DPD_FP32, 16, 128, 4)
  DPD_CASE(DPD_BF16, 4, 20, 2)
  DPD_CASE(DPD_BF16, 10, 64, 3)
  DPD_CASE(DPD_BF16, 16, 128, 4)
#undef DPD_CASE
  return false;
}

// (TDNN, GMP) pairs the fused backward kernel is built for.
template <class F>
bool bwd_dispatch(int prec, int T, int H, int NL, int K, int M, int L, F&& f) {
#define DPD_CASE(P_, T_, H_, NL_, K_, M_, L_)                                                  \
  if (prec == P_ && T == T_ && H == H_ && NL == NL_ && K == K_ && M == M_ && L == L_) {         \
    f.template operator()<P_, T_, H_, NL_, K_, M_, L_>();                                      \
    return true;                                                                               \
  }
  DPD_CASE(DPD_FP32, 4, 20, 2, 5, 3, 2)
  DPD_CASE(DPD_FP32, 10, 64, 3, 7, 5, 3)
  DPD_CASE(DPD_FP32, 16, 128, 4, 9, 7, 4)
  DPD_CASE(DPD_BF16, 4, 20, 2, 5, 3, 2)
  DPD_CASE(DPD_BF16, 10, 64, 3, 7, 5, 3)
  DPD_CASE(DPD_BF16, 16, 128, 4, 9, 7, 4)
#undef DPD_CASE
  return false;
}

// ------------------------------------------------------------------ pack
// Source offsets inside the packed float32 weight vector.
struct SrcOff {
  int64_t w[DPD_MAX_LAYERS + 1], b[DPD_MAX_LAYERS + 1];
};

template <int PREC, int T, int H, int NL>
__global__ void k_pack(const float* __restrict__ w, int64_t w_stride, SrcOff so,
                       char* __restrict__ pack) {
  using C = Cfg<PREC, T, H, NL>;
  const int set = blockIdx.y;
  const float* ws = w + set * w_stride;
  char* ps = pack + set * C::PACK;
  const int64_t n1 = (int64_t)C::NB * C::NKS1 * 64;
  const int64_t nh = (int64_t)(NL - 1) * C::NB * C::NKSH * 64;
  const int64_t total = n1 + 2 * nh + C::NVEC;
  constexpr int EPL = PREC == DPD_BF16 ? 8 : 1;   // values per lane entry
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * blockDim.x) {
    float v[EPL];
    int64_t e = idx;
    if (e < n1 + 2 * nh) {
      int lane = (int)(e % 64);
      int rowl = lane % 32, h = lane / 32;
      int64_t q = e / 64;
      int sec, layer = 0, mb, ks;
      if (e < n1) {
        sec = 0; mb = (int)(q / C::NKS1); ks = (int)(q % C::NKS1);
      } else {
        int64_t r = e < n1 + nh ? (e - n1) / 64 : (e - n1 - nh) / 64;
        sec = e < n1 + nh ? 1 : 2;
        layer = (int)(r / ((int64_t)C::NB * C::NKSH)) + 2;   // layer index i = 2..NL
        int64_t rr = r % ((int64_t)C::NB * C::NKSH);
        mb = (int)(rr / C::NKSH); ks = (int)(rr % C::NKSH);
      }
      for (int ee = 0; ee < EPL; ++ee) {
        float val = 0.f;
        if (sec == 0) {
          int o = 32 * mb + rowl;
          int k = PREC == DPD_BF16 ? 16 * ks + 8 * h + ee : 2 * ks + h;
          if (o < H && k < C::KIN) val = ws[so.w[0] + (int64_t)o * C::KIN + k];
        } else {
          // K index of a hidden-layer input in accumulator-row order
          int kk = PREC == DPD_BF16 ? 32 * (ks / 2) + mfma_row(8 * (ks % 2) + ee, h)
                                    : 32 * (ks / 16) + mfma_row(ks % 16, h);
          int m = 32 * mb + rowl;
          const float* Wi = ws + so.w[layer - 1];          // W_i is [H][H]
          if (sec == 1) {        // forward: A[o = m][k = kk]
            if (m < H && kk < H) val = Wi[(int64_t)m * H + kk];
          } else {               // backward: A[i = m][o = kk] = W_i[o][i]
            if (m < H && kk < H) val = Wi[(int64_t)kk * H + m];
          }
        }
        v[ee] = val;
      }
      if constexpr (PREC == DPD_BF16) {
        bf16x8 a;
        for (int ee = 0; ee < 8; ++ee) a[ee] = (__bf16)v[ee];
        reinterpret_cast<bf16x8*>(ps)[e] = a;
      } else {
        reinterpret_cast<float*>(ps)[e] = v[0];
      }
    } else {
      int f = (int)(e - n1 - 2 * nh);
      float val = 0.f;
      if (f < NL * C::HP) {                  // bias [i][mb][h][j]
        int i = f / C::HP, r = f % C::HP;
        int mb = r / 32, h = (r % 32) / 16, j = r % 16;
        int o = 32 * mb + mfma_row(j, h);
        if (o < H) val = ws[so.b[i] + o];
      } else if (f < NL * C::HP + 2 * C::HP) {   // wo [c][mb][h][j]
        int r0 = f - NL * C::HP;
        int c = r0 / C::HP, r = r0 % C::HP;
        int mb = r / 32, h = (r % 32) / 16, j = r % 16;
        int o = 32 * mb + mfma_row(j, h);
        if (o < H) val = ws[so.w[NL] + (int64_t)c * H + o];
      } else {
        int c = f - NL * C::HP - 2 * C::HP;
        if (c < 2) val = ws[so.b[NL] + c];
      }
      reinterpret_cast<float*>(ps + C::OFF_VEC)[f] = val;
    }
  }
}

// ------------------------------------------------------------------ MLP pieces
// Per-lane state of one wave's 32-sample block.
template <class C>
struct Acts {
  typename C::A feat[C::NKS1];                   // layer-1 B operands (features)
  typename C::A hb[C::NB][C::KS == 16 ? 2 : 16]; // B operands of layer i+1 (= h_i), per layer below
};

// Features of the lane's sample: xw points at x[n] in an LDS window (xw[-t] = x[n-t]).
template <class C>
__device__ __forceinline__ void make_features(const float2* xw, int h, typename C::A (&feat)[C::NKS1]) {
  float f[C::KIN_P];
#pragma unroll
  for (int t = 0; t < C::KIN / 5; ++t) {
    float2 z = xw[-t];
    float m2 = z.x * z.x + z.y * z.y;
    float m = sqrtf(m2);
    f[5 * t + 0] = z.x;
    f[5 * t + 1] = z.y;
    f[5 * t + 2] = m;
    f[5 * t + 3] = m2;
    f[5 * t + 4] = m2 * m;
  }
#pragma unroll
  for (int k = C::KIN; k < C::KIN_P; ++k) f[k] = 0.f;
#pragma unroll
  for (int ks = 0; ks < C::NKS1; ++ks) {
    if constexpr (C::KS == 16) {
      bf16x8 a;
#pragma unroll
      for (int e = 0; e < 8; ++e) a[e] = (__bf16)(h ? f[16 * ks + 8 + e] : f[16 * ks + e]);
      feat[ks] = a;
    } else {
      feat[ks] = h ? f[2 * ks + 1] : f[2 * ks];
    }
  }
}

// B operand of K step ks of a hidden layer from the previous layer's per-lane values.
template <class C>
__device__ __forceinline__ typename C::A b_operand(const typename C::A (&hb)[C::NB][C::KS == 16 ? 2 : 16], int ks) {
  if constexpr (C::KS == 16) return hb[ks / 2][ks % 2];
  else return hb[ks / 16][ks % 16];
}

// Store fp32 accumulator-layout values v[mb][j] as B operands.
template <class C>
__device__ __forceinline__ void to_operands(const float (&v)[C::NB][16], typename C::A (&hb)[C::NB][C::KS == 16 ? 2 : 16]) {
#pragma unroll
  for (int mb = 0; mb < C::NB; ++mb) {
    if constexpr (C::KS == 16) {
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        bf16x8 a;
#pragma unroll
        for (int e = 0; e < 8; ++e) a[e] = (__bf16)v[mb][8 * q + e];
        hb[mb][q] = a;
      }
    } else {
#pragma unroll
      for (int j = 0; j < 16; ++j) hb[mb][j] = v[mb][j];
    }
  }
}

template <class C>
__device__ __forceinline__ float operand_value(const typename C::A (&hb)[C::NB][C::KS == 16 ? 2 : 16], int mb, int j) {
  if constexpr (C::KS == 16) return (float)hb[mb][j / 8][j % 8];
  else return hb[mb][j];
}

template <class C>
__device__ __forceinline__ f32x16 mfma(typename C::A a, typename C::A b, f32x16 c) {
  if constexpr (C::KS == 16) return mfma_bf16(a, b, c);
  else return mfma_f32(a, b, c);
}

// One dense layer: acc[mb] = sum_ks A(mb, ks) B(ks).  Apk: packed [NB][nks][64].
template <class C, int NKS, class BF>
__device__ __forceinline__ void dense(const typename C::A* __restrict__ Apk, int lane, BF&& bop,
                                      f32x16 (&acc)[C::NB]) {
#pragma unroll
  for (int mb = 0; mb < C::NB; ++mb)
#pragma unroll
    for (int j = 0; j < 16; ++j) acc[mb][j] = 0.f;
#pragma unroll
  for (int ks = 0; ks < NKS; ++ks) {
    typename C::A b = bop(ks);
#pragma unroll
    for (int mb = 0; mb < C::NB; ++mb) {
      typename C::A a = Apk[((int64_t)mb * NKS + ks) * 64 + lane];
      acc[mb] = mfma<C>(a, b, acc[mb]);
    }
  }
}

// Forward through all hidden layers; keeps every layer's operands in `st` and the
// last layer's fp32 values in `last`.  vec: LDS copy of the float vector block.
template <class C, int NL>
__device__ __forceinline__ void mlp_forward(const char* __restrict__ pk, const float* vec, int lane,
                                            int h, const float2* xw,
                                            typename C::A (&feat)[C::NKS1],
                                            typename C::A (&hb)[NL][C::NB][C::KS == 16 ? 2 : 16],
                                            float (&last)[C::NB][16]) {
  make_features<C>(xw, h, feat);
  f32x16 acc[C::NB];
  const typename C::A* A1 = reinterpret_cast<const typename C::A*>(pk + C::OFF_FWD1);
  dense<C, C::NKS1>(A1, lane, [&](int ks) { return feat[ks]; }, acc);
#pragma unroll
  for (int i = 0; i < NL; ++i) {
    if (i > 0) {
      const typename C::A* Ah =
          reinterpret_cast<const typename C::A*>(pk + C::OFF_FWDH) + (int64_t)(i - 1) * C::NB * C::NKSH * 64;
      dense<C, C::NKSH>(Ah, lane, [&](int ks) { return b_operand<C>(hb[i - 1], ks); }, acc);
    }
    float v[C::NB][16];
#pragma unroll
    for (int mb = 0; mb < C::NB; ++mb) {
      const float* bias = vec + (i * C::NB + mb) * 32 + h * 16;
#pragma unroll
      for (int j = 0; j < 16; ++j) v[mb][j] = tanh_f32(acc[mb][j] + bias[j]);
    }
    to_operands<C>(v, hb[i]);
    if (i == NL - 1) {
#pragma unroll
      for (int mb = 0; mb < C::NB; ++mb)
#pragma unroll
        for (int j = 0; j < 16; ++j) last[mb][j] = v[mb][j];
    }
  }
}

template <class C>
__device__ __forceinline__ float2 output_layer(const float* vec, int h, const float (&last)[C::NB][16], int nl) {
  const float* wo = vec + nl * C::HP;
  float o0 = 0.f, o1 = 0.f;
#pragma unroll
  for (int mb = 0; mb < C::NB; ++mb)
#pragma unroll
    for (int j = 0; j < 16; ++j) {
      o0 = fmaf(wo[(0 * C::NB + mb) * 32 + h * 16 + j], last[mb][j], o0);
      o1 = fmaf(wo[(1 * C::NB + mb) * 32 + h * 16 + j], last[mb][j], o1);
    }
  o0 += __shfl_xor(o0, 32);
  o1 += __shfl_xor(o1, 32);
  const float* bo = vec + nl * C::HP + 2 * C::HP;
  return make_float2(o0 + bo[0], o1 + bo[1]);
}

// ------------------------------------------------------------------ forward kernel
template <int PREC, int T, int H, int NL>
__global__ __launch_bounds__(kThreads) void k_tdnn_fwd(StreamTable st, const float* __restrict__ x,
                                                       const char* __restrict__ pack, int residual,
                                                       float* __restrict__ u) {
  using C = Cfg<PREC, T, H, NL>;
  constexpr int XW = kTile + T - 1;
  __shared__ float2 xw[XW];
  __shared__ float vec[C::NVEC];
  const int lane = threadIdx.x % 64, wave = threadIdx.x / 64, h = lane / 32, sl = lane % 32;
  int cur_set = -1;
  for (int t = blockIdx.x; t < st.n_tiles; t += gridDim.x) {
    int s = stream_of_tile(st, t);
    int set = st.per_stream ? s : 0;
    int64_t lo = st.off[s], hi = st.off[s + 1];
    int64_t t0 = lo + (int64_t)(t - st.tile0[s]) * kTile;
    const char* pk = pack + set * C::PACK;
    __syncthreads();   // previous tile done with the LDS windows
    if (set != cur_set) {
      const float* src = reinterpret_cast<const float*>(pk + C::OFF_VEC);
      for (int i = threadIdx.x; i < C::NVEC; i += kThreads) vec[i] = src[i];
      cur_set = set;
    }
    for (int i = threadIdx.x; i < XW; i += kThreads) {
      int64_t p = t0 - (T - 1) + i;
      xw[i] = (p >= lo && p < hi) ? ld2(x, p) : make_float2(0.f, 0.f);
    }
    __syncthreads();
    typename C::A feat[C::NKS1];
    typename C::A hb[NL][C::NB][C::KS == 16 ? 2 : 16];
    float last[C::NB][16];
    int col = 32 * wave + sl;
    mlp_forward<C, NL>(pk, vec, lane, h, &xw[col + T - 1], feat, hb, last);
    float2 o = output_layer<C>(vec, h, last, NL);
    int64_t n = t0 + col;
    if (h == 0 && n < hi) {
      if (residual) {
        float2 xv = xw[col + T - 1];
        o.x += xv.x;
        o.y += xv.y;
      }
      st2(u, n, o);
    }
  }
}

// ------------------------------------------------------------------ backward kernel
template <int PREC, int T, int H, int NL, int K, int M, int L>
struct BwdLds {
  using C = Cfg<PREC, T, H, NL>;
  using G = Gmp<K, M, L>;
  static constexpr int S = kTile;
  static constexpr int XB = cmax(T - 1, L);
  static constexpr int XW = S + XB + M + L;       // x  [t0 - XB, t0 + S + M + L)
  static constexpr int UB = M + 2 * L;
  static constexpr int UW = S + 2 * UB;           // u  [t0 - UB, t0 + S + UB)
  static constexpr int QB = M + L;
  static constexpr int QW = S + 2 * QB;           // Q  [t0 - QB, t0 + S + QB)
  static constexpr int YW = S + M + 2 * L;        // gy [t0 - L, t0 + S + M + L)
  static constexpr int LD = S + (PREC == DPD_BF16 ? 8 : 4);   // staging row stride (elements)
  static constexpr int HROWS = cmax(C::C1, C::HP);
  // union: GMP phase vs. dW staging
  static constexpr int GMP_BYTES = (2 * G::J + QW * (M + 1) + YW) * 8;
  static constexpr int STAGE_BYTES = (C::HP + HROWS) * LD * (int)sizeof(typename C::E);
  static constexpr int UNION_BYTES = cmax(GMP_BYTES, STAGE_BYTES);
};

template <class C>
__device__ __forceinline__ void stage_acc_rows(typename C::E* stage, int ld, int col, int h,
                                               const float (&v)[C::NB][16]) {
#pragma unroll
  for (int mb = 0; mb < C::NB; ++mb)
#pragma unroll
    for (int j = 0; j < 16; ++j) stage[(32 * mb + mfma_row(j, h)) * ld + col] = (typename C::E)v[mb][j];
}

// dW blocks of one layer: rows = NMB*32 (delta staging), cols = NNB*32 (h staging).
// Accumulates into the slot's W block [rows][cols] and bias [rows] (bias from the
// row sums of delta).  Blocks are dealt to the waves round-robin.
template <class C, int NMB, int NNB>
__device__ __forceinline__ void dw_layer(const typename C::E* dst, const typename C::E* hst, int ld,
                                         int wave, int lane, float* __restrict__ slotW,
                                         float* __restrict__ slotB, bool first) {
  const int h = lane / 32, r = lane % 32;
  constexpr int NSTEP = kTile / C::KS;
  for (int bi = wave; bi < NMB * NNB; bi += kThreads / 64) {
    const int mb = bi / NNB, nb = bi % NNB;
    f32x16 acc;
    float* out = slotW + (int64_t)(32 * mb) * (NNB * 32) + 32 * nb + r;
#pragma unroll
    for (int j = 0; j < 16; ++j) acc[j] = first ? 0.f : out[(int64_t)mfma_row(j, h) * (NNB * 32)];
    const typename C::E* arow = dst + (32 * mb + r) * ld;
    const typename C::E* brow = hst + (32 * nb + r) * ld;
#pragma unroll 8
    for (int ks = 0; ks < NSTEP; ++ks) {
      typename C::A a, b;
      if constexpr (C::KS == 16) {
        a = *reinterpret_cast<const bf16x8*>(arow + 16 * ks + 8 * h);
        b = *reinterpret_cast<const bf16x8*>(brow + 16 * ks + 8 * h);
      } else {
        a = arow[2 * ks + h];
        b = brow[2 * ks + h];
      }
      acc = mfma<C>(a, b, acc);
    }
#pragma unroll
    for (int j = 0; j < 16; ++j) out[(int64_t)mfma_row(j, h) * (NNB * 32)] = acc[j];
    if (nb == 0) {
      // bias gradient: row sums of delta over the tile's samples
      float sum = 0.f;
      for (int c = h * (kTile / 2); c < (h + 1) * (kTile / 2); ++c) sum += (float)arow[c];
      sum += __shfl_xor(sum, 32);
      if (h == 0) {
        float* bo = slotB + 32 * mb + r;
        *bo = first ? sum : *bo + sum;
      }
    }
  }
}

template <int PREC, int T, int H, int NL, int K, int M, int L>
__global__ __launch_bounds__(kThreads) void k_tdnn_bwd(StreamTable st, const float* __restrict__ x,
                                                       const float* __restrict__ u,
                                                       const float* __restrict__ coef, float g_re,
                                                       float g_im, const char* __restrict__ pack,
                                                       float2* __restrict__ tile_part,
                                                       float* __restrict__ slots) {
  using C = Cfg<PREC, T, H, NL>;
  using G = Gmp<K, M, L>;
  using B = BwdLds<PREC, T, H, NL, K, M, L>;
  using E = typename C::E;
  constexpr int S = kTile;
  __shared__ float2 xw[B::XW];
  __shared__ float2 uw[B::UW];
  __shared__ float rw[B::UW];
  __shared__ float2 guw[S];
  __shared__ float vec[C::NVEC];
  __shared__ float red[4 * kThreads];
  __shared__ __attribute__((aligned(16))) char un[B::UNION_BYTES];
  float2* cf = reinterpret_cast<float2*>(un);
  float2* dcf = cf + G::J;
  float2(*qw)[M + 1] = reinterpret_cast<float2(*)[M + 1]>(dcf + G::J);
  float2* gyw = reinterpret_cast<float2*>(qw + B::QW);
  E* dst = reinterpret_cast<E*>(un);
  E* hst = dst + C::HP * B::LD;

  const int tid = threadIdx.x, lane = tid % 64, wave = tid / 64, h = lane / 32, sl = lane % 32;
  const int g_wg = blockIdx.x, G_wg = gridDim.x;
  const int t_begin = wg_tile_start(g_wg, G_wg, st.n_tiles);
  const int t_end = wg_tile_start(g_wg + 1, G_wg, st.n_tiles);
  int prev_stream = -1;
  for (int t = t_begin; t < t_end; ++t) {
    const int s = stream_of_tile(st, t);
    const int set = st.per_stream ? s : 0;
    const bool first = s != prev_stream;
    prev_stream = s;
    const int64_t lo = st.off[s], hi = st.off[s + 1];
    const int64_t t0 = lo + (int64_t)(t - st.tile0[s]) * S;
    const char* pk = pack + set * C::PACK;
    const float* cs = coef + (st.per_stream ? (int64_t)s * 2 * G::J : 0);
    float* slot = slots + (int64_t)(g_wg + s) * C::SLOT;

    __syncthreads();   // previous tile finished with every LDS buffer
    for (int j = tid; j < G::J; j += kThreads) {
      float2 c = make_float2(cs[2 * j], cs[2 * j + 1]);
      cf[j] = c;
      float k = (float)G::order(j);
      dcf[j] = make_float2(k * c.x, k * c.y);
    }
    {
      const float* src = reinterpret_cast<const float*>(pk + C::OFF_VEC);
      for (int i = tid; i < C::NVEC; i += kThreads) vec[i] = src[i];
    }
    for (int i = tid; i < B::XW; i += kThreads) {
      int64_t p = t0 - B::XB + i;
      xw[i] = (p >= lo && p < hi) ? ld2(x, p) : make_float2(0.f, 0.f);
    }
    for (int i = tid; i < B::UW; i += kThreads) {
      int64_t p = t0 - B::UB + i;
      float2 v = (p >= lo && p < hi) ? ld2(u, p) : make_float2(0.f, 0.f);
      uw[i] = v;
      rw[i] = sqrtf(v.x * v.x + v.y * v.y);
    }
    __syncthreads();
    // ---- GMP: Q_l(p) on the Q window
    for (int i = tid; i < B::QW; i += kThreads) {
      float2 Q[M + 1];
      gmp_q<K, M, L>(&rw[i + L], cf, Q);
#pragma unroll
      for (int l = 0; l <= M; ++l) qw[i][l] = Q[l];
    }
    __syncthreads();
    // ---- y, g_y = 2(y - Gx) (zero outside the stream), E and R on the tile
    Comp Ec, Rc;
    for (int i = tid; i < B::YW; i += kThreads) {
      int64_t n = t0 - L + i;
      float2 g = make_float2(0.f, 0.f);
      if (n >= lo && n < hi) {
        float2 y = make_float2(0.f, 0.f);
#pragma unroll
        for (int l = 0; l <= M; ++l) {
          float2 v = cmul(uw[i + M + L - l], qw[i + M - l][l]);
          y.x += v.x;
          y.y += v.y;
        }
        float2 xv = xw[i - L + B::XB];
        float tr = g_re * xv.x - g_im * xv.y, ti = g_re * xv.y + g_im * xv.x;
        float er = y.x - tr, ei = y.y - ti;
        g = make_float2(2.f * er, 2.f * ei);
        if (i >= L && i < L + S) {
          Ec.add(er * er + ei * ei);
          Rc.add(tr * tr + ti * ti);
        }
      }
      gyw[i] = g;
    }
    // E/R tile partial (fixed tree)
    red[tid] = Ec.s; red[kThreads + tid] = Ec.c; red[2 * kThreads + tid] = Rc.s; red[3 * kThreads + tid] = Rc.c;
    __syncthreads();
    for (int w2 = kThreads / 2; w2 > 0; w2 >>= 1) {
      if (tid < w2) {
        Comp a{red[tid], red[kThreads + tid]}, b{red[2 * kThreads + tid], red[3 * kThreads + tid]};
        a.add(red[tid + w2]); a.add(red[kThreads + tid + w2]);
        b.add(red[2 * kThreads + tid + w2]); b.add(red[3 * kThreads + tid + w2]);
        red[tid] = a.s; red[kThreads + tid] = a.c; red[2 * kThreads + tid] = b.s; red[3 * kThreads + tid] = b.c;
      }
      __syncthreads();
    }
    if (tid == 0) tile_part[t] = make_float2(red[0] + red[kThreads], red[2 * kThreads] + red[3 * kThreads]);
    // ---- g_u on the tile
    if (tid < S) {
      int64_t m = t0 + tid;
      float2 gu = make_float2(0.f, 0.f);
      if (m < hi) {
        float2 Qm[M + 1];
#pragma unroll
        for (int l = 0; l <= M; ++l) Qm[l] = qw[tid + B::QB][l];
        gu = gmp_grad<K, M, L>(&uw[tid + B::UB], &rw[tid + B::UB], &gyw[tid + L], Qm, cf, dcf);
      }
      guw[tid] = gu;
    }
    __syncthreads();   // g_u ready; the GMP part of the union is free from here on

    // ---- TDNN: recompute this wave's 32 samples, then the reverse mode
    const int col = 32 * wave + sl;
    typename C::A feat[C::NKS1];
    typename C::A hb[NL][C::NB][C::KS == 16 ? 2 : 16];
    float last[C::NB][16];
    mlp_forward<C, NL>(pk, vec, lane, h, &xw[col + B::XB], feat, hb, last);
    const float2 g = guw[col];
    // output layer: delta_o = (Re g_u, Im g_u) in rows 0, 1 of a 32-row block
    {
#pragma unroll
      for (int j = 0; j < 16; ++j) {
        int row = mfma_row(j, h);
        float v = row == 0 ? g.x : (row == 1 ? g.y : 0.f);
        dst[row * B::LD + col] = (E)v;
      }
      stage_acc_rows<C>(hst, B::LD, col, h, last);
    }
    __syncthreads();
    dw_layer<C, 1, C::NB>(dst, hst, B::LD, wave, lane, slot + C::dw_off(NL),
                          slot + C::dw_off(NL) + 32 * C::HP, first);
    // delta_nl = (Wo^T delta_o) * (1 - h_nl^2)
    float dl[C::NB][16];
    {
      const float* wo = vec + NL * C::HP;
#pragma unroll
      for (int mb = 0; mb < C::NB; ++mb)
#pragma unroll
        for (int j = 0; j < 16; ++j) {
          float hv = operand_value<C>(hb[NL - 1], mb, j);
          float w0 = wo[(0 * C::NB + mb) * 32 + h * 16 + j], w1 = wo[(1 * C::NB + mb) * 32 + h * 16 + j];
          dl[mb][j] = (w0 * g.x + w1 * g.y) * (1.f - hv * hv);
        }
    }
#pragma unroll
    for (int i = NL; i >= 1; --i) {   // hidden layer i: delta_i in dl, input h_{i-1}
      __syncthreads();                // staging free
      stage_acc_rows<C>(dst, B::LD, col, h, dl);
      if (i >= 2) {
        float hv[C::NB][16];
#pragma unroll
        for (int mb = 0; mb < C::NB; ++mb)
#pragma unroll
          for (int j = 0; j < 16; ++j) hv[mb][j] = operand_value<C>(hb[i - 2], mb, j);
        stage_acc_rows<C>(hst, B::LD, col, h, hv);
      } else {
        // features in natural order: row k = KS*ks + (KS/2)*h + e
#pragma unroll
        for (int ks = 0; ks < C::NKS1; ++ks) {
          if constexpr (C::KS == 16) {
#pragma unroll
            for (int e = 0; e < 8; ++e) hst[(16 * ks + 8 * h + e) * B::LD + col] = feat[ks][e];
          } else {
            hst[(2 * ks + h) * B::LD + col] = feat[ks];
          }
        }
#pragma unroll
        for (int k = C::KIN_P; k < C::C1; ++k)
          if ((k & 1) == h) hst[k * B::LD + col] = (E)0.f;
      }
      // delta_{i-1} = (W_i^T delta_i) * (1 - h_{i-1}^2) while the staging settles
      float dn[C::NB][16];
      if (i >= 2) {
        typename C::A db[C::NB][C::KS == 16 ? 2 : 16];
        to_operands<C>(dl, db);
        f32x16 acc[C::NB];
        const typename C::A* Ab =
            reinterpret_cast<const typename C::A*>(pk + C::OFF_BWDH) + (int64_t)(i - 2) * C::NB * C::NKSH * 64;
        dense<C, C::NKSH>(Ab, lane, [&](int ks) { return b_operand<C>(db, ks); }, acc);
#pragma unroll
        for (int mb = 0; mb < C::NB; ++mb)
#pragma unroll
          for (int j = 0; j < 16; ++j) {
            float hv = operand_value<C>(hb[i - 2], mb, j);
            dn[mb][j] = acc[mb][j] * (1.f - hv * hv);
          }
      }
      __syncthreads();
      if (i >= 2)
        dw_layer<C, C::NB, C::NB>(dst, hst, B::LD, wave, lane, slot + C::dw_off(i - 1),
                                  slot + C::dw_off(i - 1) + (int64_t)C::HP * C::HP, first);
      else
        dw_layer<C, C::NB, C::NN1>(dst, hst, B::LD, wave, lane, slot + C::dw_off(0),
                                   slot + C::dw_off(0) + (int64_t)C::HP * C::C1, first);
      if (i >= 2) {
#pragma unroll
        for (int mb = 0; mb < C::NB; ++mb)
#pragma unroll
          for (int j = 0; j < 16; ++j) dl[mb][j] = dn[mb][j];
      }
    }
  }
}

// ------------------------------------------------------------------ dW finalize
// dw[set][packed j] = inv_r[set] * sum over (stream s of set, workgroup g touching s)
// of slot[g + s] at the natural position of j.  Fixed order: s ascending, g ascending.
template <int PREC, int T, int H, int NL>
__global__ void k_dw_finalize(StreamTable st, int G_wg, const float* __restrict__ slots,
                              const float* __restrict__ inv_r, int64_t P, float* __restrict__ dw) {
  using C = Cfg<PREC, T, H, NL>;
  const int set = blockIdx.y;
  int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= P) return;
  // natural offset of packed index j
  int64_t nat;
  {
    int64_t pos = 0;
    int din = C::KIN;
    nat = -1;
    for (int li = 0; li <= NL && nat < 0; ++li) {
      int dout = li == NL ? 2 : H;
      int cols = li == 0 ? C::C1 : C::HP;
      int rows = li == NL ? 32 : C::HP;
      int64_t nw = (int64_t)dout * din;
      if (j < pos + nw) {
        int64_t r = j - pos;
        int o = (int)(r / din), k = (int)(r % din);
        nat = C::dw_off(li) + (int64_t)o * cols + k;
      } else if (j < pos + nw + dout) {
        int o = (int)(j - pos - nw);
        nat = C::dw_off(li) + (int64_t)rows * cols + o;
      }
      pos += nw + dout;
      din = H;
    }
  }
  float acc = 0.f;
  for (int s = 0; s < st.n; ++s) {
    if ((st.per_stream ? s : 0) != set) continue;
    int g0 = wg_of_tile(st.tile0[s], G_wg, st.n_tiles);
    int g1 = wg_of_tile(st.tile0[s + 1] - 1, G_wg, st.n_tiles);
    for (int g = g0; g <= g1; ++g) acc += slots[(int64_t)(g + s) * C::SLOT + nat];
  }
  dw[set * P + j] = acc * inv_r[set];
}

SrcOff src_offsets(int T, int H, int NL) {
  SrcOff so;
  int64_t pos = 0;
  int din = 5 * T;
  for (int i = 0; i <= NL; ++i) {
    int dout = i == NL ? 2 : H;
    so.w[i] = pos;
    pos += (int64_t)dout * din;
    so.b[i] = pos;
    pos += dout;
    din = H;
  }
  return so;
}

}  // namespace

// ------------------------------------------------------------------ host side
bool tdnn_dims(const dpd_tdnn_desc& d, TdnnDims* out) {
  TdnnDims td{};
  td.taps = d.taps;
  td.n_hidden = d.n_hidden;
  td.hidden = d.hidden;
  td.residual = d.residual;
  td.prec = d.precision;
  bool ok = tdnn_dispatch(d.precision, d.taps, d.hidden, d.n_hidden, [&]<int P_, int T_, int H_, int NL_>() {
    using C = Cfg<P_, T_, H_, NL_>;
    td.kin = C::KIN;
    td.hp = C::HP;
    td.kin_p = C::KIN_P;
    td.nks1 = C::NKS1;
    td.nksh = C::NKSH;
    td.pack_bytes = C::PACK;
    td.dw_slot = C::SLOT;
  });
  *out = td;
  return ok;
}

bool tuned_supported(const dpd_tdnn_desc& d, const dpd_gmp_desc* g) {
  if (!g) return tdnn_dispatch(d.precision, d.taps, d.hidden, d.n_hidden, [&]<int P_, int T_, int H_, int NL_>() {});
  return bwd_dispatch(d.precision, d.taps, d.hidden, d.n_hidden, g->K, g->M, g->L,
                      [&]<int P_, int T_, int H_, int NL_, int K_, int M_, int L_>() {});
}

void launch_pack(const TdnnDims& td, const float* w, int n_sets, int64_t w_stride, void* pack,
                 hipStream_t s) {
  SrcOff so = src_offsets(td.taps, td.hidden, td.n_hidden);
  tdnn_dispatch(td.prec, td.taps, td.hidden, td.n_hidden, [&]<int P_, int T_, int H_, int NL_>() {
    dim3 grid(64, n_sets);
    (void)sizeof(Cfg<P_, T_, H_, NL_>);
    k_pack<P_, T_, H_, NL_><<<grid, 256, 0, s>>>(w, w_stride, so, static_cast<char*>(pack));
  });
}

void launch_tdnn_fwd(const TdnnDims& td, const StreamTable& st, const float* x, const void* pack,
                     float* u, int grid, hipStream_t s) {
  tdnn_dispatch(td.prec, td.taps, td.hidden, td.n_hidden, [&]<int P_, int T_, int H_, int NL_>() {
    k_tdnn_fwd<P_, T_, H_, NL_><<<grid, kThreads, 0, s>>>(st, x, static_cast<const char*>(pack),
                                                         td.residual, u);
  });
}

void launch_tdnn_bwd(const TdnnDims& td, const dpd_gmp_desc& g, const StreamTable& st,
                     const float* x, const float* u, const float* coef, float g_re, float g_im,
                     const void* pack, float2* tile_part, float* slots, int grid, hipStream_t s) {
  bwd_dispatch(td.prec, td.taps, td.hidden, td.n_hidden, g.K, g.M, g.L,
               [&]<int P_, int T_, int H_, int NL_, int K_, int M_, int L_>() {
                 k_tdnn_bwd<P_, T_, H_, NL_, K_, M_, L_><<<grid, kThreads, 0, s>>>(
                     st, x, u, coef, g_re, g_im, static_cast<const char*>(pack), tile_part, slots);
               });
}

void launch_dw_finalize(const TdnnDims& td, const StreamTable& st, int grid, const float* slots,
                        const float* inv_r_set, float* dw, hipStream_t s) {
  int64_t P = (int64_t)td.hidden * (5 * td.taps) + td.hidden +
              (int64_t)(td.n_hidden - 1) * ((int64_t)td.hidden * td.hidden + td.hidden) +
              2 * (int64_t)td.hidden + 2;
  int n_sets = st.per_stream ? st.n : 1;
  tdnn_dispatch(td.prec, td.taps, td.hidden, td.n_hidden, [&]<int P_, int T_, int H_, int NL_>() {
    dim3 g2((unsigned)((P + 255) / 256), n_sets);
    k_dw_finalize<P_, T_, H_, NL_><<<g2, 256, 0, s>>>(st, grid, slots, inv_r_set, P, dw);
  });
}

}  // namespace dpdmi
