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
#include <type_traits>

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
// B operands of one 32-row block: 2 x 8 bf16 (bf16) or 16 floats (fp32), i.e. the 16
// accumulator rows of the lane in K-step order.
template <class C>
using BlockOps = typename C::A[C::KS == 16 ? 2 : 16];

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

// B operand of K step ks of a hidden layer from the previous layer's blocks.
template <class C>
__device__ __forceinline__ typename C::A b_operand(const BlockOps<C> (&hb)[C::NB], int ks) {
  if constexpr (C::KS == 16) return hb[ks / 2][ks % 2];
  else return hb[ks / 16][ks % 16];
}

template <class C>
__device__ __forceinline__ void block_to_operands(const float (&v)[16], BlockOps<C>& out) {
  if constexpr (C::KS == 16) {
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      bf16x8 a;
#pragma unroll
      for (int e = 0; e < 8; ++e) a[e] = (__bf16)v[8 * q + e];
      out[q] = a;
    }
  } else {
#pragma unroll
    for (int j = 0; j < 16; ++j) out[j] = v[j];
  }
}

template <class C>
__device__ __forceinline__ float operand_value(const BlockOps<C>& b, int j) {
  if constexpr (C::KS == 16) return (float)b[j / 8][j % 8];
  else return b[j];
}

template <class C>
__device__ __forceinline__ f32x16 mfma(typename C::A a, typename C::A b, f32x16 c) {
  if constexpr (C::KS == 16) return mfma_bf16(a, b, c);
  else return mfma_f32(a, b, c);
}

// One 32-row block mb of a dense layer: sum_ks A(mb, ks) B(ks); Apk is [NB][NKS][64].
template <class C, int NKS, class BF>
__device__ __forceinline__ f32x16 dense_block(const typename C::A* __restrict__ Apk, int mb,
                                              int lane, BF&& bop) {
  f32x16 acc;
#pragma unroll
  for (int j = 0; j < 16; ++j) acc[j] = 0.f;
#pragma unroll
  for (int ks = 0; ks < NKS; ++ks) {
    typename C::A a = Apk[((int64_t)mb * NKS + ks) * 64 + lane];
    acc = mfma<C>(a, bop(ks), acc);
  }
  return acc;
}

// Forward through all hidden layers one 32-neuron block at a time.  Keeps every
// layer's B operands in hb (hb[i] = h_{i+1}) and returns the two linear outputs.
// wf: the forward weight operands (layer 1 then hidden layers, packed order; global
// or LDS); vec: LDS copy of the float vector block (biases, output layer).
template <class C, int NL>
__device__ __forceinline__ float2 mlp_forward(const typename C::A* __restrict__ wf, const float* vec,
                                              int lane, int h, const float2* xw,
                                              BlockOps<C> (&hb)[NL][C::NB]) {
  using A = typename C::A;
  A feat[C::NKS1];
  make_features<C>(xw, h, feat);
  const float* wo = vec + NL * C::HP;
  float o0 = 0.f, o1 = 0.f;
#pragma unroll
  for (int i = 0; i < NL; ++i) {
#pragma unroll
    for (int mb = 0; mb < C::NB; ++mb) {
      DPD_KEEP_LOADS_LOCAL();
      f32x16 acc;
      if (i == 0) {
        acc = dense_block<C, C::NKS1>(wf, mb, lane, [&](int ks) { return feat[ks]; });
      } else {
        const A* Ah = wf + (int64_t)C::NB * C::NKS1 * 64 + (int64_t)(i - 1) * C::NB * C::NKSH * 64;
        acc = dense_block<C, C::NKSH>(Ah, mb, lane, [&](int ks) { return b_operand<C>(hb[i - 1], ks); });
      }
      const float* bias = vec + (i * C::NB + mb) * 32 + h * 16;
      float v[16];
#pragma unroll
      for (int j = 0; j < 16; ++j) {
        if constexpr (C::KS == 16) v[j] = tanh_bf16(acc[j] + bias[j]);
        else v[j] = tanh_f32(acc[j] + bias[j]);
      }
      block_to_operands<C>(v, hb[i][mb]);
      if (i == NL - 1) {
#pragma unroll
        for (int j = 0; j < 16; ++j) {
          o0 = fmaf(wo[(0 * C::NB + mb) * 32 + h * 16 + j], v[j], o0);
          o1 = fmaf(wo[(1 * C::NB + mb) * 32 + h * 16 + j], v[j], o1);
        }
      }
    }
  }
  o0 += __shfl_xor(o0, 32);
  o1 += __shfl_xor(o1, 32);
  const float* bo = vec + NL * C::HP + 2 * C::HP;
  return make_float2(o0 + bo[0], o1 + bo[1]);
}

// ------------------------------------------------------------------ forward kernel
// Each workgroup owns a contiguous range of tiles; the forward weight operands of the
// current parameter set live in LDS (reloaded only when the set changes), so every
// MFMA A operand is one conflict-free 16-byte (bf16) or 4-byte (fp32) LDS read.
template <int PREC, int T, int H, int NL>
__global__ __launch_bounds__(kThreads) void k_tdnn_fwd(StreamTable st, const float* __restrict__ x,
                                                       const char* __restrict__ pack, int residual,
                                                       float* __restrict__ u) {
  using C = Cfg<PREC, T, H, NL>;
  using A = typename C::A;
  constexpr int XW = kTile + T - 1;
  // forward operands in 16-byte units; models whose forward weights exceed the LDS
  // budget read them from global memory (L2) instead
  constexpr bool kLdsWeights = C::OFF_BWDH <= 144 * 1024;
  constexpr int NWF = kLdsWeights ? (int)(C::OFF_BWDH / 16) : 1;
  __shared__ float2 xw[XW];
  __shared__ float vec[C::NVEC];
  __shared__ __attribute__((aligned(16))) uint4 wf[NWF];
  const int lane = threadIdx.x % 64, wave = threadIdx.x / 64, h = lane / 32, sl = lane % 32;
  const int t_begin = wg_tile_start(blockIdx.x, gridDim.x, st.n_tiles);
  const int t_end = wg_tile_start(blockIdx.x + 1, gridDim.x, st.n_tiles);
  int cur_set = -1;
  for (int t = t_begin; t < t_end; ++t) {
    int s = stream_of_tile(st, t);
    int set = st.per_stream ? s : 0;
    int64_t lo = st.off[s], hi = st.off[s + 1];
    int64_t t0 = lo + (int64_t)(t - st.tile0[s]) * kTile;
    const char* pk = pack + set * C::PACK;
    __syncthreads();   // previous tile done with the LDS windows
    if (set != cur_set) {
      const float* src = reinterpret_cast<const float*>(pk + C::OFF_VEC);
      for (int i = threadIdx.x; i < C::NVEC; i += kThreads) vec[i] = src[i];
      if constexpr (kLdsWeights) {
        const uint4* wsrc = reinterpret_cast<const uint4*>(pk);
        for (int i = threadIdx.x; i < NWF; i += kThreads) wf[i] = wsrc[i];
      }
      cur_set = set;
    }
    for (int i = threadIdx.x; i < XW; i += kThreads) {
      int64_t p = t0 - (T - 1) + i;
      xw[i] = (p >= lo && p < hi) ? ld2(x, p) : make_float2(0.f, 0.f);
    }
    __syncthreads();
    BlockOps<C> hb[NL][C::NB];
    int col = 32 * wave + sl;
    const A* wops = kLdsWeights ? reinterpret_cast<const A*>(wf) : reinterpret_cast<const A*>(pk);
    float2 o = mlp_forward<C, NL>(wops, vec, lane, h, &xw[col + T - 1], hb);
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
  // dW blocks per layer and the register-resident accumulators that hold them:
  // layer blocks bi = 4q + wave, q = 0..ceil(blocks/4)-1, in dwacc[Q0 + q].
  static constexpr int NBL1 = C::NB * C::NN1, NBLH = C::NB * C::NB, NBLO = C::NB;
  static constexpr int Q1 = (NBL1 + 3) / 4, QH = (NBLH + 3) / 4, QO = (NBLO + 3) / 4;
  static constexpr int NQ = Q1 + (NL - 1) * QH + QO;
  static constexpr int BIAS = NL * C::HP + 32;   // bias-gradient accumulators
};

// Stage the lane's 16 accumulator-order values of every block (one sample column).
template <class C>
__device__ __forceinline__ void stage_ops(typename C::E* stage, int ld, int col, int h,
                                          const BlockOps<C> (&b)[C::NB]) {
#pragma unroll
  for (int mb = 0; mb < C::NB; ++mb)
#pragma unroll
    for (int j = 0; j < 16; ++j)
      stage[(32 * mb + mfma_row(j, h)) * ld + col] = (typename C::E)operand_value<C>(b[mb], j);
}

// One 32x32 dW block over the tile's samples: rows mb of the delta staging against
// rows nb of the activation staging (both [row][sample]).
template <class C>
__device__ __forceinline__ f32x16 dw_block(const typename C::E* dst, const typename C::E* hst, int ld,
                                           int mb, int nb, int lane, f32x16 acc) {
  const int h = lane / 32, r = lane % 32;
  const typename C::E* arow = dst + (32 * mb + r) * ld;
  const typename C::E* brow = hst + (32 * nb + r) * ld;
#pragma unroll
  for (int ks = 0; ks < kTile / C::KS; ++ks) {
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
  return acc;
}

// Sum over the tile's samples of delta row 32*mb + lane%32 (the bias gradient).
template <class C>
__device__ __forceinline__ float delta_row_sum(const typename C::E* dst, int ld, int mb, int lane) {
  const int h = lane / 32, r = lane % 32;
  const typename C::E* arow = dst + (32 * mb + r) * ld + h * (kTile / 2);
  float sum = 0.f;
  if constexpr (C::KS == 16) {
#pragma unroll
    for (int c = 0; c < kTile / 2; c += 8) {
      bf16x8 v = *reinterpret_cast<const bf16x8*>(arow + c);
#pragma unroll
      for (int e = 0; e < 8; ++e) sum += (float)v[e];
    }
  } else {
#pragma unroll
    for (int c = 0; c < kTile / 2; c += 4) {
      float4 v = *reinterpret_cast<const float4*>(arow + c);
      sum += (v.x + v.y) + (v.z + v.w);
    }
  }
  return sum + __shfl_xor(sum, 32);
}

template <int PREC, int T, int H, int NL, int K, int M, int L>
__global__ __launch_bounds__(kThreads) void k_tdnn_bwd(StreamTable st, const float* __restrict__ x,
                                                       const float* __restrict__ u,
                                                       const float* __restrict__ coef, float g_re,
                                                       float g_im, const char* __restrict__ pack,
                                                       float2* __restrict__ tile_part,
                                                       float* __restrict__ slots,
                                                       float* __restrict__ y_out) {
  using C = Cfg<PREC, T, H, NL>;
  using G = Gmp<K, M, L>;
  using B = BwdLds<PREC, T, H, NL, K, M, L>;
  using E = typename C::E;
  using A = typename C::A;
  constexpr int S = kTile;
  __shared__ float2 xw[B::XW];
  __shared__ float2 uw[B::UW];
  __shared__ float rw[B::UW];
  __shared__ float2 guw[2 * S];        // g_u partial sums of the two tap halves
  __shared__ float vec[C::NVEC];
  __shared__ float red[4 * kThreads];
  __shared__ float bacc[B::BIAS];
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

  // dW accumulators of this wave's blocks, kept in registers for the whole tile range
  // of one stream and written to its slot once.
  f32x16 dwacc[B::NQ];
#pragma unroll
  for (int q = 0; q < B::NQ; ++q)
#pragma unroll
    for (int j = 0; j < 16; ++j) dwacc[q][j] = 0.f;
  for (int i = tid; i < B::BIAS; i += kThreads) bacc[i] = 0.f;

  // Write this workgroup's partial dW of stream s (plain stores: each (workgroup,
  // stream) slot is written exactly once) and reset the accumulators.  Caller syncs.
  auto flush = [&](int s) {
    float* slot = slots + (int64_t)(g_wg + s) * C::SLOT;
#pragma unroll
    for (int q = 0; q < B::NQ; ++q) {
      // decode (layer, block) of dwacc[q] for this wave
      int li, ql, nnb, nbl;
      if (q < B::Q1) { li = 0; ql = q; nnb = C::NN1; nbl = B::NBL1; }
      else if (q < B::Q1 + (NL - 1) * B::QH) { li = 1 + (q - B::Q1) / B::QH; ql = (q - B::Q1) % B::QH; nnb = C::NB; nbl = B::NBLH; }
      else { li = NL; ql = q - B::Q1 - (NL - 1) * B::QH; nnb = C::NB; nbl = B::NBLO; }
      int bi = 4 * ql + wave;
      if (bi < nbl) {
        int mb = bi / nnb, nb = bi % nnb;
        float* out = slot + C::dw_off(li) + (int64_t)(32 * mb) * (nnb * 32) + 32 * nb + sl;
#pragma unroll
        for (int j = 0; j < 16; ++j) out[(int64_t)mfma_row(j, h) * (nnb * 32)] = dwacc[q][j];
      }
#pragma unroll
      for (int j = 0; j < 16; ++j) dwacc[q][j] = 0.f;
    }
    for (int i = tid; i < B::BIAS; i += kThreads) {
      int li = i / C::HP, o = i % C::HP;
      float* dstb = li < NL ? slot + C::dw_off(li) + (int64_t)C::HP * (li == 0 ? C::C1 : C::HP) + o
                            : slot + C::dw_off(NL) + 32 * C::HP + (i - NL * C::HP);
      *dstb = bacc[i];
      bacc[i] = 0.f;
    }
  };

  // accumulate the owned blocks of one layer (li: 0 = input layer, NL = output layer)
  auto accumulate = [&](auto li_c) {
    constexpr int li = decltype(li_c)::value;
    constexpr int nnb = li == 0 ? C::NN1 : C::NB;
    constexpr int nbl = li == 0 ? B::NBL1 : (li == NL ? B::NBLO : B::NBLH);
    constexpr int q0 = li == 0 ? 0 : (li == NL ? B::Q1 + (NL - 1) * B::QH : B::Q1 + (li - 1) * B::QH);
    constexpr int nql = li == 0 ? B::Q1 : (li == NL ? B::QO : B::QH);
    float* bl = bacc + (li == NL ? NL * C::HP : li * C::HP);
#pragma unroll
    for (int q = 0; q < nql; ++q) {
      DPD_KEEP_LOADS_LOCAL();
      int bi = 4 * q + wave;
      if (bi < nbl) {
        int mb = bi / nnb, nb = bi % nnb;
        dwacc[q0 + q] = dw_block<C>(dst, hst, B::LD, mb, nb, lane, dwacc[q0 + q]);
        if (nb == 0) {
          float sum = delta_row_sum<C>(dst, B::LD, mb, lane);
          if (h == 0) bl[32 * mb + sl] += sum;
        }
      }
    }
  };

  int cur_stream = -1;
  for (int t = t_begin; t < t_end; ++t) {
    const int s = stream_of_tile(st, t);
    const int set = st.per_stream ? s : 0;
    const int64_t lo = st.off[s], hi = st.off[s + 1];
    const int64_t t0 = lo + (int64_t)(t - st.tile0[s]) * S;
    const char* pk = pack + set * C::PACK;
    const float* cs = coef + (st.per_stream ? (int64_t)s * 2 * G::J : 0);

    __syncthreads();   // previous tile finished with every LDS buffer and accumulator
    if (s != cur_stream) {
      if (cur_stream >= 0) flush(cur_stream);
      cur_stream = s;
    }
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
    // ---- GMP: Q_l(p) on the Q window; waves 0-1 take taps [0, LH), waves 2-3 [LH, M]
    constexpr int LH = (M + 1) / 2;
    const bool upper = tid >= kThreads / 2;
    for (int i = tid % (kThreads / 2); i < B::QW; i += kThreads / 2) {
      DPD_KEEP_LOADS_LOCAL();
      float2 Q[M + 1];
      if (upper) {
        gmp_q<K, M, L, LH, M + 1>(&rw[i + L], cf, Q);
#pragma unroll
        for (int l = LH; l <= M; ++l) qw[i][l] = Q[l];
      } else {
        gmp_q<K, M, L, 0, LH>(&rw[i + L], cf, Q);
#pragma unroll
        for (int l = 0; l < LH; ++l) qw[i][l] = Q[l];
      }
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
          if (y_out) st2(y_out, n, y);
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
    // ---- g_u on the tile: the two halves of the taps in two partial sums
    {
      static_assert(S == kThreads / 2, "one sample per thread and tap half");
      const int i = tid % S;
      int64_t m = t0 + i;
      float2 gu = make_float2(0.f, 0.f);
      if (m < hi) {
        float2 Qm[M + 1];
#pragma unroll
        for (int l = 0; l <= M; ++l) Qm[l] = qw[i + B::QB][l];
        if (upper)
          gu = gmp_grad<K, M, L, LH, M + 1>(&uw[i + B::UB], &rw[i + B::UB], &gyw[i + L], Qm, cf, dcf);
        else
          gu = gmp_grad<K, M, L, 0, LH>(&uw[i + B::UB], &rw[i + B::UB], &gyw[i + L], Qm, cf, dcf);
      }
      guw[tid] = gu;
    }
    __syncthreads();   // g_u ready; the GMP part of the union is free from here on

    // ---- TDNN: recompute this wave's 32 samples, then the reverse mode
    const int col = 32 * wave + sl;
    BlockOps<C> hb[NL][C::NB];
    (void)mlp_forward<C, NL>(reinterpret_cast<const A*>(pk + C::OFF_FWD1), vec, lane, h,
                             &xw[col + B::XB], hb);
    const float2 g = make_float2(guw[col].x + guw[S + col].x, guw[col].y + guw[S + col].y);
    // output layer: delta_o = (Re g_u, Im g_u) in rows 0, 1 of a 32-row block
#pragma unroll
    for (int j = 0; j < 16; ++j) {
      int row = mfma_row(j, h);
      dst[row * B::LD + col] = (E)(row == 0 ? g.x : (row == 1 ? g.y : 0.f));
    }
    stage_ops<C>(hst, B::LD, col, h, hb[NL - 1]);
    __syncthreads();
    accumulate(std::integral_constant<int, NL>{});
    // delta_nl = (Wo^T delta_o) * (1 - h_nl^2)
    BlockOps<C> db[C::NB];
    {
      const float* wo = vec + NL * C::HP;
#pragma unroll
      for (int mb = 0; mb < C::NB; ++mb) {
        float v[16];
#pragma unroll
        for (int j = 0; j < 16; ++j) {
          float hv = operand_value<C>(hb[NL - 1][mb], j);
          float w0 = wo[(0 * C::NB + mb) * 32 + h * 16 + j], w1 = wo[(1 * C::NB + mb) * 32 + h * 16 + j];
          v[j] = (w0 * g.x + w1 * g.y) * (1.f - hv * hv);
        }
        block_to_operands<C>(v, db[mb]);
      }
    }
    auto layer = [&](auto i_c) {       // hidden layer i: delta_i in db, input h_{i-1}
      constexpr int i = decltype(i_c)::value;
      __syncthreads();                 // staging free
      stage_ops<C>(dst, B::LD, col, h, db);
      if constexpr (i >= 2) {
        stage_ops<C>(hst, B::LD, col, h, hb[i - 2]);
      } else {
        A feat[C::NKS1];
        make_features<C>(&xw[col + B::XB], h, feat);
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
      BlockOps<C> dn[C::NB];
      if constexpr (i >= 2) {
        const A* Ab = reinterpret_cast<const A*>(pk + C::OFF_BWDH) + (int64_t)(i - 2) * C::NB * C::NKSH * 64;
#pragma unroll
        for (int mb = 0; mb < C::NB; ++mb) {
          DPD_KEEP_LOADS_LOCAL();
          f32x16 acc = dense_block<C, C::NKSH>(Ab, mb, lane, [&](int ks) { return b_operand<C>(db, ks); });
          float v[16];
#pragma unroll
          for (int j = 0; j < 16; ++j) {
            float hv = operand_value<C>(hb[i - 2][mb], j);
            v[j] = acc[j] * (1.f - hv * hv);
          }
          block_to_operands<C>(v, dn[mb]);
        }
      }
      __syncthreads();
      accumulate(std::integral_constant<int, i - 1>{});
      if constexpr (i >= 2) {
#pragma unroll
        for (int mb = 0; mb < C::NB; ++mb) {
          if constexpr (C::KS == 16) {
            db[mb][0] = dn[mb][0];
            db[mb][1] = dn[mb][1];
          } else {
#pragma unroll
            for (int j = 0; j < 16; ++j) db[mb][j] = dn[mb][j];
          }
        }
      }
    };
    static_assert(NL >= 1 && NL <= 4, "hidden layer count of the tuned kernel");
    if constexpr (NL >= 4) layer(std::integral_constant<int, 4>{});
    if constexpr (NL >= 3) layer(std::integral_constant<int, 3>{});
    if constexpr (NL >= 2) layer(std::integral_constant<int, 2>{});
    layer(std::integral_constant<int, 1>{});
  }
  __syncthreads();
  if (cur_stream >= 0) flush(cur_stream);
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
    td.fwd_lds = (C::OFF_BWDH <= 144 * 1024 ? C::OFF_BWDH : 16) + 8 * (kTile + T_) + 4 * C::NVEC;
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
                     const void* pack, float2* tile_part, float* slots, float* y, int grid,
                     hipStream_t s) {
  bwd_dispatch(td.prec, td.taps, td.hidden, td.n_hidden, g.K, g.M, g.L,
               [&]<int P_, int T_, int H_, int NL_, int K_, int M_, int L_>() {
                 k_tdnn_bwd<P_, T_, H_, NL_, K_, M_, L_><<<grid, kThreads, 0, s>>>(
                     st, x, u, coef, g_re, g_im, static_cast<const char*>(pack), tile_part, slots, y);
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
