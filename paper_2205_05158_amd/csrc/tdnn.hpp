// Common pieces of the tuned TDNN kernels (tdnn_kernels.hpp): MFMA geometry,
// the packed parameter layout, the pack kernel, layer building blocks and the LDS
// staging of the reverse mode.  See tdnn.hip for the formulation.
#pragma once

#include <algorithm>
#include <type_traits>

#include "gmp.hpp"
#include "kernels.hpp"

namespace dpdmi {

namespace {


constexpr int kWaves = 4;               // backward kernel: one wave per SIMD
constexpr int kThreads = 64 * kWaves;
// Forward kernel waves per workgroup (a tile shape chosen at run time among the compiled
// variants): the workgroup shares one LDS copy of the weights, so its wave count sets the
// waves per SIMD.  Default: three per SIMD for the bf16 kernel of width 128 (it fits in
// registers), two for the others.
__host__ __device__ constexpr int fwd_waves(int prec, int hidden) {
  return prec == DPD_BF16 && hidden >= 128 ? 12 : 8;
}

constexpr int cmax(int a, int b) { return a > b ? a : b; }

// ------------------------------------------------------------------ MFMA geometry
// MT: rows (neurons) and columns (samples) of a tile; KS: K per instruction; NR:
// accumulator values per lane; LG = 64 / MT lane groups, each holding one K-slice of
// an operand; EPL: operand elements per lane.  row(j, g): neuron row of accumulator
// value j in lane group g.  A layer's value (row block mb, value j) is element
// e_of(mb, j) of the next layer's B operand for K step ks_of(mb, j); mb_of and j_of
// invert that map.
template <int PREC, int MT> struct Mma;

template <> struct Mma<DPD_BF16, 32> {
  static constexpr int MT = 32, KS = 16, NR = 16, LG = 2, EPL = 8;
  using A = bf16x8;
  using Acc = f32x16;
  using E = __bf16;
  __device__ static Acc mma(A a, A b, Acc c) { return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0); }
  __host__ __device__ static constexpr int row(int j, int g) { return 8 * (j >> 2) + 4 * g + (j & 3); }
  __host__ __device__ static constexpr int ks_of(int mb, int j) { return 2 * mb + j / 8; }
  __host__ __device__ static constexpr int e_of(int, int j) { return j % 8; }
  __host__ __device__ static constexpr int mb_of(int ks, int) { return ks / 2; }
  __host__ __device__ static constexpr int j_of(int ks, int e) { return 8 * (ks % 2) + e; }
};

template <> struct Mma<DPD_BF16, 16> {
  static constexpr int MT = 16, KS = 32, NR = 4, LG = 4, EPL = 8;
  using A = bf16x8;
  using Acc = f32x4;
  using E = __bf16;
  __device__ static Acc mma(A a, A b, Acc c) { return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0); }
  __host__ __device__ static constexpr int row(int j, int g) { return 4 * g + j; }
  __host__ __device__ static constexpr int ks_of(int mb, int) { return mb / 2; }
  __host__ __device__ static constexpr int e_of(int mb, int j) { return 4 * (mb % 2) + j; }
  __host__ __device__ static constexpr int mb_of(int ks, int e) { return 2 * ks + e / 4; }
  __host__ __device__ static constexpr int j_of(int, int e) { return e % 4; }
};

template <> struct Mma<DPD_FP32, 32> {
  static constexpr int MT = 32, KS = 2, NR = 16, LG = 2, EPL = 1;
  using A = float;
  using Acc = f32x16;
  using E = float;
  __device__ static Acc mma(A a, A b, Acc c) { return __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, c, 0, 0, 0); }
  __host__ __device__ static constexpr int row(int j, int g) { return 8 * (j >> 2) + 4 * g + (j & 3); }
  __host__ __device__ static constexpr int ks_of(int mb, int j) { return 16 * mb + j; }
  __host__ __device__ static constexpr int e_of(int, int) { return 0; }
  __host__ __device__ static constexpr int mb_of(int ks, int) { return ks / 16; }
  __host__ __device__ static constexpr int j_of(int ks, int) { return ks % 16; }
};

template <int PREC, int T, int H, int NL>
struct Cfg {
  using X = Mma<PREC, PREC == DPD_BF16 ? 16 : 32>;    // layer tiles
  using D = Mma<PREC, 32>;                              // dW tiles
  using A = typename X::A;
  using E = typename X::E;
  static constexpr int MT = X::MT, KS = X::KS, NR = X::NR, LG = X::LG;
  static constexpr int S = MT * kWaves;                // samples per workgroup tile
  static constexpr int KIN = 5 * T;
  // bf16 tanh layers run on weights and biases pre-scaled by 2 log2 e (the MFMA then
  // yields the exp2 argument of tanh_bf16_scaled directly; its accumulators start at the
  // scaled bias), so the delta chain through them carries a factor WS per layer, which
  // k_dw_finalize removes.  The output layer is not scaled.
  static constexpr float WS = X::EPL == 8 ? kTanhScale : 1.0f;
  // Layer-1 K order: lane group g holds the features of its own taps [g*TPG, (g+1)*TPG):
  // element f = EPL*ks + e of its K-slices is feature f%5 of tap g*TPG + f/5 (zero when
  // f >= 5*TPG or the tap is >= T), so each lane computes only its own taps' features.
  static constexpr int TPG = (T + LG - 1) / LG;
  static constexpr int FPG = 5 * TPG;
  static constexpr int NKS1 = (FPG + X::EPL - 1) / X::EPL;
  static constexpr int KIN_P = NKS1 * KS;
  static constexpr int HP = round_up(H, 32);
  static constexpr int NB = HP / MT;                    // row blocks of a layer
  static constexpr int NKSH = HP / KS;                  // K steps of a hidden layer
  static constexpr int C1 = round_up(KIN, 32);          // dW columns of layer 1
  static constexpr int NN1 = C1 / 32;
  static constexpr int NBD = HP / 32;                   // dW row blocks
  // packed parameter set (bytes)
  static constexpr int64_t ES = sizeof(A);
  static constexpr int64_t OFF_FWD1 = 0;
  static constexpr int64_t OFF_FWDH = OFF_FWD1 + (int64_t)NB * NKS1 * 64 * ES;
  static constexpr int64_t OFF_BWDH = OFF_FWDH + (int64_t)(NL - 1) * NB * NKSH * 64 * ES;
  static constexpr int64_t OFF_VEC = OFF_BWDH + (int64_t)(NL - 1) * NB * NKSH * 64 * ES;
  // float vector block: bias [NL][NB][LG][NR], wo [2][NB][LG][NR], bo[2] (+2 pad)
  static constexpr int NVEC = NL * HP + 2 * HP + 4;
  // bf16 models: the output layer as one 16-row MFMA A block (rows 0, 1 = the two outputs,
  // K in the accumulator order of the last hidden layer), [K step][64 lanes]
  static constexpr bool OUT_MMA = X::EPL == 8;
  static constexpr int64_t OFF_WO = OFF_VEC + (int64_t)NVEC * 4;
  static constexpr int64_t PACK = OFF_WO + (OUT_MMA ? (int64_t)NKSH * 64 * 16 : 0);
  // natural dW slot (floats): per layer W block [rows][cols] then bias [rows]
  static constexpr int64_t DW_L1 = (int64_t)HP * C1 + HP;
  static constexpr int64_t DW_H = (int64_t)HP * HP + HP;
  static constexpr int64_t DW_O = 32LL * HP + 32;
  static constexpr int64_t SLOT = DW_L1 + (NL - 1) * DW_H + DW_O;
  __host__ __device__ static constexpr int64_t dw_off(int li) {   // li = 0..NL (NL = output)
    return li == 0 ? 0 : DW_L1 + (int64_t)(li - 1) * DW_H;
  }
  // feature index held by element e of K step ks in lane group g (layer 1), -1 for padding
  __host__ __device__ static constexpr int feat_k(int ks, int g, int e) {
    return (X::EPL * ks + e < FPG && g * TPG + (X::EPL * ks + e) / 5 < T) ? FPG * g + X::EPL * ks + e : -1;
  }
  // previous-layer neuron held by element e of K step ks in lane group g (hidden layers)
  __host__ __device__ static constexpr int hid_k(int ks, int g, int e) {
    return MT * X::mb_of(ks, e) + X::row(X::j_of(ks, e), g);
  }
};

// ------------------------------------------------------------------ pack
// Source offsets inside the packed float32 weight vector.
struct SrcOff {
  int64_t w[DPD_MAX_LAYERS + 1], b[DPD_MAX_LAYERS + 1];
};

// Packs parameter set blockIdx.y of a model with tn taps and width hn (at most the
// compiled T and padded width; the padding rows and columns are zero).
template <int PREC, int T, int H, int NL>
__global__ void k_pack(const float* __restrict__ w, int64_t w_stride, SrcOff so,
                       int tn, int hn, char* __restrict__ pack) {
  using C = Cfg<PREC, T, H, NL>;
  using X = typename C::X;
  constexpr int EPL = X::EPL;
  const int set = blockIdx.y;
  const float* ws = w + set * w_stride;
  char* ps = pack + set * C::PACK;
  const int64_t n1 = (int64_t)C::NB * C::NKS1 * 64;
  const int64_t nh = (int64_t)(NL - 1) * C::NB * C::NKSH * 64;
  const int64_t no = C::OUT_MMA ? (int64_t)C::NKSH * 64 : 0;
  const int64_t total = n1 + 2 * nh + C::NVEC + no;
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * blockDim.x) {
    if (idx >= n1 + 2 * nh + C::NVEC) {
      // output-layer A block (bf16)
      if constexpr (C::OUT_MMA) {
        const int64_t f = idx - (n1 + 2 * nh + C::NVEC);
        const int lane = (int)(f % 64), ks = (int)(f / 64);
        const int m = lane % C::MT, g = lane / C::MT;
        bf16x8 a;
        for (int ee = 0; ee < 8; ++ee) {
          const int kk = C::hid_k(ks, g, ee);
          a[ee] = (__bf16)((m < 2 && kk < hn) ? ws[so.w[NL] + (int64_t)m * hn + kk] : 0.f);
        }
        reinterpret_cast<bf16x8*>(ps + C::OFF_WO)[f] = a;
      }
    } else if (idx < n1 + 2 * nh) {
      const int lane = (int)(idx % 64);
      const int rowl = lane % C::MT, g = lane / C::MT;
      const int64_t q = idx / 64;
      int sec, layer = 0, mb, ks;
      if (idx < n1) {
        sec = 0; mb = (int)(q / C::NKS1); ks = (int)(q % C::NKS1);
      } else {
        const int64_t r = idx < n1 + nh ? (idx - n1) / 64 : (idx - n1 - nh) / 64;
        sec = idx < n1 + nh ? 1 : 2;
        layer = (int)(r / ((int64_t)C::NB * C::NKSH)) + 2;   // layer index i = 2..NL
        const int64_t rr = r % ((int64_t)C::NB * C::NKSH);
        mb = (int)(rr / C::NKSH); ks = (int)(rr % C::NKSH);
      }
      const int m = C::MT * mb + rowl;                        // A-operand row
      float v[EPL];
      for (int ee = 0; ee < EPL; ++ee) {
        float val = 0.f;
        if (sec == 0) {
          const int k = C::feat_k(ks, g, ee);
          if (m < hn && k >= 0 && k < 5 * tn) val = ws[so.w[0] + (int64_t)m * (5 * tn) + k];
        } else {
          const int kk = C::hid_k(ks, g, ee);
          const float* Wi = ws + so.w[layer - 1];             // W_i is [hn][hn]
          if (m < hn && kk < hn)
            val = sec == 1 ? Wi[(int64_t)m * hn + kk]           // forward: A[o][k] = W_i[o][k]
                           : Wi[(int64_t)kk * hn + m];          // backward: A[k][o] = W_i[o][k]
        }
        v[ee] = val * C::WS;
      }
      if constexpr (EPL == 8) {
        bf16x8 a;
        for (int ee = 0; ee < 8; ++ee) a[ee] = (__bf16)v[ee];
        reinterpret_cast<bf16x8*>(ps)[idx] = a;
      } else {
        reinterpret_cast<float*>(ps)[idx] = v[0];
      }
    } else {
      // float vector block, rows in accumulator order: r = MT*mb + NR*g + j holds
      // neuron MT*mb + row(j, g)
      const int f = (int)(idx - n1 - 2 * nh);
      auto neuron = [&](int r) {
        const int mb = r / C::MT, g = (r % C::MT) / C::NR, j = r % C::NR;
        return C::MT * mb + X::row(j, g);
      };
      float val = 0.f;
      if (f < NL * C::HP) {
        // bf16 layers take their bias pre-scaled by 2 log2 e (see tanh_bf16_scaled)
        const int i = f / C::HP, o = neuron(f % C::HP);
        if (o < hn) val = ws[so.b[i] + o] * (EPL == 8 ? kTanhScale : 1.0f);
      } else if (f < NL * C::HP + 2 * C::HP) {
        const int r0 = f - NL * C::HP;
        const int c = r0 / C::HP, o = neuron(r0 % C::HP);
        if (o < hn) val = ws[so.w[NL] + (int64_t)c * hn + o];
      } else {
        const int c = f - NL * C::HP - 2 * C::HP;
        if (c < 2) val = ws[so.b[NL] + c];
      }
      reinterpret_cast<float*>(ps + C::OFF_VEC)[f] = val;
    }
  }
}

// ------------------------------------------------------------------ layer pieces
// A layer's values in B-operand form: NKS operands per lane.
template <class C, int NKS>
using Ops = typename C::A[NKS];

template <class C>
__device__ __forceinline__ void set_elem(typename C::A& a, int e, float v) {
  if constexpr (C::X::EPL == 8) a[e] = (__bf16)v;
  else { (void)e; a = v; }
}
template <class C>
__device__ __forceinline__ float get_elem(const typename C::A& a, int e) {
  if constexpr (C::X::EPL == 8) return (float)a[e];
  else { (void)e; return a; }
}
// Hides the value of a layer held in bf16 operand form from the optimiser: otherwise it
// keeps the float32 values the operands were rounded from (twice the registers) and
// redoes the rounding wherever a bf16 value is read back.  No-op for float32 operands.
template <class C, int NKS>
__device__ __forceinline__ void opaque_ops(Ops<C, NKS>& ops) {
  if constexpr (C::X::EPL == 8) {
#pragma unroll
    for (int ks = 0; ks < NKS; ++ks) {
      uint4 w = __builtin_bit_cast(uint4, ops[ks]);
      asm volatile("" : "+v"(w.x), "+v"(w.y), "+v"(w.z), "+v"(w.w));
      ops[ks] = __builtin_bit_cast(typename C::A, w);
    }
  }
}

// value j of row block mb of a layer held in operand form
template <class C, int NKS>
__device__ __forceinline__ float value_at(const Ops<C, NKS>& ops, int mb, int j) {
  return get_elem<C>(ops[C::X::ks_of(mb, j)], C::X::e_of(mb, j));
}

// Features (I, Q, |x|, |x|^2, |x|^3 per tap) of the lane's sample for the taps of its
// lane group g (see Cfg::feat_k): xw points at x[n] in an LDS window (xw[-t] = x[n-t]).
// RT: the model has tn <= T taps; the features of taps >= tn are zero (their weights are
// zero too, but a non-finite sample there must not reach the sum).
template <class C, bool RT = false>
__device__ __forceinline__ void make_features(const float2* xw, int g, Ops<C, C::NKS1>& feat, int tn = 0) {
  constexpr int T = C::KIN / 5, EPL = C::X::EPL;
  float f[C::NKS1 * EPL];
  const int tb = g * C::TPG;
#pragma unroll
  for (int t = 0; t < C::TPG; ++t) {
    float2 z;
    if constexpr (T % C::LG == 0) {
      z = xw[-(tb + t)];
    } else {
      const bool ok = tb + t < T;
      z = xw[-(ok ? tb + t : T - 1)];
      z = ok ? z : make_float2(0.f, 0.f);
    }
    if constexpr (RT) z = tb + t < tn ? z : make_float2(0.f, 0.f);
    const float m2 = z.x * z.x + z.y * z.y;
    const float m = __builtin_amdgcn_sqrtf(m2);   // hardware square root (within 1 ulp)
    f[5 * t + 0] = z.x;
    f[5 * t + 1] = z.y;
    f[5 * t + 2] = m;
    f[5 * t + 3] = m2;
    f[5 * t + 4] = m2 * m;
  }
#pragma unroll
  for (int k = C::FPG; k < C::NKS1 * EPL; ++k) f[k] = 0.f;
#pragma unroll
  for (int ks = 0; ks < C::NKS1; ++ks)
#pragma unroll
    for (int e = 0; e < EPL; ++e) set_elem<C>(feat[ks], e, f[EPL * ks + e]);
}

// One row block mb of a dense layer: sum_ks A(mb, ks) B(ks); Apk is [NB][NKS][64].
template <class C, int NKS, class BF>
__device__ __forceinline__ typename C::X::Acc dense_block(const typename C::A* __restrict__ Apk, int mb,
                                                          int lane, BF&& bop) {
  typename C::X::Acc acc;
#pragma unroll
  for (int j = 0; j < C::NR; ++j) acc[j] = 0.f;
#pragma unroll
  for (int ks = 0; ks < NKS; ++ks) {
    const typename C::A a = Apk[((int64_t)mb * NKS + ks) * 64 + lane];
    acc = C::X::mma(a, bop(ks), acc);
  }
  return acc;
}

// A whole layer, block by block: epi(mb, acc) receives sum_ks A(mb, ks) B(ks) for
// mb = 0..NB-1.  For short K (bf16 operands) the A operands of block mb+1 are read
// while block mb's MFMAs run, and block mb's epilogue runs after block mb+1's MFMAs
// are issued, so the loads, the matrix cores and the vector ALU overlap within the
// wave.  Long K (fp32 operands) runs one block at a time.
// A-operand loaders: la(mb, ks) returns the lane's operand of row block mb, K step ks.
// Packed operand order ([row block][K step][64 lanes]):
template <class C, int NKS>
struct PackedA {
  const typename C::A* __restrict__ p;
  int lane;
  __device__ typename C::A operator()(int mb, int ks) const { return p[((int64_t)mb * NKS + ks) * 64 + lane]; }
};
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));

// Accumulators of a block start at zero ...
struct ZeroInit {
  template <class Acc> __device__ Acc operator()(int, Acc* tag) const {
    (void)tag;
    Acc a;
#pragma unroll
    for (int j = 0; j < (int)(sizeof(Acc) / sizeof(float)); ++j) a[j] = 0.f;
    return a;
  }
};
// ... or at the lane's rows of a bias vector in accumulator order (the bf16 forward
// layers: their scaled bias, read from LDS along with the block's weight operands).
template <class C>
struct BiasInit {
  const float* bias;   // layer's bias block, rows in accumulator order
  int g;
  template <class Acc> __device__ Acc operator()(int mb, Acc* tag) const {
    (void)tag;
    return *reinterpret_cast<const Acc*>(bias + (mb * C::LG + g) * C::NR);
  }
};

template <class C, int NKS, class LA, class BF, class EPI, class INIT = ZeroInit>
__device__ __forceinline__ void dense_layer(LA&& la, BF&& bop, EPI&& epi, INIT&& init = INIT{}) {
  using A = typename C::A;
  using Acc = typename C::X::Acc;
  Acc* const tag = nullptr;
  if constexpr (NKS <= 8) {
    A cur[NKS], nxt[NKS];
#pragma unroll
    for (int ks = 0; ks < NKS; ++ks) cur[ks] = la(0, ks);
    Acc a_cur = init(0, tag), a_nxt;
    Acc prev;
#pragma unroll
    for (int mb = 0; mb < C::NB; ++mb) {
      if (mb + 1 < C::NB) {
#pragma unroll
        for (int ks = 0; ks < NKS; ++ks) nxt[ks] = la(mb + 1, ks);
        a_nxt = init(mb + 1, tag);
      }
      DPD_KEEP_LOADS_LOCAL();
      Acc acc = a_cur;
#pragma unroll
      for (int ks = 0; ks < NKS; ++ks) acc = C::X::mma(cur[ks], bop(ks), acc);
      if (mb > 0) epi(mb - 1, prev);
      prev = acc;
#pragma unroll
      for (int ks = 0; ks < NKS; ++ks) cur[ks] = nxt[ks];
      a_cur = a_nxt;
    }
    epi(C::NB - 1, prev);
  } else {
#pragma unroll
    for (int mb = 0; mb < C::NB; ++mb) {
      DPD_KEEP_LOADS_LOCAL();
      Acc acc = init(mb, tag);
#pragma unroll
      for (int ks = 0; ks < NKS; ++ks) acc = C::X::mma(la(mb, ks), bop(ks), acc);
      epi(mb, acc);
    }
  }
}

// Sum over the LG lane groups that share a sample column.
template <class C>
__device__ __forceinline__ float lane_group_sum(float v) {
  if constexpr (C::LG == 4) v += __shfl_xor(v, 16);
  return v + __shfl_xor(v, 32);
}

// Forward through all hidden layers one row block at a time.  hb[i] holds h_{i+1} in
// operand form; returns the two linear outputs (valid in every lane group).
// wf: forward weight operands (layer 1, then the hidden layers; global or LDS).  vec:
// LDS copy of the float vector block (biases, output layer).
// sink(i, hb[i]) receives each hidden layer's activations as soon as they are formed.
struct NoSink {
  template <class O> __device__ void operator()(int, const O&) const {}
};
template <class C, int NL, bool RT = false, class SINK = NoSink>
__device__ __forceinline__ float2 mlp_forward(const typename C::A* __restrict__ wf,
                                              const typename C::A* __restrict__ wout,
                                              const float* vec, int lane, int g, const float2* xw,
                                              Ops<C, C::NKSH> (&hb)[NL], int tn = 0, SINK&& sink = SINK{}) {
  using A = typename C::A;
  Ops<C, C::NKS1> feat;
  make_features<C, RT>(xw, g, feat, tn);
  const float* wo = vec + NL * C::HP;
  float o0 = 0.f, o1 = 0.f;
#pragma unroll
  for (int i = 0; i < NL; ++i) {
    auto epi = [&](int mb, const typename C::X::Acc& acc) {
      const int vb = (mb * C::LG + g) * C::NR;
      const float* bias = vec + i * C::HP + vb;
#pragma unroll
      for (int j = 0; j < C::NR; ++j) {
        float v;
        if constexpr (C::X::EPL == 8) {
          (void)bias;
          v = tanh_bf16_scaled(acc[j]);          // accumulators started at the scaled bias
        } else {
          v = tanh_f32(acc[j] + bias[j]);
          if (i == NL - 1) {
            o0 = fmaf(wo[vb + j], v, o0);
            o1 = fmaf(wo[C::HP + vb + j], v, o1);
          }
        }
        set_elem<C>(hb[i][C::X::ks_of(mb, j)], C::X::e_of(mb, j), v);
      }
    };
    using Init = std::conditional_t<C::X::EPL == 8, BiasInit<C>, ZeroInit>;
    Init init;
    if constexpr (C::X::EPL == 8) init = BiasInit<C>{vec + i * C::HP, g};
    if (i == 0) {
      dense_layer<C, C::NKS1>(PackedA<C, C::NKS1>{wf, lane}, [&](int ks) { return feat[ks]; }, epi, init);
    }
    if (i > 0) {
      const A* Ah = wf + (int64_t)C::NB * C::NKS1 * 64 + (int64_t)(i - 1) * C::NB * C::NKSH * 64;
      dense_layer<C, C::NKSH>(PackedA<C, C::NKSH>{Ah, lane}, [&](int ks) { return hb[i - 1][ks]; }, epi,
                              init);
    }
    opaque_ops<C, C::NKSH>(hb[i]);
    sink(i, hb[i]);
  }
  const float* bo = vec + NL * C::HP + 2 * C::HP;
  if constexpr (C::X::EPL == 8) {
    // output layer on the matrix cores: rows 0 and 1 of a 16-row block land in lane
    // group 0 (accumulator values 0 and 1); other lane groups return garbage
    typename C::X::Acc acc;
#pragma unroll
    for (int j = 0; j < C::NR; ++j) acc[j] = 0.f;
#pragma unroll
    for (int ks = 0; ks < C::NKSH; ++ks) acc = C::X::mma(wout[ks * 64 + lane], hb[NL - 1][ks], acc);
    return make_float2(acc[0] + bo[0], acc[1] + bo[1]);
  } else {
    o0 = lane_group_sum<C>(o0);
    o1 = lane_group_sum<C>(o1);
    return make_float2(o0 + bo[0], o1 + bo[1]);
  }
}

// ------------------------------------------------------------------ backward kernel
template <int PREC, int T, int H, int NL>
struct BwdLds {
  using C = Cfg<PREC, T, H, NL>;
  static constexpr int S = C::S;
  static constexpr int XB = T - 1;
  static constexpr int XW = S + XB;               // x  [t0 - XB, t0 + S)
  static constexpr int HROWS = cmax(C::C1, C::HP);
  // dW staging.  bf16 (SM): sample-major [sample][RW neurons]; the 8-byte chunk c (4
  // neurons) of sample s sits at chunk position c ^ tsw(s), so the 8-byte writes of a
  // lane group's 4 consecutive neurons over 16 consecutive samples, and the transposing
  // reads of 4 samples x 4 chunks per 16 lanes that build the dW MFMA operands, hit
  // distinct banks.  With 256-byte sample rows (one sweep of the 64 banks), s mod 16 =
  // 4q + i (i = i1 i0, q = q1 q0 in bits) and tsw = 16 i1 + 8 i0 + 4 (i1 ^ q1) + 2 q0 + q1:
  // its bits 4..1 and 3..0 each take 16 values over 16 samples (writes, 32- and 16-lane
  // halves) and bits 4..3 and 3..2 each 4 values over 4 samples (reads).  Narrower rows
  // use 4 i + q within the row's chunks.  fp32: [row][sample], rows padded by 4 floats.
  static constexpr bool SM = PREC == DPD_BF16;
  static_assert(!SM || (S == 64 && C::MT == 16), "sample-major staging of 64-sample bf16 tiles");
  static constexpr int RW = HROWS;                // SM: neurons per staged sample
  static constexpr int NPR = RW / 4;              // SM: 8-byte chunks per sample row
  static constexpr int LD = S + 4;                // fp32: staging row stride (elements)
  __host__ __device__ static int tsw(int s) {
    if (NPR == 32) {
      const int i0 = s & 1, i1 = (s >> 1) & 1, q0 = (s >> 2) & 1, q1 = (s >> 3) & 1;
      return 16 * i1 + 8 * i0 + 4 * (i1 ^ q1) + 2 * q0 + q1;
    }
    return ((4 * (s & 3)) | ((s >> 2) & 3)) & (NPR - 1);
  }
  __device__ static int off(int row, int col) {
    if constexpr (SM) return col * RW + 4 * ((row >> 2) ^ tsw(col)) + (row & 3);
    else return row * LD + col;
  }
  // fp32: rows of lane group g in a layer block are row(j, 0) + 4g, so the staging element
  // of (row MT*mb + row(j, g), column col) is (MT*mb + row(j, 0))*LD + lb[0] with
  // lb[0] = 4g*LD + col.  bf16: neuron chunk 4 mb + g of sample col is at position
  // 4 (mb ^ (tsw >> 2)) + (g ^ (tsw & 3)), i.e. element lb[0] + 16 (mb ^ lb[1]).
  __device__ static void lane_bases(int g, int col, int (&lb)[2]) {
    if constexpr (SM) {
      const int t = tsw(col);
      lb[0] = col * RW + 4 * (g ^ (t & 3));
      lb[1] = t >> 2;
    } else {
      lb[0] = 4 * g * LD + col;
      lb[1] = 0;
    }
  }
  static constexpr int STAGE_BYTES = SM ? 2 * S * RW * 2 : (C::HP + HROWS) * LD * 4;
  // bytes of static LDS besides the weight operands
  // bf16 layers with one delta row block per wave (BREG) keep their bias-gradient sums in
  // registers (each wave the rows of its own block); the others accumulate them in LDS.
  static constexpr bool BREG = SM && C::NBD == kWaves;
  static constexpr int BIAS_N = BREG ? 0 : NL * C::HP + 32;  // LDS bias-gradient accumulators
  static constexpr int DSTO_BYTES = SM ? 2 * S * 2 : 0;   // bf16: output-layer delta, [2][S]
  static constexpr int BASE_BYTES = (SM ? 2 : 1) * XW * 8 + C::NVEC * 4 + BIAS_N * 4 + STAGE_BYTES + DSTO_BYTES;
  // Weight operands staged in LDS, the byte range [W_LO, W_HI) of the packed set: both
  // packs when they fit, else the backward (transposed) pack, whose short delta-chain
  // blocks hide global-memory latency worse than the tanh-heavy recompute blocks, else
  // the forward pack, else none.
  static constexpr int kLdsBudget = 160 * 1024;
  static constexpr bool FIT_ALL = BASE_BYTES + C::OFF_VEC <= kLdsBudget;
  static constexpr bool FIT_BWD = BASE_BYTES + (C::OFF_VEC - C::OFF_BWDH) <= kLdsBudget;
  static constexpr bool FIT_FWD = BASE_BYTES + C::OFF_BWDH <= kLdsBudget;
  static constexpr int64_t W_LO = FIT_ALL ? 0 : (FIT_BWD ? C::OFF_BWDH : 0);
  static constexpr int64_t W_HI = FIT_ALL ? C::OFF_VEC : (FIT_BWD ? C::OFF_VEC : (FIT_FWD ? C::OFF_BWDH : 0));
  static constexpr bool W_FWD = W_LO == 0 && W_HI >= C::OFF_BWDH;
  static constexpr bool W_BWD = W_LO <= C::OFF_BWDH && W_HI == C::OFF_VEC;
  static constexpr int64_t W_BYTES = W_HI > W_LO ? W_HI - W_LO : 16;
  // 32x32 dW blocks of the tanh layers (layer 1, then the hidden layers), dealt
  // round-robin over the waves: block bi is held by wave bi % kWaves in dwacc[bi / kWaves].
  // The output layer's 2 x HP dW is one register per thread instead (2*HP <= threads).
  static constexpr int NBL1 = C::NBD * C::NN1, NBLH = C::NBD * C::NBD;
  static constexpr int NBT = NBL1 + (NL - 1) * NBLH;
  static constexpr int NQ = (NBT + kWaves - 1) / kWaves;
  static_assert(2 * C::HP <= kThreads, "one output-layer dW element per thread");
  __host__ __device__ static constexpr int blk_off(int li) {   // li = 0..NL-1
    return li == 0 ? 0 : NBL1 + (li - 1) * NBLH;
  }
  __host__ __device__ static constexpr int blk_cnt(int li) { return li == 0 ? NBL1 : NBLH; }
  __host__ __device__ static constexpr int blk_cols(int li) { return li == 0 ? C::NN1 : C::NBD; }
  // bf16 layers with one delta row block per wave: each wave's blocks share operands, a
  // 2x2 quadrant of a 4x4 layer (QUAD) or one row block of the others (STRIP), so every
  // staged operand a wave needs is read from LDS once per tile.
  __host__ __device__ static constexpr bool QUAD(int nnb) { return SM && C::NBD == kWaves && nnb == 4; }
  __host__ __device__ static constexpr bool STRIP(int nnb) { return SM && C::NBD == kWaves && nnb != 4; }
  // (row block, column block) of block blk of a layer with nnb column blocks (block blk is
  // held by wave blk % kWaves; the layer offsets are multiples of kWaves when QUAD or
  // STRIP applies).  Otherwise the column index is rotated by the row index so the bias
  // rows (column block 0) spread over the waves.
  __device__ static void blk_rc(int blk, int nnb, int& mb, int& nb) {
    if (QUAD(nnb)) {
      const int w = blk % kWaves, k = blk / kWaves;
      mb = 2 * (w / 2) + k / 2;
      nb = 2 * (w % 2) + k % 2;
    } else if (STRIP(nnb)) {
      mb = blk % kWaves;
      nb = blk / kWaves;
    } else {
      mb = blk / nnb;
      nb = (blk % nnb + mb) % nnb;
    }
  }
};

// One 32x32 dW block over the tile's samples: rows mb of the delta staging against
// rows nb of the activation staging (both [row][sample]).  All operand reads are
// issued before the MFMAs.
//
// bf16 (sample-major staging): the 32x32x16 operand of lane (row r = lane%32, K half
// h = lane/32) holds neuron 32 blk + r over samples 16 ks + 8 h + (0..7).  It is built by
// two transposing 8-byte reads per K step: in 16-lane group G = lane/16, lane l supplies
// the chunk of neurons 32 blk + 16 (G%2) + 4 (l%4) .. +3 of sample 16 ks + 8 (G/2) + 4 t +
// l/4 (t = 0, 1) and receives neuron 32 blk + 16 (G%2) + l over those 4 samples.  The
// bias row sums come from the same operand registers.
struct DwOps {
  bf16x8 a[4], b[4];
};
template <class B, class P>
__device__ __forceinline__ void dw_tr_operand(const P* stage, int blk, int lane, bf16x8 (&op)[4]) {
  static_assert(sizeof(P) == 2, "bf16 staging");
  const __bf16* arr = reinterpret_cast<const __bf16*>(stage);
  const int G = lane / 16, l = lane % 16;
  const int c = 8 * blk + 4 * (G % 2) + l % 4;
  int base[2];
#pragma unroll
  for (int t = 0; t < 2; ++t) {
    const int sm = 8 * (G / 2) + 4 * t + l / 4;   // sample mod 16
    base[t] = sm * B::RW + 4 * (c ^ B::tsw(sm));
  }
  typedef __attribute__((address_space(3))) bf16x4 lds_bf16x4;
#pragma unroll
  for (int ks = 0; ks < 4; ++ks) {
    const bf16x4 lo = __builtin_amdgcn_ds_read_tr16_b64_v4bf16((lds_bf16x4*)(arr + base[0] + 16 * ks * B::RW));
    const bf16x4 hi = __builtin_amdgcn_ds_read_tr16_b64_v4bf16((lds_bf16x4*)(arr + base[1] + 16 * ks * B::RW));
    op[ks] = __builtin_shufflevector(lo, hi, 0, 1, 2, 3, 4, 5, 6, 7);
  }
}
template <class C, class B>
__device__ __forceinline__ void dw_load_bf16(const __bf16* dst, const __bf16* hst, int mb, int nb,
                                             int lane, DwOps& o) {
  static_assert(C::S == 64, "four K steps of 16 samples");
  dw_tr_operand<B>(dst, mb, lane, o.a);
  dw_tr_operand<B>(hst, nb, lane, o.b);
}
template <class C>
__device__ __forceinline__ void dw_mma_bf16(const bf16x8 (&a)[4], const bf16x8 (&b)[4], f32x16& acc) {
#pragma unroll
  for (int ks = 0; ks < 4; ++ks) acc = C::D::mma(a[ks], b[ks], acc);
}
template <class C>
__device__ __forceinline__ void dw_mma_bf16(const DwOps& o, f32x16& acc) {
  dw_mma_bf16<C>(o.a, o.b, acc);
}
// sum over the tile's samples of the delta row held in a (both lane halves)
__device__ __forceinline__ float dw_rowsum_bf16(const bf16x8 (&a)[4]) {
  typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
  const bf16x2 one = {(__bf16)1.0f, (__bf16)1.0f};
  float sum = 0.f;
#pragma unroll
  for (int ks = 0; ks < 4; ++ks)
#pragma unroll
    for (int e = 0; e < 8; e += 2) {
      const bf16x2 pr = {a[ks][e], a[ks][e + 1]};
      sum = __builtin_amdgcn_fdot2_f32_bf16(pr, one, sum, false);
    }
  return sum + __shfl_xor(sum, 32);
}

template <class C, class B>
__device__ __forceinline__ f32x16 dw_block(const typename C::E* dst, const typename C::E* hst,
                                           int mb, int nb, int lane, f32x16 acc) {
  using D = typename C::D;
  constexpr int NK = C::S / D::KS;
  const int h = lane / 32, r = lane % 32;
  const int ra = 32 * mb + r, rb = 32 * nb + r;
  typename D::A a[NK], b[NK];
#pragma unroll
  for (int ks = 0; ks < NK; ++ks) {
    if constexpr (D::EPL == 8) {
      a[ks] = *reinterpret_cast<const bf16x8*>(dst + B::off(ra, 16 * ks + 8 * h));
      b[ks] = *reinterpret_cast<const bf16x8*>(hst + B::off(rb, 16 * ks + 8 * h));
    } else {
      a[ks] = dst[B::off(ra, 2 * ks + h)];
      b[ks] = hst[B::off(rb, 2 * ks + h)];
    }
  }
#pragma unroll
  for (int ks = 0; ks < NK; ++ks) acc = D::mma(a[ks], b[ks], acc);
  return acc;
}

// Sum over the tile's samples of delta row 32*mb + lane%32 (the bias gradient).
template <class C, class B>
__device__ __forceinline__ float delta_row_sum(const typename C::E* dst, int mb, int lane) {
  const int h = lane / 32, r = lane % 32;
  const int row = 32 * mb + r;
  float sum = 0.f;
  if constexpr (C::D::EPL == 8) {
#pragma unroll
    for (int c = 0; c < C::S / 2; c += 8) {
      const bf16x8 v = *reinterpret_cast<const bf16x8*>(dst + B::off(row, h * (C::S / 2) + c));
#pragma unroll
      for (int e = 0; e < 8; ++e) sum += (float)v[e];
    }
  } else {
    const typename C::E* arow = dst + B::off(row, h * (C::S / 2));
#pragma unroll
    for (int c = 0; c < C::S / 2; c += 4) {
      const float4 v = *reinterpret_cast<const float4*>(arow + c);
      sum += (v.x + v.y) + (v.z + v.w);
    }
  }
  return sum + __shfl_xor(sum, 32);
}

// Stage a layer held in operand form (lane bases of BwdLds::lane_bases).  bf16: the
// lane's 4 consecutive neurons 16 mb + 4 g + (0..3) of row block mb are 4 consecutive
// elements of its operand register (one 8-byte write); fp32: value (mb, j) goes to row
// MT*mb + row(j, g), column col.
template <class C, class B, int NKS>
__device__ __forceinline__ void stage_layer(typename C::E* stage, const int (&lb)[2],
                                            const Ops<C, NKS>& ops) {
  if constexpr (B::SM) {
    // opaque copies: the per-block addresses are formed here, not kept live across layers
    int b0 = lb[0], th = lb[1];
    asm volatile("" : "+v"(b0), "+v"(th));
#pragma unroll
    for (int ks = 0; ks < NKS; ++ks) {
      const uint4 w = __builtin_bit_cast(uint4, ops[ks]);
#pragma unroll
      for (int h2 = 0; h2 < 2; ++h2) {
        const int mb = C::X::mb_of(ks, 4 * h2);          // elements 4 h2 .. 4 h2 + 3
        const uint2 v = h2 ? make_uint2(w.z, w.w) : make_uint2(w.x, w.y);
        *reinterpret_cast<uint2*>(stage + b0 + 16 * (mb ^ th)) = v;
      }
    }
  } else {
#pragma unroll
    for (int ks = 0; ks < NKS; ++ks)
#pragma unroll
      for (int e = 0; e < C::X::EPL; ++e) {
        const int mb = C::X::mb_of(ks, e), j = C::X::j_of(ks, e);
        stage[(C::MT * mb + C::X::row(j, 0)) * B::LD + lb[0]] = (typename C::E)get_elem<C>(ops[ks], e);
      }
  }
}

}  // namespace

}  // namespace dpdmi
