// The tuned TDNN kernels (forward, reverse mode, pack, dW finalize) and their launchers,
// templated on the compiled shape; included by the translation units that instantiate
// shapes (tdnn.hip: the exact shapes; tdnn_gen.hip: the generic grid, one unit per
// precision and padded width).
#pragma once

#include "tdnn.hpp"

namespace dpdmi {

typedef unsigned act_u32x4 __attribute__((ext_vector_type(4)));   // one stored operand register

// Generic instantiations (tdnn_gen.hip, one unit per precision and padded width): the
// shape compiled for tp taps (8, 16 or 32) and nl hidden layers (1..4).
const TdnnKernels* tdnn_gen_bf16_32(int tp, int nl);
const TdnnKernels* tdnn_gen_bf16_64(int tp, int nl);
const TdnnKernels* tdnn_gen_bf16_128(int tp, int nl);
const TdnnKernels* tdnn_gen_fp32_32(int tp, int nl);
const TdnnKernels* tdnn_gen_fp32_64(int tp, int nl);
const TdnnKernels* tdnn_gen_fp32_128(int tp, int nl);

namespace {

// ------------------------------------------------------------------ forward kernel
// Each workgroup (FW waves, MT samples each) owns a contiguous range of tiles; the
// forward weight operands of the current parameter set live in LDS (reloaded only when
// the set changes) unless they exceed the LDS budget, in which case they are read from
// global memory (L2).
template <int PREC, int T, int H, int NL, int FW, bool RT>
__global__ __launch_bounds__(64 * FW) void k_tdnn_fwd(StreamTable st, const float* __restrict__ x,
                                                          const char* __restrict__ pack, int residual,
                                                          int tn, float* __restrict__ u,
                                                          act_u32x4* __restrict__ act) {
  using C = Cfg<PREC, T, H, NL>;
  using A = typename C::A;
  constexpr int kFwdThreads = 64 * FW;
  constexpr int S = C::MT * FW;
  constexpr int XW = S + T - 1;
  constexpr bool kLdsWeights = C::OFF_BWDH <= 144 * 1024;
  constexpr int NWF = kLdsWeights ? (int)(C::OFF_BWDH / 16) : 1;
  __shared__ float2 xw[XW];
  __shared__ __attribute__((aligned(16))) float vec[C::NVEC];
  __shared__ __attribute__((aligned(16))) uint4 wf[NWF];
  const int lane = threadIdx.x % 64, wave = threadIdx.x / 64;
  const int g = lane / C::MT, sl = lane % C::MT;
  const int t_begin = wg_tile_start(blockIdx.x, gridDim.x, st.n_tiles);
  const int t_end = wg_tile_start(blockIdx.x + 1, gridDim.x, st.n_tiles);
  int cur_set = -1;
  for (int t = t_begin; t < t_end; ++t) {
    const int s = stream_of_tile(st, t);
    const int set = st.per_stream ? s : 0;
    const int64_t lo = st.off[s], hi = st.off[s + 1];
    const int64_t t0 = lo + (int64_t)(t - st.tile0[s]) * S;
    const char* pk = pack + set * C::PACK;
    __syncthreads();   // previous tile done with the LDS windows
    if (set != cur_set) {
      const float* src = reinterpret_cast<const float*>(pk + C::OFF_VEC);
      for (int i = threadIdx.x; i < C::NVEC; i += kFwdThreads) vec[i] = src[i];
      if constexpr (kLdsWeights) {
        const uint4* wsrc = reinterpret_cast<const uint4*>(pk);
        for (int i = threadIdx.x; i < NWF; i += kFwdThreads) wf[i] = wsrc[i];
      }
      cur_set = set;
    }
    for (int i = threadIdx.x; i < XW; i += kFwdThreads) {
      const int64_t p = t0 - (T - 1) + i;
      xw[i] = (p >= lo && p < hi) ? ld2(x, p) : make_float2(0.f, 0.f);
    }
    __syncthreads();
    Ops<C, C::NKSH> hb[NL];
    const int col = C::MT * wave + sl;
    const A* wops = kLdsWeights ? reinterpret_cast<const A*>(wf) : reinterpret_cast<const A*>(pk);
    // bf16 with a reverse mode to follow: each layer's activations of the wave (operand
    // form, one 16-byte store per lane and operand) go to the stream's 16-sample group, for
    // every group of the stream's reverse-mode tiles (those past the stream hold the zero
    // input's)
    static_assert(C::X::EPL != 8 || C::MT == 16, "16-sample activation groups");
    const int64_t grp = (int64_t)(t - st.tile0[s]) * FW + wave;
    act_u32x4* dsta = (C::X::EPL == 8 && act && grp < st.grp0[s + 1] - st.grp0[s])
                          ? act + (st.grp0[s] + grp) * (NL * C::NKSH * 64) + lane
                          : nullptr;
    auto sink = [&](int i, const Ops<C, C::NKSH>& h) {
      if constexpr (C::X::EPL == 8) {
        if (dsta) {
#pragma unroll
          for (int ks = 0; ks < C::NKSH; ++ks)
            __builtin_nontemporal_store(__builtin_bit_cast(act_u32x4, h[ks]), dsta + (i * C::NKSH + ks) * 64);
        }
      }
    };
    float2 o = mlp_forward<C, NL, RT>(wops, reinterpret_cast<const A*>(pk + C::OFF_WO), vec, lane,
                                      g, &xw[col + T - 1], hb, tn, sink);
    const int64_t n = t0 + col;
    if (g == 0 && n < hi) {
      if (residual) {
        const float2 xv = xw[col + T - 1];
        o.x += xv.x;
        o.y += xv.y;
      }
      st2(u, n, o);
    }
  }
}

// Reverse mode of the TDNN over the stream table's tiles, from g_u (= dL/du per sample,
// zero-extended outside the streams): each workgroup owns a contiguous tile range, takes
// its samples' hidden activations from the forward's store (bf16) or recomputes them
// (fp32), runs the delta chain and accumulates dW over its tiles in registers; one slot
// per (workgroup, stream) is written.
template <int PREC, int T, int H, int NL, bool RT>
__global__ __launch_bounds__(kThreads) void k_tdnn_bwd(StreamTable st, const float* __restrict__ x,
                                                       const float* __restrict__ gu,
                                                       const char* __restrict__ pack, int tn,
                                                       float* __restrict__ slots,
                                                       const act_u32x4* __restrict__ act) {
  using C = Cfg<PREC, T, H, NL>;
  using X = typename C::X;
  using B = BwdLds<PREC, T, H, NL>;
  using E = typename C::E;
  using A = typename C::A;
  constexpr int S = C::S;
  // bf16: x windows of this tile and the next (buffer t % 2), stored at the end of the
  // previous tile; fp32: one window, stored at the top of the tile
  constexpr int NXB = B::SM ? 2 : 1;
  __shared__ float2 xw[NXB][B::XW];
  __shared__ __attribute__((aligned(16))) float vec[C::NVEC];
  __shared__ float bacc[B::BIAS_N > 0 ? B::BIAS_N : 1];
  __shared__ __attribute__((aligned(16))) char un[B::STAGE_BYTES];
  __shared__ __attribute__((aligned(16))) uint4 wlds[B::W_BYTES / 16];
  __shared__ __attribute__((aligned(16))) __bf16 dsto[B::SM ? 2 * S : 8];
  E* dst = reinterpret_cast<E*>(un);
  E* hst = dst + (B::SM ? S * B::RW : C::HP * B::LD);

  const int tid = threadIdx.x;
  const int wave_u = __builtin_amdgcn_readfirstlane(tid / 64);
  __builtin_assume(wave_u >= 0 && wave_u < kWaves);
  const int g_wg = blockIdx.x, G_wg = gridDim.x;
  const int t_begin = wg_tile_start(g_wg, G_wg, st.n_tiles);
  const int t_end = wg_tile_start(g_wg + 1, G_wg, st.n_tiles);

  // Lane-dependent values are re-derived at the top of every tile from an opaque copy of
  // the thread index, so the compiler cannot precompute the hundreds of per-block LDS and
  // global addresses outside the tile loop (they would not fit in registers).
  int lane = tid % 64;

  // dW accumulators of this wave's blocks, kept in registers for the whole tile range
  // of one stream and written to its slot once.
  f32x16 dwacc[B::NQ];
#pragma unroll
  for (int q = 0; q < B::NQ; ++q)
#pragma unroll
    for (int j = 0; j < 16; ++j) dwacc[q][j] = 0.f;
  // output-layer dW: fp32, element (tid / HP, tid % HP); bf16, rows 0 and 1 at column
  // 32 wave + lane of the lanes lane < 32 of waves wave < HP / 32
  float dwo = 0.f, dwo1 = 0.f;
  // BREG: bias-gradient sums of rows 32 wave + lane % 32 of each tanh layer (both lane
  // halves hold them) and, in wave 0, of the two outputs (lanes 0 and 1)
  float bsr[NL + 1];
#pragma unroll
  for (int li = 0; li <= NL; ++li) bsr[li] = 0.f;
  for (int i = tid; i < B::BIAS_N; i += kThreads) bacc[i] = 0.f;

  // Write this workgroup's partial dW of stream s (plain stores: each (workgroup,
  // stream) slot is written exactly once) and reset the accumulators.  Caller syncs.
  auto flush = [&](int s) {
    float* slot = slots + (int64_t)(g_wg + s) * C::SLOT;
    int ln = lane, wv = wave_u;
    asm volatile("" : "+v"(ln), "+s"(wv));
    const int h = ln / 32, r = ln % 32;
#pragma unroll
    for (int q = 0; q < B::NQ; ++q) {
      const int bi = kWaves * q + wv;
      int li = -1;
#pragma unroll
      for (int l2 = 0; l2 < NL; ++l2)
        if (bi >= B::blk_off(l2) && bi < B::blk_off(l2) + B::blk_cnt(l2)) li = l2;
      if (li >= 0) {
        const int nnb = li == 0 ? C::NN1 : C::NBD;
        int mb, nb;
        B::blk_rc(bi - B::blk_off(li), nnb, mb, nb);
        float* out = slot + C::dw_off(li) + (32 * mb) * (nnb * 32) + 32 * nb + r;
#pragma unroll
        for (int j = 0; j < 16; ++j) out[C::D::row(j, h) * (nnb * 32)] = dwacc[q][j];
      }
#pragma unroll
      for (int j = 0; j < 16; ++j) dwacc[q][j] = 0.f;
    }
    if constexpr (B::SM) {
      if (wv < C::NBD && ln < 32) {
        slot[C::dw_off(NL) + 32 * wv + ln] = dwo;
        slot[C::dw_off(NL) + C::HP + 32 * wv + ln] = dwo1;
      }
    } else {
      if (tid < 2 * C::HP) slot[C::dw_off(NL) + tid] = dwo;   // row tid / HP, column tid % HP
    }
    dwo = dwo1 = 0.f;
    if constexpr (B::BREG) {
      if (ln < 32) {
#pragma unroll
        for (int li = 0; li < NL; ++li)
          slot[C::dw_off(li) + (int64_t)C::HP * (li == 0 ? C::C1 : C::HP) + 32 * wv + ln] = bsr[li];
        if (wv == 0) slot[C::dw_off(NL) + 32 * C::HP + ln] = ln < 2 ? bsr[NL] : 0.f;
      }
#pragma unroll
      for (int li = 0; li <= NL; ++li) bsr[li] = 0.f;
    }
    for (int i = tid; i < B::BIAS_N; i += kThreads) {
      const int li = i / C::HP, o = i % C::HP;
      float* dstb = li < NL ? slot + C::dw_off(li) + (int64_t)C::HP * (li == 0 ? C::C1 : C::HP) + o
                            : slot + C::dw_off(NL) + 32 * C::HP + (i - NL * C::HP);
      *dstb = bacc[i];
      bacc[i] = 0.f;
    }
  };

  // Accumulate this wave's dW blocks of layer li (0 = input layer, NL = output layer)
  // from the staged delta and activation rows.
  auto accumulate = [&](auto li_c) {
    constexpr int li = decltype(li_c)::value;
    constexpr int off = B::blk_off(li), cnt = B::blk_cnt(li), nnb = B::blk_cols(li);
    constexpr int q0 = off / kWaves, q1 = (off + cnt - 1) / kWaves;
    float* bl = bacc + li * C::HP;
    const int h = lane / 32, r = lane % 32;
    if constexpr (B::QUAD(nnb)) {
      // the wave's 2x2 quadrant: delta row blocks mb0, mb0 + 1 x activation column blocks
      // nb0, nb0 + 1 (dwacc[q0 .. q0 + 3] in blk_rc order)
      static_assert(off % kWaves == 0 && cnt == 4 * kWaves, "quadrant layout");
      const int mb0 = 2 * (wave_u / 2), nb0 = 2 * (wave_u % 2);
      bf16x8 a0[4], a1[4], b0[4], b1[4];
      dw_tr_operand<B>(dst, mb0, lane, a0);
      dw_tr_operand<B>(hst, nb0, lane, b0);
      dw_tr_operand<B>(hst, nb0 + 1, lane, b1);
      dw_tr_operand<B>(dst, mb0 + 1, lane, a1);
      dw_mma_bf16<C>(a0, b0, dwacc[q0]);
      dw_mma_bf16<C>(a0, b1, dwacc[q0 + 1]);
      dw_mma_bf16<C>(a1, b0, dwacc[q0 + 2]);
      dw_mma_bf16<C>(a1, b1, dwacc[q0 + 3]);
      // the bias sums of the wave's own row block (mb0 + wave % 2 = wave)
      if (wave_u % 2) bsr[li] += dw_rowsum_bf16(a1);
      else bsr[li] += dw_rowsum_bf16(a0);
      (void)bl; (void)h; (void)r;
      return;
    } else if constexpr (B::STRIP(nnb)) {
      // the wave's row block mb = wave against every activation column block; the next
      // column operand is read while the current block's MFMAs run
      static_assert(off % kWaves == 0 && cnt == nnb * kWaves, "strip layout");
      bf16x8 a[4], b[2][4];
      dw_tr_operand<B>(dst, wave_u, lane, a);
      dw_tr_operand<B>(hst, 0, lane, b[0]);
#pragma unroll
      for (int k = 0; k < nnb; ++k) {
        if (k + 1 < nnb) dw_tr_operand<B>(hst, k + 1, lane, b[(k + 1) & 1]);
        DPD_KEEP_LOADS_LOCAL();
        dw_mma_bf16<C>(a, b[k & 1], dwacc[q0 + k]);
      }
      bsr[li] += dw_rowsum_bf16(a);
      (void)bl; (void)h; (void)r;
      return;
    } else if constexpr (B::SM) {
      // the operands of the wave's next block are read while this block's MFMAs run
      DwOps ops[2];
      auto valid = [&](int q) { const int bi = kWaves * q + wave_u; return bi >= off && bi < off + cnt; };
      auto load = [&](int q, DwOps& o) {
        int mb, nb;
        B::blk_rc(kWaves * q + wave_u - off, nnb, mb, nb);
        dw_load_bf16<C, B>(dst, hst, mb, nb, lane, o);
      };
      if (valid(q0)) load(q0, ops[0]);
#pragma unroll
      for (int q = q0; q <= q1; ++q) {
        if (q + 1 <= q1 && valid(q + 1)) load(q + 1, ops[(q + 1 - q0) & 1]);
        DPD_KEEP_LOADS_LOCAL();
        if (valid(q)) {
          const DwOps& o = ops[(q - q0) & 1];
          dw_mma_bf16<C>(o, dwacc[q]);
          int mb, nb;
          B::blk_rc(kWaves * q + wave_u - off, nnb, mb, nb);
          if (nb == 0) {
            const float sum = dw_rowsum_bf16(o.a);
            if (h == 0) bl[32 * mb + r] += sum;
          }
        }
      }
      return;
    }
#pragma unroll
    for (int q = q0; q <= q1; ++q) {
      DPD_KEEP_LOADS_LOCAL();
      const int bi = kWaves * q + wave_u;
      if (bi >= off && bi < off + cnt) {
        int mb, nb;
        B::blk_rc(bi - off, nnb, mb, nb);
        {
          dwacc[q] = dw_block<C, B>(dst, hst, mb, nb, lane, dwacc[q]);
          if (nb == 0) {
            const float sum = delta_row_sum<C, B>(dst, mb, lane);
            if (h == 0) bl[32 * mb + r] += sum;
          }
        }
      }
    }
  };

  // the x window and g_u of the next tile are read one tile ahead, into registers, and the
  // window is stored to its LDS buffer at the end of the current tile
  static_assert(B::XW <= kThreads, "one x-window element per thread");
  float2 xpre = make_float2(0.f, 0.f), gpre = make_float2(0.f, 0.f), gcur = gpre;
  // stream of the last prefetched tile and its bounds, advanced only when a tile of a
  // later stream is prefetched (no per-tile lookups in the stream table)
  int ps = t_begin < t_end ? stream_of_tile(st, t_begin) : 0;
  int64_t p_lo = st.off[ps], p_hi = st.off[ps + 1];
  int p_t0 = st.tile0[ps], p_t1 = st.tile0[ps + 1];
  auto prefetch = [&](int tt) {
    if (tt >= p_t1) {                  // tile0[n] = n_tiles > tt ends the scan
      do { ++ps; } while (tt >= st.tile0[ps + 1]);
      p_lo = st.off[ps];
      p_hi = st.off[ps + 1];
      p_t0 = st.tile0[ps];
      p_t1 = st.tile0[ps + 1];
    }
    const int64_t lo2 = p_lo, hi2 = p_hi;
    const int64_t t02 = lo2 + (int64_t)(tt - p_t0) * S;
    const int64_t p = t02 - B::XB + tid;
    xpre = (tid < B::XW && p >= lo2 && p < hi2) ? ld2(x, p) : make_float2(0.f, 0.f);
    const int64_t n2 = t02 + C::MT * wave_u + (tid % 64) % C::MT;
    gpre = n2 < hi2 ? ld2(gu, n2) : make_float2(0.f, 0.f);
  };
  if (t_begin < t_end) {
    prefetch(t_begin);
    if constexpr (NXB == 2) {
      if (tid < B::XW) xw[t_begin % 2][tid] = xpre;
      gcur = gpre;
    }
  }

  // bf16: the hidden activations come from the forward's store (group 4 t + wave of tile
  // t) instead of a recompute; h_NL of the next tile is read as soon as its registers free
  // up, the other layers at the top of the tile (they are needed a phase later)
  constexpr bool kAct = B::SM;
  Ops<C, C::NKSH> hb[NL];
  auto load_hb = [&](int tt, int i) {
    if constexpr (kAct) {
      int ln = tid;
      asm volatile("" : "+v"(ln));
      const act_u32x4* srca = act + ((int64_t)tt * kWaves + wave_u) * (NL * C::NKSH * 64) + ln % 64 +
                              (int64_t)i * C::NKSH * 64;
#pragma unroll
      for (int ks = 0; ks < C::NKSH; ++ks)
        hb[i][ks] = __builtin_bit_cast(A, __builtin_nontemporal_load(srca + ks * 64));
    }
  };
  if constexpr (kAct)
    if (t_begin < t_end) load_hb(t_begin, NL - 1);
  int cur_stream = -1;
  for (int t = t_begin; t < t_end; ++t) {
    const int s = ps;                  // tile t was the last one prefetched
    const int set = st.per_stream ? s : 0;
    const char* pk = pack + set * C::PACK;
    int tq = tid;
    asm volatile("" : "+v"(tq));
    lane = tq % 64;
    const int g = lane / C::MT, sl = lane % C::MT;
    const int col = C::MT * wave_u + sl;

    __syncthreads();   // previous tile finished with every LDS buffer; this tile's x window stored
    if (s != cur_stream) {
      if (cur_stream >= 0) flush(cur_stream);
      // a new stream may bring a new parameter set: stage its vector block and weights
      const float* src = reinterpret_cast<const float*>(pk + C::OFF_VEC);
      for (int i = tid; i < C::NVEC; i += kThreads) vec[i] = src[i];
      if constexpr (B::W_HI > B::W_LO) {
        const uint4* wsrc = reinterpret_cast<const uint4*>(pk + B::W_LO);
        for (int i = tid; i < (int)(B::W_BYTES / 16); i += kThreads) wlds[i] = wsrc[i];
      }
      cur_stream = s;
      if constexpr (NXB == 2) __syncthreads();
    }
    if constexpr (NXB == 1) {
      if (tid < B::XW) xw[0][tid] = xpre;
      gcur = gpre;
    }
    const float2 gsum = gcur;          // g_u of this lane's sample (zero past the stream)
    if (t + 1 < t_end) prefetch(t + 1);
    if constexpr (NXB == 1) __syncthreads();
    const float2* xwt = xw[t % NXB];

    // ---- TDNN: this wave's hidden activations (stored, or recomputed), then the reverse mode
    const A* wfwd = B::W_FWD ? reinterpret_cast<const A*>(wlds) : reinterpret_cast<const A*>(pk);
    const A* wbwd = B::W_BWD ? reinterpret_cast<const A*>(reinterpret_cast<const char*>(wlds) + (C::OFF_BWDH - B::W_LO))
                             : reinterpret_cast<const A*>(pk + C::OFF_BWDH);
    if constexpr (kAct) {
#pragma unroll
      for (int i = 0; i < NL - 1; ++i) load_hb(t, i);
    } else {
      (void)mlp_forward<C, NL, RT>(wfwd, reinterpret_cast<const A*>(pk + C::OFF_WO), vec, lane, g,
                                           &xwt[col + B::XB], hb, tn);
    }
    (void)wfwd;
    int lb[2];
    B::lane_bases(g, col, lb);
    // output layer: delta_o = (Re g_u, Im g_u) (bf16: its own [2][S] array; fp32: staging
    // rows 0 and 1)
    if (g == 0) {
      if constexpr (B::SM) {
        dsto[col] = (__bf16)gsum.x;
        dsto[S + col] = (__bf16)gsum.y;
      } else {
        dst[B::off(0, col)] = (E)gsum.x;
        dst[B::off(1, col)] = (E)gsum.y;
      }
    }
    stage_layer<C, B, C::NKSH>(hst, lb, hb[NL - 1]);
    __syncthreads();
    if constexpr (B::SM) {
      // output-layer dW on the matrix cores: wave w takes neurons 32 w .. 32 w + 31 of
      // h_NL; A rows 0, 1 = delta_o (other rows zero), so rows 0 and 1 of the product are
      // dW_o for those columns (accumulator values 0 and 1 of lanes 0..31)
      if (wave_u < C::NBD) {
        bf16x8 bop[4], aop[4];
        dw_tr_operand<B>(hst, wave_u, lane, bop);
        const int r = lane % 32, h = lane / 32;
#pragma unroll
        for (int ks = 0; ks < 4; ++ks) {
          bf16x8 z;
#pragma unroll
          for (int e = 0; e < 8; ++e) z[e] = (__bf16)0.f;
          aop[ks] = r < 2 ? *reinterpret_cast<const bf16x8*>(dsto + r * S + 16 * ks + 8 * h) : z;
        }
        f32x16 tmp;
#pragma unroll
        for (int j = 0; j < 16; ++j) tmp[j] = 0.f;
#pragma unroll
        for (int ks = 0; ks < 4; ++ks) tmp = C::D::mma(aop[ks], bop[ks], tmp);
        if (h == 0) {
          dwo += tmp[0];
          dwo1 += tmp[1];
        }
        if (wave_u == 0) {        // output-layer bias: rows 0 and 1 summed over the samples
          const float sum = dw_rowsum_bf16(aop);
          if constexpr (B::BREG) bsr[NL] += sum;
          else if (h == 0 && r < 2) bacc[NL * C::HP + r] += sum;
        }
      }
    } else if (tid < 2 * C::HP) {
      // fp32: output-layer dW element (c, n) += sum_s delta_o[c][s] h_NL[n][s]; bias by n == 0
      const int c = tid / C::HP, n = tid % C::HP;
      float acc = 0.f, bsum = 0.f;
#pragma unroll 2
      for (int k = 0; k < S; k += 4) {
        const float4 da = *reinterpret_cast<const float4*>(dst + B::off(c, k));
        const float4 hv = *reinterpret_cast<const float4*>(hst + B::off(n, k));
        acc = fmaf(da.x, hv.x, fmaf(da.y, hv.y, fmaf(da.z, hv.z, fmaf(da.w, hv.w, acc))));
        bsum += (da.x + da.y) + (da.z + da.w);
      }
      dwo += acc;
      if (n == 0) bacc[NL * C::HP + c] += bsum;
    }
    // delta_NL = (Wo^T delta_o) * (1 - h_NL^2)
    Ops<C, C::NKSH> db;
    {
      const float* wo = vec + NL * C::HP;
#pragma unroll
      for (int mb = 0; mb < C::NB; ++mb)
#pragma unroll
        for (int j = 0; j < C::NR; ++j) {
          const float hv = value_at<C, C::NKSH>(hb[NL - 1], mb, j);
          const int vi = (mb * C::LG + g) * C::NR + j;
          const float v = (wo[vi] * gsum.x + wo[C::HP + vi] * gsum.y) * (1.f - hv * hv);
          set_elem<C>(db[X::ks_of(mb, j)], X::e_of(mb, j), v);
        }
      opaque_ops<C, C::NKSH>(db);
    }
    if constexpr (kAct)
      if (t + 1 < t_end) load_hb(t + 1, NL - 1);
    auto layer = [&](auto i_c) {       // hidden layer i: delta_i in db, input h_{i-1}
      constexpr int i = decltype(i_c)::value;
      __syncthreads();                 // staging free
      stage_layer<C, B, C::NKSH>(dst, lb, db);
      if constexpr (i >= 2) {
        stage_layer<C, B, C::NKSH>(hst, lb, hb[i - 2]);
      } else {
        // features at their natural rows: lane group g holds rows [g*FPG, g*FPG + FPG)
        Ops<C, C::NKS1> feat;
        make_features<C, RT>(&xwt[col + B::XB], g, feat, tn);
        if constexpr (B::SM && C::FPG % 4 == 0) {
          // 4 consecutive features per 8-byte write; chunks of the padding rows zeroed by
          // lane group 0
#pragma unroll
          for (int f = 0; f < C::FPG; f += 4) {
            const int k = C::FPG * g + f;
            const uint4 w = __builtin_bit_cast(uint4, feat[f / 8]);
            const uint2 v = (f / 4) % 2 ? make_uint2(w.z, w.w) : make_uint2(w.x, w.y);
            if (k < C::KIN) *reinterpret_cast<uint2*>(hst + B::off(k, col)) = v;
          }
          if (g == 0) {
#pragma unroll
            for (int k = C::KIN; k < C::C1; k += 4) *reinterpret_cast<uint2*>(hst + B::off(k, col)) = make_uint2(0, 0);
          }
        } else {
#pragma unroll
          for (int ks = 0; ks < C::NKS1; ++ks)
#pragma unroll
            for (int e = 0; e < X::EPL; ++e) {
              const int f = X::EPL * ks + e;
              const int k = C::FPG * g + f;
              if (f < C::FPG && k < C::KIN) hst[B::off(k, col)] = (E)get_elem<C>(feat[ks], e);
            }
#pragma unroll
          for (int k = C::KIN; k < C::C1; ++k)
            if (k % C::LG == g) hst[B::off(k, col)] = (E)0.f;
        }
      }
      // delta_{i-1} = (W_i^T delta_i) * (1 - h_{i-1}^2) while the staging settles
      Ops<C, C::NKSH> dn;
      if constexpr (i >= 2) {
        auto epi = [&](int mb, const typename X::Acc& acc) {
#pragma unroll
          for (int j = 0; j < C::NR; ++j) {
            const float hv = value_at<C, C::NKSH>(hb[i - 2], mb, j);
            set_elem<C>(dn[X::ks_of(mb, j)], X::e_of(mb, j), acc[j] * (1.f - hv * hv));
          }
        };
        const A* Ab = wbwd + (int64_t)(i - 2) * C::NB * C::NKSH * 64;
        dense_layer<C, C::NKSH>(PackedA<C, C::NKSH>{Ab, lane}, [&](int ks) { return db[ks]; }, epi);
        opaque_ops<C, C::NKSH>(dn);
      }
      __syncthreads();
      accumulate(std::integral_constant<int, i - 1>{});
      if constexpr (i >= 2) {
#pragma unroll
        for (int ks = 0; ks < C::NKSH; ++ks) db[ks] = dn[ks];
      }
    };
    static_assert(NL >= 1 && NL <= 4, "hidden layer count of the tuned kernel");
    if constexpr (NL >= 4) layer(std::integral_constant<int, 4>{});
    if constexpr (NL >= 3) layer(std::integral_constant<int, 3>{});
    if constexpr (NL >= 2) layer(std::integral_constant<int, 2>{});
    layer(std::integral_constant<int, 1>{});
    if (NXB == 2 && t + 1 < t_end) {   // the next tile's x window (its buffer was last read by tile t - 1)
      if (tid < B::XW) xw[(t + 1) % NXB][tid] = xpre;
      gcur = gpre;
    }
  }
  __syncthreads();
  if (cur_stream >= 0) flush(cur_stream);
}

// ------------------------------------------------------------------ dW finalize
// dw[set][packed j] = inv_r[set] * sum over (stream s of set, workgroup g touching s)
// of slot[g + s] at the natural position of j (model of tn taps and width hn).  Fixed
// order: the (s ascending, g ascending) list of slots is cut into kFinChunks consecutive
// chunks; each thread of a column sums one chunk in list order, and the chunk sums are
// added in chunk order.  A workgroup covers kFinCols packed indices.
constexpr int kFinCols = 32, kFinChunks = 8;
template <int PREC, int T, int H, int NL>
__global__ __launch_bounds__(kFinCols * kFinChunks) void k_dw_finalize(StreamTable st, int G_wg,
                                                                     const float* __restrict__ slots,
                                                                     const float* __restrict__ inv_r,
                                                                     int64_t P, int tn, int hn,
                                                                     float* __restrict__ dw) {
  using C = Cfg<PREC, T, H, NL>;
  __shared__ float part[kFinChunks][kFinCols];
  const int set = blockIdx.y;
  const int e = threadIdx.x % kFinCols, c = threadIdx.x / kFinCols;
  const int64_t j = (int64_t)blockIdx.x * kFinCols + e;
  int64_t nat = -1;
  float lscale = 1.f;   // 1 / WS^(NL - 1 - li): the delta-chain scale of layer li
  if (j < P) {
    int64_t pos = 0;
    int din = 5 * tn;
    for (int li = 0; li <= NL && nat < 0; ++li) {
      const int dout = li == NL ? 2 : hn;
      const int cols = li == 0 ? C::C1 : C::HP;
      const int rows = li == NL ? 32 : C::HP;
      const int64_t nw = (int64_t)dout * din;
      if (j < pos + nw) {
        const int64_t r = j - pos;
        const int o = (int)(r / din), k = (int)(r % din);
        nat = C::dw_off(li) + (int64_t)o * cols + k;
      } else if (j < pos + nw + dout) {
        const int o = (int)(j - pos - nw);
        nat = C::dw_off(li) + (int64_t)rows * cols + o;
      }
      if (nat >= 0)
        for (int q = li; q < NL - 1; ++q) lscale *= 1.0f / C::WS;
      pos += nw + dout;
      din = hn;
    }
  }
  // this thread's chunk [lo, hi) of the set's slot list
  int64_t total = 0;
  for (int s = 0; s < st.n; ++s) {
    if ((st.per_stream ? s : 0) != set) continue;
    total += wg_of_tile(st.tile0[s + 1] - 1, G_wg, st.n_tiles) - wg_of_tile(st.tile0[s], G_wg, st.n_tiles) + 1;
  }
  const int64_t lo = total * c / kFinChunks, hi = total * (c + 1) / kFinChunks;
  float acc = 0.f;
  if (nat >= 0) {
    int64_t idx = 0;
    for (int s = 0; s < st.n && idx < hi; ++s) {
      if ((st.per_stream ? s : 0) != set) continue;
      const int g0 = wg_of_tile(st.tile0[s], G_wg, st.n_tiles);
      const int g1 = wg_of_tile(st.tile0[s + 1] - 1, G_wg, st.n_tiles);
      const int64_t n = g1 - g0 + 1;
      const int64_t a = lo > idx ? lo : idx, b = hi < idx + n ? hi : idx + n;
      for (int64_t q = a; q < b; ++q) acc += slots[(int64_t)(g0 + (q - idx) + s) * C::SLOT + nat];
      idx += n;
    }
  }
  part[c][e] = acc;
  __syncthreads();
  if (c == 0 && j < P) {
    float t = part[0][e];
#pragma unroll
    for (int c2 = 1; c2 < kFinChunks; ++c2) t += part[c2][e];
    dw[set * P + j] = t * (inv_r[set] * lscale);
  }
}

SrcOff src_offsets(int T, int H, int NL) {
  SrcOff so;
  int64_t pos = 0;
  int din = 5 * T;
  for (int i = 0; i <= NL; ++i) {
    const int dout = i == NL ? 2 : H;
    so.w[i] = pos;
    pos += (int64_t)dout * din;
    so.b[i] = pos;
    pos += dout;
    din = H;
  }
  return so;
}

// Launchers of one compiled shape.  RT: a generic instantiation (T and H are the compiled
// bounds; the model's tap count and width td.taps <= T, td.hidden <= H come at run time).
template <int PREC, int T, int H, int NL, bool RT>
struct TdnnShape {
  using C = Cfg<PREC, T, H, NL>;

  static void dims(TdnnDims* td) {
    td->kin = 5 * td->taps;
    td->hp = C::HP;
    td->kin_p = C::KIN_P;
    td->nks1 = C::NKS1;
    td->nksh = C::NKSH;
    td->tile = C::S;
    td->fwd_mt = C::MT;
    td->fwd_waves = fwd_waves(PREC, C::HP);
    td->fwd_tile = C::MT * td->fwd_waves;
    td->pack_bytes = C::PACK;
    td->fwd_lds = (C::OFF_BWDH <= 144 * 1024 ? C::OFF_BWDH : 16) + 8 * (td->fwd_tile + T) + 4 * C::NVEC;
    td->dw_slot = C::SLOT;
    td->act_group = PREC == DPD_BF16 ? (int64_t)NL * C::NKSH * 64 * 16 : 0;
  }

  static void pack(const TdnnDims& td, const float* w, int n_sets, int64_t w_stride, void* pk, hipStream_t s) {
    const SrcOff so = src_offsets(td.taps, td.hidden, NL);
    dim3 grid(64, n_sets);
    k_pack<PREC, T, H, NL><<<grid, 256, 0, s>>>(w, w_stride, so, td.taps, td.hidden, static_cast<char*>(pk));
  }

  static void fwd(const TdnnDims& td, const StreamTable& st, const float* x, const void* pk, float* u,
                  int grid, int waves, void* act, hipStream_t s) {
    auto go = [&]<int FW>() {
      static_assert(FW % 4 == 0, "forward tiles cover whole reverse-mode tiles");
      k_tdnn_fwd<PREC, T, H, NL, FW, RT><<<grid, 64 * FW, 0, s>>>(st, x, static_cast<const char*>(pk),
                                                                  td.residual, td.taps, u,
                                                                  static_cast<act_u32x4*>(act));
    };
    if (waves == 16) go.template operator()<16>();
    else if (waves == 12) go.template operator()<12>();
    else go.template operator()<8>();
  }

  static void bwd(const TdnnDims& td, const StreamTable& st, const float* x, const float* gu, const void* pk,
                  float* slots, int grid, const void* act, hipStream_t s) {
    k_tdnn_bwd<PREC, T, H, NL, RT><<<grid, kThreads, 0, s>>>(st, x, gu, static_cast<const char*>(pk),
                                                             td.taps, slots, static_cast<const act_u32x4*>(act));
  }

  static void finalize(const TdnnDims& td, const StreamTable& st, int grid, const float* slots,
                       const float* inv_r_set, float* dw, hipStream_t s) {
    const int64_t P = (int64_t)td.hidden * (5 * td.taps) + td.hidden +
                      (int64_t)(NL - 1) * ((int64_t)td.hidden * td.hidden + td.hidden) + 2 * (int64_t)td.hidden + 2;
    const int n_sets = st.per_stream ? st.n : 1;
    dim3 g2((unsigned)((P + kFinCols - 1) / kFinCols), n_sets);
    k_dw_finalize<PREC, T, H, NL><<<g2, kFinCols * kFinChunks, 0, s>>>(st, grid, slots, inv_r_set, P, td.taps,
                                                                     td.hidden, dw);
  }

  static constexpr TdnnKernels table{&dims, &pack, &fwd, &bwd, &finalize};
};

}  // namespace

}  // namespace dpdmi
