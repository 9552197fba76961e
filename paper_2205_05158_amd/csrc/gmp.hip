// Stand-alone GMP PA forward (eq. (9)) over the stream table: one workgroup per
// tile of samples; u and |u| of the tile plus its halo staged in LDS with
// coalesced 8-byte loads; Q_l(p) (all polynomials in |u| around p) computed once
// per position with Horner's rule on coefficients broadcast from LDS; then
// y[n] = sum_l u[n-l] Q_l(n-l).
#include "gmp.hpp"
#include "kernels.hpp"

namespace dpdmi {

namespace {

constexpr int kGmpThreads = 128;

// PAD: the coefficients are of the smaller order (ku, mu, lu), zero-padded into (K, M, L).
template <int K, int M, int L, bool PAD = false>
__global__ __launch_bounds__(kGmpThreads) void k_gmp_fwd(StreamTable st, const float* __restrict__ u,
                                                         const float* __restrict__ coef,
                                                         float* __restrict__ y, int ku = K, int mu = M,
                                                         int lu = L) {
  using G = Gmp<K, M, L>;
  constexpr int S = kGmpThreads;        // samples per tile (st.tile == S)
  constexpr int UB = M + L;             // u halo behind the first output
  constexpr int UW = S + M + 2 * L;     // u window [t0 - M - L, t0 + S + L)
  constexpr int QW = S + M;             // Q window [t0 - M, t0 + S)
  __shared__ float2 cf[G::J];
  __shared__ float2 uw[UW];
  __shared__ float rw[UW];
  __shared__ float2 qw[QW][M + 1];

  int t = blockIdx.x;
  int s = stream_of_tile(st, t);
  int64_t lo = st.off[s], hi = st.off[s + 1];
  int64_t t0 = lo + (int64_t)(t - st.tile0[s]) * S;
  if constexpr (PAD) {
    const int Ju = ku * (mu + 1) + 2 * (ku - 1) * (mu + 1) * lu;
    const float* cs = coef + (st.per_stream ? (int64_t)s * 2 * Ju : 0);
    for (int q = threadIdx.x; q < G::J; q += S) {
      int k;
      const int j = gmp_pad_src<K, M, L>(q, ku, mu, lu, k);
      cf[q] = j >= 0 ? make_float2(cs[2 * j], cs[2 * j + 1]) : make_float2(0.f, 0.f);
    }
  } else {
    const float* cs = coef + (st.per_stream ? (int64_t)s * 2 * G::J : 0);
    for (int j = threadIdx.x; j < G::J; j += S) cf[G::tpos(j)] = make_float2(cs[2 * j], cs[2 * j + 1]);
  }
  for (int i = threadIdx.x; i < UW; i += S) {
    int64_t p = t0 - UB + i;
    float2 v = (p >= lo && p < hi) ? ld2(u, p) : make_float2(0.f, 0.f);
    uw[i] = v;
    rw[i] = sqrtf(v.x * v.x + v.y * v.y);
  }
  __syncthreads();
  for (int i = threadIdx.x; i < QW; i += S) {
    DPD_KEEP_LOADS_LOCAL();
    float2 Q[M + 1];
    gmp_q<K, M, L>(&rw[i + L], cf, Q);     // position t0 - M + i sits at u index i + L
#pragma unroll
    for (int l = 0; l <= M; ++l) qw[i][l] = Q[l];
  }
  __syncthreads();
  int64_t n = t0 + threadIdx.x;
  if (n < hi) {
    int qi = threadIdx.x + M;          // Q index of position n
    int ui = threadIdx.x + UB;         // u index of position n
    float2 acc = make_float2(0.f, 0.f);
#pragma unroll
    for (int l = 0; l <= M; ++l) {
      float2 v = cmul(uw[ui - l], qw[qi - l][l]);
      acc.x += v.x;
      acc.y += v.y;
    }
    st2(y, n, acc);
  }
}

// Per parameter set, the coefficient table read by k_gmp_bwd, in the kernels' order
// (Gmp::tpos): tab[set][tpos(j)] = C_j and tab[set][J + tpos(j)] = order(j) * C_j (the
// coefficients of the envelope derivative).
template <int K, int M, int L>
__global__ void k_gmp_table(const float* __restrict__ coef, float2* __restrict__ tab) {
  using G = Gmp<K, M, L>;
  const int set = blockIdx.y;
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= G::J) return;
  const float* cs = coef + (int64_t)set * 2 * G::J;
  const float2 c = make_float2(cs[2 * j], cs[2 * j + 1]);
  const float k = (float)G::order(j);
  tab[(int64_t)set * 2 * G::J + G::tpos(j)] = c;
  tab[(int64_t)set * 2 * G::J + G::J + G::tpos(j)] = make_float2(k * c.x, k * c.y);
}

// The same table for a smaller order (K, M, L) run on the (KP, MP, LP) kernels: every
// position of the padded table holds the coefficient of the same monomial, or zero where
// the order has none.
template <int KP, int MP, int LP>
__global__ void k_gmp_table_pad(const float* __restrict__ coef, int K, int M, int L, float2* __restrict__ tab) {
  using G = Gmp<KP, MP, LP>;
  const int set = blockIdx.y;
  const int q = blockIdx.x * blockDim.x + threadIdx.x;   // position in the padded table
  if (q >= G::J) return;
  const int J = K * (M + 1) + 2 * (K - 1) * (M + 1) * L;
  int k;
  const int j = gmp_pad_src<KP, MP, LP>(q, K, M, L, k);
  const float* cs = coef + (int64_t)set * 2 * J;
  const float2 c = j >= 0 ? make_float2(cs[2 * j], cs[2 * j + 1]) : make_float2(0.f, 0.f);
  tab[(int64_t)set * 2 * G::J + q] = c;
  tab[(int64_t)set * 2 * G::J + G::J + q] = make_float2((float)k * c.x, (float)k * c.y);
}

// GMP forward and reverse mode over tiles of S samples (one per thread), one workgroup per tile
// (no persistent state, so it runs at the occupancy its registers allow).  The
// coefficients are read from the table (wave-uniform addresses: scalar loads into
// SGPRs, used directly as FMA operands):
//   y = GMP(u) (stored when y_out is not null), g_y = 2 (y - G x) inside the stream,
//   the tile's E = sum |y - G x|^2, R = sum |G x|^2 and count of samples where either
//   square is not finite (fixed reduction tree), and
//   g_u[m] = dL/du[m] of L = sum |y - G x|^2 (the gather form in gmp.hpp).
template <int K, int M, int L, int S>
__global__ __launch_bounds__(S) void k_gmp_bwd(StreamTable st, const float* __restrict__ x,
                                                            const float* __restrict__ u,
                                                            const float2* __restrict__ tab, float g_re,
                                                            float g_im, float4* __restrict__ tile_part,
                                                            float* __restrict__ gu_out,
                                                            float* __restrict__ y_out) {
  using G = Gmp<K, M, L>;
  constexpr int UB = M + 2 * L;
  constexpr int UW = S + 2 * UB;        // u  [t0 - UB, t0 + S + UB)
  constexpr int QB = M + L;
  constexpr int QW = S + 2 * QB;        // Q  [t0 - QB, t0 + S + QB)
  constexpr int YW = S + M + 2 * L;     // gy [t0 - L, t0 + S + M + L), also the x window
  __shared__ float2 uw[UW];
  __shared__ float rw[UW];
  __shared__ float2 xw[YW];
  __shared__ float2 qw[QW][M + 1];
  __shared__ float2 gyw[YW];
  // the E/R reduction tree runs after the reverse mode, in the Q window's memory (5 KB
  // less LDS per workgroup: six workgroups per CU instead of five)
  static_assert(sizeof(float2) * QW * (M + 1) >= 5 * sizeof(float) * S, "tree fits the Q window");
  float* red = reinterpret_cast<float*>(&qw[0][0]);
  uint32_t* redn = reinterpret_cast<uint32_t*>(red + 4 * S);

  const int tid = threadIdx.x;
  const int t = blockIdx.x;
  const int s = stream_of_tile(st, t);
  const int64_t lo = st.off[s], hi = st.off[s + 1];
  const int64_t t0 = lo + (int64_t)(t - st.tile0[s]) * S;
  const float2* cf = tab + (st.per_stream ? (int64_t)s * 2 * G::J : 0);
  const float2* dcf = cf + G::J;
  for (int i = tid; i < UW; i += S) {
    const int64_t p = t0 - UB + i;
    const float2 v = (p >= lo && p < hi) ? ld2(u, p) : make_float2(0.f, 0.f);
    uw[i] = v;
    rw[i] = sqrtf(v.x * v.x + v.y * v.y);
  }
  for (int i = tid; i < YW; i += S) {
    const int64_t p = t0 - L + i;
    xw[i] = (p >= lo && p < hi) ? ld2(x, p) : make_float2(0.f, 0.f);
  }
  __syncthreads();
  // Q_l(p) for every position of the Q window (qw[i] is position t0 - QB + i)
  for (int i = tid; i < QW; i += S) {
    DPD_KEEP_LOADS_LOCAL();
    float2 Q[M + 1];
    gmp_q<K, M, L>(&rw[i + L], cf, Q);
#pragma unroll
    for (int l = 0; l <= M; ++l) qw[i][l] = Q[l];
  }
  __syncthreads();
  // y and g_y on [t0 - L, t0 + S + M + L); E and R on the tile's own samples
  Comp Ec, Rc;
  uint32_t nf = 0;
  for (int i = tid; i < YW; i += S) {
    const int64_t n = t0 - L + i;
    float2 gyv = make_float2(0.f, 0.f);
    if (n >= lo && n < hi) {
      float2 y = make_float2(0.f, 0.f);
#pragma unroll
      for (int l = 0; l <= M; ++l) {
        const float2 v = cmul(uw[i + M + L - l], qw[i + M - l][l]);
        y.x += v.x;
        y.y += v.y;
      }
      const float2 xv = xw[i];
      const float tr = g_re * xv.x - g_im * xv.y, ti = g_re * xv.y + g_im * xv.x;
      const float er = y.x - tr, ei = y.y - ti;
      gyv = make_float2(2.f * er, 2.f * ei);
      if (i >= L && i < L + S) {
        const float e2 = er * er + ei * ei, r2 = tr * tr + ti * ti;
        nf += !isfinite(e2 + r2);
        Ec.add(e2);
        Rc.add(r2);
        if (y_out) st2(y_out, n, y);
      }
    }
    gyw[i] = gyv;
  }
  __syncthreads();
  // g_u at the tile's own samples
  const int64_t m = t0 + tid;
  if (m < hi) {
    float2 Qm[M + 1];
#pragma unroll
    for (int l = 0; l <= M; ++l) Qm[l] = qw[tid + QB][l];
    const float2 gu = gmp_grad<K, M, L>(&uw[tid + UB], &rw[tid + UB], &gyw[tid + L], Qm, cf, dcf);
    st2(gu_out, m, gu);
  }
  __syncthreads();                      // Q window free for the tree
  red[tid] = Ec.s; red[S + tid] = Ec.c; red[2 * S + tid] = Rc.s; red[3 * S + tid] = Rc.c;
  redn[tid] = nf;
  __syncthreads();
  for (int w2 = S / 2; w2 > 0; w2 >>= 1) {
    if (tid < w2) {
      Comp a{red[tid], red[S + tid]}, b{red[2 * S + tid], red[3 * S + tid]};
      a.add(red[tid + w2]); a.add(red[S + tid + w2]);
      b.add(red[2 * S + tid + w2]); b.add(red[3 * S + tid + w2]);
      red[tid] = a.s; red[S + tid] = a.c; red[2 * S + tid] = b.s; red[3 * S + tid] = b.c;
      redn[tid] += redn[tid + w2];
    }
    __syncthreads();
  }
  if (tid == 0) tile_part[t] = make_float4(red[0] + red[S], red[2 * S] + red[3 * S], (float)redn[0], 0.f);
}

}  // namespace

int64_t gmp_table_coeffs(const dpd_gmp_desc& g) {
  int64_t J = 0;
  if (!gmp_dispatch(g.K, g.M, g.L, [&]<int K, int M, int L>() { J = Gmp<K, M, L>::J; }) &&
      gmp_pad_fits(g.K, g.M, g.L))
    J = Gmp<kGmpPadK, kGmpPadM, kGmpPadL>::J;
  return J;
}

void launch_gmp_bwd(const dpd_gmp_desc& g, const StreamTable& st, const float* x, const float* u,
                    const float* coef, float2* tab, float g_re, float g_im, float4* tile_part,
                    float* gu, float* y, hipStream_t s) {
  const int n_sets = st.per_stream ? st.n : 1;
  auto run = [&]<int K, int M, int L>() {
    if (st.tile == 512)
      k_gmp_bwd<K, M, L, 512><<<st.n_tiles, 512, 0, s>>>(st, x, u, tab, g_re, g_im, tile_part, gu, y);
    else
      k_gmp_bwd<K, M, L, 256><<<st.n_tiles, 256, 0, s>>>(st, x, u, tab, g_re, g_im, tile_part, gu, y);
  };
  const bool exact = gmp_dispatch(g.K, g.M, g.L, [&]<int K, int M, int L>() {
    dim3 tg((Gmp<K, M, L>::J + 255) / 256, n_sets);
    k_gmp_table<K, M, L><<<tg, 256, 0, s>>>(coef, tab);
    run.template operator()<K, M, L>();
  });
  if (!exact && gmp_pad_fits(g.K, g.M, g.L)) {
    constexpr int KP = kGmpPadK, MP = kGmpPadM, LP = kGmpPadL;
    dim3 tg((Gmp<KP, MP, LP>::J + 255) / 256, n_sets);
    k_gmp_table_pad<KP, MP, LP><<<tg, 256, 0, s>>>(coef, g.K, g.M, g.L, tab);
    run.template operator()<KP, MP, LP>();
  }
}

void launch_gmp_fwd(const dpd_gmp_desc& g, const StreamTable& st, const float* u, const float* coef,
                    float* y, hipStream_t s) {
  StreamTable t2 = st;
  // re-tile with this kernel's tile
  int32_t tt = 0;
  for (int i = 0; i < st.n; ++i) {
    t2.tile0[i] = tt;
    tt += (int32_t)ceil_div64(st.off[i + 1] - st.off[i], kGmpThreads);
  }
  t2.tile0[st.n] = tt;
  t2.n_tiles = tt;
  t2.tile = kGmpThreads;
  bool ok = gmp_dispatch(g.K, g.M, g.L, [&]<int K, int M, int L>() {
    k_gmp_fwd<K, M, L><<<t2.n_tiles, kGmpThreads, 0, s>>>(t2, u, coef, y);
  });
  if (!ok && gmp_pad_fits(g.K, g.M, g.L)) {
    k_gmp_fwd<kGmpPadK, kGmpPadM, kGmpPadL, true><<<t2.n_tiles, kGmpThreads, 0, s>>>(t2, u, coef, y, g.K, g.M, g.L);
    ok = true;
  }
  if (!ok) {
    int64_t J = (int64_t)g.K * (g.M + 1) + 2 * (int64_t)(g.K - 1) * (g.M + 1) * g.L;
    for (int i = 0; i < st.n; ++i)
      launch_plain_gmp_fwd(u, st.off[i], st.off[i + 1], coef + (st.per_stream ? i * 2 * J : 0), g.K,
                           g.M, g.L, y, s);
  }
}

}  // namespace dpdmi
