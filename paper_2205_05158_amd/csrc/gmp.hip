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

template <int K, int M, int L>
__global__ __launch_bounds__(kGmpThreads) void k_gmp_fwd(StreamTable st, const float* __restrict__ u,
                                                         const float* __restrict__ coef,
                                                         float* __restrict__ y) {
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
  const float* cs = coef + (st.per_stream ? (int64_t)s * 2 * G::J : 0);
  for (int j = threadIdx.x; j < G::J; j += S) cf[j] = make_float2(cs[2 * j], cs[2 * j + 1]);
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

}  // namespace

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
  if (!ok) {
    int64_t J = (int64_t)g.K * (g.M + 1) + 2 * (int64_t)(g.K - 1) * (g.M + 1) * g.L;
    for (int i = 0; i < st.n; ++i)
      launch_plain_gmp_fwd(u, st.off[i], st.off[i + 1], coef + (st.per_stream ? i * 2 * J : 0), g.K,
                           g.M, g.L, y, s);
  }
}

}  // namespace dpdmi
