// GMP power-amplifier model of eq. (9) on LDS windows, with compile-time (K, M, L).
//
// Factorisation used by the kernels: for each position p and memory tap l,
//   Q_l(p) = sum_k a_{k,l} r[p]^k + sum_g ( sum_{k>=1} b_{k,l,g} r[p-g]^k
//                                         + sum_{k>=1} c_{k,l,g} r[p+g]^k ),
// r = |u|, so that eq. (9) reads  y[n] = sum_l u[n-l] Q_l(n-l).
// Reverse mode (real convention g_z = dL/dRe z + j dL/dIm z) for one sample m:
//   g_u[m] = sum_l conj(Q_l(m)) g_y[m+l]                                   (u[m] multiplied)
//          + unit(u[m]) * s1 + u[m] * s2                                   (u[m] in an envelope)
//   s1 = sum Re(w C_1),  s2 = sum Re(w sum_{k>=2} k C_k r[m]^{k-2})
// over the monomial families with envelope sample m: a_l (w = conj(g_y[m+l]) u[m]),
// b_{l,g} (w = conj(g_y[m+l+g]) u[m+g]), c_{l,g} (w = conj(g_y[m+l-g]) u[m-g]);
// unit(u) = u/|u|, taken as 0 at u = 0.
#pragma once

#include "common.hpp"

namespace dpdmi {

template <int K, int M, int L>
struct Gmp {
  static constexpr int KA = K * (M + 1);
  static constexpr int KB = (K - 1) * (M + 1) * L;
  static constexpr int J = KA + 2 * KB;
  __host__ __device__ static constexpr int ia(int k, int l) { return k * (M + 1) + l; }
  __host__ __device__ static constexpr int ib(int k, int l, int g) {
    return KA + ((k - 1) * (M + 1) + l) * L + (g - 1);
  }
  __host__ __device__ static constexpr int ic(int k, int l, int g) {
    return KA + KB + ((k - 1) * (M + 1) + l) * L + (g - 1);
  }
  // power of k of the coefficient at packed index j (for the derivative table)
  __host__ __device__ static constexpr int order(int j) {
    return j < KA ? j / (M + 1) : ((j - KA) % KB) / ((M + 1) * L) + 1;
  }
  // The kernels' coefficient order: per memory tap l, the K coefficients of a_{.,l}, then
  // per lag g the K - 1 coefficients of b_{.,l,g} and those of c_{.,l,g}, so that every
  // Horner chain reads one contiguous run (a few wide scalar loads instead of one load
  // per coefficient).
  static constexpr int P = K + 2 * L * (K - 1);
  __host__ __device__ static constexpr int ta(int k, int l) { return l * P + k; }
  __host__ __device__ static constexpr int tb(int k, int l, int g) {
    return l * P + K + 2 * (g - 1) * (K - 1) + (k - 1);
  }
  __host__ __device__ static constexpr int tc(int k, int l, int g) { return tb(k, l, g) + (K - 1); }
  // position in the kernels' order of the coefficient at packed index j
  __host__ __device__ static constexpr int tpos(int j) {
    if (j < KA) return ta(j / (M + 1), j % (M + 1));
    const bool fc = j >= KA + KB;
    const int r = j - KA - (fc ? KB : 0);   // ((k - 1)(M + 1) + l) L + g - 1
    const int g = r % L + 1, kl = r / L, l = kl % (M + 1), k = kl / (M + 1) + 1;
    return fc ? tc(k, l, g) : tb(k, l, g);
  }
};

__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ float2 cmulc(float2 a, float2 b) {   // conj(a) * b
  return make_float2(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x);
}
__device__ __forceinline__ float2 cfma_r(float2 acc, float r, float2 c) {   // acc * r + c
  return make_float2(fmaf(acc.x, r, c.x), fmaf(acc.y, r, c.y));
}

// Q_l(p) for l = L0..L1-1 (default: all taps); cf holds the coefficients in the kernels'
// order (Gmp::tpos); rw points at r[p] inside a window that
// covers p-L..p+L.
template <int K, int M, int L, int L0 = 0, int L1 = M + 1>
__device__ __forceinline__ void gmp_q(const float* rw, const float2* cf, float2 (&Q)[M + 1]) {
  using G = Gmp<K, M, L>;
  float r0 = rw[0];
  float rl[L + 1], rr[L + 1];
#pragma unroll
  for (int g = 1; g <= L; ++g) {
    rl[g] = rw[-g];
    rr[g] = rw[g];
  }
#pragma unroll
  for (int l = L0; l < L1; ++l) {
    DPD_KEEP_LOADS_LOCAL();
    float2 acc = cf[G::ta(K - 1, l)];
#pragma unroll
    for (int k = K - 2; k >= 0; --k) acc = cfma_r(acc, r0, cf[G::ta(k, l)]);
    if (K > 1) {
#pragma unroll
      for (int g = 1; g <= L; ++g) {
        DPD_KEEP_LOADS_LOCAL();
        float2 hb = cf[G::tb(K - 1, l, g)];
#pragma unroll
        for (int k = K - 2; k >= 1; --k) hb = cfma_r(hb, rl[g], cf[G::tb(k, l, g)]);
        float2 hc = cf[G::tc(K - 1, l, g)];
#pragma unroll
        for (int k = K - 2; k >= 1; --k) hc = cfma_r(hc, rr[g], cf[G::tc(k, l, g)]);
        acc.x = fmaf(hb.x, rl[g], fmaf(hc.x, rr[g], acc.x));
        acc.y = fmaf(hb.y, rl[g], fmaf(hc.y, rr[g], acc.y));
      }
    }
    Q[l] = acc;
  }
}

// sum_{k>=2} k C_k r^{k-2} by Horner on the table dcf[j] = order(j) * cf[j].
template <int K, int M, int L, int FAM>
__device__ __forceinline__ float2 gmp_d2(const float2* dcf, int l, int g, float r) {
  using G = Gmp<K, M, L>;
  auto idx = [&](int k) { return FAM == 0 ? G::ta(k, l) : (FAM == 1 ? G::tb(k, l, g) : G::tc(k, l, g)); };
  float2 acc = make_float2(0.f, 0.f);
  if (K >= 3) {
    acc = dcf[idx(K - 1)];
#pragma unroll
    for (int k = K - 2; k >= 2; --k) acc = cfma_r(acc, r, dcf[idx(k)]);
  }
  return acc;
}

// Backward contribution at sample m of the memory taps l = L0..L1-1 (default: all;
// the full gradient is the sum over a partition of the taps).
//   uw, rw: u and |u| at m inside a window covering m-L..m+L
//   gyw: g_y at m inside a window covering m-L..m+M+L
//   Qm: Q_l(m) (entries L0..L1-1 used)
template <int K, int M, int L, int L0 = 0, int L1 = M + 1>
__device__ __forceinline__ float2 gmp_grad(const float2* uw, const float* rw, const float2* gyw,
                                           const float2 (&Qm)[M + 1], const float2* cf,
                                           const float2* dcf) {
  using G = Gmp<K, M, L>;
  float2 um = uw[0];
  float r = rw[0];
  float inv = r > 0.f ? __builtin_amdgcn_rcpf(r) : 0.f;
  float2 unit = make_float2(um.x * inv, um.y * inv);
  float2 gu = make_float2(0.f, 0.f);
  float s1 = 0.f, s2 = 0.f;
#pragma unroll
  for (int l = L0; l < L1; ++l) {
    DPD_KEEP_LOADS_LOCAL();
    float2 gyl = gyw[l];
    float2 t = cmulc(Qm[l], gyl);
    gu.x += t.x;
    gu.y += t.y;
    if (K > 1) {
      float2 w = cmulc(gyl, um);                         // conj(g_y[m+l]) u[m]
      float2 c1 = cf[G::ta(1, l)];
      s1 += w.x * c1.x - w.y * c1.y;
      float2 d = gmp_d2<K, M, L, 0>(dcf, l, 0, r);
      s2 += w.x * d.x - w.y * d.y;
#pragma unroll
      for (int g = 1; g <= L; ++g) {
        DPD_KEEP_LOADS_LOCAL();
        float2 wb = cmulc(gyw[l + g], uw[g]);            // conj(g_y[m+l+g]) u[m+g]
        float2 cb = cf[G::tb(1, l, g)];
        s1 += wb.x * cb.x - wb.y * cb.y;
        float2 db = gmp_d2<K, M, L, 1>(dcf, l, g, r);
        s2 += wb.x * db.x - wb.y * db.y;
        float2 wc = cmulc(gyw[l - g], uw[-g]);           // conj(g_y[m+l-g]) u[m-g]
        float2 cc = cf[G::tc(1, l, g)];
        s1 += wc.x * cc.x - wc.y * cc.y;
        float2 dc = gmp_d2<K, M, L, 2>(dcf, l, g, r);
        s2 += wc.x * dc.x - wc.y * dc.y;
      }
    }
  }
  gu.x += unit.x * s1 + um.x * s2;
  gu.y += unit.y * s1 + um.y * s2;
  return gu;
}

// Orders with no instantiation of their own run on the (9, 7, 4) kernels with their
// coefficients zero-padded to that order (a polynomial with zero leading coefficients,
// taps and lags with zero coefficients change no value for finite inputs).
constexpr int kGmpPadK = 9, kGmpPadM = 7, kGmpPadL = 4;
__host__ inline bool gmp_pad_fits(int K, int M, int L) {
  return K >= 1 && K <= kGmpPadK && M >= 0 && M <= kGmpPadM && L >= 0 && L <= kGmpPadL;
}

// Packed index, in the order (K, M, L), of the monomial at position q of the padded
// (KP, MP, LP) table in the kernels' order, and its power k; -1 where (K, M, L) has none.
template <int KP, int MP, int LP>
__device__ inline int gmp_pad_src(int q, int K, int M, int L, int& k) {
  constexpr int P = Gmp<KP, MP, LP>::P;
  const int l = q / P, r = q % P;
  int g = 0, fam = 0;
  if (r < KP) {
    k = r;
  } else {
    const int r2 = r - KP;
    g = r2 / (2 * (KP - 1)) + 1;
    fam = (r2 % (2 * (KP - 1))) < KP - 1 ? 1 : 2;
    k = r2 % (KP - 1) + 1;
  }
  if (k >= K || l > M || (fam != 0 && g > L)) return -1;
  const int KA = K * (M + 1), KB = (K - 1) * (M + 1) * L;
  return fam == 0 ? k * (M + 1) + l : KA + (fam == 2 ? KB : 0) + ((k - 1) * (M + 1) + l) * L + (g - 1);
}

// Supported (K, M, L) for the tuned kernels; call f.template operator()<K,M,L>().
template <class F>
__host__ bool gmp_dispatch(int K, int M, int L, F&& f) {
  if (K == 5 && M == 3 && L == 2) { f.template operator()<5, 3, 2>(); return true; }
  if (K == 7 && M == 5 && L == 3) { f.template operator()<7, 5, 3>(); return true; }
  if (K == 9 && M == 7 && L == 4) { f.template operator()<9, 7, 4>(); return true; }
  if (K == 7 && M == 3 && L == 1) { f.template operator()<7, 3, 1>(); return true; }
  return false;
}

}  // namespace dpdmi
