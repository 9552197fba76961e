// Plain FP32 path: one thread per output element, activations kept in HBM, no LDS
// tiling and no MFMA.  It is the straightforward GPU reading of the definitions
// (tapped delay line + FC layers, eq. (9), reverse mode) and the comparison
// baseline for the tuned kernels.  The host drives it stream by stream and
// chunk by chunk, so every kernel sees one stream [lo, hi) and one parameter set.
#include "kernels.hpp"

namespace dpdmi {

namespace {

__global__ void k_plain_features(const float* __restrict__ x, int64_t lo, int64_t c0, int cn,
                                 int taps, float* __restrict__ F) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= cn) return;
  int64_t n = c0 + i;
  float* f = F + (int64_t)i * 5 * taps;
  for (int t = 0; t < taps; ++t) {
    float2 z = make_float2(0.f, 0.f);
    if (n - t >= lo) z = ld2(x, n - t);
    float m2 = z.x * z.x + z.y * z.y;
    float m = sqrtf(m2);
    f[5 * t + 0] = z.x;
    f[5 * t + 1] = z.y;
    f[5 * t + 2] = m;
    f[5 * t + 3] = m2;
    f[5 * t + 4] = m2 * m;
  }
}

__global__ void k_plain_dense(const float* __restrict__ in, int din, const float* __restrict__ W,
                              const float* __restrict__ b, float* __restrict__ out, int dout,
                              int cn, int act) {
  int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)cn * dout) return;
  int i = (int)(idx / dout), o = (int)(idx % dout);
  const float* a = in + (int64_t)i * din;
  const float* wr = W + (int64_t)o * din;
  float acc = b[o];
  for (int k = 0; k < din; ++k) acc = fmaf(wr[k], a[k], acc);
  out[idx] = act ? tanhf(acc) : acc;
}

__global__ void k_plain_u(const float* __restrict__ o2, const float* __restrict__ x, int64_t c0,
                          int cn, int residual, float* __restrict__ u) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= cn) return;
  float2 v = make_float2(o2[2 * i], o2[2 * i + 1]);
  if (residual) {
    float2 xv = ld2(x, c0 + i);
    v.x += xv.x;
    v.y += xv.y;
  }
  st2(u, c0 + i, v);
}

// |u[p]| and u[p] with zero outside [lo, hi)
__device__ __forceinline__ float2 u_at(const float* u, int64_t p, int64_t lo, int64_t hi) {
  return (p >= lo && p < hi) ? ld2(u, p) : make_float2(0.f, 0.f);
}

__device__ __forceinline__ float2 coef_at(const float* coef, int j) {
  return make_float2(coef[2 * j], coef[2 * j + 1]);
}

// Index of the coefficient of monomial (family, k, l, g) in the packed layout.
__device__ __forceinline__ int cidx(int fam, int k, int l, int g, int K, int M, int L) {
  if (fam == 0) return k * (M + 1) + l;
  int base = K * (M + 1) + (fam == 2 ? (K - 1) * (M + 1) * L : 0);
  return base + ((k - 1) * (M + 1) + l) * L + (g - 1);
}

__global__ void k_plain_gmp_fwd(const float* __restrict__ u, int64_t lo, int64_t hi,
                                const float* __restrict__ coef, int K, int M, int L,
                                float* __restrict__ y) {
  int64_t n = lo + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= hi) return;
  float yr = 0.f, yi = 0.f;
  for (int l = 0; l <= M; ++l) {
    float2 up = u_at(u, n - l, lo, hi);
    for (int fam = 0; fam < 3; ++fam) {
      int gmax = fam == 0 ? 0 : L;
      for (int g = (fam == 0 ? 0 : 1); g <= gmax; ++g) {
        int d = fam == 0 ? l : (fam == 1 ? l + g : l - g);
        float2 uq = u_at(u, n - d, lo, hi);
        float r = sqrtf(uq.x * uq.x + uq.y * uq.y);
        float rk = 1.f;
        for (int k = 0; k < K; ++k) {
          if (k >= 1 || fam == 0) {
            float2 c = coef_at(coef, cidx(fam, k, l, g, K, M, L));
            float tr = c.x * up.x - c.y * up.y;
            float ti = c.x * up.y + c.y * up.x;
            yr = fmaf(tr, rk, yr);
            yi = fmaf(ti, rk, yi);
          }
          rk *= r;
        }
      }
    }
  }
  st2(y, n, make_float2(yr, yi));
}

// g_u[m] for the real-convention gradient of sum|y - Gx|^2 (unscaled: g_y = 2(y - Gx)).
__global__ void k_plain_gmp_bwd(const float* __restrict__ u, const float* __restrict__ y,
                                const float* __restrict__ x, int64_t lo, int64_t hi,
                                const float* __restrict__ coef, int K, int M, int L, float g_re,
                                float g_im, float* __restrict__ gu) {
  int64_t m = lo + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= hi) return;
  float2 um = ld2(u, m);
  float rm = sqrtf(um.x * um.x + um.y * um.y);
  float2 unit = rm > 0.f ? make_float2(um.x / rm, um.y / rm) : make_float2(0.f, 0.f);
  float gr = 0.f, gi = 0.f;
  for (int l = 0; l <= M; ++l) {
    for (int fam = 0; fam < 3; ++fam) {
      int gmax = fam == 0 ? 0 : L;
      for (int g = (fam == 0 ? 0 : 1); g <= gmax; ++g) {
        int d = fam == 0 ? l : (fam == 1 ? l + g : l - g);
        for (int k = (fam == 0 ? 0 : 1); k < K; ++k) {
          float2 c = coef_at(coef, cidx(fam, k, l, g, K, M, L));
          // (1) m is the multiplied sample p = n - l, output n = m + l
          int64_t n = m + l;
          if (n < hi) {
            float2 yn = ld2(y, n), xn = ld2(x, n);
            float ger = 2.f * (yn.x - (g_re * xn.x - g_im * xn.y));
            float gei = 2.f * (yn.y - (g_re * xn.y + g_im * xn.x));
            float2 uq = u_at(u, n - d, lo, hi);
            float rq = sqrtf(uq.x * uq.x + uq.y * uq.y);
            float rk = powf(rq, (float)k);
            if (k == 0) rk = 1.f;
            // conj(c rk) * g_y
            gr += rk * (c.x * ger + c.y * gei);
            gi += rk * (c.x * gei - c.y * ger);
          }
          // (2) m is the envelope sample q = n - d, output n = m + d
          if (k >= 1) {
            int64_t n2 = m + d;
            if (n2 >= lo && n2 < hi) {
              float2 yn = ld2(y, n2), xn = ld2(x, n2);
              float ger = 2.f * (yn.x - (g_re * xn.x - g_im * xn.y));
              float gei = 2.f * (yn.y - (g_re * xn.y + g_im * xn.x));
              float2 up = u_at(u, n2 - l, lo, hi);
              // Re(conj(g_y) c u_p)
              float cr = c.x * up.x - c.y * up.y, ci = c.x * up.y + c.y * up.x;
              float re = ger * cr + gei * ci;
              float s = (float)k * re;
              if (k == 1) {
                gr += s * unit.x;
                gi += s * unit.y;
              } else {
                float rk2 = powf(rm, (float)(k - 2));
                if (k == 2) rk2 = 1.f;
                gr += s * rk2 * um.x;
                gi += s * rk2 * um.y;
              }
            }
          }
        }
      }
    }
  }
  st2(gu, m, make_float2(gr, gi));
}

__global__ void k_plain_delta_out(const float* __restrict__ gu, int64_t c0, int cn,
                                  float* __restrict__ d) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= cn) return;
  float2 g = ld2(gu, c0 + i);
  d[2 * i] = g.x;
  d[2 * i + 1] = g.y;
}

__global__ void k_plain_dense_bwd(const float* __restrict__ dout, int n_out,
                                  const float* __restrict__ W, const float* __restrict__ hin,
                                  int n_in, float* __restrict__ din, int cn) {
  int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)cn * n_in) return;
  int i = (int)(idx / n_in), k = (int)(idx % n_in);
  float acc = 0.f;
  for (int o = 0; o < n_out; ++o) acc = fmaf(W[(int64_t)o * n_in + k], dout[(int64_t)i * n_out + o], acc);
  float h = hin[idx];
  din[idx] = acc * (1.f - h * h);
}

// part[b][o][k] = sum_{i in block b} dout[i][o] * (k < n_in ? hin[i][k] : 1)
__global__ void k_plain_dw(const float* __restrict__ dout, int n_out,
                           const float* __restrict__ hin, int n_in, int cn, int blk,
                           float* __restrict__ part) {
  int cols = n_in + 1;
  int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n_out * cols) return;
  int o = j / cols, k = j % cols;
  int b = blockIdx.y;
  int i0 = b * blk, i1 = min(cn, i0 + blk);
  float acc = 0.f;
  for (int i = i0; i < i1; ++i) {
    float h = k < n_in ? hin[(int64_t)i * n_in + k] : 1.f;
    acc = fmaf(dout[(int64_t)i * n_out + o], h, acc);
  }
  part[(int64_t)b * n_out * cols + j] = acc;
}

__global__ void k_plain_dw_accum(const float* __restrict__ part, int nblk, int count,
                                 float* __restrict__ acc) {
  int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= count) return;
  float s = acc[j];
  for (int b = 0; b < nblk; ++b) s += part[(int64_t)b * count + j];
  acc[j] = s;
}

// acc layout per set: for each layer, [dout][din + 1] (bias in the last column).
__global__ void k_plain_finalize(const float* __restrict__ acc, int taps, int n_hidden, int hidden,
                                 int64_t acc_stride, int64_t P, const float* __restrict__ inv_r,
                                 float* __restrict__ dw) {
  int set = blockIdx.y;
  int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= P) return;
  // walk the layers to find (layer, o, k) of packed index j
  int64_t pos = 0, apos = 0;
  int din = 5 * taps;
  for (int layer = 0; layer <= n_hidden; ++layer) {
    int dout = layer == n_hidden ? 2 : hidden;
    int64_t nw = (int64_t)dout * din;
    if (j < pos + nw) {
      int64_t r = j - pos;
      int o = (int)(r / din), k = (int)(r % din);
      dw[set * P + j] = acc[set * acc_stride + apos + (int64_t)o * (din + 1) + k] * inv_r[set];
      return;
    }
    pos += nw;
    if (j < pos + dout) {
      int o = (int)(j - pos);
      dw[set * P + j] = acc[set * acc_stride + apos + (int64_t)o * (din + 1) + din] * inv_r[set];
      return;
    }
    pos += dout;
    apos += (int64_t)dout * (din + 1);
    din = hidden;
  }
}

__global__ void k_fill(float* p, int64_t n, float v) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

inline unsigned blocks_for(int64_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }

}  // namespace

void launch_plain_features(const float* x, int64_t lo, int64_t c0, int cn, int taps, float* F,
                           hipStream_t s) {
  k_plain_features<<<blocks_for(cn, 256), 256, 0, s>>>(x, lo, c0, cn, taps, F);
}
void launch_plain_dense(const float* in, int din, const float* W, const float* b, float* out,
                        int dout, int cn, int act, hipStream_t s) {
  k_plain_dense<<<blocks_for((int64_t)cn * dout, 256), 256, 0, s>>>(in, din, W, b, out, dout, cn, act);
}
void launch_plain_u(const float* o2, const float* x, int64_t c0, int cn, int residual, float* u,
                    hipStream_t s) {
  k_plain_u<<<blocks_for(cn, 256), 256, 0, s>>>(o2, x, c0, cn, residual, u);
}
void launch_plain_gmp_fwd(const float* u, int64_t lo, int64_t hi, const float* coef, int K, int M,
                          int L, float* y, hipStream_t s) {
  k_plain_gmp_fwd<<<blocks_for(hi - lo, 256), 256, 0, s>>>(u, lo, hi, coef, K, M, L, y);
}
void launch_plain_gmp_bwd(const float* u, const float* y, const float* x, int64_t lo, int64_t hi,
                          const float* coef, int K, int M, int L, float g_re, float g_im, float* gu,
                          hipStream_t s) {
  k_plain_gmp_bwd<<<blocks_for(hi - lo, 256), 256, 0, s>>>(u, y, x, lo, hi, coef, K, M, L, g_re,
                                                           g_im, gu);
}
void launch_plain_delta_out(const float* gu, int64_t c0, int cn, float* d, hipStream_t s) {
  k_plain_delta_out<<<blocks_for(cn, 256), 256, 0, s>>>(gu, c0, cn, d);
}
void launch_plain_dense_bwd(const float* dout, int n_out, const float* W, const float* hin,
                            int n_in, float* din, int cn, hipStream_t s) {
  k_plain_dense_bwd<<<blocks_for((int64_t)cn * n_in, 256), 256, 0, s>>>(dout, n_out, W, hin, n_in,
                                                                         din, cn);
}
void launch_plain_dw(const float* dout, int n_out, const float* hin, int n_in, int cn, int blk,
                     float* part, hipStream_t s) {
  int nblk = (cn + blk - 1) / blk;
  dim3 grid(blocks_for((int64_t)n_out * (n_in + 1), 256), nblk);
  k_plain_dw<<<grid, 256, 0, s>>>(dout, n_out, hin, n_in, cn, blk, part);
}
void launch_plain_dw_accum(const float* part, int nblk, int count, float* acc, hipStream_t s) {
  k_plain_dw_accum<<<blocks_for(count, 256), 256, 0, s>>>(part, nblk, count, acc);
}
void launch_fill(float* p, int64_t n, float v, hipStream_t s) {
  if (n > 0) k_fill<<<blocks_for(n, 256), 256, 0, s>>>(p, n, v);
}

// Full-argument form used by the ABI.
void launch_plain_finalize_sets(const float* acc, int taps, int n_hidden, int hidden,
                                int64_t acc_stride, int64_t P, int n_sets, const float* inv_r,
                                float* dw, hipStream_t s) {
  dim3 grid(blocks_for(P, 256), n_sets);
  k_plain_finalize<<<grid, 256, 0, s>>>(acc, taps, n_hidden, hidden, acc_stride, P, inv_r, dw);
}

}  // namespace dpdmi
